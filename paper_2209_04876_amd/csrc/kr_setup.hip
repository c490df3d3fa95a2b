// Factor preprocessing of Algorithm 2 (lines computing the Gram matrix, its
// eigen-decomposition and the leverage scores, and the product-distribution
// data structure), one mode per workgroup:
//   k_promote_all : factors -> FP64 workspace copies (one launch), finiteness check
//   k_gram      : G_n = A_n^T A_n (FP64, LDS row tiles, fixed summation order)
//   k_eig       : cyclic Jacobi eigen-decomposition G_n = V diag(lambda) V^T in one
//                 wave, plus G_n^{-1} = V diag(1/lambda) V^T
//   k_leverage  : l_i = sum_k (a_i . v_k)^2 / lambda_k over the numerical rank
//                 (definition of statistical leverage via the Gram
//                 eigen-decomposition), integer weights Q on the 2^32 grid and the
//                 inclusive CDF used by the sampler.
#include "kr_internal.h"

namespace kr {

#define KR_RMAX 64

// dst[e] = src[e] for e < n by the threads of a workgroup: each thread issues
// SB loads before its LDS stores, so that one memory round trip covers SB
// entries per thread instead of one.
template <int SB>
__device__ __forceinline__ void copy_to_lds(double* dst, const double* __restrict__ src, int n) {
  const int bd = blockDim.x, tid = threadIdx.x;
  for (int e0 = tid; e0 < n; e0 += SB * bd) {
    double v[SB];
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = e0 + u * bd;
      v[u] = src[e < n ? e : n - 1];
    }
#pragma unroll
    for (int u = 0; u < SB; ++u) {
      const int e = e0 + u * bd;
      if (e < n) dst[e] = v[u];
    }
  }
}

// Every mode's factor -> FP64 copy in one launch: blockIdx.y is the mode.
struct PromoteArgs {
  const void* src[KR_MAXN];
  double* dst[KR_MAXN];
  int64_t cnt[KR_MAXN];
};
__global__ void k_promote_all(PromoteArgs a, int dtype, int32_t* __restrict__ flags) {
  const int n = blockIdx.y;
  const void* __restrict__ src = a.src[n];
  double* __restrict__ dst = a.dst[n];
  const int64_t cnt = a.cnt[n];
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = dtype == KR_F32 ? (double)((const float*)src)[i] : ((const double*)src)[i];
    dst[i] = v;
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flags, KR_FLAG_NONFINITE);
}

// One workgroup (256 threads, four waves) per mode, on v_mfma_f64_16x16x4: for
// each 16 x 16 tile (a, b) of G = A^T A, a step takes four rows k..k+3 of A as the
// A operand (A^T: lane l holds A[k + l/16][16a + l%16]) and the B operand (lane l
// holds A[k + l/16][16b + l%16]); wave w takes the steps of rows 4w, 4w + 16, ...
// (coalesced 4-row blocks, eight steps' loads issued together), and the four
// waves' tiles are added in wave order through LDS.  Only the tiles and entries
// on and above the diagonal are formed; each is written to both halves.
typedef double gm_f64x4 __attribute__((ext_vector_type(4)));
#define GM_UNROLL 8
__global__ void __launch_bounds__(256) k_gram(ModeTables T, Geom g, double* __restrict__ gram) {
  __shared__ double part[4 * 256];
  const int n = blockIdx.x;
  const int I = g.I[n], R = g.R[n];
  const double* __restrict__ A = T.A[n];
  double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int nb = (R + 15) / 16;
  // tiles a <= b only; G[c][r] is written as G[r][c] (exactly symmetric)
  for (int tile = 0; tile < nb * nb; ++tile) {
    if (tile / nb > tile % nb) continue;   // uniform
    const int a0 = 16 * (tile / nb), b0 = 16 * (tile % nb);
    const int ca = a0 + col, cb = b0 + col;
    gm_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    // rows k = 16 t + 4 w + kq for step t of this wave
    for (int t0 = 0; 16 * t0 < I; t0 += GM_UNROLL) {
      double va[GM_UNROLL], vb[GM_UNROLL];
#pragma unroll
      for (int u = 0; u < GM_UNROLL; ++u) {
        const int k = 16 * (t0 + u) + 4 * w + kq;
        const bool ok = k < I;
        va[u] = (ok && ca < R) ? A[(size_t)k * R + ca] : 0.0;
        vb[u] = (ok && cb < R) ? A[(size_t)k * R + cb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < GM_UNROLL; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], vb[u], acc, 0, 0, 0);
    }
    // D lane l item v = G[a0 + l/16 + 4v][b0 + l%16]
#pragma unroll
    for (int v = 0; v < 4; ++v) part[w * 256 + (kq + 4 * v) * 16 + col] = acc[v];
    __syncthreads();
    {
      const int e = threadIdx.x, r = a0 + e / 16, c = b0 + e % 16;
      const double sum = ((part[e] + part[256 + e]) + part[512 + e]) + part[768 + e];
      if (r < R && c < R && r <= c) {
        G[r * R + c] = sum;
        G[c * R + r] = sum;
      }
    }
    __syncthreads();
  }
}

// One wave per mode.  Two-sided Jacobi with the round-robin (tournament)
// ordering: each round applies floor(R/2) disjoint rotations at once, A <- J^T A J
// and V <- V J; R-1 rounds (R even; R rounds with a dummy player when R is odd)
// make a sweep.  The rotations of a round act on disjoint index pairs, so the
// update splits into independent 2x2 blocks (rows of pair k, columns of pair l),
// each transformed by one lane.  A rotation is skipped when |a_pq| <=
// 1e-16 sqrt(|a_pp a_qq|) (the rounding level); sweeps stop when a sweep performs
// no rotation.
__global__ void __launch_bounds__(64) k_eig(ModeTables T, Geom g, const double* __restrict__ gram,
                                            int32_t* __restrict__ flags) {
  __shared__ double a[KR_RMAX * KR_RMAX];
  __shared__ double v[KR_RMAX * KR_RMAX];
  __shared__ double cs_c[KR_RMAX / 2], cs_s[KR_RMAX / 2];
  __shared__ int cs_p[KR_RMAX / 2], cs_q[KR_RMAX / 2];
  __shared__ int rotated;
  const int n = blockIdx.x;
  const int R = g.R[n], I = g.I[n];
  const int lane = threadIdx.x;
  const double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  copy_to_lds<16>(a, G, R * R);
  for (int e = lane; e < R * R; e += 64) v[e] = (e / R == e % R) ? 1.0 : 0.0;
  const int mpl = (R & 1) ? R + 1 : R;   // players in the round-robin (dummy = R when odd)
  const int npair = mpl / 2;
  const int nblk = npair * npair;
  __syncthreads();
  for (int sweep = 0; sweep < 60 && R > 1; ++sweep) {
    if (lane == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < mpl - 1; ++round) {
      if (lane < npair) {
        int p, q;
        if (lane == 0) { p = mpl - 1; q = round; }
        else {
          p = round + lane; if (p >= mpl - 1) p -= mpl - 1;
          q = round - lane; if (q < 0) q += mpl - 1;
        }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, sn = 0.0;
        if (q < R) {
          const double apq = a[p * R + q], app = a[p * R + p], aqq = a[q * R + q];
          if (!(apq == 0.0 || fabs(apq) <= 1e-16 * sqrt(fabs(app * aqq)))) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            rotated = 1;
          }
        }
        cs_c[lane] = c; cs_s[lane] = sn;
        cs_p[lane] = p; cs_q[lane] = q;   // q == R marks the dummy
      }
      __syncthreads();
      // A <- J^T A J by 2x2 blocks: rows {p_k, q_k} x columns {p_l, q_l}
      for (int b = lane; b < nblk; b += 64) {
        const int k = b / npair, l = b - k * npair;
        const int pk = cs_p[k], qk = cs_q[k], pl = cs_p[l], ql = cs_q[l];
        const double ck = cs_c[k], sk = cs_s[k], cl = cs_c[l], sl = cs_s[l];
        const bool qkv = qk < R, qlv = ql < R;
        const double b00 = a[pk * R + pl];
        const double b01 = qlv ? a[pk * R + ql] : 0.0;
        const double b10 = qkv ? a[qk * R + pl] : 0.0;
        const double b11 = (qkv && qlv) ? a[qk * R + ql] : 0.0;
        // columns: [x0 x1] <- [c x0 - s x1, s x0 + c x1] with pair l
        const double c00 = cl * b00 - sl * b01, c01 = sl * b00 + cl * b01;
        const double c10 = cl * b10 - sl * b11, c11 = sl * b10 + cl * b11;
        // rows with pair k; the element a rotation annihilates is set to exactly
        // zero (left to rounding it would keep re-triggering rotations)
        const bool annihilated = k == l && sk != 0.0;
        a[pk * R + pl] = ck * c00 - sk * c10;
        if (qlv) a[pk * R + ql] = annihilated ? 0.0 : ck * c01 - sk * c11;
        if (qkv) a[qk * R + pl] = annihilated ? 0.0 : sk * c00 + ck * c10;
        if (qkv && qlv) a[qk * R + ql] = sk * c01 + ck * c11;
      }
      // V <- V J: row i, pair l
      for (int e = lane; e < R * npair; e += 64) {
        const int i = e / npair, l = e - i * npair;
        const int pl = cs_p[l], ql = cs_q[l];
        if (ql >= R) continue;
        const double cl = cs_c[l], sl = cs_s[l];
        const double vip = v[i * R + pl], viq = v[i * R + ql];
        v[i * R + pl] = cl * vip - sl * viq;
        v[i * R + ql] = sl * vip + cl * viq;
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  __syncthreads();
  double* V = T.V[n];
  double* ev = T.evals[n];
  for (int e = lane; e < R * R; e += 64) V[e] = v[e];
  double lmax = 0.0;
  for (int k = 0; k < R; ++k) lmax = fmax(lmax, a[k * R + k]);
  const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
  const double thr = eps_r * eps_r * lmax;
  bool sing = false;
  for (int k = 0; k < R; ++k) sing |= !(a[k * R + k] > thr);
  for (int k = lane; k < R; k += 64) ev[k] = a[k * R + k];
  if (sing) {
    if (lane == 0) atomicOr(flags, KR_FLAG_SINGULAR);
  }
  // G^{-1} = V diag(1/lambda) V^T over the numerical rank (pseudo-inverse)
  double* Gi = T.Ginv[n];
  for (int e = lane; e < R * R; e += 64) {
    const int p = e / R, q = e % R;
    double s = 0.0;
    for (int k = 0; k < R; ++k) {
      const double lk = a[k * R + k];
      if (lk > thr) s += v[p * R + k] * v[q * R + k] / lk;
    }
    Gi[e] = s;
  }
}

// The value of lane l (uniform l) of a float64 register.
__device__ __forceinline__ double chol_lane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// lambda = 0 without the eigenvectors: one wave per mode factors G = L L^T
// (right-looking Cholesky; a pivot at or below max(I,R) eps max_i G_ii -- the
// resolution of G itself -- flags the factor singular and is clamped there),
// forms L^{-1} column by column (lane c
// owns column c, in registers) and writes G^{-1} = L^{-T} L^{-1}, V := L^{-T} and
// unit "eigenvalues".  k_leverage then computes sum_k (a_i . V[:,k])^2 = ||L^{-1}
// a_i||^2 = a_i^T G^{-1} a_i, the leverage score of row i.
template <int RM>
__global__ void __launch_bounds__(64) k_chol(ModeTables T, Geom g, const double* __restrict__ gram,
                                             int32_t* __restrict__ flags) {
  static_assert(RM <= 16, "k_chol holds a row per lane for R <= 16");
  __shared__ double li[RM * RM];
  const int n = blockIdx.x;
  const int R = g.R[n], I = g.I[n];
  const int lane = threadIdx.x;
  const double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  // Lane i holds row i of G padded to RM x RM with the identity (R <= RM <= 16).
  // Every loop runs RM steps, so the code unrolls into straight-line selects with
  // compile-time register indices; the padding leaves the leading R x R block's
  // operations exactly those of the unpadded factorisation (padded entries meet
  // the real ones only through exact zeros) and is never stored.
  double row[RM];
  {
    const int li0 = lane < R ? lane : R - 1;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
      const double gv = G[li0 * R + (k < R ? k : R - 1)];   // unconditional loads
      row[k] = (lane < R && k < R) ? gv : (k == lane ? 1.0 : 0.0);
    }
  }
  double dmax = 0.0;
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    const double dk = chol_lane(row[k], k);
    dmax = k < R ? fmax(dmax, dk) : dmax;
  }
  const double thr = (double)max(I, R) * 2.220446049250313e-16 * dmax;
  // Right-looking factorisation: column j's diagonal and entries L_kj reach every
  // lane by readlane.  Each entry sees the same operations in the same order as a
  // column-by-column update in memory.
  bool sing = false;
  double dinv[RM];
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    double d = chol_lane(row[j], j);
    const bool bad = j < R && !(d > thr);
    sing = sing || bad;
    d = bad ? (thr > 0.0 ? thr : 1.0) : d;
    const double l = sqrt(d);
    const double di = 1.0 / l;
    dinv[j] = di;
    const double sc = row[j] * di;
    row[j] = lane == j ? l : (lane > j ? sc : row[j]);
#pragma unroll
    for (int k = j + 1; k < RM; ++k) {
      const double lkj = chol_lane(row[j], k);
      const double upd = row[k] - row[j] * lkj;
      row[k] = (lane > j && k <= lane) ? upd : row[k];
    }
  }
  // column c = lane of L^{-1}: x_i = 0 (i < c), x_c = 1 / L_cc,
  // x_i = -(sum_{k<i} L_ik x_k) / L_ii, with L_ik = row[k] of lane i
  double x[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < i; ++k) acc = fma(chol_lane(row[k], i), x[k], acc);
    x[i] = i < R ? (i < lane ? 0.0 : (i == lane ? dinv[i] : -acc * dinv[i])) : 0.0;
  }
  if (lane < RM)
#pragma unroll
    for (int i = 0; i < RM; ++i) li[i * RM + lane] = x[i];
  __syncthreads();
  // lane p: V[p][q] = (L^{-1})_qp and G^{-1}[p][q] = sum_{k >= max(p,q)} (L^{-1})_kp (L^{-1})_kq,
  // summed in increasing k (the terms below max(p,q) are exact zeros, so acc
  // meets its first nonzero term at k = max(p,q); the terms k >= R are skipped)
  double* V = T.V[n];
  double* ev = T.evals[n];
  double* Gi = T.Ginv[n];
#pragma unroll
  for (int q = 0; q < RM; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RM; ++k) {
      const double t = fma(x[k], li[k * RM + q], acc);
      acc = k < R ? t : acc;
    }
    if (lane < R && q < R) {
      V[lane * R + q] = x[q];
      Gi[lane * R + q] = acc;
    }
  }
  for (int k = lane; k < R; k += 64) ev[k] = 1.0;
  if (lane == 0 && sing) atomicOr(flags, KR_FLAG_SINGULAR);
}

// The same factorisation for 16 < R <= RM (32 or 64), with the row's updates
// under lane conditions: unrolled straight-line code would not fit the registers there.
template <int RM>
__global__ void __launch_bounds__(64) k_chol_wide(ModeTables T, Geom g, const double* __restrict__ gram,
                                             int32_t* __restrict__ flags) {
  __shared__ double a[KR_RMAX * KR_RMAX];
  __shared__ double li[KR_RMAX * KR_RMAX];
  __shared__ double dinv[KR_RMAX];
  __shared__ int sing;
  const int n = blockIdx.x;
  const int R = g.R[n], I = g.I[n];
  const int lane = threadIdx.x;
  const double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  copy_to_lds<16>(a, G, R * R);
  if (lane == 0) sing = 0;
  __syncthreads();
  double dmax = 0.0;
  for (int k = 0; k < R; ++k) dmax = fmax(dmax, a[k * R + k]);
  const double thr = (double)max(I, R) * 2.220446049250313e-16 * dmax;
  // Right-looking factorisation with lane i holding row i in registers (R <= RM
  // <= 64): column j's diagonal and entries L_kj reach every lane by readlane, so
  // the steps need neither LDS round trips nor barriers.  Each entry sees the same
  // operations in the same order as a column-by-column update in memory.
  {
    double row[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) row[k] = (lane < R && k < R) ? a[lane * R + k] : 0.0;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j < R) {
        double d = chol_lane(row[j], j);
        if (!(d > thr)) {
          if (lane == 0) sing = 1;
          d = thr > 0.0 ? thr : 1.0;
        }
        const double l = sqrt(d);
        const double di = 1.0 / l;
        if (lane == j) row[j] = l;
        if (lane > j) row[j] *= di;
        if (lane == 0) dinv[j] = di;
#pragma unroll
        for (int k = j + 1; k < RM; ++k) {
          if (k < R) {
            const double lkj = chol_lane(row[j], k);
            if (lane > j && k <= lane) row[k] -= row[j] * lkj;
          }
        }
      }
    }
    if (lane < R)
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k < R) a[lane * R + k] = row[k];
  }
  __syncthreads();
  // column c of L^{-1}: x_i = 0 (i < c), x_c = 1 / L_cc, x_i = -(sum_{k<i} L_ik x_k) / L_ii
  if (lane < R) {
    const int c = lane;
    double x[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) acc = fma(i < R ? a[i * R + k] : 0.0, x[k], acc);
      x[i] = i < c ? 0.0 : (i == c ? dinv[i] : (i < R ? -acc * dinv[i] : 0.0));
    }
#pragma unroll
    for (int i = 0; i < RM; ++i)
      if (i < R) li[i * R + c] = x[i];
  }
  __syncthreads();
  double* V = T.V[n];
  double* ev = T.evals[n];
  double* Gi = T.Ginv[n];
  for (int e = lane; e < R * R; e += 64) {
    const int p = e / R, q = e % R;
    V[e] = li[q * R + p];
    double acc = 0.0;
    for (int k = max(p, q); k < R; ++k) acc = fma(li[k * R + p], li[k * R + q], acc);
    Gi[e] = acc;
  }
  for (int k = lane; k < R; k += 64) ev[k] = 1.0;
  if (lane == 0 && sing) atomicOr(flags, KR_FLAG_SINGULAR);
}

// One workgroup (256 threads) per mode.  A thread takes rows tid, tid + 256, ...;
// when every row of the mode fits LV rows per thread, its rows' scores and
// weights stay in registers from the leverage through the CDF (no global round
// trips between the stages), and the CDF is a wave-shuffle scan.
template <int RM>
__global__ void __launch_bounds__(256) k_leverage(ModeTables T, Geom g, int32_t* __restrict__ flags) {
  constexpr int LV = RM <= 8 ? 4 : (RM <= 16 ? 2 : 1);
  __shared__ double vs[KR_RMAX * KR_RMAX];
  __shared__ double inv[2 * KR_RMAX];
  __shared__ double red[8];
  __shared__ unsigned long long ured[4];
  __shared__ unsigned long long umax[4];
  __shared__ unsigned long long wtot[4];
  __shared__ long long fixv[2];
  const int n = blockIdx.x;
  const int I = g.I[n], R = g.R[n];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* A = T.A[n];
  double* lev = T.lev[n];
  uint64_t* Q = T.Q[n];
  uint64_t* C = T.C[n];
  copy_to_lds<16>(vs, T.V[n], R * R);
  if (tid < R) inv[tid] = T.evals[n][tid];
  __syncthreads();
  if (tid < R) {
    double lmax = 0.0;
    for (int k = 0; k < R; ++k) lmax = fmax(lmax, inv[k]);
    const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
    const double lk = inv[tid];
    inv[tid + KR_RMAX] = lk > eps_r * eps_r * lmax ? 1.0 / lk : 0.0;
  }
  __syncthreads();
  if (tid < R) inv[tid] = inv[tid + KR_RMAX];
  __syncthreads();
  const bool one = I <= LV * 256;   // one trip: every row of this thread in registers
  // leverage per row; thread-local partial sums in increasing row order
  double lr[LV];
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < LV; ++u) lr[u] = 0.0;
  for (int i0 = tid; i0 < I; i0 += LV * 256) {
    // every load unconditional (clamped indices), so the trip's rows are in flight together
    double x[LV][RM];
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int i = i0 + u * 256;
      const double* ai = A + (size_t)(i < I ? i : I - 1) * R;
#pragma unroll
      for (int r = 0; r < RM; ++r) x[u][r] = ai[r < R ? r : R - 1];
    }
    bool zero[LV];
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      zero[u] = true;
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        x[u][r] = r < R ? x[u][r] : 0.0;
        zero[u] &= (x[u][r] == 0.0);
      }
    }
    double l[LV];
#pragma unroll
    for (int u = 0; u < LV; ++u) l[u] = 0.0;
    for (int k = 0; k < R; ++k) {
      double dot[LV];
#pragma unroll
      for (int u = 0; u < LV; ++u) dot[u] = 0.0;
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const double v = vs[(r < R ? r : 0) * R + k];
#pragma unroll
        for (int u = 0; u < LV; ++u) {
          const double t = fma(x[u][r], v, dot[u]);
          dot[u] = r < R ? t : dot[u];
        }
      }
#pragma unroll
      for (int u = 0; u < LV; ++u) l[u] = fma(dot[u] * dot[u], inv[k], l[u]);
    }
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int i = i0 + u * 256;
      const double li = zero[u] ? 0.0 : l[u];
      lr[u] = li;
      if (i < I) {
        lev[i] = li;
        part += li;
      }
    }
  }
  const double S = block_sum(part, red);
  if (!(S > 0.0) || !isfinite(S)) {
    if (tid == 0) atomicOr(flags, KR_FLAG_QUANT);
    return;
  }
  // Q_i = max(1, nearest integer to 2^32 l_i / S) for l_i > 0; exact integer sum and argmax
  unsigned long long qsum = 0ull, best = 0ull;
  uint64_t qr[LV];
#pragma unroll
  for (int u = 0; u < LV; ++u) qr[u] = 0ull;
  for (int i0 = tid; i0 < I; i0 += LV * 256) {
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int i = i0 + u * 256;
      if (i < I) {
        const double l = one ? lr[u] : lev[i];
        uint64_t q = 0;
        if (l > 0.0) {
          q = (uint64_t)floor((l / S) * 4294967296.0 + 0.5);
          if (q < 1) q = 1;
        }
        Q[i] = q;
        qr[u] = q;
        qsum += q;
        // pack (q, lowest index wins on ties) into a comparable key: q high, ~i low
        const unsigned long long key = ((unsigned long long)q << 24) | (unsigned long long)(0xFFFFFF - i);
        best = key > best ? key : best;
      }
    }
  }
  // reductions (integer: order-independent); the deficit 2^32 - sum goes to the
  // largest weight (lowest index on ties)
  for (int o = 32; o > 0; o >>= 1) {
    qsum += __shfl_xor(qsum, o, 64);
    const unsigned long long ob = __shfl_xor(best, o, 64);
    best = ob > best ? ob : best;
  }
  if (lane == 0) { ured[w] = qsum; umax[w] = best; }
  __syncthreads();
  if (tid == 0) {
    unsigned long long s2 = 0, b2 = 0;
    for (int k = 0; k < 4; ++k) { s2 += ured[k]; b2 = umax[k] > b2 ? umax[k] : b2; }
    const int j = 0xFFFFFF - (int)(b2 & 0xFFFFFFull);
    const long long deficit = (long long)(1ull << 32) - (long long)s2;
    fixv[0] = j;
    fixv[1] = deficit;
    if (!one) {
      const long long qj = (long long)Q[j] + deficit;
      if (qj < 1) atomicOr(flags, KR_FLAG_QUANT);
      else Q[j] = (uint64_t)qj;
    }
  }
  __syncthreads();
  if (one) {
    const int j = (int)fixv[0];
    if ((j & 255) == tid) {
#pragma unroll
      for (int u = 0; u < LV; ++u)
        if (u == (j >> 8)) {
          const long long qj = (long long)qr[u] + fixv[1];
          if (qj < 1) {
            atomicOr(flags, KR_FLAG_QUANT);
          } else {
            qr[u] = (uint64_t)qj;
            Q[j] = (uint64_t)qj;
          }
        }
    }
  }
  // inclusive CDF over 256-entry blocks (block b: entries 256 b + tid), each a
  // wave-shuffle scan plus the preceding waves' totals, with a running carry
  unsigned long long carry = 0ull;
  for (int c0 = 0; c0 < I; c0 += LV * 256) {
#pragma unroll
    for (int u = 0; u < LV; ++u) {
      const int base = c0 + u * 256;
      if (base < I) {   // uniform
        const int i = base + tid;
        unsigned long long v = i < I ? (one ? qr[u] : Q[i]) : 0ull;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const unsigned long long t = __shfl_up(v, o, 64);
          if (lane >= o) v += t;
        }
        if (lane == 63) wtot[w] = v;
        __syncthreads();
        unsigned long long before = 0ull, total = 0ull;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          before += k < w ? wtot[k] : 0ull;
          total += wtot[k];
        }
        if (i < I) C[i] = carry + before + v;
        carry += total;
        __syncthreads();   // wtot is rewritten by the next block
      }
    }
  }
}

}  // namespace kr
