// Factor preprocessing of Algorithm 2 for large factors, spread over many
// workgroups (the single-workgroup kernels of kr_setup.hip serve small I_n):
//
//   k_gram_part / k_gram_sum  G_n = A_n^T A_n as per-block partial Grams summed in
//                             block order (fixed summation order)
//   k_row_quadform            per row l_i = sum_c w_c (a_i . p_c)^2 for a projection
//                             P staged in LDS: exact leverage (P = V, w = 1/lambda
//                             over the numerical rank), the squared row norms
//                             (P = I), or the Johnson-Lindenstrauss scores (P = Z^T)
//   k_quant_blocks / k_quant_fix / k_cdf_blocks
//                             the integer weights Q on the 2^32 grid and their
//                             inclusive CDF, block by block
//   k_mix_uniform             the even mixture of the squared row norms and the
//                             uniform distribution (the rows' sampling weights)
//   k_approx_rows             the rows of the spectral approximation A~ = S A
//   k_jl_project              Z = (G / sqrt(r)) A~ M, M = (1 + eps/4) (A~^T A~)^+
//
// The approximate path follows Algorithm 2's first loop: a spectral
// approximation A~ by row sampling (Lemma block_sketch_is_spectral_approx) from
// the even mixture of the squared row norms (a beta-overestimate of the leverage
// distribution with beta >= 1/kappa(A)^2) and the uniform distribution (beta = R
// / (I max l)), the eigen-decomposition of A~^T A~ (which also gives the
// preconditioner's V and Sigma), and the approximate scores of Lemma fast-ls-comp
// ||G A~ M a_i||^2 / ((1 + eps/4)(1 - eps/20)) with a Gaussian projection G of r
// rows (Lemma random-projection).
// Random bits: Philox4x64-10, key (seed, stream); row t of A~ for mode n from
// word 0 of counter (t, n, 0, 1) (top 32 bits against the CDF); entry (c, t) of G
// for mode n by Box-Muller on words 0 and 1 of counter (t, c, n, 2).
#include "kr_internal.h"

namespace kr {

#define LV_THREADS 256
#define LV_RPB 4096   // rows per workgroup of the row passes

struct LevPass {
  const double* A[KR_MAXN];
  const double* P[KR_MAXN];     // projection: element (r, c) at P[r * ldr + c * ldc]
  const double* evals[KR_MAXN]; // exact mode: weights 1/lambda_c over the numerical rank
  double wscale;                // JL mode: every weight
  int ldr[KR_MAXN], ldc[KR_MAXN], nc[KR_MAXN];
  double* out[KR_MAXN];
  double* part[KR_MAXN];        // per-block sums of out
  int I[KR_MAXN], R[KR_MAXN];
  int mode;                     // 0: squared row norms; 1: exact (P = V); 2: JL (P = Z^T)
};

// One workgroup per LV_RPB rows of one mode (blockIdx.y).  Rows are held in
// registers; partial sums in increasing row order, then the block's fixed-order sum.
template <int RM>
__global__ void __launch_bounds__(LV_THREADS) k_row_quadform(LevPass a) {
  __shared__ double P[KR_RMAX * KR_RMAX];
  __shared__ double w[KR_RMAX];
  __shared__ double red[LV_THREADS / 64];
  const int n = blockIdx.y;
  const int I = a.I[n], R = a.R[n];
  const int64_t r0 = (int64_t)blockIdx.x * LV_RPB;
  if (r0 >= I) return;
  const int nc = a.mode == 0 ? 0 : a.nc[n];
  if (a.mode != 0) {
    for (int e = threadIdx.x; e < R * nc; e += blockDim.x) {
      const int r = e / nc, c = e - r * nc;
      P[r * nc + c] = a.P[n][(int64_t)r * a.ldr[n] + (int64_t)c * a.ldc[n]];
    }
    if (threadIdx.x < nc) {
      if (a.mode == 1) {
        double lmax = 0.0;
        for (int k = 0; k < nc; ++k) lmax = fmax(lmax, a.evals[n][k]);
        const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
        const double lk = a.evals[n][threadIdx.x];
        w[threadIdx.x] = lk > eps_r * eps_r * lmax ? 1.0 / lk : 0.0;
      } else {
        w[threadIdx.x] = a.wscale;
      }
    }
  }
  __syncthreads();
  const int64_t r1 = min((int64_t)I, r0 + LV_RPB);
  const double* A = a.A[n];
  double* out = a.out[n];
  double part = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double* ai = A + i * R;
    double x[RM];
    bool zero = true;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      x[r] = r < R ? ai[r] : 0.0;
      zero &= (x[r] == 0.0);
    }
    double l = 0.0;
    if (a.mode == 0) {
#pragma unroll
      for (int r = 0; r < RM; ++r) l = fma(x[r], x[r], l);
    } else {
      for (int c = 0; c < nc; ++c) {
        double dot = 0.0;
#pragma unroll
        for (int r = 0; r < RM; ++r)
          if (r < R) dot = fma(x[r], P[r * nc + c], dot);
        l = fma(dot * dot, w[c], l);
      }
    }
    if (zero) l = 0.0;
    out[i] = l;
    part += l;
  }
  const double s = block_sum(part, red);
  if (threadIdx.x == 0) a.part[n][blockIdx.x] = s;
}

// Row weights of the spectral approximation: the even mixture of the squared row
// norms and the uniform distribution, w_i <- w_i / S + 1/I (S the row-norm block
// sums added in block order), with the new block sums in part_out (a separate
// array: other blocks still read part_in).
struct MixPass {
  double* w[KR_MAXN];
  const double* part_in[KR_MAXN];
  double* part_out[KR_MAXN];
  int I[KR_MAXN], nb[KR_MAXN];
};

__global__ void __launch_bounds__(LV_THREADS) k_mix_uniform(MixPass a) {
  __shared__ double red[LV_THREADS / 64];
  __shared__ double Ssh;
  const int n = blockIdx.y;
  if (blockIdx.x >= (unsigned)a.nb[n]) return;
  const int I = a.I[n];
  if (threadIdx.x == 0) {
    double S = 0.0;
    for (int b = 0; b < a.nb[n]; ++b) S += a.part_in[n][b];
    Ssh = S;
  }
  __syncthreads();
  const double S = Ssh, u = 1.0 / (double)I;
  const int64_t r0 = (int64_t)blockIdx.x * LV_RPB;
  const int64_t r1 = min((int64_t)I, r0 + LV_RPB);
  double part = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double v = (S > 0.0 ? a.w[n][i] / S : 0.0) + u;
    a.w[n][i] = v;
    part += v;
  }
  const double t = block_sum(part, red);
  if (threadIdx.x == 0) a.part_out[n][blockIdx.x] = t;
}

struct QuantPass {
  const double* w[KR_MAXN];     // non-negative weights (I_n)
  const double* part[KR_MAXN];  // their per-block sums (nb_n)
  uint64_t* Q[KR_MAXN];
  uint64_t* C[KR_MAXN];
  uint64_t* qpart[KR_MAXN];     // per-block sums of Q, then exclusive block offsets
  uint64_t* qbest[KR_MAXN];     // per-block argmax keys
  int I[KR_MAXN];
  int nb[KR_MAXN];
};

// Q_i = max(1, nearest integer to 2^32 w_i / S) for w_i > 0 (S = the block sums
// added in block order, the same in every block); the block's integer sum and its
// argmax key (q high, the complement of i low: lowest index wins on ties).
__global__ void __launch_bounds__(LV_THREADS) k_quant_blocks(QuantPass a, int32_t* __restrict__ flags) {
  __shared__ unsigned long long us[LV_THREADS / 64], ub[LV_THREADS / 64];
  __shared__ double Ssh;
  const int n = blockIdx.y;
  const int I = a.I[n];
  const int64_t r0 = (int64_t)blockIdx.x * LV_RPB;
  if (blockIdx.x >= (unsigned)a.nb[n]) return;
  if (threadIdx.x == 0) {
    double S = 0.0;
    for (int b = 0; b < a.nb[n]; ++b) S += a.part[n][b];
    Ssh = S;
  }
  __syncthreads();
  const double S = Ssh;
  if (!(S > 0.0) || !isfinite(S)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(flags, KR_FLAG_QUANT);
    return;
  }
  const int64_t r1 = min((int64_t)I, r0 + LV_RPB);
  unsigned long long qsum = 0ull, best = 0ull;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double l = a.w[n][i];
    uint64_t q = 0;
    if (l > 0.0) {
      q = (uint64_t)floor((l / S) * 4294967296.0 + 0.5);
      if (q < 1) q = 1;
    }
    a.Q[n][i] = q;
    qsum += q;
    const unsigned long long key = ((unsigned long long)q << 24) | (unsigned long long)(0xFFFFFF - i);
    best = key > best ? key : best;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    qsum += __shfl_xor(qsum, o, 64);
    const unsigned long long ob = __shfl_xor(best, o, 64);
    best = ob > best ? ob : best;
  }
  if (lane == 0) { us[wv] = qsum; ub[wv] = best; }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0, b = 0;
    for (int k = 0; k < LV_THREADS / 64; ++k) { s += us[k]; b = ub[k] > b ? ub[k] : b; }
    a.qpart[n][blockIdx.x] = s;
    a.qbest[n][blockIdx.x] = b;
  }
}

// One thread per mode: the rounding deficit 2^32 - sum Q goes to the largest
// weight; the block sums become exclusive offsets for the CDF.
__global__ void k_quant_fix(QuantPass a, int N, int32_t* __restrict__ flags) {
  const int n = threadIdx.x;
  if (n >= N) return;
  const int nb = a.nb[n];
  unsigned long long s = 0, b = 0;
  for (int k = 0; k < nb; ++k) { s += a.qpart[n][k]; b = a.qbest[n][k] > b ? a.qbest[n][k] : b; }
  if (s == 0ull) return;   // k_quant_blocks has flagged it
  const int64_t j = 0xFFFFFF - (int64_t)(b & 0xFFFFFFull);
  const long long deficit = (long long)(1ull << 32) - (long long)s;
  const long long qj = (long long)a.Q[n][j] + deficit;
  if (qj < 1) { atomicOr(flags, KR_FLAG_QUANT); return; }
  a.Q[n][j] = (uint64_t)qj;
  const int bj = (int)(j / LV_RPB);
  unsigned long long off = 0;
  for (int k = 0; k < nb; ++k) {
    const unsigned long long v = a.qpart[n][k] + (k == bj ? (unsigned long long)deficit : 0ull);
    a.qpart[n][k] = off;
    off += v;
  }
}

// Inclusive CDF of each block's Q from its offset, 256 entries per step.
__global__ void __launch_bounds__(LV_THREADS) k_cdf_blocks(QuantPass a) {
  __shared__ unsigned long long scan[LV_THREADS];
  __shared__ unsigned long long carry;
  const int n = blockIdx.y;
  if (blockIdx.x >= (unsigned)a.nb[n]) return;
  const int I = a.I[n];
  const int64_t r0 = (int64_t)blockIdx.x * LV_RPB;
  const int64_t r1 = min((int64_t)I, r0 + LV_RPB);
  if (threadIdx.x == 0) carry = a.qpart[n][blockIdx.x];
  __syncthreads();
  for (int64_t base = r0; base < r1; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    scan[threadIdx.x] = i < r1 ? a.Q[n][i] : 0ull;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const unsigned long long add = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0ull;
      __syncthreads();
      scan[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < r1) a.C[n][i] = carry + scan[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) carry += scan[blockDim.x - 1];
    __syncthreads();
  }
}

// Per-block partial Grams: block b of mode n sums rows [b LV_RPB, (b+1) LV_RPB)
// in increasing order into its own R x R slot (thread t owns entries t, t+256, ...).
struct GramPass {
  const double* A[KR_MAXN];
  double* part[KR_MAXN];   // nb_n x R_n^2
  double* gram;            // N x 64 x 64 (the layout k_eig / k_chol read)
  int I[KR_MAXN], R[KR_MAXN], nb[KR_MAXN];
};

__global__ void __launch_bounds__(256) k_gram_part(GramPass a) {
  __shared__ double tile[64 * KR_RMAX];
  const int n = blockIdx.y;
  if (blockIdx.x >= (unsigned)a.nb[n]) return;
  const int I = a.I[n], R = a.R[n];
  const int64_t r0 = (int64_t)blockIdx.x * LV_RPB;
  const int64_t r1 = min((int64_t)I, r0 + LV_RPB);
  const double* A = a.A[n];
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int rows = (int)min((int64_t)64, r1 - rb);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * R; e += blockDim.x) tile[e] = A[rb * R + e];
    __syncthreads();
    int k = 0;
    for (int pq = threadIdx.x; pq < R * R; pq += blockDim.x, ++k) {
      const int p = pq / R, q = pq % R;
      double s = acc[k];
#pragma unroll 8
      for (int i = 0; i < rows; ++i) s = fma(tile[i * R + p], tile[i * R + q], s);
      acc[k] = s;
    }
  }
  double* out = a.part[n] + (size_t)blockIdx.x * R * R;
  int k = 0;
  for (int pq = threadIdx.x; pq < R * R; pq += blockDim.x, ++k) out[pq] = acc[k];
}

__global__ void __launch_bounds__(256) k_gram_sum(GramPass a) {
  const int n = blockIdx.x;
  const int R = a.R[n], nb = a.nb[n];
  double* G = a.gram + (size_t)n * KR_RMAX * KR_RMAX;
  for (int pq = threadIdx.x; pq < R * R; pq += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += a.part[n][(size_t)b * R * R + pq];
    G[pq] = s;
  }
}

// Rows of the spectral approximation: A~[t] = a_i / sqrt(k q'_i), i drawn from the
// inclusive CDF C of the quantised squared row norms Q (q'_i = Q_i 2^-32).
struct ApproxRows {
  const double* A[KR_MAXN];
  const uint64_t* Q[KR_MAXN];
  const uint64_t* C[KR_MAXN];
  double* At[KR_MAXN];    // k_n x R_n
  int I[KR_MAXN], R[KR_MAXN], k[KR_MAXN];
};

__global__ void __launch_bounds__(256) k_approx_rows(ApproxRows a, uint64_t seed, uint64_t stream) {
  const int n = blockIdx.y;
  const int k = a.k[n], R = a.R[n], I = a.I[n];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k) return;
  const u64x4 w = philox4x64_10((uint64_t)t, (uint64_t)n, 0ull, 1ull, seed, stream);
  const uint64_t u = w.v[0] >> 32;
  // first index with C[i] > u
  int lo = 0, hi = I - 1;
  const uint64_t* C = a.C[n];
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (C[mid] > u) hi = mid; else lo = mid + 1;
  }
  const double qp = (double)a.Q[n][lo] * 0x1p-32;
  const double sc = 1.0 / sqrt((double)k * qp);
  const double* ai = a.A[n] + (int64_t)lo * R;
  double* dst = a.At[n] + (int64_t)t * R;
  for (int r = 0; r < R; ++r) dst[r] = ai[r] * sc;
}

// Z[c] = (1 + eps/4) (g_c A~) N^+ for row c of the projection (g_c = G[c, :] /
// sqrt(r)); one workgroup per (c, mode).  Each thread sums its samples t in
// increasing order, then waves and workgroup combine in fixed order.
struct JLPass {
  const double* At[KR_MAXN];
  const double* Ninv[KR_MAXN];   // R_n x R_n
  double* Z[KR_MAXN];            // r x R_n, row-major
  int R[KR_MAXN], k[KR_MAXN];
  int r;
  double coef;                   // 1 + eps/4
};

__device__ __forceinline__ double philox_normal(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t seed,
                                                uint64_t stream) {
  const u64x4 w = philox4x64_10(c0, c1, c2, c3, seed, stream);
  const double u1 = (double)((w.v[0] >> 11) + 1ull) * 0x1p-53;
  const double u2 = (double)(w.v[1] >> 11) * 0x1p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

template <int RM>
__global__ void __launch_bounds__(256) k_jl_project(JLPass a, uint64_t seed, uint64_t stream) {
  __shared__ double red[4][KR_RMAX];
  __shared__ double ga[KR_RMAX];
  const int n = blockIdx.y, c = blockIdx.x;
  const int R = a.R[n], k = a.k[n];
  const double inv_sqrt_r = 1.0 / sqrt((double)a.r);
  double acc[RM];
#pragma unroll
  for (int q = 0; q < RM; ++q) acc[q] = 0.0;
  for (int t = threadIdx.x; t < k; t += blockDim.x) {
    const double gv = philox_normal((uint64_t)t, (uint64_t)c, (uint64_t)n, 2ull, seed, stream) * inv_sqrt_r;
    const double* row = a.At[n] + (int64_t)t * R;
#pragma unroll
    for (int q = 0; q < RM; ++q)
      if (q < R) acc[q] = fma(gv, row[q], acc[q]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < RM; ++q) {
    double v = acc[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0 && q < R) red[wv][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < R) ga[threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
                                         red[3][threadIdx.x];
  __syncthreads();
  if (threadIdx.x < R) {
    const int q = threadIdx.x;
    const double* Ni = a.Ninv[n];
    double s = 0.0;
    for (int p = 0; p < R; ++p) s = fma(ga[p], Ni[p * R + q], s);
    a.Z[n][(int64_t)c * R + q] = a.coef * s;
  }
}

}  // namespace kr
