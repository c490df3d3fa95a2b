// Algorithm 3 (FastFactorMatrixUpdate): the factor update of Tucker ALS for
// mode n, every row i of A(n) solved as its own sketched, penalised regression
//     min_z sum_j Omega_ij (k_j z - X_(n)[i, j])^2 + lam ||(G^T)^+ z||^2 + w ||N z||^2,
//     a_i = (G^T)^+ z,
// with K the Kronecker product of the other factors, G = G_(n) the mode-n
// unfolding of the core, N = I - G^T (G^T)^+ and w = (1 + 12/eps) prod_{m != n}
// lambda_max(G_m) (Lemmas constrained_least_squares and constraint-reg).
//
// The rows become segments of one sample tree: a pseudo-mode 0 whose index is the
// row (no factor), followed by the other modes in increasing order.  Each row
// draws its own sketch (Philox counter word 2 = row).  The shared level kernels
// give every row's sketched gradient part K~^T Omega (K~ z - b~) at its level-1
// node.  The update kernel adds w z + G^+ (lam (G^T)^+ - w G) z and applies
//     M^-1 = A^-1 - A^-1 U (I + V A^-1 U)^-1 V A^-1,
//     A = K^T K + w I,  U = G^+,  V = lam (G^T)^+ - w G
// (Lemma fast_factor_richardson_step, read with the minus sign of the Woodbury
// identity), with A^-1 = (kron V_m) (kron Lambda_m + w)^-1 (kron V_m)^T.
#include "kr_internal.h"

namespace kr {

// Tensor geometry of X for the gathers: mode n of X holds the row; the other
// modes of X are the tree modes 1..N-1 in increasing order.
struct TuckerGeom {
  int Nx;                 // order of X
  int mode;               // n
  int Ix[KR_MAXN];        // dims of X
  int tmode[KR_MAXN];     // X mode of tree mode k (tmode[0] = n)
  int Rn;                 // R_n
  int Rr;                 // prod_{m != n} R_m
  int64_t m_row;          // samples per row
};

// Small dense helpers, one workgroup ------------------------------------------

// In-place inverse of an n x n matrix in LDS by Gauss-Jordan with partial
// pivoting (n <= 64).  Returns false (uniformly) when a pivot is not positive
// relative to the largest diagonal scale.
__device__ bool wg_invert(double* M, double* Inv, int n, int* piv_s, double* scale_s) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) Inv[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(M[i * n + i]));
    *scale_s = mx;
  }
  __syncthreads();
  const double tiny = 1e-13 * (*scale_s);
  for (int c = 0; c < n; ++c) {
    if (threadIdx.x == 0) {
      int p = c;
      double best = fabs(M[c * n + c]);
      for (int r = c + 1; r < n; ++r)
        if (fabs(M[r * n + c]) > best) { best = fabs(M[r * n + c]); p = r; }
      *piv_s = best > tiny ? p : -1;
    }
    __syncthreads();
    const int p = *piv_s;
    if (p < 0) return false;
    if (p != c) {
      for (int k = threadIdx.x; k < n; k += blockDim.x) {
        double t = M[c * n + k]; M[c * n + k] = M[p * n + k]; M[p * n + k] = t;
        t = Inv[c * n + k]; Inv[c * n + k] = Inv[p * n + k]; Inv[p * n + k] = t;
      }
      __syncthreads();
    }
    const double d = M[c * n + c];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) { M[c * n + k] /= d; Inv[c * n + k] /= d; }
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = e / n, k = e % n;
      if (r != c) {
        const double f = M[r * n + c];
        if (k != c) M[r * n + k] -= f * M[c * n + k];
        Inv[r * n + k] -= f * Inv[c * n + k];
      }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x)
      if (r != c) M[r * n + c] = 0.0;
    __syncthreads();
  }
  return true;
}

// A^-1 v for A = K^T K + w I on an R_1 x .. x R_{N-1} vector held in LDS (tree
// modes 1..N-1): t = v x_m V_m^T (all m), t *= 1/(kron Lambda + w), t x_m V_m.
// buf is scratch of the same size.  Works on one vector per workgroup.
__device__ void wg_apply_Ainv(const Geom& g, const ModeTables& T, double w, double* v, double* buf) {
  const int Rr = (int)g.rsuf[1];
  double* cur = v;
  double* nxt = buf;
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 1; k < g.N; ++k) {
      const int Rk = g.R[k];
      const int post = (int)g.rsuf[k + 1];
      const double* V = T.V[k];
      for (int e = threadIdx.x; e < Rr; e += blockDim.x) {
        const int blk = e / (Rk * post), rem = e - blk * Rk * post, a = rem / post, c = rem - a * post;
        const double* src = cur + blk * Rk * post + c;
        double acc = 0.0;
        for (int b = 0; b < Rk; ++b) acc = fma(pass == 0 ? V[b * Rk + a] : V[a * Rk + b], src[b * post], acc);
        nxt[e] = acc;
      }
      __syncthreads();
      double* t = cur; cur = nxt; nxt = t;
    }
    if (pass == 0) {
      for (int e = threadIdx.x; e < Rr; e += blockDim.x) {
        int r = e;
        double prod = 1.0;
        for (int k = g.N - 1; k >= 1; --k) {
          const int rk = r % g.R[k];
          r /= g.R[k];
          prod *= T.evals[k][rk];
        }
        cur[e] /= (prod + w);
      }
      __syncthreads();
    }
  }
  if (cur != v) {
    for (int e = threadIdx.x; e < Rr; e += blockDim.x) v[e] = cur[e];
    __syncthreads();
  }
}

// Row-independent matrices.  One workgroup of 256 threads; LDS holds G G^T and
// its inverse.  Outputs (global, row-major):
//   Gn   R_n x Rr   mode-n unfolding of the core
//   GtP  R_n x Rr   (G^T)^+ = (G G^T)^-1 G
//   Vw   R_n x Rr   lam (G^T)^+ - w G
//   *w_out          the penalty weight
// stage: the unfolding is also kept in dynamic LDS (Rn Rr doubles) and read from
// there by the products below, instead of from global memory inside their loops.
__global__ void __launch_bounds__(256) k_tucker_setup(ModeTables T, Geom g, TuckerGeom tg, const double* __restrict__ core,
                                                     double lambda, double eps, double* __restrict__ Gn,
                                                     double* __restrict__ GtP, double* __restrict__ Vw,
                                                     double* __restrict__ w_out, int32_t* __restrict__ flags,
                                                     int stage) {
  __shared__ double GG[64 * 64];
  __shared__ double Gi[64 * 64];
  __shared__ int piv;
  __shared__ double scl;
  extern __shared__ double ts_dyn[];
  const double* Gr = stage ? (const double*)ts_dyn : (const double*)Gn;
  const int Rn = tg.Rn, Rr = tg.Rr, Nx = tg.Nx, n = tg.mode;
  // core dims R_0..R_{Nx-1} of X order: tree mode k >= 1 carries X mode tmode[k]
  int Rx[KR_MAXN];
  for (int k = 1; k < g.N; ++k) Rx[tg.tmode[k]] = g.R[k];
  Rx[n] = Rn;
  // Gn[r][c]: c is the row-major index over the other modes (tree order = X order)
  for (int e = threadIdx.x; e < Rn * Rr; e += blockDim.x) {
    const int r = e / Rr;
    int c = e - r * Rr;
    int64_t lin = 0;
    int64_t mul = 1;
    for (int m = Nx - 1; m >= 0; --m) {
      int im;
      if (m == n) im = r;
      else { im = c % Rx[m]; c /= Rx[m]; }
      lin += im * mul;
      mul *= Rx[m];
    }
    const double v = core[lin];
    Gn[e] = v;
    if (stage) ts_dyn[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < Rn * Rn; e += blockDim.x) {
    const int a = e / Rn, b = e % Rn;
    double s = 0.0;
    for (int c = 0; c < Rr; ++c) s = fma(Gr[a * Rr + c], Gr[b * Rr + c], s);
    GG[e] = s;
  }
  __syncthreads();
  const bool ok = wg_invert(GG, Gi, Rn, &piv, &scl);
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(flags, KR_FLAG_CORE);
    return;
  }
  double w = 1.0 + 12.0 / eps;
  for (int k = 1; k < g.N; ++k) {
    double mx = 0.0;
    for (int r = 0; r < g.R[k]; ++r) mx = fmax(mx, T.evals[k][r]);
    w *= mx;
  }
  if (threadIdx.x == 0) *w_out = w;
  for (int e = threadIdx.x; e < Rn * Rr; e += blockDim.x) {
    const int r = e / Rr, c = e - r * Rr;
    double s = 0.0;
    for (int b = 0; b < Rn; ++b) s = fma(Gi[r * Rn + b], Gr[b * Rr + c], s);
    GtP[e] = s;
    Vw[e] = lambda * s - w * Gr[e];
  }
}

// AinvU[:, k] = A^-1 U[:, k] with U = G^+ = GtP^T; one workgroup per column k.
// Stored row-major Rr x R_n.
__global__ void __launch_bounds__(256) k_tucker_ainvu(ModeTables T, Geom g, TuckerGeom tg, const double* __restrict__ GtP,
                                                     const double* __restrict__ w_in, double* __restrict__ AinvU) {
  extern __shared__ double sm[];
  const int Rr = tg.Rr, Rn = tg.Rn, k = blockIdx.x;
  double* v = sm;
  double* buf = sm + Rr;
  for (int e = threadIdx.x; e < Rr; e += blockDim.x) v[e] = GtP[k * Rr + e];
  __syncthreads();
  wg_apply_Ainv(g, T, *w_in, v, buf);
  for (int e = threadIdx.x; e < Rr; e += blockDim.x) AinvU[e * Rn + k] = v[e];
}

// Cinv = (I + V A^-1 U)^-1, R_n x R_n; one workgroup.
// stage: Vw and AinvU are first copied to dynamic LDS (2 Rn Rr doubles) with
// coalesced loads, and the product reads them there.
__global__ void __launch_bounds__(256) k_tucker_cinv(TuckerGeom tg, const double* __restrict__ Vw,
                                                    const double* __restrict__ AinvU, double* __restrict__ Cinv,
                                                    int32_t* __restrict__ flags, int stage) {
  __shared__ double C[64 * 64];
  __shared__ double Ci[64 * 64];
  __shared__ int piv;
  __shared__ double scl;
  extern __shared__ double tc_dyn[];
  const int Rn = tg.Rn, Rr = tg.Rr;
  const double* Vr = Vw;
  const double* Ar = AinvU;
  if (stage) {
    for (int e = threadIdx.x; e < Rn * Rr; e += blockDim.x) {
      tc_dyn[e] = Vw[e];
      tc_dyn[Rn * Rr + e] = AinvU[e];
    }
    __syncthreads();
    Vr = tc_dyn;
    Ar = tc_dyn + Rn * Rr;
  }
  for (int e = threadIdx.x; e < Rn * Rn; e += blockDim.x) {
    const int a = e / Rn, b = e % Rn;
    double s = (a == b) ? 1.0 : 0.0;
    for (int c = 0; c < Rr; ++c) s = fma(Vr[a * Rr + c], Ar[c * Rn + b], s);
    C[e] = s;
  }
  __syncthreads();
  if (!wg_invert(C, Ci, Rn, &piv, &scl)) {
    if (threadIdx.x == 0) atomicOr(flags, KR_FLAG_CORE);
    return;
  }
  for (int e = threadIdx.x; e < Rn * Rn; e += blockDim.x) Cinv[e] = Ci[e];
}

// Sampling for all rows: sample T = row * m_row + t draws, for tree modes k >= 1,
// the word (k-1)%4 of Philox block (t, (k-1)/4, row, 0).
__global__ void __launch_bounds__(256) k_sample_rows(ModeTables T, Geom g, TuckerGeom tg, uint64_t seed,
                                                    uint64_t stream, uint64_t* __restrict__ keys) {
  for (int64_t Tt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; Tt < g.m; Tt += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = Tt / tg.m_row, t = Tt - row * tg.m_row;
    uint64_t key = (uint64_t)row << g.shift[0];
    for (int grp = 0; grp * 4 < g.N - 1; ++grp) {
      const u64x4 w = philox4x64_10((uint64_t)t, (uint64_t)grp, (uint64_t)row, 0ull, seed, stream);
      for (int q = 0; q < 4 && grp * 4 + q < g.N - 1; ++q) {
        const int k = 1 + grp * 4 + q;
        const uint64_t u = w.v[q] >> 32;
        int lo = 0, hi = g.I[k];
        const uint64_t* c = T.C[k];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (c[mid] <= u) lo = mid + 1; else hi = mid;
        }
        key |= (uint64_t)lo << g.shift[k];
      }
    }
    keys[Tt] = key;
  }
}

// Distinct rows of all sketches: Omega_j = count_j / (m_row prod_{k>=1} p'_{i_k});
// b~_j = X[row, i_1, ...] with the row in X mode n.
__global__ void __launch_bounds__(256) k_rows_tucker(ModeTables T, Geom g, TuckerGeom tg, Tree tr,
                                                    const void* __restrict__ X, int x_dtype,
                                                    double* __restrict__ Omega, double* __restrict__ bD,
                                                    int32_t* __restrict__ counts, int32_t* __restrict__ flags) {
  const int64_t D = tr.cnt[g.N];
  int bad = 0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < D; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = tr.rstart[j + 1] - tr.rstart[j];
    const uint64_t key = tr.rkey[j];
    int ix[KR_MAXN];
    double den = (double)tg.m_row;
    for (int k = 0; k < g.N; ++k) {
      const int i = (int)((key >> g.shift[k]) & ((1ull << g.bits[k]) - 1ull));
      ix[tg.tmode[k]] = i;
      if (k >= 1) den = den * ((double)T.Q[k][i] * 0x1p-32);
    }
    int64_t lin = 0;
    for (int m = 0; m < tg.Nx; ++m) lin = lin * tg.Ix[m] + ix[m];
    Omega[j] = (double)c * (1.0 / den);
    counts[j] = c;
    const double v = x_dtype == KR_F32 ? (double)((const float*)X)[lin] : ((const double*)X)[lin];
    bD[j] = v;
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flags, KR_FLAG_NONFINITE);
}

__device__ void tucker_row_stop(int i, double dd, double zz, double eta, double tol, int it,
                                int32_t* __restrict__ seg_done, int32_t* __restrict__ seg_iters,
                                double* __restrict__ seg_rel, double* __restrict__ seg_d0,
                                double* __restrict__ seg_best, int32_t* __restrict__ seg_stall,
                                int32_t* __restrict__ ndone, int32_t* __restrict__ diverged);

// Per-row update, one workgroup per row i (the level-1 node of row i is node i:
// every row has at least one sample and rows sort first):
//   h = Q1[i] + w z + U (V z);  d = A^-1 h - AinvU Cinv V A^-1 h;  z -= eta d
// and the row's stopping rule (relative step <= tol, or stagnation on the
// rounding floor).  seg_done / seg_iters / seg_rel / seg_best / seg_stall are per
// row; *ndone counts converged rows.
__global__ void __launch_bounds__(256) k_tucker_update(ModeTables T, Geom g, TuckerGeom tg, const double* __restrict__ Q1,
                                                      double* __restrict__ Z, const double* __restrict__ GtP,
                                                      const double* __restrict__ Vw, const double* __restrict__ AinvU,
                                                      const double* __restrict__ Cinv, const double* __restrict__ w_in,
                                                      double eta, double tol, int it, int max_iter,
                                                      int32_t* __restrict__ seg_done, int32_t* __restrict__ seg_iters,
                                                      double* __restrict__ seg_rel, double* __restrict__ seg_d0,
                                                      double* __restrict__ seg_best, int32_t* __restrict__ seg_stall,
                                                      int32_t* __restrict__ ndone, int32_t* __restrict__ diverged,
                                                      IterState* __restrict__ st) {
  extern __shared__ double sm[];
  __shared__ double red[8];
  __shared__ double vv[64];
  __shared__ double uu[64];
  // every row done (one workgroup per row) or a row diverged: nothing to update
  if (*ndone >= (int)gridDim.x || *diverged) return;
  const int i = blockIdx.x;
  if (seg_done[i]) return;
  const int Rr = tg.Rr, Rn = tg.Rn;
  const double w = *w_in;
  double* z = sm;
  double* h = sm + Rr;
  double* buf = sm + 2 * Rr;
  for (int e = threadIdx.x; e < Rr; e += blockDim.x) z[e] = Z[(size_t)i * Rr + e];
  __syncthreads();
  // vv[a] = sum_c V[a][c] v[c] by 16 lanes per output a: lane p sums the terms
  // c = p, p + 16, ... and a butterfly over the 16 lanes adds the partial sums
  // (fixed order; the 16 lanes of a group always run the same a)
  auto v_times = [&](const double* v) {
    const int p = threadIdx.x & 15;
    for (int a = threadIdx.x >> 4; a < Rn; a += blockDim.x >> 4) {
      double s = 0.0;
      for (int c = p; c < Rr; c += 16) s = fma(Vw[a * Rr + c], v[c], s);
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      if (p == 0) vv[a] = s;
    }
    __syncthreads();
  };
  v_times(z);
  // h = Q1 + w z + G^+ vv   (G^+ = GtP^T)
  for (int e = threadIdx.x; e < Rr; e += blockDim.x) {
    double s = Q1[(size_t)i * Rr + e] + w * z[e];
    for (int a = 0; a < Rn; ++a) s = fma(GtP[a * Rr + e], vv[a], s);
    h[e] = s;
  }
  __syncthreads();
  wg_apply_Ainv(g, T, w, h, buf);          // h <- A^-1 h
  v_times(h);
  for (int a = threadIdx.x; a < Rn; a += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < Rn; ++b) s = fma(Cinv[a * Rn + b], vv[b], s);
    uu[a] = s;
  }
  __syncthreads();
  double dd = 0.0, zz = 0.0;
  for (int e = threadIdx.x; e < Rr; e += blockDim.x) {
    double d = h[e];
    for (int a = 0; a < Rn; ++a) d = fma(-AinvU[e * Rn + a], uu[a], d);
    const double zn = fma(-eta, d, z[e]);
    Z[(size_t)i * Rr + e] = zn;
    dd = fma(d, d, dd);
    zz = fma(zn, zn, zz);
  }
  dd = block_sum(dd, red);
  zz = block_sum(zz, red);
  if (threadIdx.x == 0)
    tucker_row_stop(i, dd, zz, eta, tol, it, seg_done, seg_iters, seg_rel, seg_d0, seg_best, seg_stall, ndone, diverged);
}

// The stopping rule of row i from the squared norms of its step d and new z.
__device__ void tucker_row_stop(int i, double dd, double zz, double eta, double tol, int it,
                                int32_t* __restrict__ seg_done, int32_t* __restrict__ seg_iters,
                                double* __restrict__ seg_rel, double* __restrict__ seg_d0,
                                double* __restrict__ seg_best, int32_t* __restrict__ seg_stall,
                                int32_t* __restrict__ ndone, int32_t* __restrict__ diverged) {
  {
    const double dn = sqrt(dd), zn = sqrt(zz);
    const double rel = zn > 0.0 ? eta * dn / zn : (dn > 0.0 ? INFINITY : 0.0);
    // stagnation: the terms w z and w G^+ G z of h cancel at O(w ||z||), so the
    // relative step has a rounding floor near tol; a row whose step has not
    // halved in 4 iterations while below 1e3 tol sits on that floor and stops
    if (it == 0) {
      seg_d0[i] = dn;
      seg_best[i] = rel;
      seg_stall[i] = 0;
    } else if (rel < 0.5 * seg_best[i]) {
      seg_best[i] = rel;
      seg_stall[i] = 0;
    } else {
      seg_stall[i] += 1;
    }
    const bool stalled = seg_stall[i] >= 4 && rel <= 1e3 * tol;
    const bool bad = !isfinite(dn) || !isfinite(zn) || (it > 0 && dn > 1e6 * seg_d0[i] && dn > 0.0);
    seg_rel[i] = rel;
    if (bad) atomicOr(diverged, 1);
    if (rel <= tol || bad || stalled) {
      seg_done[i] = 1;
      seg_iters[i] = it + 1;
      atomicAdd(ndone, 1);
    }
  }
}

// The same per-row update with every row-independent operand requested once, up
// front, for rows of Rr <= 256 entries (one per thread) and R_n <= 16: thread e
// holds column e of GtP and row e of AinvU, the 16-lane group a holds row a of
// Vw (lane p its entries p, p + 16, ...), and the tree modes' eigenvectors and
// Cinv are staged in LDS.  The original reads those operands from global memory
// inside each step, a chain of about ten dependent round trips per iteration;
// here the steps wait only on LDS and barriers.  The arithmetic and its order are
// those of k_tucker_update (the same results, bit for bit).  Dynamic LDS: 3 Rr
// doubles for z, h and scratch, then sum_k R_k^2 + R_n^2 for the staged matrices.
#define TU_RN 16
__global__ void __launch_bounds__(256) k_tucker_update_st(ModeTables T, Geom g, TuckerGeom tg,
                                                         const double* __restrict__ Q1, double* __restrict__ Z,
                                                         const double* __restrict__ GtP, const double* __restrict__ Vw,
                                                         const double* __restrict__ AinvU,
                                                         const double* __restrict__ Cinv, const double* __restrict__ w_in,
                                                         double eta, double tol, int it, int max_iter,
                                                         int32_t* __restrict__ seg_done, int32_t* __restrict__ seg_iters,
                                                         double* __restrict__ seg_rel, double* __restrict__ seg_d0,
                                                         double* __restrict__ seg_best, int32_t* __restrict__ seg_stall,
                                                         int32_t* __restrict__ ndone, int32_t* __restrict__ diverged,
                                                         IterState* __restrict__ st) {
  extern __shared__ double sm[];
  __shared__ double red[8];
  __shared__ double vv[64];
  __shared__ double uu[64];
  // every row done (one workgroup per row) or a row diverged: nothing to update
  if (*ndone >= (int)gridDim.x || *diverged) return;
  const int i = blockIdx.x;
  if (seg_done[i]) return;
  const int Rr = tg.Rr, Rn = tg.Rn;
  const int e = threadIdx.x;
  const bool own = e < Rr;
  double* z = sm;
  double* h = sm + Rr;
  double* buf = sm + 2 * Rr;
  double* Vs = sm + 3 * Rr;
  int voff[KR_MAXN];
  int nv = 0;
  for (int k = 1; k < g.N; ++k) {
    voff[k] = nv;
    nv += g.R[k] * g.R[k];
  }
  double* Cs = Vs + nv;
  // every operand requested before the first use
  for (int k = 1; k < g.N; ++k)
    for (int t = threadIdx.x; t < g.R[k] * g.R[k]; t += blockDim.x) Vs[voff[k] + t] = T.V[k][t];
  for (int t = threadIdx.x; t < Rn * Rn; t += blockDim.x) Cs[t] = Cinv[t];
  const double w = *w_in;
  const double zq = own ? Z[(size_t)i * Rr + e] : 0.0;
  const double q1 = own ? Q1[(size_t)i * Rr + e] : 0.0;
  double gt[TU_RN], au[TU_RN], vw[TU_RN];
#pragma unroll
  for (int a = 0; a < TU_RN; ++a) {
    gt[a] = own && a < Rn ? GtP[a * Rr + e] : 0.0;
    au[a] = own && a < Rn ? AinvU[e * Rn + a] : 0.0;
  }
  const int ga = threadIdx.x >> 4, gp = threadIdx.x & 15;
#pragma unroll
  for (int j = 0; j < TU_RN; ++j) {
    const int c = gp + 16 * j;
    vw[j] = ga < Rn && c < Rr ? Vw[ga * Rr + c] : 0.0;
  }
  // the diagonal of A for entry e (the eigenvalue products plus w)
  double den = 1.0;
  if (own) {
    int r = e;
    double prod = 1.0;
    for (int k = g.N - 1; k >= 1; --k) {
      const int rk = r % g.R[k];
      r /= g.R[k];
      prod *= T.evals[k][rk];
    }
    den = prod + w;
  }
  if (own) z[e] = zq;
  __syncthreads();
  // vv[a] = sum_c V[a][c] v[c]: group a, lane p sums c = p, p + 16, ..., then a
  // butterfly over the group's 16 lanes
  auto v_times = [&](const double* v) {
    if (ga < Rn) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < TU_RN; ++j) {
        const int c = gp + 16 * j;
        if (c < Rr) s = fma(vw[j], v[c], s);
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) s += __shfl_xor(s, o, 16);
      if (gp == 0) vv[ga] = s;
    }
    __syncthreads();
  };
  v_times(z);
  if (own) {
    double sh = q1 + w * zq;
#pragma unroll
    for (int a = 0; a < TU_RN; ++a)
      if (a < Rn) sh = fma(gt[a], vv[a], sh);
    h[e] = sh;
  }
  __syncthreads();
  // h <- A^-1 h: the mode products with V_k^T, the diagonal, the products with V_k
  double* cur = h;
  double* nxt = buf;
  for (int pass = 0; pass < 2; ++pass) {
    for (int k = 1; k < g.N; ++k) {
      const int Rk = g.R[k];
      const int post = (int)g.rsuf[k + 1];
      const double* V = Vs + voff[k];
      if (own) {
        const int blk = e / (Rk * post), rem = e - blk * Rk * post, a = rem / post, c = rem - a * post;
        const double* src = cur + blk * Rk * post + c;
        double acc = 0.0;
        for (int b = 0; b < Rk; ++b) acc = fma(pass == 0 ? V[b * Rk + a] : V[a * Rk + b], src[b * post], acc);
        nxt[e] = acc;
      }
      __syncthreads();
      double* t = cur;
      cur = nxt;
      nxt = t;
    }
    if (pass == 0) {
      if (own) cur[e] /= den;
      __syncthreads();
    }
  }
  const double he = own ? cur[e] : 0.0;
  v_times(cur);
  for (int a = threadIdx.x; a < Rn; a += blockDim.x) {
    double sa = 0.0;
    for (int b = 0; b < Rn; ++b) sa = fma(Cs[a * Rn + b], vv[b], sa);
    uu[a] = sa;
  }
  __syncthreads();
  double dd = 0.0, zz = 0.0;
  if (own) {
    double d = he;
#pragma unroll
    for (int a = 0; a < TU_RN; ++a)
      if (a < Rn) d = fma(-au[a], uu[a], d);
    const double zn = fma(-eta, d, zq);
    Z[(size_t)i * Rr + e] = zn;
    dd = d * d;
    zz = zn * zn;
  }
  dd = block_sum(dd, red);
  zz = block_sum(zz, red);
  if (threadIdx.x == 0)
    tucker_row_stop(i, dd, zz, eta, tol, it, seg_done, seg_iters, seg_rel, seg_d0, seg_best, seg_stall, ndone, diverged);
}

// A_out[i][r] = sum_c GtP[r][c] z_i[c]
__global__ void __launch_bounds__(256) k_tucker_rows_out(TuckerGeom tg, const double* __restrict__ Z,
                                                        const double* __restrict__ GtP, int nrows,
                                                        double* __restrict__ Aout) {
  const int Rn = tg.Rn, Rr = tg.Rr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)nrows * Rn;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / Rn;
    const int r = (int)(e - i * Rn);
    double s = 0.0;
    for (int c = 0; c < Rr; ++c) s = fma(GtP[r * Rr + c], Z[i * Rr + c], s);
    Aout[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Exact factor update of Algorithm 1 (the ALS baseline the paper compares
// with): every row i of factor n solves (G_(n) K^T K G_(n)^T + lambda I) y =
// G_(n) K^T X_(n)[i]^T with K^T K = kron_{m != n} A_m^T A_m.  K^T X_(n)^T is the
// tensor-times-matrix chain T = X x_{m != n} A_m^T (mode products, the first one
// reading X in its own dtype); the right-hand sides and the R_n x R_n matrix are
// contractions of T and of core x_{m != n} (A_m^T A_m) with the core over every
// mode but n.
// ---------------------------------------------------------------------------

// out[pre][o][post] = sum_{i < Rin} A[i][o] in[pre][i][post] for a float32 input
// (the first mode product of the chain; A is Rin x Rout row-major).
__global__ void __launch_bounds__(256) k_ttm_f32(const float* __restrict__ in, double* __restrict__ out,
                                                int64_t pre, int Rin, int Rout, int64_t post,
                                                const double* __restrict__ A) {
  const int64_t total = pre * Rout * post;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ((int64_t)Rout * post);
    const int64_t rem = e - b * Rout * post;
    const int o = (int)(rem / post);
    const int64_t c = rem - (int64_t)o * post;
    const float* src = in + b * Rin * post + c;
    double acc = 0.0;
    for (int r = 0; r < Rin; ++r) acc = fma(A[(int64_t)r * Rout + o], (double)src[(int64_t)r * post], acc);
    out[e] = acc;
  }
}

// out[i][r] = sum_{a < pre, c < post} T[a][i][c] G[a][r][c]: T has In entries on
// the contracted-out mode, G (the core) Rn; every other mode has the core's size.
__global__ void __launch_bounds__(256) k_contract_all_but(const double* __restrict__ T, const double* __restrict__ G,
                                                         int64_t pre, int In, int Rn, int64_t post,
                                                         double* __restrict__ out) {
  const int64_t total = (int64_t)In * Rn;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / Rn;
    const int r = (int)(e - i * Rn);
    double acc = 0.0;
    for (int64_t a = 0; a < pre; ++a) {
      const double* t = T + (a * In + i) * post;
      const double* gg = G + (a * Rn + r) * post;
      for (int64_t c = 0; c < post; ++c) acc = fma(t[c], gg[c], acc);
    }
    out[e] = acc;
  }
}

// Rows of the new factor: y_i = (H + lambda I)^{-1} P[i] by the Cholesky factor of
// H + lambda I, formed in LDS by every workgroup (R_n <= 64); a non-positive
// pivot raises KR_FLAG_CORE.
__global__ void __launch_bounds__(256) k_factor_solve(const double* __restrict__ H, double lambda,
                                                     const double* __restrict__ P, int In, int Rn,
                                                     double* __restrict__ out, int32_t* __restrict__ flags) {
  __shared__ double L[64 * 64];
  __shared__ int bad;
  for (int e = threadIdx.x; e < Rn * Rn; e += blockDim.x) {
    const int p = e / Rn, q = e - p * Rn;
    L[e] = H[e] + (p == q ? lambda : 0.0);
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 0; j < Rn; ++j) {
      double d = L[j * Rn + j];
      for (int k = 0; k < j; ++k) d -= L[j * Rn + k] * L[j * Rn + k];
      if (!(d > 0.0)) { bad = 1; d = 1.0; }
      const double l = sqrt(d);
      L[j * Rn + j] = l;
      for (int i = j + 1; i < Rn; ++i) {
        double v = L[i * Rn + j];
        for (int k = 0; k < j; ++k) v -= L[i * Rn + k] * L[j * Rn + k];
        L[i * Rn + j] = v / l;
      }
    }
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicOr(flags, KR_FLAG_CORE);
    return;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < In; i += (int64_t)gridDim.x * blockDim.x) {
    double y[64];
    const double* b = P + i * Rn;
    for (int r = 0; r < Rn; ++r) {      // L z = b
      double v = b[r];
      for (int k = 0; k < r; ++k) v -= L[r * Rn + k] * y[k];
      y[r] = v / L[r * Rn + r];
    }
    for (int r = Rn - 1; r >= 0; --r) { // L^T y = z
      double v = y[r];
      for (int k = r + 1; k < Rn; ++k) v -= L[k * Rn + r] * y[k];
      y[r] = v / L[r * Rn + r];
    }
    for (int r = 0; r < Rn; ++r) out[i * Rn + r] = y[r];
  }
}

}  // namespace kr
