// One preconditioned Richardson step of Algorithm 2 on the merged sketch:
//     x <- x - (1 - sqrt(eps)) M^+ (K~^T Omega (K~ x - b~) + lambda x).
//
// The sampled products follow the idea of Theorem kron_mat_mul_sqrt_decomp
// (contract with the factors only over the distinct prefixes present in the
// sample), applied at every prefix length instead of one split:
//   forward  P_0 = x;  P_k[s] = P_{k-1}[parent(s)] x_k a_{k-1}[i_{k-1}(s)]
//            (level-k node s, k = 1..N-1), u_j = <a_{N-1}[i(j)], P_{N-1}[parent(j)]> - b_j
//   adjoint  Q_{N-1}[p] = sum_{j child of p} Omega_j u_j a_{N-1}[i(j)]
//            Q_{k-1}[p] = sum_{s child of p} a_{k-1}[i(s)] (outer) Q_k[s],  g = Q_0
// so level k costs |level-k nodes| * R_{k-1} * R_k..R_{N-1} multiply-adds instead of
// m * R for the naive per-sample product.  The preconditioner M^+ =
// (kron V) D (kron V)^T (Algorithm 2, with D = (kron Lambda + lambda)^+) is applied by
// mode products (the square Kronecker mat-vec theorem); for lambda = 0 it is
// kron G_n^{-1}.  Every output is computed by one thread with a fixed
// summation order, so results are deterministic.
//
// All intermediates are stored node-major with the right-hand side innermost:
// P_k[s][c][q], c < rsuf[k], q < nrhs.
#include "kr_internal.h"

namespace kr {

__global__ void __launch_bounds__(256) k_fwd_level(ModeTables T, Geom g, Tree tr, int k,
                                                  const double* __restrict__ Pprev,
                                                  double* __restrict__ Pout,
                                                  const IterState* __restrict__ st) {
  if (st->all_done) return;
  const int64_t S = tr.cnt[k];
  const int64_t W = g.rsuf[k] * g.nrhs;         // entries per level-k node
  const int64_t Wp = g.rsuf[k - 1] * g.nrhs;    // entries per parent
  const int Rk = g.R[k - 1];
  const double* __restrict__ A = T.A[k - 1];
  const int64_t total = S * W;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / W, cq = e - s * W;
    const int p = k == 1 ? 0 : tr.parent[k][s];
    const double* a = A + (int64_t)tr.idx[k][s] * Rk;
    const double* src = Pprev + (int64_t)p * Wp + cq;
    double acc = 0.0;
    for (int r = 0; r < Rk; ++r) acc = fma(a[r], src[(int64_t)r * W], acc);
    Pout[e] = acc;
  }
}

// Rows and the last adjoint level, fused.  A group of G lanes (power of two
// >= R_{N-1}) owns one (level-(N-1) node p, rhs q); lane r keeps P[p][r][q] and
// accumulates Q[p][r][q] over the children rows of p.
template <int G>
__global__ void __launch_bounds__(256) k_rows_adj(ModeTables T, Geom g, Tree tr,
                                                 const double* __restrict__ Pprev,
                                                 const double* __restrict__ Omega,
                                                 const double* __restrict__ bD,
                                                 double* __restrict__ Qout,
                                                 const IterState* __restrict__ st) {
  if (st->all_done) return;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  const double* __restrict__ A = T.A[N - 1];
  const int64_t Sp = tr.cnt[N - 1];
  const int lane = threadIdx.x & (G - 1);
  const int64_t ngroups_total = Sp * nrhs;
  const int64_t gpb = blockDim.x / G;
  for (int64_t grp = blockIdx.x * gpb + threadIdx.x / G; grp - (threadIdx.x / G) < ngroups_total;
       grp += (int64_t)gridDim.x * gpb) {
    const bool active = grp < ngroups_total;
    const int64_t p = active ? grp / nrhs : 0;
    const int q = active ? (int)(grp - p * nrhs) : 0;
    const double pv = (active && lane < R) ? Pprev[(p * R + lane) * nrhs + q] : 0.0;
    double acc = 0.0;
    const int j0 = active ? tr.fchild[N - 1][p] : 0;
    const int j1 = active ? tr.fchild[N - 1][p + 1] : 0;
    for (int j = j0; j < j1; ++j) {
      const double a = lane < R ? A[(int64_t)tr.idx[N][j] * R + lane] : 0.0;
      double y = a * pv;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, G);
      const double w = Omega[j] * (y - bD[(int64_t)j * nrhs + q]);
      acc = fma(w, a, acc);
    }
    if (active && lane < R) Qout[(p * R + lane) * nrhs + q] = acc;
  }
}

// Adjoint level k (k = N-1 .. 1): Q_{k-1}[p][r][c][q] = sum_s a_{k-1}[i(s)][r] Q_k[s][c][q].
__global__ void __launch_bounds__(256) k_adj_level(ModeTables T, Geom g, Tree tr, int k,
                                                  const double* __restrict__ Qk,
                                                  double* __restrict__ Qout,
                                                  const IterState* __restrict__ st) {
  if (st->all_done) return;
  const int64_t Sp = tr.cnt[k - 1];
  const int64_t W = g.rsuf[k] * g.nrhs;
  const int64_t Wp = g.rsuf[k - 1] * g.nrhs;
  const int Rk = g.R[k - 1];
  const double* __restrict__ A = T.A[k - 1];
  const int64_t total = Sp * Wp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = e / Wp, rem = e - p * Wp;
    const int r = (int)(rem / W);
    const int64_t cq = rem - (int64_t)r * W;
    const int s0 = tr.fchild[k - 1][p], s1 = tr.fchild[k - 1][p + 1];
    double acc = 0.0;
    for (int s = s0; s < s1; ++s)
      acc = fma(A[(int64_t)tr.idx[k][s] * Rk + r], Qk[(int64_t)s * W + cq], acc);
    Qout[e] = acc;
  }
}

// Mode product inside one workgroup: out = in x_n M, M is R_n x R_n (M[a][b]),
// transposed when trans != 0.  Tensor layout [R_0..R_{N-1}][nrhs].
__device__ void wg_mode_product(const Geom& g, int n, const double* __restrict__ M, int trans,
                                const double* in, double* out) {
  const int Rn = g.R[n];
  const int64_t post = g.rsuf[n + 1] * g.nrhs;
  const int64_t total = g.Rtot * g.nrhs;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t blk = e / (Rn * post);
    const int64_t rem = e - blk * Rn * post;
    const int a = (int)(rem / post);
    const int64_t c = rem - (int64_t)a * post;
    const double* src = in + blk * Rn * post + c;
    double acc = 0.0;
    for (int b = 0; b < Rn; ++b) {
      const double mab = trans ? M[b * Rn + a] : M[a * Rn + b];
      acc = fma(mab, src[(int64_t)b * post], acc);
    }
    out[e] = acc;
  }
}

// d = M^+ (g + lambda x); x <- x - eta d for right-hand sides not yet converged;
// per-RHS norms, stopping rule eta ||d|| <= tol ||x||, divergence test.
// One workgroup of 1024 threads.  t0/t1 are Rtot x nrhs scratch buffers.
__global__ void __launch_bounds__(1024) k_precond_update(ModeTables T, Geom g, const double* __restrict__ grad,
                                                        double* __restrict__ x, double* __restrict__ t0,
                                                        double* __restrict__ t1, double lambda, double eta,
                                                        double tol, int max_iter, int use_ginv,
                                                        IterState* __restrict__ st) {
  __shared__ double red[16];
  if (st->all_done) return;
  const int64_t total = g.Rtot * g.nrhs;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) t0[e] = grad[e] + lambda * x[e];
  __syncthreads();
  double* cur = t0;
  double* nxt = t1;
  if (use_ginv) {
    for (int n = 0; n < g.N; ++n) {
      wg_mode_product(g, n, T.Ginv[n], 0, cur, nxt);
      __syncthreads();
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
  } else {
    for (int n = 0; n < g.N; ++n) {
      wg_mode_product(g, n, T.V[n], 1, cur, nxt);
      __syncthreads();
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      int64_t r = e / g.nrhs;
      double prod = 1.0;
      for (int n = g.N - 1; n >= 0; --n) {
        const int rn = (int)(r % g.R[n]);
        r /= g.R[n];
        prod *= T.evals[n][rn];
      }
      const double den = prod + lambda;
      cur[e] = den > 0.0 ? cur[e] / den : 0.0;
    }
    __syncthreads();
    for (int n = 0; n < g.N; ++n) {
      wg_mode_product(g, n, T.V[n], 0, cur, nxt);
      __syncthreads();
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
  }
  // cur = d.  Update and norms per right-hand side.
  const int it = st->iters;
  int all = 1, div = 0;
  for (int q = 0; q < g.nrhs; ++q) {
    const int done = st->done[q];
    double dd = 0.0, xx = 0.0;
    for (int64_t r = threadIdx.x; r < g.Rtot; r += blockDim.x) {
      const int64_t e = r * g.nrhs + q;
      const double d = cur[e];
      double xv = x[e];
      if (!done) { xv = fma(-eta, d, xv); x[e] = xv; }
      dd = fma(d, d, dd);
      xx = fma(xv, xv, xx);
    }
    dd = block_sum(dd, red);
    xx = block_sum(xx, red);
    if (threadIdx.x == 0 && !done) {
      const double dn = sqrt(dd), xn = sqrt(xx);
      const double rel = xn > 0.0 ? eta * dn / xn : (dn > 0.0 ? INFINITY : 0.0);
      st->rel[q] = rel;
      if (it == 0) st->dnorm0[q] = dn;
      const bool bad = !isfinite(dn) || !isfinite(xn) || (it > 0 && dn > 1e6 * st->dnorm0[q] && dn > 0.0);
      if (bad) { div = 1; }
      if (rel <= tol || bad) { st->done[q] = 1; st->it_rhs[q] = it + 1; }
    }
    if (threadIdx.x == 0) all &= st->done[q];
  }
  if (threadIdx.x == 0) {
    st->iters = it + 1;
    if (div) st->diverged = 1;
    if (all || div || it + 1 >= max_iter) st->all_done = 1;
  }
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_zero_bytes(uint32_t* __restrict__ p, int64_t nwords) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template __global__ void k_rows_adj<8>(ModeTables, Geom, Tree, const double*, const double*, const double*,
                                       double*, const IterState*);
template __global__ void k_rows_adj<16>(ModeTables, Geom, Tree, const double*, const double*, const double*,
                                        double*, const IterState*);
template __global__ void k_rows_adj<32>(ModeTables, Geom, Tree, const double*, const double*, const double*,
                                        double*, const IterState*);
template __global__ void k_rows_adj<64>(ModeTables, Geom, Tree, const double*, const double*, const double*,
                                        double*, const IterState*);

}  // namespace kr
