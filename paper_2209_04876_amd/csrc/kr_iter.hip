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

// (q, r) = divmod(e, W) for a grid-stride loop without dividing inside the loop.
struct GDiv {
  unsigned q, r, dq, dr, W;
  __device__ __forceinline__ GDiv(unsigned e0, unsigned W_, unsigned step) : W(W_) {
    q = e0 / W; r = e0 - q * W; dq = step / W; dr = step - dq * W;
  }
  __device__ __forceinline__ void next() {
    q += dq; r += dr;
    if (r >= W) { r -= W; ++q; }
  }
};

// Gathered factor rows of level k in the arithmetic type of the products.
template <typename T> __device__ __forceinline__ const T* node_rows(const Tree& tr, int k);
template <> __device__ __forceinline__ const double* node_rows<double>(const Tree& tr, int k) { return tr.arow[k]; }
template <> __device__ __forceinline__ const float* node_rows<float>(const Tree& tr, int k) { return tr.arow32[k]; }

// Forward level k (always float64: the residual K~x - b~ cancels, so it is formed
// in float64 in every precision mode).
__global__ void __launch_bounds__(256) k_fwd_level(ModeTables TT, Geom g, Tree tr, int k,
                                                  const double* __restrict__ Pprev,
                                                  double* __restrict__ Pout,
                                                  const IterState* __restrict__ st) {
  if (st->all_done) return;
  const unsigned S = (unsigned)tr.cnt[k];
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs);         // entries per level-k node
  const unsigned Wp = (unsigned)(g.rsuf[k - 1] * g.nrhs);    // entries per parent
  const int Rk = g.R[k - 1];
  const double* __restrict__ arow = tr.arow[k];
  const unsigned total = S * W;
  const unsigned step = gridDim.x * blockDim.x;
  const unsigned e0 = blockIdx.x * blockDim.x + threadIdx.x;
  GDiv di(e0, W, step);
  if (k == 1 && g.seg_root) {
    // segment roots: copy the segment's own iterate (Pprev is segments x W)
    for (unsigned e = e0; e < total; e += step, di.next())
      Pout[e] = Pprev[(size_t)tr.idx[1][di.q] * W + di.r];
    return;
  }
  for (unsigned e = e0; e < total; e += step, di.next()) {
    const unsigned s = di.q, cq = di.r;
    const unsigned p = k == 1 ? 0u : (unsigned)tr.parent[k][s];
    const double* a = arow + (size_t)s * Rk;
    const double* src = Pprev + (size_t)p * Wp + cq;
    double acc = 0.0;
#pragma unroll 4
    for (int r = 0; r < Rk; ++r) acc = fma(a[r], src[r * W], acc);
    Pout[e] = acc;
  }
}

// Rows and the last adjoint level, fused.  A group of G lanes (power of two
// >= R_{N-1}) owns one (level-(N-1) node p, rhs q); lane r keeps P[p][r][q] and
// accumulates Q[p][r][q] over the children rows of p, four rows per step.  The
// row dot product and the residual u_j = <a, P> - b_j are float64; the weighted
// residual Omega_j u_j is then accumulated in T (float64, or float32 in the
// refined modes).
template <int G, typename T>
__global__ void __launch_bounds__(256) k_rows_adj(ModeTables TT, Geom g, Tree tr,
                                                 const double* __restrict__ Pprev,
                                                 const double* __restrict__ Omega,
                                                 const double* __restrict__ bD,
                                                 T* __restrict__ Qout,
                                                 const IterState* __restrict__ st) {
  if (st->all_done) return;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  const double* __restrict__ AL = tr.arow[N];
  const int64_t Sp = tr.cnt[N - 1];
  const int lane = threadIdx.x & (G - 1);
  const int64_t ngroups_total = Sp * nrhs;
  const int64_t gpb = blockDim.x / G;
  for (int64_t grp = blockIdx.x * gpb + threadIdx.x / G; grp - (threadIdx.x / G) < ngroups_total;
       grp += (int64_t)gridDim.x * gpb) {
    const bool active = grp < ngroups_total;
    const int64_t p = active ? grp / nrhs : 0;
    const int q = active ? (int)(grp - p * nrhs) : 0;
    const bool ln = active && lane < R;
    const double pv = ln ? Pprev[(p * R + lane) * nrhs + q] : 0.0;
    T acc = 0;
    const int j0 = active ? tr.fchild[N - 1][p] : 0;
    const int j1 = active ? tr.fchild[N - 1][p + 1] : 0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      double av[4], y[4], om[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = ln ? AL[(int64_t)(j + u) * R + lane] : 0.0;
        om[u] = Omega[j + u];
        bb[u] = bD[(int64_t)(j + u) * nrhs + q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = av[u] * pv;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] += __shfl_xor(y[u], o, G);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma((T)(om[u] * (y[u] - bb[u])), (T)av[u], acc);
    }
    for (; j < j1; ++j) {
      const double a = ln ? AL[(int64_t)j * R + lane] : 0.0;
      double y = a * pv;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) y += __shfl_xor(y, o, G);
      acc = fma((T)(Omega[j] * (y - bD[(int64_t)j * nrhs + q])), (T)a, acc);
    }
    if (ln) Qout[(p * R + lane) * nrhs + q] = acc;
  }
}

// Adjoint level k (k = N-1 .. 2): Q_{k-1}[p][r][c][q] = sum_s a_{k-1}[i(s)][r] Q_k[s][c][q].
template <typename T>
__global__ void __launch_bounds__(256) k_adj_level(ModeTables TT, Geom g, Tree tr, int k,
                                                  const T* __restrict__ Qk,
                                                  T* __restrict__ Qout,
                                                  const IterState* __restrict__ st) {
  if (st->all_done) return;
  const unsigned Sp = (unsigned)tr.cnt[k - 1];
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs);
  const unsigned Wp = (unsigned)(g.rsuf[k - 1] * g.nrhs);
  const int Rk = g.R[k - 1];
  const T* __restrict__ arow = node_rows<T>(tr, k);
  const unsigned total = Sp * Wp;
  const unsigned step = gridDim.x * blockDim.x;
  const unsigned e0 = blockIdx.x * blockDim.x + threadIdx.x;
  GDiv di(e0, Wp, step);
  for (unsigned e = e0; e < total; e += step, di.next()) {
    const unsigned p = di.q, rem = di.r;
    const unsigned r = rem / W, cq = rem - r * W;
    const int s0 = tr.fchild[k - 1][p], s1 = tr.fchild[k - 1][p + 1];
    T acc = 0;
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
      T av[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = arow[(size_t)(s + u) * Rk + r];
        qv[u] = Qk[(size_t)(s + u) * W + cq];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
    }
    for (; s < s1; ++s) acc = fma(arow[(size_t)s * Rk + r], Qk[(size_t)s * W + cq], acc);
    Qout[e] = acc;
  }
}

// Root adjoint, split over blocks of level-1 nodes: partial[b][r0][c] =
// sum_{s in block b} a_0[i(s)][r0] Q_1[s][c].  Workgroup (column block, node block)
// stages its node block's factor rows and Q_1 columns in LDS.
#define RA_NODES 32
template <typename T>
__global__ void __launch_bounds__(256) k_adj_root_partial(Geom g, Tree tr, const T* __restrict__ Q1,
                                                         T* __restrict__ partial,
                                                         const IterState* __restrict__ st) {
  if (st->all_done) return;
  __shared__ T as[RA_NODES * 64];
  __shared__ T qs[RA_NODES * 256];
  const T* __restrict__ arow1 = node_rows<T>(tr, 1);
  const unsigned S1 = (unsigned)tr.cnt[1];
  const int R0 = g.R[0];
  const unsigned W1 = (unsigned)(g.rsuf[1] * g.nrhs);
  const unsigned CE = R0 >= 256 ? 1u : 256u / (unsigned)R0;
  const unsigned ncb = (W1 + CE - 1) / CE;
  const unsigned nnb = (S1 + RA_NODES - 1) / RA_NODES;
  for (unsigned task = blockIdx.x; task < ncb * nnb; task += gridDim.x) {
    const unsigned cb = task % ncb, nbk = task / ncb;
    const unsigned e0 = cb * CE, s0 = nbk * RA_NODES;
    const unsigned ns = (S1 - s0) < RA_NODES ? (S1 - s0) : RA_NODES;
    for (unsigned i = threadIdx.x; i < ns * (unsigned)R0; i += blockDim.x) as[i] = arow1[(size_t)s0 * R0 + i];
    for (unsigned i = threadIdx.x; i < ns * CE; i += blockDim.x) {
      const unsigned sn = i / CE, c = i - sn * CE;
      qs[i] = e0 + c < W1 ? Q1[(size_t)(s0 + sn) * W1 + e0 + c] : T(0);
    }
    __syncthreads();
    const unsigned r0 = threadIdx.x / CE, c = threadIdx.x - r0 * CE;
    if (r0 < (unsigned)R0 && e0 + c < W1) {
      T acc = 0;
      for (unsigned sn = 0; sn < ns; ++sn) acc = fma(as[sn * R0 + r0], qs[sn * CE + c], acc);
      partial[(size_t)nbk * g.Rtot * g.nrhs + (size_t)r0 * W1 + e0 + c] = acc;
    }
    __syncthreads();
  }
}

// g = sum over node blocks of the partials, in block order (deterministic).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_root_sum(Geom g, Tree tr, const T* __restrict__ partial,
                                                     T* __restrict__ grad, const IterState* __restrict__ st) {
  if (st->all_done) return;
  const unsigned S1 = (unsigned)tr.cnt[1];
  const unsigned nnb = (S1 + RA_NODES - 1) / RA_NODES;
  const size_t RT = (size_t)g.Rtot * g.nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < RT; e += (size_t)gridDim.x * blockDim.x) {
    T acc = 0;
    for (unsigned b = 0; b < nnb; ++b) acc += partial[(size_t)b * RT + e];
    grad[e] = acc;
  }
}

// Mode product inside one workgroup: out = in x_n M, M is R_n x R_n (M[a][b]),
// transposed when trans != 0.  Tensor layout [R_0..R_{N-1}][nrhs].  Each thread
// owns whole mode-n fibres: it reads the fibre once into registers and forms all
// R_n outputs.
template <int RM>
__device__ void wg_mode_fibre(const Geom& g, int n, const double* __restrict__ M, int trans,
                              const double* in, double* out) {
  const int Rn = g.R[n];
  const unsigned post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
  const unsigned nfib = (unsigned)(g.Rtot * g.nrhs) / (unsigned)Rn;
  GDiv di(threadIdx.x, post, blockDim.x);
  for (unsigned f = threadIdx.x; f < nfib; f += blockDim.x, di.next()) {
    const size_t base = (size_t)di.q * Rn * post + di.r;
    double v[RM];
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = b < Rn ? in[base + (size_t)b * post] : 0.0;
    for (int a = 0; a < Rn; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < Rn) acc = fma(trans ? M[b * Rn + a] : M[a * Rn + b], v[b], acc);
      out[base + (size_t)a * post] = acc;
    }
  }
}

// d = M^+ (g + lambda x); x <- x - eta d for right-hand sides not yet converged;
// per-RHS norms, stopping rule eta ||d|| <= tol ||x||, divergence test.
// One workgroup of 256 threads.  t0/t1 are Rtot x nrhs scratch buffers; each
// factor matrix is staged in LDS before its mode product.  RM (8, 16, 32 or 64)
// bounds every R_n: one fibre width per kernel keeps the fibre in registers.
template <int RM>
__global__ void __launch_bounds__(256) k_precond_update(ModeTables T, Geom g, const double* __restrict__ grad,
                                                        double* __restrict__ x, double* __restrict__ t0,
                                                        double* __restrict__ t1, double lambda, double eta,
                                                        double tol, int max_iter, int use_ginv,
                                                        IterState* __restrict__ st) {
  __shared__ double red[16];
  __shared__ double ms[64 * 64];
  if (st->all_done) return;
  const int64_t total = g.Rtot * g.nrhs;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) t0[e] = grad[e] + lambda * x[e];
  double* cur = t0;
  double* nxt = t1;
  auto stage = [&](const double* M, int n) {
    __syncthreads();
    for (int e = threadIdx.x; e < g.R[n] * g.R[n]; e += blockDim.x) ms[e] = M[e];
    __syncthreads();
  };
  if (use_ginv) {
    for (int n = 0; n < g.N; ++n) {
      stage(T.Ginv[n], n);
      wg_mode_fibre<RM>(g, n, ms, 0, cur, nxt);
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
  } else {
    for (int n = 0; n < g.N; ++n) {
      stage(T.V[n], n);
      wg_mode_fibre<RM>(g, n, ms, 1, cur, nxt);
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
    __syncthreads();
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
    for (int n = 0; n < g.N; ++n) {
      stage(T.V[n], n);
      wg_mode_fibre<RM>(g, n, ms, 0, cur, nxt);
      double* tmp = cur; cur = nxt; nxt = tmp;
    }
  }
  __syncthreads();
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

}  // namespace kr
