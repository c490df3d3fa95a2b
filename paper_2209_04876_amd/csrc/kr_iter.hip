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
// accumulates Q[p][r][q] over the children rows of p, eight rows per step (their
// loads issued together).  The
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
    for (; j + 8 <= j1; j += 8) {
      double av[8], y[8], om[8], bb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        av[u] = ln ? AL[(int64_t)(j + u) * R + lane] : 0.0;
        om[u] = Omega[j + u];
        bb[u] = bD[(int64_t)(j + u) * nrhs + q];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = av[u] * pv;
#pragma unroll
      for (int o = G / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int u = 0; u < 8; ++u) y[u] += __shfl_xor(y[u], o, G);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = fma((T)(om[u] * (y[u] - bb[u])), (T)av[u], acc);
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

// Adjoint of one block of nodes: out[r][e0 + c] = sum_{s in [s0, s1)} a[s][r] q[s][e0 + c]
// for r < Rk and the column block c < CE of the W columns.  Thread (r, c) keeps one
// sum; up to RA_NODES nodes' factor rows and q columns (at most ADJ_QS entries)
// are staged in LDS at a time and added in increasing node order.  Used for the
// adjoint levels (the children of one parent) and the root adjoint (a block of
// level-1 nodes).
#define RA_NODES 32
#define ADJ_QS 2048
template <typename T>
__device__ void adj_block(const T* __restrict__ arow, int Rk, const T* __restrict__ q, unsigned W, unsigned s0,
                          unsigned s1, unsigned e0, unsigned CE, T* __restrict__ out, T* as, T* qs) {
  const unsigned r0 = threadIdx.x / CE, c = threadIdx.x - r0 * CE;
  const bool mine = r0 < (unsigned)Rk && e0 + c < W;
  const unsigned chunk = min((unsigned)RA_NODES, (unsigned)ADJ_QS / CE);
  T acc = 0;
  for (unsigned b0 = s0; b0 < s1; b0 += chunk) {
    const unsigned ns = min(chunk, s1 - b0);
    __syncthreads();
    for (unsigned i = threadIdx.x; i < ns * (unsigned)Rk; i += blockDim.x) as[i] = arow[(size_t)b0 * Rk + i];
    for (unsigned i = threadIdx.x; i < ns * CE; i += blockDim.x) {
      const unsigned sn = i / CE, cc = i - sn * CE;
      qs[i] = e0 + cc < W ? q[(size_t)(b0 + sn) * W + e0 + cc] : T(0);
    }
    __syncthreads();
    if (mine)
      for (unsigned sn = 0; sn < ns; ++sn) acc = fma(as[sn * Rk + r0], qs[sn * CE + c], acc);
  }
  if (mine) out[(size_t)r0 * W + e0 + c] = acc;
}

__host__ __device__ __forceinline__ unsigned adj_cols(int Rk) { return Rk >= 256 ? 1u : 256u / (unsigned)Rk; }

// Adjoint level k (k = N-1 .. 2): Q_{k-1}[p][r][c] = sum_{s child of p} a_{k-1}[i(s)][r]
// Q_k[s][c] (c < rsuf[k] nrhs).  One task per (parent, column block).
template <typename T>
__global__ void __launch_bounds__(256) k_adj_level(ModeTables TT, Geom g, Tree tr, int k,
                                                  const T* __restrict__ Qk,
                                                  T* __restrict__ Qout,
                                                  const IterState* __restrict__ st) {
  if (st->all_done) return;
  __shared__ T as[RA_NODES * 64];
  __shared__ T qs[ADJ_QS];
  const unsigned Sp = (unsigned)tr.cnt[k - 1];
  const int Rk = g.R[k - 1];
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs);
  const unsigned CE = adj_cols(Rk);
  const unsigned ncb = (W + CE - 1) / CE;
  const T* __restrict__ arow = node_rows<T>(tr, k);
  for (unsigned task = blockIdx.x; task < Sp * ncb; task += gridDim.x) {
    const unsigned p = task / ncb, cb = task - p * ncb;
    adj_block(arow, Rk, Qk, W, (unsigned)tr.fchild[k - 1][p], (unsigned)tr.fchild[k - 1][p + 1], cb * CE, CE,
              Qout + (size_t)p * Rk * W, as, qs);
  }
}

// Root adjoint, split over blocks of npb level-1 nodes (npb a multiple of
// RA_NODES): partial[b][r0][c] = sum_{s in block b} a_0[i(s)][r0] Q_1[s][c].
template <typename T>
__global__ void __launch_bounds__(256) k_adj_root_partial(Geom g, Tree tr, const T* __restrict__ Q1,
                                                         T* __restrict__ partial, int npb,
                                                         const IterState* __restrict__ st) {
  if (st->all_done) return;
  __shared__ T as[RA_NODES * 64];
  __shared__ T qs[ADJ_QS];
  const unsigned S1 = (unsigned)tr.cnt[1];
  const int R0 = g.R[0];
  const unsigned W1 = (unsigned)(g.rsuf[1] * g.nrhs);
  const unsigned CE = adj_cols(R0);
  const unsigned ncb = (W1 + CE - 1) / CE;
  const unsigned nnb = (S1 + npb - 1) / npb;
  for (unsigned task = blockIdx.x; task < ncb * nnb; task += gridDim.x) {
    const unsigned cb = task % ncb, nbk = task / ncb;
    const unsigned b0 = nbk * (unsigned)npb;
    adj_block(node_rows<T>(tr, 1), R0, Q1, W1, b0, min(S1, b0 + (unsigned)npb), cb * CE, CE,
              partial + (size_t)nbk * g.Rtot * g.nrhs, as, qs);
  }
}

// Partial blocks of the root adjoint: ceil(S_1 / npb); npb = 0 means the
// gradient was written directly (one block).
__device__ __forceinline__ unsigned root_blocks(const int64_t* __restrict__ cnt, int npb) {
  return npb > 0 ? (unsigned)((cnt[1] + npb - 1) / npb) : 1u;
}

// g = sum over the partial blocks in block order (deterministic).  Each thread
// issues the loads of up to 16 blocks at once before adding them in order.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_root_sum(Geom g, Tree tr, const T* __restrict__ partial, int npb,
                                                     T* __restrict__ grad, const IterState* __restrict__ st) {
  if (st->all_done) return;
  const unsigned nnb = root_blocks(tr.cnt, npb);
  const size_t RT = (size_t)g.Rtot * g.nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < RT; e += (size_t)gridDim.x * blockDim.x) {
    T acc = 0;
    for (unsigned b0 = 0; b0 < nnb; b0 += 16) {
      T v[16];
#pragma unroll
      for (unsigned u = 0; u < 16; ++u) v[u] = b0 + u < nnb ? partial[(size_t)(b0 + u) * RT + e] : T(0);
#pragma unroll
      for (unsigned u = 0; u < 16; ++u)
        if (b0 + u < nnb) acc += v[u];
    }
    grad[e] = acc;
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
