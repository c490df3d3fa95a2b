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

// sum_{r < n} a[r] src[r * step] in increasing r, with the loads of 16 terms issued
// together (a serial load-FMA chain is latency-bound).
__device__ __forceinline__ double dot_batched(const double* __restrict__ a, const double* __restrict__ src,
                                              int64_t step, int n) {
  double acc = 0.0;
  for (int r0 = 0; r0 < n; r0 += 16) {
    double av[16], sv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      av[u] = r0 + u < n ? a[r0 + u] : 0.0;
      sv[u] = r0 + u < n ? src[(int64_t)(r0 + u) * step] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (r0 + u < n) acc = fma(av[u], sv[u], acc);
  }
  return acc;
}

// base[byte offset]: a 32-bit offset from a (wave-uniform) base pointer.
__device__ __forceinline__ double ld_at(const double* __restrict__ base, unsigned off) {
  return *(const double*)((const char*)base + off);
}

// Lane exchanges of float64 values inside a wave, without LDS address registers:
// DPP moves within a row of 16 lanes, swizzles within 32, a permute across 32.
template <int CTRL> __device__ __forceinline__ double dpp64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
template <int PAT> __device__ __forceinline__ double swz64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(uint32_t)b, PAT);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), PAT);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// the value of lane (lane ^ O)
template <int O> __device__ __forceinline__ double xor_lane(double v) {
  if constexpr (O == 1) return dpp64<0xB1>(v);        // quad_perm [1,0,3,2]
  else if constexpr (O == 2) return dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  else if constexpr (O == 8) return dpp64<0x128>(v);  // row_ror:8
  else if constexpr (O == 32) return __shfl_xor(v, 32, 64);
  else return swz64<0x1F | (O << 10)>(v);             // bit-mode swizzle, xor mask O
}
// Sum over each aligned group of G lanes; every lane of a group ends with the same
// bits (each step adds a pair in either order, and addition commutes).
template <int G> __device__ __forceinline__ double grp_sum(double v) {
  if constexpr (G > 1) v += xor_lane<1>(v);
  if constexpr (G > 2) v += xor_lane<2>(v);
  if constexpr (G > 4) v += dpp64<0x141>(v);  // row_half_mirror: the other quad of 8 lanes
  if constexpr (G > 8) v += xor_lane<8>(v);
  if constexpr (G > 16) v += xor_lane<16>(v);
  if constexpr (G > 32) v += xor_lane<32>(v);
  return v;
}
// Sum of lane l's value over the 64 / G groups (lanes l ^ G k), in the order G, 2G, ...
template <int G> __device__ __forceinline__ double xgrp_sum(double v) {
  static_assert(G >= 4 && G <= 64, "group width");
  if constexpr (G <= 4) v += xor_lane<4>(v);
  if constexpr (G <= 8) v += xor_lane<8>(v);
  if constexpr (G <= 16) v += xor_lane<16>(v);
  if constexpr (G <= 32) v += xor_lane<32>(v);
  return v;
}

// The level kernels do not test for convergence: the host stops launching them,
// and the few passes launched after the last iteration only rewrite scratch
// levels (the preconditioner kernel leaves x unchanged then).  Level counts come
// from tr.ncnt (host copies), so no dependent load precedes the work.
//
// Forward level k (always float64: the residual K~x - b~ cancels, so it is formed
// in float64 in every precision mode).
__global__ void __launch_bounds__(256) k_fwd_level(ModeTables TT, Geom g, Tree tr, int k,
                                                  const double* __restrict__ Pprev,
                                                  double* __restrict__ Pout,
                                                  const IterState* __restrict__ st) {
  const unsigned S = (unsigned)tr.ncnt[k];
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
    Pout[e] = dot_batched(arow + (size_t)s * Rk, Pprev + (size_t)p * Wp + cq, W, Rk);
  }
}

// The last forward level, the rows and the last adjoint level, fused.  One wave
// owns one (level-(N-1) node p, rhs q).  Its NGR = 64/G lane groups (G a power of
// two >= R_{N-1}) first form P_{N-1}[p][r][q] in lane r: from P_{N-2}[parent(p)]
// and the gathered factor row a_{N-2}[i(p)] (P_0 = x with the root as parent;
// for N = 1 it is x itself; for a segment root it is the segment's own iterate).
// Group gi then takes rows j0 + gi, j0 + gi + NGR, ... of p, KR_ROWS_PER_STEP per
// step (the first step's requested before the node's forward value):
// u_j = <a_{N-1}[i(j)], P_{N-1}[p]> - b_j in float64 and Q[p][r][q] +=
// (Omega_j u_j) a_{N-1}[i(j)][r] in T; the groups' sums are added in a fixed order.
// Measured: the wave-uniform task with scalar row bases, DPP group sums and one
// register set (92 VGPRs, 5 waves per SIMD) beat a prefetching second set; the
// compiler waits for all loads at the loop head either way.
#ifndef KR_ROWS_PER_STEP
#define KR_ROWS_PER_STEP 4
#endif
template <int G, typename T>
__global__ void __launch_bounds__(256) k_rows_adj(ModeTables TT, Geom g, Tree tr,
                                                 const double* __restrict__ Pprev,
                                                 const double* __restrict__ Omega,
                                                 const double* __restrict__ bD,
                                                 T* __restrict__ Qout,
                                                 const IterState* __restrict__ st) {
  constexpr int NGR = 64 / G;
  constexpr int RPS = KR_ROWS_PER_STEP;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  const double* __restrict__ AL = tr.arow[N];
  const int64_t ntask = tr.ncnt[N - 1] * nrhs;
  const int lane = threadIdx.x & (G - 1);
  const int gi = (threadIdx.x & 63) / G;
  const bool ln = lane < R;
  const int64_t wpb = blockDim.x >> 6;
  // the task index is wave-uniform, so the node's bounds and row bases live in
  // scalar registers and every lane addresses its rows by a small 32-bit offset
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int64_t task = blockIdx.x * wpb + w; task < ntask; task += (int64_t)gridDim.x * wpb) {
    const int64_t p = task / nrhs;
    const int q = (int)(task - p * nrhs);
    const int j0 = tr.fchild[N - 1][p], j1 = tr.fchild[N - 1][p + 1];
    const double* __restrict__ ab = AL + (int64_t)j0 * R;
    const double* __restrict__ ob = Omega + j0;
    const double* __restrict__ bp = bD + (int64_t)j0 * nrhs + q;
    // Steps of RPS NGR rows; group gi takes rows gi + NGR u (u < RPS) of a step,
    // all requested at once.  The loads are unconditional: an absent row re-reads
    // the step's first row and gets weight 0 where it is used, and lanes r >= R
    // re-read entry R - 1, which meets P_{N-1} = 0 there.  32-bit offsets from
    // the scalar bases.
    const int nrow = j1 - j0;
    if (nrow <= 0) {  // a node always has rows; kept for safety (uniform branch)
      if (gi == 0 && ln) Qout[(p * R + lane) * nrhs + q] = (T)0;
      continue;
    }
    const unsigned lc = ln ? lane : R - 1;
    auto load_step = [&](double (&av)[RPS], double (&om)[RPS], double (&bb)[RPS], int k) {
      const int nl = nrow - k * RPS * NGR;
      const double* __restrict__ abk = ab + (int64_t)k * RPS * NGR * R;
      const double* __restrict__ obk = ob + k * RPS * NGR;
      const double* __restrict__ bpk = bp + (int64_t)k * RPS * NGR * nrhs;
#pragma unroll
      for (int u = 0; u < RPS; ++u) {
        const int jl = gi + u * NGR;
        const unsigned jc = jl < nl ? (unsigned)jl : 0u;
        av[u] = ld_at(abk, (jc * (unsigned)R + lc) * 8u);
        om[u] = ld_at(obk, jc * 8u);
        bb[u] = ld_at(bpk, jc * (unsigned)nrhs * 8u);
      }
    };
    double aA[RPS], oA[RPS], bA[RPS];
    // the first step's rows are requested before the forward value of the node,
    // so that both memory round trips overlap
    load_step(aA, oA, bA, 0);
    // P_{N-1}[p][lane][q]; from a parent level, group gi sums the terms
    // s = gi, gi + NGR, ... of the contraction over R_{N-2} and the groups' partial
    // sums are combined by a butterfly (the same rounding in every group)
    double pv = 0.0;
    if (N == 1) {
      if (ln) pv = Pprev[(int64_t)lane * nrhs + q];
    } else if (N == 2 && g.seg_root) {
      if (ln) pv = Pprev[((int64_t)tr.idx[1][p] * R + lane) * nrhs + q];
    } else {
      const int Rp = g.R[N - 2];
      const int64_t par = N >= 3 ? tr.parent[N - 1][p] : 0;
      const double* __restrict__ a = tr.arow[N - 1] + p * Rp;
      const int64_t step = (int64_t)R * nrhs;
      const double* __restrict__ src = Pprev + par * (int64_t)Rp * step + q;
      if (ln) {
        for (int s0 = gi; s0 < Rp; s0 += 4 * NGR) {
          double as[4], sv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * NGR;
            as[u] = s < Rp ? a[s] : 0.0;
            sv[u] = s < Rp ? src[(int64_t)s * step + lane * nrhs] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) pv = fma(as[u], sv[u], pv);
        }
      }
      pv = xgrp_sum<G>(pv);
    }
    T acc = 0;
    auto step = [&](const double (&av)[RPS], const double (&om)[RPS], const double (&bb)[RPS], int k) {
      const int nl = nrow - k * RPS * NGR;
      double y[RPS];
#pragma unroll
      for (int u = 0; u < RPS; ++u) y[u] = grp_sum<G>(av[u] * pv);
#pragma unroll
      for (int u = 0; u < RPS; ++u) {
        const double w = gi + u * NGR < nl ? om[u] : 0.0;
        acc = fma((T)(w * (y[u] - bb[u])), (T)av[u], acc);
      }
    };
    const int nstep = (nrow + RPS * NGR - 1) / (RPS * NGR);
    for (int k = 0;;) {
      step(aA, oA, bA, k);
      if (++k >= nstep) break;
      load_step(aA, oA, bA, k);
    }
    // sum over the groups of the wave (fixed pairing order)
#pragma unroll
    for (int o = G; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (gi == 0 && ln) Qout[(p * R + lane) * nrhs + q] = acc;
  }
}

// Adjoint of one block of nodes: out[r][e0 + c] = sum_{s in [s0, s1)} a[s][r] q[s][e0 + c]
// for r < Rk and the column block c < CE of the W columns.  Output (r, c) belongs to
// threads (r, c) + 256 k of a workgroup of 256 k threads; up to ADJ_CHUNK nodes' factor rows and q columns (at most ADJ_QS entries
// each) are staged in LDS at a time and added in increasing node order.  Used for the
// adjoint levels (the children of one parent) and the root adjoint (a block of
// level-1 nodes).
#define RA_NODES 32
#define ADJ_CHUNK 128
#define ADJ_QS 2048
#define ADJ_THREADS 1024
template <typename T>
__device__ void adj_block(const T* __restrict__ arow, int Rk, const T* __restrict__ q, unsigned W, unsigned s0,
                          unsigned s1, unsigned e0, unsigned CE, T* __restrict__ out, T* as, T* qs, T* red) {
  constexpr int NPF = ADJ_QS / ADJ_THREADS;   // staged entries per thread
  const unsigned r0 = (threadIdx.x & 255) / CE, c = (threadIdx.x & 255) - r0 * CE;
  const bool mine = r0 < (unsigned)Rk && e0 + c < W;
  const unsigned chunk = min((unsigned)ADJ_CHUNK, min((unsigned)ADJ_QS / CE, (unsigned)ADJ_QS / (unsigned)Rk));
  // a chunk's staged entries fit in NPF per thread; the next chunk's loads are
  // issued before the current chunk is summed
  T va[NPF], vq[NPF];
  auto load = [&](unsigned b0) {
    const unsigned ns = min(chunk, s1 - b0);
    const unsigned na = ns * (unsigned)Rk, nq = ns * CE;
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const unsigned i = threadIdx.x + u * ADJ_THREADS;
      va[u] = i < na ? arow[(size_t)b0 * Rk + i] : T(0);
      const unsigned sn = i / CE, cc = i - sn * CE;
      vq[u] = (i < nq && e0 + cc < W) ? q[(size_t)(b0 + sn) * W + e0 + cc] : T(0);
    }
  };
  auto store = [&](unsigned b0) {
    const unsigned ns = min(chunk, s1 - b0);
    const unsigned na = ns * (unsigned)Rk, nq = ns * CE;
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const unsigned i = threadIdx.x + u * ADJ_THREADS;
      if (i < na) as[i] = va[u];
      if (i < nq) qs[i] = vq[u];
    }
  };
  // ADJ_THREADS / 256 threads share an output: part p sums nodes p, p + nparts,
  // ... of every chunk, four at a time, and the parts are added in order at the end
  const unsigned nparts = ADJ_THREADS >> 8, part = threadIdx.x >> 8;
  T acc = 0;
  __syncthreads();
  if (s0 < s1) {
    load(s0);
    store(s0);
  }
  __syncthreads();
  for (unsigned b0 = s0; b0 < s1; b0 += chunk) {
    const unsigned ns = min(chunk, s1 - b0);
    const bool more = b0 + chunk < s1;
    if (more) load(b0 + chunk);
    if (mine) {
      unsigned sn = part;
      for (; sn + 3 * nparts < ns; sn += 4 * nparts) {
        T av[4], qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = as[(sn + u * nparts) * Rk + r0];
          qv[u] = qs[(sn + u * nparts) * CE + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
      }
      for (; sn < ns; sn += nparts) acc = fma(as[sn * Rk + r0], qs[sn * CE + c], acc);
    }
    __syncthreads();
    if (more) store(b0 + chunk);
    __syncthreads();
  }
  if (nparts > 1) {
    red[threadIdx.x] = acc;
    __syncthreads();
    if (part == 0) {
      for (unsigned k = 1; k < nparts; ++k) acc += red[threadIdx.x + 256 * k];
    }
    __syncthreads();
  }
  if (mine && part == 0) out[(size_t)r0 * W + e0 + c] = acc;
}

__host__ __device__ __forceinline__ unsigned adj_cols(int Rk) { return Rk >= 256 ? 1u : 256u / (unsigned)Rk; }

// Adjoint level k (k = N-1 .. 2): Q_{k-1}[p][r][c] = sum_{s child of p} a_{k-1}[i(s)][r]
// Q_k[s][c] (c < rsuf[k] nrhs).  One task per (parent, column block).
template <typename T>
__global__ void __launch_bounds__(ADJ_THREADS) k_adj_level(ModeTables TT, Geom g, Tree tr, int k,
                                                  const T* __restrict__ Qk,
                                                  T* __restrict__ Qout,
                                                  const IterState* __restrict__ st) {
  __shared__ T as[ADJ_QS];
  __shared__ T qs[ADJ_QS];
  __shared__ T red[ADJ_THREADS];
  const unsigned Sp = (unsigned)tr.ncnt[k - 1];
  const int Rk = g.R[k - 1];
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs);
  const unsigned CE = adj_cols(Rk);
  const unsigned ncb = (W + CE - 1) / CE;
  const T* __restrict__ arow = node_rows<T>(tr, k);
  for (unsigned task = blockIdx.x; task < Sp * ncb; task += gridDim.x) {
    const unsigned p = task / ncb, cb = task - p * ncb;
    adj_block(arow, Rk, Qk, W, (unsigned)tr.fchild[k - 1][p], (unsigned)tr.fchild[k - 1][p + 1], cb * CE, CE,
              Qout + (size_t)p * Rk * W, as, qs, red);
  }
}

// Root adjoint, split over blocks of npb level-1 nodes (npb a multiple of
// RA_NODES): partial[b][r0][c] = sum_{s in block b} a_0[i(s)][r0] Q_1[s][c].
template <typename T>
__global__ void __launch_bounds__(ADJ_THREADS) k_adj_root_partial(Geom g, Tree tr, const T* __restrict__ Q1,
                                                         T* __restrict__ partial, int npb,
                                                         const IterState* __restrict__ st) {
  __shared__ T as[ADJ_QS];
  __shared__ T qs[ADJ_QS];
  __shared__ T red[ADJ_THREADS];
  const unsigned S1 = (unsigned)tr.ncnt[1];
  const int R0 = g.R[0];
  const unsigned W1 = (unsigned)(g.rsuf[1] * g.nrhs);
  const unsigned CE = adj_cols(R0);
  const unsigned ncb = (W1 + CE - 1) / CE;
  const unsigned nnb = (S1 + npb - 1) / npb;
  for (unsigned task = blockIdx.x; task < ncb * nnb; task += gridDim.x) {
    const unsigned cb = task % ncb, nbk = task / ncb;
    const unsigned b0 = nbk * (unsigned)npb;
    adj_block(node_rows<T>(tr, 1), R0, Q1, W1, b0, min(S1, b0 + (unsigned)npb), cb * CE, CE,
              partial + (size_t)nbk * g.Rtot * g.nrhs, as, qs, red);
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
