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

#ifndef KR_ROWS_PER_STEP
#define KR_ROWS_PER_STEP 4
#endif

// The rows of one (level-(N-1) node, rhs) task, owned by one wave whose lane
// group gi takes rows gi + NGR u (u < RPS) of each step of RPS NGR rows, all
// requested at once.  The loads are unconditional: an absent row re-reads the
// step's first row and gets weight 0 where it is used, and lanes r >= R re-read
// entry R - 1, which meets P_{N-1} = 0 there.  Rows are addressed by 32-bit
// offsets from wave-uniform (scalar) bases.  load(0) is issued before the node's
// forward value is formed, so that both memory round trips overlap; run(pv)
// then returns the wave's sum of (Omega_j u_j) a_{N-1}[i(j)][lane] over the node's
// rows, u_j = <a_{N-1}[i(j)], P_{N-1}> - b_j formed in float64.
// LDSF: the last mode's factor is staged in LDS (AL points there) and each row
// streams its 4-byte index i(j) instead of its materialised factor row; the row
// is then read from LDS.
template <int G, int RPS, bool LDSF = false>
struct RowsTask {
  static constexpr int NGR = 64 / G;
  const double* __restrict__ ab;
  const int32_t* __restrict__ ib;
  const double* __restrict__ ob;
  const double* __restrict__ bp;
  int nrow, R, nrhs, gi;
  unsigned lc;
  double aA[RPS], oA[RPS], bA[RPS];
  int iA[RPS];
  __device__ __forceinline__ RowsTask(const double* AL, const int32_t* idxL, const double* Omega, const double* bD,
                                      int j0, int j1, int R_, int nrhs_, int q, int lane, int gi_)
      : ab(LDSF ? AL : AL + (int64_t)j0 * R_), ib(LDSF ? idxL + j0 : nullptr), ob(Omega + j0),
        bp(bD + (int64_t)j0 * nrhs_ + q), nrow(j1 - j0), R(R_), nrhs(nrhs_), gi(gi_),
        lc(lane < R_ ? (unsigned)lane : (unsigned)(R_ - 1)) {}
  __device__ __forceinline__ void load(int k) {
    const int nl = nrow - k * RPS * NGR;
    const double* __restrict__ abk = ab + (int64_t)k * RPS * NGR * R;
    const double* __restrict__ obk = ob + k * RPS * NGR;
    const double* __restrict__ bpk = bp + (int64_t)k * RPS * NGR * nrhs;
#pragma unroll
    for (int u = 0; u < RPS; ++u) {
      const int jl = gi + u * NGR;
      const unsigned jc = jl < nl ? (unsigned)jl : 0u;
      if constexpr (LDSF)
        iA[u] = ib[k * RPS * NGR + jc];
      else
        aA[u] = ld_at(abk, (jc * (unsigned)R + lc) * 8u);
      oA[u] = ld_at(obk, jc * 8u);
      bA[u] = ld_at(bpk, jc * (unsigned)nrhs * 8u);
    }
  }
  template <typename T>
  __device__ __forceinline__ T run(double pv) {
    T acc = 0;
    const int nstep = (nrow + RPS * NGR - 1) / (RPS * NGR);
    for (int k = 0;;) {
      const int nl = nrow - k * RPS * NGR;
      if constexpr (LDSF) {
#pragma unroll
        for (int u = 0; u < RPS; ++u) aA[u] = ab[(unsigned)iA[u] * (unsigned)R + lc];
      }
      double y[RPS];
#pragma unroll
      for (int u = 0; u < RPS; ++u) y[u] = grp_sum<G>(aA[u] * pv);
#pragma unroll
      for (int u = 0; u < RPS; ++u) {
        const double w = gi + u * NGR < nl ? oA[u] : 0.0;
        acc = fma((T)(w * (y[u] - bA[u])), (T)aA[u], acc);
      }
      if (++k >= nstep) break;
      load(k);
    }
    // sum over the groups of the wave (fixed pairing order)
#pragma unroll
    for (int o = G; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
  }
};

// P_{N-1}[p][lane][q] of a (level-(N-1) node p, rhs q) task in lane `lane` of
// every group of G lanes (0 in lanes lane >= R_{N-1}).  From a parent level, group
// gi sums the terms s = gi, gi + NGR, ... of the contraction over R_{N-2} and the
// groups' partial sums are combined by a butterfly (the same rounding in every
// group); P_0 = x with the root as parent; for N = 1 it is x itself; for a
// segment root it is the segment's own iterate.
template <int G>
__device__ __forceinline__ double rows_pnode(const Geom& g, const Tree& tr, const double* __restrict__ Pprev,
                                             int64_t p, int64_t par, int q, int lane, int gi) {
  constexpr int NGR = 64 / G;
  const int N = g.N, nrhs = g.nrhs, R = g.R[N - 1];
  const bool ln = lane < R;
  double pv = 0.0;
  if (N == 1) {
    if (ln) pv = Pprev[(int64_t)lane * nrhs + q];
  } else if (N == 2 && g.seg_root) {
    if (ln) pv = Pprev[((int64_t)tr.idx[1][p] * R + lane) * nrhs + q];
  } else {
    // 32-bit byte offsets from the wave-uniform bases of a_{N-2}[i(p)] and
    // P_{N-2}[parent(p)][:, :, q]
    const int Rp = g.R[N - 2];
    const double* __restrict__ a = tr.arow[N - 1] + p * Rp;
    const unsigned step8 = (unsigned)(R * nrhs) * 8u;
    const double* __restrict__ src = Pprev + par * (int64_t)Rp * R * nrhs + q;
    const unsigned lo8 = (unsigned)(lane * nrhs) * 8u;
    if (ln) {
      if (Rp == 4 * NGR) {   // one term per lane group and step: no bounds to test
        double as[4], sv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned s = (unsigned)(gi + u * NGR);
          as[u] = ld_at(a, s * 8u);
          sv[u] = ld_at(src, s * step8 + lo8);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pv = fma(as[u], sv[u], pv);
      } else {
        for (int s0 = gi; s0 < Rp; s0 += 4 * NGR) {
          double as[4], sv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int s = s0 + u * NGR;
            as[u] = s < Rp ? ld_at(a, (unsigned)s * 8u) : 0.0;
            sv[u] = s < Rp ? ld_at(src, (unsigned)s * step8 + lo8) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) pv = fma(as[u], sv[u], pv);
        }
      }
    }
    pv = xgrp_sum<G>(pv);
  }
  return pv;
}

// The last forward level, the rows and the last adjoint level, fused.  One wave
// owns one (level-(N-1) node p, rhs q).  Its NGR = 64/G lane groups (G a power of
// two >= R_{N-1}) first form P_{N-1}[p][r][q] in lane r: from P_{N-2}[parent(p)]
// and the gathered factor row a_{N-2}[i(p)] (P_0 = x with the root as parent;
// for N = 1 it is x itself; for a segment root it is the segment's own iterate).
// The rows then follow as in RowsTask: Q[p][r][q] = sum_j (Omega_j u_j)
// a_{N-1}[i(j)][r] in T, the groups' sums added in a fixed order.
// Measured: the wave-uniform task with scalar row bases, DPP group sums and one
// register set (92 VGPRs, 5 waves per SIMD) beat a prefetching second set; the
// compiler waits for all loads at the loop head either way.
// The LDS-staged variant runs KR_ROWS_LDS_TPB threads per workgroup with at least
// KR_ROWS_LDS_WPE waves per SIMD, so that more waves share each staged copy of the
// factor (the kernel is bound by the latency of its dependent row loads).
// Measured on the Tucker factor updates (ms per 400^3 sweep): materialised rows
// 46.4; staged, 256 threads 45.0; 512 threads at 5 waves per SIMD 39.6; 1024
// threads 39.8; 512 threads at 6 waves per SIMD 53.2 (80 VGPRs, spills); with
// the next task's bounds requested one task ahead (114 VGPRs, 4 waves per SIMD,
// two 512-thread workgroups per CU) 36.2.
#ifndef KR_ROWS_LDS_TPB
#define KR_ROWS_LDS_TPB 512
#endif
#ifndef KR_ROWS_LDS_WPE
#define KR_ROWS_LDS_WPE 4
#endif
template <int G, typename T, bool LDSF>
__global__ void __launch_bounds__(LDSF ? KR_ROWS_LDS_TPB : 256)
    __attribute__((amdgpu_waves_per_eu(LDSF ? KR_ROWS_LDS_WPE : 1, 8))) k_rows_adj(ModeTables TT, Geom g, Tree tr,
                                                 const double* __restrict__ Pprev,
                                                 const double* __restrict__ Omega,
                                                 const double* __restrict__ bD,
                                                 T* __restrict__ Qout,
                                                 const IterState* __restrict__ st) {
  extern __shared__ double rows_fac[];
  constexpr int NGR = 64 / G;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  const double* __restrict__ AL = LDSF ? (const double*)rows_fac : tr.arow[N];
  if constexpr (LDSF) {
    // the last mode's whole factor (I_{N-1} x R_{N-1}), once per workgroup
    const int nf = g.I[N - 1] * R;
    const double* __restrict__ A = TT.A[N - 1];
    for (int e = threadIdx.x; e < nf; e += blockDim.x) rows_fac[e] = A[e];
    __syncthreads();
  }
  const int64_t ntask = tr.ncnt[N - 1] * nrhs;
  const int lane = threadIdx.x & (G - 1);
  const int gi = (threadIdx.x & 63) / G;
  const bool ln = lane < R;
  const int64_t wpb = blockDim.x >> 6;
  // the task index is wave-uniform, so the node's bounds and row bases live in
  // scalar registers
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tstride = (int64_t)gridDim.x * wpb;
  // a node's row bounds and parent are requested one task ahead, so that they
  // are in registers when the task starts (one dependent round trip fewer)
  int nb0 = 0, nb1 = 0;
  int64_t npar = 0;
  auto fetch = [&](int64_t t) {
    if (t < ntask) {
      const int64_t pp = t / nrhs;
      nb0 = tr.fchild[N - 1][pp];
      nb1 = tr.fchild[N - 1][pp + 1];
      npar = N >= 3 ? tr.parent[N - 1][pp] : 0;
    }
  };
  fetch(blockIdx.x * wpb + w);
  for (int64_t task = blockIdx.x * wpb + w; task < ntask; task += tstride) {
    const int64_t p = task / nrhs;
    const int q = (int)(task - p * nrhs);
    const int j0 = nb0, j1 = nb1;
    const int64_t par = npar;
    fetch(task + tstride);
    if (j1 <= j0) {  // a node always has rows; kept for safety (uniform branch)
      if (gi == 0 && ln) Qout[(p * R + lane) * nrhs + q] = (T)0;
      continue;
    }
    RowsTask<G, KR_ROWS_PER_STEP, LDSF> rt(AL, tr.idx[N], Omega, bD, j0, j1, R, nrhs, q, lane, gi);
    rt.load(0);
    const double pv = rows_pnode<G>(g, tr, Pprev, p, par, q, lane, gi);
    const T acc = rt.template run<T>(pv);
    if (gi == 0 && ln) Qout[(p * R + lane) * nrhs + q] = acc;
  }
}

// Lane exchange (lane ^ O) of a float64 or float32 value.
template <int O, typename T> __device__ __forceinline__ T xlane(T v) {
  if constexpr (sizeof(T) == 8) return xor_lane<O>(v);
  else return __shfl_xor(v, O, 64);
}
// The permlane swaps of gfx950 (per 32-bit half): permlane32_swap exchanges x in
// lanes 32..63 with y in lanes 0..31, permlane16_swap x in the odd 16-lane rows
// with y in the even rows below them.
template <bool P32> __device__ __forceinline__ void swap_u32(uint32_t& x, uint32_t& y) {
  if constexpr (P32) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}
template <bool P32, typename T> __device__ __forceinline__ void swap_lanes(T& x, T& y) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
    uint32_t xl = (uint32_t)bx, yl = (uint32_t)by, xh = (uint32_t)(bx >> 32), yh = (uint32_t)(by >> 32);
    swap_u32<P32>(xl, yl);
    swap_u32<P32>(xh, yh);
    x = __builtin_bit_cast(T, ((uint64_t)xh << 32) | xl);
    y = __builtin_bit_cast(T, ((uint64_t)yh << 32) | yl);
  } else {
    uint32_t ux = __builtin_bit_cast(uint32_t, x), uy = __builtin_bit_cast(uint32_t, y);
    swap_u32<P32>(ux, uy);
    x = __builtin_bit_cast(T, ux);
    y = __builtin_bit_cast(T, uy);
  }
}
// DPP row rotate by 8 of a 32- or 64-bit value, written only to the lanes of the
// banks (4-lane quarters of each 16-lane row) in BANKS; the others keep `old`.
template <int BANKS, typename T> __device__ __forceinline__ T ror8_into(T old, T v) {
  if constexpr (sizeof(T) == 8) {
    const uint64_t bo = __builtin_bit_cast(uint64_t, old), bv = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)bo, (int)(uint32_t)bv, 0x128, 0xF, BANKS, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(bo >> 32), (int)(uint32_t)(bv >> 32), 0x128, 0xF, BANKS,
                                               false);
    return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                             0x128, 0xF, BANKS, false));
  }
}
// One halving step of the transpose sum over the lane pairs (l, l ^ MASK): the
// lane with bit MASK clear ends with entries 0..H-1 of the pair's sum, the other
// with entries H..2H-1, both in acc[0..H-1].  Each entry is one addition of the
// pair's two values.
template <int H, int MASK, typename T> __device__ __forceinline__ void tsum_step(T* acc, bool up) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T x = acc[i], y = acc[H + i];
    if constexpr (MASK == 32 || MASK == 16) {
      // after the swap the low lane holds (its x, the partner's x), the high lane
      // (the partner's y, its y)
      swap_lanes<MASK == 32>(x, y);
      acc[i] = x + y;
    } else if constexpr (MASK == 8) {
      acc[i] = ror8_into<0x3>(y, x) + ror8_into<0xC>(x, y);
    } else {
      const T keep = up ? y : x;
      const T give = up ? x : y;
      acc[i] = keep + xlane<MASK>(give);
    }
  }
}
// Sum over the 64 lanes of each of the RP entries acc[0..RP-1]: entry r ends in
// lanes r (64 / RP) .. r (64 / RP) + 64 / RP - 1 (all with the same bits).  Every
// lane pair adds its two values once, so the result does not depend on timing.
template <int RP, typename T> __device__ __forceinline__ T lane_transpose_sum(T (&acc)[RP], int l64) {
  static_assert(RP == 8 || RP == 16, "padded row width");
  tsum_step<RP / 2, 32>(acc, (l64 & 32) != 0);
  tsum_step<RP / 4, 16>(acc, (l64 & 16) != 0);
  tsum_step<RP / 8, 8>(acc, (l64 & 8) != 0);
  if constexpr (RP == 16) tsum_step<1, 4>(acc, (l64 & 4) != 0);
  T v = acc[0];
  if constexpr (RP == 8) v += xlane<4>(v);
  v += xlane<2>(v);
  v += xlane<1>(v);
  return v;
}
__device__ __forceinline__ double read_lane(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The LDS-staged rows with one row per lane, for R_{N-1} <= RP (8 or 16).  The
// same sums as k_rows_adj: one wave per (level-(N-1) node p, rhs q) task, Q[p][r][q]
// = sum_j (Omega_j u_j) a_{N-1}[i(j)][r] with u_j = <a_{N-1}[i(j)], P_{N-1}> - b_j
// in float64.  The rows of a task are taken 64 at a time, lane l owning row
// j0 + 64 c + l: its index, Omega and b arrive in one coalesced request per 64
// rows (the next 64 requested before the current ones are used, the first before
// the node's forward value is formed), its factor row is read from LDS (the
// factor staged zero-padded to RP columns), and P_{N-1} is held wave-uniform, so
// a lane forms u_j alone and accumulates its RP adjoint terms in registers.  A
// transpose sum across the lanes ends the task.  Against the group-per-row
// kernel a task of up to 64 rows costs one memory round trip instead of one per
// 4 G-lane steps, which is what bounds that kernel on short tasks.
#ifndef KR_LANE_TPB
#define KR_LANE_TPB 512
#endif
#ifndef KR_LANE_WPE
#define KR_LANE_WPE 4
#endif
template <int RP, typename T>
__global__ void __launch_bounds__(KR_LANE_TPB) __attribute__((amdgpu_waves_per_eu(KR_LANE_WPE, 8)))
    k_rows_lane(ModeTables TT, Geom g, Tree tr, const double* __restrict__ Pprev, const double* __restrict__ Omega,
                const double* __restrict__ bD, T* __restrict__ Qout) {
  extern __shared__ double2 lane_fac2[];
  double* rows_fac = (double*)lane_fac2;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  {
    const int nf = g.I[N - 1] * RP;
    const double* __restrict__ A = TT.A[N - 1];
    for (int e = threadIdx.x; e < nf; e += blockDim.x) {
      const int i = e / RP, r = e % RP;
      rows_fac[e] = r < R ? A[(int64_t)i * R + r] : 0.0;
    }
    __syncthreads();
  }
  const int64_t ntask = tr.ncnt[N - 1] * nrhs;
  const int l64 = threadIdx.x & 63;
  const int lane = l64 & (RP - 1), gi = l64 / RP;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t tstride = (int64_t)gridDim.x * wpb;
  const int32_t* __restrict__ idxL = tr.idx[N];
  int nb0 = 0, nb1 = 0;
  int64_t npar = 0;
  // (node, rhs) of a task; one right-hand side needs no division
  auto node_of = [&](int64_t t) { return nrhs == 1 ? t : t / nrhs; };
  auto fetch = [&](int64_t t) {
    if (t < ntask) {
      const int64_t pp = node_of(t);
      nb0 = tr.fchild[N - 1][pp];
      nb1 = tr.fchild[N - 1][pp + 1];
      npar = N >= 3 ? tr.parent[N - 1][pp] : 0;
    }
  };
  const unsigned nrhs8 = (unsigned)nrhs * 8u;
  fetch(blockIdx.x * wpb + w);
  for (int64_t task_v = blockIdx.x * wpb + w; task_v < ntask; task_v += tstride) {
    // the task index in scalar registers (tasks number below 2^31), so that the
    // node's addresses are formed by scalar arithmetic
    const int64_t task = __builtin_amdgcn_readfirstlane((int)task_v);
    const int64_t p = node_of(task);
    const int q = (int)(task - p * nrhs);
    // the bounds and parent are wave-uniform: in scalar registers they make the
    // row and parent bases scalar, and the loads take 32-bit lane offsets
    const int j0 = __builtin_amdgcn_readfirstlane(nb0), j1 = __builtin_amdgcn_readfirstlane(nb1);
    const int64_t par = __builtin_amdgcn_readfirstlane((int)npar);
    fetch(task + tstride);
    T* __restrict__ qb = Qout + p * R * nrhs + q;
    if (j1 <= j0) {  // a node always has rows; kept for safety (uniform branch)
      if (l64 < R) qb[l64 * nrhs] = (T)0;
      continue;
    }
    // row j0 + c + l, addressed by 32-bit offsets from the node's wave-uniform
    // bases (clamped to the node's first row past the end, where Omega is taken
    // as 0)
    const int nrow = j1 - j0;
    const int32_t* __restrict__ ib = idxL + j0;
    const double* __restrict__ ob = Omega + j0;
    const double* __restrict__ bq = bD + (int64_t)j0 * nrhs + q;
    auto rowload = [&](int c, int& ix, double& om, double& bb) {
      const int k = c + l64;
      const unsigned kk = k < nrow ? (unsigned)k : 0u;
      ix = *(const int32_t*)((const char*)ib + kk * 4u);
      om = ld_at(ob, kk * 8u);
      bb = ld_at(bq, kk * nrhs8);
      if (k >= nrow) om = 0.0;
    };
    int ix;
    double om, bb;
    rowload(0, ix, om, bb);
    const double pv = rows_pnode<RP>(g, tr, Pprev, p, par, q, lane, gi);
    double pvs[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) pvs[r] = read_lane(pv, r);
    T acc[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) acc[r] = (T)0;
    for (int c = 0; c < nrow; c += 64) {
      int ixn = 0;
      double omn = 0.0, bbn = 0.0;
      if (c + 64 < nrow) rowload(c + 64, ixn, omn, bbn);
      const double2* __restrict__ row = (const double2*)(rows_fac + (int64_t)ix * RP);
      double a[RP];
#pragma unroll
      for (int k = 0; k < RP / 2; ++k) {
        const double2 v = row[k];
        a[2 * k] = v.x;
        a[2 * k + 1] = v.y;
      }
      double y = 0.0;
#pragma unroll
      for (int r = 0; r < RP; ++r) y = fma(a[r], pvs[r], y);
      const T u = (T)(om * (y - bb));
#pragma unroll
      for (int r = 0; r < RP; ++r) acc[r] = fma(u, (T)a[r], acc[r]);
      ix = ixn;
      om = omn;
      bb = bbn;
    }
    const T qv = lane_transpose_sum<RP>(acc, l64);
    const int r = l64 / (64 / RP);
    if ((l64 & (64 / RP - 1)) == 0 && r < R) qb[r * nrhs] = qv;
  }
}

// The LDS-staged rows for short nodes (a few rows each; three or more modes,
// R_{N-1} <= 16, one right-hand side): one wave takes a block of MN_NODES
// consecutive level-(N-1) nodes, whose rows are contiguous.
//   1. the block's forward values P_{N-1}[p] (16 per node), one node per 16-lane
//      group and pass (the contraction of P_{N-2}[parent] with a_{N-2}[i(p)] in
//      the same order as rows_pnode), into the wave's LDS;
//   2. the block's rows 64 at a time, one per lane: its node (a search of the
//      block's row bounds), u_j = Omega_j (<a_{N-1}[i(j)], P_{N-1}[node]> - b_j),
//      with (u_j, i(j)) left in the wave's LDS;
//   3. per node, lane r of its group adds u_j a_{N-1}[i(j)][r] over the node's
//      rows of the chunk, in row order, into the node's accumulator (LDS);
// and the nodes' accumulators are written as Q[p] at the end.  Compared with one
// node per wave, a block of nodes shares each memory round trip.
#define MN_NODES 8
// a wave's LDS writes are seen by its later LDS reads (the hardware keeps a wave's
// LDS operations in order); this keeps the compiler from moving them across
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}
#define MN_WAVE_LDS (MN_NODES * 16 * 2 + 64 + 32 + 16)   // doubles per wave: pv, sums, u, indices, bounds, parents
template <typename T>
__global__ void __launch_bounds__(KR_LANE_TPB) __attribute__((amdgpu_waves_per_eu(KR_LANE_WPE, 8)))
    k_rows_multi(ModeTables TT, Geom g, Tree tr, const double* __restrict__ Pprev, const double* __restrict__ Omega,
                 const double* __restrict__ bD, T* __restrict__ Qout) {
  constexpr int RP = 16, NGR = 4;
  extern __shared__ double2 multi_fac2[];
  double* rows_fac = (double*)multi_fac2;
  const int N = g.N;
  const int R = g.R[N - 1], Rp = g.R[N - 2];
  const int IL = g.I[N - 1];
  {
    const double* __restrict__ A = TT.A[N - 1];
    for (int e = threadIdx.x; e < IL * RP; e += blockDim.x) {
      const int i = e / RP, r = e % RP;
      rows_fac[e] = r < R ? A[(int64_t)i * R + r] : 0.0;
    }
    __syncthreads();
  }
  const int l64 = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lane = l64 & 15, gi = l64 >> 4;
  double* wl = rows_fac + (size_t)IL * RP + (size_t)w * MN_WAVE_LDS;
  double* pvl = wl;                          // MN_NODES x 16 forward values
  double* accl = wl + MN_NODES * 16;         // MN_NODES x 16 adjoint sums
  double* ul = accl + MN_NODES * 16;         // 64 u_j
  int* ixl = (int*)(ul + 64);                // 64 row indices
  int* bnd = ixl + 64;                       // MN_NODES + 1 row bounds
  int* parl = bnd + MN_NODES + 1;            // MN_NODES parents
  const int64_t S = tr.ncnt[N - 1];
  const int64_t nblk = (S + MN_NODES - 1) / MN_NODES;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t wg = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * wpb + w));
  const int64_t wstride = (int64_t)gridDim.x * wpb;
  const int32_t* __restrict__ idxL = tr.idx[N];
  const int32_t* __restrict__ fch = tr.fchild[N - 1];
  const int32_t* __restrict__ parL = tr.parent[N - 1];
  const double* __restrict__ arow = tr.arow[N - 1];
  const unsigned step8 = (unsigned)R * 8u;
  for (int64_t b = wg; b < nblk; b += wstride) {
    const int64_t p0 = __builtin_amdgcn_readfirstlane((int)(b * MN_NODES));
    const int nn = (int)min((int64_t)MN_NODES, S - p0);
    // row bounds and parents of the block's nodes (one round trip)
    if (l64 <= nn) bnd[l64] = fch[p0 + l64];
    if (l64 < nn) parl[l64] = parL[p0 + l64];
    wave_sync();
    const int r0 = bnd[0], r1 = bnd[nn];
    // the first chunk's row data, requested with the forward values' operands
    int ix0;
    double om0, bb0;
    {
      const int j = r0 + l64;
      const int jj = j < r1 ? j : r0;
      ix0 = idxL[jj];
      om0 = j < r1 ? Omega[jj] : 0.0;
      bb0 = bD[jj];
    }
    // 1. forward values, node p0 + 4 pass + gi in group gi (all of a pass's
    // operands requested together when R_{N-2} <= 16)
#pragma unroll 1
    for (int pass = 0; pass * NGR < nn; ++pass) {
      const int nl = pass * NGR + gi;
      double pv = 0.0;
      if (nl < nn && lane < R) {
        const int64_t pp = p0 + nl;
        const double* __restrict__ a = arow + pp * Rp;
        const double* __restrict__ src = Pprev + (int64_t)parl[nl] * Rp * R;
        if (Rp <= 16) {
          double av[16], sv[16];
#pragma unroll
          for (int s0 = 0; s0 < 16; ++s0) {
            const bool ok = s0 < Rp;
            av[s0] = ok ? a[s0] : 0.0;
            sv[s0] = ok ? ld_at(src, (unsigned)s0 * step8 + (unsigned)lane * 8u) : 0.0;
          }
#pragma unroll
          for (int s0 = 0; s0 < 16; ++s0) pv = fma(av[s0], sv[s0], pv);
        } else {
          for (int s0 = 0; s0 < Rp; ++s0) pv = fma(a[s0], ld_at(src, (unsigned)s0 * step8 + (unsigned)lane * 8u), pv);
        }
      }
      if (nl < MN_NODES) {
        pvl[nl * 16 + lane] = pv;
        accl[nl * 16 + lane] = 0.0;
      }
    }
    wave_sync();
    for (int c = r0; c < r1; c += 64) {
      // 2. one row per lane
      const int j = c + l64;
      const bool in = j < r1;
      const int jj = in ? j : r0;
      int nl = 0;
#pragma unroll
      for (int q = 1; q < MN_NODES; ++q) nl += (q < nn && bnd[q] <= jj) ? 1 : 0;
      int ix;
      double om, bb;
      if (c == r0) {
        ix = ix0;
        om = om0;
        bb = bb0;
      } else {
        ix = idxL[jj];
        om = in ? Omega[jj] : 0.0;
        bb = bD[jj];
      }
      const double2* __restrict__ row = (const double2*)(rows_fac + (int64_t)ix * RP);
      const double2* __restrict__ pvr = (const double2*)(pvl + nl * 16);
      double y = 0.0;
#pragma unroll
      for (int k = 0; k < RP / 2; ++k) {
        const double2 a = row[k], v = pvr[k];
        y = fma(a.x, v.x, y);
        y = fma(a.y, v.y, y);
      }
      ul[l64] = in ? om * (y - bb) : 0.0;
      ixl[l64] = ix;
      wave_sync();
      // 3. per node, lane r of its group over the node's rows of this chunk
      for (int pass = 0; pass * NGR < nn; ++pass) {
        const int nl2 = pass * NGR + gi;
        if (nl2 < nn) {
          const int a0 = max(bnd[nl2], c), a1 = min(bnd[nl2 + 1], min(c + 64, r1));
          T acc = (T)accl[nl2 * 16 + lane];
          for (int jr = a0; jr < a1; ++jr) {
            const int t = jr - c;
            acc = fma((T)ul[t], (T)rows_fac[(int64_t)ixl[t] * RP + lane], acc);
          }
          accl[nl2 * 16 + lane] = (double)acc;
        }
      }
      wave_sync();
    }
    // the block's adjoints
    for (int pass = 0; pass * NGR < nn; ++pass) {
      const int nl = pass * NGR + gi;
      if (nl < nn && lane < R) Qout[(p0 + nl) * R + lane] = (T)accl[nl * 16 + lane];
    }
    wave_sync();
  }
}

// The chunk table of the fused three-mode pass: the children of level-1 node p
// (n_p of them) split into k_p = ceil(n_p / ch) runs, run j starting at child
// floor(j n_p / k_p), numbered in node order by an exclusive scan of k_p over
// the level-1 nodes.  One workgroup of CH_THREADS threads.
#define CH_THREADS 1024
__global__ void __launch_bounds__(CH_THREADS) k_chunk_table(Tree tr, Chunks ck, int R0, int f32) {
  __shared__ int wsum[CH_THREADS / 64];
  const int S1 = (int)tr.cnt[1];
  const int32_t* __restrict__ fc = tr.fchild[1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int running = 0;
  for (int b0 = 0; b0 < S1; b0 += CH_THREADS) {
    const int p = b0 + (int)threadIdx.x;
    int f = 0, n = 0, k = 0;
    if (p < S1) {
      f = fc[p];
      n = fc[p + 1] - f;
      k = (n + ck.ch - 1) / ck.ch;
    }
    int v = k;   // inclusive scan of k over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(v, o, 64);
      if (lane >= o) v += t;
    }
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    int before = 0, total = 0;
    for (int i = 0; i < CH_THREADS / 64; ++i) {
      const int t = wsum[i];
      before += i < w ? t : 0;
      total += t;
    }
    const int off = running + before + v - k;
    if (off + k <= ck.cap)
      for (int j = 0; j < k; ++j) {
        ck.beg[off + j] = f + (int)(((int64_t)j * n) / k);
        ck.par[off + j] = p;
      }
    running += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ck.count = running;
    if (running <= ck.cap) ck.beg[running] = (int)tr.cnt[2];
  }
  if (running > ck.cap) return;
  __syncthreads();
  // the runs' factor rows, CH_U entries per thread per trip with every trip's
  // loads issued before its stores (the stores could alias ck.par as far as the
  // compiler knows, so it would not hoist them itself)
  const double* __restrict__ a0 = tr.arow[1];
  const int total = running * R0;
  constexpr int CH_U = 8;
  for (int e0 = threadIdx.x; e0 < total; e0 += CH_U * CH_THREADS) {
    int pr[CH_U];
    double a[CH_U];
#pragma unroll
    for (int u = 0; u < CH_U; ++u) {
      const int e = e0 + u * CH_THREADS;
      pr[u] = e < total ? ck.par[e / R0] : 0;
    }
#pragma unroll
    for (int u = 0; u < CH_U; ++u) {
      const int e = e0 + u * CH_THREADS;
      a[u] = e < total ? a0[(int64_t)pr[u] * R0 + (e % R0)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH_U; ++u) {
      const int e = e0 + u * CH_THREADS;
      if (e < total) {
        ck.arow[e] = a[u];
        if (f32) ck.arow32[e] = (float)a[u];
      }
    }
  }
}

// The fused pass of a three-mode problem (no segment roots), one workgroup of
// 256 threads per chunk c (the children s in [beg[c], beg[c+1]) of the level-1
// node p = par[c]):
//   P_1[p] = x contracted with a_0[i(p)], in LDS, summed as the forward level;
//   per (child s, rhs), one wave: P_2[s] from P_1[p] and a_1[i(s)], then the rows
//   of s as in the rows kernel, giving Q_2[s] in LDS;
//   Q1c[c][r][e] = sum_s a_1[i(s)][r] Q_2[s][e] in increasing s.
// The root adjoint sums the chunks in place of the level-1 nodes (each with the
// factor row of its node): the same sum, grouped by chunk.  Workgroups are
// independent, so the forward level, the rows and the last adjoint level cost
// one launch.  Dynamic LDS: W1 doubles for P_1, then ch R_1 and ch R_2 nrhs
// entries of T for the children's factor rows and Q_2.
template <int G, typename T>
// Threads per workgroup of the fused pass.  Measured at the 512^3 workload
// (bf16-refined solves/s): 256 threads 824; 512 781 (runs of 8), 774 (runs of 16);
// 1024 759 (runs of 16): wider workgroups leave more waves idle on short runs.
#ifndef KR_SUB_THREADS
#define KR_SUB_THREADS 256
#endif
__global__ void __launch_bounds__(KR_SUB_THREADS) k_subtree3(Geom g, Tree tr, Chunks ck, const double* __restrict__ x,
                                                 const double* __restrict__ Omega,
                                                 const double* __restrict__ bD, T* __restrict__ Q1c) {
  extern __shared__ double sub_lds[];
  constexpr int NGR = 64 / G;
  const int nrhs = g.nrhs;
  const int R0 = g.R[0], R1 = g.R[1], R = g.R[2];
  const unsigned W2 = (unsigned)(R * nrhs);
  const unsigned W1 = (unsigned)R1 * W2;
  double* P1 = sub_lds;
  T* A1 = (T*)(sub_lds + W1);
  T* Q2 = A1 + ck.ch * R1;
  const int c = blockIdx.x;
  const int p = ck.par[c];
  const int s0 = ck.beg[c], ns = ck.beg[c + 1] - s0;
  const int lane = threadIdx.x & (G - 1);
  const int gi = (threadIdx.x & 63) / G;
  const bool ln = lane < R;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int ntask = ns * nrhs;
  // the first task's rows are requested before P_1 is formed
  int task = w;
  int j0 = 0, j1 = 0;
  if (task < ntask) {
    j0 = tr.fchild[2][s0 + task / nrhs];
    j1 = tr.fchild[2][s0 + task / nrhs + 1];
  }
  RowsTask<G, KR_ROWS_PER_STEP> rt(tr.arow[3], nullptr, Omega, bD, j0, j1, R, nrhs, task < ntask ? task % nrhs : 0,
                                   lane, gi);
  if (task < ntask && j1 > j0) rt.load(0);
  // a wave's later tasks have their bounds requested one task ahead
  const int tstep = blockDim.x >> 6;
  int nj0 = 0, nj1 = 0;
  auto fetch = [&](int t) {
    if (t < ntask) {
      nj0 = tr.fchild[2][s0 + t / nrhs];
      nj1 = tr.fchild[2][s0 + t / nrhs + 1];
    }
  };
  fetch(task + tstep);
  {
    const double* __restrict__ a0 = tr.arow[1] + (int64_t)p * R0;
    for (unsigned e = threadIdx.x; e < W1; e += blockDim.x) P1[e] = dot_batched(a0, x + e, W1, R0);
    const T* __restrict__ a1 = node_rows<T>(tr, 2) + (int64_t)s0 * R1;
    for (int e = threadIdx.x; e < ns * R1; e += blockDim.x) A1[e] = a1[e];
  }
  __syncthreads();
  for (; task < ntask; task += tstep) {
    const int sl = task / nrhs, q = task - sl * nrhs;
    if (task != w) {
      j0 = nj0;
      j1 = nj1;
      fetch(task + tstep);
      rt = RowsTask<G, KR_ROWS_PER_STEP>(tr.arow[3], nullptr, Omega, bD, j0, j1, R, nrhs, q, lane, gi);
      if (j1 > j0) rt.load(0);
    }
    if (j1 <= j0) {  // a node always has rows; kept for safety (uniform branch)
      if (gi == 0 && ln) Q2[sl * W2 + lane * nrhs + q] = (T)0;
      continue;
    }
    // P_2[s][lane][q], summed as in the rows kernel (from LDS)
    double pv = 0.0;
    if (ln) {
      const double* __restrict__ a = tr.arow[2] + (int64_t)(s0 + sl) * R1;
      const unsigned step = W2;
      for (int r0 = gi; r0 < R1; r0 += 4 * NGR) {
        double as[4], sv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + u * NGR;
          as[u] = r < R1 ? a[r] : 0.0;
          sv[u] = r < R1 ? P1[r * step + lane * nrhs + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) pv = fma(as[u], sv[u], pv);
      }
    }
    pv = xgrp_sum<G>(pv);
    const T acc = rt.template run<T>(pv);
    if (gi == 0 && ln) Q2[sl * W2 + lane * nrhs + q] = acc;
  }
  __syncthreads();
  for (unsigned e = threadIdx.x; e < W1; e += blockDim.x) {
    const unsigned r = e / W2, cq = e - r * W2;
    T acc = 0;
    for (int sl = 0; sl < ns; ++sl) acc = fma(A1[sl * R1 + r], Q2[sl * W2 + cq], acc);
    Q1c[(size_t)c * W1 + e] = acc;
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

// Adjoint level k on v_mfma_f64_16x16x4 for R_{k-1} <= 16 (float64): one
// workgroup of 4 waves per (parent p, block of 16 columns), Q_{k-1}[p][r][c] =
// sum over the children s of p of a_{k-1}[i(s)][r] Q_k[s][c], an (R x children)
// (children x 16) product taken four children per matrix step.  Wave w takes the
// steps w, w + 4, ... (two per trip, their loads issued together); the waves'
// 16 x 16 accumulators are added in wave order through LDS.  Rows r >= R and
// columns c >= W are zero padding.  Against the one-workgroup-per-task VALU
// kernel this moves the contraction onto the matrix cores and shortens each
// task's chain of LDS staging steps.
typedef double it_f64x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_adj_level_mfma(Geom g, Tree tr, int k, const double* __restrict__ Qk,
                                                        double* __restrict__ Qout) {
  __shared__ double accs[3][4][64];
  const int Rk = g.R[k - 1];
  const int64_t W = g.rsuf[k] * g.nrhs;
  const int64_t ncb = (W + 15) / 16;
  const int64_t p = blockIdx.x / ncb;
  const int64_t c0 = (blockIdx.x - p * ncb) * 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int64_t s0 = tr.fchild[k - 1][p], s1 = tr.fchild[k - 1][p + 1];
  const double* __restrict__ arow = tr.arow[k];
  const int64_t cq = c0 + col;
  const bool rok = col < Rk, cok = cq < W;
  it_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  int64_t sb = s0 + 4 * w;
  for (; sb + 20 <= s1; sb += 32) {   // steps sb and sb + 16, all four children present
    const int64_t sa = sb + kq, sc = sb + 16 + kq;
    const double a0 = rok ? arow[sa * Rk + col] : 0.0;
    const double b0 = cok ? Qk[sa * W + cq] : 0.0;
    const double a1 = rok ? arow[sc * Rk + col] : 0.0;
    const double b1 = cok ? Qk[sc * W + cq] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
  }
  for (; sb < s1; sb += 16) {
    const int64_t sl = sb + kq;
    const double a = (sl < s1 && rok) ? arow[sl * Rk + col] : 0.0;
    const double b = (sl < s1 && cok) ? Qk[sl * W + cq] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  if (w > 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) accs[w - 1][u][lane] = acc[u];
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += accs[q][u][lane];
    double* __restrict__ Qo = Qout + p * Rk * W;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = kq + 4 * u;
      if (r < Rk && cok) Qo[(int64_t)r * W + cq] = acc[u];
    }
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
