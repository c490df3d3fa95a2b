// Refined (mixed-precision) Richardson step of Algorithm 2.
//
// The fixed point of  x <- x - eta M~^+ g(x)  is g(x) = 0 for any M~^+ close
// enough to M^+ for the iteration to contract, so the preconditioner can be
// applied in low precision and the accuracy is won back by the iteration
// itself (iterative refinement; the paper only remarks on the bit complexity of
// its arithmetic).  In the refined modes:
//   residual  u = K~x - b~          float64 (it cancels; see k_rows_adj)
//   adjoint   g = K~^T Omega u       float32 accumulation
//   correction d = M^+ (g + lambda x) with every mode product in
//               KR_PREC_F32   float32 VALU,
//               KR_PREC_BF16  bf16 MFMA 16x16x16, float32 accumulation,
//               KR_PREC_FP8   fp8 (OCP e4m3) MFMA 16x16x32, float32 accumulation,
//                             per-operand scales to the e4m3 range,
//   update    x <- x - eta d, norms and the stopping rule in float64.
// M^+ is the same operator as in the float64 path: kron G_n^{-1} for lambda = 0,
// (kron V) (kron Lambda + lambda)^+ (kron V)^T otherwise (the square Kronecker
// mat-vec theorem applies it by mode products).
#include "kr_internal.h"

namespace kr {

typedef short mp_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mp_f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (NaN stays NaN, overflow goes to inf).
__device__ __forceinline__ short mp_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Two floats -> two e4m3 bytes (low 16 bits), hardware conversion with rounding
// to nearest even and saturation.
__device__ __forceinline__ unsigned mp_to_fp8x2(float a, float b) {
  return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

__device__ __forceinline__ float mp_block_max(float v, float* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  float r = 0.0f;
  for (int i = 0; i < nw; ++i) r = fmaxf(r, red[i]);
  __syncthreads();
  return r;
}

// out = in x_n M (trans: M^T), float32 VALU; each thread owns whole fibres.
template <int RM>
__device__ void mp_fibre_f32(const Geom& g, int n, const float* __restrict__ M, int trans, const float* in,
                             float* out) {
  const int Rn = g.R[n];
  const unsigned post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
  const unsigned nfib = (unsigned)(g.Rtot * g.nrhs) / (unsigned)Rn;
  for (unsigned f = threadIdx.x; f < nfib; f += blockDim.x) {
    const unsigned fq = f / post;
    const size_t base = (size_t)fq * Rn * post + (f - fq * post);
    float v[RM];
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = b < Rn ? in[base + (size_t)b * post] : 0.0f;
    for (int a = 0; a < Rn; ++a) {
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < Rn) acc = fmaf(trans ? M[b * Rn + a] : M[a * Rn + b], v[b], acc);
      out[base + (size_t)a * post] = acc;
    }
  }
}

// bf16 MFMA mode product.  Tiles of 16 fibres; NB = ceil(R_n / 16) blocks along
// the mode.  For a tile, D[a][f] = sum_b M[a][b] T[b][f] with A = M block
// (lane l: row l%16, k 4(l/16)..+3), B = fibre block (lane l: k 4(l/16)..+3 of
// fibre l%16), D (lane l: rows 4(l/16)..+3 of fibre l%16).
template <int NB>
__device__ void mp_mfma_bf16(const Geom& g, int n, const float* M, int trans, const float* in,
                             float* out) {
  const int Rn = g.R[n];
  const unsigned post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
  const unsigned nfib = (unsigned)(g.Rtot * g.nrhs) / (unsigned)Rn;
  const unsigned ntile = (nfib + 15u) / 16u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  // A fragment of block (ab, bb) from the LDS copy of M; with one block it is
  // loaded once, otherwise per use (a register copy of every block would spill)
  auto afrag = [&](int ab, int bb) {
    mp_bf16x4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = ab * 16 + col, k = bb * 16 + 4 * kq + i;
      v[i] = mp_to_bf16((a < Rn && k < Rn) ? (trans ? M[k * Rn + a] : M[a * Rn + k]) : 0.0f);
    }
    return v;
  };
  const mp_bf16x4 A1 = afrag(0, 0);
  for (unsigned t = wave; t < ntile; t += nw) {
    const unsigned f = t * 16u + col;
    const bool valid = f < nfib;
    const unsigned fq = valid ? f / post : 0u;
    const size_t base = valid ? (size_t)fq * Rn * post + (f - fq * post) : 0;
    mp_bf16x4 Bv[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = bb * 16 + 4 * kq + i;
        Bv[bb][i] = mp_to_bf16(valid && k < Rn ? in[base + (size_t)k * post] : 0.0f);
      }
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) {
      mp_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(NB == 1 ? A1 : afrag(ab, bb), Bv[bb], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = ab * 16 + 4 * kq + i;
        if (valid && a < Rn) out[base + (size_t)a * post] = acc[i];
      }
    }
  }
}

// fp8 (e4m3) MFMA mode product, 16x16x32 tiles: A lane l holds row l%16, k
// 8(l/16)..+7; B lane l holds k 8(l/16)..+7 of fibre l%16; D as for bf16.
// NA = ceil(R_n / 16) row blocks, NK = ceil(R_n / 32) contraction blocks.  The
// operands are scaled by sm (matrix) and st (tensor) into the e4m3 range and the
// float32 result is scaled back.
template <int NA, int NK>
__device__ void mp_mfma_fp8(const Geom& g, int n, const float* M, int trans, float sm, float st,
                            const float* in, float* out) {
  const int Rn = g.R[n];
  const unsigned post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
  const unsigned nfib = (unsigned)(g.Rtot * g.nrhs) / (unsigned)Rn;
  const unsigned ntile = (nfib + 15u) / 16u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const float unscale = 1.0f / (sm * st);
  auto afrag = [&](int ab, int kb) {
    unsigned long long pk = 0;
#pragma unroll
    for (int i = 0; i < 8; i += 2) {
      float v[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int a = ab * 16 + col, k = kb * 32 + 8 * kq + i + h;
        v[h] = (a < Rn && k < Rn) ? sm * (trans ? M[k * Rn + a] : M[a * Rn + k]) : 0.0f;
      }
      pk |= (unsigned long long)mp_to_fp8x2(v[0], v[1]) << (8 * i);
    }
    return (long)pk;
  };
  const long A1 = afrag(0, 0);
  for (unsigned t = wave; t < ntile; t += nw) {
    const unsigned f = t * 16u + col;
    const bool valid = f < nfib;
    const unsigned fq = valid ? f / post : 0u;
    const size_t base = valid ? (size_t)fq * Rn * post + (f - fq * post) : 0;
    long Bv[NK];
#pragma unroll
    for (int kb = 0; kb < NK; ++kb) {
      unsigned long long pk = 0;
#pragma unroll
      for (int i = 0; i < 8; i += 2) {
        float v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = kb * 32 + 8 * kq + i + h;
          v[h] = valid && k < Rn ? st * in[base + (size_t)k * post] : 0.0f;
        }
        pk |= (unsigned long long)mp_to_fp8x2(v[0], v[1]) << (8 * i);
      }
      Bv[kb] = (long)pk;
    }
#pragma unroll
    for (int ab = 0; ab < NA; ++ab) {
      mp_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(NA == 1 ? A1 : afrag(ab, kb), Bv[kb], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = ab * 16 + 4 * kq + i;
        if (valid && a < Rn) out[base + (size_t)a * post] = acc[i] * unscale;
      }
    }
  }
}

// e4m3 scale for values of largest magnitude mx: the largest maps to 224, half
// the e4m3 maximum, so that the rounding of the products cannot saturate.
__device__ __forceinline__ float mp_fp8_scale(float mx) {
  return (mx > 0.0f && isfinite(mx)) ? 224.0f / mx : 1.0f;
}

// One mode product in the precision MODE.  NB = ceil(max_n R_n / 16) is fixed per
// kernel (a mode with fewer 16-blocks is zero padded): instantiating every block
// count inside one kernel makes the register allocator spill.
template <int MODE, int NB>
__device__ void mp_mode_product(const Geom& g, int n, const float* M, int trans, float mscale, const float* in,
                                float* out, float* red) {
  if (MODE == KR_PREC_F32) {
    mp_fibre_f32<16 * NB>(g, n, M, trans, in, out);
  } else if (MODE == KR_PREC_BF16) {
    mp_mfma_bf16<NB>(g, n, M, trans, in, out);
  } else {
    float mx = 0.0f;
    const int64_t RT = g.Rtot * g.nrhs;
    for (int64_t e = threadIdx.x; e < RT; e += blockDim.x) mx = fmaxf(mx, fabsf(in[e]));
    const float st = mp_fp8_scale(mp_block_max(mx, red));
    mp_mfma_fp8<NB, (NB + 1) / 2>(g, n, M, trans, mscale, st, in, out);
  }
}

// d = M^+ (g + lambda x) in the precision MODE, x <- x - eta d for right-hand sides
// not yet converged, then the float64 norms and stopping rule of the float64
// path.  One workgroup of 256 threads.  The two tensor buffers live in dynamic
// LDS when lds != 0 (2 Rtot nrhs floats), else in t0/t1.
template <int MODE, int NB>
__global__ void __launch_bounds__(256) k_precond_mp(ModeTables T, Geom g, const float* __restrict__ grad,
                                                    double* __restrict__ x, float* __restrict__ t0,
                                                    float* __restrict__ t1, int lds, double lambda, double eta,
                                                    double tol, int max_iter, int use_ginv,
                                                    IterState* __restrict__ st) {
  extern __shared__ float mp_dyn[];
  __shared__ double red[16];
  __shared__ float redf[16];
  __shared__ float ms[64 * 64];
  __shared__ float mscale;
  if (st->all_done) return;
  const int64_t total = g.Rtot * g.nrhs;
  float* cur = lds ? mp_dyn : t0;
  float* nxt = lds ? mp_dyn + total : t1;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) cur[e] = (float)((double)grad[e] + lambda * x[e]);
  // stage M (float64 table) into LDS as float; fp8 also needs its scale
  auto stage = [&](const double* M, int n) {
    __syncthreads();
    float mx = 0.0f;
    for (int e = threadIdx.x; e < g.R[n] * g.R[n]; e += blockDim.x) {
      ms[e] = (float)M[e];
      mx = fmaxf(mx, fabsf(ms[e]));
    }
    if (MODE == KR_PREC_FP8) {
      mx = mp_block_max(mx, redf);
      if (threadIdx.x == 0) mscale = mp_fp8_scale(mx);
    }
    __syncthreads();
  };
  // fp8 takes the eigenvector form also for lambda = 0: its orthogonal factors
  // round far better in e4m3 than the inverse Grams (measured: fewer iterations)
  if (use_ginv && MODE != KR_PREC_FP8) {
    for (int n = 0; n < g.N; ++n) {
      stage(T.Ginv[n], n);
      mp_mode_product<MODE, NB>(g, n, ms, 0, mscale, cur, nxt, redf);
      float* tmp = cur; cur = nxt; nxt = tmp;
    }
  } else {
    for (int n = 0; n < g.N; ++n) {
      stage(T.V[n], n);
      mp_mode_product<MODE, NB>(g, n, ms, 1, mscale, cur, nxt, redf);
      float* tmp = cur; cur = nxt; nxt = tmp;
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
      cur[e] = den > 0.0 ? (float)((double)cur[e] / den) : 0.0f;
    }
    for (int n = 0; n < g.N; ++n) {
      stage(T.V[n], n);
      mp_mode_product<MODE, NB>(g, n, ms, 0, mscale, cur, nxt, redf);
      float* tmp = cur; cur = nxt; nxt = tmp;
    }
  }
  __syncthreads();
  const int it = st->iters;
  int all = 1, div = 0;
  for (int q = 0; q < g.nrhs; ++q) {
    const int done = st->done[q];
    double dd = 0.0, xx = 0.0;
    for (int64_t r = threadIdx.x; r < g.Rtot; r += blockDim.x) {
      const int64_t e = r * g.nrhs + q;
      const double d = (double)cur[e];
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

// float copies of the gathered factor rows of levels 1..N-1 (the adjoint levels).
__global__ void k_rows_to_f32(Geom g, Tree tr) {
  for (int k = 1; k < g.N; ++k) {
    const int64_t n = tr.cnt[k] * g.R[k - 1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      tr.arow32[k][i] = (float)tr.arow[k][i];
  }
}

}  // namespace kr
