// Preconditioner step of Algorithm 2's Richardson iteration, one workgroup:
//     h = g + lambda x,   d = M^+ h,   x <- x - (1 - sqrt(eps)) d
// with M^+ = kron G_n^{-1} (lambda = 0) or (kron V) diag(1 / (kron Lambda + lambda))
// (kron V)^T (the square Kronecker mat-vec theorem: mode products with the
// R_n x R_n factors).  Then the per-RHS stopping rule eta ||d|| <= tol ||x|| and
// the divergence test.
//
// Mode products are dense 16x16 tiles on the matrix cores: 16 fibres of the
// R-tensor per tile, the factor matrix as the A operand, zero padded to multiples
// of 16 (NB = ceil(max R_n / 16) blocks).  Float64 uses v_mfma_f64_16x16x4; the
// refined precisions (float32 tensor) use float32 VALU, bf16 16x16x16 or e4m3
// 16x16x32 MFMA with float32 accumulation.  The tensor sits in LDS when two
// copies fit (else in t0/t1), all factor matrices are staged in LDS once per
// launch when they fit, and elementwise phases issue their loads in batches.
//
// Refined (mixed-precision) iteration.  The fixed point of x <- x - eta M~^+ g(x)
// is g(x) = 0 for any M~^+ close enough to M^+ for the iteration to contract, so
// the preconditioner can be applied in low precision and the accuracy is won back
// by the iteration itself (iterative refinement; the paper only remarks on the
// bit complexity of its arithmetic).  In the refined modes the residual
// u = K~x - b~ is float64 (it cancels; see k_rows_adj), the adjoint K~^T Omega u
// accumulates in float32 over float copies of the adjoint levels' factor rows
// (k_rows_to_f32), the mode products of M^+ run as described above, and the
// update, norms and stopping rule stay float64.
#include "kr_internal.h"

namespace kr {

// float copies of the gathered factor rows of levels 1..N-1 (the adjoint levels).
__global__ void k_rows_to_f32(Geom g, Tree tr) {
  for (int k = 1; k < g.N; ++k) {
    const int64_t n = tr.cnt[k] * g.R[k - 1];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
      tr.arow32[k][i] = (float)tr.arow[k][i];
  }
}

typedef double pc_f64x4 __attribute__((ext_vector_type(4)));
typedef short pc_bf16x4 __attribute__((ext_vector_type(4)));
typedef float pc_f32x4 __attribute__((ext_vector_type(4)));

#define PC_MATS 4096   // LDS entries for the staged factor matrices
#ifndef PC_THREADS
#define PC_THREADS 512 // threads of the single-problem preconditioner kernels
#endif
#define PC_BATCH 8     // elements per thread whose loads are issued together

// Offset of mode n's matrix in the staged table.
__device__ __forceinline__ int pc_mat_off(const Geom& g, int n) {
  int o = 0;
  for (int m = 0; m < n; ++m) o += (int)(g.R[m] * g.R[m]);
  return o;
}

__device__ __forceinline__ bool pc_mats_fit(const Geom& g) { return pc_mat_off(g, g.N) <= PC_MATS; }

// Stage mode n's matrix (or all modes when they fit) into ms; caller syncs.  The
// loads of all staged entries of a thread are issued before the LDS stores.
template <typename TM>
__device__ void pc_stage(const Geom& g, const double* const* Ms, int n, bool all, TM* ms) {
  const int n0 = all ? 0 : n, n1 = all ? g.N : n + 1;
  int off = 0;
  for (int m = n0; m < n1; ++m) {
    const int RR = (int)(g.R[m] * g.R[m]);
    const double* __restrict__ M = Ms[m];
    for (int e0 = threadIdx.x; e0 < RR; e0 += PC_BATCH * blockDim.x) {
      double v[PC_BATCH];
#pragma unroll
      for (int u = 0; u < PC_BATCH; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        v[u] = e < RR ? M[e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PC_BATCH; ++u) {
        const int e = e0 + u * (int)blockDim.x;
        if (e < RR) ms[off + e] = (TM)v[u];
      }
    }
    off += RR;
  }
}

// h = g + lambda x into cur, where g is the sum, in block order, of nnb partial
// blocks of total entries each (the root adjoint's split; one block unless the
// tree has very many level-1 nodes).  Loads of PC_HB elements x 4 blocks are
// issued together.
#define PC_HB 4
template <typename TG, typename TT>
__device__ void pc_load_h(const TG* __restrict__ part, unsigned nnb, const double* __restrict__ x, double lambda,
                          TT* cur, int64_t total) {
  const int64_t bd = blockDim.x;
  for (int64_t e0 = threadIdx.x; e0 < total; e0 += PC_HB * bd) {
    TG gs[PC_HB];
    double xv[PC_HB];
#pragma unroll
    for (int u = 0; u < PC_HB; ++u) {
      const int64_t e = e0 + u * bd;
      gs[u] = TG(0);
      xv[u] = (e < total && lambda != 0.0) ? x[e] : 0.0;
    }
    for (unsigned b0 = 0; b0 < nnb; b0 += 4) {
      TG v[PC_HB][4];
#pragma unroll
      for (int u = 0; u < PC_HB; ++u)
#pragma unroll
        for (unsigned k = 0; k < 4; ++k) {
          const int64_t e = e0 + u * bd;
          v[u][k] = (e < total && b0 + k < nnb) ? part[(size_t)(b0 + k) * total + e] : TG(0);
        }
#pragma unroll
      for (int u = 0; u < PC_HB; ++u)
#pragma unroll
        for (unsigned k = 0; k < 4; ++k)
          if (b0 + k < nnb) gs[u] += v[u][k];
    }
#pragma unroll
    for (int u = 0; u < PC_HB; ++u) {
      const int64_t e = e0 + u * bd;
      if (e < total) cur[e] = (TT)((double)gs[u] + lambda * xv[u]);
    }
  }
}

// cur[r][q] *= dinv[r] (the diagonal (kron Lambda + lambda)^+), batched.
template <typename TT>
__device__ void pc_scale(const Geom& g, const double* __restrict__ dinv, TT* cur) {
  const int64_t total = g.Rtot * g.nrhs, bd = blockDim.x;
  for (int64_t e0 = threadIdx.x; e0 < total; e0 += PC_BATCH * bd) {
    double dv[PC_BATCH];
#pragma unroll
    for (int u = 0; u < PC_BATCH; ++u) {
      const int64_t e = e0 + u * bd;
      dv[u] = e < total ? dinv[e / g.nrhs] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PC_BATCH; ++u) {
      const int64_t e = e0 + u * bd;
      if (e < total) cur[e] = (TT)((double)cur[e] * dv[u]);
    }
  }
}

// The iterate's entries r = threadIdx.x + u blockDim.x (u < PC_BATCH) of a
// one-RHS problem whose x fits PC_BATCH entries per thread, loaded at kernel
// start together with the gradient, so that the update waits on no global load
// (ok = false: the update loads x itself).
struct PcX {
  double v[PC_BATCH];
  bool ok;
};
__device__ __forceinline__ void pc_prefetch_x(const Geom& g, const double* __restrict__ x, PcX& xr) {
  xr.ok = g.nrhs == 1 && g.Rtot <= (int64_t)PC_BATCH * blockDim.x;
  if (!xr.ok) return;
#pragma unroll
  for (int u = 0; u < PC_BATCH; ++u) {
    const int64_t r = threadIdx.x + (int64_t)u * blockDim.x;
    xr.v[u] = r < g.Rtot ? x[r] : 0.0;
  }
}

// Block-wide sums of two values with one set of barriers (fixed order, every
// thread gets both).  red holds 2 blockDim.x / 64 doubles.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int i = 0; i < nw; ++i) {
    ta += red[2 * i];
    tb += red[2 * i + 1];
  }
  __syncthreads();
  a = ta;
  b = tb;
}

// x <- x - eta d for right-hand sides not yet converged; float64 norms, the
// stopping rule and the divergence test; the iteration counter.
// it, done_lane and dn0_lane (lane q of every wave holds done[q] and dnorm0[q]) are
// read at kernel start; so is xr when xr.ok.
template <typename TT>
__device__ void pc_update(const Geom& g, const TT* d_t, double* __restrict__ x, double eta, double tol, int max_iter,
                          IterState* __restrict__ st, double* red, int it, int done_lane, double dn0_lane,
                          const PcX& xr) {
  int all = 1, div = 0;
  const int64_t bd = blockDim.x;
  for (int q = 0; q < g.nrhs; ++q) {
    const int done = __shfl(done_lane, q, 64);
    double dd = 0.0, xx = 0.0;
    for (int64_t r0 = threadIdx.x; r0 < g.Rtot; r0 += PC_BATCH * bd) {
      double xv[PC_BATCH], dv[PC_BATCH];
#pragma unroll
      for (int u = 0; u < PC_BATCH; ++u) {
        const int64_t r = r0 + u * bd;
        xv[u] = xr.ok ? xr.v[u] : (r < g.Rtot ? x[r * g.nrhs + q] : 0.0);
        dv[u] = r < g.Rtot ? (double)d_t[r * g.nrhs + q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PC_BATCH; ++u) {
        const int64_t r = r0 + u * bd;
        if (r < g.Rtot) {
          double xn = xv[u];
          if (!done) { xn = fma(-eta, dv[u], xn); x[r * g.nrhs + q] = xn; }
          dd = fma(dv[u], dv[u], dd);
          xx = fma(xn, xn, xx);
        }
      }
    }
    block_sum2(dd, xx, red);
    // the first norm comes from the launch's first loads (dn0_lane), and the
    // stopping flags are kept in registers: no global load waits here
    const double dn0 = __shfl(dn0_lane, q, 64);
    if (threadIdx.x == 0) {
      bool dq = done;
      if (!done) {
        const double dn = sqrt(dd), xn = sqrt(xx);
        const double rel = xn > 0.0 ? eta * dn / xn : (dn > 0.0 ? INFINITY : 0.0);
        st->rel[q] = rel;
        if (it == 0) { st->dnorm0[q] = dn; st->rel_first[q] = rel; }
        const bool bad = !isfinite(dn) || !isfinite(xn) || (it > 0 && dn > 1e6 * dn0 && dn > 0.0);
        if (bad) div = 1;
        if (rel <= tol || bad) { st->done[q] = 1; st->it_rhs[q] = it + 1; dq = true; }
      }
      all &= dq;
    }
  }
  if (threadIdx.x == 0) {
    st->iters = it + 1;
    if (div) st->diverged = 1;
    if (all || div || it + 1 >= max_iter) st->all_done = 1;
  }
}

// Fibre geometry of mode n: nfib fibres of R_n entries, stride post; fibre f
// starts at (f / post) R_n post + f % post.
struct PcFib {
  int Rn;
  unsigned post, nfib, ntile;
  __device__ PcFib(const Geom& g, int n) {
    Rn = (int)g.R[n];
    post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
    nfib = (unsigned)(g.Rtot * g.nrhs) / (unsigned)Rn;
    ntile = (nfib + 15u) / 16u;
  }
  __device__ __forceinline__ size_t base(unsigned f) const {
    const unsigned fq = f / post;
    return (size_t)fq * Rn * post + (f - fq * post);
  }
};

// float64 MFMA mode product: out = in x_n M (M^T when trans).  Tile of fibres
// t*16 .. t*16+15; v_mfma_f64_16x16x4: A lane l = M[a = l%16][k = l/16], B lane l
// = T[k = l/16][fibre l%16], D lane l item v = out[a = l/16 + 4v][fibre l%16].
template <int NB>
__device__ void pc_mode_f64(const Geom& g, int n, const double* M, int trans, const double* in, double* out) {
  const PcFib fb(g, n);
  const int Rn = fb.Rn;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  auto aval = [&](int a, int k) -> double {
    return (a < Rn && k < Rn) ? (trans ? M[k * Rn + a] : M[a * Rn + k]) : 0.0;
  };
  double A1[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) A1[ks] = aval(col, 4 * ks + kq);
  for (unsigned t = wave; t < fb.ntile; t += nw) {
    const unsigned f = t * 16u + col;
    const bool valid = f < fb.nfib;
    const size_t base = valid ? fb.base(f) : 0;
    double Bv[NB][4];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int k = bb * 16 + 4 * ks + kq;
        Bv[bb][ks] = valid && k < Rn ? in[base + (size_t)k * fb.post] : 0.0;
      }
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) {
      pc_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const double a = NB == 1 ? A1[ks] : aval(ab * 16 + col, bb * 16 + 4 * ks + kq);
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bv[bb][ks], acc, 0, 0, 0);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = ab * 16 + kq + 4 * v;
        if (valid && a < Rn) out[base + (size_t)a * fb.post] = acc[v];
      }
    }
  }
}

// float32 VALU mode product; each thread owns whole fibres (RM >= R_n).
template <int RM>
__device__ void pc_mode_f32(const Geom& g, int n, const float* M, int trans, const float* in, float* out) {
  const PcFib fb(g, n);
  const int Rn = fb.Rn;
  for (unsigned f = threadIdx.x; f < fb.nfib; f += blockDim.x) {
    const size_t base = fb.base(f);
    float v[RM];
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = b < Rn ? in[base + (size_t)b * fb.post] : 0.0f;
    for (int a = 0; a < Rn; ++a) {
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < Rn) acc = fmaf(trans ? M[b * Rn + a] : M[a * Rn + b], v[b], acc);
      out[base + (size_t)a * fb.post] = acc;
    }
  }
}

// float -> bf16 bits, round to nearest even (NaN stays NaN, overflow goes to inf).
__device__ __forceinline__ short pc_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// Two floats -> two e4m3 bytes (low 16 bits), hardware conversion with rounding
// to nearest even and saturation.
__device__ __forceinline__ unsigned pc_to_fp8x2(float a, float b) {
  return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xFFFFu;
}

// bf16 MFMA mode product, 16x16x16 tiles: A lane l = M[l%16][4(l/16)..+3], B lane l
// = T[4(l/16)..+3][fibre l%16], D lane l = out[4(l/16)..+3][fibre l%16].
template <int NB>
__device__ void pc_mode_bf16(const Geom& g, int n, const float* M, int trans, const float* in, float* out) {
  const PcFib fb(g, n);
  const int Rn = fb.Rn;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  auto afrag = [&](int ab, int bb) {
    pc_bf16x4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = ab * 16 + col, k = bb * 16 + 4 * kq + i;
      v[i] = pc_to_bf16((a < Rn && k < Rn) ? (trans ? M[k * Rn + a] : M[a * Rn + k]) : 0.0f);
    }
    return v;
  };
  const pc_bf16x4 A1 = afrag(0, 0);
  for (unsigned t = wave; t < fb.ntile; t += nw) {
    const unsigned f = t * 16u + col;
    const bool valid = f < fb.nfib;
    const size_t base = valid ? fb.base(f) : 0;
    pc_bf16x4 Bv[NB];
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = bb * 16 + 4 * kq + i;
        Bv[bb][i] = pc_to_bf16(valid && k < Rn ? in[base + (size_t)k * fb.post] : 0.0f);
      }
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) {
      pc_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(NB == 1 ? A1 : afrag(ab, bb), Bv[bb], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = ab * 16 + 4 * kq + i;
        if (valid && a < Rn) out[base + (size_t)a * fb.post] = acc[i];
      }
    }
  }
}

// e4m3 MFMA mode product, 16x16x32 tiles: A lane l = row l%16, k 8(l/16)..+7; B
// lane l = k 8(l/16)..+7 of fibre l%16; D as for bf16.  NA = ceil(R_n/16) row
// blocks, NK = ceil(R_n/32) contraction blocks.  Operands are scaled by sm
// (matrix) and st (tensor) into the e4m3 range; the result is scaled back.
template <int NA, int NK>
__device__ void pc_mode_fp8(const Geom& g, int n, const float* M, int trans, float sm, float st, const float* in,
                            float* out) {
  const PcFib fb(g, n);
  const int Rn = fb.Rn;
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
      pk |= (unsigned long long)pc_to_fp8x2(v[0], v[1]) << (8 * i);
    }
    return (long)pk;
  };
  const long A1 = afrag(0, 0);
  for (unsigned t = wave; t < fb.ntile; t += nw) {
    const unsigned f = t * 16u + col;
    const bool valid = f < fb.nfib;
    const size_t base = valid ? fb.base(f) : 0;
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
          v[h] = valid && k < Rn ? st * in[base + (size_t)k * fb.post] : 0.0f;
        }
        pk |= (unsigned long long)pc_to_fp8x2(v[0], v[1]) << (8 * i);
      }
      Bv[kb] = (long)pk;
    }
#pragma unroll
    for (int ab = 0; ab < NA; ++ab) {
      pc_f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kb = 0; kb < NK; ++kb)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(NA == 1 ? A1 : afrag(ab, kb), Bv[kb], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = ab * 16 + 4 * kq + i;
        if (valid && a < Rn) out[base + (size_t)a * fb.post] = acc[i] * unscale;
      }
    }
  }
}

__device__ __forceinline__ float pc_block_max(float v, float* red) {
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

// e4m3 scale for values of largest magnitude mx: the largest maps to 224, half the
// e4m3 maximum, so that rounding cannot saturate.
__device__ __forceinline__ float pc_fp8_scale(float mx) { return (mx > 0.0f && isfinite(mx)) ? 224.0f / mx : 1.0f; }

// The precision-specific mode product.  mscale: e4m3 scale of M (fp8 only).
template <int MODE, int NB>
__device__ void pc_mode_lp(const Geom& g, int n, const float* M, int trans, float mscale, const float* in, float* out,
                           float* redf) {
  if (MODE == KR_PREC_F32) {
    pc_mode_f32<16 * NB>(g, n, M, trans, in, out);
  } else if (MODE == KR_PREC_BF16) {
    pc_mode_bf16<NB>(g, n, M, trans, in, out);
  } else {
    float mx = 0.0f;
    const int64_t RT = g.Rtot * g.nrhs;
    for (int64_t e = threadIdx.x; e < RT; e += blockDim.x) mx = fmaxf(mx, fabsf(in[e]));
    const float st = pc_fp8_scale(pc_block_max(mx, redf));
    pc_mode_fp8<NB, (NB + 1) / 2>(g, n, M, trans, mscale, st, in, out);
  }
}

// Float64 step of one workgroup (any multiple of 64 threads).  grad holds the
// gradient as nnb partial blocks (summed here); dinv (Rtot) holds
// 1 / (kron Lambda + lambda) (0 where the sum vanishes) for the eigenvector form.
// cur/nxt are the two tensor buffers (LDS or global); ms stages factor matrices
// (PC_MATS entries), red holds 16 doubles.  Returns without touching x when the
// state is already converged.
template <int NB>
__device__ void pc_step_f64(const ModeTables& T, const Geom& g, const double* __restrict__ grad, unsigned nnb,
                            const double* __restrict__ dinv, double* __restrict__ x, double* cur, double* nxt,
                            double lambda, double eta, double tol, int max_iter, int use_ginv,
                            IterState* __restrict__ st, double* red, double* ms) {
  // state loads issued together with the staging and h loads below
  const int all_done = st->all_done;
  const int it0 = st->iters;
  const int done_lane = (int)(threadIdx.x & 63) < g.nrhs ? st->done[threadIdx.x & 63] : 1;
  const double dn0_lane = (int)(threadIdx.x & 63) < g.nrhs ? st->dnorm0[threadIdx.x & 63] : 0.0;
  const int64_t total = g.Rtot * g.nrhs;
  const bool all = pc_mats_fit(g);
  const double* const* Ms = use_ginv ? T.Ginv : T.V;
  PcX xr;
  pc_prefetch_x(g, x, xr);
  if (all) pc_stage(g, Ms, 0, true, ms);
  pc_load_h(grad, nnb, x, lambda, cur, total);
  __syncthreads();
  if (all_done) return;
  auto product = [&](int n, int trans) {
    if (!all) {
      pc_stage(g, Ms, n, false, ms);
      __syncthreads();
    }
    pc_mode_f64<NB>(g, n, all ? ms + pc_mat_off(g, n) : ms, trans, cur, nxt);
    __syncthreads();
    double* tmp = cur; cur = nxt; nxt = tmp;
  };
  if (use_ginv) {
    for (int n = 0; n < g.N; ++n) product(n, 0);
  } else {
    for (int n = 0; n < g.N; ++n) product(n, 1);
    pc_scale(g, dinv, cur);
    __syncthreads();
    for (int n = 0; n < g.N; ++n) product(n, 0);
  }
  pc_update(g, cur, x, eta, tol, max_iter, st, red, it0, done_lane, dn0_lane, xr);
}

// Float64 step as its own launch (one workgroup of PC_THREADS threads); the tensor
// buffers are in dynamic LDS when lds != 0, else t0/t1.
template <int NB>
__global__ void __launch_bounds__(PC_THREADS) k_precond_update(ModeTables T, Geom g, const double* __restrict__ grad,
                                                       unsigned nnb,
                                                       const double* __restrict__ dinv, double* __restrict__ x,
                                                       double* __restrict__ t0, double* __restrict__ t1, int lds,
                                                       double lambda, double eta, double tol, int max_iter,
                                                       int use_ginv, IterState* __restrict__ st) {
  extern __shared__ double pd_dyn[];
  __shared__ double red[2 * PC_THREADS / 64];
  __shared__ double ms[PC_MATS];
  const int64_t total = g.Rtot * g.nrhs;
  pc_step_f64<NB>(T, g, grad, nnb, dinv, x, lds ? pd_dyn : t0, lds ? pd_dyn + total : t1, lambda, eta, tol, max_iter,
                  use_ginv, st, red, ms);
}

// Refined-precision step: float32 gradient and tensor, mode products in MODE.
// fp8 takes the eigenvector form also for lambda = 0: its orthogonal factors
// round far better in e4m3 than the inverse Grams (fewer iterations, measured).
// One workgroup of any multiple of 64 threads; cur/nxt are the tensor buffers,
// red holds 2 blockDim.x / 64 doubles, redf blockDim.x / 64 floats, ms PC_MATS
// floats and mscale KR_MAXN floats (all LDS).  Returns without touching x when
// the state is already converged.
template <int MODE, int NB>
__device__ void pc_step_mp(const ModeTables& T, const Geom& g, const float* __restrict__ grad, unsigned nnb,
                           const double* __restrict__ dinv, double* __restrict__ x, float* cur, float* nxt,
                           double lambda, double eta, double tol, int max_iter, int use_ginv,
                           IterState* __restrict__ st, double* red, float* redf, float* ms, float* mscale) {
  // state loads issued together with the staging and h loads below
  const int all_done = st->all_done;
  const int it0 = st->iters;
  const int done_lane = (int)(threadIdx.x & 63) < g.nrhs ? st->done[threadIdx.x & 63] : 1;
  const double dn0_lane = (int)(threadIdx.x & 63) < g.nrhs ? st->dnorm0[threadIdx.x & 63] : 0.0;
  const int64_t total = g.Rtot * g.nrhs;
  const bool ginv = use_ginv && MODE != KR_PREC_FP8;
  const bool all = pc_mats_fit(g);
  const double* const* Ms = ginv ? T.Ginv : T.V;
  PcX xr;
  pc_prefetch_x(g, x, xr);
  if (all) pc_stage(g, Ms, 0, true, ms);
  pc_load_h(grad, nnb, x, lambda, cur, total);
  __syncthreads();
  if (all_done) return;
  auto scale_of = [&](int n, const float* M) {
    if (MODE == KR_PREC_FP8) {
      float mx = 0.0f;
      for (int e = threadIdx.x; e < g.R[n] * g.R[n]; e += blockDim.x) mx = fmaxf(mx, fabsf(M[e]));
      mx = pc_block_max(mx, redf);
      if (threadIdx.x == 0) mscale[n] = pc_fp8_scale(mx);
      __syncthreads();
    }
  };
  if (all)
    for (int n = 0; n < g.N; ++n) scale_of(n, ms + pc_mat_off(g, n));
  auto product = [&](int n, int trans) {
    if (!all) {
      pc_stage(g, Ms, n, false, ms);
      __syncthreads();
      scale_of(n, ms);
    }
    pc_mode_lp<MODE, NB>(g, n, all ? ms + pc_mat_off(g, n) : ms, trans, MODE == KR_PREC_FP8 ? mscale[n] : 1.0f, cur,
                         nxt, redf);
    __syncthreads();
    float* tmp = cur; cur = nxt; nxt = tmp;
  };
  if (ginv) {
    for (int n = 0; n < g.N; ++n) product(n, 0);
  } else {
    for (int n = 0; n < g.N; ++n) product(n, 1);
    pc_scale(g, dinv, cur);
    __syncthreads();
    for (int n = 0; n < g.N; ++n) product(n, 0);
  }
  pc_update(g, cur, x, eta, tol, max_iter, st, red, it0, done_lane, dn0_lane, xr);
}

// Refined-precision step as its own launch (one workgroup of PC_THREADS threads);
// the tensor buffers are in dynamic LDS when lds != 0, else t0/t1.
template <int MODE, int NB>
__global__ void __launch_bounds__(PC_THREADS) k_precond_mp(ModeTables T, Geom g, const float* __restrict__ grad,
                                                   unsigned nnb,
                                                   const double* __restrict__ dinv, double* __restrict__ x,
                                                   float* __restrict__ t0, float* __restrict__ t1, int lds,
                                                   double lambda, double eta, double tol, int max_iter, int use_ginv,
                                                   IterState* __restrict__ st) {
  extern __shared__ float mp_dyn[];
  __shared__ double red[2 * PC_THREADS / 64];
  __shared__ float redf[PC_THREADS / 64];
  __shared__ float ms[PC_MATS];
  __shared__ float mscale[KR_MAXN];
  const int64_t total = g.Rtot * g.nrhs;
  pc_step_mp<MODE, NB>(T, g, grad, nnb, dinv, x, lds ? mp_dyn : t0, lds ? mp_dyn + total : t1, lambda, eta, tol,
                       max_iter, use_ginv, st, red, redf, ms, mscale);
}

// dinv[r] = 1 / (prod_n lambda_n[r_n] + lambda), 0 where that sum is not positive.
__global__ void k_precond_diag(ModeTables T, Geom g, double lambda, double* __restrict__ dinv) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < g.Rtot; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e;
    double prod = 1.0;
    for (int n = g.N - 1; n >= 0; --n) {
      const int rn = (int)(r % g.R[n]);
      r /= g.R[n];
      prod *= T.evals[n][rn];
    }
    const double den = prod + lambda;
    dinv[e] = den > 0.0 ? 1.0 / den : 0.0;
  }
}

}  // namespace kr
