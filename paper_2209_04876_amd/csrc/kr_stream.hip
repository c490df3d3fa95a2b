// Streaming KronMatMul kernels (Lemma kron_mat_mul): the full-size products that
// touch every entry of b.
//   kron_loss  f(x) = ||K x - b||^2 + lambda ||x||^2.  Y = x x_{N-1} A_{N-1} .. x_1 A_1
//              is expanded by mode products (all modes but the first); the last
//              stage (K x)[i_0][c] = sum_{r_0} A_0[i_0][r_0] Y[r_0][c] is fused with the
//              read of b and the squared residual, so b is read exactly once.
//   kron_exact x* = (kron V) diag(kron s / (kron s^2 + lambda)) (kron U)^T b with
//              A_n = U_n S_n V_n^T from the Gram eigen-decomposition (the exact
//              KronMatMul baseline); the first contraction (U_0^T over i_0) streams b.
// One thread owns one column c of the [I_0][C] view of b (C = prod_{n>0} I_n * nrhs)
// and walks i_0, so consecutive lanes read consecutive addresses.
#include "kr_internal.h"

namespace kr {

// out[pre][o][post] = sum_{r < Rin} M(o, r) in[pre][r][post];
// M(o, r) = M[o * Rin + r], or M[r * Rout + o] when trans.
__global__ void __launch_bounds__(256) k_mode_product(const double* __restrict__ in, double* __restrict__ out,
                                                     int64_t pre, int Rin, int Rout, int64_t post,
                                                     const double* __restrict__ M, int trans) {
  const int64_t total = pre * Rout * post;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / ((int64_t)Rout * post);
    const int64_t rem = e - b * Rout * post;
    const int o = (int)(rem / post);
    const int64_t c = rem - (int64_t)o * post;
    const double* src = in + b * Rin * post + c;
    double acc = 0.0;
    if (trans) {
      for (int r = 0; r < Rin; ++r) acc = fma(M[(int64_t)r * Rout + o], src[(int64_t)r * post], acc);
    } else {
      const double* mo = M + (int64_t)o * Rin;
      for (int r = 0; r < Rin; ++r) acc = fma(mo[r], src[(int64_t)r * post], acc);
    }
    out[e] = acc;
  }
}

// The same product for R_in <= RIN: workgroup (c block, block of MP_OUT outputs
// o, pre index) -- o is uniform over the workgroup, so M is read through the
// scalar cache; each thread loads its input fibre in[pre][.][c] once and forms
// MP_OUT outputs from it.
#define MP_OUT 16
template <int RIN>
__global__ void __launch_bounds__(256) k_mode_product_fibre(const double* __restrict__ in, double* __restrict__ out,
                                                           int64_t pre, int Rin, int Rout, int64_t post,
                                                           const double* __restrict__ M, int trans) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= post) return;
  const int o0 = blockIdx.y * MP_OUT;
  for (int64_t b = blockIdx.z; b < pre; b += gridDim.z) {
    const double* src = in + b * Rin * post + c;
    double v[RIN];
#pragma unroll
    for (int r = 0; r < RIN; ++r) v[r] = r < Rin ? src[(int64_t)r * post] : 0.0;
#pragma unroll 4
    for (int oo = 0; oo < MP_OUT; ++oo) {
      const int o = o0 + oo;
      if (o >= Rout) break;
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < RIN; ++r)
        if (r < Rin) acc = fma(trans ? M[(int64_t)r * Rout + o] : M[(int64_t)o * Rin + r], v[r], acc);
      out[(b * Rout + o) * post + c] = acc;
    }
  }
}

#define STREAM_ROWS 64

typedef double ks_f64x4 __attribute__((ext_vector_type(4)));

// Squared residual, streaming b once: acc[c] = sum_{i0} ((A0 Y)[i0][c] - b[i0][c])^2 for
// the [I_0][C] view of b (b of dtype bdt).  (A0 Y) is formed on the matrix cores:
// each wave owns 16 columns and walks the rows in blocks of 16 with
// v_mfma_f64_16x16x4 (A = A0 block, lane l: row l%16, k l/16; B = Y block, lane
// l: k l/16, column l%16; D lane l item v: row l/16 + 4v, column l%16), KS
// k-steps of 4.  A0 is staged in LDS per workgroup (rows padded against bank
// conflicts), in chunks when large.  Two row blocks' loads of b are in flight.
// The workgroup writes its per-RHS sums partial[blockIdx.x * nrhs + q] (columns
// c = col * nrhs + q).
#define SL_WAVES 16
#define SL_LDS 8192
template <int KS>
__global__ void __launch_bounds__(64 * SL_WAVES) k_stream_loss(const double* __restrict__ A0, int I0, int R0,
                                                              const double* __restrict__ Y, const void* __restrict__ b,
                                                              int bdt, int64_t C, int nrhs,
                                                              double* __restrict__ partial) {
  __shared__ double a_s[SL_LDS];
  __shared__ double red[SL_WAVES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int stride = 4 * KS + 1;   // padded row of A0 in LDS
  const int64_t c0 = ((int64_t)blockIdx.x * SL_WAVES + wave) * 16;
  const int64_t c = c0 + col;
  const bool act = c < C;
  const int64_t cc = act ? c : C - 1;   // inactive lanes read a valid column, discarded
  double yb[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int r = 4 * ks + kq;
    yb[ks] = r < R0 ? Y[(int64_t)r * C + cc] : 0.0;
  }
  const int chunk = (SL_LDS / stride) & ~15;   // rows per LDS chunk, a multiple of 16
  double acc = 0.0;
  for (int ic = 0; ic < I0; ic += chunk) {
    const int rows = min(chunk, I0 - ic);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * 4 * KS; e += blockDim.x) {
      const int i = e / (4 * KS), r = e - i * (4 * KS);
      a_s[i * stride + r] = r < R0 ? A0[(int64_t)(ic + i) * R0 + r] : 0.0;
    }
    __syncthreads();
    auto block = [&](int i0, const double* bv) {
      ks_f64x4 d = {0.0, 0.0, 0.0, 0.0};
      const int ia = i0 + col;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const double av = ia < rows ? a_s[ia * stride + 4 * ks + kq] : 0.0;
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(av, yb[ks], d, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + kq + 4 * v;
        if (i < rows) {
          const double e = d[v] - bv[v];
          acc = fma(e, e, acc);
        }
      }
    };
    auto load_b = [&](int i0, double* bv) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + kq + 4 * v;
        const int64_t off = (int64_t)(ic + min(i, rows - 1)) * C + cc;
        bv[v] = bdt == KR_F32 ? (double)((const float*)b)[off] : ((const double*)b)[off];
      }
    };
    int i0 = 0;
    for (; i0 + 32 <= rows; i0 += 32) {
      double b0[4], b1[4];
      load_b(i0, b0);
      load_b(i0 + 16, b1);
      block(i0, b0);
      block(i0 + 16, b1);
    }
    for (; i0 < rows; i0 += 16) {
      double b0[4];
      load_b(i0, b0);
      block(i0, b0);
    }
  }
  if (!act) acc = 0.0;
  for (int q = 0; q < nrhs; ++q) {
    const double t = block_sum((act && (int)(c % nrhs) == q) ? acc : 0.0, red);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.x * nrhs + q] = t;
  }
}

// Z[r][c] = sum_{i0} U0[i0][r] b[i0][c]
template <int RM>
__global__ void __launch_bounds__(256) k_stream_contract0(const double* __restrict__ U0, int I0, int R0,
                                                         const void* __restrict__ b, int bdt, int64_t C,
                                                         double* __restrict__ Z) {
  __shared__ double u_s[STREAM_ROWS * RM];
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = c < C;
  double z[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) z[r] = 0.0;
  for (int base = 0; base < I0; base += STREAM_ROWS) {
    const int rows = min(STREAM_ROWS, I0 - base);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * RM; e += blockDim.x) {
      const int i = e / RM, r = e % RM;
      u_s[e] = r < R0 ? U0[(int64_t)(base + i) * R0 + r] : 0.0;
    }
    __syncthreads();
    if (act) {
#pragma unroll 4
      for (int i = 0; i < rows; ++i) {
        const int64_t off = (int64_t)(base + i) * C + c;
        const double bv = bdt == KR_F32 ? (double)((const float*)b)[off] : ((const double*)b)[off];
#pragma unroll
        for (int r = 0; r < RM; ++r) z[r] = fma(u_s[i * RM + r], bv, z[r]);
      }
    }
  }
  if (act) {
#pragma unroll
    for (int r = 0; r < RM; ++r)
      if (r < R0) Z[(int64_t)r * C + c] = z[r];
  }
}

// out[q] = sum over the nparts block sums of partial[p * nrhs + q] + lambda * sum_r
// x[r][q]^2.  One workgroup per right-hand side; fixed summation order.
__global__ void __launch_bounds__(1024) k_finish_loss(const double* __restrict__ partial, int64_t nparts,
                                                     const double* __restrict__ x, int64_t Rtot, int nrhs,
                                                     double lambda, double* __restrict__ out) {
  __shared__ double red[16];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int64_t p0 = threadIdx.x; p0 < nparts; p0 += 8 * (int64_t)blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t p = p0 + u * (int64_t)blockDim.x;
      v[u] = p < nparts ? partial[p * nrhs + q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  double xx = 0.0;
  for (int64_t r = threadIdx.x; r < Rtot; r += blockDim.x) {
    const double v = x[r * nrhs + q];
    xx = fma(v, v, xx);
  }
  s = block_sum(s, red);
  xx = block_sum(xx, red);
  if (threadIdx.x == 0) out[q] = s + lambda * xx;
}

// U_n = A_n V_n diag(1/s) over the numerical rank (zero columns elsewhere); s = sqrt(lambda_k).
__global__ void __launch_bounds__(256) k_left_singular(const double* __restrict__ A, const double* __restrict__ V,
                                                      const double* __restrict__ ev, int I, int R,
                                                      double* __restrict__ U) {
  double lmax = 0.0;
  for (int k = 0; k < R; ++k) lmax = fmax(lmax, ev[k]);
  const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
  const double thr = eps_r * eps_r * lmax;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)I * R;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / R;
    const int k = (int)(e - i * R);
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = fma(A[i * R + r], V[r * R + k], acc);
    U[e] = ev[k] > thr ? acc / sqrt(ev[k]) : 0.0;
  }
}

// t[r][q] *= s_r / (s_r^2 + lambda) with s_r = prod_n sqrt(lambda_n[r_n]) over the
// numerical rank of every mode (zero otherwise).
__global__ void __launch_bounds__(256) k_exact_scale(ModeTables T, Geom g, double lambda, double* __restrict__ t) {
  const int64_t total = g.Rtot * g.nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / g.nrhs;
    double sig = 1.0;
    bool zero = false;
    for (int n = g.N - 1; n >= 0; --n) {
      const int rn = (int)(r % g.R[n]);
      r /= g.R[n];
      double lmax = 0.0;
      for (int k = 0; k < g.R[n]; ++k) lmax = fmax(lmax, T.evals[n][k]);
      const double eps_r = (double)max(g.I[n], g.R[n]) * 2.220446049250313e-16;
      const double lk = T.evals[n][rn];
      if (!(lk > eps_r * eps_r * lmax)) zero = true;
      sig *= sqrt(fmax(lk, 0.0));
    }
    const double den = sig * sig + lambda;
    t[e] = (zero || !(den > 0.0)) ? 0.0 : t[e] * (sig / den);
  }
}

template __global__ void k_stream_contract0<8>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<16>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<32>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<64>(const double*, int, int, const void*, int, int64_t, double*);

// ---------------------------------------------------------------------------
// Implicit responses b = K X_true + sigma E (E[i][q] the Philox Box-Muller normal
// of K's row i, see kron_regress.h): the loss and the exact minimiser need only
// s = K^T E (R x nrhs) and e2 = ||E||^2 per right-hand side, since with
// v = x - X_true
//   f(x)    = v^T (kron G) v - 2 sigma v^T s + sigma^2 e2 + lambda ||x||^2,
//   K^T b   = (kron G) X_true + sigma s,   x* = (kron G + lambda I)^+ K^T b,
// so one pass generates every E entry once.  k_noise_adjoint contracts the last
// two modes while generating: workgroup (p, q) covers the rows whose first N-2
// indices form prefix p, 16 rows of mode N-2 by 256 columns of mode N-1 at a time
// in LDS; the other modes follow as mode products.
// ---------------------------------------------------------------------------
struct NoiseArgs {
  const double* A1;   // factor of mode N-2 (M1 x R1)
  const double* A2;   // factor of mode N-1 (M2 x R2)
  int M1, M2, R1, R2;
  int nrhs;
  uint64_t seed, stream;
  double* Y;          // P x R1 x R2 x nrhs
  double* e2part;     // P x nrhs
};

#define NA_ROWS 16
#define NA_COLS 256
__global__ void __launch_bounds__(256) k_noise_adjoint(NoiseArgs a) {
  __shared__ double tile[NA_ROWS * NA_COLS];
  __shared__ double zt[NA_ROWS * 64];
  __shared__ double red[4];
  const int64_t p = blockIdx.x;
  const int q = blockIdx.y;
  const int M1 = a.M1, M2 = a.M2, R1 = a.R1, R2 = a.R2;
  const int nout = R1 * R2;
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  double e2 = 0.0;
  const uint64_t base = (uint64_t)p * (uint64_t)M1 * (uint64_t)M2;
  for (int i0 = 0; i0 < M1; i0 += NA_ROWS) {
    const int rows = min(NA_ROWS, M1 - i0);
    for (int e = threadIdx.x; e < rows * R2; e += blockDim.x) zt[e] = 0.0;
    for (int j0 = 0; j0 < M2; j0 += NA_COLS) {
      const int cols = min(NA_COLS, M2 - j0);
      __syncthreads();
      for (int e = threadIdx.x; e < rows * cols; e += blockDim.x) {
        const int ii = e / cols, jj = e - ii * cols;
        const uint64_t row = base + (uint64_t)(i0 + ii) * (uint64_t)M2 + (uint64_t)(j0 + jj);
        const u64x4 w = philox4x64_10(row, (uint64_t)q, 0ull, 0ull, a.seed, a.stream);
        const double u1 = (double)((w.v[0] >> 11) + 1ull) * 0x1p-53;
        const double u2 = (double)(w.v[1] >> 11) * 0x1p-53;
        const double v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        tile[ii * NA_COLS + jj] = v;
        e2 = fma(v, v, e2);
      }
      __syncthreads();
      // zt[ii][r2] += sum_jj tile[ii][jj] A2[j0 + jj][r2]
      for (int o = threadIdx.x; o < rows * R2; o += blockDim.x) {
        const int ii = o / R2, r2 = o - ii * R2;
        double z = zt[o];
        for (int jj = 0; jj < cols; ++jj) z = fma(tile[ii * NA_COLS + jj], a.A2[(int64_t)(j0 + jj) * R2 + r2], z);
        zt[o] = z;
      }
    }
    __syncthreads();
    // acc[r1][r2] += sum_ii A1[i0 + ii][r1] zt[ii][r2]
    int k = 0;
    for (int o = threadIdx.x; o < nout; o += blockDim.x, ++k) {
      const int r1 = o / R2, r2 = o - r1 * R2;
      double s = acc[k];
      for (int ii = 0; ii < rows; ++ii) s = fma(a.A1[(int64_t)(i0 + ii) * R1 + r1], zt[ii * R2 + r2], s);
      acc[k] = s;
    }
    __syncthreads();
  }
  int k = 0;
  for (int o = threadIdx.x; o < nout; o += blockDim.x, ++k) a.Y[(p * nout + o) * a.nrhs + q] = acc[k];
  const double t = block_sum(e2, red);
  if (threadIdx.x == 0) a.e2part[p * a.nrhs + q] = t;
}

// e2[q] = sum_p e2part[p][q] in prefix order; one workgroup per right-hand side.
__global__ void __launch_bounds__(256) k_noise_e2(const double* __restrict__ part, int64_t P, int nrhs,
                                                 double* __restrict__ e2) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int64_t p = threadIdx.x; p < P; p += blockDim.x) s += part[p * nrhs + q];
  s = block_sum(s, red);
  if (threadIdx.x == 0) e2[q] = s;
}

// out[e] = a[e] + c * b[e] (a may be NULL for 0)
__global__ void __launch_bounds__(256) k_axpy_into(const double* __restrict__ a, const double* __restrict__ b,
                                                  double c, int64_t n, double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (a ? a[e] : 0.0) + c * b[e];
}

// f[q] = v^T w - 2 sigma v^T s + sigma^2 e2[q] + lambda ||x||^2 with v = x - X_true
// and w = (kron G) v (one workgroup per right-hand side).
__global__ void __launch_bounds__(256) k_gen_loss_finish(const double* __restrict__ x, const double* __restrict__ X,
                                                        const double* __restrict__ w, const double* __restrict__ s,
                                                        const double* __restrict__ e2, int64_t Rtot, int nrhs,
                                                        double sigma, double lambda, double* __restrict__ out) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  double vw = 0.0, vs = 0.0, xx = 0.0;
  for (int64_t r = threadIdx.x; r < Rtot; r += blockDim.x) {
    const int64_t e = r * nrhs + q;
    const double v = x[e] - X[e];
    vw = fma(v, w[e], vw);
    vs = fma(v, s[e], vs);
    xx = fma(x[e], x[e], xx);
  }
  vw = block_sum(vw, red);
  vs = block_sum(vs, red);
  xx = block_sum(xx, red);
  if (threadIdx.x == 0) out[q] = vw - 2.0 * sigma * vs + sigma * sigma * e2[q] + lambda * xx;
}

// t <- t / (kron lambda + lambda_reg) in the eigenbasis, zero where a mode's
// eigenvalue is below its rank threshold (the pseudo-inverse of kron G + lambda I
// restricted like the exact path's).
__global__ void __launch_bounds__(256) k_gen_exact_scale(ModeTables T, Geom g, double lambda, double* __restrict__ t) {
  const int64_t total = g.Rtot * g.nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = e / g.nrhs;
    double prod = 1.0;
    bool zero = false;
    for (int n = g.N - 1; n >= 0; --n) {
      const int rn = (int)(r % g.R[n]);
      r /= g.R[n];
      double lmax = 0.0;
      for (int k = 0; k < g.R[n]; ++k) lmax = fmax(lmax, T.evals[n][k]);
      const double eps_r = (double)max(g.I[n], g.R[n]) * 2.220446049250313e-16;
      const double lk = T.evals[n][rn];
      if (!(lk > eps_r * eps_r * lmax)) zero = true;
      prod *= fmax(lk, 0.0);
    }
    const double den = prod + lambda;
    t[e] = (zero || !(den > 0.0)) ? 0.0 : t[e] / den;
  }
}

}  // namespace kr
