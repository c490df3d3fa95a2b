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

#define STREAM_ROWS 64

// partial[c] = sum_{i0} ((sum_r A0[i0][r] Y[r][c]) - b[i0][c])^2, b of dtype bdt.
template <int RM>
__global__ void __launch_bounds__(256) k_stream_loss(const double* __restrict__ A0, int I0, int R0,
                                                    const double* __restrict__ Y, const void* __restrict__ b,
                                                    int bdt, int64_t C, double* __restrict__ partial) {
  __shared__ double a_s[STREAM_ROWS * RM];
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool act = c < C;
  double y[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) y[r] = (act && r < R0) ? Y[(int64_t)r * C + c] : 0.0;
  double acc = 0.0;
  for (int base = 0; base < I0; base += STREAM_ROWS) {
    const int rows = min(STREAM_ROWS, I0 - base);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * RM; e += blockDim.x) {
      const int i = e / RM, r = e % RM;
      a_s[e] = r < R0 ? A0[(int64_t)(base + i) * R0 + r] : 0.0;
    }
    __syncthreads();
    if (act) {
      if (bdt == KR_F32) {
        const float* bb = (const float*)b + (int64_t)base * C + c;
#pragma unroll 4
        for (int i = 0; i < rows; ++i) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < RM; ++r) v = fma(a_s[i * RM + r], y[r], v);
          const double d = v - (double)bb[(int64_t)i * C];
          acc = fma(d, d, acc);
        }
      } else {
        const double* bb = (const double*)b + (int64_t)base * C + c;
#pragma unroll 4
        for (int i = 0; i < rows; ++i) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < RM; ++r) v = fma(a_s[i * RM + r], y[r], v);
          const double d = v - bb[(int64_t)i * C];
          acc = fma(d, d, acc);
        }
      }
    }
  }
  if (act) partial[c] = acc;
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

// out[q] = sum over c = q (mod nrhs) of partial[c] + lambda * sum_r x[r][q]^2.
// One workgroup per right-hand side; fixed summation order.
__global__ void __launch_bounds__(1024) k_finish_loss(const double* __restrict__ partial, int64_t C,
                                                     const double* __restrict__ x, int64_t Rtot, int nrhs,
                                                     double lambda, double* __restrict__ out) {
  __shared__ double red[16];
  const int q = blockIdx.x;
  double s = 0.0;
  for (int64_t c = (int64_t)threadIdx.x * nrhs + q; c < C; c += (int64_t)blockDim.x * nrhs) s += partial[c];
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

template __global__ void k_stream_loss<8>(const double*, int, int, const double*, const void*, int, int64_t, double*);
template __global__ void k_stream_loss<16>(const double*, int, int, const double*, const void*, int, int64_t, double*);
template __global__ void k_stream_loss<32>(const double*, int, int, const double*, const void*, int, int64_t, double*);
template __global__ void k_stream_loss<64>(const double*, int, int, const double*, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<8>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<16>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<32>(const double*, int, int, const void*, int, int64_t, double*);
template __global__ void k_stream_contract0<64>(const double*, int, int, const void*, int, int64_t, double*);

}  // namespace kr
