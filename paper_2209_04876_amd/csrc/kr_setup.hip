// Factor preprocessing of Algorithm 2 (lines computing the Gram matrix, its
// eigen-decomposition and the leverage scores, and the product-distribution
// data structure), one mode per workgroup:
//   k_promote   : factor -> FP64 workspace copy, finiteness check
//   k_gram      : G_n = A_n^T A_n (FP64, LDS row tiles, fixed summation order)
//   k_eig       : cyclic Jacobi eigen-decomposition G_n = V diag(lambda) V^T in one
//                 wave, plus G_n^{-1} = V diag(1/lambda) V^T
//   k_leverage  : l_i = sum_k (a_i . v_k)^2 / lambda_k over the numerical rank
//                 (definition of statistical leverage via the Gram
//                 eigen-decomposition), integer weights Q on the 2^32 grid and the
//                 inclusive CDF used by the sampler.
#include "kr_internal.h"

namespace kr {

#define KR_RMAX 64

__global__ void k_promote(const void* __restrict__ src, int dtype, double* __restrict__ dst,
                          int64_t n, int32_t* __restrict__ flags) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = dtype == KR_F32 ? (double)((const float*)src)[i] : ((const double*)src)[i];
    dst[i] = v;
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flags, KR_FLAG_NONFINITE);
}

// One workgroup (256 threads) per mode.  Thread t owns Gram entries t, t+256, ...
// (upper triangle mirrored) and sums over rows in increasing order.
__global__ void __launch_bounds__(256) k_gram(ModeTables T, Geom g, double* __restrict__ gram) {
  __shared__ double tile[64 * KR_RMAX];
  const int n = blockIdx.x;
  const int I = g.I[n], R = g.R[n];
  const double* A = T.A[n];
  double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  double acc[16];
  int npair = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int r0 = 0; r0 < I; r0 += 64) {
    const int rows = min(64, I - r0);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * R; e += blockDim.x) tile[e] = A[(size_t)r0 * R + e];
    __syncthreads();
    int k = 0;
    for (int pq = threadIdx.x; pq < R * R; pq += blockDim.x, ++k) {
      const int p = pq / R, q = pq % R;
      double s = acc[k];
      for (int i = 0; i < rows; ++i) s = fma(tile[i * R + p], tile[i * R + q], s);
      acc[k] = s;
    }
    npair = k;
  }
  int k = 0;
  for (int pq = threadIdx.x; pq < R * R && k < npair; pq += blockDim.x, ++k) G[pq] = acc[k];
}

// One wave per mode.  Cyclic-by-row Jacobi rotations on the symmetric Gram
// matrix held in LDS; lanes update the rows/columns touched by a rotation in
// parallel.  A rotation is skipped when |a_pq| is below rounding relative to
// sqrt(|a_pp a_qq|); sweeps stop when a sweep performs no rotation.
__global__ void __launch_bounds__(64) k_eig(ModeTables T, Geom g, const double* __restrict__ gram,
                                            int32_t* __restrict__ flags) {
  __shared__ double a[KR_RMAX * KR_RMAX];
  __shared__ double v[KR_RMAX * KR_RMAX];
  __shared__ int rotated;
  const int n = blockIdx.x;
  const int R = g.R[n], I = g.I[n];
  const int lane = threadIdx.x;
  const double* G = gram + (size_t)n * KR_RMAX * KR_RMAX;
  for (int e = lane; e < R * R; e += 64) {
    a[e] = G[e];
    v[e] = (e / R == e % R) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (lane == 0) rotated = 0;
    __syncthreads();
    for (int p = 0; p < R - 1; ++p) {
      for (int q = p + 1; q < R; ++q) {
        const double apq = a[p * R + q], app = a[p * R + p], aqq = a[q * R + q];
        const bool skip = fabs(apq) <= 1e-17 * sqrt(fabs(app * aqq)) || apq == 0.0;
        __syncthreads();
        if (skip) continue;
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = lane; k < R; k += 64) {
          if (k != p && k != q) {
            const double akp = a[k * R + p], akq = a[k * R + q];
            const double nkp = c * akp - s * akq, nkq = s * akp + c * akq;
            a[k * R + p] = nkp; a[p * R + k] = nkp;
            a[k * R + q] = nkq; a[q * R + k] = nkq;
          }
          const double vkp = v[k * R + p], vkq = v[k * R + q];
          v[k * R + p] = c * vkp - s * vkq;
          v[k * R + q] = s * vkp + c * vkq;
        }
        if (lane == 0) {
          a[p * R + p] = app - t * apq;
          a[q * R + q] = aqq + t * apq;
          a[p * R + q] = 0.0; a[q * R + p] = 0.0;
          rotated = 1;
        }
        __syncthreads();
      }
    }
    __syncthreads();
    if (!rotated) break;
  }
  __syncthreads();
  double* V = T.V[n];
  double* ev = T.evals[n];
  for (int e = lane; e < R * R; e += 64) V[e] = v[e];
  double lmax = 0.0;
  for (int k = 0; k < R; ++k) lmax = fmax(lmax, a[k * R + k]);
  const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
  const double thr = eps_r * eps_r * lmax;
  bool sing = false;
  for (int k = 0; k < R; ++k) sing |= !(a[k * R + k] > thr);
  for (int k = lane; k < R; k += 64) ev[k] = a[k * R + k];
  if (sing) {
    if (lane == 0) atomicOr(flags, KR_FLAG_SINGULAR);
  }
  // G^{-1} = V diag(1/lambda) V^T over the numerical rank (pseudo-inverse)
  double* Gi = T.Ginv[n];
  for (int e = lane; e < R * R; e += 64) {
    const int p = e / R, q = e % R;
    double s = 0.0;
    for (int k = 0; k < R; ++k) {
      const double lk = a[k * R + k];
      if (lk > thr) s += v[p * R + k] * v[q * R + k] / lk;
    }
    Gi[e] = s;
  }
}

// One workgroup (256 threads) per mode.
__global__ void __launch_bounds__(256) k_leverage(ModeTables T, Geom g, int32_t* __restrict__ flags) {
  __shared__ double vs[KR_RMAX * KR_RMAX];
  __shared__ double inv[KR_RMAX];
  __shared__ double red[8];
  __shared__ unsigned long long ured[4];
  __shared__ unsigned long long umax[4];
  __shared__ unsigned long long carry;
  __shared__ unsigned long long scan[256];
  const int n = blockIdx.x;
  const int I = g.I[n], R = g.R[n];
  const double* A = T.A[n];
  double* lev = T.lev[n];
  uint64_t* Q = T.Q[n];
  uint64_t* C = T.C[n];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) vs[e] = T.V[n][e];
  if (threadIdx.x < R) {
    double lmax = 0.0;
    for (int k = 0; k < R; ++k) lmax = fmax(lmax, T.evals[n][k]);
    const double eps_r = (double)max(I, R) * 2.220446049250313e-16;
    const double lk = T.evals[n][threadIdx.x];
    inv[threadIdx.x] = lk > eps_r * eps_r * lmax ? 1.0 / lk : 0.0;
  }
  __syncthreads();
  // leverage per row; thread-local partial sums in increasing row order
  double part = 0.0;
  for (int i = threadIdx.x; i < I; i += blockDim.x) {
    const double* ai = A + (size_t)i * R;
    double l = 0.0;
    bool zero = true;
    for (int k = 0; k < R; ++k) {
      double dot = 0.0;
      for (int r = 0; r < R; ++r) {
        const double x = ai[r];
        zero &= (x == 0.0);
        dot = fma(x, vs[r * R + k], dot);
      }
      l = fma(dot * dot, inv[k], l);
    }
    if (zero) l = 0.0;
    lev[i] = l;
    part += l;
  }
  const double S = block_sum(part, red);
  if (!(S > 0.0) || !isfinite(S)) {
    if (threadIdx.x == 0) atomicOr(flags, KR_FLAG_QUANT);
    return;
  }
  // Q_i = max(1, floor(2^32 l_i / S)) for l_i > 0; exact integer sum and argmax
  unsigned long long qsum = 0ull, best = 0ull;
  for (int i = threadIdx.x; i < I; i += blockDim.x) {
    const double l = lev[i];
    uint64_t q = 0;
    if (l > 0.0) {
      q = (uint64_t)floor((l / S) * 4294967296.0);
      if (q < 1) q = 1;
    }
    Q[i] = q;
    qsum += q;
    // pack (q, lowest index wins on ties) into a comparable key: q high, ~i low
    const unsigned long long key = ((unsigned long long)q << 24) | (unsigned long long)(0xFFFFFF - i);
    best = key > best ? key : best;
  }
  // reductions (integer: order-independent)
  {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) {
      qsum += __shfl_xor(qsum, o, 64);
      const unsigned long long ob = __shfl_xor(best, o, 64);
      best = ob > best ? ob : best;
    }
    if (lane == 0) { ured[w] = qsum; umax[w] = best; }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long s = 0, b = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { s += ured[k]; b = umax[k] > b ? umax[k] : b; }
      const int j = 0xFFFFFF - (int)(b & 0xFFFFFFull);
      const long long deficit = (long long)(1ull << 32) - (long long)s;
      const long long qj = (long long)Q[j] + deficit;
      if (qj < 1) atomicOr(flags, KR_FLAG_QUANT);
      else Q[j] = (uint64_t)qj;
      carry = 0ull;
    }
    __syncthreads();
  }
  // inclusive CDF, 256 entries per step with a running carry
  for (int base = 0; base < I; base += blockDim.x) {
    const int i = base + threadIdx.x;
    scan[threadIdx.x] = i < I ? Q[i] : 0ull;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const unsigned long long add = threadIdx.x >= (unsigned)o ? scan[threadIdx.x - o] : 0ull;
      __syncthreads();
      scan[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < I) C[i] = carry + scan[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) carry += scan[blockDim.x - 1];
    __syncthreads();
  }
}

}  // namespace kr
