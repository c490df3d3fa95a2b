// Refined (mixed-precision) Richardson iteration of Algorithm 2.
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
// mat-vec theorem applies it by mode products).  The preconditioner kernels are
// in kr_precond.hip; this file holds the float copies of the adjoint's rows.
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

}  // namespace kr
