// Internal declarations shared by the HIP translation units of the library.
// Everything here is gfx950 (CDNA4, wave64) code; no other target is built.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kron_regress.h"

#define KR_WAVE 64
#define KR_MAXN KR_MAX_MODES

namespace kr {

// ---------------------------------------------------------------------------
// Problem geometry passed by value to kernels.
// Modes are numbered 0..N-1 (mode n of the paper is n+1).  Level k of the
// sample tree (k = 0..N) holds the distinct prefixes (i_0..i_{k-1}) of the
// sampled rows; level 0 is a single root, level N the distinct rows.
// rsuf[k] = R_k * ... * R_{N-1} is the size of a level-k intermediate.
// ---------------------------------------------------------------------------
struct Geom {
  int N;
  int nrhs;
  int I[KR_MAXN];
  int R[KR_MAXN];
  int64_t rsuf[KR_MAXN + 1];
  int shift[KR_MAXN];   // bit offset of mode n inside the packed sort key
  int bits[KR_MAXN];    // bits of mode n (ceil(log2 I_n), at least 1)
  int lshift[KR_MAXN + 1];  // key >> lshift[k] is the level-k prefix (lshift[N] = 0)
  int keybits;
  int64_t Rtot;
  int64_t Itot;
  int64_t m;
  int seg_root;         // 1: mode 0 indexes independent segments (no factor); the
                        //    level-1 node of segment i reads its own iterate row i
  int orig[KR_MAXN];    // the caller's mode of tree mode n (identity unless the
  int inv[KR_MAXN];     //    modes were reordered); inv is its inverse
  int approx;           // 1: approximate leverage (spectral approximation + JL)
  int lev_r;            //    rows of its Johnson-Lindenstrauss projection
  int lev_k[KR_MAXN];   //    rows of each spectral approximation A~
  double lev_eps;       //    the eps of the scores' constants (Lemma fast-ls-comp)
};

// Per-mode results of the setup kernel.
struct ModeTables {
  const double* A[KR_MAXN];     // FP64 factor copies, row-major I_n x R_n
  double* V[KR_MAXN];           // eigenvectors of G_n (R_n x R_n, column k = vector k)
  double* evals[KR_MAXN];       // eigenvalues of G_n (R_n)
  double* Ginv[KR_MAXN];        // G_n^{-1} (R_n x R_n) when G_n is non-singular
  double* lev[KR_MAXN];         // leverage scores (I_n)
  uint64_t* Q[KR_MAXN];         // integer weights on the 2^32 grid (I_n)
  uint64_t* C[KR_MAXN];         // inclusive CDF of Q (I_n)
};

// The sample tree built from the sorted keys.  For level k = 1..N:
//   idx[k][s]    mode-(k-1) index of node s
//   parent[k][s] level-(k-1) node containing s (root = 0 for k = 1)
//   fchild[k][s] first level-(k+1) child of s, with fchild[k][S_k] = S_{k+1}
//                (k = 0..N-1; fchild[0] = {0, S_1})
//   cnt[k]       S_k (device side; cnt[0] = 1)
//   arow[k]      the factor row a_{k-1}[i_{k-1}(s)] of every level-k node, gathered
//                once so the iteration reads node data contiguously
// Level N nodes are the distinct rows; rstart[j] is the first sorted sample of
// row j and rstart[D] = m.
struct Tree {
  int32_t* idx[KR_MAXN + 1];
  double* arow[KR_MAXN + 1];    // arow[k][s][r] = A_{k-1}[idx[k][s]][r], contiguous per node
  float* arow32[KR_MAXN + 1];   // float copies of arow[1..N-1] for the float32 adjoint (refined modes)
  int32_t* parent[KR_MAXN + 1];
  int32_t* fchild[KR_MAXN + 1];
  int32_t* rstart;
  uint64_t* rkey;
  int64_t* cnt;                 // KR_MAXN + 1 entries (device)
  int64_t ncnt[KR_MAXN + 1];    // the same counts, copied to the host once the tree is
                                // built and passed by value to the iteration kernels
};

// Chunks of the level-2 nodes for the fused pass of three-mode problems: chunk c
// covers the level-2 nodes [beg[c], beg[c+1]), all children of the level-1 node
// par[c] (a node's children are split into runs of at most `ch` nodes), and
// arow[c] / arow32[c] hold that node's factor row a_0[i_0(par[c])].  Built on the
// device once the tree is; *count is the number of chunks (written even when it
// exceeds cap, in which case the table is not).
struct Chunks {
  int32_t* beg;
  int32_t* par;
  double* arow;
  float* arow32;
  int64_t* count;
  int cap;
  int ch;
};

// Solver state shared between the iteration kernels (device memory).
struct IterState {
  int32_t iters;        // iterations completed
  int32_t all_done;     // 1 when every RHS has converged or the solve stopped
  int32_t diverged;     // 1 when a non-finite or exploding update was seen
  int32_t pad;
  int32_t done[64];     // per RHS
  int32_t it_rhs[64];   // iterations at which each RHS stopped
  double dnorm0[64];    // ||d|| of the first iteration, per RHS
  double rel[64];       // eta ||d|| / ||x|| of the last iteration, per RHS
  double rel_first[64]; // the same after the first iteration (rate estimate for polling)
};

#define KR_MAX_RHS 64

// Status bits raised by kernels (device int32 at ws.flags).
enum : int32_t {
  KR_FLAG_NONFINITE = 1,
  KR_FLAG_SINGULAR = 2,
  KR_FLAG_QUANT = 4,
  KR_FLAG_CORE = 8,     // the core unfolding G_(n) G_(n)^T (or the Woodbury C) is singular
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): two 64x64->128 products per round,
// Weyl key schedule.  Written from the published definition.
// ---------------------------------------------------------------------------
struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                               uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  u64x4 o; o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, KR_WAVE);
  return v;
}

// Block-wide sum with a fixed reduction order (deterministic).  `scratch` holds
// at least blockDim.x / 64 doubles.  Result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  __syncthreads();
  return t;
}

}  // namespace kr
