// Batched Algorithm 2: many independent ridge problems of uneven N, I_n, R_n and
// right-hand sides, iterated by two persistent kernels.
//
// Each problem's setup and sketch (Gram, leverage, sampling, sort, sample tree,
// gathered rows) is enqueued with the single-problem kernels.  The Richardson
// iterations then run in two persistent launches:
//
//   queue  k_batched_queue: workgroups take the next small problem from a queue
//          (largest first) and run its whole iteration -- forward levels, rows,
//          adjoint levels, root adjoint, preconditioner and update -- with
//          workgroup barriers only, until the stopping rule holds or max_iter;
//   team   k_batched_team: all workgroups iterate all large problems together.
//          Each problem's iteration is a list of stages (forward levels, fused
//          rows, adjoint levels, root, one stage per preconditioner mode product,
//          update); at every step each active problem runs its next stage, and
//          the work items of all those stages form one index space that the team
//          strides over (workgroup w takes item blocks w, w + teams, ...: every
//          workgroup samples every problem, which balances stages of very
//          different cost).  A team-wide barrier separates steps.  Problems
//          with short stage lists simply iterate more often; a problem leaves
//          the index space when its stopping rule holds.
//
// Every output of a stage has one owning thread (or lane group) with a fixed
// summation order, and the update's norms are reduced in chunk order, so results
// do not depend on the number of workgroups or on which workgroup runs what.
#include "kr_internal.h"

namespace kr {

#define BT_THREADS 512   // threads per workgroup of the queue kernel
#define TM_THREADS 256   // threads per workgroup of the team kernel

// Everything one problem's iteration needs (device array, one entry per problem).
struct BatchDesc {
  Geom g;
  ModeTables T;
  Tree tr;
  double* P[KR_MAXN + 1];   // P[0] = iterate x
  double* Q[KR_MAXN + 1];   // Q[0] = gradient
  double* Omega;
  double* bD;
  double* t0;
  double* t1;
  double* dinv;
  IterState* st;
  const int32_t* flags;     // setup flags of the problem
  double lambda;
  int32_t use_ginv;
  int32_t pad;
};

// Forward level k of one problem: P_k[s][cq] = <a_{k-1}[i(s)], P_{k-1}[parent(s)][:, cq]>.
__device__ void bt_forward(const BatchDesc& d, int k, unsigned S) {
  const Geom& g = d.g;
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs), Wp = (unsigned)(g.rsuf[k - 1] * g.nrhs);
  const int Rk = g.R[k - 1];
  const double* __restrict__ Pp = d.P[k - 1];
  double* __restrict__ Po = d.P[k];
  for (unsigned e = threadIdx.x; e < S * W; e += blockDim.x) {
    const unsigned s = e / W, cq = e - s * W;
    const unsigned p = k == 1 ? 0u : (unsigned)d.tr.parent[k][s];
    Po[e] = dot_batched(d.tr.arow[k] + (size_t)s * Rk, Pp + (size_t)p * Wp + cq, W, Rk);
  }
}

// Last forward level, rows and last adjoint level of one problem (R_{N-1} <= 16):
// a group of 16 lanes per (level-(N-1) node, rhs), as in k_rows_adj.
__device__ void bt_rows(const BatchDesc& d, unsigned Sp) {
  const Geom& g = d.g;
  const int N = g.N, nrhs = g.nrhs;
  const int R = g.R[N - 1];
  const double* __restrict__ AL = d.tr.arow[N];
  const double* __restrict__ Pprev = d.P[N >= 2 ? N - 2 : 0];
  double* __restrict__ Qout = d.Q[N - 1];
  const unsigned lane = threadIdx.x & 15;
  const bool ln = (int)lane < R;
  const unsigned ntask = Sp * (unsigned)nrhs, gpb = blockDim.x >> 4;
  for (unsigned t0 = 0; t0 < ntask; t0 += gpb) {
    const unsigned task = t0 + (threadIdx.x >> 4);
    const bool active = task < ntask;
    const unsigned p = active ? task / nrhs : 0u;
    const int q = active ? (int)(task - p * nrhs) : 0;
    double pv = 0.0;
    if (active && ln) {
      if (N == 1) {
        pv = Pprev[(int64_t)lane * nrhs + q];
      } else {
        const int Rp = g.R[N - 2];
        const int64_t par = N >= 3 ? d.tr.parent[N - 1][p] : 0;
        pv = dot_batched(d.tr.arow[N - 1] + (size_t)p * Rp,
                         Pprev + par * (int64_t)Rp * R * nrhs + (int64_t)lane * nrhs + q, (int64_t)R * nrhs, Rp);
      }
    }
    double acc = 0.0;
    const int j0 = active ? d.tr.fchild[N - 1][p] : 0;
    const int j1 = active ? d.tr.fchild[N - 1][p + 1] : 0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      double av[4], y[4], om[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = ln ? AL[(int64_t)(j + u) * R + lane] : 0.0;
        om[u] = d.Omega[j + u];
        bb[u] = d.bD[(int64_t)(j + u) * nrhs + q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = av[u] * pv;
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) y[u] += __shfl_xor(y[u], o, 16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(om[u] * (y[u] - bb[u]), av[u], acc);
    }
    for (; j < j1; ++j) {
      const double a = ln ? AL[(int64_t)j * R + lane] : 0.0;
      double y = a * pv;
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) y += __shfl_xor(y, o, 16);
      acc = fma(d.Omega[j] * (y - d.bD[(int64_t)j * nrhs + q]), a, acc);
    }
    if (active && ln) Qout[((int64_t)p * R + lane) * nrhs + q] = acc;
  }
}

// Adjoint level k: Q_{k-1}[p][r][cq] = sum_{s child of p} a_{k-1}[i(s)][r] Q_k[s][cq].
__device__ void bt_adjoint(const BatchDesc& d, int k, unsigned Sp) {
  const Geom& g = d.g;
  const unsigned W = (unsigned)(g.rsuf[k] * g.nrhs), Wp = (unsigned)(g.rsuf[k - 1] * g.nrhs);
  const int Rk = g.R[k - 1];
  const double* __restrict__ arow = d.tr.arow[k];
  const double* __restrict__ Qk = d.Q[k];
  double* __restrict__ Qo = d.Q[k - 1];
  for (unsigned e = threadIdx.x; e < Sp * Wp; e += blockDim.x) {
    const unsigned p = e / Wp, rem = e - p * Wp;
    const unsigned r = rem / W, cq = rem - r * W;
    const int s0 = d.tr.fchild[k - 1][p], s1 = d.tr.fchild[k - 1][p + 1];
    double acc = 0.0;
    int s = s0;
    for (; s + 4 <= s1; s += 4) {
      double av[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = arow[(size_t)(s + u) * Rk + r];
        qv[u] = Qk[(size_t)(s + u) * W + cq];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
    }
    for (; s < s1; ++s) acc = fma(arow[(size_t)s * Rk + r], Qk[(size_t)s * W + cq], acc);
    Qo[e] = acc;
  }
}

// Root adjoint: g[r0][c] = sum_{s < S_1} a_0[i(s)][r0] Q_1[s][c].
__device__ void bt_root(const BatchDesc& d, unsigned S1) {
  const Geom& g = d.g;
  const unsigned W1 = (unsigned)(g.rsuf[1] * g.nrhs);
  const int R0 = g.R[0];
  const unsigned total = (unsigned)(g.Rtot * g.nrhs);
  const double* __restrict__ a0 = d.tr.arow[1];
  const double* __restrict__ Q1 = d.Q[1];
  double* __restrict__ grad = d.Q[0];
  for (unsigned e = threadIdx.x; e < total; e += blockDim.x) {
    const unsigned r0 = e / W1, c = e - r0 * W1;
    double acc = 0.0;
    unsigned s = 0;
    for (; s + 4 <= S1; s += 4) {
      double av[4], qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = a0[(size_t)(s + u) * R0 + r0];
        qv[u] = Q1[(size_t)(s + u) * W1 + c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
    }
    for (; s < S1; ++s) acc = fma(a0[(size_t)s * R0 + r0], Q1[(size_t)s * W1 + c], acc);
    grad[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// Team stages (large problems)
// ---------------------------------------------------------------------------
#define LS_MAXST 24      // stages per iteration: N forward/adjoint + 2N mode products + 2
#define LS_MAXP 1024     // large problems per launch
#define LS_MAXRHS 64

enum : int32_t { LS_FWD = 0, LS_ROWS = 1, LS_ROWS2 = 2, LS_ADJ = 3, LS_ROOT = 4, LS_MODE = 5, LS_UPD = 6 };

struct LStage {
  int32_t kind;     // LS_*
  int32_t k;        // level (FWD, ADJ) or mode (MODE)
  int32_t trans;    // MODE: multiply by M^T
  int32_t io;       // MODE: bit 0 input is h = g + lambda x, bit 1 scale the output by dinv,
                    //       bit 2 output to t1 (else t0), bit 3 input from t1 (else t0)
  const double* M;  // MODE: the R_k x R_k matrix
};

struct LExtra {
  LStage st[LS_MAXST];
  int32_t nst;
  int32_t nchunk;       // update chunks of TM_THREADS rows
  int32_t dfin;         // buffer holding M^+ h after the last mode product: 0 = t0, 1 = t1
  int32_t pad;
  double* part;         // update partial norms: nchunk x nrhs x 2
  int32_t* ticket;      // update arrivals
};

// Work items (threads, a multiple of TM_THREADS) of stage st of problem d.
__device__ int64_t ls_threads(const BatchDesc& d, const LExtra& L, const LStage& st) {
  const Geom& g = d.g;
  int64_t n = 0;
  switch (st.kind) {
    case LS_FWD: n = (d.tr.cnt[st.k] + 15) / 16 * ((g.rsuf[st.k] * g.nrhs + 15) / 16) * 64; break;
    case LS_ROWS: n = (g.N >= 2 ? d.tr.cnt[g.N - 1] : 1) * g.nrhs * 16; break;
    case LS_ROWS2: n = d.tr.cnt[g.N - 2] * 64; break;
    case LS_ADJ: n = d.tr.cnt[st.k - 1] * ((g.rsuf[st.k] * g.nrhs + 15) / 16) * 64; break;
    case LS_ROOT: n = ((g.rsuf[1] * g.nrhs + 15) / 16) * 64; break;
    case LS_MODE: n = ((g.Rtot * g.nrhs / g.R[st.k] + 15) / 16) * 64; break;
    case LS_UPD: n = (int64_t)L.nchunk * TM_THREADS; break;
  }
  return (n + TM_THREADS - 1) / TM_THREADS * TM_THREADS;
}

// Forward level k on v_mfma_f64_16x16x4, one wave per tile of 16 consecutive
// level-k nodes x 16 columns cq: P_k[s][cq] = sum_r a_k[s][r] P_{k-1}[parent(s)][r][cq]
// is, per parent, a (children x R_k) (R_k x W) product.  A tile whose 16 nodes
// have one parent (nodes are grouped by parent) uses the matrix cores; a tile
// that spans parents falls back to per-lane dot products.
__device__ __forceinline__ void ls_forward(const BatchDesc& d, int k, int64_t v) {
  const Geom& g = d.g;
  const int64_t W = g.rsuf[k] * g.nrhs, Wp = g.rsuf[k - 1] * g.nrhs;
  const int64_t S = d.tr.cnt[k];
  const int64_t nct = (W + 15) / 16;
  const int64_t tile = v >> 6;
  const int lane = (int)(v & 63);
  if (tile >= ((S + 15) / 16) * nct) return;   // uniform over the wave
  const int64_t st = tile / nct;
  const int64_t s0 = st * 16, c0 = (tile - st * nct) * 16;
  const int Rk = g.R[k - 1];
  const int col = lane & 15, kq = lane >> 4;
  const int64_t slast = s0 + 15 < S ? s0 + 15 : S - 1;
  const int64_t p0 = k == 1 ? 0 : d.tr.parent[k][s0];
  const int64_t p1 = k == 1 ? 0 : d.tr.parent[k][slast];
  const double* __restrict__ arow = d.tr.arow[k];
  const double* __restrict__ Pp = d.P[k - 1];
  double* __restrict__ Po = d.P[k];
  const int64_t cq = c0 + col;
  if (p0 == p1) {
    double A[4], B[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = 4 * ks + kq;
      const int64_t s = s0 + col;
      A[ks] = (s < S && kk < Rk) ? arow[s * Rk + kk] : 0.0;
      B[ks] = (kk < Rk && cq < W) ? Pp[p0 * Wp + (int64_t)kk * W + cq] : 0.0;
    }
    pc_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[ks], B[ks], acc, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t s = s0 + kq + 4 * u;
      if (s < S && cq < W) Po[s * W + cq] = acc[u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t s = s0 + kq + 4 * u;
      if (s < S && cq < W) {
        const int64_t p = d.tr.parent[k][s];
        Po[s * W + cq] = dot_batched(arow + s * Rk, Pp + p * Wp + cq, W, Rk);
      }
    }
  }
}

// Adjoint level k (and the root, k = 1) on v_mfma_f64_16x16x4, one wave per
// (level-(k-1) node p, 16 columns cq): Q_{k-1}[p][r][cq] = sum over the children
// s of p of a_k[s][r] Q_k[s][cq], an (R_k x children) (children x W) product
// accumulated four children per step.  Rows r >= R_k and columns cq >= W are
// zero padding.
__device__ __forceinline__ void ls_adjoint(const BatchDesc& d, int k, int64_t v) {
  const Geom& g = d.g;
  const int64_t W = g.rsuf[k] * g.nrhs, Wp = g.rsuf[k - 1] * g.nrhs;
  const int64_t Sp = k == 1 ? 1 : d.tr.cnt[k - 1];
  const int64_t nct = (W + 15) / 16;
  const int64_t tile = v >> 6;
  const int lane = (int)(v & 63);
  if (tile >= Sp * nct) return;   // uniform over the wave
  const int64_t p = tile / nct;
  const int64_t c0 = (tile - p * nct) * 16;
  const int Rk = g.R[k - 1];
  const int col = lane & 15, kq = lane >> 4;
  const int64_t s0 = k == 1 ? 0 : d.tr.fchild[k - 1][p];
  const int64_t s1 = k == 1 ? d.tr.cnt[1] : d.tr.fchild[k - 1][p + 1];
  const double* __restrict__ arow = d.tr.arow[k];
  const double* __restrict__ Qk = d.Q[k];
  const int64_t cq = c0 + col;
  const bool rok = col < Rk, cok = cq < W;
  pc_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  // children sb + kq (lane group kq) per step; the trip counts are uniform
  int64_t sb = s0;
  for (; sb + 8 <= s1; sb += 8) {   // two steps per trip, loads issued together
    const int64_t sa = sb + kq, sc = sb + 4 + kq;
    const double a0 = rok ? arow[sa * Rk + col] : 0.0;
    const double b0 = cok ? Qk[sa * W + cq] : 0.0;
    const double a1 = rok ? arow[sc * Rk + col] : 0.0;
    const double b1 = cok ? Qk[sc * W + cq] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
  }
  for (; sb < s1; sb += 4) {
    const int64_t sl = sb + kq;
    const double a = (sl < s1 && rok) ? arow[sl * Rk + col] : 0.0;
    const double b = (sl < s1 && cok) ? Qk[sl * W + cq] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  double* __restrict__ Qo = d.Q[k - 1];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = kq + 4 * u;
    if (r < Rk && cok) Qo[p * Wp + (int64_t)r * W + cq] = acc[u];
  }
}

// Residual sum of one level-(N-1) node's rows for a 16-lane group: returns
// sum_j a_N[j][lane] Omega_j (<a_N[j], pv> - b_j[q]) over rows j0..j1.
__device__ __forceinline__ double ls_rows_of(const BatchDesc& d, int j0, int j1, double pv, int q, unsigned lane,
                                             bool ln) {
  const Geom& g = d.g;
  const int R = g.R[g.N - 1], nrhs = g.nrhs;
  const double* __restrict__ AL = d.tr.arow[g.N];
  double acc = 0.0;
  int j = j0;
  for (; j + 4 <= j1; j += 4) {
    double av[4], y[4], om[4], bb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = ln ? AL[(int64_t)(j + u) * R + lane] : 0.0;
      om[u] = d.Omega[j + u];
      bb[u] = d.bD[(int64_t)(j + u) * nrhs + q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) y[u] = av[u] * pv;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] += __shfl_xor(y[u], o, 16);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(om[u] * (y[u] - bb[u]), av[u], acc);
  }
  for (; j < j1; ++j) {
    const double a = ln ? AL[(int64_t)j * R + lane] : 0.0;
    double y = a * pv;
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) y += __shfl_xor(y, o, 16);
    acc = fma(d.Omega[j] * (y - d.bD[(int64_t)j * nrhs + q]), a, acc);
  }
  return acc;
}

// Rows stage for N <= 2: a 16-lane group per (level-(N-1) node, rhs) forms the
// node's last forward value, its rows' residuals and Q_{N-1}[node].
__device__ __forceinline__ void ls_rows(const BatchDesc& d, int64_t v) {
  const Geom& g = d.g;
  const int N = g.N, nrhs = g.nrhs, R = g.R[N - 1];
  const int64_t task = v >> 4;
  const unsigned lane = (unsigned)v & 15u;
  const int64_t S = N >= 2 ? d.tr.cnt[N - 1] : 1;
  if (task >= S * nrhs) return;   // uniform over the group
  const int64_t p = task / nrhs;
  const int q = (int)(task - p * nrhs);
  const bool ln = (int)lane < R;
  double pv = 0.0;
  if (ln) {
    if (N == 1) {
      pv = d.P[0][(int64_t)lane * nrhs + q];
    } else {
      const int Rp = g.R[N - 2];
      pv = dot_batched(d.tr.arow[N - 1] + p * Rp, d.P[0] + (int64_t)lane * nrhs + q, (int64_t)R * nrhs, Rp);
    }
  }
  const int j0 = N >= 2 ? d.tr.fchild[N - 1][p] : 0;
  const int j1 = N >= 2 ? d.tr.fchild[N - 1][p + 1] : (int)d.tr.cnt[N];
  const double acc = ls_rows_of(d, j0, j1, pv, q, lane, ln);
  if (ln) d.Q[N - 1][(p * R + lane) * nrhs + q] = acc;
}

#define LS_FACT 4096   // LDS entries per staged factor (I_n x R_n <= 4096)

// Stage the factors of modes N-2 and N-1 of problem i into LDS unless they are
// there already (the tag holds the problem whose factors are staged, -1 none).
// Called by the whole workgroup; returns whether they are staged.
__device__ bool ls_stage_factors(const BatchDesc& d, int i, double* fa, int* tag) {
  const Geom& g = d.g;
  const int N = g.N;
  const int nP = g.I[N - 2] * g.R[N - 2], nL = g.I[N - 1] * g.R[N - 1];
  if (nP > LS_FACT || nL > LS_FACT) return false;
  if (*tag == i) return true;
  __syncthreads();   // every thread is done with the previous factors
  const double* __restrict__ AP = d.T.A[N - 2];
  const double* __restrict__ AL = d.T.A[N - 1];
  for (int e = threadIdx.x; e < nP; e += blockDim.x) fa[e] = AP[e];
  for (int e = threadIdx.x; e < nL; e += blockDim.x) fa[LS_FACT + e] = AL[e];
  if (threadIdx.x == 0) *tag = i;
  __syncthreads();   // factors and tag visible to every thread
  return true;
}

// The rows j0..j1 of one level-(N-2) subtree for right-hand sides q and, when
// two, q + 1, one wave (see ls_rows2 for the contraction).  B0, B1 hold the B
// operands of M = AV P in tile layout; the adjoints accumulate into acc0, acc1
// (Q[r' = gq + 4 v][c]).  The two right-hand sides share each block's keys,
// weights and factor-row gathers.  Row data streams in 64-row chunks with the
// next chunk in flight; AP and AL are the mode-(N-2) and last-mode factors (LDS
// or global).
typedef const __attribute__((address_space(1))) double* ls_gd;     // global
typedef const __attribute__((address_space(1))) uint64_t* ls_gu;   // global
typedef const __attribute__((address_space(3))) double* ls_ld;     // LDS

// FP is ls_ld (factors staged in LDS) or ls_gd: a pointer of one address space,
// so that the gathers compile to ds_read or global_load (a generic pointer would
// make them flat loads, whose waits also drain the streamed rows in flight).
template <typename FP>
__device__ __forceinline__ void ls_subtree_rows(const BatchDesc& d, int j0, int j1, int q, bool two,
                                                const double* B0, const double* B1, FP AP, FP AL,
                                                int lane, pc_f64x4& acc0, pc_f64x4& acc1) {
  const Geom& g = d.g;
  const int N = g.N, nrhs = g.nrhs;
  const int RL = g.R[N - 1], RP = g.R[N - 2];
  const int c = lane & 15, gq = lane >> 4;
  const int shP = g.shift[N - 2], shL = g.shift[N - 1];
  const uint64_t mP = (1ull << g.bits[N - 2]) - 1ull, mL = (1ull << g.bits[N - 1]) - 1ull;
  const ls_gu keys = (ls_gu)d.tr.rkey;
  const ls_gd Om = (ls_gd)d.Omega;
  const ls_gd bD = (ls_gd)d.bD;
  auto load_chunk = [&](int jc, uint64_t& k, double& om, double& b0, double& b1) {
    const int j = jc + lane;
    const bool ok = j < j1;
    k = ok ? keys[j] : 0ull;
    om = ok ? Om[j] : 0.0;
    b0 = ok ? bD[(int64_t)j * nrhs + q] : 0.0;
    b1 = (ok && two) ? bD[(int64_t)j * nrhs + q + 1] : 0.0;
  };
  uint64_t kc = 0;
  double oc = 0.0, bc0 = 0.0, bc1 = 0.0;
  if (j0 < j1) load_chunk(j0, kc, oc, bc0, bc1);
  for (int jc = j0; jc < j1; jc += 64) {
    uint64_t kn = 0;
    double on = 0.0, bn0 = 0.0, bn1 = 0.0;
    if (jc + 64 < j1) load_chunk(jc + 64, kn, on, bn0, bn1);
    const int nblk = (j1 - jc) >= 64 ? 4 : (j1 - jc + 15) / 16;
    for (int ub = 0; ub < nblk; ++ub) {
      const int jb = jc + 16 * ub;
      const uint64_t ka = __shfl(kc, 16 * ub + c, 64);
      const bool va = jb + c < j1;
      const int iPa = (int)((ka >> shP) & mP);
      double Af[4];
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int r1 = 4 * ks + gq;
        Af[ks] = (va && r1 < RP) ? AP[iPa * RP + r1] : 0.0;
      }
      pc_f64x4 M0 = {0.0, 0.0, 0.0, 0.0}, M1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        M0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Af[ks], B0[ks], M0, 0, 0, 0);
        if (two) M1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Af[ks], B1[ks], M1, 0, 0, 0);
      }
      double an[4], Aa[4], om[4], y0[4], y1[4], W0[4], W1[4], b0[4], b1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int src = 16 * ub + gq + 4 * u;
        const uint64_t kd = __shfl(kc, src, 64);
        om[u] = __shfl(oc, src, 64);
        b0[u] = __shfl(bc0, src, 64);
        b1[u] = __shfl(bc1, src, 64);
        const bool vd = jb + gq + 4 * u < j1;
        const int iPd = (int)((kd >> shP) & mP), iLd = (int)((kd >> shL) & mL);
        an[u] = (vd && c < RL) ? AL[iLd * RL + c] : 0.0;
        Aa[u] = (vd && c < RP) ? AP[iPd * RP + c] : 0.0;
        if (!vd) om[u] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        y0[u] = an[u] * M0[u];
        y1[u] = an[u] * M1[u];
      }
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          y0[u] += __shfl_xor(y0[u], o, 16);
          y1[u] += __shfl_xor(y1[u], o, 16);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        W0[u] = an[u] * (om[u] * (y0[u] - b0[u]));
        W1[u] = an[u] * (om[u] * (y1[u] - b1[u]));
      }
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Aa[ks], W0[ks], acc0, 0, 0, 0);
        if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Aa[ks], W1[ks], acc1, 0, 0, 0);
      }
    }
    kc = kn;
    oc = on;
    bc0 = bn0;
    bc1 = bn1;
  }
}

// Fused last two levels for N >= 3, one wave per level-(N-2) node p (all
// right-hand sides in turn), on v_mfma_f64_16x16x4.  The rows j of p's subtree
// are contiguous; per block of 16 rows, with AV the rows' mode-(N-2) factor rows
// (16 x R_{N-1}), AN their last-mode factor rows (16 x R_N) and
// P = P_{N-2}[p][:, :, q] (R_{N-1} x R_N):
//   M = AV P                      (the rows' level-(N-1) values, one MFMA chain)
//   y_j = sum_r AN[j][r] M[j][r]  (k_j x, a 16-lane reduction)
//   u_j = Omega_j (y_j - b_j)
//   Q += AV^T diag(u) AN          (the adjoint of both levels, one MFMA chain)
// and Q is Q_{N-2}[p][:, :, q].  Neither level-(N-1) product is formed.  Lane
// l = 16 g + c: c indexes the tile's columns, g its row quarter.  Right-hand
// sides go in pairs (ls_subtree_rows): row data (keys, weights, responses)
// streams in chunks of 64 rows, one row per lane, and reaches the tile layouts
// by shuffles; the next chunk is loaded while the current one is processed.
// The factor rows come from LDS (fa) when the workgroup has staged them, else
// from global memory (fa = nullptr).
__device__ __forceinline__ void ls_rows2(const BatchDesc& d, int64_t v, const double* fa) {
  const Geom& g = d.g;
  const int N = g.N, nrhs = g.nrhs;
  const int RL = g.R[N - 1], RP = g.R[N - 2];
  const int64_t p = v >> 6;
  const int lane = (int)(v & 63);
  if (p >= d.tr.cnt[N - 2]) return;   // uniform over the wave
  const int c = lane & 15, gq = lane >> 4;
  const int64_t pb = p * (int64_t)RP * RL * nrhs;
  const double* __restrict__ Pn2 = d.P[N - 2];
  const int c0 = d.tr.fchild[N - 2][p], c1 = d.tr.fchild[N - 2][p + 1];
  const int j0 = d.tr.fchild[N - 1][c0], j1 = d.tr.fchild[N - 1][c1];
  double* __restrict__ Qo = d.Q[N - 2];
  // B operand of M = AV P for rhs q: P[r' = 4 ks + gq][c]
  auto load_B = [&](int q, double* B) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int r1 = 4 * ks + gq;
      B[ks] = (r1 < RP && c < RL) ? Pn2[pb + ((int64_t)r1 * RL + c) * nrhs + q] : 0.0;
    }
  };
  auto store = [&](int q, const pc_f64x4& acc2) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r1 = gq + 4 * u;
      if (r1 < RP && c < RL) Qo[pb + ((int64_t)r1 * RL + c) * nrhs + q] = acc2[u];
    }
  };
  // right-hand sides in pairs; each pair walks the subtree's rows once
  for (int q = 0; q < nrhs; q += 2) {
    const bool two = q + 1 < nrhs;
    double B0[4], B1[4] = {0.0, 0.0, 0.0, 0.0};
    load_B(q, B0);
    if (two) load_B(q + 1, B1);
    pc_f64x4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    if (fa)
      ls_subtree_rows(d, j0, j1, q, two, B0, B1, (ls_ld)fa, (ls_ld)(fa + LS_FACT), lane, acc0, acc1);
    else
      ls_subtree_rows(d, j0, j1, q, two, B0, B1, (ls_gd)d.T.A[N - 2], (ls_gd)d.T.A[N - 1], lane, acc0, acc1);
    store(q, acc0);
    if (two) store(q + 1, acc1);
  }
}

// One 16-fibre tile of a mode product on v_mfma_f64_16x16x4 (R_n <= 16), one
// wave: out = in x_n M (M^T when trans), in = g + lambda x for the first product,
// the output scaled by dinv for the last product of the eigenvector form.
__device__ __forceinline__ void ls_mode(const BatchDesc& d, const LStage& st, int64_t v) {
  const double* __restrict__ M = st.M;
  const Geom& g = d.g;
  const PcFib fb(g, st.k);
  const unsigned tile = (unsigned)(v >> 6), lane = (unsigned)v & 63u;
  if (tile >= fb.ntile) return;   // uniform over the wave
  const int Rn = fb.Rn;
  const int col = lane & 15, kq = lane >> 4;
  const bool hin = st.io & 1;
  const double* __restrict__ in = hin ? d.Q[0] : ((st.io & 8) ? d.t1 : d.t0);
  double* __restrict__ out = (st.io & 4) ? d.t1 : d.t0;
  double A1[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + kq;
    A1[ks] = (col < Rn && k < Rn) ? (st.trans ? M[k * Rn + col] : M[col * Rn + k]) : 0.0;
  }
  const unsigned f = tile * 16u + (unsigned)col;
  const bool valid = f < fb.nfib;
  const size_t base = valid ? fb.base(f) : 0;
  double Bv[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int k = 4 * ks + kq;
    const size_t e = base + (size_t)k * fb.post;
    double b = 0.0;
    if (valid && k < Rn) {
      b = in[e];
      if (hin) b = fma(d.lambda, d.P[0][e], b);
    }
    Bv[ks] = b;
  }
  pc_f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A1[ks], Bv[ks], acc, 0, 0, 0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a = kq + 4 * u;
    if (valid && a < Rn) {
      const size_t e = base + (size_t)a * fb.post;
      double o = acc[u];
      if (st.io & 2) o *= d.dinv[e / (size_t)g.nrhs];
      out[e] = o;
    }
  }
}

// Update stage, one workgroup per chunk of TM_THREADS rows r of x (all RHS):
// x <- x - eta d for RHS not yet converged, chunk partial norms of d and x per
// RHS.  The last chunk to arrive sums the partials in chunk order and applies the
// stopping rule and the divergence test (as the single-problem update does).
// Returns true in the workgroup that finished the iteration of a problem whose
// solve is over.
__device__ bool ls_update(const BatchDesc& d, const LExtra& L, int64_t chunk, double eta, double tol, int max_iter,
                          double* red2 /* waves x LS_MAXRHS x 2 */, int* flag_s) {
  const Geom& g = d.g;
  const int nrhs = g.nrhs;
  IterState* __restrict__ st = d.st;
  const double* __restrict__ dt = L.dfin ? d.t1 : d.t0;
  double* __restrict__ x = d.P[0];
  const int64_t r = chunk * TM_THREADS + threadIdx.x;
  const bool ok = r < g.Rtot;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int q = 0; q < nrhs; ++q) {
    const int done = st->done[q];
    double xv = ok ? x[r * nrhs + q] : 0.0;
    const double dv = ok ? dt[r * nrhs + q] : 0.0;
    if (ok && !done) {
      xv = fma(-eta, dv, xv);
      x[r * nrhs + q] = xv;
    }
    const double dd = wave_sum(dv * dv), xx = wave_sum(xv * xv);
    if (lane == 0) {
      red2[(w * LS_MAXRHS + q) * 2] = dd;
      red2[(w * LS_MAXRHS + q) * 2 + 1] = xx;
    }
  }
  __syncthreads();
  if (threadIdx.x < nrhs) {
    const int q = threadIdx.x;
    double dd = 0.0, xx = 0.0;
    for (int i = 0; i < nw; ++i) {
      dd += red2[(i * LS_MAXRHS + q) * 2];
      xx += red2[(i * LS_MAXRHS + q) * 2 + 1];
    }
    L.part[(chunk * nrhs + q) * 2] = dd;
    L.part[(chunk * nrhs + q) * 2 + 1] = xx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const int prev = atomicAdd(L.ticket, 1);
    *flag_s = prev == L.nchunk - 1;
  }
  __syncthreads();
  if (!*flag_s) return false;
  __threadfence();
  const int it = st->iters;
  __syncthreads();
  int fin = 0;
  if (threadIdx.x < 64) {
    const int q = threadIdx.x;
    int all = 1, div = 0;
    if (q < nrhs) {
      const int done = st->done[q];
      double dd = 0.0, xx = 0.0;
      for (int c = 0; c < L.nchunk; ++c) {
        dd += L.part[((int64_t)c * nrhs + q) * 2];
        xx += L.part[((int64_t)c * nrhs + q) * 2 + 1];
      }
      if (!done) {
        const double dn = sqrt(dd), xn = sqrt(xx);
        const double rel = xn > 0.0 ? eta * dn / xn : (dn > 0.0 ? INFINITY : 0.0);
        st->rel[q] = rel;
        if (it == 0) { st->dnorm0[q] = dn; st->rel_first[q] = rel; }
        const bool bad = !isfinite(dn) || !isfinite(xn) || (it > 0 && dn > 1e6 * st->dnorm0[q] && dn > 0.0);
        if (bad) div = 1;
        if (rel <= tol || bad) { st->done[q] = 1; st->it_rhs[q] = it + 1; }
        else all = 0;
      }
    }
    // wave-wide AND / OR over the RHS lanes
    all = __all(all);
    div = __any(div);
    if (q == 0) {
      st->iters = it + 1;
      if (div) st->diverged = 1;
      if (all || div || it + 1 >= max_iter) {
        st->all_done = 1;
        fin = 1;
      }
      *L.ticket = 0;
      *flag_s = fin;
    }
  }
  __syncthreads();
  return *flag_s != 0;
}

// Team-wide barrier over nblocks workgroups with a wall-clock bound: a workgroup
// that waits longer than `limit` ticks raises the abort flag, and every
// workgroup that sees the flag returns false.
__device__ bool team_sync(unsigned* bar, unsigned nblocks, int32_t* abortf, uint64_t limit) {
  __shared__ int ok_s;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      unsigned spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0u &&
            (wall_clock64() - t0 > limit || __hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
          __hip_atomic_store(abortf, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    if (__hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    __threadfence();
    ok_s = ok;
  }
  __syncthreads();
  return ok_s != 0;
}

struct BatchArgs {
  const BatchDesc* descs;   // all problems: queue problems first, then team problems
  const int32_t* order;     // queue problems, largest first
  int nqueue;               // problems on the queue
  int nteam_prob;           // problems of the team (descs[nqueue + i], L[i])
  const LExtra* L;
  int64_t* done_step;       // per team problem: 0 while active, else the first step it is inactive
  int32_t* queue;           // queue counter (0 at launch)
  unsigned* bar;            // team barrier: [0] arrivals, [1] generation
  int32_t* abortf;
  int max_iter;
  double eta, tol;
  uint64_t limit;           // barrier wait bound (wall-clock ticks)
};

// The small-problem body: one workgroup per problem, workgroup barriers only.
__device__ void batched_queue(const BatchArgs& a, double* ms, double* red) {
  __shared__ int cur_s, stop_s;
  for (;;) {
    if (threadIdx.x == 0) cur_s = atomicAdd(a.queue, 1);
    __syncthreads();
    const int qi = __builtin_amdgcn_readfirstlane(cur_s);
    __syncthreads();
    if (qi >= a.nqueue) break;
    const BatchDesc& d = a.descs[__builtin_amdgcn_readfirstlane(a.order[qi])];
    const Geom& g = d.g;
    const int N = g.N;
    const int32_t fl = *d.flags;
    const bool bad = (fl & (KR_FLAG_NONFINITE | KR_FLAG_QUANT)) || ((fl & KR_FLAG_SINGULAR) && d.lambda == 0.0);
    if (bad) continue;   // uniform over the workgroup
    unsigned S[KR_MAXN + 1];
    for (int k = 0; k <= N; ++k) S[k] = (unsigned)d.tr.cnt[k];
    for (int it = 0; it < a.max_iter; ++it) {
      for (int k = 1; k < N - 1; ++k) {
        bt_forward(d, k, S[k]);
        __syncthreads();
      }
      bt_rows(d, S[N - 1]);
      __syncthreads();
      for (int k = N - 1; k >= 2; --k) {
        bt_adjoint(d, k, S[k - 1]);
        __syncthreads();
      }
      if (N >= 2) {
        bt_root(d, S[1]);
        __syncthreads();
      }
      pc_step_f64<1>(d.T, g, d.Q[0], 1u, d.dinv, d.P[0], d.t0, d.t1, d.lambda, a.eta, a.tol, a.max_iter,
                     d.use_ginv, d.st, red, ms);
      // thread 0 wrote the state; it decides and broadcasts, so that the whole
      // workgroup leaves the loop together
      if (threadIdx.x == 0) stop_s = d.st->all_done;
      __syncthreads();
      if (stop_s) break;
    }
    __syncthreads();
  }
}

// The large-problem body: the team's lockstep over stage steps.  LDS (from the
// queue body's matrix buffer): the offsets of every problem's work items in this
// step, a scan buffer and the update's per-wave partial norms.
#define LS_WAVES (TM_THREADS / 64)
__device__ void batched_team(const BatchArgs& a, unsigned rank, unsigned nteam, char* lds) {
  int64_t* off = (int64_t*)lds;                                  // LS_MAXP + 1
  int64_t* wtot = off + LS_MAXP + 1;                             // LS_WAVES
  double* red2 = (double*)(wtot + LS_WAVES);                     // LS_WAVES x LS_MAXRHS x 2
  double* fact = red2 + LS_WAVES * LS_MAXRHS * 2;                // 2 x LS_FACT staged factors
  __shared__ int flag_s, any_s, tag_s;
  if (threadIdx.x == 0) tag_s = -1;
  const int np = a.nteam_prob;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t t = 0;; ++t) {
    // work items of every active problem's stage at step t (multiples of
    // TM_THREADS), and their exclusive prefix sums
    if (threadIdx.x == 0) { any_s = 0; off[0] = 0; }
    __syncthreads();
    int64_t carry = 0;
    for (int b0 = 0; b0 < np; b0 += TM_THREADS) {
      const int i = b0 + threadIdx.x;
      int64_t n = 0;
      if (i < np) {
        const BatchDesc& d = a.descs[a.nqueue + i];
        const int32_t fl = *d.flags;
        const bool bad = (fl & (KR_FLAG_NONFINITE | KR_FLAG_QUANT)) || ((fl & KR_FLAG_SINGULAR) && d.lambda == 0.0);
        const int64_t ds = a.done_step[i];
        if (!bad && (ds == 0 || ds > t)) {
          const LExtra& L = a.L[i];
          n = ls_threads(d, L, L.st[t % L.nst]);
          any_s = 1;
        }
      }
      int64_t incl = n;   // inclusive scan within the wave
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
      }
      if (lane == 63) wtot[wv] = incl;
      __syncthreads();
      int64_t before = carry;
      for (int w = 0; w < wv; ++w) before += wtot[w];
      if (i < np) off[i + 1] = before + incl;
      for (int w = 0; w < LS_WAVES; ++w) carry += wtot[w];
      __syncthreads();
    }
    if (!any_s) break;   // every problem is done (the same memory state in every workgroup)
    const int64_t total = off[np];
    for (int64_t base = (int64_t)rank * TM_THREADS; base < total; base += (int64_t)nteam * TM_THREADS) {
      // the problem owning items base .. base + TM_THREADS - 1 (uniform)
      int lo = 0, hi = np;   // off[lo] <= base < off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= base) lo = mid; else hi = mid;
      }
      // uniform values in scalar registers: the descriptor fields then load
      // through the scalar cache instead of occupying vector registers
      const int i = __builtin_amdgcn_readfirstlane(lo);
      const BatchDesc& d = a.descs[a.nqueue + i];
      const LExtra& L = a.L[i];
      const LStage st = L.st[t % L.nst];
      const int64_t oi = off[i];
      const int64_t v0 = base - (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(oi >> 32)) << 32) |
                                          (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)oi));
      const int64_t v = v0 + threadIdx.x;
      switch (st.kind) {
        case LS_FWD: ls_forward(d, st.k, v); break;
        case LS_ROWS: ls_rows(d, v); break;
        case LS_ROWS2: ls_rows2(d, v, ls_stage_factors(d, i, fact, &tag_s) ? fact : nullptr); break;
        case LS_ADJ: ls_adjoint(d, st.k, v); break;
        case LS_ROOT: ls_adjoint(d, 1, v); break;
        case LS_MODE: ls_mode(d, st, v); break;
        default:
          if (v0 / TM_THREADS < L.nchunk &&
              ls_update(d, L, v0 / TM_THREADS, a.eta, a.tol, a.max_iter, red2, &flag_s) && threadIdx.x == 0)
            a.done_step[i] = t + 1;
          break;
      }
    }
    if (!team_sync(a.bar, nteam, a.abortf, a.limit)) break;
  }
}

#define TM_LDS_BYTES ((LS_MAXP + 1 + LS_WAVES) * 8 + LS_WAVES * LS_MAXRHS * 2 * 8 + 2 * LS_FACT * 8)

// Small problems: one workgroup per problem from the queue.
__global__ void __launch_bounds__(BT_THREADS) k_batched_queue(BatchArgs a) {
  __shared__ double ms[PC_MATS];
  __shared__ double red[2 * BT_THREADS / 64];
  batched_queue(a, ms, red);
}

// Large problems: the team, every workgroup resident (cooperative launch).
__global__ void __launch_bounds__(TM_THREADS) k_batched_team(BatchArgs a) {
  __shared__ __attribute__((aligned(16))) char lds[TM_LDS_BYTES];
  batched_team(a, blockIdx.x, gridDim.x, lds);
}

}  // namespace kr
