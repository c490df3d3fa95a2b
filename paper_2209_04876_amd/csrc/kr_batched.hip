// Batched Algorithm 2: many independent ridge problems of uneven N, I_n, R_n and
// right-hand sides in one persistent launch.
//
// Each problem's setup and sketch (Gram, leverage, sampling, sort, sample tree,
// gathered rows) is enqueued with the single-problem kernels.  The Richardson
// iterations of all problems then run in one launch of k_batched_richardson,
// whose workgroups split into two groups:
//
//   queue  workgroups that take the next small problem from a device queue
//          (largest first) and run its whole iteration -- forward levels, rows,
//          adjoint levels, root adjoint, preconditioner and update -- with
//          workgroup barriers only, until the stopping rule holds or max_iter;
//   team   the other workgroups, which iterate all large problems together.
//          Each problem's iteration is a list of stages (forward levels, fused
//          rows, adjoint levels, root, one stage per preconditioner mode product,
//          update); at every step each active problem runs its next stage, and
//          the work items of all those stages form one index space that the team
//          strides over.  A team-wide barrier separates steps.  Problems with
//          short stage lists simply iterate more often; a problem leaves the
//          index space when its stopping rule holds.
//
// Every output of a stage has one owning thread (or lane group) with a fixed
// summation order, and the update's norms are reduced in chunk order, so results
// do not depend on the number of workgroups or on which workgroup runs what.
#include "kr_internal.h"

namespace kr {

#define BT_THREADS 512   // threads per workgroup of the batched launch

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
  int32_t nchunk;       // update chunks of BT_THREADS rows
  int32_t dfin;         // buffer holding M^+ h after the last mode product: 0 = t0, 1 = t1
  int32_t pad;
  double* part;         // update partial norms: nchunk x nrhs x 2
  int32_t* ticket;      // update arrivals
};

// Work items (threads, a multiple of BT_THREADS) of stage st of problem d.
__device__ int64_t ls_threads(const BatchDesc& d, const LExtra& L, const LStage& st) {
  const Geom& g = d.g;
  int64_t n = 0;
  switch (st.kind) {
    case LS_FWD: n = d.tr.cnt[st.k] * g.rsuf[st.k] * g.nrhs; break;
    case LS_ROWS: n = (g.N >= 2 ? d.tr.cnt[g.N - 1] : 1) * g.nrhs * 16; break;
    case LS_ROWS2: n = d.tr.cnt[g.N - 2] * g.nrhs * 16; break;
    case LS_ADJ: n = d.tr.cnt[st.k - 1] * g.rsuf[st.k - 1] * g.nrhs; break;
    case LS_ROOT: n = g.Rtot * g.nrhs; break;
    case LS_MODE: n = ((g.Rtot * g.nrhs / g.R[st.k] + 15) / 16) * 64; break;
    case LS_UPD: n = (int64_t)L.nchunk * BT_THREADS; break;
  }
  return (n + BT_THREADS - 1) / BT_THREADS * BT_THREADS;
}

// Forward level k, output element e.
__device__ __forceinline__ void ls_forward(const BatchDesc& d, int k, int64_t e) {
  const Geom& g = d.g;
  const int64_t W = g.rsuf[k] * g.nrhs, Wp = g.rsuf[k - 1] * g.nrhs;
  if (e >= d.tr.cnt[k] * W) return;
  const int Rk = g.R[k - 1];
  const int64_t s = e / W, cq = e - s * W;
  const int64_t p = k == 1 ? 0 : d.tr.parent[k][s];
  d.P[k][e] = dot_batched(d.tr.arow[k] + s * Rk, d.P[k - 1] + p * Wp + cq, W, Rk);
}

// Adjoint level k, output element e of Q_{k-1}.
__device__ __forceinline__ void ls_adjoint(const BatchDesc& d, int k, int64_t e) {
  const Geom& g = d.g;
  const int64_t W = g.rsuf[k] * g.nrhs, Wp = g.rsuf[k - 1] * g.nrhs;
  if (e >= d.tr.cnt[k - 1] * Wp) return;
  const int Rk = g.R[k - 1];
  const int64_t p = e / Wp, rem = e - p * Wp;
  const int64_t r = rem / W, cq = rem - r * W;
  const int s0 = d.tr.fchild[k - 1][p], s1 = d.tr.fchild[k - 1][p + 1];
  const double* __restrict__ arow = d.tr.arow[k];
  const double* __restrict__ Qk = d.Q[k];
  double acc = 0.0;
  int s = s0;
  for (; s + 4 <= s1; s += 4) {
    double av[4], qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = arow[(int64_t)(s + u) * Rk + r];
      qv[u] = Qk[(int64_t)(s + u) * W + cq];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
  }
  for (; s < s1; ++s) acc = fma(arow[(int64_t)s * Rk + r], Qk[(int64_t)s * W + cq], acc);
  d.Q[k - 1][e] = acc;
}

// Root adjoint, output element e of the gradient.
__device__ __forceinline__ void ls_root(const BatchDesc& d, int64_t e) {
  const Geom& g = d.g;
  if (e >= g.Rtot * g.nrhs) return;
  const int64_t W1 = g.rsuf[1] * g.nrhs;
  const int R0 = g.R[0];
  const int64_t S1 = d.tr.cnt[1];
  const int64_t r0 = e / W1, c = e - r0 * W1;
  const double* __restrict__ a0 = d.tr.arow[1];
  const double* __restrict__ Q1 = d.Q[1];
  double acc = 0.0;
  int64_t s = 0;
  for (; s + 4 <= S1; s += 4) {
    double av[4], qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a0[(s + u) * R0 + r0];
      qv[u] = Q1[(s + u) * W1 + c];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
  }
  for (; s < S1; ++s) acc = fma(a0[s * R0 + r0], Q1[s * W1 + c], acc);
  d.Q[0][e] = acc;
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

// Fused last two levels for N >= 3: a 16-lane group per (level-(N-2) node p,
// rhs q), lane = r_N.  For every child s of p: the forward value
// P_{N-1}[s] = a_{N-1}[s] . P_{N-2}[p], the residuals of s's rows, their
// adjoint Q_{N-1}[s], and its outer product with a_{N-1}[s] accumulated into
// Q_{N-2}[p].  Neither P_{N-1} nor Q_{N-1} is written.
__device__ __forceinline__ void ls_rows2(const BatchDesc& d, int64_t v) {
  const Geom& g = d.g;
  const int N = g.N, nrhs = g.nrhs;
  const int RL = g.R[N - 1], RP = g.R[N - 2];
  const int64_t task = v >> 4;
  const unsigned lane = (unsigned)v & 15u;
  if (task >= d.tr.cnt[N - 2] * nrhs) return;   // uniform over the group
  const int64_t p = task / nrhs;
  const int q = (int)(task - p * nrhs);
  const bool ln = (int)lane < RL;
  const int64_t pbase = p * (int64_t)RP * RL * nrhs + (int64_t)lane * nrhs + q;
  const double* __restrict__ Pn2 = d.P[N - 2];
  double pp[16], acc2[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    pp[r] = (ln && r < RP) ? Pn2[pbase + (int64_t)r * RL * nrhs] : 0.0;
    acc2[r] = 0.0;
  }
  const int s0 = d.tr.fchild[N - 2][p], s1 = d.tr.fchild[N - 2][p + 1];
  const double* __restrict__ aP = d.tr.arow[N - 1];
  for (int s = s0; s < s1; ++s) {
    double av[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) av[r] = r < RP ? aP[(int64_t)s * RP + r] : 0.0;
    double pv = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) pv = fma(av[r], pp[r], pv);
    const double acc1 = ls_rows_of(d, d.tr.fchild[N - 1][s], d.tr.fchild[N - 1][s + 1], pv, q, lane, ln);
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[r] = fma(av[r], acc1, acc2[r]);
  }
  if (ln) {
    double* __restrict__ Qo = d.Q[N - 2];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (r < RP) Qo[pbase + (int64_t)r * RL * nrhs] = acc2[r];
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

// Update stage, one workgroup per chunk of BT_THREADS rows r of x (all RHS):
// x <- x - eta d for RHS not yet converged, chunk partial norms of d and x per
// RHS.  The last chunk to arrive sums the partials in chunk order and applies the
// stopping rule and the divergence test (as the single-problem update does).
// Returns true in the workgroup that finished the iteration of a problem whose
// solve is over.
__device__ bool ls_update(const BatchDesc& d, const LExtra& L, int64_t chunk, double eta, double tol, int max_iter,
                          double* red2 /* 16 x LS_MAXRHS x 2 */, int* flag_s) {
  const Geom& g = d.g;
  const int nrhs = g.nrhs;
  IterState* __restrict__ st = d.st;
  const double* __restrict__ dt = L.dfin ? d.t1 : d.t0;
  double* __restrict__ x = d.P[0];
  const int64_t r = chunk * BT_THREADS + threadIdx.x;
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
  int nqueue_wg;            // workgroups 0 .. nqueue_wg-1 serve the queue, the rest form the team
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
    const int qi = cur_s;
    __syncthreads();
    if (qi >= a.nqueue) break;
    const BatchDesc& d = a.descs[a.order[qi]];
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
#define LS_WAVES (BT_THREADS / 64)
__device__ void batched_team(const BatchArgs& a, unsigned rank, unsigned nteam, char* lds) {
  int64_t* off = (int64_t*)lds;                                  // LS_MAXP + 1
  int64_t* wtot = off + LS_MAXP + 1;                             // LS_WAVES
  double* red2 = (double*)(wtot + LS_WAVES);                     // LS_WAVES x LS_MAXRHS x 2
  __shared__ int flag_s, any_s;
  const int np = a.nteam_prob;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t t = 0;; ++t) {
    // work items of every active problem's stage at step t (multiples of
    // BT_THREADS), and their exclusive prefix sums
    if (threadIdx.x == 0) { any_s = 0; off[0] = 0; }
    __syncthreads();
    int64_t carry = 0;
    for (int b0 = 0; b0 < np; b0 += BT_THREADS) {
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
    for (int64_t base = (int64_t)rank * BT_THREADS; base < total; base += (int64_t)nteam * BT_THREADS) {
      // the problem owning items base .. base + BT_THREADS - 1 (uniform)
      int lo = 0, hi = np;   // off[lo] <= base < off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= base) lo = mid; else hi = mid;
      }
      const int i = lo;
      const BatchDesc& d = a.descs[a.nqueue + i];
      const LExtra& L = a.L[i];
      const LStage st = L.st[t % L.nst];
      const int64_t v0 = base - off[i];
      const int64_t v = v0 + threadIdx.x;
      switch (st.kind) {
        case LS_FWD: ls_forward(d, st.k, v); break;
        case LS_ROWS: ls_rows(d, v); break;
        case LS_ROWS2: ls_rows2(d, v); break;
        case LS_ADJ: ls_adjoint(d, st.k, v); break;
        case LS_ROOT: ls_root(d, v); break;
        case LS_MODE: ls_mode(d, st, v); break;
        default:
          if (v0 / BT_THREADS < L.nchunk &&
              ls_update(d, L, v0 / BT_THREADS, a.eta, a.tol, a.max_iter, red2, &flag_s) && threadIdx.x == 0)
            a.done_step[i] = t + 1;
          break;
      }
    }
    if (!team_sync(a.bar, nteam, a.abortf, a.limit)) break;
  }
}

static_assert((LS_MAXP + 1 + LS_WAVES) * 8 + LS_WAVES * LS_MAXRHS * 2 * 8 <= PC_MATS * 8,
              "the team's LDS must fit in the queue body's matrix buffer");

__global__ void __launch_bounds__(BT_THREADS) k_batched_richardson(BatchArgs a) {
  __shared__ double ms[PC_MATS];
  __shared__ double red[16];
  if ((int)blockIdx.x < a.nqueue_wg) batched_queue(a, ms, red);
  else batched_team(a, blockIdx.x - a.nqueue_wg, gridDim.x - a.nqueue_wg, (char*)ms);
}

}  // namespace kr
