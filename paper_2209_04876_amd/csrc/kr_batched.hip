// Batched Algorithm 2: many independent ridge problems of uneven N, I_n, R_n and
// right-hand sides in one persistent launch.
//
// Each problem's setup and sketch (Gram, leverage, sampling, sort, sample tree,
// gathered rows) is enqueued with the single-problem kernels.  The Richardson
// iterations of all problems then run in one launch of k_batched_richardson: a
// workgroup takes the next problem from a device queue (problems ordered by
// estimated cost, largest first) and runs that problem's whole iteration --
// forward levels, rows, adjoint levels, root adjoint, preconditioner and update
// -- with workgroup barriers only, until the stopping rule holds or max_iter;
// then it takes the next problem.  No per-iteration launches, no host polling,
// no grid barriers.  Every output of a pass has one owning thread with a fixed
// summation order, so results do not depend on which workgroup runs a problem.
#include "kr_internal.h"

namespace kr {

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

// The persistent batched iteration.  queue[0] must be 0 at launch; order lists the
// problems largest first.  A problem whose setup flagged an error is skipped (its
// state stays at zero iterations; the host reports the error).
#define BT_THREADS 512
template <int NB>
__global__ void __launch_bounds__(BT_THREADS) k_batched_richardson(const BatchDesc* __restrict__ descs,
                                                                  const int32_t* __restrict__ order, int nprob,
                                                                  int32_t* __restrict__ queue, double eta,
                                                                  double tol, int max_iter) {
  __shared__ int cur_s, stop_s;
  __shared__ double red[16];
  __shared__ double ms[PC_MATS];
  for (;;) {
    if (threadIdx.x == 0) cur_s = atomicAdd(queue, 1);
    __syncthreads();
    const int qi = cur_s;
    __syncthreads();
    if (qi >= nprob) break;
    const BatchDesc& d = descs[order[qi]];
    const Geom& g = d.g;
    const int N = g.N;
    const int32_t fl = *d.flags;
    const bool bad = (fl & (KR_FLAG_NONFINITE | KR_FLAG_QUANT)) || ((fl & KR_FLAG_SINGULAR) && d.lambda == 0.0);
    if (bad) continue;   // uniform over the workgroup
    unsigned S[KR_MAXN + 1];
    for (int k = 0; k <= N; ++k) S[k] = (unsigned)d.tr.cnt[k];
    for (int it = 0; it < max_iter; ++it) {
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
      pc_step_f64<NB>(d.T, g, d.Q[0], 1u, d.dinv, d.P[0], d.t0, d.t1, d.lambda, eta, tol, max_iter, d.use_ginv,
                      d.st, red, ms);
      // thread 0 wrote the state; it decides and broadcasts, so that the whole
      // workgroup leaves the loop together
      if (threadIdx.x == 0) stop_s = d.st->all_done;
      __syncthreads();
      if (stop_s) break;
    }
    __syncthreads();
  }
}

}  // namespace kr
