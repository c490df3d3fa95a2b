// The whole preconditioned Richardson loop of Algorithm 2 in one cooperative
// launch (for prod(R) * nrhs small enough that every workgroup can hold the
// iterate in LDS).  Per iteration, two grid-wide barriers separate:
//   phase G  each workgroup owns a contiguous range of level-1 nodes (distinct
//            first indices i_0) holding about D / workgroups rows and walks their
//            subtrees level by level: forward products down to the rows, the
//            residuals Omega_j (k_j x - b_j), and the adjoint back up to Q_1[s]
//            (Theorem kron_mat_mul_sqrt_decomp, applied per prefix);
//   phase R  a block of columns of g = sum_s a_0[i_0(s)] (outer) Q_1[s] for every r_0,
//            plus lambda x, with the preconditioner's mode-0 product applied
//            locally;
//   update   every workgroup finishes M^+ (modes 1..N-1 and, for lambda > 0, the
//            diagonal and the V products) on its own LDS copy, forms
//            x <- x - (1 - sqrt(eps)) d, the norms and the stopping decision.
// The update is computed redundantly with identical arithmetic in every
// workgroup, so all reach the same decision without another barrier.
// The grid barrier spins with a bound and an abort flag: a workgroup that waits
// too long raises the flag and every workgroup leaves the loop.
#include "kr_internal.h"

namespace kr {

struct PArgs {
  ModeTables T;
  Geom g;
  Tree tr;
  const double* Omega;
  const double* bD;
  double* P[KR_MAXN];     // level scratch, k = 1..N-1 (node-major)
  double* Q[KR_MAXN];     // level scratch, k = 1..N-1
  double* gp;             // phase-R output, Rtot x nrhs
  double* wrow;           // Omega_j (k_j x - b_j) per distinct row, D x nrhs
  const int64_t* rs1;     // first row of each level-1 subtree, S_1 + 1 entries
  double* xout;           // final iterate
  IterState* st;
  unsigned* bar;          // [0] arrivals, [1] generation
  int32_t* abortf;
  const int32_t* setup_flags;
  double lambda, eta, tol;
  int max_iter;
  int use_ginv;
};

__device__ bool grid_sync(unsigned* bar, unsigned nblocks, int32_t* abortf) {
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
      long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if ((++spins & 1023) == 0 &&
            (spins > (1L << 24) || __hip_atomic_load(abortf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
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

// out = in x_n M over a tensor with dims R[lo..N-1] and nrhs innermost (LDS or
// global).  M is R_n x R_n; trans selects M^T.
__device__ __forceinline__ void mode_prod_slice(const Geom& g, int lo, int n, const double* __restrict__ M,
                                                int trans, const double* in, double* out) {
  const int Rn = g.R[n];
  const int64_t post = g.rsuf[n + 1] * g.nrhs;
  const int64_t total = g.rsuf[lo] * g.nrhs;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t blk = e / (Rn * post);
    const int64_t rem = e - blk * Rn * post;
    const int a = (int)(rem / post);
    const int64_t c = rem - (int64_t)a * post;
    const double* src = in + blk * Rn * post + c;
    double acc = 0.0;
    for (int b = 0; b < Rn; ++b) acc = fma(trans ? M[b * Rn + a] : M[a * Rn + b], src[(int64_t)b * post], acc);
    out[e] = acc;
  }
}

// Copy n doubles global -> LDS with eight independent loads in flight per thread.
__device__ __forceinline__ void bulk_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t base = 0; base < n; base += (int64_t)blockDim.x * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      v[u] = i < n ? src[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      if (i < n) dst[i] = v[u];
    }
  }
}

// (q, r) = divmod(e, W) for e = e0, e0 + step, ... without dividing in the loop.
struct DivIter {
  unsigned q, r, dq, dr, W;
  __device__ __forceinline__ DivIter(unsigned e0, unsigned W_, unsigned step) : W(W_) {
    q = e0 / W; r = e0 - q * W; dq = step / W; dr = step - dq * W;
  }
  __device__ __forceinline__ void next() {
    q += dq; r += dr;
    if (r >= W) { r -= W; ++q; }
  }
};

// out = in x_n M for a tensor [R_0..R_{N-1}][nrhs] in LDS; M (Rn x Rn, row-major,
// transposed when trans) in LDS.  Each thread owns whole mode-n fibres (blk, c):
// it loads the fibre into registers once and forms all Rn outputs, reading M as
// wave-uniform broadcasts.
template <int RM>
__device__ __forceinline__ void mode_prod_fibre(const Geom& g, int n, const double* __restrict__ M, int trans,
                                                const double* in, double* out) {
  const int Rn = g.R[n];
  const unsigned post = (unsigned)(g.rsuf[n + 1] * g.nrhs);
  const unsigned nfib = (unsigned)(g.rsuf[0] * g.nrhs) / (unsigned)Rn;
  DivIter it(threadIdx.x, post, blockDim.x);
  for (unsigned f = threadIdx.x; f < nfib; f += blockDim.x, it.next()) {
    const unsigned base = it.q * (unsigned)Rn * post + it.r;
    double v[RM];
#pragma unroll
    for (int b = 0; b < RM; ++b) v[b] = b < Rn ? in[base + b * post] : 0.0;
    for (int a = 0; a < Rn; ++a) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < Rn) acc = fma(trans ? M[b * Rn + a] : M[a * Rn + b], v[b], acc);
      out[base + a * post] = acc;
    }
  }
}

__device__ __forceinline__ void mode_prod_any(const Geom& g, int n, const double* M, int trans, const double* in,
                                              double* out) {
  const int Rn = g.R[n];
  if (Rn <= 8) mode_prod_fibre<8>(g, n, M, trans, in, out);
  else if (Rn <= 16) mode_prod_fibre<16>(g, n, M, trans, in, out);
  else if (Rn <= 32) mode_prod_fibre<32>(g, n, M, trans, in, out);
  else mode_prod_fibre<64>(g, n, M, trans, in, out);
}

template <int G>
__global__ void __launch_bounds__(1024) k_richardson_persistent(PArgs a) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  __shared__ int done_s[KR_MAX_RHS];
  __shared__ double dn0_s[KR_MAX_RHS];
  __shared__ int64_t range_s[2];
  const Geom& g = a.g;
  const int N = g.N, nrhs = g.nrhs;
  const unsigned RT = (unsigned)(g.Rtot * nrhs);
  const unsigned W1 = (unsigned)(g.rsuf[1] * nrhs);
  const int R0 = g.R[0];
  const unsigned BD = blockDim.x;
  // LDS: iterate x, two work regions of MR = max(RT, blockDim) doubles, the ridge
  // diagonal (lambda > 0) and the preconditioner matrices
  const unsigned MR = RT > BD ? RT : BD;
  double* xs = lds;
  double* ts = lds + MR;
  double* us = lds + 2 * MR;
  double* dg = lds + 3 * MR;
  double* mats = dg + (a.use_ginv ? 0 : RT);
  int moff[KR_MAXN];
  {
    int off = 0;
    for (int n = 0; n < N; ++n) { moff[n] = off; off += g.R[n] * g.R[n]; }
  }
  const unsigned nb = gridDim.x;
  for (unsigned e = threadIdx.x; e < RT; e += BD) xs[e] = 0.0;
  for (int n = 0; n < N; ++n) {
    const double* M = a.use_ginv ? a.T.Ginv[n] : a.T.V[n];
    for (int e = threadIdx.x; e < g.R[n] * g.R[n]; e += BD) mats[moff[n] + e] = M[e];
  }
  if (!a.use_ginv) {
    // D = (kron Lambda + lambda)^-1 on the row-major multi-index, once
    for (unsigned e = threadIdx.x; e < RT; e += BD) {
      unsigned r = e / (unsigned)nrhs;
      double prod = 1.0;
      for (int n = N - 1; n >= 0; --n) {
        const unsigned rn = r % (unsigned)g.R[n];
        r /= (unsigned)g.R[n];
        prod *= a.T.evals[n][rn];
      }
      const double den = prod + a.lambda;
      dg[e] = den > 0.0 ? 1.0 / den : 0.0;
    }
  }
  for (int q = threadIdx.x; q < nrhs; q += BD) done_s[q] = 0;
  const int64_t S1 = a.tr.cnt[1];
  const int64_t D = a.tr.cnt[N];
  // contiguous range of level-1 nodes holding about D / nb rows (row starts of
  // level-1 nodes are non-decreasing)
  if (threadIdx.x < 2) {
    const int64_t w = blockIdx.x + threadIdx.x;
    int64_t sv;
    if (w == 0) sv = 0;
    else if (w >= (int64_t)nb) sv = S1;
    else {
      const int64_t target = (w * D + nb - 1) / nb;
      int64_t lo = 0, hi = S1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.rs1[mid] < target) lo = mid + 1; else hi = mid;
      }
      sv = lo;
    }
    range_s[threadIdx.x] = sv;
  }
  __syncthreads();
  const unsigned sa = (unsigned)range_s[0], sb = (unsigned)range_s[1];
  int it = 0;
  bool aborted = false;
  // inputs that make the iteration meaningless are reported by the host
  if (*a.setup_flags & (KR_FLAG_NONFINITE | KR_FLAG_QUANT | (a.use_ginv ? KR_FLAG_SINGULAR : 0)))
    return;
  const unsigned CE = (unsigned)R0 >= BD ? 1u : BD / (unsigned)R0;   // phase-R columns per task
  const unsigned ntaskR = (W1 + CE - 1) / CE;
  const unsigned WA = 2 * MR;                                         // staging doubles (ts..us)
  const unsigned S1u = (unsigned)S1;
  for (; it < a.max_iter; ++it) {
    // ---------------- phase G: the subtrees of level-1 nodes [sa, sb), level by level
    if (sa < sb) {
      unsigned lo[KR_MAXN + 1], hi[KR_MAXN + 1];
      lo[1] = sa; hi[1] = sb;
      {
        const unsigned cnt = (sb - sa) * W1;
        DivIter di(threadIdx.x, W1, BD);
        for (unsigned e = threadIdx.x; e < cnt; e += BD, di.next()) {
          const unsigned s = sa + di.q, c = di.r;
          const double* ar = a.tr.arow[1] + (size_t)s * R0;
          double acc = 0.0;
#pragma unroll 4
          for (int r = 0; r < R0; ++r) acc = fma(ar[r], xs[r * W1 + c], acc);
          a.P[1][(size_t)s * W1 + c] = acc;
        }
        __syncthreads();
      }
      for (int k = 2; k <= N - 1; ++k) {
        lo[k] = a.tr.fchild[k - 1][lo[k - 1]];
        hi[k] = a.tr.fchild[k - 1][hi[k - 1]];
        const unsigned Wk = (unsigned)(g.rsuf[k] * nrhs), Wp = (unsigned)(g.rsuf[k - 1] * nrhs);
        const int Rk = g.R[k - 1];
        const double* __restrict__ arow = a.tr.arow[k];
        const unsigned cnt = (hi[k] - lo[k]) * Wk;
        DivIter di(threadIdx.x, Wk, BD);
        for (unsigned e = threadIdx.x; e < cnt; e += BD, di.next()) {
          const unsigned sn = lo[k] + di.q, cq = di.r;
          const double* src = a.P[k - 1] + (size_t)a.tr.parent[k][sn] * Wp + cq;
          const double* ak = arow + (size_t)sn * Rk;
          double acc = 0.0;
#pragma unroll 4
          for (int r = 0; r < Rk; ++r) acc = fma(ak[r], src[r * Wk], acc);
          a.P[k][(size_t)sn * Wk + cq] = acc;
        }
        __syncthreads();
      }
      // rows: w_j = Omega_j (k_j x - b_j), one thread per (row, rhs)
      const int L = N - 1;
      const int R = g.R[N - 1];
      const double* __restrict__ AL = a.tr.arow[N];
      const unsigned jlo = a.tr.fchild[L][lo[L]], jhi = a.tr.fchild[L][hi[L]];
      {
        const unsigned cnt = (jhi - jlo) * nrhs;
        DivIter di(threadIdx.x, nrhs, BD);
        for (unsigned e = threadIdx.x; e < cnt; e += BD, di.next()) {
          const unsigned j = jlo + di.q, q = di.r;
          const double* Pp = a.P[L] + (size_t)a.tr.parent[N][j] * R * nrhs + q;
          const double* aj = AL + (size_t)j * R;
          double y = 0.0;
#pragma unroll 4
          for (int r = 0; r < R; ++r) y = fma(aj[r], Pp[r * nrhs], y);
          a.wrow[(size_t)j * nrhs + q] = a.Omega[j] * (y - a.bD[(size_t)j * nrhs + q]);
        }
        __syncthreads();
      }
      // adjoint of the rows: Q_{N-1}[p][r][q] = sum_{j child of p} w_j a_{N-1}[i(j)][r]
      {
        const unsigned RW = (unsigned)R * nrhs;
        const unsigned cnt = (hi[L] - lo[L]) * RW;
        DivIter di(threadIdx.x, RW, BD);
        for (unsigned e = threadIdx.x; e < cnt; e += BD, di.next()) {
          const unsigned p = lo[L] + di.q, rem = di.r;
          const unsigned r = rem / (unsigned)nrhs, q = rem - r * nrhs;
          const int j0 = a.tr.fchild[L][p], j1 = a.tr.fchild[L][p + 1];
          double acc = 0.0;
          int j = j0;
          for (; j + 4 <= j1; j += 4) {
            double av[4], wv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              av[u] = AL[(size_t)(j + u) * R + r];
              wv[u] = a.wrow[(size_t)(j + u) * nrhs + q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = fma(wv[u], av[u], acc);
          }
          for (; j < j1; ++j) acc = fma(a.wrow[(size_t)j * nrhs + q], AL[(size_t)j * R + r], acc);
          a.Q[L][(size_t)p * RW + rem] = acc;
        }
        __syncthreads();
      }
      for (int k = N - 1; k >= 2; --k) {
        const unsigned Wk = (unsigned)(g.rsuf[k] * nrhs), Wp = (unsigned)(g.rsuf[k - 1] * nrhs);
        const int Rk = g.R[k - 1];
        const double* __restrict__ arow = a.tr.arow[k];
        const double* __restrict__ Qk = a.Q[k];
        const unsigned cnt = (hi[k - 1] - lo[k - 1]) * Wp;
        DivIter di(threadIdx.x, Wp, BD);
        for (unsigned e = threadIdx.x; e < cnt; e += BD, di.next()) {
          const unsigned p = lo[k - 1] + di.q, rem = di.r;
          const unsigned r = rem / Wk, cq = rem - r * Wk;
          const int s0 = a.tr.fchild[k - 1][p], s1e = a.tr.fchild[k - 1][p + 1];
          double acc = 0.0;
          int sn = s0;
          for (; sn + 4 <= s1e; sn += 4) {
            double av[4], qv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              av[u] = arow[(size_t)(sn + u) * Rk + r];
              qv[u] = Qk[(size_t)(sn + u) * Wk + cq];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = fma(av[u], qv[u], acc);
          }
          for (; sn < s1e; ++sn) acc = fma(arow[(size_t)sn * Rk + r], Qk[(size_t)sn * Wk + cq], acc);
          a.Q[k - 1][(size_t)p * Wp + rem] = acc;
        }
        __syncthreads();
      }
    }
    if (!grid_sync(a.bar, nb, a.abortf)) { aborted = true; break; }
    // ---------------- phase R: columns [e0, e0 + CE) of g for every r_0, then mode 0 of M^+
    for (unsigned task = blockIdx.x; task < ntaskR; task += nb) {
      const unsigned e0 = task * CE;
      const unsigned r0 = threadIdx.x / CE, ce = threadIdx.x - r0 * CE;
      const unsigned e = e0 + ce;
      const bool act = r0 < (unsigned)R0 && e < W1;
      const unsigned CEv = (W1 - e0) < CE ? (W1 - e0) : CE;   // valid columns in this block
      const unsigned SC = WA / ((unsigned)R0 + CE);            // level-1 nodes per staged chunk
      double* ast = ts;                 // SC x R0
      double* qst = ts + SC * R0;       // SC x CE
      double acc = 0.0;
      for (unsigned sbase = 0; sbase < S1u; sbase += SC) {
        const unsigned ns = (S1u - sbase) < SC ? (S1u - sbase) : SC;
        bulk_copy(ast, a.tr.arow[1] + (size_t)sbase * R0, (int64_t)ns * R0);
        {
          DivIter di(threadIdx.x, CE, BD);
          for (unsigned i = threadIdx.x; i < ns * CE; i += BD, di.next())
            qst[i] = di.r < CEv ? a.Q[1][(size_t)(sbase + di.q) * W1 + e0 + di.r] : 0.0;
        }
        __syncthreads();
        if (act) {
          for (unsigned sn = 0; sn < ns; ++sn) acc = fma(ast[sn * R0 + r0], qst[sn * CE + ce], acc);
        }
        __syncthreads();
      }
      if (act) acc += a.lambda * xs[r0 * W1 + e];
      if (threadIdx.x < (unsigned)R0 * CE) us[threadIdx.x] = acc;
      __syncthreads();
      if (act) {
        const double* M = mats + moff[0];
        double out = 0.0;
        for (int b = 0; b < R0; ++b) out = fma(a.use_ginv ? M[r0 * R0 + b] : M[b * R0 + r0], us[b * CE + ce], out);
        a.gp[(size_t)r0 * W1 + e] = out;
      }
      __syncthreads();
    }
    if (!grid_sync(a.bar, nb, a.abortf)) { aborted = true; break; }
    // ---------------- redundant update: remaining modes of M^+, x update, stopping rule
    bulk_copy(ts, a.gp, RT);
    __syncthreads();
    double* cur = ts;
    double* nxt = us;
    if (a.use_ginv) {
      for (int n = 1; n < N; ++n) {
        mode_prod_any(g, n, mats + moff[n], 0, cur, nxt);
        __syncthreads();
        double* t = cur; cur = nxt; nxt = t;
      }
    } else {
      for (int n = 1; n < N; ++n) {
        mode_prod_any(g, n, mats + moff[n], 1, cur, nxt);
        __syncthreads();
        double* t = cur; cur = nxt; nxt = t;
      }
      for (unsigned e = threadIdx.x; e < RT; e += BD) cur[e] *= dg[e];
      __syncthreads();
      for (int n = 0; n < N; ++n) {
        mode_prod_any(g, n, mats + moff[n], 0, cur, nxt);
        __syncthreads();
        double* t = cur; cur = nxt; nxt = t;
      }
    }
    const double* d = cur;
    int all = 1, div = 0;
    for (int q = 0; q < nrhs; ++q) {
      const int done = done_s[q];
      double dd = 0.0, xx = 0.0;
      for (unsigned r = threadIdx.x; r < (unsigned)g.Rtot; r += BD) {
        const unsigned e = r * nrhs + q;
        const double dv = d[e];
        double xv = xs[e];
        if (!done) { xv = fma(-a.eta, dv, xv); xs[e] = xv; }
        dd = fma(dv, dv, dd);
        xx = fma(xv, xv, xx);
      }
      dd = block_sum(dd, red);
      xx = block_sum(xx, red);
      if (!done) {
        const double dn = sqrt(dd), xn = sqrt(xx);
        const double rel = xn > 0.0 ? a.eta * dn / xn : (dn > 0.0 ? INFINITY : 0.0);
        const double d0 = it > 0 ? dn0_s[q] : dn;
        const bool bad = !isfinite(dn) || !isfinite(xn) || (it > 0 && dn > 1e6 * d0 && dn > 0.0);
        div |= bad;
        __syncthreads();
        if (threadIdx.x == 0) {
          if (it == 0) dn0_s[q] = dn;
          if (blockIdx.x == 0) {
            a.st->rel[q] = rel;
            if (it == 0) a.st->dnorm0[q] = dn;
            if (rel <= a.tol || bad) a.st->it_rhs[q] = it + 1;
          }
          if (rel <= a.tol || bad) done_s[q] = 1;
        }
        __syncthreads();
      }
      all &= done_s[q];
    }
    if (div || all) {
      if (threadIdx.x == 0 && blockIdx.x == 0 && div) a.st->diverged = 1;
      ++it;
      break;
    }
  }
  if (blockIdx.x == 0) {
    for (unsigned e = threadIdx.x; e < RT; e += BD) a.xout[e] = xs[e];
    if (threadIdx.x == 0) {
      a.st->iters = it;
      a.st->all_done = 1;
      for (int q = 0; q < nrhs; ++q) a.st->done[q] = done_s[q];
      if (aborted) a.st->diverged = 2;
    }
  }
}

// Row start of every level-1 node (rs1[S_1] = D): the first row of its subtree.
__global__ void __launch_bounds__(256) k_level1_rows(Geom g, Tree tr, int64_t* __restrict__ rs1) {
  const int64_t S1 = tr.cnt[1];
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s <= S1; s += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = s;
    for (int k = 1; k < g.N; ++k) v = tr.fchild[k][v];
    rs1[s] = v;
  }
}

template __global__ void k_richardson_persistent<8>(PArgs);
template __global__ void k_richardson_persistent<16>(PArgs);
template __global__ void k_richardson_persistent<32>(PArgs);
template __global__ void k_richardson_persistent<64>(PArgs);

}  // namespace kr
