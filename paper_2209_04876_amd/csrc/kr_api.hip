// C ABI of the library: handles, workspace, validation and the launch sequence
// of Algorithm 2 (FastKroneckerRegression) and of the exact KronMatMul
// baseline and loss.  Single translation unit: the kernel files are included.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "kr_internal.h"
#include "kr_setup.hip"
#include "kr_leverage.hip"
#include "kr_sketch.hip"
#include "kr_iter.hip"
#include "kr_stream.hip"
#include "kr_tucker.hip"
#include "kr_precond.hip"
#include "kr_batched.hip"

using namespace kr;

namespace {

struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Where one solve's sketch lives in the workspace: geometry (with the mode
// order of its tree), tables, tree, merged weights and multiplicities.
struct SketchRec {
  bool valid = false;
  Geom g{};
  ModeTables T{};
  Tree tr{};
  double* Omega = nullptr;
  int32_t* counts = nullptr;
  bool redraw = false;          // drawn by k_sample with (seed, stream), row 0
  uint64_t seed = 0, stream = 0;
};

}  // namespace

struct kr_handle_s {
  hipStream_t stream = nullptr;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* aux = nullptr;
  size_t aux_bytes = 0;
  void* als_zero = nullptr;       // zero core of kr_tucker_als's ||X||^2
  size_t als_zero_bytes = 0;
  IterState* h_state = nullptr;   // pinned
  int64_t* h_small = nullptr;     // pinned scratch (flags, counts)
  void* h_batch = nullptr;         // pinned staging of batched descriptors and results
  size_t h_batch_bytes = 0;
  // batched solves: the captured graph of the last KR_OPT_GRAPH call and its
  // signature, and the autotuned launch configuration per batch shape
  hipGraphExec_t bgraph = nullptr;
  std::vector<uint64_t> bgraph_sig;
  std::map<std::vector<int64_t>, std::pair<double, int>> tune;
  // iterations the last solve of a problem shape took (the first chunk of the next)
  std::map<std::vector<int64_t>, int> iter_hint;
  bool capturing = false;
  // side streams (default priority) over which a batched call spreads the
  // problems' setup and sketch, forked from and joined to the handle's stream
  hipStream_t side[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // last single solve's sketch (kr_export_sketch, kr_export_leverage) and every
  // problem's sketch of the last batched call (kr_export_batched_sketch); the
  // pointers reference the workspace, valid until the next call
  SketchRec last;
  std::vector<SketchRec> batch;
  // optional per-kernel timing with HIP events on the handle's stream
  bool prof_on = false;
  std::string prof_filter;
  std::unordered_map<const char*, bool> prof_hit;   // filter match per kernel-name literal
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof;
};

namespace {

hipEvent_t pool_event(kr_handle h) {
  if (h->ev_pool.empty()) {
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  hipEvent_t e = h->ev_pool.back();
  h->ev_pool.pop_back();
  return e;
}

// Records an event pair around one launch when profiling is enabled.
// Does kernel name n contain one of the '|'-separated alternatives of filter (an
// empty filter matches every kernel)?
static bool prof_match(const std::string& filter, const char* n) {
  if (filter.empty()) return true;
  size_t b = 0;
  while (b <= filter.size()) {
    size_t e = filter.find('|', b);
    if (e == std::string::npos) e = filter.size();
    if (e > b && std::strstr(n, filter.substr(b, e - b).c_str())) return true;
    b = e + 1;
  }
  return false;
}

// prof_match, cached per name literal (launch names are string literals), so
// that a profiled run's launches pay one hash lookup each.
static bool prof_wanted(kr_handle h, const char* n) {
  auto it = h->prof_hit.find(n);
  if (it != h->prof_hit.end()) return it->second;
  const bool hit = prof_match(h->prof_filter, n);
  h->prof_hit.emplace(n, hit);
  return hit;
}

struct ProfScope {
  kr_handle h;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(kr_handle h_, const char* n, hipStream_t s_) : h(h_), name(n), s(s_) {
    if (h->prof_on && !h->capturing && prof_wanted(h, n)) {
      a = pool_event(h);
      hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = pool_event(h);
      hipEventRecord(b, s);
      h->prof[name].push_back({a, b});
    }
  }
};

void prof_clear(kr_handle h) {
  for (auto& kv : h->prof)
    for (auto& pr : kv.second) {
      h->ev_pool.push_back(pr.first);
      h->ev_pool.push_back(pr.second);
    }
  h->prof.clear();
}

}  // namespace

// Events of a profiled launch (h->prof_on, name matching the filter); false when
// the launch is not profiled.
static bool prof_take(kr_handle h, const char* name, hipEvent_t* a, hipEvent_t* b) {
  if (!(h->prof_on && !h->capturing && prof_wanted(h, name))) return false;
  *a = pool_event(h);
  *b = pool_event(h);
  h->prof[name].push_back({*a, *b});
  return true;
}

// Launch with an explicit profiling name (for kernels instantiated per type); a
// profiled launch carries its two events in the dispatch itself
// (hipExtLaunchKernelGGL), so they time the kernel alone, without the dispatch
// gap that marker events around the launch would include.  Its host path is
// longer (4-6% per bf16 solve when every launch is profiled), so callers profile
// a few solves, not the whole timed stretch.
#define KLN(h, name, kern, grid, block, shm, strm, ...)                          \
  do {                                                                         \
    hipEvent_t _pa = nullptr, _pb = nullptr;                                   \
    if (prof_take((h), (name), &_pa, &_pb)) {                                  \
      hipExtLaunchKernelGGL(kern, grid, block, shm, strm, _pa, _pb, 0u,        \
                            __VA_ARGS__);                                      \
    } else                                                                     \
      hipLaunchKernelGGL(kern, grid, block, shm, strm, __VA_ARGS__);           \
  } while (0)

#define KL(h, kern, ...) KLN(h, #kern, kern, __VA_ARGS__)

#define KR_FAIL(h, code, ...)                                   \
  do {                                                          \
    char _b[512];                                               \
    snprintf(_b, sizeof(_b), __VA_ARGS__);                      \
    (h)->err = _b;                                              \
    return (code);                                              \
  } while (0)

#define HIPCHK(h, expr)                                                          \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess)                                                        \
      KR_FAIL(h, KR_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));        \
  } while (0)

static int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

// workgroups of the rows kernel at most (4 waves each; 1280 and 2048 measured no better)
#ifndef KR_ROWS_GRID_CAP
#define KR_ROWS_GRID_CAP 1024
#endif
#ifndef KR_ROWS_LDS_GRID
#define KR_ROWS_LDS_GRID 512    // two workgroups of 512 threads per CU for the LDS-staged rows kernel
#endif
static int64_t grid_for(int64_t work, int64_t threads, int64_t cap = 4096) {
  int64_t b = (work + threads - 1) / threads;
  return std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

static kr_status ensure(kr_handle h, void** buf, size_t* cap, size_t need) {
  if (need <= *cap) return KR_OK;
  if (*buf) {
    hipStreamSynchronize(h->stream);
    hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
  }
  size_t want = std::max(need, size_t(64) << 20);
  if (hipMalloc(buf, want) != hipSuccess) {
    *buf = nullptr;
    KR_FAIL(h, KR_ENOMEM, "device workspace of %zu bytes could not be allocated", want);
  }
  *cap = want;
  h->last.valid = false;
  h->batch.clear();
  return KR_OK;
}

// Validate a problem and fill the geometry (m set by the caller).
static kr_status make_geom(kr_handle h, const kr_problem* p, Geom* g) {
  if (!p) KR_FAIL(h, KR_EINVAL, "problem is NULL");
  if (p->N < 1 || p->N > KR_MAX_MODES) KR_FAIL(h, KR_EINVAL, "N=%d outside 1..%d", p->N, KR_MAX_MODES);
  if (p->nrhs < 1 || p->nrhs > KR_MAX_RHS) KR_FAIL(h, KR_EINVAL, "nrhs=%d outside 1..%d", p->nrhs, KR_MAX_RHS);
  if (p->a_dtype != KR_F64 && p->a_dtype != KR_F32) KR_FAIL(h, KR_EINVAL, "bad a_dtype");
  if (p->b_dtype != KR_F64 && p->b_dtype != KR_F32) KR_FAIL(h, KR_EINVAL, "bad b_dtype");
  std::memset(g, 0, sizeof(*g));
  g->N = p->N;
  g->nrhs = p->nrhs;
  int64_t Rtot = 1, Itot = 1;
  for (int n = 0; n < p->N; ++n) {
    if (!p->A[n]) KR_FAIL(h, KR_EINVAL, "A[%d] is NULL", n);
    if (p->R[n] < 1 || p->R[n] > 64) KR_FAIL(h, KR_EUNSUPPORTED, "R[%d]=%lld outside 1..64", n, (long long)p->R[n]);
    if (p->I[n] < p->R[n]) KR_FAIL(h, KR_EINVAL, "I[%d]=%lld < R[%d]=%lld", n, (long long)p->I[n], n, (long long)p->R[n]);
    if (p->I[n] > (int64_t(1) << 24)) KR_FAIL(h, KR_EUNSUPPORTED, "I[%d] > 2^24", n);
    g->I[n] = (int)p->I[n];
    g->R[n] = (int)p->R[n];
    Rtot *= p->R[n];
    Itot *= p->I[n];
    if (Itot > (int64_t(1) << 46)) KR_FAIL(h, KR_EUNSUPPORTED, "prod(I) too large");
  }
  if (Rtot * p->nrhs > (int64_t(1) << 26)) KR_FAIL(h, KR_EUNSUPPORTED, "prod(R)*nrhs too large");
  g->Rtot = Rtot;
  g->Itot = Itot;
  g->rsuf[p->N] = 1;
  for (int k = p->N - 1; k >= 0; --k) g->rsuf[k] = g->rsuf[k + 1] * g->R[k];
  int kb = 0;
  for (int n = 0; n < p->N; ++n) {
    g->bits[n] = std::max(1, ceil_log2(g->I[n]));
    kb += g->bits[n];
  }
  if (kb > 64) KR_FAIL(h, KR_EUNSUPPORTED, "packed row key needs %d > 64 bits", kb);
  g->keybits = kb;
  g->shift[p->N - 1] = 0;
  for (int n = p->N - 2; n >= 0; --n) g->shift[n] = g->shift[n + 1] + g->bits[n + 1];
  for (int k = 1; k <= p->N; ++k) g->lshift[k] = g->shift[k - 1];
  g->lshift[0] = kb;
  for (int n = 0; n < p->N; ++n) g->orig[n] = g->inv[n] = n;
  return KR_OK;
}

// Device scratch of the allocation-free entry point: one copy per device, held
// until the process ends.  Host code never uses the array's name as an address
// (it is a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, fetched once per device (at kr_create, or on the
// entry point's first call on a device) and kept in g_scratch_ptr.
#define KR_SCRATCH_BYTES (size_t(64) << 20)
#define KR_SCRATCH_DEVICES 64
static __device__ __align__(256) char kr_scratch[KR_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[KR_SCRATCH_DEVICES] = {};

static kr_status scratch_address(kr_handle h, void** out) {
  int dev = 0;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= KR_SCRATCH_DEVICES) KR_FAIL(h, KR_EUNSUPPORTED, "device %d has no scratch slot", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(kr_scratch));
    if (e != hipSuccess || !p)
      KR_FAIL(h, KR_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KR_OK;
}

extern "C" {

const char* kr_version(void) { return "kron_regress gfx950 0.2"; }

kr_status kr_create(kr_handle* out, void* stream) {
  if (!out) return KR_EINVAL;
  kr_handle h = new kr_handle_s();
  h->stream = (hipStream_t)stream;
  if (hipHostMalloc((void**)&h->h_state, sizeof(IterState)) != hipSuccess ||
      hipHostMalloc((void**)&h->h_small, 64 * sizeof(int64_t)) != hipSuccess) {
    delete h;
    return KR_ENOMEM;
  }
  // the scratch address of the current device (the entry point fetches it on its
  // first call on another device; a failure here is reported by that call)
  void* sp = nullptr;
  (void)scratch_address(h, &sp);
  h->err.clear();
  *out = h;
  return KR_OK;
}

kr_status kr_destroy(kr_handle h) {
  if (!h) return KR_EINVAL;
  hipStreamSynchronize(h->stream);
  prof_clear(h);
  for (hipEvent_t e : h->ev_pool) hipEventDestroy(e);
  if (h->ws) hipFree(h->ws);
  if (h->aux) hipFree(h->aux);
  if (h->als_zero) hipFree(h->als_zero);
  if (h->h_state) hipHostFree(h->h_state);
  if (h->h_small) hipHostFree(h->h_small);
  if (h->h_batch) hipHostFree(h->h_batch);
  if (h->bgraph) hipGraphExecDestroy(h->bgraph);
  for (int k = 0; k < 4; ++k) {
    if (h->side[k]) hipStreamDestroy(h->side[k]);
    if (h->join_ev[k]) hipEventDestroy(h->join_ev[k]);
  }
  if (h->fork_ev) hipEventDestroy(h->fork_ev);
  delete h;
  return KR_OK;
}

kr_status kr_set_stream(kr_handle h, void* stream) {
  if (!h) return KR_EINVAL;
  h->stream = (hipStream_t)stream;
  return KR_OK;
}

const char* kr_last_error(kr_handle h) { return h ? h->err.c_str() : "null handle"; }

kr_status kr_profile_enable(kr_handle h, int32_t enable, const char* filter) {
  if (!h) return KR_EINVAL;
  hipStreamSynchronize(h->stream);
  prof_clear(h);
  h->prof_on = enable != 0;
  h->prof_filter = filter ? filter : "";
  h->prof_hit.clear();
  // events are created here rather than inside a profiled (timed) stretch
  if (h->prof_on)
    while (h->ev_pool.size() < 4096) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      h->ev_pool.push_back(e);
    }
  return KR_OK;
}

kr_status kr_profile_list(kr_handle h, char* h_buf, int64_t cap) {
  if (!h || !h_buf || cap < 1) return KR_EINVAL;
  std::string all;
  for (auto& kv : h->prof) {
    all += kv.first;
    all += '\n';
  }
  const size_t n = std::min<size_t>(all.size(), (size_t)cap - 1);
  std::memcpy(h_buf, all.data(), n);
  h_buf[n] = 0;
  return all.size() + 1 > (size_t)cap ? KR_EINVAL : KR_OK;
}

kr_status kr_profile_query(kr_handle h, const char* kernel, int64_t* launches, double* total_ms) {
  if (!h || !kernel) return KR_EINVAL;
  auto it = h->prof.find(kernel);
  int64_t n = 0;
  double tot = 0.0;
  if (it != h->prof.end()) {
    for (auto& pr : it->second) {
      HIPCHK(h, hipEventSynchronize(pr.second));
      float ms = 0.f;
      HIPCHK(h, hipEventElapsedTime(&ms, pr.first, pr.second));
      tot += ms;
      ++n;
    }
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = tot;
  return KR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Setup shared by the solvers and the exact baseline: FP64 factors, Gram
// eigen-decompositions, leverage scores, quantised weights and CDFs.
// ---------------------------------------------------------------------------
struct SetupBufs {
  double* A64[KR_MAXN];
  double* gram;
  int32_t* flags;
  // large-factor passes (see setup_large): per-block sums of the row passes and
  // of the integer weights, per-block argmax keys, per-block partial Grams (exact
  // route) or the spectral approximations and projections (approximate route)
  double* lpart[KR_MAXN];
  double* lpart2[KR_MAXN];
  uint64_t* qpart[KR_MAXN];
  uint64_t* qbest[KR_MAXN];
  double* gpart[KR_MAXN];
  double* At[KR_MAXN];
  double* Z[KR_MAXN];
};

// Factors with more rows than this, and every factor of an approximate-leverage
// solve, take the many-workgroup setup passes of kr_leverage.hip.
#define LV_SMALL_I 16384

static bool setup_large(const Geom& g) {
  if (g.approx) return true;
  for (int n = 0; n < g.N; ++n)
    if (g.I[n] > LV_SMALL_I) return true;
  return false;
}

static int lv_blocks(int I) { return (I + LV_RPB - 1) / LV_RPB; }

static void carve_setup(Arena& a, const Geom& g, ModeTables* T, SetupBufs* s) {
  for (int n = 0; n < g.N; ++n) {
    s->A64[n] = a.take<double>((size_t)g.I[n] * g.R[n]);
    T->A[n] = s->A64[n];
    T->V[n] = a.take<double>((size_t)g.R[n] * g.R[n]);
    T->evals[n] = a.take<double>(g.R[n]);
    T->Ginv[n] = a.take<double>((size_t)g.R[n] * g.R[n]);
    T->lev[n] = a.take<double>(g.I[n]);
    T->Q[n] = a.take<uint64_t>(g.I[n]);
    T->C[n] = a.take<uint64_t>(g.I[n]);
  }
  s->gram = a.take<double>((size_t)g.N * 64 * 64);
  s->flags = a.take<int32_t>(64);
  for (int n = 0; n < KR_MAXN; ++n)
    s->lpart[n] = s->lpart2[n] = nullptr, s->qpart[n] = s->qbest[n] = nullptr,
    s->gpart[n] = s->At[n] = s->Z[n] = nullptr;
  if (!setup_large(g)) return;
  for (int n = 0; n < g.N; ++n) {
    const int nb = lv_blocks(g.I[n]);
    s->lpart[n] = a.take<double>(nb);
    s->lpart2[n] = a.take<double>(nb);
    s->qpart[n] = a.take<uint64_t>(nb);
    s->qbest[n] = a.take<uint64_t>(nb);
    if (g.approx) {
      s->At[n] = a.take<double>((size_t)g.lev_k[n] * g.R[n]);
      s->Z[n] = a.take<double>((size_t)g.lev_r * g.R[n]);
    } else {
      s->gpart[n] = a.take<double>((size_t)nb * g.R[n] * g.R[n]);
    }
  }
}

static size_t setup_bytes(const Geom& g) {
  size_t b = 0;
  for (int n = 0; n < g.N; ++n)
    b += 8 * ((size_t)g.I[n] * g.R[n] + 2 * (size_t)g.R[n] * g.R[n] + g.R[n] + 3 * (size_t)g.I[n]) + 7 * 256;
  if (setup_large(g))
    for (int n = 0; n < g.N; ++n) {
      const size_t nb = lv_blocks(g.I[n]);
      b += 32 * nb + 4 * 256;
      b += g.approx ? 8 * ((size_t)g.lev_k[n] * g.R[n] + (size_t)g.lev_r * g.R[n]) + 2 * 256
                    : 8 * nb * g.R[n] * g.R[n] + 256;
    }
  return b + 8 * (size_t)g.N * 4096 + 1024;
}

// FP64 copies of every factor (one launch; blockIdx.y is the mode).
static void launch_promote(kr_handle h, const kr_problem* p, const Geom& g, double* const* dst, int32_t* flags,
                           hipStream_t s) {
  PromoteArgs pa{};
  int64_t cmax = 1;
  for (int n = 0; n < g.N; ++n) {
    pa.src[n] = p->A[n];
    pa.dst[n] = dst[n];
    pa.cnt[n] = (int64_t)g.I[n] * g.R[n];
    cmax = std::max(cmax, pa.cnt[n]);
  }
  KL(h, k_promote_all, dim3(grid_for(cmax, 256, 1024), g.N), dim3(256), 0, s, pa, p->a_dtype, flags);
}

// The Gram matrices' eigen-decomposition (eig) or Cholesky factor (lambda = 0
// solves that need only G^{-1}).
static void launch_factor(kr_handle h, const Geom& g, const ModeTables& T, const SetupBufs& s, bool eig, int maxR) {
  if (eig) {
    KL(h, k_eig, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  } else if (maxR <= 8) {
    KLN(h, "k_chol<8>", k_chol<8>, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  } else if (maxR <= 16) {
    KLN(h, "k_chol<16>", k_chol<16>, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  } else if (maxR <= 32) {
    KLN(h, "k_chol_wide<32>", k_chol_wide<32>, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  } else {
    KLN(h, "k_chol_wide<64>", k_chol_wide<64>, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  }
}

template <int RM>
static void launch_quadform(kr_handle h, const Geom& g, const LevPass& lp) {
  int nbmax = 1;
  for (int n = 0; n < g.N; ++n) nbmax = std::max(nbmax, lv_blocks(g.I[n]));
  KLN(h, "k_row_quadform", k_row_quadform<RM>, dim3(nbmax, g.N), dim3(LV_THREADS), 0, h->stream, lp);
}

// The integer weights and CDF of every mode from the weights T.lev and their
// per-block sums s.lpart (many workgroups per mode).
static void launch_quantise(kr_handle h, const Geom& g, const ModeTables& T, const SetupBufs& s,
                            bool second = false) {
  QuantPass qp{};
  int nbmax = 1;
  for (int n = 0; n < g.N; ++n) {
    qp.w[n] = T.lev[n];
    qp.part[n] = second ? s.lpart2[n] : s.lpart[n];
    qp.Q[n] = T.Q[n];
    qp.C[n] = T.C[n];
    qp.qpart[n] = s.qpart[n];
    qp.qbest[n] = s.qbest[n];
    qp.I[n] = g.I[n];
    qp.nb[n] = lv_blocks(g.I[n]);
    nbmax = std::max(nbmax, qp.nb[n]);
  }
  KL(h, k_quant_blocks, dim3(nbmax, g.N), dim3(LV_THREADS), 0, h->stream, qp, s.flags);
  KL(h, k_quant_fix, dim3(1), dim3(64), 0, h->stream, qp, g.N, s.flags);
  KL(h, k_cdf_blocks, dim3(nbmax, g.N), dim3(LV_THREADS), 0, h->stream, qp);
}

// Setup of large factors (or approximate leverage) on many workgroups per mode.
// Exact route: partial Grams summed in block order, the eigen-decomposition or
// Cholesky factor, then l_i = sum_k (a_i . v_k)^2 / lambda_k.  Approximate route
// (Algorithm 2's first loop): squared row norms and their tables, k_n rows of the
// spectral approximation A~, the eigen-decomposition of A~^T A~ (the
// preconditioner's V and Sigma), the projection Z = (G / sqrt(r)) A~ M, and the
// scores ||Z a_i||^2 / ((1 + eps/4)(1 - eps/20)).  Then the integer weights and CDF.
static kr_status launch_setup_large(kr_handle h, const Geom& g, const ModeTables& T, const SetupBufs& s,
                                    bool leverage, bool eig, uint64_t seed, uint64_t stream) {
  int maxR = 1, nbmax = 1;
  for (int n = 0; n < g.N; ++n) {
    maxR = std::max<int>(maxR, (int)g.R[n]);
    nbmax = std::max(nbmax, lv_blocks(g.I[n]));
  }
  auto quadform = [&](const LevPass& lp) {
    if (maxR <= 8) launch_quadform<8>(h, g, lp);
    else if (maxR <= 16) launch_quadform<16>(h, g, lp);
    else if (maxR <= 32) launch_quadform<32>(h, g, lp);
    else launch_quadform<64>(h, g, lp);
  };
  LevPass lp{};
  for (int n = 0; n < g.N; ++n) {
    lp.A[n] = T.A[n];
    lp.out[n] = T.lev[n];
    lp.part[n] = s.lpart[n];
    lp.I[n] = g.I[n];
    lp.R[n] = g.R[n];
  }
  if (!g.approx) {
    GramPass gp{};
    for (int n = 0; n < g.N; ++n) {
      gp.A[n] = T.A[n];
      gp.part[n] = s.gpart[n];
      gp.I[n] = g.I[n];
      gp.R[n] = g.R[n];
      gp.nb[n] = lv_blocks(g.I[n]);
    }
    gp.gram = s.gram;
    KL(h, k_gram_part, dim3(nbmax, g.N), dim3(256), 0, h->stream, gp);
    KL(h, k_gram_sum, dim3(g.N), dim3(256), 0, h->stream, gp);
    launch_factor(h, g, T, s, eig, maxR);
    if (!leverage) return KR_OK;
    lp.mode = 1;
    for (int n = 0; n < g.N; ++n) {
      lp.P[n] = T.V[n];
      lp.evals[n] = T.evals[n];
      lp.ldr[n] = g.R[n];
      lp.ldc[n] = 1;
      lp.nc[n] = g.R[n];
    }
    quadform(lp);
    launch_quantise(h, g, T, s);
    HIPCHK(h, hipGetLastError());
    return KR_OK;
  }
  // approximate route: squared row norms, mixed with the uniform distribution ->
  // their tables -> rows of A~
  lp.mode = 0;
  quadform(lp);
  {
    MixPass mp{};
    for (int n = 0; n < g.N; ++n) {
      mp.w[n] = T.lev[n];
      mp.part_in[n] = s.lpart[n];
      mp.part_out[n] = s.lpart2[n];
      mp.I[n] = g.I[n];
      mp.nb[n] = lv_blocks(g.I[n]);
    }
    KL(h, k_mix_uniform, dim3(nbmax, g.N), dim3(LV_THREADS), 0, h->stream, mp);
  }
  launch_quantise(h, g, T, s, true);
  ApproxRows ar{};
  int kmax = 1;
  for (int n = 0; n < g.N; ++n) {
    ar.A[n] = T.A[n];
    ar.Q[n] = T.Q[n];
    ar.C[n] = T.C[n];
    ar.At[n] = s.At[n];
    ar.I[n] = g.I[n];
    ar.R[n] = g.R[n];
    ar.k[n] = g.lev_k[n];
    kmax = std::max(kmax, g.lev_k[n]);
  }
  KL(h, k_approx_rows, dim3((kmax + 255) / 256, g.N), dim3(256), 0, h->stream, ar, seed, stream);
  // N_n = A~^T A~ (the k_n rows of A~ as a factor) and its eigen-decomposition
  {
    Geom ga = g;
    ModeTables Ta = T;
    for (int n = 0; n < g.N; ++n) {
      ga.I[n] = g.lev_k[n];
      Ta.A[n] = s.At[n];
    }
    KL(h, k_gram, dim3(g.N), dim3(256), 0, h->stream, Ta, ga, s.gram);
  }
  KL(h, k_eig, dim3(g.N), dim3(64), 0, h->stream, T, g, (const double*)s.gram, s.flags);
  if (!leverage) return KR_OK;
  JLPass jp{};
  for (int n = 0; n < g.N; ++n) {
    jp.At[n] = s.At[n];
    jp.Ninv[n] = T.Ginv[n];
    jp.Z[n] = s.Z[n];
    jp.R[n] = g.R[n];
    jp.k[n] = g.lev_k[n];
  }
  jp.r = g.lev_r;
  jp.coef = 1.0 + g.lev_eps / 4.0;
  if (maxR <= 8) KLN(h, "k_jl_project", k_jl_project<8>, dim3(g.lev_r, g.N), dim3(256), 0, h->stream, jp, seed, stream);
  else if (maxR <= 16) KLN(h, "k_jl_project", k_jl_project<16>, dim3(g.lev_r, g.N), dim3(256), 0, h->stream, jp, seed, stream);
  else if (maxR <= 32) KLN(h, "k_jl_project", k_jl_project<32>, dim3(g.lev_r, g.N), dim3(256), 0, h->stream, jp, seed, stream);
  else KLN(h, "k_jl_project", k_jl_project<64>, dim3(g.lev_r, g.N), dim3(256), 0, h->stream, jp, seed, stream);
  lp.mode = 2;
  lp.wscale = 1.0 / ((1.0 + g.lev_eps / 4.0) * (1.0 - g.lev_eps / 20.0));
  for (int n = 0; n < g.N; ++n) {
    lp.P[n] = s.Z[n];
    lp.ldr[n] = 1;
    lp.ldc[n] = g.R[n];
    lp.nc[n] = g.lev_r;
  }
  quadform(lp);
  launch_quantise(h, g, T, s);
  HIPCHK(h, hipGetLastError());
  return KR_OK;
}

// Factor setup: float64 copies, Grams, then the eigen-decomposition (eig) or, when
// only G^{-1} is needed (lambda = 0 solves), the Cholesky route; then the
// leverage tables.  Large factors and approximate leverage take launch_setup_large.
static kr_status launch_setup(kr_handle h, const kr_problem* p, const Geom& g, const ModeTables& T,
                              const SetupBufs& s, bool leverage, bool eig = true, uint64_t seed = 0,
                              uint64_t stream = 0) {
  KL(h, k_zero_bytes, dim3(1), dim3(64), 0, h->stream, (uint32_t*)s.flags, (int64_t)64);
  launch_promote(h, p, g, s.A64, s.flags, h->stream);
  if (setup_large(g)) return launch_setup_large(h, g, T, s, leverage, eig || g.approx, seed, stream);
  KL(h, k_gram, dim3(g.N), dim3(256), 0, h->stream, T, g, s.gram);
  int maxR = 1;
  for (int n = 0; n < g.N; ++n) maxR = std::max<int>(maxR, (int)g.R[n]);
  launch_factor(h, g, T, s, eig, maxR);
  if (leverage) {
    if (maxR <= 8) KLN(h, "k_leverage<8>", k_leverage<8>, dim3(g.N), dim3(256), 0, h->stream, T, g, s.flags);
    else if (maxR <= 16) KLN(h, "k_leverage<16>", k_leverage<16>, dim3(g.N), dim3(256), 0, h->stream, T, g, s.flags);
    else if (maxR <= 32) KLN(h, "k_leverage<32>", k_leverage<32>, dim3(g.N), dim3(256), 0, h->stream, T, g, s.flags);
    else KLN(h, "k_leverage<64>", k_leverage<64>, dim3(g.N), dim3(256), 0, h->stream, T, g, s.flags);
  }
  HIPCHK(h, hipGetLastError());
  return KR_OK;
}

// ---------------------------------------------------------------------------
// Algorithm 2
// ---------------------------------------------------------------------------
struct SolveBufs {
  SetupBufs s;
  uint64_t* keys;
  uint64_t* keys_alt;
  uint32_t* hist;
  int64_t* tiletot;
  double* Omega;
  double* bD;
  int32_t* counts;
  double* P[KR_MAXN + 1];
  double* Q[KR_MAXN + 1];
  double* t0;
  double* t1;
  double* dinv;
  double* part;
  IterState* state;
  Chunks ck;      // fused three-mode pass (ck.cap = 0: not carved)
  void* Q1c;      // its per-chunk level-1 adjoints (float64 or float32)
};

static int64_t level_cap(const Geom& g, int k) {
  // level k holds distinct prefixes of length k: at most min(m, prod_{n<k} I_n)
  if (k == 0) return 1;
  double prod = 1.0;
  for (int n = 0; n < k; ++n) prod *= (double)g.I[n];
  return (int64_t)std::min<double>((double)g.m, prod);
}

// The fused three-mode pass (k_subtree3): three factors without segment roots,
// R_2 <= 16 (one lane group per row), its LDS (P_1, and the factor rows and
// Q_2 of at most ch children) within 48 KB, and at most 65536 level-1 nodes
// (the chunk table is one workgroup's scan).
#ifndef KR_FUSED_RUN
#define KR_FUSED_RUN 8     // (node, rhs) tasks per run of the fused pass
#endif
static int fused3_ch(const Geom& g) { return std::max(1, KR_FUSED_RUN / g.nrhs); }
static size_t fused3_lds(const Geom& g, size_t elem) {
  const size_t W2 = (size_t)g.R[2] * g.nrhs;
  return 8 * (size_t)g.R[1] * W2 + elem * (size_t)fused3_ch(g) * ((size_t)g.R[1] + W2);
}
static bool fused3_eligible(const Geom& g) {
  return g.N == 3 && !g.seg_root && g.R[2] <= 16 && (int64_t)g.R[1] * g.R[2] * g.nrhs <= 4096 &&
         (int64_t)g.R[2] * g.nrhs <= 256 && fused3_lds(g, 8) <= 48 * 1024 && level_cap(g, 1) <= 65536;
}
// Chunks the table may hold: beyond about two per level-1 node the root adjoint
// over the chunks costs more than the adjoint level it replaces, and the
// level-wise passes are used.
static int64_t fused3_cap(const Geom& g) {
  const int64_t ch = fused3_ch(g);
  return std::min<int64_t>(level_cap(g, 1) + (level_cap(g, 2) + ch - 1) / ch, 2 * level_cap(g, 1) + 4096);
}

// Partial blocks of the root adjoint (see root_npb): one per 32 level-1 nodes,
// and up to 64 when the fused pass's chunks take their place.
static int64_t part_blocks(const Geom& g) {
  const int64_t b = (level_cap(g, 1) + 31) / 32;
  return fused3_eligible(g) ? std::max<int64_t>(b, 64) : b;
}

// Workspace of one solve.  lean: the batched team's layout, which never forms
// the level-(N-1) products (N >= 3) nor the single-problem iteration's row and
// partial-sum buffers.
// Key tiles up to which each scatter workgroup forms its own offsets from the
// raw histogram (reading all of it) instead of a scan launch.
#ifndef SORT_OWN_SCAN_TILES
#define SORT_OWN_SCAN_TILES 128
#endif

// Words of the sort's histogram buffer for nblocks key tiles: SORT_DIGITS_MAX
// counts per tile, then the tile totals of the many-workgroup scan.
static size_t hist_words(int64_t nblocks) {
  const size_t nh = (size_t)SORT_DIGITS_MAX * nblocks;
  return nh + (nh + SCANP_TILE - 1) / SCANP_TILE + 16;
}

// Tiles of the tree kernels over m sorted keys (tiletot holds KR_MAXN + 1 counts
// per tile).
static int tree_tiles(int64_t m) { return (int)((m + TREE_TILE - 1) / TREE_TILE); }

static size_t solve_bytes(const Geom& g, int ntiles, int nblocks, bool lean = false) {
  size_t b = setup_bytes(g);
  b += 2 * 8 * (size_t)g.m + 4 * hist_words(nblocks) + 8 * (size_t)ntiles * (KR_MAXN + 1);
  const int64_t D = level_cap(g, g.N);
  b += (size_t)D * (8 + 8 * g.nrhs + 4);
  for (int k = 1; k <= g.N; ++k) b += 3 * 4 * (size_t)(level_cap(g, k) + 2) + 8 * (size_t)level_cap(g, k) * g.R[k - 1] + 1024;
  b += 4 * (size_t)(D + 2) + 8 * (size_t)D;
  for (int k = 1; k < g.N; ++k)
    if (!(lean && g.N >= 3 && k == g.N - 1)) b += 2 * 8 * (size_t)level_cap(g, k) * g.rsuf[k] * g.nrhs + 512;
  b += 3 * 8 * (size_t)g.Rtot * g.nrhs + 8 * (size_t)g.Rtot + sizeof(IterState) + 8 * (KR_MAXN + 2) + 768;
  if (lean) return b + 8 * (size_t)(level_cap(g, 1) + 2) + 64 * 256 + 8192;
  b += 8 * (size_t)D * g.nrhs + 8 * (size_t)(level_cap(g, 1) + 2) + 512;
  b += 8 * (size_t)part_blocks(g) * g.Rtot * g.nrhs + 512;
  if (fused3_eligible(g)) {
    const size_t c = (size_t)fused3_cap(g);
    b += 8 * (c + 2) + 12 * c * g.R[0] + 8 * c * (size_t)g.R[1] * g.R[2] * g.nrhs + 6 * 256;
  }
  for (int k = 1; k < g.N; ++k) b += 4 * (size_t)level_cap(g, k) * g.R[k - 1] + 256;
  return b + 64 * 256 + 4096;
}


// Stable LSD radix sort of the g.m packed keys (9-bit digits when that takes
// fewer passes over g.keybits than 8-bit digits and the tiles are few, else
// 8-bit) and the per-level run-length encoding into the sample tree.
static void launch_sort_tree(kr_handle h, const Geom& g, uint64_t* keys, uint64_t* keys_alt, uint32_t* hist,
                             int64_t* tiletot, int nblocks, const Tree& tr) {
  hipStream_t s = h->stream;
  const int64_t m = g.m;
  uint64_t* kin = keys;
  uint64_t* kout = keys_alt;
  // 9-bit digits when they take fewer passes over g.keybits than 8-bit ones.
  // Measured: at 340k keys (27-bit) three 9-bit passes beat four 8-bit ones by
  // ~1.5% of the whole solve (three fewer launch triples), although the kernels
  // alone take about as long.  The histogram scan is one workgroup while it is
  // one tile, else many (k_scan_part, k_scan_tiles).
  const int rb = (g.keybits + 8) / 9 < (g.keybits + 7) / 8 ? 9 : 8;
  uint32_t* part = hist + (size_t)SORT_DIGITS_MAX * nblocks;
  auto scan = [&](int64_t nh) {
    if (nh <= 1024 * SCAN_K) {
      KL(h, k_scan_u32, dim3(1), dim3(1024), 0, s, hist, nh);
    } else {
      const int nt = (int)((nh + SCANP_TILE - 1) / SCANP_TILE);
      KL(h, k_scan_part, dim3(nt), dim3(SCANP_THREADS), 0, s, (const uint32_t*)hist, nh, part);
      KL(h, k_scan_tiles, dim3(nt), dim3(SCANP_THREADS), 0, s, hist, nh, (const uint32_t*)part);
    }
  };
  // With few tiles every scatter workgroup reads the whole histogram and forms
  // its own offsets, in place of a scan launch.
  const bool own = nblocks <= SORT_OWN_SCAN_TILES;
  for (int sh = 0; sh < g.keybits; sh += rb) {
    if (rb == 9 && own) {
      KLN(h, "k_radix_hist", (k_radix_hist<9, true>), dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, m, sh, hist, nblocks);
      KLN(h, "k_radix_scatter", (k_radix_scatter<9, true>), dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, kout, m, sh,
          hist, nblocks);
    } else if (rb == 9) {
      KLN(h, "k_radix_hist", k_radix_hist<9>, dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, m, sh, hist, nblocks);
      scan((int64_t)512 * nblocks);
      KLN(h, "k_radix_scatter", k_radix_scatter<9>, dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, kout, m, sh, hist,
          nblocks);
    } else if (own) {
      KLN(h, "k_radix_hist", (k_radix_hist<8, true>), dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, m, sh, hist, nblocks);
      KLN(h, "k_radix_scatter", (k_radix_scatter<8, true>), dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, kout, m, sh,
          hist, nblocks);
    } else {
      KLN(h, "k_radix_hist", k_radix_hist<8>, dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, m, sh, hist, nblocks);
      scan((int64_t)256 * nblocks);
      KLN(h, "k_radix_scatter", k_radix_scatter<8>, dim3(nblocks), dim3(SORT_THREADS), 0, s, kin, kout, m, sh, hist,
          nblocks);
    }
    std::swap(kin, kout);
  }
  const int ntree = tree_tiles(m);
  KL(h, k_tree_count, dim3(ntree), dim3(SORT_THREADS), 0, s, kin, g, tiletot);
  KL(h, k_tree_scan, dim3(1), dim3(64 * g.N), 0, s, tiletot, ntree, g, tr);
  KL(h, k_tree_sentinels, dim3(1), dim3(64), 0, s, g, tr);
  KL(h, k_tree_emit, dim3(ntree), dim3(SORT_THREADS), 0, s, kin, g, tiletot, tr);
}

// Nodes per root-adjoint block (a multiple of RA_NODES): all level-1 nodes in one
// block up to 2048 of them (the root adjoint then writes g itself), else at most
// 64 blocks, which the preconditioner kernel sums.  Needs tr.ncnt.
static int root_npb(const Tree& tr) {
  // up to 2048 level-1 nodes: about four partial blocks of at least 128 nodes
  // (their sum costs the preconditioner little, and the root adjoint spreads
  // over more workgroups); beyond, 64 blocks
#ifndef KR_ROOT_BLOCKS
#define KR_ROOT_BLOCKS 4   // partial blocks of the root adjoint up to 2048 level-1 nodes
#endif
  const int64_t S1 = std::max<int64_t>(1, tr.ncnt[1]);
  const int64_t per = S1 <= 2048 ? std::max<int64_t>(std::min<int64_t>(S1, 512 / KR_ROOT_BLOCKS),
                                                      (S1 + KR_ROOT_BLOCKS - 1) / KR_ROOT_BLOCKS)
                                 : (S1 + 63) / 64;
  return (int)(RA_NODES * ((per + RA_NODES - 1) / RA_NODES));
}

// The rows kernel reads the last mode's factor from LDS (rows stream 4-byte
// indices, not materialised factor rows) when that factor fits 64 KB and the
// distinct rows outnumber its rows 16 times (staging it once per workgroup then
// costs little against the row traffic it saves).  Needs tr.ncnt.
#ifndef KR_ROWS_LDS_MAX
#define KR_ROWS_LDS_MAX (64 * 1024)
#endif
static bool rows_ldsf(const Geom& g, const Tree& tr) {
  const int64_t IL = g.I[g.N - 1];
  return IL * g.R[g.N - 1] * 8 <= KR_ROWS_LDS_MAX && tr.ncnt[g.N] >= 16 * IL;
}
#ifndef KR_MULTI_ROWS
#define KR_MULTI_ROWS 6
#endif
// Padded row width of the lane-per-row kernel (k_rows_lane), 0 where it does not
// apply: R_{N-1} <= 16 and the factor zero-padded to 8 or 16 columns fits the
// same LDS budget.
static int rows_lane_width(const Geom& g, const Tree& tr) {
  const int Rl = g.R[g.N - 1];
  const int RP = Rl <= 8 ? 8 : 16;
  if (Rl > 16 || !rows_ldsf(g, tr) || (int64_t)g.I[g.N - 1] * RP * 8 > KR_ROWS_LDS_MAX) return 0;
  return RP;
}

// One pass of the sampled products K~^T Omega (K~ x - b~) down and up the sample
// tree: forward levels 1..N-2, the last forward level with the rows and the last
// adjoint level, and adjoint levels N-1..2.  Returns whether the root adjoint
// (launch_root) follows: without segment roots and for N >= 2 (for N = 1 the rows
// write Q[0]; with segment roots the level-1 adjoints are the per-segment
// gradients).  P[0] is the iterate; Q[k] holds the adjoint type T (float64, or
// float32 in the refined precisions).
template <typename T>
static bool launch_level_products(kr_handle h, const ModeTables& TT, const Geom& g, const Tree& tr, double* const* P,
                                  void* const* Qv, const double* Omega, const double* bD, const IterState* state) {
  hipStream_t s = h->stream;
  T* Q[KR_MAXN + 1];
  for (int k = 0; k <= KR_MAXN; ++k) Q[k] = (T*)Qv[k];
  const bool f32 = sizeof(T) == 4;
  const int Rl = g.R[g.N - 1];
  const int G = Rl <= 8 ? 8 : Rl <= 16 ? 16 : Rl <= 32 ? 32 : 64;
  {
    // forward levels 1..N-2; the rows kernel forms level N-1 itself
    for (int k = 1; k < g.N - 1; ++k) {
      // segment roots whose level-1 nodes are the segments in order: P_1 is the
      // iterate itself (the caller passes it as P[1])
      if (k == 1 && g.seg_root && P[1] == P[0]) continue;
      const int64_t work = tr.ncnt[k] * g.rsuf[k] * g.nrhs;
      KL(h, k_fwd_level, dim3(grid_for(work, 256, 2048)), dim3(256), 0, s, TT, g, tr, k, (const double*)P[k - 1],
         P[k], state);
    }
    T* qlast = Q[g.N - 1];
    const double* plast = P[g.N >= 2 ? g.N - 2 : 0];
    // one wave per (node, rhs), grid-stride, at most a few workgroups per CU
    const dim3 rg(grid_for(tr.ncnt[g.N - 1] * g.nrhs, 4, KR_ROWS_GRID_CAP));
    const bool ldsf = rows_ldsf(g, tr);
    const size_t fl = ldsf ? 8 * (size_t)g.I[g.N - 1] * g.R[g.N - 1] : 0;
    const dim3 rgl(grid_for(tr.ncnt[g.N - 1] * g.nrhs, KR_ROWS_LDS_TPB / 64, KR_ROWS_LDS_GRID));
#define KR_ROWS_LAUNCH(GG, NAME)                                                                          \
  if (ldsf)                                                                                               \
    KLN(h, f32 ? NAME ",f32,lds>" : NAME ",lds>", (k_rows_adj<GG, T, true>), rgl, dim3(KR_ROWS_LDS_TPB), fl, s, \
        TT, g, tr, plast, Omega, bD, qlast, state);                                                       \
  else                                                                                                    \
    KLN(h, f32 ? NAME ",f32>" : NAME ">", (k_rows_adj<GG, T, false>), rg, dim3(256), 0, s, TT, g, tr, plast, \
        Omega, bD, qlast, state);
    const int RP = rows_lane_width(g, tr);
    const size_t flp = 8 * (size_t)g.I[g.N - 1] * RP;
    const dim3 rgp(grid_for(tr.ncnt[g.N - 1] * g.nrhs, KR_LANE_TPB / 64, KR_ROWS_LDS_GRID));
    // short nodes (under KR_MULTI_ROWS rows on average): blocks of nodes per wave
    const bool multi = RP == 16 && g.N >= 3 && g.nrhs == 1 &&
                       tr.ncnt[g.N] < (int64_t)KR_MULTI_ROWS * tr.ncnt[g.N - 1];
    if (multi) {
      const int64_t nblk = (tr.ncnt[g.N - 1] + MN_NODES - 1) / MN_NODES;
      const size_t flm = flp + 8 * (size_t)(KR_LANE_TPB / 64) * MN_WAVE_LDS;
      KLN(h, f32 ? "k_rows_multi<f32>" : "k_rows_multi", k_rows_multi<T>,
          dim3(grid_for(nblk, KR_LANE_TPB / 64, KR_ROWS_LDS_GRID)), dim3(KR_LANE_TPB), flm, s, TT, g, tr, plast, Omega,
          bD, qlast);
    } else if (RP == 8)
      KLN(h, f32 ? "k_rows_lane<8,f32>" : "k_rows_lane<8>", (k_rows_lane<8, T>), rgp, dim3(KR_LANE_TPB), flp, s, TT, g,
          tr, plast, Omega, bD, qlast);
    else if (RP == 16)
      KLN(h, f32 ? "k_rows_lane<16,f32>" : "k_rows_lane<16>", (k_rows_lane<16, T>), rgp, dim3(KR_LANE_TPB), flp, s, TT,
          g, tr, plast, Omega, bD, qlast);
    else
    switch (G) {
      case 8: KR_ROWS_LAUNCH(8, "k_rows_adj<8") break;
      case 16: KR_ROWS_LAUNCH(16, "k_rows_adj<16") break;
      case 32: KR_ROWS_LAUNCH(32, "k_rows_adj<32") break;
      default: KR_ROWS_LAUNCH(64, "k_rows_adj<64") break;
    }
#undef KR_ROWS_LAUNCH
    for (int k = g.N - 1; k >= 2; --k) {
      if (!f32 && g.R[k - 1] <= 16) {
        const int64_t tasks = tr.ncnt[k - 1] * ((g.rsuf[k] * g.nrhs + 15) / 16);
        KL(h, k_adj_level_mfma, dim3((unsigned)tasks), dim3(256), 0, s, g, tr, k, (const double*)Q[k], (double*)Q[k - 1]);
        continue;
      }
      const int64_t CE = adj_cols((int)g.R[k - 1]);
      const int64_t tasks = tr.ncnt[k - 1] * ((g.rsuf[k] * g.nrhs + CE - 1) / CE);
      KLN(h, f32 ? "k_adj_level<f32>" : "k_adj_level", k_adj_level<T>, dim3(grid_for(tasks, 1, 2048)), dim3(ADJ_THREADS), 0,
          s, TT, g, tr, k, (const T*)Q[k], Q[k - 1], state);
    }
  }
  return g.N >= 2 && !g.seg_root;
}

// The fused three-mode pass over nchunk chunks (k_subtree3: forward level 1,
// rows and adjoint level 2 in one launch).  The root adjoint (launch_root) then
// sums the chunks as if they were level-1 nodes (root_tree).
template <typename T>
static void launch_fused3(kr_handle h, const Geom& g, const Tree& tr, const Chunks& ck, int64_t nchunk,
                          const double* x, const double* Omega, const double* bD, void* Q1cv) {
  hipStream_t s = h->stream;
  T* Q1c = (T*)Q1cv;
  const bool f32 = sizeof(T) == 4;
  const size_t lds = fused3_lds(g, sizeof(T));
  const dim3 grid((unsigned)nchunk);
  if (g.R[2] <= 8)
    KLN(h, f32 ? "k_subtree3<8,f32>" : "k_subtree3<8>", (k_subtree3<8, T>), grid, dim3(KR_SUB_THREADS), lds, s, g, tr, ck, x,
        Omega, bD, Q1c);
  else
    KLN(h, f32 ? "k_subtree3<16,f32>" : "k_subtree3<16>", (k_subtree3<16, T>), grid, dim3(KR_SUB_THREADS), lds, s, g, tr, ck,
        x, Omega, bD, Q1c);
}

// The tree the root adjoint sums over after the fused pass: the chunks in place
// of the level-1 nodes, each with the factor row of its node.
static Tree root_tree(const Tree& tr, const Chunks& ck, int64_t nchunk) {
  Tree trc = tr;
  trc.ncnt[1] = nchunk;
  trc.arow[1] = ck.arow;
  trc.arow32[1] = ck.arow32;
  return trc;
}

// Dynamic LDS for the two tensor buffers of a preconditioner kernel, or 0 (then
// the kernel works in t0/t1): at most 64 KB beside its static matrix stage.
static size_t precond_lds(const Geom& g, size_t elem) {
  const size_t b = 2 * elem * (size_t)(g.Rtot * g.nrhs);
  return b <= 64 * 1024 ? b : 0;
}

// Allow `bytes` of dynamic LDS for kernel fn (beyond the default limit); false
// when the device refuses, and the caller then works without it.
static bool allow_dynamic_lds(const void* fn, size_t bytes) {
  if (bytes == 0) return true;
  // the attribute persists per function and device: set it once per size
  // (the preconditioner launches every iteration, and the call is host time)
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> granted;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lock(mu);
  auto it = granted.find({fn, dev});
  if (it != granted.end() && it->second >= bytes) return true;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return false;
  granted[{fn, dev}] = bytes;
  return true;
}

// Number of 16-blocks along the widest mode (1..4).
static int mode_blocks(const Geom& g) {
  int maxR = 1;
  for (int n = 0; n < g.N; ++n) maxR = std::max<int>(maxR, (int)g.R[n]);
  return std::min(4, (maxR + 15) / 16);
}

struct PrecondArgs {
  const void* grad;     // float64 or float32 gradient (Rtot x nrhs), as nnb partial blocks
  unsigned nnb;
  const double* dinv;   // diagonal of the eigenvector form (Rtot)
  double* x;
  void* t0;
  void* t1;
  double lambda, eta, tol;
  int max_iter, use_ginv;
  IterState* st;
};

template <int NB>
static void launch_precond_f64_nb(kr_handle h, const ModeTables& T, const Geom& g, const PrecondArgs& a) {
  static const char* names[] = {"k_precond_update<1>", "k_precond_update<2>", "k_precond_update<3>",
                                "k_precond_update<4>"};
  size_t lds = precond_lds(g, 8);
  if (!allow_dynamic_lds((const void*)k_precond_update<NB>, lds)) {
    (void)hipGetLastError();
    lds = 0;
  }
  KLN(h, names[NB - 1], k_precond_update<NB>, dim3(1), dim3(PC_THREADS), lds, h->stream, T, g, (const double*)a.grad,
      a.nnb, a.dinv, a.x, (double*)a.t0, (double*)a.t1, (int)(lds > 0), a.lambda, a.eta, a.tol, a.max_iter, a.use_ginv,
      a.st);
}

template <int MODE, int NB>
static void launch_precond_mp_nb(kr_handle h, const ModeTables& T, const Geom& g, const PrecondArgs& a) {
  static const char* names[4][4] = {
      {"", "", "", ""},
      {"k_precond_mp<f32,1>", "k_precond_mp<f32,2>", "k_precond_mp<f32,3>", "k_precond_mp<f32,4>"},
      {"k_precond_mp<bf16,1>", "k_precond_mp<bf16,2>", "k_precond_mp<bf16,3>", "k_precond_mp<bf16,4>"},
      {"k_precond_mp<fp8,1>", "k_precond_mp<fp8,2>", "k_precond_mp<fp8,3>", "k_precond_mp<fp8,4>"}};
  size_t lds = precond_lds(g, 4);
  if (!allow_dynamic_lds((const void*)k_precond_mp<MODE, NB>, lds)) {
    (void)hipGetLastError();
    lds = 0;
  }
  KLN(h, names[MODE][NB - 1], (k_precond_mp<MODE, NB>), dim3(1), dim3(PC_THREADS), lds, h->stream, T, g,
      (const float*)a.grad, a.nnb, a.dinv, a.x, (float*)a.t0, (float*)a.t1, (int)(lds > 0), a.lambda, a.eta, a.tol,
      a.max_iter, a.use_ginv, a.st);
}

template <int MODE>
static void launch_precond_mode(kr_handle h, int nb, const ModeTables& T, const Geom& g, const PrecondArgs& a) {
  if (MODE == KR_PREC_F64) {
    if (nb == 1) launch_precond_f64_nb<1>(h, T, g, a);
    else if (nb == 2) launch_precond_f64_nb<2>(h, T, g, a);
    else if (nb == 3) launch_precond_f64_nb<3>(h, T, g, a);
    else launch_precond_f64_nb<4>(h, T, g, a);
  } else {
    constexpr int M = MODE == KR_PREC_F64 ? KR_PREC_F32 : MODE;
    if (nb == 1) launch_precond_mp_nb<M, 1>(h, T, g, a);
    else if (nb == 2) launch_precond_mp_nb<M, 2>(h, T, g, a);
    else if (nb == 3) launch_precond_mp_nb<M, 3>(h, T, g, a);
    else launch_precond_mp_nb<M, 4>(h, T, g, a);
  }
}

// One preconditioner step in precision prec.
static void launch_precond(kr_handle h, int prec, const ModeTables& T, const Geom& g, const PrecondArgs& a) {
  const int nb = mode_blocks(g);
  if (prec == KR_PREC_F64) launch_precond_mode<KR_PREC_F64>(h, nb, T, g, a);
  else if (prec == KR_PREC_F32) launch_precond_mode<KR_PREC_F32>(h, nb, T, g, a);
  else if (prec == KR_PREC_BF16) launch_precond_mode<KR_PREC_BF16>(h, nb, T, g, a);
  else launch_precond_mode<KR_PREC_FP8>(h, nb, T, g, a);
}

// The root adjoint over trr's level-1 nodes (nodes, or the fused pass's chunks)
// into partial blocks of npb nodes, which the preconditioner step sums.  Returns
// npb.
template <typename T>
static int launch_root(kr_handle h, const Geom& g, const Tree& trr, const T* Q1, T* part, const IterState* state) {
  const bool f32 = sizeof(T) == 4;
  const int npb = root_npb(trr);
  const int64_t CEr = adj_cols((int)g.R[0]);
  const int64_t ncb = (g.rsuf[1] * g.nrhs + CEr - 1) / CEr;
  const int64_t nnb = (trr.ncnt[1] + npb - 1) / npb;
  KLN(h, f32 ? "k_adj_root_partial<f32>" : "k_adj_root_partial", k_adj_root_partial<T>,
      dim3(grid_for(ncb * nnb, 1, 4096)), dim3(ADJ_THREADS), 0, h->stream, g, trr, Q1, part, npb, state);
  return npb;
}

// Validation, the sample count and the geometry of one Algorithm 2 problem.
static kr_status prepare_problem(kr_handle h, const kr_problem* p, double lambda, double eps, double delta,
                                 const kr_opts& o, Geom* gout) {
  Geom& g = *gout;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  if (!p->b && !p->gen) KR_FAIL(h, KR_EINVAL, "b is NULL and no response generator is given");
  if (p->gen) {
    if (p->b) KR_FAIL(h, KR_EINVAL, "give either b or a response generator, not both");
    if (!p->gen->X_true) KR_FAIL(h, KR_EINVAL, "response generator without X_true");
    if (!std::isfinite(p->gen->sigma)) KR_FAIL(h, KR_EINVAL, "response generator sigma is not finite");
  }
  if (!(eps > 0.0 && eps < 1.0)) KR_FAIL(h, KR_EINVAL, "eps=%g outside (0, 1)", eps);
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda=%g invalid", lambda);
  int64_t m = o.m;
  if (m <= 0 && (o.flags & KR_OPT_M_RLNR)) {
    const double R = (double)g.Rtot;
    m = std::max<int64_t>(1, (int64_t)std::ceil(R * std::log(R) / eps));
  } else if (m <= 0) {
    if (!(delta > 0.0 && delta < 1.0)) KR_FAIL(h, KR_EINVAL, "delta=%g outside (0, 1)", delta);
    const double R = (double)g.Rtot;
    const double sc = std::ceil(1680.0 * R * std::log(40.0 * R) * std::log(1.0 / delta) / eps);
    if (sc > 2.0e9) KR_FAIL(h, KR_EUNSUPPORTED, "theory sample count %.3g too large; pass opts.m", sc);
    m = (int64_t)sc;
  }
  if (m > (int64_t(1) << 31) - 2) KR_FAIL(h, KR_EUNSUPPORTED, "m=%lld too large", (long long)m);
  g.m = m;
  if (o.flags & KR_OPT_APPROX_LEVERAGE) {
    if (o.lev_proj < 0 || o.lev_proj > 64 || o.lev_rows < 0)
      KR_FAIL(h, KR_EINVAL, "opts.lev_proj=%d (1..64, 0 = default) or opts.lev_rows=%d invalid", o.lev_proj,
              o.lev_rows);
    g.approx = 1;
    g.lev_r = o.lev_proj > 0 ? o.lev_proj : 32;
    g.lev_eps = eps;
    for (int n = 0; n < g.N; ++n)
      g.lev_k[n] = o.lev_rows > 0 ? o.lev_rows : 64 * g.R[n] * std::max(1, ceil_log2(2 * (int64_t)g.R[n]));
  }
  for (int k = 0; k <= g.N; ++k)
    if ((double)level_cap(g, k) * (double)g.rsuf[k] * g.nrhs >= 2147483647.0)
      KR_FAIL(h, KR_EUNSUPPORTED, "level %d of the sample tree needs more than 2^31 entries", k);
  return KR_OK;
}

// Workspace of one problem's solve, carved from a.  P[0] is the caller's x.
static void carve_solve(Arena& a, const Geom& g, bool f32rows, void* d_x, ModeTables* T, SolveBufs* B, Tree* tr,
                        bool lean = false) {
  const int64_t m = g.m;
  const int nblocks = (int)((m + SORT_TILE - 1) / SORT_TILE);
  carve_setup(a, g, T, &B->s);
  B->keys = a.take<uint64_t>(m);
  B->keys_alt = a.take<uint64_t>(m);
  B->hist = a.take<uint32_t>(hist_words(nblocks));
  B->tiletot = a.take<int64_t>((size_t)tree_tiles(m) * (KR_MAXN + 1));
  for (int k = 1; k <= g.N; ++k) {
    const int64_t c = level_cap(g, k);
    tr->idx[k] = a.take<int32_t>(c + 2);
    tr->parent[k] = a.take<int32_t>(c + 2);
    tr->fchild[k] = a.take<int32_t>(c + 2);
    tr->arow[k] = a.take<double>((size_t)c * g.R[k - 1]);
  }
  tr->fchild[0] = a.take<int32_t>(4);
  const int64_t Dcap = level_cap(g, g.N);
  tr->rstart = a.take<int32_t>(Dcap + 2);
  tr->rkey = a.take<uint64_t>(Dcap + 1);
  tr->cnt = a.take<int64_t>(KR_MAXN + 2);   // [KR_MAXN + 1]: chunks of the fused pass
  B->Omega = a.take<double>(Dcap);
  B->counts = a.take<int32_t>(Dcap);
  B->bD = a.take<double>((size_t)Dcap * g.nrhs);
  B->P[0] = (double*)d_x;
  for (int k = 1; k < g.N; ++k) {
    if (lean && g.N >= 3 && k == g.N - 1) {
      B->P[k] = B->Q[k] = nullptr;
      continue;
    }
    B->P[k] = a.take<double>((size_t)level_cap(g, k) * g.rsuf[k] * g.nrhs);
    B->Q[k] = a.take<double>((size_t)level_cap(g, k) * g.rsuf[k] * g.nrhs);
  }
  B->Q[0] = a.take<double>((size_t)g.Rtot * g.nrhs);
  B->t0 = a.take<double>((size_t)g.Rtot * g.nrhs);
  B->t1 = a.take<double>((size_t)g.Rtot * g.nrhs);
  B->dinv = a.take<double>((size_t)g.Rtot);
  B->part = lean ? nullptr : a.take<double>((size_t)part_blocks(g) * g.Rtot * g.nrhs);
  B->state = a.take<IterState>(1);
  if (f32rows)
    for (int k = 1; k < g.N; ++k) tr->arow32[k] = a.take<float>((size_t)level_cap(g, k) * g.R[k - 1]);
  B->ck = Chunks{};
  B->Q1c = nullptr;
  if (!lean && fused3_eligible(g)) {
    const int64_t c = fused3_cap(g);
    B->ck.beg = a.take<int32_t>(c + 1);
    B->ck.par = a.take<int32_t>(c);
    B->ck.arow = a.take<double>((size_t)c * g.R[0]);
    B->ck.arow32 = a.take<float>((size_t)c * g.R[0]);
    B->ck.count = tr->cnt + KR_MAXN + 1;
    B->ck.cap = (int)c;
    B->ck.ch = fused3_ch(g);
    B->Q1c = a.take<double>((size_t)c * g.R[1] * g.R[2] * g.nrhs);
  }
}

// The part of a sketch after sampling: stable radix sort, sample tree, gathered
// rows and weights, and (implicit response) the rows of b.
static kr_status launch_sketch_rest(kr_handle h, const kr_problem* p, const Geom& g, const ModeTables& T,
                                    SolveBufs& B, Tree& tr) {
  hipStream_t s = h->stream;
  const int nblocks = (int)((g.m + SORT_TILE - 1) / SORT_TILE);
  launch_sort_tree(h, g, B.keys, B.keys_alt, B.hist, B.tiletot, nblocks, tr);
  const int64_t Dcap = level_cap(g, g.N);
  KL(h, k_node_rows, dim3(grid_for(Dcap * g.R[g.N - 1], 256, 2048)), dim3(256), 0, s, T, g, tr, g.N);
  KL(h, k_rows, dim3(grid_for(Dcap, 256, 2048)), dim3(256), 0, s, T, g, tr, p->b, p->b_dtype, B.Omega, B.bD,
     B.counts, B.s.flags);
  if (p->gen) {
    // implicit response: forward levels 1..N-2 of X_true, then the rows
    const double* X = p->gen->X_true;
    for (int k = 1; k <= g.N - 2; ++k)
      KL(h, k_gen_level, dim3(grid_for(level_cap(g, k) * g.rsuf[k] * g.nrhs, 256, 4096)), dim3(256), 0, s, g, tr, k,
         k == 1 ? X : (const double*)B.P[k - 1], B.P[k]);
    KL(h, k_gen_rows, dim3(grid_for(Dcap * g.nrhs, 256, 8192)), dim3(256), 0, s, g, tr,
       g.N >= 3 ? (const double*)B.P[g.N - 2] : X, p->gen->sigma, p->gen->seed, p->gen->stream, B.bD, B.s.flags);
  }
  HIPCHK(h, hipGetLastError());
  return KR_OK;
}

// Setup (Gram, eigen or Cholesky route, leverage tables), sampling, the stable
// radix sort, the sample tree and the gathered rows of one problem, enqueued on
// the handle's stream without host synchronisation.
static kr_status launch_sketch(kr_handle h, const kr_problem* p, const Geom& g, const ModeTables& T, SolveBufs& B,
                               Tree& tr, const kr_opts& o, bool need_eig) {
  hipStream_t s = h->stream;
  const int64_t m = g.m;
  kr_status st = launch_setup(h, p, g, T, B.s, true, need_eig, o.seed, o.stream);
  if (st != KR_OK) return st;
  int64_t sumI = 0;
  for (int n = 0; n < g.N; ++n) sumI += g.I[n];
  const int in_lds = sumI * 8 <= 48 * 1024;
  KL(h, k_sample, dim3(grid_for(m, 256, 2048)), dim3(256), in_lds ? sumI * 8 : 0, s, T, g, o.seed, o.stream,
     (uint64_t)0, in_lds, B.keys);
  return launch_sketch_rest(h, p, g, T, B, tr);
}

// ext_ws/ext_cap: a caller-provided device workspace used instead of the
// handle's (which is then neither allocated nor grown); the solve fails with
// KR_EUNSUPPORTED when it needs more than ext_cap bytes.
static kr_status solve(kr_handle h, const kr_problem* p, double lambda, double eps, double delta,
                       const kr_opts* opts, void* d_x, kr_info* info, void* ext_ws = nullptr,
                       size_t ext_cap = 0) {
  if (!h) return KR_EINVAL;
  kr_opts o{};
  if (opts) o = *opts;
  Geom g;
  kr_status st = prepare_problem(h, p, lambda, eps, delta, o, &g);
  if (st != KR_OK) return st;
  if (!d_x) KR_FAIL(h, KR_EINVAL, "x is NULL");
  const int64_t m = g.m;
  const int prec = o.precision;
  if (prec < KR_PREC_F64 || prec > KR_PREC_FP8 || o.reserved != 0)
    KR_FAIL(h, KR_EINVAL, "opts.precision=%d invalid (or opts.reserved != 0)", prec);
  if (o.flags & 1) KR_FAIL(h, KR_EINVAL, "opts.flags bit 0 is reserved");
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const int check_every = o.check_every > 0 ? o.check_every : 8;
  const double tol = o.tol > 0.0 ? o.tol : (prec == KR_PREC_F64 ? 1e-12 : 1e-9);
  const double eta = 1.0 - std::sqrt(eps);

  const int nblocks = (int)((m + SORT_TILE - 1) / SORT_TILE);
  const size_t need = solve_bytes(g, tree_tiles(g.m), nblocks);
  if (ext_ws) {
    if (need > ext_cap)
      KR_FAIL(h, KR_EUNSUPPORTED,
              "this problem needs %zu bytes of device scratch; the allocation-free entry point holds %zu", need,
              ext_cap);
  } else {
    st = ensure(h, &h->ws, &h->ws_bytes, need);
    if (st != KR_OK) return st;
  }
  Arena a{ext_ws ? (char*)ext_ws : (char*)h->ws, ext_ws ? ext_cap : h->ws_bytes, 0};
  ModeTables T{};
  SolveBufs B{};
  Tree tr{};
  carve_solve(a, g, prec != KR_PREC_F64, d_x, &T, &B, &tr);
  if (a.off > a.cap) KR_FAIL(h, KR_EHIP, "internal: workspace overflow (%zu > %zu)", a.off, a.cap);

  hipStream_t s = h->stream;
  // the eigenvectors are needed for lambda > 0 (the (kron Lambda + lambda)^+ form),
  // fp8 (eigenvector form); otherwise G^{-1} suffices
  const bool need_eig = lambda > 0.0 || prec == KR_PREC_FP8;
  st = launch_sketch(h, p, g, T, B, tr, o, need_eig);
  if (st != KR_OK) return st;
  const bool fused = B.ck.cap > 0 && !(o.flags & KR_OPT_LEVEL_PASSES);
  if (fused)
    KL(h, k_chunk_table, dim3(1), dim3(CH_THREADS), 0, s, tr, B.ck, (int)g.R[0], prec != KR_PREC_F64 ? 1 : 0);
  // one host round trip: the setup flags, the level counts of the sample tree
  // (which the iteration kernels take by value) and the fused pass's chunks
  HIPCHK(h, hipMemcpyAsync(h->h_small + 8, tr.cnt, (KR_MAXN + 2) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(h->h_small, B.s.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  {
    const int32_t fl = (int32_t)(h->h_small[0] & 0xFFFFFFFF);
    if (fl & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in A or b");
    if (fl & KR_FLAG_QUANT) KR_FAIL(h, KR_EINVAL, "a factor has no non-zero leverage to sample from");
    if ((fl & KR_FLAG_SINGULAR) && lambda == 0.0)
      KR_FAIL(h, KR_ESINGULAR, "a factor Gram matrix is singular and lambda = 0");
    for (int k = 0; k <= KR_MAXN; ++k) tr.ncnt[k] = (int64_t)h->h_small[8 + k];
  }
  int64_t nchunk = fused ? (int64_t)h->h_small[8 + KR_MAXN + 1] : 0;
  if (nchunk < 1 || nchunk > B.ck.cap) nchunk = 0;   // more chunks than the table holds: level passes
  if (prec != KR_PREC_F64 && g.N >= 2) {
    int64_t rows32 = 0;
    for (int k = 1; k < g.N; ++k) rows32 = std::max<int64_t>(rows32, level_cap(g, k) * g.R[k - 1]);
    KL(h, k_rows_to_f32, dim3(grid_for(rows32, 256, 1024)), dim3(256), 0, s, g, tr);
  }
  // -- Richardson
  if (lambda > 0.0 || prec == KR_PREC_FP8)
    KL(h, k_precond_diag, dim3(grid_for(g.Rtot, 256, 1024)), dim3(256), 0, s, T, g, lambda, B.dinv);
  KL(h, k_fill, dim3(grid_for(g.Rtot * g.nrhs, 256, 1024)), dim3(256), 0, s, (double*)d_x,
                     g.Rtot * g.nrhs, 0.0);
  KL(h, k_zero_bytes, dim3(1), dim3(256), 0, s, (uint32_t*)B.state,
                     (int64_t)(sizeof(IterState) / 4));
  HIPCHK(h, hipGetLastError());
  kr_status result = KR_OK;
  {
    PrecondArgs pa{};
    pa.grad = B.Q[0];
    pa.nnb = 1;
    pa.dinv = B.dinv;
    pa.x = (double*)d_x;
    pa.t0 = B.t0;
    pa.t1 = B.t1;
    pa.lambda = lambda;
    pa.eta = eta;
    pa.tol = tol;
    pa.max_iter = max_iter;
    pa.use_ginv = lambda == 0.0 ? 1 : 0;
    pa.st = B.state;
    // Host checks: after the first check_every iterations, the next chunk is the
    // number of iterations the observed per-RHS contraction rate predicts to
    // reach tol (plus one), so a solve usually needs two checks and launches few
    // iterations that find the state already converged.
    int iters_enqueued = 0;
    int chunk = std::min(check_every, max_iter);
    // a solve of the same shape and parameters took iter_hint iterations last
    // time: enqueue that many before the first host check (one round trip per
    // solve instead of two when it holds; passes enqueued after convergence
    // return at once)
    std::vector<int64_t> hint_key = {g.N, g.nrhs, g.m, prec, lambda > 0.0 ? 1 : 0, (int64_t)g.approx};
    for (int n = 0; n < g.N; ++n) { hint_key.push_back(g.I[n]); hint_key.push_back(g.R[n]); }
    {
      int64_t tb, eb;
      std::memcpy(&tb, &tol, 8);
      std::memcpy(&eb, &eps, 8);
      hint_key.push_back(tb);
      hint_key.push_back(eb);
    }
    if (o.check_every <= 0) {
      auto hit = h->iter_hint.find(hint_key);
      if (hit != h->iter_hint.end()) chunk = std::max(1, std::min(hit->second, max_iter));
    }
    while (iters_enqueued < max_iter) {
      chunk = std::max(1, std::min(chunk, max_iter - iters_enqueued));
      for (int it = 0; it < chunk; ++it) {
        // the sampled products, the root adjoint (over the chunks after the fused
        // pass) and the step on its partial blocks (without a root adjoint, on Q[0])
        const IterState* stc = (const IterState*)B.state;
        const Tree trr = nchunk > 0 ? root_tree(tr, B.ck, nchunk) : tr;
        const void* Q1 = nchunk > 0 ? B.Q1c : (const void*)B.Q[1];
        bool root;
        int npb = 0;
        if (prec == KR_PREC_F64) {
          if (nchunk > 0) launch_fused3<double>(h, g, tr, B.ck, nchunk, B.P[0], B.Omega, B.bD, B.Q1c);
          root = nchunk > 0 || launch_level_products<double>(h, T, g, tr, B.P, (void* const*)B.Q, B.Omega, B.bD, stc);
          if (root) npb = launch_root<double>(h, g, trr, (const double*)Q1, (double*)B.part, stc);
        } else {
          if (nchunk > 0) launch_fused3<float>(h, g, tr, B.ck, nchunk, B.P[0], B.Omega, B.bD, B.Q1c);
          root = nchunk > 0 || launch_level_products<float>(h, T, g, tr, B.P, (void* const*)B.Q, B.Omega, B.bD, stc);
          if (root) npb = launch_root<float>(h, g, trr, (const float*)Q1, (float*)B.part, stc);
        }
        pa.grad = root ? (const void*)B.part : (const void*)B.Q[0];
        pa.nnb = root ? (unsigned)((trr.ncnt[1] + npb - 1) / npb) : 1u;
        launch_precond(h, prec, T, g, pa);
      }
      iters_enqueued += chunk;
      HIPCHK(h, hipGetLastError());
      // (the setup flags were checked at the setup round trip; no iteration kernel sets them)
      HIPCHK(h, hipMemcpyAsync(h->h_state, B.state, sizeof(IterState), hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
      if (h->h_state->all_done) break;
      const IterState& S0 = *h->h_state;
      int predict = 0;
      for (int q = 0; q < g.nrhs; ++q) {
        if (S0.done[q]) continue;
        const double r1 = S0.rel_first[q], rk = S0.rel[q];
        const int k = S0.iters;
        int need = check_every;
        if (k > 1 && r1 > 0.0 && rk > 0.0 && rk < r1 && std::isfinite(r1) && std::isfinite(rk)) {
          const double rho = std::pow(rk / r1, 1.0 / (k - 1));
          if (rho > 0.0 && rho < 0.999)
            need = (int)std::ceil(std::log(tol / rk) / std::log(rho)) + 1;
        }
        predict = std::max(predict, std::max(1, need));
      }
      chunk = predict;
    }
    if (h->h_state->all_done && !h->h_state->diverged) {
      if (h->iter_hint.size() > 64) h->iter_hint.clear();
      h->iter_hint[hint_key] = h->h_state->iters;
    }
  }
  // the tree's level counts were read at the setup round trip (the tree does not
  // change while iterating); the last check already synchronised the stream
  HIPCHK(h, hipStreamSynchronize(s));
  const IterState& S = *h->h_state;
  double rel = 0.0;
  bool all = true;
  for (int q = 0; q < g.nrhs; ++q) {
    rel = std::max(rel, S.rel[q]);
    all = all && S.done[q];
  }
  if (S.diverged) {
    result = KR_EDIVERGED;
    h->err = "Richardson iteration diverged (non-finite or exploding update)";
  } else if (!all) {
    result = KR_WMAXITER;
    h->err = "iteration limit reached before the stopping rule was met";
  }
  if (info) {
    info->iters = S.iters;
    info->status = result;
    info->m = m;
    info->distinct_rows = tr.ncnt[g.N];
    info->rel_update = rel;
  }
  h->last.valid = true;
  h->last.g = g;
  h->last.T = T;
  h->last.tr = tr;
  h->last.Omega = B.Omega;
  h->last.counts = B.counts;
  h->last.redraw = true;
  h->last.seed = o.seed;
  h->last.stream = o.stream;
  return result;
}

// Per-problem result of a batched solve, gathered on the device.
struct BatchResult {
  int32_t iters, all_done, diverged, flags;
  int64_t distinct_rows;
  double rel;
};

__global__ void k_batch_collect(const BatchDesc* __restrict__ descs, int count, BatchResult* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const BatchDesc& d = descs[i];
    const IterState* st = d.st;
    BatchResult r;
    r.iters = st->iters;
    int all = 1;
    double rel = 0.0;
    for (int q = 0; q < d.g.nrhs; ++q) {
      all &= st->done[q];
      rel = fmax(rel, st->rel[q]);
    }
    r.all_done = all;
    r.diverged = st->diverged;
    r.flags = *d.flags;
    r.distinct_rows = d.tr.cnt[d.g.N];
    r.rel = rel;
    out[i] = r;
  }
}

// Stage list of one team problem's iteration (see kr_batched.hip).
static void team_stages(const Geom& g, const ModeTables& T, bool use_ginv, LExtra* L) {
  int n = 0;
  auto add = [&](int kind, int k, int trans, int io, const double* M) {
    L->st[n].kind = kind;
    L->st[n].k = k;
    L->st[n].trans = trans;
    L->st[n].io = io;
    L->st[n].M = M;
    ++n;
  };
  const int N = g.N;
  if (N <= 2) {
    add(LS_ROWS, 0, 0, 0, nullptr);
  } else {
    for (int k = 1; k <= N - 2; ++k) add(LS_FWD, k, 0, 0, nullptr);
    add(LS_ROWS2, 0, 0, 0, nullptr);
    for (int k = N - 2; k >= 2; --k) add(LS_ADJ, k, 0, 0, nullptr);
  }
  if (N >= 2) add(LS_ROOT, 0, 0, 0, nullptr);
  int j = 0;   // mode products alternate t0, t1; the first reads h = g + lambda x
  auto mode = [&](int k, int trans, bool scale, const double* M) {
    int io = (j == 0 ? 1 : 0) | (scale ? 2 : 0) | ((j & 1) ? 4 : 0) | (j > 0 && ((j - 1) & 1) ? 8 : 0);
    add(LS_MODE, k, trans, io, M);
    ++j;
  };
  if (use_ginv) {
    for (int k = 0; k < N; ++k) mode(k, 0, false, T.Ginv[k]);
  } else {
    for (int k = 0; k < N; ++k) mode(k, 1, k == N - 1, T.V[k]);
    for (int k = 0; k < N; ++k) mode(k, 0, false, T.V[k]);
  }
  L->dfin = (j - 1) & 1;
  add(LS_UPD, 0, 0, 0, nullptr);
  L->nst = n;
  L->nchunk = (int32_t)((g.Rtot + TM_THREADS - 1) / TM_THREADS);
}

// Launch configuration of a batched solve: problems with more sampled rows x
// right-hand sides than big_rows go to the team; the team kernel runs
// team_per_cu workgroups per compute unit (0 = as many as fit).
struct BatchCfg {
  double big_rows = 8192.0;
  int team_per_cu = 0;
};

static kr_status solve_batched(kr_handle h, int32_t count, const kr_problem* probs, const double* lambda, double eps,
                               double delta, const kr_opts* opts, void* const* d_x, kr_info* info,
                               const BatchCfg& cfg, bool graph) {
  if (!h) return KR_EINVAL;
  if (count < 0) KR_FAIL(h, KR_EINVAL, "count=%d", count);
  if (count == 0) return KR_OK;
  if (!probs || !lambda || !d_x) KR_FAIL(h, KR_EINVAL, "probs, lambda or x is NULL");
  kr_opts o{};
  if (opts) o = *opts;
  if (o.precision != KR_PREC_F64 || o.reserved != 0)
    KR_FAIL(h, KR_EUNSUPPORTED, "batched solves run in float64 only (opts.precision=%d)", o.precision);
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const double tol = o.tol > 0.0 ? o.tol : 1e-12;
  const double eta = 1.0 - std::sqrt(eps);
  // pass 1: geometry, limits and routes.  A queue workgroup walks a problem's
  // rows 32 (node, rhs) pairs at a time, so problems with more than cfg.big_rows
  // sampled rows x right-hand sides go to the team instead (up to LS_MAXP of
  // them); a large single-factor problem has no tree level to split over and
  // takes the multi-kernel path (outside any captured graph).
  const double BATCH_BIG_ROWS = cfg.big_rows;
  enum Route : char { QUEUE = 0, TEAM = 1, SOLO = 2 };
  std::vector<Geom> G(count);
  std::vector<double> cost(count);
  std::vector<char> route(count, QUEUE);
  int nteam_p = 0;
  // Reordered modes (N >= 3): the tree's level-(N-2) products hold
  // S_{N-2} x R_{N-2} R_{N-1} entries per right-hand side, S_{N-2} <= min(m,
  // prod of the first N-2 sizes); the two modes that minimise that product go
  // last (the others keep their order).  The sample is the same (the sampler
  // draws by the caller's mode), and x and X_true are transposed in and out.
  std::vector<kr_problem> pp(probs, probs + count);
  std::vector<kr_response_gen> pgen(count);
  std::vector<char> permuted(count, 0);
  std::vector<std::array<int, KR_MAXN>> perm(count);
  for (int i = 0; i < count; ++i) {
    kr_opts oi = o;
    oi.stream = o.stream + (uint64_t)i;
    kr_status st = prepare_problem(h, &probs[i], lambda[i], eps, delta, oi, &G[i]);
    if (st != KR_OK) return st;
    if (!d_x[i]) KR_FAIL(h, KR_EINVAL, "x of problem %d is NULL", i);
    const int N = probs[i].N;
    for (int n = 0; n < KR_MAXN; ++n) perm[i][n] = n;
    if (N >= 3) {
      auto level_size = [&](int a, int b) {
        double Ip = 1.0;
        for (int n = 0; n < N; ++n)
          if (n != a && n != b) Ip *= (double)probs[i].I[n];
        return std::min(Ip, (double)G[i].m) * (double)probs[i].R[a] * (double)probs[i].R[b];
      };
      const double base = level_size(N - 2, N - 1);
      double best = base;
      int ba = N - 2, bb = N - 1;
      for (int a = 0; a < N; ++a)
        for (int b = a + 1; b < N; ++b) {
          const double c = level_size(a, b);
          if (c < best) { best = c; ba = a; bb = b; }
        }
      if (best * 1.25 < base) {
        int k = 0;
        for (int n = 0; n < N; ++n)
          if (n != ba && n != bb) perm[i][k++] = n;
        perm[i][k++] = ba;
        perm[i][k++] = bb;
        kr_problem& q = pp[i];
        for (int n = 0; n < N; ++n) {
          q.A[n] = probs[i].A[perm[i][n]];
          q.I[n] = probs[i].I[perm[i][n]];
          q.R[n] = probs[i].R[perm[i][n]];
        }
        if (probs[i].gen) {
          pgen[i] = *probs[i].gen;
          q.gen = &pgen[i];   // X_true is replaced by its transposed copy in pass 2
        }
        st = prepare_problem(h, &q, lambda[i], eps, delta, oi, &G[i]);
        if (st != KR_OK) return st;
        for (int n = 0; n < N; ++n) {
          G[i].orig[n] = perm[i][n];
          G[i].inv[perm[i][n]] = n;
        }
        permuted[i] = 1;
      }
    }
    for (int n = 0; n < G[i].N; ++n)
      if (G[i].R[n] > 16) KR_FAIL(h, KR_EUNSUPPORTED, "batched solves need R_n <= 16 (problem %d)", i);
    const Geom& g = G[i];
    if ((double)g.Rtot * g.nrhs > 2147483647.0)
      KR_FAIL(h, KR_EUNSUPPORTED, "batched solves need prod(R) x nrhs < 2^31 (problem %d)", i);
    double sumR = 0.0;
    for (int n = 0; n < g.N; ++n) sumR += (double)g.R[n];
    cost[i] = (double)level_cap(g, g.N) * g.R[g.N - 1] * g.nrhs + (double)level_cap(g, 1) * g.Rtot * g.nrhs +
              (double)g.Rtot * g.nrhs * sumR;
    if ((double)level_cap(g, g.N) * g.nrhs > BATCH_BIG_ROWS) {
      if (g.N == 1) route[i] = SOLO;
      else if (nteam_p < LS_MAXP) { route[i] = TEAM; ++nteam_p; }
    }
  }
  kr_status first = KR_OK;
  std::string first_msg;
  auto note = [&](int i, kr_status si, const std::string& msg) {
    if (si != KR_OK && first == KR_OK) {
      first = si;
      first_msg = "problem " + std::to_string(i) + ": " + msg;
    }
  };
  for (int i = 0; i < count; ++i) {
    if (route[i] != SOLO) continue;
    kr_opts oi = o;
    oi.stream = o.stream + (uint64_t)i;
    kr_info inf{};
    const kr_status si = solve(h, &probs[i], lambda[i], eps, delta, &oi, d_x[i], &inf);
    if (si == KR_EHIP || si == KR_ENOMEM) return si;
    if (info) info[i] = inf;
    note(i, si, si == KR_OK ? std::string() : h->err);
  }
  // descriptor slots: queue problems first, then the team's
  std::vector<int32_t> slot(count, -1), idx;
  for (int i = 0; i < count; ++i)
    if (route[i] == QUEUE) { slot[i] = (int32_t)idx.size(); idx.push_back(i); }
  const int nq = (int)idx.size();
  for (int i = 0; i < count; ++i)
    if (route[i] == TEAM) { slot[i] = (int32_t)idx.size(); idx.push_back(i); }
  const int nall = (int)idx.size();
  if (nall == 0) {
    h->last.valid = false;
    if (first != KR_OK) h->err = first_msg;
    return first;
  }
  size_t total = 0, nparts = 0;
  for (int i : idx) {
    const int nb = (int)((G[i].m + SORT_TILE - 1) / SORT_TILE);
    total += solve_bytes(G[i], tree_tiles(G[i].m), nb, route[i] == TEAM) + 1024;
    if (permuted[i]) total += 2 * 8 * (size_t)G[i].Rtot * G[i].nrhs + 1024;   // x and X_true in tree order
    if (route[i] == TEAM) nparts += (size_t)((G[i].Rtot + TM_THREADS - 1) / TM_THREADS) * G[i].nrhs * 2;
  }
  total += (size_t)nall * (sizeof(BatchDesc) + sizeof(BatchResult) + sizeof(SampleJob) + 8) + 4096 + 256;
  total += (size_t)nteam_p * (sizeof(LExtra) + 8 + 4) + nparts * 8 + 8192;
  kr_status st = ensure(h, &h->ws, &h->ws_bytes, total);
  if (st != KR_OK) return st;
  const size_t host_bytes = (size_t)nall * (sizeof(BatchDesc) + sizeof(BatchResult) + sizeof(SampleJob) + 8) + 64 +
                            (size_t)nteam_p * sizeof(LExtra) + 1024;
  if (host_bytes > h->h_batch_bytes) {
    if (h->h_batch) HIPCHK(h, hipHostFree(h->h_batch));
    h->h_batch = nullptr;
    h->h_batch_bytes = 0;
    HIPCHK(h, hipHostMalloc(&h->h_batch, host_bytes, hipHostMallocDefault));
    h->h_batch_bytes = host_bytes;
  }
  char* hb = (char*)h->h_batch;
  BatchDesc* hd = (BatchDesc*)hb;
  LExtra* hl = (LExtra*)(((uintptr_t)(hd + nall) + 15) & ~(uintptr_t)15);
  int32_t* horder = (int32_t*)(hl + nteam_p);
  BatchResult* hres = (BatchResult*)(((uintptr_t)(horder + nall) + 15) & ~(uintptr_t)15);
  int32_t* habort = (int32_t*)(hres + nall);
  SampleJob* hjobs = (SampleJob*)(((uintptr_t)(habort + 4) + 15) & ~(uintptr_t)15);
  Arena a{(char*)h->ws, h->ws_bytes, 0};
  BatchDesc* d_descs = a.take<BatchDesc>(nall);
  LExtra* d_l = a.take<LExtra>(std::max(1, nteam_p));
  int32_t* d_order = a.take<int32_t>(nall);
  BatchResult* d_res = a.take<BatchResult>(nall);
  // launch-wide counters, cleared together: queue counter, team barrier, abort
  // flag, then per team problem a ticket and a done step
  const size_t cnt_words = 64 + (size_t)nteam_p * 3;
  uint32_t* d_cnt = a.take<uint32_t>(cnt_words);
  int32_t* d_queue = (int32_t*)d_cnt;
  unsigned* d_bar = d_cnt + 16;
  int32_t* d_abort = (int32_t*)(d_cnt + 32);
  int32_t* d_ticket = (int32_t*)(d_cnt + 64);
  int64_t* d_done = a.take<int64_t>(std::max(1, nteam_p));
  double* d_part = a.take<double>(std::max<size_t>(1, nparts));
  SampleJob* d_jobs = a.take<SampleJob>(nall);
  hipStream_t s = h->stream;
  // graph mode: the work enqueued below (everything but the multi-kernel
  // problems above) is captured once and replayed while the signature -- every
  // pointer, shape and parameter it depends on -- is unchanged
  bool replay = false;
  std::vector<uint64_t> sig;
  if (graph) {
    auto put = [&](uint64_t v) { sig.push_back(v); };
    auto putd = [&](double v) { uint64_t u; std::memcpy(&u, &v, 8); sig.push_back(u); };
    put((uint64_t)count); putd(eps); putd(delta); put((uint64_t)o.m); put((uint64_t)max_iter); putd(tol);
    put(o.seed); put(o.stream); put((uint64_t)o.flags); putd(cfg.big_rows); put((uint64_t)cfg.team_per_cu);
    put((uint64_t)(uintptr_t)h->ws); put((uint64_t)h->ws_bytes); put((uint64_t)(uintptr_t)h->h_batch);
    put((uint64_t)(uintptr_t)s);
    for (int i = 0; i < count; ++i) {
      const kr_problem& pr = probs[i];
      put((uint64_t)pr.N); put((uint64_t)pr.nrhs); put((uint64_t)pr.a_dtype); put((uint64_t)pr.b_dtype);
      for (int n = 0; n < pr.N; ++n) { put((uint64_t)pr.I[n]); put((uint64_t)pr.R[n]); put((uint64_t)(uintptr_t)pr.A[n]); }
      put((uint64_t)(uintptr_t)pr.b);
      if (pr.gen) { put((uint64_t)(uintptr_t)pr.gen->X_true); putd(pr.gen->sigma); put(pr.gen->seed); put(pr.gen->stream); }
      else put(0);
      putd(lambda[i]);
      put((uint64_t)(uintptr_t)d_x[i]);
    }
    replay = h->bgraph && sig == h->bgraph_sig;
  }
  if (!h->fork_ev) {
    HIPCHK(h, hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
    for (int k = 0; k < 4; ++k) {
      HIPCHK(h, hipStreamCreateWithFlags(&h->side[k], hipStreamNonBlocking));
      HIPCHK(h, hipEventCreateWithFlags(&h->join_ev[k], hipEventDisableTiming));
    }
  }
  struct CaptureGuard {   // ends an unfinished capture on every early return
    kr_handle h;
    hipStream_t s;
    bool active = false;
    ~CaptureGuard() {
      if (!active) return;
      hipGraph_t gr = nullptr;
      (void)hipStreamEndCapture(s, &gr);
      if (gr) (void)hipGraphDestroy(gr);
      h->capturing = false;
    }
  } cap_guard{h, s};
  if (graph && !replay) {
    if (!s) KR_FAIL(h, KR_EUNSUPPORTED, "graph capture needs a stream other than the legacy default stream");
    if (h->bgraph) {
      (void)hipGraphExecDestroy(h->bgraph);
      h->bgraph = nullptr;
      h->bgraph_sig.clear();
    }
    HIPCHK(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    cap_guard.active = true;
    h->capturing = true;
  }
  const bool enq = !replay;   // enqueue work (else only rebuild the host descriptors)
  // pass 2: carve, and enqueue every problem's setup and sketch, spread over the
  // side streams (fork here, join before the persistent kernels)
  size_t part_off = 0;
  std::vector<double*> xtree(count, nullptr);   // tree-order iterate of a reordered problem
  struct StreamRestore {   // the handle's stream back on every return
    kr_handle h;
    hipStream_t s;
    ~StreamRestore() { h->stream = s; }
  } stream_restore{h, s};
  if (enq) {
    HIPCHK(h, hipEventRecord(h->fork_ev, s));
    for (int k = 0; k < 4; ++k) HIPCHK(h, hipStreamWaitEvent(h->side[k], h->fork_ev, 0));
  }
  h->batch.assign(count, SketchRec{});
  std::vector<ModeTables> pT(count);
  std::vector<SolveBufs> pB(count);
  std::vector<Tree> ptr(count);
  std::vector<double*> pxi(count, nullptr);
  int pidx = 0;
  for (int i : idx) {
    h->stream = h->side[pidx++ & 3];
    const Geom& g = G[i];
    const bool team = route[i] == TEAM;
    ModeTables T{};
    SolveBufs B{};
    Tree tr{};
    double* xi = (double*)d_x[i];
    double* Xt = nullptr;
    if (permuted[i]) {
      xi = a.take<double>((size_t)g.Rtot * g.nrhs);
      Xt = a.take<double>((size_t)g.Rtot * g.nrhs);
      xtree[i] = xi;
      if (pp[i].gen) pgen[i].X_true = Xt;
    }
    carve_solve(a, g, false, xi, &T, &B, &tr, team);
    if (a.off > a.cap) KR_FAIL(h, KR_EHIP, "internal: workspace overflow (%zu > %zu)", a.off, a.cap);
    kr_opts oi = o;
    oi.stream = o.stream + (uint64_t)i;
    if (enq) {
      if (permuted[i] && pp[i].gen)
        KL(h, k_permute_modes, dim3(grid_for(g.Rtot * g.nrhs, 256, 1024)), dim3(256), 0, h->stream, g,
           probs[i].gen->X_true, Xt, 1);
      st = launch_setup(h, &pp[i], g, T, B.s, true, lambda[i] > 0.0, oi.seed, oi.stream);
      if (st != KR_OK) return st;
    }
    // this problem's share of the batched sampling launch
    {
      SampleJob& jb = hjobs[slot[i]];
      std::memset(&jb, 0, sizeof(SampleJob));
      for (int n = 0; n < g.N; ++n) {
        jb.C[n] = T.C[n];
        jb.I[n] = g.I[n];
        jb.shift[n] = g.shift[n];
        jb.inv[n] = g.inv[n];
      }
      jb.N = g.N;
      jb.m = g.m;
      jb.seed = oi.seed;
      jb.stream = oi.stream;
      jb.keys = B.keys;
    }
    pT[i] = T;
    pB[i] = B;
    ptr[i] = tr;
    pxi[i] = xi;
    SketchRec& rec = h->batch[i];
    rec.valid = true;
    rec.g = g;
    rec.T = T;
    rec.tr = tr;
    rec.Omega = B.Omega;
    rec.counts = B.counts;
    BatchDesc& d = hd[slot[i]];
    std::memset(&d, 0, sizeof(BatchDesc));
    d.g = g;
    d.T = T;
    d.tr = tr;
    for (int k = 0; k <= KR_MAXN; ++k) { d.P[k] = B.P[k]; d.Q[k] = B.Q[k]; }
    d.Omega = B.Omega;
    d.bD = B.bD;
    d.t0 = B.t0;
    d.t1 = B.t1;
    d.dinv = B.dinv;
    d.st = B.state;
    d.flags = B.s.flags;
    d.lambda = lambda[i];
    d.use_ginv = lambda[i] == 0.0 ? 1 : 0;
    if (team) {
      const int ti = slot[i] - nq;
      LExtra& L = hl[ti];
      std::memset(&L, 0, sizeof(LExtra));
      team_stages(g, T, d.use_ginv != 0, &L);
      L.part = d_part + part_off;
      part_off += (size_t)L.nchunk * g.nrhs * 2;
      L.ticket = d_ticket + ti;
    }
  }
  h->stream = s;
  // every problem's samples in one launch (8 samples per thread), then the rest of
  // each sketch on the side streams again.  The job table is rebuilt on every call
  // (a replayed graph copies it from the pinned staging again).
  int64_t nb = 0;
  for (int j = 0; j < nall; ++j) {
    hjobs[j].b0 = nb;
    nb += std::max<int64_t>(1, (hjobs[j].m + 2047) / 2048);
  }
  if (enq) {
    for (int k = 0; k < 4; ++k) {
      HIPCHK(h, hipEventRecord(h->join_ev[k], h->side[k]));
      HIPCHK(h, hipStreamWaitEvent(s, h->join_ev[k], 0));
    }
    HIPCHK(h, hipMemcpyAsync(d_jobs, hjobs, nall * sizeof(SampleJob), hipMemcpyHostToDevice, s));
    if (nb > 2147483647LL) KR_FAIL(h, KR_EUNSUPPORTED, "too many samples in one batch");
    KL(h, k_sample_batched, dim3((unsigned)nb), dim3(256), 0, s, (const SampleJob*)d_jobs, nall);
    HIPCHK(h, hipEventRecord(h->fork_ev, s));
    for (int k = 0; k < 4; ++k) HIPCHK(h, hipStreamWaitEvent(h->side[k], h->fork_ev, 0));
    pidx = 0;
    for (int i : idx) {
      h->stream = h->side[pidx++ & 3];
      const Geom& g = G[i];
      st = launch_sketch_rest(h, &pp[i], g, pT[i], pB[i], ptr[i]);
      if (st != KR_OK) return st;
      if (lambda[i] > 0.0)
        KL(h, k_precond_diag, dim3(grid_for(g.Rtot, 256, 1024)), dim3(256), 0, h->stream, pT[i], g, lambda[i],
           pB[i].dinv);
      KL(h, k_fill, dim3(grid_for(g.Rtot * g.nrhs, 256, 1024)), dim3(256), 0, h->stream, pxi[i], g.Rtot * g.nrhs,
         0.0);
      KL(h, k_zero_bytes, dim3(1), dim3(256), 0, h->stream, (uint32_t*)pB[i].state, (int64_t)(sizeof(IterState) / 4));
    }
    h->stream = s;
    for (int k = 0; k < 4; ++k) {
      HIPCHK(h, hipEventRecord(h->join_ev[k], h->side[k]));
      HIPCHK(h, hipStreamWaitEvent(s, h->join_ev[k], 0));
    }
  }
  // queue problems largest first
  std::vector<int32_t> ord(nq);
  for (int k = 0; k < nq; ++k) ord[k] = k;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return cost[idx[x]] > cost[idx[y]]; });
  std::memcpy(horder, ord.data(), nq * sizeof(int32_t));
  if (enq) {
    HIPCHK(h, hipMemcpyAsync(d_descs, hd, nall * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    if (nteam_p) HIPCHK(h, hipMemcpyAsync(d_l, hl, nteam_p * sizeof(LExtra), hipMemcpyHostToDevice, s));
    if (nq) HIPCHK(h, hipMemcpyAsync(d_order, horder, nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KL(h, k_zero_bytes, dim3(1), dim3(256), 0, s, d_cnt, (int64_t)cnt_words);
    KL(h, k_zero_bytes, dim3(grid_for(std::max(1, nteam_p) * 2, 256, 64)), dim3(256), 0, s, (uint32_t*)d_done,
       (int64_t)std::max(1, nteam_p) * 2);
    // launch shapes: the queue kernel, then the team kernel with every workgroup
    // resident
    int dev = 0, ncu = 0, wclk = 0;
    HIPCHK(h, hipGetDevice(&dev));
    HIPCHK(h, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(h, hipDeviceGetAttribute(&wclk, hipDeviceAttributeWallClockRate, dev));   // kHz
    BatchArgs ba{};
    ba.descs = d_descs;
    ba.order = d_order;
    ba.nqueue = nq;
    ba.nteam_prob = nteam_p;
    ba.L = d_l;
    ba.done_step = d_done;
    ba.queue = d_queue;
    ba.bar = d_bar;
    ba.abortf = d_abort;
    ba.max_iter = max_iter;
    ba.eta = eta;
    ba.tol = tol;
    ba.limit = (uint64_t)std::max(1, wclk) * 1000ull * 30ull;   // 30 s of waiting at one barrier
    if (nq > 0) {
      int per_cu = 0;
      HIPCHK(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batched_queue, BT_THREADS, 0));
      const int grid = std::max(1, std::min(nq, std::max(1, per_cu) * ncu));
      KLN(h, "k_batched_queue", k_batched_queue, dim3(grid), dim3(BT_THREADS), 0, s, ba);
    }
    if (nteam_p > 0) {
      int per_cu = 0;
      HIPCHK(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batched_team, TM_THREADS, 0));
      per_cu = std::max(1, per_cu);
      if (cfg.team_per_cu > 0) per_cu = std::min(per_cu, cfg.team_per_cu);
      const int grid = per_cu * ncu;
      hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
      HIPCHK(h, hipStreamIsCapturing(s, &cap));
      if (cap == hipStreamCaptureStatusNone) {
        // the team's barrier needs every workgroup resident: a cooperative launch
        // guarantees it (or fails)
        void* args[] = {&ba};
        hipError_t e;
        {
          ProfScope ps(h, "k_batched_team", s);
          e = hipLaunchCooperativeKernel((const void*)k_batched_team, dim3(grid), dim3(TM_THREADS), args, 0, s);
        }
        HIPCHK(h, e);
      } else {
        KLN(h, "k_batched_team", k_batched_team, dim3(grid), dim3(TM_THREADS), 0, s, ba);
      }
    }
    for (int i : idx)   // reordered problems: x back to the caller's mode order
      if (permuted[i])
        KL(h, k_permute_modes, dim3(grid_for(G[i].Rtot * G[i].nrhs, 256, 1024)), dim3(256), 0, s, G[i],
           (const double*)xtree[i], (double*)d_x[i], 0);
    KL(h, k_batch_collect, dim3(grid_for(nall, 256, 64)), dim3(256), 0, s, (const BatchDesc*)d_descs, nall, d_res);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(hres, d_res, nall * sizeof(BatchResult), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(habort, d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  if (graph && !replay) {
    hipGraph_t gr = nullptr;
    cap_guard.active = false;
    h->capturing = false;
    HIPCHK(h, hipStreamEndCapture(s, &gr));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIPCHK(h, e);
    h->bgraph = ex;
    h->bgraph_sig = sig;
  }
  if (graph) HIPCHK(h, hipGraphLaunch(h->bgraph, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (*habort) KR_FAIL(h, KR_EHIP, "the batched team's barrier timed out (workgroups not resident?)");
  for (int i = 0; i < count; ++i) {
    if (route[i] == SOLO) continue;
    const BatchResult& r = hres[slot[i]];
    kr_status si = KR_OK;
    const char* msg = "";
    if (r.flags & KR_FLAG_NONFINITE) { si = KR_EINVAL; msg = "non-finite entries in A or b"; }
    else if (r.flags & KR_FLAG_QUANT) { si = KR_EINVAL; msg = "a factor has no non-zero leverage to sample from"; }
    else if ((r.flags & KR_FLAG_SINGULAR) && lambda[i] == 0.0) { si = KR_ESINGULAR; msg = "a factor Gram matrix is singular and lambda = 0"; }
    else if (r.diverged) { si = KR_EDIVERGED; msg = "Richardson iteration diverged"; }
    else if (!r.all_done) { si = KR_WMAXITER; msg = "iteration limit reached before the stopping rule was met"; }
    if (info) {
      info[i].iters = r.iters;
      info[i].status = si;
      info[i].m = G[i].m;
      info[i].distinct_rows = r.distinct_rows;
      info[i].rel_update = r.rel;
    }
    note(i, si, msg);
  }
  h->last.valid = false;
  if (first != KR_OK) h->err = first_msg;
  return first;
}

extern "C" {

}  // extern "C"

// The timed solve behind the entry points: kr_info.ms (host wall clock of the
// whole call) and, with KR_OPT_LOSS, kr_info.loss (max over RHS of f(x)).
static kr_status solve_entry(kr_handle h, const kr_problem* p, double lambda, double eps, double delta,
                             const kr_opts* opts, void* d_x, kr_info* info, void* ext_ws = nullptr,
                             size_t ext_cap = 0) {
  const auto t0 = std::chrono::steady_clock::now();
  kr_status st = solve(h, p, lambda, eps, delta, opts, d_x, info, ext_ws, ext_cap);
  if (info) info->loss = std::nan("");
  if ((st == KR_OK || st == KR_WMAXITER) && info && opts && (opts->flags & KR_OPT_LOSS)) {
    double f[KR_MAX_RHS];
    const std::string keep = h->err;
    const kr_status sl = kron_loss(h, p, lambda, d_x, f);
    if (sl != KR_OK) return sl;
    double mx = f[0];
    for (int q = 1; q < p->nrhs; ++q) mx = std::max(mx, f[q]);
    info->loss = mx;
    h->err = keep;
  }
  if (info) info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

extern "C" {

kr_status kron_regress(kr_handle h, const kr_problem* p, double eps, double delta, const kr_opts* opts,
                       void* d_x, kr_info* info) {
  return solve_entry(h, p, 0.0, eps, delta, opts, d_x, info);
}

kr_status kron_ridge(kr_handle h, const kr_problem* p, double lambda, double eps, double delta,
                     const kr_opts* opts, void* d_x, kr_info* info) {
  return solve_entry(h, p, lambda, eps, delta, opts, d_x, info);
}

kr_status kron_ridge_noalloc(kr_handle h, const kr_problem* p, double lambda, double eps, double delta,
                             const kr_opts* opts, void* d_x, kr_info* info) {
  if (!h) return KR_EINVAL;
  if (opts && (opts->flags & KR_OPT_LOSS))
    KR_FAIL(h, KR_EUNSUPPORTED, "KR_OPT_LOSS allocates the loss pass's workspace; not available here");
  void* ws = nullptr;
  const kr_status st = scratch_address(h, &ws);
  if (st != KR_OK) return st;
  return solve_entry(h, p, lambda, eps, delta, opts, d_x, info, ws, KR_SCRATCH_BYTES);
}

int64_t kr_noalloc_capacity(void) { return (int64_t)KR_SCRATCH_BYTES; }

static kr_status ridge_batched(kr_handle h, int32_t count, const kr_problem* probs, const double* lambda, double eps,
                               double delta, const kr_opts* opts, void* const* d_x, kr_info* info);

kr_status kron_ridge_batched(kr_handle h, int32_t count, const kr_problem* probs, const double* lambda, double eps,
                             double delta, const kr_opts* opts, void* const* d_x, kr_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  const kr_status st = ridge_batched(h, count, probs, lambda, eps, delta, opts, d_x, info);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info)
    for (int i = 0; i < count; ++i) {
      info[i].ms = ms;
      info[i].loss = std::nan("");
    }
  return st;
}

}  // extern "C"

static kr_status ridge_batched(kr_handle h, int32_t count, const kr_problem* probs, const double* lambda, double eps,
                               double delta, const kr_opts* opts, void* const* d_x, kr_info* info) {
  if (!h) return KR_EINVAL;
  kr_opts o{};
  if (opts) o = *opts;
  const bool graph = (o.flags & KR_OPT_GRAPH) != 0;
  BatchCfg cfg;
  if ((o.flags & KR_OPT_AUTOTUNE) && count > 0 && probs && lambda && d_x) {
    // batch shape class: count, sum of N, and the binary magnitudes of the summed
    // unknowns and of the summed design rows (capped by the sample count)
    int64_t sumN = 0;
    double sumR = 0.0, sumRows = 0.0;
    for (int i = 0; i < count; ++i) {
      double R = 1.0, I = 1.0;
      for (int n = 0; n < probs[i].N && n < KR_MAX_MODES; ++n) { R *= (double)probs[i].R[n]; I *= (double)probs[i].I[n]; }
      sumN += probs[i].N;
      sumR += R * std::max(1, probs[i].nrhs);
      sumRows += std::min(I, std::max(R, 1.0) * 100.0) * std::max(1, probs[i].nrhs);
    }
    const std::vector<int64_t> key = {count, sumN, (int64_t)std::floor(4.0 * std::log2(sumR + 1.0)),
                                      (int64_t)std::floor(4.0 * std::log2(sumRows + 1.0)), o.m, o.flags & KR_OPT_M_RLNR};
    auto it = h->tune.find(key);
    if (it == h->tune.end()) {
      // time every candidate on this batch (full solves; the last, chosen run
      // below produces the returned results)
      const double rows_c[] = {2048.0, 8192.0, 32768.0};
      const int wg_c[] = {1, 0};
      double best_ms = 1e300;
      BatchCfg best;
      for (double br : rows_c)
        for (int wg : wg_c) {
          BatchCfg c;
          c.big_rows = br;
          c.team_per_cu = wg;
          const auto t0 = std::chrono::steady_clock::now();
          const kr_status st = solve_batched(h, count, probs, lambda, eps, delta, opts, d_x, info, c, false);
          const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
          if (st == KR_EHIP || st == KR_ENOMEM || st == KR_EUNSUPPORTED) return st;
          if (ms < best_ms) { best_ms = ms; best = c; }
        }
      it = h->tune.emplace(key, std::make_pair(best.big_rows, best.team_per_cu)).first;
    }
    cfg.big_rows = it->second.first;
    cfg.team_per_cu = it->second.second;
  }
  return solve_batched(h, count, probs, lambda, eps, delta, opts, d_x, info, cfg, graph);
}

extern "C" {

kr_status kr_batched_config(kr_handle h, double* big_rows, int32_t* team_per_cu) {
  if (!h) return KR_EINVAL;
  if (h->tune.empty()) {
    const BatchCfg c;
    if (big_rows) *big_rows = c.big_rows;
    if (team_per_cu) *team_per_cu = c.team_per_cu;
    return KR_OK;
  }
  const auto& v = h->tune.rbegin()->second;
  if (big_rows) *big_rows = v.first;
  if (team_per_cu) *team_per_cu = v.second;
  return KR_OK;
}

}  // extern "C"

// Copy one recorded sketch to host memory in the caller's mode order: the tree
// of a reordered batched problem packs its modes in tree order, so its rows are
// mapped back (tree mode n is the caller's mode g.orig[n]) and re-sorted by the
// caller's linear row index, with their weights and multiplicities.
static kr_status export_rec(kr_handle h, const SketchRec& r, uint64_t* h_Q, int32_t* h_rows, double* h_Omega,
                            int32_t* h_counts, int64_t cap, int64_t* h_D) {
  const Geom& g = r.g;
  int64_t D = 0;
  HIPCHK(h, hipMemcpy(&D, r.tr.cnt + g.N, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (h_D) *h_D = D;
  if (h_Q) {
    std::vector<int64_t> off(g.N + 1, 0);
    for (int o = 0; o < g.N; ++o) off[o + 1] = off[o] + g.I[g.inv[o]];
    for (int n = 0; n < g.N; ++n) {
      uint64_t* dst = h_Q + off[g.orig[n]];
      if (r.T.Q[n])
        HIPCHK(h, hipMemcpy(dst, r.T.Q[n], g.I[n] * sizeof(uint64_t), hipMemcpyDeviceToHost));
      else
        std::memset(dst, 0, g.I[n] * sizeof(uint64_t));
    }
  }
  if (D > cap) {
    if (h_rows || h_Omega || h_counts) KR_FAIL(h, KR_EINVAL, "capacity %lld < D=%lld", (long long)cap, (long long)D);
    return KR_OK;
  }
  if (!h_rows && !h_Omega && !h_counts) return KR_OK;
  std::vector<uint64_t> keys(D);
  std::vector<double> om(D);
  std::vector<int32_t> ct(D);
  HIPCHK(h, hipMemcpy(keys.data(), r.tr.rkey, D * sizeof(uint64_t), hipMemcpyDeviceToHost));
  HIPCHK(h, hipMemcpy(om.data(), r.Omega, D * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(h, hipMemcpy(ct.data(), r.counts, D * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int32_t> rows((size_t)D * g.N);
  for (int64_t j = 0; j < D; ++j)
    for (int n = 0; n < g.N; ++n)
      rows[j * g.N + g.orig[n]] = (int32_t)((keys[j] >> g.shift[n]) & ((1ull << g.bits[n]) - 1ull));
  bool ident = true;
  for (int n = 0; n < g.N; ++n) ident = ident && g.orig[n] == n;
  std::vector<int64_t> ord(D);
  for (int64_t j = 0; j < D; ++j) ord[j] = j;
  if (!ident)
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
      return std::lexicographical_compare(rows.begin() + a * g.N, rows.begin() + (a + 1) * g.N,
                                          rows.begin() + b * g.N, rows.begin() + (b + 1) * g.N);
    });
  for (int64_t j = 0; j < D; ++j) {
    const int64_t k = ord[j];
    if (h_rows) std::memcpy(h_rows + j * g.N, rows.data() + k * g.N, g.N * sizeof(int32_t));
    if (h_Omega) h_Omega[j] = om[k];
    if (h_counts) h_counts[j] = ct[k];
  }
  return KR_OK;
}

static kr_status export_lev(kr_handle h, const SketchRec& r, double* h_lev, int64_t cap) {
  const Geom& g = r.g;
  int64_t sumI = 0;
  for (int n = 0; n < g.N; ++n) sumI += g.I[n];
  if (cap < sumI) KR_FAIL(h, KR_EINVAL, "capacity %lld < sum I_n = %lld", (long long)cap, (long long)sumI);
  std::vector<int64_t> off(g.N + 1, 0);
  for (int o = 0; o < g.N; ++o) off[o + 1] = off[o] + g.I[g.inv[o]];
  for (int n = 0; n < g.N; ++n) {
    double* dst = h_lev + off[g.orig[n]];
    if (r.T.lev[n] && r.T.Q[n])
      HIPCHK(h, hipMemcpy(dst, r.T.lev[n], g.I[n] * sizeof(double), hipMemcpyDeviceToHost));
    else
      for (int i = 0; i < g.I[n]; ++i) dst[i] = 0.0;
  }
  return KR_OK;
}

extern "C" {

kr_status kr_export_sketch(kr_handle h, uint64_t* h_Q, int32_t* h_rows, double* h_Omega, int32_t* h_counts,
                           int64_t cap, int64_t* h_D) {
  if (!h) return KR_EINVAL;
  if (!h->last.valid) KR_FAIL(h, KR_EINVAL, "no sketch to export");
  return export_rec(h, h->last, h_Q, h_rows, h_Omega, h_counts, cap, h_D);
}

kr_status kr_export_samples(kr_handle h, int64_t first, int64_t count, int32_t* h_idx) {
  if (!h) return KR_EINVAL;
  const SketchRec& r = h->last;
  if (!r.valid || !r.redraw) KR_FAIL(h, KR_EINVAL, "no single-solve sketch to redraw");
  const Geom& g = r.g;
  if (!h_idx || first < 0 || count < 0 || first + count > g.m)
    KR_FAIL(h, KR_EINVAL, "samples [%lld, %lld) outside [0, %lld) or h_idx NULL", (long long)first,
            (long long)(first + count), (long long)g.m);
  if (count == 0) return KR_OK;
  // the sampler again, from the kept tables, into a temporary buffer
  uint64_t* d_keys = nullptr;
  if (hipMalloc(&d_keys, (size_t)g.m * sizeof(uint64_t)) != hipSuccess)
    KR_FAIL(h, KR_ENOMEM, "sample buffer of %lld keys", (long long)g.m);
  KL(h, k_sample, dim3(grid_for(g.m, 256, 2048)), dim3(256), 0, h->stream, r.T, g, r.seed, r.stream, (uint64_t)0, 0,
     d_keys);
  std::vector<uint64_t> keys((size_t)count);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(keys.data(), d_keys + first, (size_t)count * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  hipFree(d_keys);
  if (e != hipSuccess) KR_FAIL(h, KR_EHIP, "redraw failed: %s", hipGetErrorString(e));
  for (int64_t t = 0; t < count; ++t)
    for (int n = 0; n < g.N; ++n)
      h_idx[t * g.N + g.orig[n]] = (int32_t)((keys[t] >> g.shift[n]) & ((1ull << g.bits[n]) - 1ull));
  return KR_OK;
}

kr_status kr_export_batched_sketch(kr_handle h, int32_t problem, uint64_t* h_Q, int32_t* h_rows, double* h_Omega,
                                   int32_t* h_counts, int64_t cap, int64_t* h_D) {
  if (!h) return KR_EINVAL;
  if (problem < 0 || problem >= (int32_t)h->batch.size())
    KR_FAIL(h, KR_EINVAL, "problem %d outside the last batched call (%zu problems)", problem, h->batch.size());
  if (!h->batch[problem].valid)
    KR_FAIL(h, KR_EINVAL, "problem %d took the single-problem path; its sketch is not kept", problem);
  return export_rec(h, h->batch[problem], h_Q, h_rows, h_Omega, h_counts, cap, h_D);
}

kr_status kr_export_leverage(kr_handle h, int32_t problem, double* h_lev, int64_t cap) {
  if (!h || !h_lev) return KR_EINVAL;
  if (problem < 0) {
    if (!h->last.valid) KR_FAIL(h, KR_EINVAL, "no sketch to export");
    return export_lev(h, h->last, h_lev, cap);
  }
  if (problem >= (int32_t)h->batch.size() || !h->batch[problem].valid)
    KR_FAIL(h, KR_EINVAL, "no kept sketch for problem %d of the last batched call", problem);
  return export_lev(h, h->batch[problem], h_lev, cap);
}

// ---------------------------------------------------------------------------
// Loss and exact baseline
// ---------------------------------------------------------------------------
static int rm_bucket(int R) { return R <= 8 ? 8 : R <= 16 ? 16 : R <= 32 ? 32 : 64; }

// out[pre][o][post] = sum_r M(o, r) in[pre][r][post]: the fibre kernel for R_in <= 64
// and post >= 64, the general one otherwise.
static void launch_mode_product(kr_handle h, const double* in, double* out, int64_t pre, int Rin, int Rout,
                                int64_t post, const double* M, int trans) {
  hipStream_t s = h->stream;
  if (Rin > 64 || post < 64) {   // the fibre kernel needs fibres long enough to fill its lanes
    KL(h, k_mode_product, dim3(grid_for(pre * Rout * post, 256)), dim3(256), 0, s, in, out, pre, Rin, Rout, post, M,
       trans);
    return;
  }
  const dim3 grid((unsigned)((post + 255) / 256), (unsigned)((Rout + MP_OUT - 1) / MP_OUT),
                  (unsigned)std::min<int64_t>(pre, 65535));
  switch (rm_bucket(Rin)) {
    case 8: KLN(h, "k_mode_product_fibre<8>", k_mode_product_fibre<8>, grid, dim3(256), 0, s, in, out, pre, Rin, Rout, post, M, trans); break;
    case 16: KLN(h, "k_mode_product_fibre<16>", k_mode_product_fibre<16>, grid, dim3(256), 0, s, in, out, pre, Rin, Rout, post, M, trans); break;
    case 32: KLN(h, "k_mode_product_fibre<32>", k_mode_product_fibre<32>, grid, dim3(256), 0, s, in, out, pre, Rin, Rout, post, M, trans); break;
    default: KLN(h, "k_mode_product_fibre<64>", k_mode_product_fibre<64>, grid, dim3(256), 0, s, in, out, pre, Rin, Rout, post, M, trans); break;
  }
}

}  // extern "C"

// Bytes of the implicit-response statistics (noise_stats) of a problem.
static size_t noise_bytes(const Geom& g) {
  int64_t P = 1;
  for (int n = 0; n + 2 < g.N; ++n) P *= g.I[n];
  const int R1 = g.N >= 2 ? g.R[g.N - 2] : 1;
  size_t b = 8 * (size_t)P * R1 * g.R[g.N - 1] * g.nrhs * 2 + 8 * (size_t)P * g.nrhs + 8 * 64 + 3 * 256;
  return b + 8 * (size_t)g.Rtot * g.nrhs * 4 + 4 * 256;
}

// s = K^T E (Rtot x nrhs) and e2[q] = ||E[:, q]||^2 of the implicit response's noise,
// every E entry generated once (k_noise_adjoint), then the prefix modes' products.
static kr_status noise_stats(kr_handle h, const kr_problem* p, const Geom& g, const SetupBufs& S, Arena& a,
                             double* s_out, double* e2) {
  hipStream_t st = h->stream;
  const int N = g.N;
  int64_t P = 1;
  for (int n = 0; n + 2 < N; ++n) P *= g.I[n];
  NoiseArgs na{};
  double* one = a.take<double>(1);
  if (N == 1) {
    KL(h, k_fill, dim3(1), dim3(64), 0, st, one, (int64_t)1, 1.0);
    na.A1 = one; na.M1 = 1; na.R1 = 1;
  } else {
    na.A1 = S.A64[N - 2]; na.M1 = g.I[N - 2]; na.R1 = g.R[N - 2];
  }
  na.A2 = S.A64[N - 1]; na.M2 = g.I[N - 1]; na.R2 = g.R[N - 1];
  na.nrhs = g.nrhs;
  na.seed = p->gen->seed;
  na.stream = p->gen->stream;
  const size_t ysz = (size_t)P * na.R1 * na.R2 * g.nrhs;
  double* Y = a.take<double>(ysz);
  double* Y2 = a.take<double>(ysz);
  na.Y = Y;
  na.e2part = a.take<double>((size_t)P * g.nrhs);
  if (a.off > a.cap) KR_FAIL(h, KR_EHIP, "internal: workspace overflow");
  if (P > 2147483647LL) KR_FAIL(h, KR_EUNSUPPORTED, "too many row prefixes for the noise pass");
  KL(h, k_noise_adjoint, dim3((unsigned)P, g.nrhs), dim3(256), 0, st, na);
  KL(h, k_noise_e2, dim3(g.nrhs), dim3(256), 0, st, (const double*)na.e2part, P, g.nrhs, e2);
  // prefix modes N-3 .. 0: I_n -> R_n
  int64_t dims[KR_MAXN];
  for (int n = 0; n + 2 < N; ++n) dims[n] = g.I[n];
  const double* cur = Y;
  double* dst = Y2;
  const int64_t tail = (int64_t)na.R1 * na.R2 * g.nrhs;
  for (int n = N - 3; n >= 0; --n) {
    int64_t pre = 1, post = tail;
    for (int k = 0; k < n; ++k) pre *= dims[k];
    for (int k = n + 1; k + 2 < N; ++k) post *= dims[k];
    double* o = n == 0 ? s_out : dst;
    KL(h, k_mode_product, dim3(grid_for(pre * g.R[n] * post, 256)), dim3(256), 0, st, cur, o, pre, g.I[n], g.R[n],
       post, (const double*)S.A64[n], 1);
    dims[n] = g.R[n];
    cur = o;
    dst = (o == Y2) ? Y : Y2;
  }
  if (N <= 2)
    KL(h, k_axpy_into, dim3(grid_for(g.Rtot * g.nrhs, 256, 1024)), dim3(256), 0, st, (const double*)nullptr,
       (const double*)Y, 1.0, g.Rtot * g.nrhs, s_out);
  return KR_OK;
}

// out = (kron M_n) in over the R-tensor (nrhs innermost); M_n (R_n x R_n) at
// mats + n * stride, transposed when trans.
static void kron_apply(kr_handle h, const Geom& g, const double* const* M, int trans, const double* in, double* out,
                       double* tmp) {
  const double* cur = in;
  for (int n = 0; n < g.N; ++n) {
    int64_t pre = 1, post = g.nrhs;
    for (int k = 0; k < n; ++k) pre *= g.R[k];
    for (int k = n + 1; k < g.N; ++k) post *= g.R[k];
    double* o = ((g.N - 1 - n) % 2 == 0) ? out : tmp;
    KL(h, k_mode_product, dim3(grid_for(pre * g.R[n] * post, 256)), dim3(256), 0, h->stream, cur, o, pre, g.R[n],
       g.R[n], post, M[n], trans);
    cur = o;
  }
}

// kron_loss for an implicit response: f(x) = v^T (kron G) v - 2 sigma v^T s +
// sigma^2 e2 + lambda ||x||^2, v = x - X_true.
static kr_status gen_loss(kr_handle h, const kr_problem* p, const Geom& g, double lambda, const double* x,
                          double* h_loss, double* h_opt = nullptr) {
  const size_t need = setup_bytes(g) + noise_bytes(g) + 8 * 3 * (size_t)g.Rtot * g.nrhs + 4096;
  kr_status st = ensure(h, &h->aux, &h->aux_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->aux, h->aux_bytes, 0};
  ModeTables T{};
  SetupBufs S{};
  carve_setup(a, g, &T, &S);
  const int64_t RT = g.Rtot * g.nrhs;
  double* sv = a.take<double>(RT);
  double* v = a.take<double>(RT);
  double* w = a.take<double>(RT);
  double* t = a.take<double>(RT);
  double* e2 = a.take<double>(64);
  double* out = a.take<double>(128);
  double* xs = a.take<double>(RT);
  double* u0 = a.take<double>(RT);
  double* u1 = a.take<double>(RT);
  hipStream_t s = h->stream;
  if (h_opt) {
    // Gram eigen-decompositions for x*, then x* = (kron V) D (kron V)^T K^T b
    st = launch_setup(h, p, g, T, S, false, true);
    if (st != KR_OK) return st;
  } else {
    KL(h, k_zero_bytes, dim3(1), dim3(64), 0, s, (uint32_t*)S.flags, (int64_t)64);
    launch_promote(h, p, g, S.A64, S.flags, s);
    KL(h, k_gram, dim3(g.N), dim3(256), 0, s, T, g, S.gram);
  }
  st = noise_stats(h, p, g, S, a, sv, e2);
  if (st != KR_OK) return st;
  const double* X = p->gen->X_true;
  const double* Gm[KR_MAXN];
  for (int n = 0; n < g.N; ++n) Gm[n] = S.gram + (size_t)n * 64 * 64;
  KL(h, k_axpy_into, dim3(grid_for(RT, 256, 1024)), dim3(256), 0, s, x, X, -1.0, RT, v);
  kron_apply(h, g, Gm, 0, v, w, t);
  KL(h, k_gen_loss_finish, dim3(g.nrhs), dim3(256), 0, s, x, X, (const double*)w, (const double*)sv,
     (const double*)e2, g.Rtot, g.nrhs, p->gen->sigma, lambda, out);
  if (h_opt) {
    const double* Vm[KR_MAXN];
    for (int n = 0; n < g.N; ++n) Vm[n] = T.V[n];
    kron_apply(h, g, Gm, 0, X, w, t);
    KL(h, k_axpy_into, dim3(grid_for(RT, 256, 1024)), dim3(256), 0, s, (const double*)w, (const double*)sv,
       p->gen->sigma, RT, u0);
    kron_apply(h, g, Vm, 1, u0, w, t);
    KL(h, k_gen_exact_scale, dim3(grid_for(RT, 256)), dim3(256), 0, s, T, g, lambda, w);
    kron_apply(h, g, Vm, 0, w, xs, t);
    KL(h, k_axpy_into, dim3(grid_for(RT, 256, 1024)), dim3(256), 0, s, (const double*)xs, X, -1.0, RT, u1);
    kron_apply(h, g, Gm, 0, u1, w, t);
    KL(h, k_gen_loss_finish, dim3(g.nrhs), dim3(256), 0, s, (const double*)xs, X, (const double*)w,
       (const double*)sv, (const double*)e2, g.Rtot, g.nrhs, p->gen->sigma, lambda, out + 64);
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h_loss, out, g.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  if (h_opt) HIPCHK(h, hipMemcpyAsync(h_opt, out + 64, g.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if ((int32_t)(h->h_small[0] & 0xFFFFFFFF) & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in A");
  return KR_OK;
}

// kron_exact for an implicit response: x* = (kron V) diag(1 / (kron Lambda + lambda))
// (kron V)^T ((kron G) X_true + sigma s).
static kr_status gen_exact(kr_handle h, const kr_problem* p, const Geom& g, double lambda, double* x) {
  const size_t need = setup_bytes(g) + noise_bytes(g) + 4096;
  kr_status st = ensure(h, &h->aux, &h->aux_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->aux, h->aux_bytes, 0};
  ModeTables T{};
  SetupBufs S{};
  carve_setup(a, g, &T, &S);
  const int64_t RT = g.Rtot * g.nrhs;
  double* sv = a.take<double>(RT);
  double* w = a.take<double>(RT);
  double* t0 = a.take<double>(RT);
  double* t1 = a.take<double>(RT);
  double* e2 = a.take<double>(64);
  hipStream_t s = h->stream;
  st = launch_setup(h, p, g, T, S, false, true);
  if (st != KR_OK) return st;
  st = noise_stats(h, p, g, S, a, sv, e2);
  if (st != KR_OK) return st;
  const double* Gm[KR_MAXN];
  const double* Vm[KR_MAXN];
  for (int n = 0; n < g.N; ++n) {
    Gm[n] = S.gram + (size_t)n * 64 * 64;
    Vm[n] = T.V[n];
  }
  kron_apply(h, g, Gm, 0, p->gen->X_true, w, t0);
  KL(h, k_axpy_into, dim3(grid_for(RT, 256, 1024)), dim3(256), 0, s, (const double*)w, (const double*)sv,
     p->gen->sigma, RT, t1);
  kron_apply(h, g, Vm, 1, t1, w, t0);
  KL(h, k_gen_exact_scale, dim3(grid_for(RT, 256)), dim3(256), 0, s, T, g, lambda, w);
  kron_apply(h, g, Vm, 0, w, x, t0);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if ((int32_t)(h->h_small[0] & 0xFFFFFFFF) & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in A");
  return KR_OK;
}

extern "C" {

kr_status kron_loss(kr_handle h, const kr_problem* p, double lambda, const void* d_x, double* h_loss) {
  if (!h) return KR_EINVAL;
  Geom g;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
  if (p->gen && !p->b && d_x && h_loss) {
    if (!p->gen->X_true || !std::isfinite(p->gen->sigma)) KR_FAIL(h, KR_EINVAL, "invalid response generator");
    return gen_loss(h, p, g, lambda, (const double*)d_x, h_loss);
  }
  if (!p->b || !d_x || !h_loss) KR_FAIL(h, KR_EINVAL, "b, x or loss is NULL");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
  // largest intermediate of the expansion x x_{N-1} A_{N-1} .. x_1 A_1
  int64_t dims[KR_MAXN];
  for (int n = 0; n < g.N; ++n) dims[n] = g.R[n];
  int64_t maxsz = g.Rtot * g.nrhs;
  for (int n = g.N - 1; n >= 1; --n) {
    dims[n] = g.I[n];
    int64_t sz = g.nrhs;
    for (int k = 0; k < g.N; ++k) sz *= dims[k];
    maxsz = std::max(maxsz, sz);
  }
  const int64_t C = (g.Itot / g.I[0]) * g.nrhs;
  // block sums of the stream: one per workgroup of 16 * SL_WAVES columns and RHS
  const size_t nparts_max = (size_t)((C + 16 * SL_WAVES - 1) / (16 * SL_WAVES)) * g.nrhs;
  size_t need = setup_bytes(g) + 2 * 8 * (size_t)maxsz + 8 * nparts_max + 8 * 64 + 4096;
  st = ensure(h, &h->aux, &h->aux_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->aux, h->aux_bytes, 0};
  ModeTables T{};
  SetupBufs S{};
  carve_setup(a, g, &T, &S);
  double* buf0 = a.take<double>(maxsz);
  double* buf1 = a.take<double>(maxsz);
  double* partial = a.take<double>(nparts_max);
  double* out = a.take<double>(64);
  hipStream_t s = h->stream;
  KL(h, k_zero_bytes, dim3(1), dim3(64), 0, s, (uint32_t*)S.flags, (int64_t)64);
  launch_promote(h, p, g, S.A64, S.flags, s);
  const double* cur = (const double*)d_x;
  for (int n = 0; n < g.N; ++n) dims[n] = g.R[n];
  double* dst = buf0;
  for (int n = g.N - 1; n >= 1; --n) {
    int64_t pre = 1, post = g.nrhs;
    for (int k = 0; k < n; ++k) pre *= dims[k];
    for (int k = n + 1; k < g.N; ++k) post *= dims[k];
    launch_mode_product(h, cur, dst, pre, (int)g.R[n], (int)g.I[n], post, (const double*)S.A64[n], 0);
    dims[n] = g.I[n];
    cur = dst;
    dst = dst == buf0 ? buf1 : buf0;
  }
  // one workgroup of SL_WAVES waves per 16 * SL_WAVES columns
  const int64_t nbx = (C + 16 * SL_WAVES - 1) / (16 * SL_WAVES);
  const dim3 sg((unsigned)nbx);
  const dim3 sb(64 * SL_WAVES);
  switch (rm_bucket(g.R[0])) {
    case 8: KLN(h, "k_stream_loss<8>", k_stream_loss<2>, sg, sb, 0, s, (const double*)S.A64[0], g.I[0], g.R[0], cur, p->b, p->b_dtype, C, g.nrhs, partial); break;
    case 16: KLN(h, "k_stream_loss<16>", k_stream_loss<4>, sg, sb, 0, s, (const double*)S.A64[0], g.I[0], g.R[0], cur, p->b, p->b_dtype, C, g.nrhs, partial); break;
    case 32: KLN(h, "k_stream_loss<32>", k_stream_loss<8>, sg, sb, 0, s, (const double*)S.A64[0], g.I[0], g.R[0], cur, p->b, p->b_dtype, C, g.nrhs, partial); break;
    default: KLN(h, "k_stream_loss<64>", k_stream_loss<16>, sg, sb, 0, s, (const double*)S.A64[0], g.I[0], g.R[0], cur, p->b, p->b_dtype, C, g.nrhs, partial); break;
  }
  KL(h, k_finish_loss, dim3(g.nrhs), dim3(1024), 0, s, (const double*)partial, nbx, (const double*)d_x,
                     g.Rtot, g.nrhs, lambda, out);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h_loss, out, g.nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if ((int32_t)(h->h_small[0] & 0xFFFFFFFF) & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in A");
  return KR_OK;
}

kr_status kron_loss_opt(kr_handle h, const kr_problem* p, double lambda, const void* d_x, double* h_loss,
                        double* h_opt) {
  if (!h) return KR_EINVAL;
  Geom g;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  if (!p->gen || p->b || !d_x || !h_loss || !h_opt)
    KR_FAIL(h, KR_EINVAL, "kron_loss_opt needs an implicit response, x, and both outputs");
  if (!p->gen->X_true || !std::isfinite(p->gen->sigma)) KR_FAIL(h, KR_EINVAL, "invalid response generator");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
  return gen_loss(h, p, g, lambda, (const double*)d_x, h_loss, h_opt);
}

kr_status kron_exact(kr_handle h, const kr_problem* p, double lambda, void* d_x) {
  if (!h) return KR_EINVAL;
  Geom g;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  if (p->gen && !p->b && d_x) {
    if (!p->gen->X_true || !std::isfinite(p->gen->sigma)) KR_FAIL(h, KR_EINVAL, "invalid response generator");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
    return gen_exact(h, p, g, lambda, (double*)d_x);
  }
  if (!p->b || !d_x) KR_FAIL(h, KR_EINVAL, "b or x is NULL");
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
  const int64_t C = (g.Itot / g.I[0]) * g.nrhs;
  int64_t maxsz = (int64_t)g.R[0] * C;
  size_t need = setup_bytes(g) + 2 * 8 * (size_t)maxsz + 4096;
  for (int n = 0; n < g.N; ++n) need += 8 * (size_t)g.I[n] * g.R[n] + 256;
  st = ensure(h, &h->aux, &h->aux_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->aux, h->aux_bytes, 0};
  ModeTables T{};
  SetupBufs S{};
  carve_setup(a, g, &T, &S);
  double* U[KR_MAXN];
  for (int n = 0; n < g.N; ++n) U[n] = a.take<double>((size_t)g.I[n] * g.R[n]);
  double* buf0 = a.take<double>(maxsz);
  double* buf1 = a.take<double>(maxsz);
  hipStream_t s = h->stream;
  st = launch_setup(h, p, g, T, S, false);
  if (st != KR_OK) return st;
  for (int n = 0; n < g.N; ++n)
    KL(h, k_left_singular, dim3(grid_for((int64_t)g.I[n] * g.R[n], 256, 1024)), dim3(256), 0, s,
                       (const double*)S.A64[n], (const double*)T.V[n], (const double*)T.evals[n], g.I[n], g.R[n],
                       U[n]);
  const dim3 sg(grid_for(C, 256, int64_t(1) << 30));
  switch (rm_bucket(g.R[0])) {
    case 8: KL(h, k_stream_contract0<8>, sg, dim3(256), 0, s, (const double*)U[0], g.I[0], g.R[0], p->b, p->b_dtype, C, buf0); break;
    case 16: KL(h, k_stream_contract0<16>, sg, dim3(256), 0, s, (const double*)U[0], g.I[0], g.R[0], p->b, p->b_dtype, C, buf0); break;
    case 32: KL(h, k_stream_contract0<32>, sg, dim3(256), 0, s, (const double*)U[0], g.I[0], g.R[0], p->b, p->b_dtype, C, buf0); break;
    default: KL(h, k_stream_contract0<64>, sg, dim3(256), 0, s, (const double*)U[0], g.I[0], g.R[0], p->b, p->b_dtype, C, buf0); break;
  }
  int64_t dims[KR_MAXN];
  dims[0] = g.R[0];
  for (int n = 1; n < g.N; ++n) dims[n] = g.I[n];
  double* cur = buf0;
  double* dst = buf1;
  for (int n = 1; n < g.N; ++n) {
    int64_t pre = 1, post = g.nrhs;
    for (int k = 0; k < n; ++k) pre *= dims[k];
    for (int k = n + 1; k < g.N; ++k) post *= dims[k];
    KL(h, k_mode_product, dim3(grid_for(pre * g.R[n] * post, 256)), dim3(256), 0, s,
                       (const double*)cur, dst, pre, g.I[n], g.R[n], post, (const double*)U[n], 1);
    dims[n] = g.R[n];
    std::swap(cur, dst);
  }
  KL(h, k_exact_scale, dim3(grid_for(g.Rtot * g.nrhs, 256)), dim3(256), 0, s, T, g, lambda, cur);
  for (int n = 0; n < g.N; ++n) {
    int64_t pre = 1, post = g.nrhs;
    for (int k = 0; k < n; ++k) pre *= g.R[k];
    for (int k = n + 1; k < g.N; ++k) post *= g.R[k];
    double* o = (n == g.N - 1) ? (double*)d_x : dst;
    launch_mode_product(h, (const double*)cur, o, pre, (int)g.R[n], (int)g.R[n], post, (const double*)T.V[n], 0);
    if (n != g.N - 1) std::swap(cur, dst);
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if ((int32_t)(h->h_small[0] & 0xFFFFFFFF) & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in A");
  return KR_OK;
}


// ---------------------------------------------------------------------------
// Algorithm 3 (FastFactorMatrixUpdate) for one mode of Tucker ALS
// ---------------------------------------------------------------------------
static kr_status factor_update(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode, double lambda,
                               double eps, double delta, const kr_opts* opts, void* d_A_out, kr_info* info);

kr_status tucker_factor_update(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode, double lambda,
                               double eps, double delta, const kr_opts* opts, void* d_A_out, kr_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  const kr_status st = factor_update(h, p, d_core, mode, lambda, eps, delta, opts, d_A_out, info);
  if (info) {
    info->loss = std::nan("");
    info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return st;
}

}  // extern "C"

static kr_status factor_update(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode, double lambda,
                               double eps, double delta, const kr_opts* opts, void* d_A_out, kr_info* info) {
  if (!h) return KR_EINVAL;
  Geom gx;   // the tensor X with its factors (validated like a regression problem)
  kr_status st = make_geom(h, p, &gx);
  if (st != KR_OK) return st;
  if (p->N < 2) KR_FAIL(h, KR_EINVAL, "a factor update needs N >= 2");
  if (mode < 0 || mode >= p->N) KR_FAIL(h, KR_EINVAL, "mode %d outside 0..%d", mode, p->N - 1);
  if (p->nrhs != 1) KR_FAIL(h, KR_EINVAL, "the tensor is a single right-hand side");
  if (p->gen) KR_FAIL(h, KR_EINVAL, "a factor update needs the dense tensor X, not a response generator");
  if (!p->b || !d_core || !d_A_out) KR_FAIL(h, KR_EINVAL, "X, core or output is NULL");
  if (!(eps > 0.0 && eps < 1.0)) KR_FAIL(h, KR_EINVAL, "eps=%g outside (0, 1)", eps);
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda=%g invalid", lambda);
  const int N = p->N;
  const int In = (int)p->I[mode], Rn = (int)p->R[mode];
  // problem of the other factors (setup) and the sample-tree geometry (row first)
  kr_problem po = *p;
  po.N = N - 1;
  TuckerGeom tg{};
  tg.Nx = N;
  tg.mode = mode;
  tg.Rn = Rn;
  for (int m = 0; m < N; ++m) tg.Ix[m] = (int)p->I[m];
  tg.tmode[0] = mode;
  int Rr = 1;
  for (int m = 0, k = 0; m < N; ++m) {
    if (m == mode) continue;
    po.I[k] = p->I[m];
    po.R[k] = p->R[m];
    po.A[k] = p->A[m];
    tg.tmode[k + 1] = m;
    Rr *= (int)p->R[m];
    ++k;
  }
  tg.Rr = Rr;
  if (Rr > 2048) KR_FAIL(h, KR_EUNSUPPORTED, "prod_{m != n} R_m = %d > 2048", Rr);
  Geom go;
  st = make_geom(h, &po, &go);
  if (st != KR_OK) return st;
  kr_problem pt = po;  // tree geometry: pseudo-mode 0 = row, then the other modes
  pt.N = N;
  for (int k = N - 1; k >= 1; --k) { pt.I[k] = po.I[k - 1]; pt.R[k] = po.R[k - 1]; pt.A[k] = po.A[k - 1]; }
  pt.I[0] = In;
  pt.R[0] = 1;
  pt.A[0] = p->A[mode];
  Geom g;
  st = make_geom(h, &pt, &g);
  if (st != KR_OK) return st;
  g.seg_root = 1;
  kr_opts o{};
  if (opts) o = *opts;
  if (o.precision != KR_PREC_F64)
    KR_FAIL(h, KR_EUNSUPPORTED, "tucker_factor_update runs in float64 only (opts.precision=%d)", o.precision);
  int64_t mrow = o.m;
  if (mrow <= 0) {
    if (!(delta > 0.0 && delta < 1.0)) KR_FAIL(h, KR_EINVAL, "delta=%g outside (0, 1)", delta);
    const double Rd = (double)Rr;
    const double sc = std::ceil(1680.0 * Rd * std::log(40.0 * Rd) * std::log((double)In / delta) / eps);
    if (sc * In > 2.0e9) KR_FAIL(h, KR_EUNSUPPORTED, "theory sample count %.3g per row too large; pass opts.m", sc);
    mrow = (int64_t)sc;
  }
  if ((double)mrow * In > 2.0e9) KR_FAIL(h, KR_EUNSUPPORTED, "rows x samples = %.3g too large", (double)mrow * In);
  tg.m_row = mrow;
  g.m = mrow * In;
  go.m = g.m;
  for (int k = 0; k <= g.N; ++k)
    if ((double)level_cap(g, k) * (double)g.rsuf[k] >= 2147483647.0)
      KR_FAIL(h, KR_EUNSUPPORTED, "level %d of the sample tree needs more than 2^31 entries", k);
  const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
  const int check_every = o.check_every > 0 ? o.check_every : 8;
  const double tol = o.tol > 0.0 ? o.tol : 1e-12;
  const double eta = 1.0 - std::sqrt(eps);
  const int64_t m = g.m;
  const int nblocks = (int)((m + SORT_TILE - 1) / SORT_TILE);

  // workspace
  size_t need = setup_bytes(go) + 2 * 8 * (size_t)m + 4 * hist_words(nblocks) +
                8 * (size_t)tree_tiles(m) * (KR_MAXN + 1) + 4096;
  const int64_t Dcap = level_cap(g, g.N);
  for (int k = 1; k <= g.N; ++k) need += 3 * 4 * (size_t)(level_cap(g, k) + 2) + 8 * (size_t)level_cap(g, k) * g.R[k - 1] + 1024;
  need += (size_t)Dcap * (8 + 8 + 4) + 4 * (size_t)(Dcap + 2) + 8 * (size_t)Dcap + 2048;
  for (int k = 1; k < g.N; ++k) need += 2 * 8 * (size_t)level_cap(g, k) * g.rsuf[k] + 512;
  need += 8 * ((size_t)In * Rr + 3 * (size_t)Rn * Rr + (size_t)Rr * Rn + (size_t)Rn * Rn + 8) + 4 * 4 * (size_t)In +
          8 * 3 * (size_t)In + 4 * (size_t)In + sizeof(IterState) + 18 * 256;
  st = ensure(h, &h->ws, &h->ws_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->ws, h->ws_bytes, 0};
  ModeTables To{};
  SetupBufs S{};
  carve_setup(a, go, &To, &S);
  uint64_t* keys = a.take<uint64_t>(m);
  uint64_t* keys_alt = a.take<uint64_t>(m);
  uint32_t* hist = a.take<uint32_t>(hist_words(nblocks));
  int64_t* tiletot = a.take<int64_t>((size_t)tree_tiles(m) * (KR_MAXN + 1));
  Tree tr{};
  for (int k = 1; k <= g.N; ++k) {
    const int64_t c = level_cap(g, k);
    tr.idx[k] = a.take<int32_t>(c + 2);
    tr.parent[k] = a.take<int32_t>(c + 2);
    tr.fchild[k] = a.take<int32_t>(c + 2);
    tr.arow[k] = a.take<double>((size_t)c * g.R[k - 1]);
  }
  tr.fchild[0] = a.take<int32_t>(4);
  tr.rstart = a.take<int32_t>(Dcap + 2);
  tr.rkey = a.take<uint64_t>(Dcap + 1);
  tr.cnt = a.take<int64_t>(KR_MAXN + 1);
  double* Omega = a.take<double>(Dcap);
  int32_t* counts = a.take<int32_t>(Dcap);
  double* bD = a.take<double>(Dcap);
  double* P[KR_MAXN + 1] = {};
  double* Q[KR_MAXN + 1] = {};
  for (int k = 1; k < g.N; ++k) {
    P[k] = a.take<double>((size_t)level_cap(g, k) * g.rsuf[k]);
    Q[k] = a.take<double>((size_t)level_cap(g, k) * g.rsuf[k]);
  }
  double* Z = a.take<double>((size_t)In * Rr);
  P[0] = Z;
  double* Gn = a.take<double>((size_t)Rn * Rr);
  double* GtP = a.take<double>((size_t)Rn * Rr);
  double* Vw = a.take<double>((size_t)Rn * Rr);
  double* AinvU = a.take<double>((size_t)Rr * Rn);
  double* Cinv = a.take<double>((size_t)Rn * Rn);
  double* wbuf = a.take<double>(8);
  int32_t* seg_done = a.take<int32_t>(In);
  int32_t* seg_iters = a.take<int32_t>(In);
  int32_t* counters = a.take<int32_t>(64);   // [0] rows done, [1] diverged
  double* seg_rel = a.take<double>(In);
  double* seg_d0 = a.take<double>(In);
  double* seg_best = a.take<double>(In);
  int32_t* seg_stall = a.take<int32_t>(In);
  IterState* state = a.take<IterState>(1);
  if (a.off > a.cap) KR_FAIL(h, KR_EHIP, "internal: workspace overflow (%zu > %zu)", a.off, a.cap);

  hipStream_t s = h->stream;
  st = launch_setup(h, &po, go, To, S, true);
  if (st != KR_OK) return st;
  ModeTables T{};
  for (int k = 1; k < g.N; ++k) {
    T.A[k] = To.A[k - 1]; T.V[k] = To.V[k - 1]; T.evals[k] = To.evals[k - 1]; T.Ginv[k] = To.Ginv[k - 1];
    T.lev[k] = To.lev[k - 1]; T.Q[k] = To.Q[k - 1]; T.C[k] = To.C[k - 1];
  }
  // the row-independent matrices staged in LDS while one of them fits 32 KB
  const int tstage = (int64_t)Rn * Rr <= 4096 ? 1 : 0;
  KL(h, k_tucker_setup, dim3(1), dim3(256), tstage ? 8 * (size_t)Rn * Rr : 0, s, T, g, tg, (const double*)d_core,
     lambda, eps, Gn, GtP, Vw, wbuf, S.flags, tstage);
  KL(h, k_tucker_ainvu, dim3(Rn), dim3(256), 2 * 8 * (size_t)Rr, s, T, g, tg, (const double*)GtP,
     (const double*)wbuf, AinvU);
  KL(h, k_tucker_cinv, dim3(1), dim3(256), tstage ? 2 * 8 * (size_t)Rn * Rr : 0, s, tg, (const double*)Vw,
     (const double*)AinvU, Cinv, S.flags, tstage);
  KL(h, k_sample_rows, dim3(grid_for(m, 256, 4096)), dim3(256), 0, s, T, g, tg, o.seed, o.stream, keys);
  launch_sort_tree(h, g, keys, keys_alt, hist, tiletot, nblocks, tr);
  KL(h, k_rows_tucker, dim3(grid_for(Dcap, 256, 2048)), dim3(256), 0, s, T, g, tg, tr, p->b, p->b_dtype, Omega, bD,
     counts, S.flags);
  // level counts of the sample tree for the iteration kernels (one host round trip)
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h->h_small + 8, tr.cnt, (KR_MAXN + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  for (int k = 0; k <= KR_MAXN; ++k) tr.ncnt[k] = (int64_t)h->h_small[8 + k];
  // every row drawn (level-1 node s is row s): the forward level 1, a copy of the
  // rows' iterates, is Z itself
  if (g.N >= 3 && tr.ncnt[1] == In) P[1] = Z;
  // the rows' own factor rows are materialised only when the rows kernel does not
  // read them from the LDS-staged factor
  KL(h, k_node_rows, dim3(grid_for(Dcap * g.R[g.N - 1], 256, 2048)), dim3(256), 0, s, T, g, tr,
     rows_ldsf(g, tr) ? g.N - 1 : g.N);
  KL(h, k_fill, dim3(grid_for((int64_t)In * Rr, 256, 1024)), dim3(256), 0, s, Z, (int64_t)In * Rr, 0.0);
  KL(h, k_zero_bytes, dim3(grid_for(In, 256, 64)), dim3(256), 0, s, (uint32_t*)seg_done, (int64_t)In);
  KL(h, k_zero_bytes, dim3(1), dim3(64), 0, s, (uint32_t*)counters, (int64_t)64);
  KL(h, k_zero_bytes, dim3(1), dim3(256), 0, s, (uint32_t*)state, (int64_t)(sizeof(IterState) / 4));
  HIPCHK(h, hipGetLastError());
  // the per-row update with its operands staged up front (rows of at most 256
  // entries, R_n <= 16, the tree modes' eigenvectors and Cinv within 8 KB)
  int64_t nstage = (int64_t)Rn * Rn;
  for (int k = 1; k < g.N; ++k) nstage += (int64_t)g.R[k] * g.R[k];
  const bool staged = Rr <= 256 && Rn <= TU_RN && nstage <= 1024;
  int enq = 0;
  bool checked = false;
  while (enq < max_iter) {
    const int chunk = std::min(check_every, max_iter - enq);
    for (int it = 0; it < chunk; ++it) {
      launch_level_products<double>(h, T, g, tr, P, (void* const*)Q, Omega, bD, (const IterState*)state);
      if (staged)
        KL(h, k_tucker_update_st, dim3(In), dim3(256), 8 * (3 * (size_t)Rr + (size_t)nstage), s, T, g, tg,
           (const double*)Q[1], Z, (const double*)GtP, (const double*)Vw, (const double*)AinvU, (const double*)Cinv,
           (const double*)wbuf, eta, tol, enq + it, max_iter, seg_done, seg_iters, seg_rel, seg_d0, seg_best, seg_stall,
           counters, counters + 1, state);
      else
        KL(h, k_tucker_update, dim3(In), dim3(256), 3 * 8 * (size_t)Rr, s, T, g, tg, (const double*)Q[1], Z,
           (const double*)GtP, (const double*)Vw, (const double*)AinvU, (const double*)Cinv, (const double*)wbuf, eta,
           tol, enq + it, max_iter, seg_done, seg_iters, seg_rel, seg_d0, seg_best, seg_stall, counters, counters + 1,
           state);
    }
    enq += chunk;
    HIPCHK(h, hipGetLastError());
    // rows done and the divergence flag (the updates test them themselves)
    HIPCHK(h, hipMemcpyAsync(h->h_small + 4, counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (!checked) HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (!checked) {
      checked = true;
      const int32_t fl = (int32_t)(h->h_small[0] & 0xFFFFFFFF);
      if (fl & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in the factors or X");
      if (fl & KR_FLAG_QUANT) KR_FAIL(h, KR_EINVAL, "a factor has no non-zero leverage to sample from");
      if (fl & KR_FLAG_CORE) KR_FAIL(h, KR_ESINGULAR, "G_(n) G_(n)^T or the Woodbury matrix is singular");
    }
    const int32_t* cnt = (const int32_t*)(h->h_small + 4);
    if (cnt[0] >= In || cnt[1]) break;
  }
  KL(h, k_tucker_rows_out, dim3(grid_for((int64_t)In * Rn, 256, 1024)), dim3(256), 0, s, tg, (const double*)Z,
     (const double*)GtP, In, (double*)d_A_out);
  HIPCHK(h, hipGetLastError());
  // per-row status
  std::vector<int32_t> done(In), its(In);
  std::vector<double> rel(In);
  int32_t cnt_h[2];
  HIPCHK(h, hipMemcpyAsync(done.data(), seg_done, In * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(its.data(), seg_iters, In * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(rel.data(), seg_rel, In * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(cnt_h, counters, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(h->h_small + 8, tr.cnt, (KR_MAXN + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  kr_status result = KR_OK;
  bool all = true;
  double relmax = 0.0;
  int itmax = 0;
  for (int i = 0; i < In; ++i) {
    all = all && done[i];
    relmax = std::max(relmax, rel[i]);
    itmax = std::max(itmax, done[i] ? its[i] : enq);
  }
  if (cnt_h[1]) {
    result = KR_EDIVERGED;
    h->err = "Richardson iteration diverged for at least one row";
  } else if (!all) {
    result = KR_WMAXITER;
    h->err = "iteration limit reached before every row met the stopping rule";
  }
  if (info) {
    info->iters = itmax;
    info->status = result;
    info->m = m;
    info->distinct_rows = h->h_small[8 + g.N];
    info->rel_update = relmax;
  }
  h->last.valid = true;
  h->last.redraw = false;   // drawn per factor row by k_sample_rows
  h->last.g = g;
  h->last.T = T;
  h->last.tr = tr;
  h->last.Omega = Omega;
  h->last.counts = counts;
  return result;
}

extern "C" {

kr_status tucker_factor_exact(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode, double lambda,
                              void* d_A_out) {
  if (!h) return KR_EINVAL;
  Geom g;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  if (!p->b || !d_core || !d_A_out) KR_FAIL(h, KR_EINVAL, "X, core or output is NULL");
  if (p->nrhs != 1) KR_FAIL(h, KR_EINVAL, "the tensor is one right-hand side (nrhs=%d)", p->nrhs);
  if (mode < 0 || mode >= g.N || g.N < 2) KR_FAIL(h, KR_EINVAL, "mode %d of an order-%d tensor", mode, g.N);
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) KR_FAIL(h, KR_EINVAL, "lambda invalid");
  const int n = mode;
  // contraction order: the first product reads X, so it takes the mode that shrinks
  // the tensor most; the rest follow in increasing mode order
  int first = -1;
  for (int m = 0; m < g.N; ++m)
    if (m != n && (first < 0 || (double)g.I[m] / g.R[m] > (double)g.I[first] / g.R[first])) first = m;
  int order[KR_MAXN], no = 0;
  order[no++] = first;
  for (int m = 0; m < g.N; ++m)
    if (m != n && m != first) order[no++] = m;
  int64_t dims[KR_MAXN];
  for (int m = 0; m < g.N; ++m) dims[m] = g.I[m];
  int64_t maxsz = 0;
  for (int k = 0; k < no; ++k) {
    dims[order[k]] = g.R[order[k]];
    int64_t sz = 1;
    for (int m = 0; m < g.N; ++m) sz *= dims[m];
    maxsz = std::max(maxsz, sz);
  }
  const size_t need = setup_bytes(g) + 2 * 8 * (size_t)maxsz + 2 * 8 * (size_t)g.Rtot +
                      8 * ((size_t)g.I[n] * g.R[n] + (size_t)g.R[n] * g.R[n]) + 8192;
  st = ensure(h, &h->aux, &h->aux_bytes, need);
  if (st != KR_OK) return st;
  Arena a{(char*)h->aux, h->aux_bytes, 0};
  ModeTables T{};
  SetupBufs S{};
  carve_setup(a, g, &T, &S);
  double* buf0 = a.take<double>(maxsz);
  double* buf1 = a.take<double>(maxsz);
  double* c0 = a.take<double>(g.Rtot);
  double* c1 = a.take<double>(g.Rtot);
  double* P = a.take<double>((size_t)g.I[n] * g.R[n]);
  double* H = a.take<double>((size_t)g.R[n] * g.R[n]);
  if (a.off > a.cap) KR_FAIL(h, KR_EHIP, "internal: workspace overflow");
  hipStream_t s = h->stream;
  KL(h, k_zero_bytes, dim3(1), dim3(64), 0, s, (uint32_t*)S.flags, (int64_t)64);
  launch_promote(h, p, g, S.A64, S.flags, s);
  KL(h, k_gram, dim3(g.N), dim3(256), 0, s, T, g, S.gram);
  // T = X x_{m != n} A_m^T
  for (int m = 0; m < g.N; ++m) dims[m] = g.I[m];
  const double* cur = nullptr;
  double* dst = buf0;
  for (int k = 0; k < no; ++k) {
    const int m = order[k];
    int64_t pre = 1, post = 1;
    for (int q = 0; q < m; ++q) pre *= dims[q];
    for (int q = m + 1; q < g.N; ++q) post *= dims[q];
    const int64_t work = pre * g.R[m] * post;
    if (k == 0 && p->b_dtype == KR_F32)
      KL(h, k_ttm_f32, dim3(grid_for(work, 256)), dim3(256), 0, s, (const float*)p->b, dst, pre, g.I[m], g.R[m],
         post, (const double*)S.A64[m]);
    else
      KL(h, k_mode_product, dim3(grid_for(work, 256)), dim3(256), 0, s, k == 0 ? (const double*)p->b : cur, dst, pre,
         g.I[m], g.R[m], post, (const double*)S.A64[m], 1);
    dims[m] = g.R[m];
    cur = dst;
    dst = dst == buf0 ? buf1 : buf0;
  }
  // core x_{m != n} (A_m^T A_m)
  const double* core = (const double*)d_core;
  const double* cc = core;
  double* cd = c0;
  for (int m = 0; m < g.N; ++m) {
    if (m == n) continue;
    int64_t pre = 1, post = 1;
    for (int q = 0; q < m; ++q) pre *= g.R[q];
    for (int q = m + 1; q < g.N; ++q) post *= g.R[q];
    KL(h, k_mode_product, dim3(grid_for(pre * g.R[m] * post, 256)), dim3(256), 0, s, cc, cd, pre, g.R[m], g.R[m],
       post, (const double*)(S.gram + (size_t)m * 64 * 64), 0);
    cc = cd;
    cd = cd == c0 ? c1 : c0;
  }
  int64_t pre = 1, post = 1;
  for (int q = 0; q < n; ++q) pre *= g.R[q];
  for (int q = n + 1; q < g.N; ++q) post *= g.R[q];
  KL(h, k_contract_all_but, dim3(grid_for((int64_t)g.I[n] * g.R[n], 256)), dim3(256), 0, s, cur, core, pre, g.I[n],
     g.R[n], post, P);
  KL(h, k_contract_all_but, dim3(grid_for((int64_t)g.R[n] * g.R[n], 256)), dim3(256), 0, s, cc, core, pre, g.R[n],
     g.R[n], post, H);
  KL(h, k_factor_solve, dim3(grid_for(g.I[n], 256, 64)), dim3(256), 0, s, (const double*)H, lambda,
     (const double*)P, g.I[n], g.R[n], (double*)d_A_out, S.flags);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(h->h_small, S.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  const int32_t fl = (int32_t)(h->h_small[0] & 0xFFFFFFFF);
  if (fl & KR_FLAG_NONFINITE) KR_FAIL(h, KR_EINVAL, "non-finite entries in the factors");
  if (fl & KR_FLAG_CORE) KR_FAIL(h, KR_ESINGULAR, "G_(n) K^T K G_(n)^T + lambda I is singular");
  return KR_OK;
}


// Algorithm 1 (TuckerALS) behind the boundary: per sweep the factor updates of
// modes 0..N-1 (Algorithm 3) and the core update (Algorithm 2 with b = vec(X)),
// then the relative reconstruction error.
kr_status kr_tucker_als(kr_handle h, const kr_problem* p, void* d_core, double lambda, double eps, double delta,
                        int32_t sweeps, const kr_opts* factor_opts, const kr_opts* core_opts, double* h_rre,
                        int32_t* h_iters, int32_t* h_failed_step) {
  if (!h) return KR_EINVAL;
  if (h_failed_step) *h_failed_step = -1;
  if (!p || !d_core || !factor_opts || !core_opts || sweeps < 0) KR_FAIL(h, KR_EINVAL, "NULL argument or sweeps < 0");
  if (p->a_dtype != KR_F64) KR_FAIL(h, KR_EINVAL, "the factors are updated in place and must be float64");
  for (int n = 0; n < p->N; ++n)
    if (!p->A[n]) KR_FAIL(h, KR_EINVAL, "factor %d is NULL", n);
  Geom g;
  kr_status st = make_geom(h, p, &g);
  if (st != KR_OK) return st;
  // ||X||^2 = the loss of the zero core
  const size_t zb = 8 * (size_t)g.Rtot;
  if (h->als_zero_bytes < zb) {
    if (h->als_zero) {
      hipStreamSynchronize(h->stream);
      hipFree(h->als_zero);
      h->als_zero = nullptr;
      h->als_zero_bytes = 0;
    }
    if (hipMalloc(&h->als_zero, zb) != hipSuccess) {
      h->als_zero = nullptr;
      KR_FAIL(h, KR_ENOMEM, "zero core of %zu bytes could not be allocated", zb);
    }
    h->als_zero_bytes = zb;
  }
  KL(h, k_fill, dim3(grid_for(g.Rtot, 256, 1024)), dim3(256), 0, h->stream, (double*)h->als_zero, g.Rtot, 0.0);
  HIPCHK(h, hipGetLastError());
  double xx = 0.0;
  st = kron_loss(h, p, 0.0, h->als_zero, &xx);
  if (st != KR_OK) return st;
  if (!(xx > 0.0)) KR_FAIL(h, KR_EINVAL, "||X|| is zero or not finite");
  kr_opts fo = *factor_opts, co = *core_opts;
  const int N = p->N;
  for (int s = 0; s < sweeps; ++s) {
    for (int step = 0; step <= N; ++step) {
      kr_info info{};
      if (step < N) {
        fo.stream = ((uint64_t)s << 8) | (uint64_t)step;
        st = tucker_factor_update(h, p, d_core, step, lambda, eps, delta, &fo, const_cast<void*>(p->A[step]), &info);
      } else {
        co.stream = ((uint64_t)s << 8) | (uint64_t)N;
        st = kron_ridge(h, p, lambda, eps, delta, &co, d_core, &info);
      }
      if (h_iters) h_iters[(size_t)s * (N + 1) + step] = info.iters;
      if (st != KR_OK) {
        if (h_failed_step) *h_failed_step = s * (N + 1) + step;
        if (st > 0) KR_FAIL(h, st, "ALS sweep %d step %d ended with status %d", s, step, (int)st);
        return st;
      }
    }
    double l = 0.0;
    st = kron_loss(h, p, 0.0, d_core, &l);
    if (st != KR_OK) return st;
    if (h_rre) h_rre[s] = l / xx;
  }
  return KR_OK;
}

}  // extern "C"
