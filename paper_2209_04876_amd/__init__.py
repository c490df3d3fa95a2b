"""Python binding of libkron_regress (gfx950): subquadratic Kronecker regression.

Argument marshalling only: every step runs in the HIP library behind the C ABI
declared in include/kron_regress.h.  Tensors are torch tensors on the GPU
(PyTorch supplies device memory and the current HIP stream).  There is no CPU
fallback: when the library or a GPU is missing the calls raise.

Functions mirror the C entry points:
  kron_regress(As, b, eps, ...)            Algorithm 2 with lambda = 0
  kron_ridge(As, b, lam, eps, ...)         Algorithm 2 with L2 regularisation
  kron_loss(As, b, x, lam)                 ||K x - b||^2 + lam ||x||^2 (float64)
  kron_exact(As, b, lam)                   exact KronMatMul optimum
  tucker_factor_update(X, As, G, mode, lam) Algorithm 3 (Tucker ALS factor update)
  tucker_factor_exact(X, As, G, mode, lam)  Algorithm 1's exact factor update
  tucker_als(X, G, As, lam, sweeps)        Algorithm 1 sequenced over the calls above
  export_sketch(handle)                    last solve's sketch (tests)
"""

import atexit
import ctypes
import os
import weakref

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkron_regress.so")
MAX_MODES = 8

KR_OK, KR_WMAXITER = 0, 1
STATUS_NAMES = {0: "OK", 1: "WMAXITER", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR",
                -5: "EDIVERGED", -6: "EUNSUPPORTED"}
KR_F64, KR_F32 = 0, 1


class KronRegressError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class ResponseGenC(ctypes.Structure):
    _fields_ = [("X_true", ctypes.c_void_p), ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_uint64)]


class Problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("I", ctypes.c_int64 * MAX_MODES), ("R", ctypes.c_int64 * MAX_MODES),
                ("A", ctypes.c_void_p * MAX_MODES), ("a_dtype", ctypes.c_int32),
                ("b_dtype", ctypes.c_int32), ("b", ctypes.c_void_p), ("gen", ctypes.POINTER(ResponseGenC))]


class ResponseGen:
    """An implicit response b = K X_true + sigma E, passed in place of b: only the
    sampled rows of b are formed (on the GPU).  E[i][q] is the Box-Muller normal of
    Philox4x64-10 words 0 and 1 at counter (i, q, 0, 0), key (seed, stream), with i
    K's row index.  X_true: contiguous float64 CUDA tensor, prod(R) or prod(R) x nrhs."""

    def __init__(self, X_true, sigma, seed=0, stream=0):
        self.X_true, self.sigma, self.seed, self.stream = X_true, float(sigma), int(seed), int(stream)

    def dim(self):
        return self.X_true.dim()


class Opts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("stream", ctypes.c_uint64),
                ("flags", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lev_rows", ctypes.c_int32), ("lev_proj", ctypes.c_int32)]


OPT_M_RLNR = 2
OPT_GRAPH = 4
OPT_AUTOTUNE = 8
OPT_APPROX_LEVERAGE = 16
OPT_LOSS = 32
OPT_LEVEL_PASSES = 64

# kr_precision: the arithmetic of the Richardson iteration (float64 plain, or
# refined: float64 residual and update, float32 adjoint, preconditioner in the
# named precision with float32 accumulation).
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}


def _precision(name):
    if name not in PRECISIONS:
        raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
    return PRECISIONS[name]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("m", ctypes.c_int64),
                ("distinct_rows", ctypes.c_int64), ("rel_update", ctypes.c_double), ("loss", ctypes.c_double),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "status": STATUS_NAMES.get(self.status, self.status),
                "m": self.m, "distinct_rows": self.distinct_rows, "rel_update": self.rel_update,
                "loss": self.loss, "ms": self.ms}


_lib = None


def load_library(path=LIB_PATH):
    """Load libkron_regress.so (built by build.py) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libkron_regress.so is not built; run paper_2209_04876_amd/build.py")
    lib = ctypes.CDLL(path)
    c_p, c_i, c_d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.kr_create.argtypes = [ctypes.POINTER(c_p), c_p]
    lib.kr_destroy.argtypes = [c_p]
    lib.kr_set_stream.argtypes = [c_p, c_p]
    lib.kr_last_error.argtypes = [c_p]
    lib.kr_last_error.restype = ctypes.c_char_p
    lib.kr_version.restype = ctypes.c_char_p
    P, O, IN = ctypes.POINTER(Problem), ctypes.POINTER(Opts), ctypes.POINTER(Info)
    lib.kron_regress.argtypes = [c_p, P, c_d, c_d, O, c_p, IN]
    lib.kron_ridge.argtypes = [c_p, P, c_d, c_d, c_d, O, c_p, IN]
    lib.kron_ridge_noalloc.argtypes = [c_p, P, c_d, c_d, c_d, O, c_p, IN]
    lib.kr_noalloc_capacity.argtypes = []
    lib.kr_noalloc_capacity.restype = ctypes.c_int64
    lib.kron_ridge_batched.argtypes = [c_p, ctypes.c_int32, P, ctypes.POINTER(c_d), c_d, c_d, O,
                                       ctypes.POINTER(c_p), IN]
    lib.kr_batched_config.argtypes = [c_p, ctypes.POINTER(c_d), ctypes.POINTER(ctypes.c_int32)]
    lib.kron_loss.argtypes = [c_p, P, c_d, c_p, ctypes.POINTER(c_d)]
    lib.kron_exact.argtypes = [c_p, P, c_d, c_p]
    lib.kron_loss_opt.argtypes = [c_p, P, c_d, c_p, ctypes.POINTER(c_d), ctypes.POINTER(c_d)]
    lib.tucker_factor_update.argtypes = [c_p, P, c_p, ctypes.c_int32, c_d, c_d, c_d, O, c_p, IN]
    lib.tucker_factor_exact.argtypes = [c_p, P, c_p, ctypes.c_int32, c_d, c_p]
    lib.kr_tucker_als.argtypes = [c_p, P, c_p, c_d, c_d, c_d, ctypes.c_int32, O, O, ctypes.POINTER(c_d),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.kr_export_sketch.argtypes = [c_p, c_p, c_p, c_p, c_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.kr_export_batched_sketch.argtypes = [c_p, ctypes.c_int32, c_p, c_p, c_p, c_p, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64)]
    lib.kr_export_leverage.argtypes = [c_p, ctypes.c_int32, c_p, ctypes.c_int64]
    lib.kr_export_samples.argtypes = [c_p, ctypes.c_int64, ctypes.c_int64, c_p]
    lib.kr_profile_enable.argtypes = [c_p, ctypes.c_int32, ctypes.c_char_p]
    lib.kr_profile_query.argtypes = [c_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(c_d)]
    lib.kr_profile_list.argtypes = [c_p, ctypes.c_char_p, ctypes.c_int64]
    for name in ("kr_batched_config", "kron_ridge_batched", "kr_profile_list", "kr_profile_enable", "kr_profile_query", "kr_create", "kr_destroy", "kr_set_stream", "kron_regress", "kron_ridge", "kron_ridge_noalloc", "kron_loss",
                 "kron_loss_opt", "kron_exact", "kr_export_sketch", "kr_export_batched_sketch", "kr_export_leverage",
                 "tucker_factor_update", "tucker_factor_exact", "kr_tucker_als", "kr_export_samples"):
        getattr(lib, name).restype = c_i
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required: the library has no CPU path")
    return torch


_live_handles = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    """Destroy every open handle while the interpreter still runs: kr_destroy then
    releases its streams, events, pinned and device memory before the HIP runtime
    (and a profiler attached to it) shuts down in the process's exit handlers.
    Leaving it to garbage collection during interpreter teardown ran those calls
    after the runtime's own finalisation had begun."""
    for h in list(_live_handles):
        try:
            h.close()
        except Exception:
            pass
    _default.clear()


class Handle:
    """A library handle bound to a HIP stream (torch's current stream by default)."""

    def __init__(self, stream=None):
        torch = _torch()
        self.lib = load_library()
        self.ptr = ctypes.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self._check(self.lib.kr_create(ctypes.byref(self.ptr), ctypes.c_void_p(s.cuda_stream)))
        _live_handles.add(self)

    def _check(self, status):
        if status < 0:
            msg = self.lib.kr_last_error(self.ptr).decode() if self.ptr else ""
            raise KronRegressError(status, msg)
        return status

    def close(self):
        if self.ptr:
            self.lib.kr_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_handle():
    torch = _torch()
    key = (torch.cuda.current_device(), torch.cuda.current_stream().cuda_stream)
    h = _default.get(key)
    if h is None:
        h = _default[key] = Handle()
    return h


def _problem(As, b):
    torch = _torch()
    if not 1 <= len(As) <= MAX_MODES:
        raise ValueError("need 1..%d factors" % MAX_MODES)
    p = Problem()
    p.N = len(As)
    keep = []
    adt = As[0].dtype
    for n, A in enumerate(As):
        if not (A.is_cuda and A.dim() == 2 and A.is_contiguous() and A.dtype == adt):
            raise ValueError("factor %d must be a contiguous 2-D CUDA tensor of one dtype" % n)
        p.I[n], p.R[n] = A.shape
        p.A[n] = A.data_ptr()
        keep.append(A)
    p.a_dtype = {torch.float64: KR_F64, torch.float32: KR_F32}[adt]
    if isinstance(b, ResponseGen):
        X = b.X_true
        if not (X.is_cuda and X.is_contiguous() and X.dim() in (1, 2) and X.dtype == torch.float64):
            raise ValueError("X_true must be a contiguous 1-D or 2-D float64 CUDA tensor")
        p.nrhs = 1 if X.dim() == 1 else X.shape[1]
        g = ResponseGenC(X.data_ptr(), b.sigma, b.seed & 0xFFFFFFFFFFFFFFFF, b.stream & 0xFFFFFFFFFFFFFFFF)
        p.gen = ctypes.pointer(g)
        keep += [g, X]
    elif b is not None:
        if not (b.is_cuda and b.is_contiguous() and b.dim() in (1, 2)):
            raise ValueError("b must be a contiguous 1-D or 2-D CUDA tensor")
        p.nrhs = 1 if b.dim() == 1 else b.shape[1]
        p.b = b.data_ptr()
        p.b_dtype = {torch.float64: KR_F64, torch.float32: KR_F32}[b.dtype]
    else:
        p.nrhs = 1
    return p, keep


def _x_like(As, nrhs, one_dim):
    torch = _torch()
    R = 1
    for A in As:
        R *= A.shape[1]
    shape = (R,) if one_dim else (R, nrhs)
    return torch.empty(shape, dtype=torch.float64, device=As[0].device)


def _opts(m, max_iter, tol, seed, stream, check_every, flags=0, workgroups=0, precision="f64",
          approx_leverage=None):
    """approx_leverage: None for exact leverage, or (k, r) -- the rows of each spectral
    approximation and of the projection (0 = the library's defaults)."""
    o = Opts()
    o.m, o.max_iter, o.seed, o.stream, o.check_every = m, max_iter, seed, stream, check_every
    o.tol = 0.0 if tol is None else tol
    o.flags, o.workgroups = flags, workgroups
    o.precision = _precision(precision)
    if approx_leverage is not None:
        o.flags |= OPT_APPROX_LEVERAGE
        o.lev_rows, o.lev_proj = int(approx_leverage[0]), int(approx_leverage[1])
    return o


def kron_ridge(As, b, lam, eps=0.1, delta=0.01, m=0, seed=0, stream=0, max_iter=200, tol=None,
               check_every=0, handle=None, x=None, allow_maxiter=True,
               precision="f64", approx_leverage=None, compute_loss=False, level_passes=False):
    """Algorithm 2 with regularisation lam.  Returns (x float64, info dict).

    tol=None takes the library default (1e-12 for "f64", 1e-9 for the refined
    precisions "f32", "bf16", "fp8").  approx_leverage=(k, r) takes Algorithm 2's
    approximate leverage scores (spectral approximation of k rows per factor, JL
    projection of r rows; 0 = defaults) instead of exact ones.  compute_loss=True
    fills info["loss"] with the float64 loss of x (max over right-hand sides).
    level_passes=True runs three-factor problems level by level instead of the
    fused pass (KR_OPT_LEVEL_PASSES)."""
    h = handle or default_handle()
    p, _keep = _problem(As, b)
    if x is None:
        x = _x_like(As, p.nrhs, b.dim() == 1)
    info = Info()
    flags = (OPT_LOSS if compute_loss else 0) | (OPT_LEVEL_PASSES if level_passes else 0)
    st = h.lib.kron_ridge(h.ptr, ctypes.byref(p), lam, eps, delta,
                          ctypes.byref(_opts(m, max_iter, tol, seed, stream, check_every,
                                             flags, 0, precision, approx_leverage)),
                          ctypes.c_void_p(x.data_ptr()), ctypes.byref(info))
    h._check(st)
    if st == KR_WMAXITER and not allow_maxiter:
        raise KronRegressError(st, "iteration limit reached")
    return x, info.as_dict()


def kron_ridge_noalloc(As, b, lam, x, eps=0.1, delta=0.01, m=0, seed=0, stream=0, max_iter=200, tol=None,
                       check_every=0, handle=None, precision="f64"):
    """kron_ridge through the allocation-free entry point: the library's fixed
    device scratch (noalloc_capacity() bytes per device) replaces the handle's
    workspace.  x (float64 CUDA tensor, prod(R) or prod(R) x nrhs) is the output,
    allocated by the caller.  Returns (x, info dict)."""
    h = handle or default_handle()
    p, _keep = _problem(As, b)
    info = Info()
    st = h.lib.kron_ridge_noalloc(h.ptr, ctypes.byref(p), lam, eps, delta,
                                  ctypes.byref(_opts(m, max_iter, tol, seed, stream, check_every, 0, 0, precision)),
                                  ctypes.c_void_p(x.data_ptr()), ctypes.byref(info))
    h._check(st)
    return x, info.as_dict()


def noalloc_capacity():
    """Bytes of device scratch behind kron_ridge_noalloc."""
    return int(load_library().kr_noalloc_capacity())


def kron_regress(As, b, eps=0.1, delta=0.01, m=0, seed=0, stream=0, max_iter=200, tol=None,
                 check_every=0, handle=None, x=None, allow_maxiter=True,
                 precision="f64", approx_leverage=None, compute_loss=False, level_passes=False):
    """Algorithm 2 (lambda = 0).  Returns (x float64, info dict); see kron_ridge
    for tol, precision, approx_leverage, compute_loss and level_passes."""
    h = handle or default_handle()
    p, _keep = _problem(As, b)
    if x is None:
        x = _x_like(As, p.nrhs, b.dim() == 1)
    info = Info()
    flags = (OPT_LOSS if compute_loss else 0) | (OPT_LEVEL_PASSES if level_passes else 0)
    st = h.lib.kron_regress(h.ptr, ctypes.byref(p), eps, delta,
                            ctypes.byref(_opts(m, max_iter, tol, seed, stream, check_every,
                                               flags, 0, precision, approx_leverage)),
                            ctypes.c_void_p(x.data_ptr()), ctypes.byref(info))
    h._check(st)
    if st == KR_WMAXITER and not allow_maxiter:
        raise KronRegressError(st, "iteration limit reached")
    return x, info.as_dict()


def kron_ridge_batched(problems, lams, eps=0.1, delta=0.01, m=0, m_rule=None, seed=0, stream=0, max_iter=200,
                       tol=None, handle=None, raise_on_error=True, graph=False, autotune=False, xs=None):
    """Many independent ridge problems in one call (persistent launches for all
    Richardson iterations).  problems: list of (As, b) with As a list of CUDA factor
    tensors (every R_n <= 16) and b a CUDA tensor or a ResponseGen; lams: one
    lambda per problem.  m_rule="rlnr" takes m = ceil(R ln R / eps) per problem
    (with m=0).  Problem i draws with Philox stream `stream + i`.  graph=True
    captures the call's work into a HIP graph and replays it on later calls with
    the same problems and outputs (pass the previous xs to reuse the buffers);
    autotune=True times the candidate launch configurations on the first call
    for a batch shape.  Returns (xs, infos) and, with raise_on_error=False, also
    the call's status (per-problem statuses are in infos)."""
    h = handle or default_handle()
    n = len(problems)
    if len(lams) != n:
        raise ValueError("one lambda per problem")
    probs = (Problem * n)()
    keep, new_xs = [], []
    for i, (As, b) in enumerate(problems):
        p, k = _problem(As, b)
        probs[i] = p
        keep.append(k)
        keep.append(b)
        new_xs.append(xs[i] if xs is not None else _x_like(As, p.nrhs, b.dim() == 1))
    xs = new_xs
    lam_arr = (ctypes.c_double * n)(*[float(v) for v in lams])
    xptr = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    infos = (Info * n)()
    flags = (OPT_M_RLNR if m_rule == "rlnr" else 0) | (OPT_GRAPH if graph else 0) | (OPT_AUTOTUNE if autotune else 0)
    if m_rule not in (None, "rlnr"):
        raise ValueError("m_rule must be None or 'rlnr'")
    st = h.lib.kron_ridge_batched(h.ptr, n, probs, lam_arr, eps, delta,
                                  ctypes.byref(_opts(m, max_iter, tol, seed, stream, 8, flags)), xptr, infos)
    out = [infos[i].as_dict() for i in range(n)]
    if raise_on_error:
        h._check(st)   # raises for a negative status (the first failing problem)
        return xs, out
    return xs, out, st


def batched_config(handle=None):
    """(team threshold in sampled rows x RHS, team workgroups per CU) last chosen
    by the handle's autotuner (the defaults before any tuning)."""
    h = handle or default_handle()
    br, wg = ctypes.c_double(), ctypes.c_int32()
    h._check(h.lib.kr_batched_config(h.ptr, ctypes.byref(br), ctypes.byref(wg)))
    return br.value, wg.value


def kron_loss(As, b, x, lam=0.0, handle=None):
    """||K x - b||^2 + lam ||x||^2 per right-hand side (list of floats)."""
    h = handle or default_handle()
    p, _keep = _problem(As, b)
    if x.dtype != _torch().float64 or not x.is_contiguous():
        raise ValueError("x must be contiguous float64")
    out = (ctypes.c_double * p.nrhs)()
    h._check(h.lib.kron_loss(h.ptr, ctypes.byref(p), lam, ctypes.c_void_p(x.data_ptr()), out))
    return list(out)


def kron_loss_opt(As, gen, x, lam=0.0, handle=None):
    """(losses, OPTs) per right-hand side of an implicit-response problem in one
    pass over its noise: f(x) and f(x*) with x* the exact minimiser."""
    h = handle or default_handle()
    p, _keep = _problem(As, gen)
    if x.dtype != _torch().float64 or not x.is_contiguous():
        raise ValueError("x must be contiguous float64")
    f = (ctypes.c_double * p.nrhs)()
    o = (ctypes.c_double * p.nrhs)()
    h._check(h.lib.kron_loss_opt(h.ptr, ctypes.byref(p), lam, ctypes.c_void_p(x.data_ptr()), f, o))
    return list(f), list(o)


def kron_exact(As, b, lam=0.0, handle=None):
    """The exact minimiser via factor SVDs and KronMatMul (float64)."""
    h = handle or default_handle()
    p, _keep = _problem(As, b)
    x = _x_like(As, p.nrhs, b.dim() == 1)
    h._check(h.lib.kron_exact(h.ptr, ctypes.byref(p), lam, ctypes.c_void_p(x.data_ptr())))
    return x


def tucker_factor_update(X, As, G, mode, lam, eps=0.1, delta=0.01, m=0, seed=0, stream=0, max_iter=400,
                         tol=1e-12, check_every=8, handle=None, out=None):
    """Algorithm 3: the new factor `mode` (float64 I_mode x R_mode) and an info dict.

    X: contiguous CUDA tensor with the full tensor (row-major); As: the N current
    factors (A[mode] supplies its shape); G: the core, float64, shape R_1..R_N."""
    torch = _torch()
    h = handle or default_handle()
    p, _keep = _problem(As, X.reshape(-1))
    if G.dtype != torch.float64 or not G.is_contiguous() or not G.is_cuda:
        raise ValueError("core must be a contiguous float64 CUDA tensor")
    if out is None:
        out = torch.empty(As[mode].shape, dtype=torch.float64, device=As[mode].device)
    info = Info()
    st = h.lib.tucker_factor_update(h.ptr, ctypes.byref(p), ctypes.c_void_p(G.data_ptr()), mode, lam, eps, delta,
                                    ctypes.byref(_opts(m, max_iter, tol, seed, stream, check_every)),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.byref(info))
    h._check(st)
    return out, info.as_dict()


def tucker_factor_exact(X, As, G, mode, lam, handle=None, out=None):
    """Algorithm 1's exact factor update (the ALS baseline): the new factor `mode`
    (float64 I_mode x R_mode).  Arguments as tucker_factor_update."""
    torch = _torch()
    h = handle or default_handle()
    p, _keep = _problem(As, X.reshape(-1))
    if G.dtype != torch.float64 or not G.is_contiguous() or not G.is_cuda:
        raise ValueError("core must be a contiguous float64 CUDA tensor")
    if out is None:
        out = torch.empty(As[mode].shape, dtype=torch.float64, device=As[mode].device)
    h._check(h.lib.tucker_factor_exact(h.ptr, ctypes.byref(p), ctypes.c_void_p(G.data_ptr()), mode, lam,
                                       ctypes.c_void_p(out.data_ptr())))
    return out


def als_stream(sweep, step):
    """Philox stream of ALS step `step` (mode n, or N for the core) of a sweep."""
    return (int(sweep) << 8) | int(step)


def tucker_als(X, G, As, lam, sweeps, eps=0.1, m_core=0, m_factor=0, seed=0, handle=None, tol=1e-12,
               factor_update="sketched", core_update="sketched", stats=None, max_iter=400, core_precision="f64",
               core_tol=None):
    """Algorithm 1 (TuckerALS) driven through the C ABI: for every sweep, the factor
    updates in mode order, then the core update, then the relative reconstruction
    error ||X^ - X||^2 / ||X||^2 from kron_loss.

    factor_update: "sketched" (Algorithm 3, tucker_factor_update with m_factor
    samples per row) or "exact" (tucker_factor_exact, the ALS baseline);
    core_update: "sketched" (Algorithm 2, kron_ridge with b = vec(X) and m_core
    samples) or "exact" (kron_exact); core_precision is the sketched core update's
    kron_ridge precision ("f64", or a refined "f32", "bf16", "fp8": float64 residual
    and update around a low-precision preconditioner) and core_tol its stopping
    tolerance (default: tol in float64, 1e-6 in the refined precisions: their
    float32 adjoint puts a floor under the relative step, about 3e-7 on a poorly
    fitted early sweep).  Every update's status is checked: one that
    does not end in OK raises KronRegressError.  stats, if a list, receives one
    dict per update (sweep, step, iterations, distinct rows, status).  X, G and the
    factors are CUDA tensors (G and the factors float64); returns (G, As, [rre per
    sweep])."""
    torch = _torch()
    if factor_update not in ("sketched", "exact") or core_update not in ("sketched", "exact"):
        raise ValueError("factor_update and core_update are 'sketched' or 'exact'")
    h = handle or default_handle()
    ctol = core_tol if core_tol is not None else (tol if core_precision == "f64" else max(tol, 1e-6))
    As = [A.clone() for A in As]
    G = G.clone()
    N = len(As)
    Xv = X.reshape(-1)
    zero = torch.zeros(G.numel(), dtype=torch.float64, device=G.device)
    xx = kron_loss(As, Xv, zero, 0.0, handle=h)[0]
    trace = []

    def record(s, step, info):
        if info["status"] != "OK":
            raise KronRegressError(KR_WMAXITER if info["status"] == "WMAXITER" else -1,
                                   "ALS sweep %d step %d ended in %s" % (s, step, info["status"]))
        if stats is not None:
            stats.append(dict(sweep=s, step=step, iters=info["iters"], distinct_rows=info["distinct_rows"],
                              status=info["status"]))

    for s in range(sweeps):
        for n in range(N):
            if factor_update == "exact":
                As[n] = tucker_factor_exact(X, As, G, n, lam, handle=h)
            else:
                As[n], info = tucker_factor_update(X, As, G, n, lam, eps=eps, m=m_factor, seed=seed,
                                                   stream=als_stream(s, n), handle=h, tol=tol, max_iter=max_iter)
                record(s, n, info)
        if core_update == "exact":
            g = kron_exact(As, Xv, lam, handle=h)
        else:
            g, info = kron_ridge(As, Xv, lam, eps=eps, m=m_core, seed=seed, stream=als_stream(s, N), handle=h,
                                 tol=ctol, max_iter=max_iter, precision=core_precision)
            record(s, N, info)
        G = g.reshape(G.shape)
        trace.append(kron_loss(As, Xv, g, 0.0, handle=h)[0] / xx)
    return G, As, trace


def tucker_als_native(X, G, As, lam, sweeps, eps=0.1, m_core=0, m_factor=0, seed=0, handle=None, tol=1e-12,
                      max_iter=400, core_precision="f64", core_tol=None, delta=0.01):
    """Algorithm 1 with the sketched updates through kr_tucker_als: the same
    updates, streams and order as tucker_als(factor_update="sketched",
    core_update="sketched"), looped inside the library.  Returns (G, As, [rre per
    sweep], [iterations per update]); raises KronRegressError at the first update
    that does not end in OK."""
    torch = _torch()
    h = handle or default_handle()
    As = [A.clone() for A in As]
    G = G.clone()
    if G.dtype != torch.float64 or any(A.dtype != torch.float64 for A in As):
        raise ValueError("the core and the factors must be float64")
    N = len(As)
    p, _keep = _problem(As, X.reshape(-1))
    ctol = core_tol if core_tol is not None else (tol if core_precision == "f64" else max(tol, 1e-6))
    fo = _opts(m_factor, max_iter, tol, seed, 0, 8)
    co = _opts(m_core, max_iter, ctol, seed, 0, 0, 0, 0, core_precision)
    rre = (ctypes.c_double * max(1, sweeps))()
    iters = (ctypes.c_int32 * max(1, sweeps * (N + 1)))()
    failed = ctypes.c_int32(-1)
    st = h.lib.kr_tucker_als(h.ptr, ctypes.byref(p), ctypes.c_void_p(G.data_ptr()), lam, eps, delta, sweeps,
                             ctypes.byref(fo), ctypes.byref(co), rre, iters, ctypes.byref(failed))
    h._check(st)
    if st != KR_OK:
        raise KronRegressError(st, "ALS update %d ended with status %s" % (failed.value, STATUS_NAMES.get(st, st)))
    return G, As, [rre[s] for s in range(sweeps)], [iters[k] for k in range(sweeps * (N + 1))]


def profile_enable(enable=True, kernel_filter="", handle=None):
    """Bracket kernel launches whose name contains kernel_filter ("" = all) with HIP
    events on the handle's stream (clears old records)."""
    h = handle or default_handle()
    h._check(h.lib.kr_profile_enable(h.ptr, 1 if enable else 0, kernel_filter.encode()))


def profile_query(kernel, handle=None):
    """(launches, total device ms) recorded for a kernel name since profile_enable."""
    h = handle or default_handle()
    n, ms = ctypes.c_int64(), ctypes.c_double()
    h._check(h.lib.kr_profile_query(h.ptr, kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def profile_names(handle=None):
    """Kernel names recorded since profile_enable."""
    h = handle or default_handle()
    buf = ctypes.create_string_buffer(65536)
    h._check(h.lib.kr_profile_list(h.ptr, buf, len(buf)))
    return [n for n in buf.value.decode().split("\n") if n]


def profile_breakdown(handle=None):
    """{kernel: (launches, total ms)} for every kernel recorded since profile_enable."""
    return {n: profile_query(n, handle) for n in profile_names(handle)}


def _export(call, sizes):
    import numpy as np
    D = ctypes.c_int64()
    call(None, None, None, None, 0, ctypes.byref(D))
    D = D.value
    N = len(sizes)
    Q = np.zeros(int(sum(sizes)), dtype=np.uint64)
    rows = np.zeros((D, N), dtype=np.int32)
    Omega = np.zeros(D, dtype=np.float64)
    counts = np.zeros(D, dtype=np.int32)
    call(Q.ctypes.data, rows.ctypes.data, Omega.ctypes.data, counts.ctypes.data, D, ctypes.byref(ctypes.c_int64()))
    offs = np.cumsum([0] + list(sizes))
    return {"Q": [Q[offs[n]:offs[n + 1]] for n in range(N)], "rows": rows.astype(np.int64),
            "Omega": Omega, "counts": counts.astype(np.int64)}


def export_sketch(sizes, handle=None):
    """The last solve's sketch: Q tables per mode, distinct rows (D x N), Omega, counts."""
    h = handle or default_handle()
    return _export(lambda *a: h._check(h.lib.kr_export_sketch(h.ptr, *a)), sizes)


def export_samples(first, count, N, handle=None):
    """Samples first .. first + count - 1 of the last single solve, drawn again from
    its kept tables before merging: an int32 (count, N) array of per-mode indices
    in sample order."""
    import numpy as np
    h = handle or default_handle()
    idx = np.zeros((int(count), int(N)), dtype=np.int32)
    h._check(h.lib.kr_export_samples(h.ptr, int(first), int(count), idx.ctypes.data))
    return idx


def export_batched_sketch(problem, sizes, handle=None):
    """The sketch of problem `problem` of the last kron_ridge_batched call, in the
    caller's mode order (same form as export_sketch)."""
    h = handle or default_handle()
    return _export(lambda *a: h._check(h.lib.kr_export_batched_sketch(h.ptr, int(problem), *a)), sizes)


def export_leverage(sizes, problem=-1, handle=None):
    """Float64 leverage scores of every factor (list per mode) of the last single
    solve (problem=-1) or of problem `problem` of the last batched call."""
    import numpy as np
    h = handle or default_handle()
    lev = np.zeros(int(sum(sizes)), dtype=np.float64)
    h._check(h.lib.kr_export_leverage(h.ptr, int(problem), lev.ctypes.data, lev.size))
    offs = np.cumsum([0] + list(sizes))
    return [lev[offs[n]:offs[n + 1]] for n in range(len(sizes))]


__all__ = ["Handle", "KronRegressError", "ResponseGen", "kron_regress", "kron_ridge", "kron_ridge_noalloc",
           "kron_loss_opt",
           "noalloc_capacity", "kron_ridge_noalloc", "kron_loss", "kron_exact",
           "tucker_factor_update", "tucker_factor_exact", "tucker_als", "als_stream",
           "export_sketch", "export_batched_sketch", "export_leverage", "load_library", "default_handle", "profile_enable", "profile_query",
           "profile_names", "profile_breakdown"]
