"""GPU parity of the refined (mixed-precision) Richardson iteration against the oracle.

The refined precisions change only the arithmetic of the iteration: the sketch
(sample indices, multiplicities, weights) is bit-exact with the oracle as in
float64 mode, and the fixed point is the sketched minimiser x~_64, which the
oracle computes directly in float64 from the same samples.  The bar is the
relative loss gap |f(x_mp) - f(x~_64)| / f(x~_64) <= 1e-6 with f the full float64
loss, plus rel-L2(x_mp, x~_64) <= 1e-6."""

import numpy as np
import pytest

import workloads
from oracle.regression import exact_solution, kron_rows, loss
from parity import check_quantised_tables, check_sketch, rel_l2, sketched_solution

pytestmark = pytest.mark.gpu

GAP = 1e-6
XTOL = 1e-6
PRECS = ["f32", "bf16", "fp8"]

CASES = [
    # name, I, R, m, nrhs, lam, heavy
    ("C1 shape ridge", (64, 64), (8, 8), 2048, 1, 0.05, 0),
    ("two blocks ragged tiles", (40, 36, 30), (12, 20, 7), 30000, 2, 0.0, 0),
    ("two blocks ridge", (40, 36, 30), (12, 20, 7), 30000, 1, 0.01, 0),
    ("global buffers nrhs 32", (20, 20, 20), (6, 6, 6), 5000, 32, 0.0, 0),
    ("N1", (50,), (9,), 400, 1, 0.0, 0),
    ("N4", (12, 10, 9, 8), (3, 4, 2, 3), 8000, 1, 0.0, 0),
]


def _torch_inputs(As, b):
    import torch
    return ([torch.tensor(A, device="cuda").contiguous() for A in As],
            torch.tensor(b, device="cuda").contiguous())


def _gap(As, b, x, x64, lam):
    b2 = np.asarray(b).reshape(np.asarray(b).shape[0], -1)
    x2, y2 = x.reshape(x.shape[0], -1), x64.reshape(x64.shape[0], -1)
    gaps = []
    for q in range(b2.shape[1]):
        f = loss(As, b2[:, q], x2[:, q], lam)
        f64 = loss(As, b2[:, q], y2[:, q], lam)
        gaps.append(abs(f - f64) / f64)
    return max(gaps)


@pytest.mark.parametrize("prec", PRECS)
def test_small_regression_refined(gpu_lib, prec):
    """The C1 workload (N=2, 64x8 factors, m=2048, Philox seed 0) in each refined
    precision: same sketch as the oracle, loss gap <= 1e-6 against x~_64."""
    w = workloads.small_regression()
    print("case small_regression precision", prec, flush=True)
    tA, tb = _torch_inputs(w["As"], w["b"])
    x, info = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"], precision=prec)
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch([A.shape[0] for A in w["As"]])
    check_quantised_tables(w["As"], sk["Q"])
    rows, ridx, counts, Omega = check_sketch(w["As"], sk, w["m"], seed=w["seed"])
    x64 = sketched_solution(w["As"], w["b"], rows, ridx, Omega, 0.0)
    xg = x.cpu().numpy()
    gap = _gap(w["As"], w["b"], xg, x64, 0.0)
    opt = loss(w["As"], w["b"], exact_solution(w["As"], w["b"]))
    f = loss(w["As"], w["b"], xg)
    print("iters %d gap %.2e rel-L2 %.2e f/opt %.6f" % (info["iters"], gap, rel_l2(xg, x64), f / opt), flush=True)
    assert gap <= GAP
    assert rel_l2(xg, x64) <= XTOL
    assert f <= (1 + w["eps"]) * opt


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_refined_parity(gpu_lib, case, prec):
    name, I, R, m, nrhs, lam, heavy = case
    print("case", name, "precision", prec, I, R, m, nrhs, lam, flush=True)
    w = workloads.random_problem(I, R, seed=len(name) * 7 + nrhs, nrhs=nrhs, heavy=heavy, sigma=0.05)
    As, b = w["As"], w["b"]
    tA, tb = _torch_inputs(As, b)
    x, info = gpu_lib.kron_ridge(tA, tb, lam, eps=0.1, m=m, seed=11, stream=2, precision=prec, max_iter=400)
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch(I)
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=11, stream=2)
    x64 = sketched_solution(As, b, rows, ridx, Omega, lam)
    xg = x.cpu().numpy()
    gap = _gap(As, b, xg, x64, lam)
    print("iters %d gap %.2e rel-L2 %.2e" % (info["iters"], gap, rel_l2(xg, x64)), flush=True)
    assert gap <= GAP
    assert rel_l2(xg, x64) <= XTOL


@pytest.mark.parametrize("prec", PRECS)
def test_refined_ill_conditioned_fails_loudly(gpu_lib, prec):
    """Heavy rows make kappa(K^T K) ~ 1e14: a low-precision preconditioner may no
    longer contract.  The solve must then end in KR_EDIVERGED (or, if it converges,
    meet the same bar) -- never return a silent wrong answer."""
    I, R, m = (12, 10, 9, 8), (3, 4, 2, 3), 8000
    name = "N4 heavy rows"
    print("case", name, "precision", prec, flush=True)
    w = workloads.random_problem(I, R, seed=len(name) * 7 + 1, heavy=2, sigma=0.05)
    As, b = w["As"], w["b"]
    tA, tb = _torch_inputs(As, b)
    try:
        x, info = gpu_lib.kron_regress(tA, tb, eps=0.1, m=m, seed=11, stream=2, precision=prec, max_iter=400)
    except gpu_lib.KronRegressError as e:
        print("status", e.status, flush=True)
        assert e.status == -5
        return
    sk = gpu_lib.export_sketch(I)
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=11, stream=2)
    x64 = sketched_solution(As, b, rows, ridx, Omega, 0.0)
    xg = x.cpu().numpy()
    print("status %s iters %d rel-L2 %.2e rel_update %.2e" % (info["status"], info["iters"], rel_l2(xg, x64),
                                                             info["rel_update"]), flush=True)
    assert info["status"] in ("OK", "WMAXITER"), info
    if info["status"] == "OK":
        assert rel_l2(xg, x64) <= XTOL
    else:
        # a truthful WMAXITER: the stopping rule (default tol 1e-9) was indeed not met
        assert info["iters"] == 400 and info["rel_update"] > 1e-9, info


def test_refined_same_samples_as_f64(gpu_lib):
    """Precision does not touch the sketch: the exported samples of a bf16 solve
    equal those of a float64 solve bit for bit."""
    w = workloads.random_problem((30, 20, 10), (3, 4, 2), seed=5)
    tA, tb = _torch_inputs(w["As"], w["b"])
    print("case same samples f64 vs bf16", flush=True)
    gpu_lib.kron_regress(tA, tb, m=3000, seed=4, precision="f64")
    a = gpu_lib.export_sketch([30, 20, 10])
    gpu_lib.kron_regress(tA, tb, m=3000, seed=4, precision="bf16")
    c = gpu_lib.export_sketch([30, 20, 10])
    for k in ("rows", "counts", "Omega"):
        np.testing.assert_array_equal(a[k], c[k])


def test_refined_rejects_tucker_and_unknown_precisions(gpu_lib):
    import torch
    w = workloads.random_problem((10, 9), (2, 3), seed=1)
    tA, tb = _torch_inputs(w["As"], w["b"])
    print("case refined error paths", flush=True)
    with pytest.raises(ValueError):
        gpu_lib.kron_regress(tA, tb, m=200, precision="fp16")
    X = torch.zeros((6, 5, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.KronRegressError) as e:
        lib = gpu_lib
        h = lib.default_handle()
        p, _keep = lib._problem([torch.ones((6, 2), dtype=torch.float64, device="cuda"),
                                 torch.ones((5, 2), dtype=torch.float64, device="cuda"),
                                 torch.ones((4, 2), dtype=torch.float64, device="cuda")], X.reshape(-1))
        G = torch.ones((2, 2, 2), dtype=torch.float64, device="cuda")
        out = torch.empty((6, 2), dtype=torch.float64, device="cuda")
        info = lib.Info()
        import ctypes
        st = h.lib.tucker_factor_update(h.ptr, ctypes.byref(p), ctypes.c_void_p(G.data_ptr()), 0, 0.1, 0.1, 0.01,
                                        ctypes.byref(lib._opts(100, 50, 0.0, 0, 0, 8, 0, 0, "bf16")),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.byref(info))
        h._check(st)
    assert e.value.status == -6
