"""GPU parity at the benchmark's full size: N=3 factors 512x16 with 26 heavy rows per
mode, K is 1.34e8 x 4096, m = 340,696 (the launch configuration bench.py times).

Every sample index is checked (bit-exact, via the GPU's quantised tables), the
leverage scores against the oracle's, the solution against the oracle's direct
sketched minimiser (rel-L2 <= 1e-10), the float64 loss against the oracle's, the
exact KronMatMul solution against the oracle's, and the (1 + eps) gate.  The
refined precisions (f32, bf16, fp8) draw the same sketch and reach the same
minimiser x~_64: loss gap |f(x_mp) - f(x~_64)| / f(x~_64) <= 1e-6 and
rel-L2(x_mp, x~_64) <= 1e-6 with f the full float64 loss."""

import numpy as np
import pytest

import workloads
from oracle.leverage import leverage_scores
from oracle.regression import exact_solution, kron_rows, loss, solve_sketched_direct
from parity import check_quantised_tables, check_sketch, rel_l2

pytestmark = pytest.mark.gpu

GAP = 1e-6
XTOL = 1e-6


@pytest.fixture(scope="module")
def skewed():
    return workloads.skewed_regression()


@pytest.fixture(scope="module")
def skewed_ref(gpu_lib, skewed):
    """The float64 solve on the GPU and the oracle's direct minimiser of the same
    (bit-exact) sketch, the loss at that minimiser and OPT."""
    import torch
    w = skewed
    print("case skewed_regression full size, m=%d" % w["m"], flush=True)
    tA = [torch.tensor(A, device="cuda") for A in w["As"]]
    tb = torch.from_numpy(w["b"]).cuda()
    x, info = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"], tol=1e-12)
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch([512, 512, 512])
    lev = gpu_lib.export_leverage([512, 512, 512])
    straddles = check_quantised_tables(w["As"], sk["Q"])
    print("quantisation straddles:", straddles, flush=True)
    rows, ridx, counts, Omega = check_sketch(w["As"], sk, w["m"], seed=w["seed"])
    KD = kron_rows(w["As"], ridx)
    xo = solve_sketched_direct(KD, Omega, w["b"][rows], 0.0)
    del KD
    xs = exact_solution(w["As"], w["b"])
    return dict(tA=tA, tb=tb, x=x.cpu().numpy(), info=info, lev=lev, counts=counts, xo=xo,
                fo=loss(w["As"], w["b"], xo), opt=loss(w["As"], w["b"], xs), xs=xs)


def test_skewed_full_size(gpu_lib, skewed, skewed_ref):
    w, r = skewed, skewed_ref
    assert r["counts"].sum() == w["m"]
    err = rel_l2(r["x"], r["xo"])
    print("rel-L2 vs direct sketched minimiser: %.3e" % err, flush=True)
    assert err < 1e-10
    import torch
    fg = gpu_lib.kron_loss(r["tA"], r["tb"], torch.from_numpy(r["x"]).cuda())[0]
    fo = loss(w["As"], w["b"], r["x"])
    assert abs(fg - fo) <= 1e-10 * fo
    xe = gpu_lib.kron_exact(r["tA"], r["tb"]).cpu().numpy()
    assert rel_l2(xe, r["xs"]) < 1e-10
    print("loss / opt = %.6f" % (fo / r["opt"]), flush=True)
    assert fo <= 1.1 * r["opt"]


def test_skewed_leverage_values(skewed, skewed_ref):
    """The GPU's float64 leverage scores (Cholesky route) against the oracle's
    (Householder QR / SVD route), every entry of every mode, within 1e-13."""
    for n, A in enumerate(skewed["As"]):
        lo = leverage_scores(A)
        d = float(np.max(np.abs(skewed_ref["lev"][n] - lo)))
        print("mode %d: max |l_gpu - l_oracle| = %.2e, sum l = %.15f" % (n, d, skewed_ref["lev"][n].sum()), flush=True)
        assert d <= 1e-13


# Stopping tolerance per precision at this size.  The loss here is about 1e12
# times more sensitive to x than at the small workload (||K x||^2 / OPT is huge:
# heavy rows scaled x100 in every mode), so the default 1e-9 leaves a loss gap of
# about 1.2e-6; 3e-10 (1e-10 for fp8, whose preconditioner contracts more slowly)
# brings it below 1e-6 (measured: f32 2.5e-8, bf16 1.4e-7, fp8 2.8e-7).
TOL = {"f32": 3e-10, "bf16": 3e-10, "fp8": 1e-10}


@pytest.mark.parametrize("prec", ["f32", "bf16", "fp8"])
def test_skewed_refined(gpu_lib, skewed, skewed_ref, prec):
    """The refined precisions at full size: the same sketch as float64 (bit for
    bit), and the sketched minimiser x~_64 reached to the refined bar."""
    w, r = skewed, skewed_ref
    print("case skewed_regression precision", prec, "tol", TOL[prec], flush=True)
    x, info = gpu_lib.kron_regress(r["tA"], r["tb"], eps=w["eps"], m=w["m"], seed=w["seed"], precision=prec,
                                   tol=TOL[prec])
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch([512, 512, 512])
    np.testing.assert_array_equal(sk["counts"], r["counts"])
    xg = x.cpu().numpy()
    f = loss(w["As"], w["b"], xg)
    gap = abs(f - r["fo"]) / r["fo"]
    err = rel_l2(xg, r["xo"])
    print("iters %d gap %.2e rel-L2 %.2e f/opt %.6f" % (info["iters"], gap, err, f / r["opt"]), flush=True)
    assert gap <= GAP
    assert err <= XTOL
    assert f <= 1.1 * r["opt"]
