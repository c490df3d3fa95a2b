"""GPU parity at the benchmark's full size: N=3 factors 512x16 with 26 heavy rows per
mode, K is 1.34e8 x 4096, m = 340,696 (the launch configuration bench.py times).

Every sample index is checked (bit-exact, via the GPU's quantised tables), the
solution against the oracle's direct sketched minimiser (rel-L2 <= 1e-10), the
float64 loss against the oracle's, the exact KronMatMul solution against the
oracle's, and the (1 + eps) gate."""

import numpy as np
import pytest

import workloads
from oracle.regression import exact_solution, kron_rows, loss, solve_sketched_direct
from parity import check_quantised_tables, check_sketch, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def skewed():
    return workloads.skewed_regression()


def test_skewed_full_size(gpu_lib, skewed):
    import torch
    w = skewed
    print("case skewed_regression full size, m=%d" % w["m"], flush=True)
    tA = [torch.tensor(A, device="cuda") for A in w["As"]]
    tb = torch.from_numpy(w["b"]).cuda()
    x, info = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"], tol=1e-12)
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch([512, 512, 512])
    straddles = check_quantised_tables(w["As"], sk["Q"])
    print("quantisation straddles:", straddles, flush=True)
    rows, ridx, counts, Omega = check_sketch(w["As"], sk, w["m"], seed=w["seed"])
    assert counts.sum() == w["m"]
    KD = kron_rows(w["As"], ridx)
    xo = solve_sketched_direct(KD, Omega, w["b"][rows], 0.0)
    xg = x.cpu().numpy()
    err = rel_l2(xg, xo)
    print("rel-L2 vs direct sketched minimiser: %.3e" % err, flush=True)
    assert err < 1e-10
    fg = gpu_lib.kron_loss(tA, tb, x)[0]
    fo = loss(w["As"], w["b"], xg)
    assert abs(fg - fo) <= 1e-10 * fo
    xs = exact_solution(w["As"], w["b"])
    xe = gpu_lib.kron_exact(tA, tb).cpu().numpy()
    assert rel_l2(xe, xs) < 1e-10
    opt = loss(w["As"], w["b"], xs)
    print("loss / opt = %.6f" % (fo / opt), flush=True)
    assert fo <= 1.1 * opt
