"""GPU parity of the fused three-factor pass (k_subtree3: forward level 1, the rows
and adjoint level 2 in one launch per run of level-2 prefixes, then the root
adjoint over the runs) against the level-by-level passes and the oracle.

For each case the solve runs twice on the same sketch: fused (the default for
three factors) and with level_passes=True.  The profiled kernel names show which
path ran; both solutions must match the oracle's direct sketched minimiser to
rel-L2 1e-10 (float64) or the refined bar (loss gap 1e-6), and each other to the
same tolerance.  A tree whose runs outnumber the chunk table's capacity must
fall back to the level passes (bit-identical to level_passes=True)."""

import zlib

import numpy as np
import pytest

import workloads
from parity import check_sketch, rel_l2, sketched_solution

pytestmark = pytest.mark.gpu

CASES = [
    # name, I, R, m, nrhs, lam, heavy, precision
    ("R3 8 lanes", (40, 33, 20), (4, 5, 3), 20000, 1, 0.0, 3, "f64"),
    ("R3 16 lanes heavy", (60, 50, 40), (3, 4, 12), 30000, 1, 0.0, 4, "f64"),
    ("nrhs 2", (30, 25, 20), (3, 3, 4), 8000, 2, 0.0, 2, "f64"),
    ("nrhs 3 ridge", (30, 25, 20), (3, 3, 4), 8000, 3, 0.3, 2, "f64"),
    ("nrhs 9 one child per run", (20, 18, 16), (2, 3, 2), 4000, 9, 0.0, 0, "f64"),
    ("ragged runs", (7, 300, 9), (2, 6, 3), 5000, 1, 0.0, 0, "f64"),
    ("bf16 refined", (60, 50, 40), (3, 4, 12), 30000, 1, 0.0, 0, "bf16"),
    ("f32 refined ridge", (40, 33, 20), (4, 5, 3), 20000, 2, 0.1, 3, "f32"),
]


def _inputs(As, b):
    import torch
    tA = [torch.tensor(A, dtype=torch.float64, device="cuda").contiguous() for A in As]
    tb = torch.tensor(b, dtype=torch.float64, device="cuda").contiguous()
    return tA, tb


def _solve(gpu_lib, tA, tb, lam, m, precision, level_passes):
    gpu_lib.profile_enable(True, "k_subtree3|k_adj_level|k_fwd_level")
    tol = 1e-12 if precision == "f64" else 1e-10
    x, info = gpu_lib.kron_ridge(tA, tb, lam, eps=0.1, m=m, seed=11, stream=5, tol=tol, max_iter=400,
                                 precision=precision, level_passes=level_passes)
    # the adjoint level runs as k_adj_level or, in float64 with R <= 16, as
    # k_adj_level_mfma: both count as the level passes
    names = set(n.split("<")[0].replace("k_adj_level_mfma", "k_adj_level") for n in gpu_lib.profile_names())
    gpu_lib.profile_enable(False)
    return x.cpu().numpy(), info, names


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused_matches_level_passes_and_oracle(gpu_lib, case):
    name, I, R, m, nrhs, lam, heavy, precision = case
    print("case fused", name, I, R, m, nrhs, lam, precision, flush=True)
    w = workloads.random_problem(I, R, seed=zlib.crc32(name.encode()) % 1000, nrhs=nrhs, heavy=heavy)
    As, b = w["As"], w["b"]
    tA, tb = _inputs(As, b)
    xf, info_f, names_f = _solve(gpu_lib, tA, tb, lam, m, precision, False)
    assert info_f["status"] == "OK", info_f
    assert "k_subtree3" in names_f and "k_adj_level" not in names_f and "k_fwd_level" not in names_f, names_f
    sk = gpu_lib.export_sketch(list(I))
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=11, stream=5)
    xl, info_l, names_l = _solve(gpu_lib, tA, tb, lam, m, precision, True)
    assert info_l["status"] == "OK", info_l
    assert "k_adj_level" in names_l and "k_subtree3" not in names_l, names_l
    xo = sketched_solution(As, b, rows, ridx, Omega, lam)
    if precision == "f64":
        for x in (xf, xl):
            assert rel_l2(x, xo) <= 1e-10, (rel_l2(xf, xo), rel_l2(xl, xo))
        assert rel_l2(xf, xl) <= 1e-10
    else:
        bD = b.reshape(-1, nrhs)[rows] if nrhs > 1 else b.reshape(-1)[rows]
        from oracle.regression import kron_rows
        KD = kron_rows(As, ridx) * np.sqrt(Omega)[:, None]
        bW = (bD.T * np.sqrt(Omega)).T

        def f(x):
            r = KD @ x.reshape(KD.shape[1], -1) - bW.reshape(KD.shape[0], -1)
            return float(np.sum(r * r) + lam * np.sum(x * x))
        fo = f(xo)
        for x in (xf, xl):
            assert abs(f(x) - fo) <= 1e-6 * fo + 1e-14 * float(np.sum(bW ** 2)), (f(xf), f(xl), fo)
            assert rel_l2(x, xo) <= 1e-6, (rel_l2(xf, xo), rel_l2(xl, xo))


def test_fused_falls_back_when_runs_exceed_the_table(gpu_lib):
    """Four level-1 prefixes over about 86,000 level-2 prefixes (mode-1 leverage of
    a 30000 x 2 Gaussian factor is about Exp(1) / 15000, so a pair is drawn with
    probability 1 - 1/(1 + 2.5 X)): about 10,700 runs of 8, more than the table's
    2 S_1 + 4096 = 4104, so the level passes run."""
    print("case fused fallback", flush=True)
    I, R, m = (4, 30000, 6), (2, 2, 2), 300000
    w = workloads.random_problem(I, R, seed=41)
    tA, tb = _inputs(w["As"], w["b"])
    x1, i1, n1 = _solve(gpu_lib, tA, tb, 0.0, m, "f64", False)
    x2, i2, n2 = _solve(gpu_lib, tA, tb, 0.0, m, "f64", True)
    assert "k_subtree3" not in n1 and "k_adj_level" in n1, n1
    assert i1["status"] == i2["status"] == "OK"
    assert np.array_equal(x1, x2)


def test_fused_is_deterministic(gpu_lib):
    print("case fused determinism", flush=True)
    w = workloads.random_problem((50, 40, 30), (4, 4, 8), seed=3, heavy=3)
    tA, tb = _inputs(w["As"], w["b"])
    xa, _, na = _solve(gpu_lib, tA, tb, 0.0, 20000, "f64", False)
    xb, _, _ = _solve(gpu_lib, tA, tb, 0.0, 20000, "f64", False)
    assert "k_subtree3" in na
    assert np.array_equal(xa, xb)
