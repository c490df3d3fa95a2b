"""GPU parity of Algorithm 2 (kron_regress / kron_ridge) against the oracle.

Each case prints its name before touching the GPU.  Sample indices, multiplicities
and merged weights must match the oracle bit for bit (using the GPU's quantised
tables, which must themselves equal the oracle's up to boundary straddles); the
solution must match the oracle's direct sketched minimiser to rel-L2 1e-10 in
float64 where kappa(K)^2 u is below that.  For the ill-conditioned cases (square
factors, heavy rows) the attainable accuracy of x from the normal-equation form
that Richardson iterates is about kappa(K)^2 u; there x is held to 20 kappa^2 u,
the fitted values sqrt(Omega) K_D x to max(1e-10, 20 kappa u) and the sketched
loss to a relative gap of 1e-10 in every case."""

import zlib

import numpy as np
import pytest

import workloads
from oracle.regression import exact_solution, loss
from parity import check_quantised_tables, check_sketch, rel_l2, sketched_solution

pytestmark = pytest.mark.gpu

CASES = [
    # name, I, R, m, nrhs, lam, heavy
    ("N1", (6,), (2,), 50, 1, 0.0, 0),
    ("N2 small", (7, 5), (2, 3), 300, 1, 0.0, 0),
    ("N3 ragged tile", (9, 6, 5), (3, 2, 2), 4097, 1, 0.0, 0),
    ("N4", (5, 4, 6, 3), (2, 2, 3, 1), 800, 1, 0.0, 0),
    ("unit mode", (1, 5, 4), (1, 2, 2), 300, 1, 0.0, 0),
    ("square factors", (4, 3, 5), (4, 3, 5), 2000, 1, 0.0, 0),   # kappa(K) ~ 5e4
    ("heavy rows", (40, 33, 20), (4, 5, 3), 20000, 1, 0.0, 3),
    ("nrhs 3", (20, 15), (3, 4), 1000, 3, 0.0, 0),
    ("ridge", (30, 20, 10), (3, 4, 2), 3000, 1, 0.5, 0),
    ("ridge nrhs 2", (12, 11, 9), (2, 3, 3), 1500, 2, 0.01, 2),
    ("R 17 lanes 32", (40, 30), (17, 5), 4000, 1, 0.0, 0),
    ("few samples", (8, 8), (2, 2), 3, 1, 0.0, 0),
]


def _torch_inputs(As, b, dtype=None):
    import torch
    dt = dtype or torch.float64
    tA = [torch.tensor(A, dtype=dt, device="cuda").contiguous() for A in As]
    tb = torch.tensor(b, dtype=dt, device="cuda").contiguous()
    return tA, tb


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_regress_parity(gpu_lib, case):
    name, I, R, m, nrhs, lam, heavy = case
    print("case", name, I, R, m, nrhs, lam, flush=True)
    w = workloads.random_problem(I, R, seed=zlib.crc32(name.encode()) % 1000, nrhs=nrhs, heavy=heavy)
    As, b = w["As"], w["b"]
    tA, tb = _torch_inputs(As, b)
    x, info = gpu_lib.kron_ridge(tA, tb, lam, eps=0.1, m=m, seed=7, stream=3, tol=1e-12, max_iter=400)
    # Richardson's attainable accuracy is about kappa(K)^2 u (normal-equation form);
    # below that floor the stopping rule cannot be met and the last iterate is returned
    kappa2u = float(np.prod([np.linalg.cond(A) for A in As])) ** 2 * 2.2e-16
    xtol = max(1e-10, 20 * kappa2u)
    assert info["status"] == "OK" or (info["status"] == "WMAXITER" and kappa2u > 1e-12), info
    sk = gpu_lib.export_sketch(I)
    check_quantised_tables(As, sk["Q"])
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=7, stream=3)
    assert info["distinct_rows"] == len(rows)
    xg = x.cpu().numpy()
    if len(rows) < int(np.prod(R)) and lam == 0.0:
        # rank-deficient sketch: the minimiser is not unique; check the sketched
        # normal equations K_D^T Omega (K_D x - b_D) = 0 instead
        from oracle.regression import kron_rows
        KD = kron_rows(As, ridx)
        bD = np.asarray(b)[rows].reshape(len(rows), -1)
        res = KD.T @ (Omega[:, None] * (KD @ xg.reshape(KD.shape[1], -1) - bD))
        ref = KD.T @ (Omega[:, None] * bD)
        assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(ref)
        return
    xo = sketched_solution(As, b, rows, ridx, Omega, lam)
    # the fitted values sqrt(Omega) K_D x of the sketched problem: their error is
    # about kappa u for a normal-equation method, where x's is kappa^2 u
    from oracle.regression import kron_rows
    KW = kron_rows(As, ridx) * np.sqrt(Omega)[:, None]
    fit = rel_l2(KW @ xg.reshape(KW.shape[1], -1), KW @ xo.reshape(KW.shape[1], -1))
    # the loss of the sketched problem at both points: its relative gap is
    # second order in the error of the fitted values
    kappau = float(np.prod([np.linalg.cond(A) for A in As])) * 2.2e-16
    fit_tol = max(1e-10, 20 * kappau)
    bW = np.asarray(b)[rows].reshape(len(rows), -1) * np.sqrt(Omega)[:, None]
    fs = np.sum((KW @ xg.reshape(KW.shape[1], -1) - bW) ** 2) + lam * np.sum(xg ** 2)
    fso = np.sum((KW @ xo.reshape(KW.shape[1], -1) - bW) ** 2) + lam * np.sum(xo ** 2)
    print("rel-L2 x %.3e (bar %.1e), fitted values %.3e (bar %.1e), sketched-loss gap %.2e" % (
        rel_l2(xg, xo), xtol, fit, fit_tol, abs(fs - fso) / fso), flush=True)
    assert rel_l2(xg, xo) < xtol, (name, rel_l2(xg, xo), xtol)
    assert fit < fit_tol, (name, fit, fit_tol)
    # (a consistent sketched problem -- square factors -- has fso ~ 0: the gap is
    # then measured against the scale of b~)
    assert abs(fs - fso) <= 1e-10 * fso + 1e-14 * float(np.sum(bW ** 2))


def test_small_regression_workload(gpu_lib):
    print("case small_regression", flush=True)
    w = workloads.small_regression()
    tA, tb = _torch_inputs(w["As"], w["b"])
    x, info = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"], tol=1e-13)
    assert info["status"] == "OK"
    sk = gpu_lib.export_sketch([64, 64])
    assert check_quantised_tables(w["As"], sk["Q"]) == 0
    rows, ridx, _, Omega = check_sketch(w["As"], sk, w["m"], seed=w["seed"])
    xo = sketched_solution(w["As"], w["b"], rows, ridx, Omega, 0.0)
    assert rel_l2(x.cpu().numpy(), xo) < 1e-10
    opt = loss(w["As"], w["b"], exact_solution(w["As"], w["b"]))
    f = gpu_lib.kron_loss(tA, tb, x)[0]
    assert abs(f - loss(w["As"], w["b"], x.cpu().numpy())) < 1e-12 * f
    assert f <= 1.1 * opt


def test_deterministic_repeat(gpu_lib):
    print("case determinism", flush=True)
    w = workloads.random_problem((30, 25, 20), (3, 3, 2), seed=4, heavy=2)
    tA, tb = _torch_inputs(w["As"], w["b"])
    x1, _ = gpu_lib.kron_regress(tA, tb, m=5000, seed=1)
    x2, _ = gpu_lib.kron_regress(tA, tb, m=5000, seed=1)
    assert bool((x1 == x2).all())


@pytest.mark.parametrize("lam,nrhs,f32", [(0.0, 1, False), (0.3, 2, False), (0.0, 1, True)])
def test_exact_and_loss(gpu_lib, lam, nrhs, f32):
    import torch
    print("case exact/loss", lam, nrhs, f32, flush=True)
    w = workloads.random_problem((11, 9, 7), (3, 2, 4), seed=5, nrhs=nrhs)
    As, b = w["As"], w["b"]
    if f32:
        As = [A.astype(np.float32).astype(np.float64) for A in As]
        b = b.astype(np.float32).astype(np.float64)
    tA, tb = _torch_inputs(As, b, torch.float32 if f32 else torch.float64)
    x = gpu_lib.kron_exact(tA, tb, lam)
    xo = exact_solution(As, b, lam)
    assert rel_l2(x.cpu().numpy(), xo) < 1e-10
    f = gpu_lib.kron_loss(tA, tb, x, lam)
    for q in range(nrhs):
        xq = xo if nrhs == 1 else xo[:, q]
        bq = b if nrhs == 1 else b[:, q]
        fo = loss(As, bq, xq, lam)
        assert abs(f[q] - fo) < 1e-11 * fo


def test_error_paths(gpu_lib):
    import torch
    print("case errors", flush=True)
    w = workloads.random_problem((10, 8), (3, 2), seed=6)
    As = [A.copy() for A in w["As"]]
    As[0][:, 2] = As[0][:, 1]            # duplicated column: singular Gram
    tA, tb = _torch_inputs(As, w["b"])
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_regress(tA, tb, m=200)
    assert e.value.status == -4
    x, info = gpu_lib.kron_ridge(tA, tb, 0.1, m=200)   # ridge tolerates it
    assert info["status"] == "OK"
    bad = [A.copy() for A in w["As"]]
    bad[1][3, 1] = np.nan
    tA, tb = _torch_inputs(bad, w["b"])
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_regress(tA, tb, m=200)
    assert e.value.status == -1
    tA, tb = _torch_inputs([w["As"][0][:2]], w["b"][:2])  # I < R
    with pytest.raises(gpu_lib.KronRegressError):
        gpu_lib.kron_regress(tA, tb, m=10)


def test_sketch_failure_detected(gpu_lib):
    # one sample of a rank-4 design: the sketch spectrum is about R/m = 4, so the
    # paper's step 1 - sqrt(eps) makes Richardson diverge; the detector reports it
    print("case divergence", flush=True)
    w = workloads.random_problem((8, 8), (2, 2), seed=8)
    tA, tb = _torch_inputs(w["As"], w["b"])
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_regress(tA, tb, m=1)
    assert e.value.status == -5


def test_default_sample_count_is_algorithm_2s(gpu_lib):
    """opts.m = 0 takes Algorithm 2's count ceil(1680 R ln(40 R) ln(1/delta) / eps)
    (the oracle's theory_sample_count, pinned to the paper's printed rows-sampled
    column); the sketch drawn with it is the oracle's, bit for bit."""
    from oracle.regression import theory_sample_count
    w = workloads.random_problem((9, 7), (2, 2), seed=21)
    As, b = w["As"], w["b"]
    tA, tb = _torch_inputs(As, b)
    m = theory_sample_count(4, 0.1, 0.01)
    print("case default sample count m=%d" % m, flush=True)
    x, info = gpu_lib.kron_regress(tA, tb, eps=0.1, delta=0.01, m=0, seed=5, stream=0)
    assert info["m"] == m, (info["m"], m)
    sk = gpu_lib.export_sketch([9, 7])
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=5, stream=0)
    assert counts.sum() == m
    xo = sketched_solution(As, b, rows, ridx, Omega, 0.0)
    assert rel_l2(x.cpu().numpy(), xo) < 1e-10


def test_info_loss_and_time(gpu_lib):
    """KR_OPT_LOSS fills kr_info.loss with f(x) of the returned x (the oracle's loss
    on the same x), for a dense and an implicit response; kr_info.ms is the call's
    wall clock."""
    import torch
    from oracle.response import implicit_response
    print("case info loss", flush=True)
    w = workloads.small_regression()
    tA, tb = _torch_inputs(w["As"], w["b"])
    x, info = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"], compute_loss=True)
    assert abs(info["loss"] - loss(w["As"], w["b"], x.cpu().numpy())) <= 1e-12 * info["loss"]
    assert info["ms"] > 0
    _, info2 = gpu_lib.kron_regress(tA, tb, eps=w["eps"], m=w["m"], seed=w["seed"])
    assert np.isnan(info2["loss"])
    rng = np.random.default_rng(3)
    X = rng.standard_normal((64, 2))
    b = implicit_response(w["As"], X, 0.1, 2, 3)
    gen = gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), 0.1, seed=2, stream=3)
    x, info = gpu_lib.kron_ridge(tA, gen, 0.01, m=3000, compute_loss=True)
    xh = x.cpu().numpy()
    ref = max(loss(w["As"], b[:, q], xh[:, q], 0.01) for q in range(2))
    assert abs(info["loss"] - ref) <= 1e-10 * ref


@pytest.mark.parametrize("case", [("N3", (9, 6, 5), (3, 2, 2), 4097), ("N4", (5, 4, 6, 3), (2, 2, 3, 1), 800),
                                  ("N2 heavy", (40, 33), (4, 5), 20000)], ids=lambda c: c[0])
def test_per_sample_draws_match_oracle(gpu_lib, case):
    """Algorithm 2's draws before merging: every sample t's indices (i_1(t), ..,
    i_N(t)) redrawn from the solve's kept tables equal the oracle sampler's, in
    sample order, bit for bit; a window [first, first + count) equals the same
    rows of the whole draw."""
    import torch
    from oracle.sampling import sample_product
    name, I, R, m = case
    print("case per-sample draws", name, I, R, m, flush=True)
    w = workloads.random_problem(I, R, seed=zlib.crc32(name.encode()) % 1000, heavy=3 if "heavy" in name else 0)
    tA = [torch.tensor(A, dtype=torch.float64, device="cuda") for A in w["As"]]
    tb = torch.tensor(w["b"], dtype=torch.float64, device="cuda")
    _, info = gpu_lib.kron_regress(tA, tb, eps=0.1, m=m, seed=23, stream=4)
    sk = gpu_lib.export_sketch(list(I))
    idx = gpu_lib.export_samples(0, m, len(I))
    oidx, _ = sample_product(sk["Q"], m, 23, 4)
    np.testing.assert_array_equal(idx, np.asarray(oidx, dtype=np.int32))
    f, c = m // 3, min(257, m - m // 3)
    np.testing.assert_array_equal(gpu_lib.export_samples(f, c, len(I)), idx[f:f + c])

