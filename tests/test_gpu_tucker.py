"""GPU parity of Algorithm 3 (tucker_factor_update) against the oracle.

Per row: the sketch (Philox counter word 2 = row) must match the oracle's draw bit
for bit; the updated factor row must match the oracle's direct solution of the
penalised sketched row problem.  At the 400^3 tensor workload a sample of rows is
checked the same way, and every row's objective against the exact row optimum."""

import numpy as np
import pytest

import workloads
from oracle.kron import kron_explicit, tucker_reconstruct, unfold
from oracle.regression import kron_rows
from oracle.tucker import FactorUpdateSetup, exact_factor_update
from parity import rel_l2

pytestmark = pytest.mark.gpu


def _tensor_case(I, R, seed, noise=0.05):
    rng = np.random.default_rng(seed)
    As = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    G = rng.standard_normal(R)
    X = tucker_reconstruct(G, As) + noise * rng.standard_normal(I)
    return X, As, G


def _gpu(X, As, G, dtype=None):
    import torch
    dt = dtype or torch.float64
    return (torch.tensor(X, dtype=dt, device="cuda").contiguous(),
            [torch.tensor(A, device="cuda") for A in As],
            torch.tensor(G, device="cuda").contiguous())


def _check_rows(kr, X, As, G, n, lam, m, seed, stream, A_gpu, rows, xtol):
    S = FactorUpdateSetup(As, G, n, lam, 0.1)
    B = unfold(X, n)
    I = list(X.shape)
    sizes = [I[n]] + [I[k] for k in range(len(I)) if k != n]
    sk = kr.export_sketch(sizes)
    for k in range(1, len(sizes)):
        np.testing.assert_array_equal(sk["Q"][k], S.Q[k - 1])
    grows = sk["rows"]
    worst = 0.0
    for i in rows:
        osk = S.row_sketch(m, seed, stream, i)
        sel = grows[:, 0] == i
        np.testing.assert_array_equal(grows[sel, 1:], osk["ridx"])
        np.testing.assert_array_equal(sk["counts"][sel], osk["counts"])
        np.testing.assert_allclose(sk["Omega"][sel], osk["Omega"], rtol=2e-16, atol=0)
        KD = kron_rows(S.As_other, osk["ridx"])
        z = S.row_direct(KD, osk["Omega"], B[i, osk["rows"]])
        worst = max(worst, rel_l2(A_gpu[i], S.GtP @ z))
    assert worst < xtol, worst
    return worst


@pytest.mark.parametrize("n", [0, 1, 2])
def test_factor_update_small(gpu_lib, n):
    print("case tucker small mode", n, flush=True)
    X, As, G = _tensor_case((20, 18, 16), (3, 3, 2), seed=11 + n)
    tX, tA, tG = _gpu(X, As, G)
    lam, m = 0.05, 300
    A_new, info = gpu_lib.tucker_factor_update(tX, tA, tG, n, lam, eps=0.1, m=m, seed=0, stream=5, tol=1e-13)
    assert info["status"] == "OK", info
    worst = _check_rows(gpu_lib, X, As, G, n, lam, m, 0, 5, A_new.cpu().numpy(), range(X.shape[n]), 1e-10)
    print("worst row rel-L2 %.2e, iterations %d" % (worst, info["iters"]), flush=True)


def test_factor_update_four_modes_f32(gpu_lib):
    import torch
    print("case tucker N=4 float32 tensor", flush=True)
    X, As, G = _tensor_case((9, 8, 7, 6), (2, 3, 2, 2), seed=21)
    X = X.astype(np.float32).astype(np.float64)
    tX, tA, tG = _gpu(X, As, G, torch.float32)
    tA = [torch.tensor(A, device="cuda") for A in As]
    A_new, info = gpu_lib.tucker_factor_update(tX, tA, tG, 2, 0.1, m=250, seed=3, stream=1, tol=1e-13)
    assert info["status"] == "OK", info
    _check_rows(gpu_lib, X, As, G, 2, 0.1, 250, 3, 1, A_new.cpu().numpy(), range(7), 1e-10)


def test_factor_update_singular_core(gpu_lib):
    print("case tucker singular core", flush=True)
    X, As, G = _tensor_case((10, 9, 8), (3, 2, 2), seed=31)
    G[1] = G[0]                   # two equal mode-0 slices: G_(0) G_(0)^T is singular
    tX, tA, tG = _gpu(X, As, G)
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.tucker_factor_update(tX, tA, tG, 0, 0.1, m=100)
    assert e.value.status == -4


def test_factor_update_tucker_tensor_workload(gpu_lib):
    """The 400^3 FP32 tensor, rank (16,16,16), lam = 1e-3, m = 14,196 per row."""
    import torch
    w = workloads.tucker_tensor()
    print("case", w["name"], "m_factor", w["m_factor"], flush=True)
    X = w["X"]
    As = [A.copy() for A in w["A_init"]]
    G = w["G_init"]
    tX = torch.from_numpy(X).cuda()
    tA = [torch.tensor(A, device="cuda") for A in As]
    tG = torch.tensor(G, device="cuda")
    n = 0
    A_new, info = gpu_lib.tucker_factor_update(tX, tA, tG, n, w["lam"], eps=w["eps"], m=w["m_factor"],
                                               seed=w["seed"], stream=7, tol=1e-12)
    assert info["status"] == "OK", info
    Xd = X.astype(np.float64)
    An = A_new.cpu().numpy()
    _check_rows(gpu_lib, Xd, As, G, n, w["lam"], w["m_factor"], w["seed"], 7, An, [0, 1, 199, 398, 399], 1e-9)
    # every row within (1 + eps) of its exact optimum
    exact = exact_factor_update(Xd, As, G, n, w["lam"])
    S = FactorUpdateSetup(As, G, n, w["lam"], w["eps"])
    D = np.kron(S.As_other[0], S.As_other[1]) @ S.Gn.T
    B = unfold(Xd, n)
    f = lambda y, i: np.sum((D @ y - B[i]) ** 2) + w["lam"] * y @ y
    ratios = np.array([f(An[i], i) / f(exact[i], i) for i in range(X.shape[0])])
    print("row objective ratio: max %.4f median %.5f" % (ratios.max(), np.median(ratios)), flush=True)
    assert ratios.max() <= 1 + w["eps"]


def test_core_update_tucker_workload(gpu_lib):
    """Core update of ALS (Algorithm 2 with b = vec(X), FP32 X, lam = 1e-3) on the
    400^3 tensor: bit-exact sketch, sketched normal equations satisfied, loss gate."""
    import torch
    from oracle.regression import exact_solution, loss
    from parity import check_quantised_tables, check_sketch
    w = workloads.tucker_tensor()
    print("case core update", w["name"], "m", w["m_core"], flush=True)
    As = w["A_init"]
    X = w["X"]
    tX = torch.from_numpy(X).cuda().reshape(-1)
    tA = [torch.tensor(A, device="cuda") for A in As]
    g, info = gpu_lib.kron_ridge(tA, tX, w["lam"], eps=w["eps"], m=w["m_core"], seed=w["seed"], stream=3,
                                 tol=1e-12)
    assert info["status"] == "OK", info
    sk = gpu_lib.export_sketch([400, 400, 400])
    check_quantised_tables(As, sk["Q"])
    rows, ridx, counts, Omega = check_sketch(As, sk, w["m_core"], seed=w["seed"], stream=3)
    gv = g.cpu().numpy()
    bD = X.reshape(-1)[rows].astype(np.float64)
    # sketched normal equations K_D^T Omega (K_D g - b_D) + lam g = 0, in row chunks
    res = w["lam"] * gv
    ref = np.zeros_like(gv)
    for c0 in range(0, len(rows), 20000):
        KD = kron_rows(As, ridx[c0:c0 + 20000])
        r = KD @ gv - bD[c0:c0 + 20000]
        res += KD.T @ (Omega[c0:c0 + 20000] * r)
        ref += KD.T @ (Omega[c0:c0 + 20000] * bD[c0:c0 + 20000])
    rel = np.linalg.norm(res) / np.linalg.norm(ref)
    print("normal-equation residual %.2e, distinct rows %d" % (rel, len(rows)), flush=True)
    assert rel < 1e-10
    Xd = X.astype(np.float64).reshape(-1)
    f = loss(As, Xd, gv, w["lam"])
    opt = loss(As, Xd, exact_solution(As, Xd, w["lam"]), w["lam"])
    print("loss / opt = %.5f" % (f / opt), flush=True)
    assert f <= (1 + w["eps"]) * opt


def test_als_matches_oracle_small(gpu_lib):
    """Two sketched ALS sweeps through the C ABI against the oracle's sketched ALS
    (same Philox streams; the oracle solves each sketched problem directly)."""
    import torch
    from oracle.tucker import tucker_als
    print("case ALS small", flush=True)
    rng = np.random.default_rng(41)
    I, R = (24, 20, 18), (3, 3, 2)
    Qs = [np.linalg.qr(rng.standard_normal((i, r)))[0] for i, r in zip(I, R)]
    X = tucker_reconstruct(rng.standard_normal(R), Qs) + 0.01 * rng.standard_normal(I)
    G0 = rng.standard_normal(R)
    A0 = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    lam, eps, mc, mf = 1e-3, 0.1, 3000, 400
    Go, Ao, to = tucker_als(X, G0, A0, lam, 2, sketched=True, eps=eps, m_factor=mf, m_core=mc, seed=0)
    Gg, Ag, tg = gpu_lib.tucker_als(torch.tensor(X, device="cuda"), torch.tensor(G0, device="cuda"),
                                    [torch.tensor(A, device="cuda") for A in A0], lam, 2, eps=eps,
                                    m_core=mc, m_factor=mf, seed=0)
    print("rre oracle", to, "gpu", tg, flush=True)
    np.testing.assert_allclose(tg, to, rtol=1e-7)
    assert rel_l2(Gg.cpu().numpy(), Go) < 1e-7
    for a, b in zip(Ag, Ao):
        assert rel_l2(a.cpu().numpy(), b) < 1e-7


def test_als_native_loop_matches_python_loop(gpu_lib):
    """kr_tucker_als (Algorithm 1 looped inside the library) against tucker_als's
    Python loop over the same C-ABI updates, on the small tensor: the same
    updates, streams and order, so the factors, core, errors and iteration counts
    are identical bit for bit; and both against the oracle's sketched ALS."""
    import torch
    from oracle.tucker import tucker_als
    print("case ALS native loop", flush=True)
    rng = np.random.default_rng(41)
    I, R = (24, 20, 18), (3, 3, 2)
    Qs = [np.linalg.qr(rng.standard_normal((i, r)))[0] for i, r in zip(I, R)]
    X = tucker_reconstruct(rng.standard_normal(R), Qs) + 0.01 * rng.standard_normal(I)
    G0 = rng.standard_normal(R)
    A0 = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    lam, eps, mc, mf = 1e-3, 0.1, 3000, 400
    tX = torch.tensor(X, device="cuda")
    tG = torch.tensor(G0, device="cuda")
    tA = [torch.tensor(A, device="cuda") for A in A0]
    stats = []
    Gp, Ap, tp = gpu_lib.tucker_als(tX, tG, tA, lam, 2, eps=eps, m_core=mc, m_factor=mf, seed=0, stats=stats)
    Gn, An, tn, iters = gpu_lib.tucker_als_native(tX, tG, tA, lam, 2, eps=eps, m_core=mc, m_factor=mf, seed=0)
    print("rre python", tp, "native", tn, "iters", iters, flush=True)
    assert tn == tp
    assert iters == [st["iters"] for st in stats]
    assert torch.equal(Gn, Gp)
    for a, b in zip(An, Ap):
        assert torch.equal(a, b)
    Go, Ao, to = tucker_als(X, G0, A0, lam, 2, sketched=True, eps=eps, m_factor=mf, m_core=mc, seed=0)
    np.testing.assert_allclose(tn, to, rtol=1e-7)
    assert rel_l2(Gn.cpu().numpy(), Go) < 1e-7


def test_als_native_loop_reports_a_failed_update(gpu_lib):
    """Updates held to one Richardson iteration end in WMAXITER: the native loop
    stops at the first one (sweep 0, the factor update of mode 0) and names it."""
    import torch
    from paper_2209_04876_amd import KronRegressError
    print("case ALS native loop failure", flush=True)
    rng = np.random.default_rng(5)
    I, R = (12, 10, 9), (2, 2, 2)
    X = torch.tensor(rng.standard_normal(I), device="cuda")
    G0 = torch.tensor(rng.standard_normal(R), device="cuda")
    A0 = [torch.tensor(rng.standard_normal((i, r)), device="cuda") for i, r in zip(I, R)]
    with pytest.raises(KronRegressError, match="update 0 "):
        gpu_lib.tucker_als_native(X, G0, A0, 1e-3, 1, m_core=500, m_factor=200, max_iter=1)


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_als_refined_core_small(gpu_lib, prec):
    """Two sketched ALS sweeps with the core update in a refined precision (float64
    residual and update around a bf16 or float32 preconditioner) against the
    oracle's sketched ALS.  The float32 adjoint of the refined precisions puts a
    floor of about 3e-7 under the core solve's relative step here (the first
    sweep's fit is poor, so the adjoint's terms cancel heavily), so the core stops
    at 1e-6 (the refined default) and the trajectory agrees to that tolerance's
    effect."""
    import torch
    from oracle.tucker import tucker_als
    print("case ALS small, core", prec, flush=True)
    rng = np.random.default_rng(41)
    I, R = (24, 20, 18), (3, 3, 2)
    Qs = [np.linalg.qr(rng.standard_normal((i, r)))[0] for i, r in zip(I, R)]
    X = tucker_reconstruct(rng.standard_normal(R), Qs) + 0.01 * rng.standard_normal(I)
    G0 = rng.standard_normal(R)
    A0 = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    lam, eps, mc, mf = 1e-3, 0.1, 3000, 400
    Go, Ao, to = tucker_als(X, G0, A0, lam, 2, sketched=True, eps=eps, m_factor=mf, m_core=mc, seed=0)
    stats = []
    Gg, Ag, tg = gpu_lib.tucker_als(torch.tensor(X, device="cuda"), torch.tensor(G0, device="cuda"),
                                    [torch.tensor(A, device="cuda") for A in A0], lam, 2, eps=eps,
                                    m_core=mc, m_factor=mf, seed=0, core_precision=prec, stats=stats)
    print("rre oracle", to, "gpu", tg, "core iterations", [s["iters"] for s in stats if s["step"] == 3], flush=True)
    np.testing.assert_allclose(tg, to, rtol=1e-5)
    assert rel_l2(Gg.cpu().numpy(), Go) < 2e-5
    for a, b in zip(Ag, Ao):
        assert rel_l2(a.cpu().numpy(), b) < 2e-5


def test_exact_als_400_trajectory(gpu_lib):
    """Exact ALS (exact factor and core updates, lambda = 1e-3) on the 400^3 tensor
    the benchmark decomposes: the relative reconstruction error after each of 10
    sweeps against the oracle's trajectory (tests/golden/tucker_400_als.txt,
    written by make_tucker_400_als.py from the oracle only)."""
    import os

    import torch
    print("case exact ALS 400^3", flush=True)
    ref = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "tucker_400_als.txt")):
        if line.strip() and not line.startswith("#"):
            ref.append(float(line.split()[1]))
    w = workloads.tucker_tensor()
    X = torch.from_numpy(w["X"]).cuda()
    del w["X"]
    G0 = torch.tensor(w["G_init"], device="cuda")
    A0 = [torch.tensor(A, device="cuda") for A in w["A_init"]]
    _, _, trace = gpu_lib.tucker_als(X, G0, A0, w["lam"], len(ref), factor_update="exact", core_update="exact")
    print("rre", ["%.6g" % v for v in trace], "oracle", ["%.6g" % v for v in ref], flush=True)
    for a, b in zip(trace, ref):
        assert abs(a - b) <= 1e-8 * b, (trace, ref)
