"""GPU parity of kron_ridge_batched (many uneven problems; their iterations in
a queue kernel and a team kernel, both persistent) against the oracle.

Problem i of a batch draws its sample with Philox stream `stream + i`; the
oracle sketches each problem from its own leverage tables with the same key and
solves the merged sketched problem directly in float64.  The batched solution
must match that minimiser to the same tolerance as a single solve, and the
distinct-row count must equal the oracle's."""

import numpy as np
import pytest

import workloads
from oracle.regression import sketch
from parity import rel_l2, sketched_solution

pytestmark = pytest.mark.gpu


def _batch(count, seed, lam_zero_every=4):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.integers(1, 5))
        I = tuple(int(v) for v in rng.integers(5, 13, size=N))
        R = tuple(int(min(v, i_)) for v, i_ in zip(rng.integers(2, 6, size=N), I))
        nrhs = int(rng.integers(1, 4))
        lam = 0.0 if i % lam_zero_every == 0 else float(10 ** rng.uniform(-4, 0))
        w = workloads.random_problem(I, R, seed=seed * 1000 + i, nrhs=nrhs, sigma=0.05)
        m = int(min(4 * int(np.prod(R)) + 50, 3000))
        out.append((w["As"], w["b"], lam, m))
    return out


def _gpu(problems):
    import torch
    res = []
    for As, b, lam, m in problems:
        tA = [torch.tensor(A, device="cuda") for A in As]
        tb = torch.tensor(b, device="cuda").contiguous()
        res.append((tA, tb))
    return res


def _check(problem, x, info, seed, stream):
    As, b, lam, m = problem
    sk = sketch(As, m, seed, stream)
    assert info["distinct_rows"] == len(sk["rows"]), (info, len(sk["rows"]))
    x64 = sketched_solution(As, b, sk["rows"], sk["ridx"], sk["Omega"], lam)
    kappa2u = float(np.prod([np.linalg.cond(A) for A in As])) ** 2 * 2.2e-16
    xtol = max(1e-10, 20 * kappa2u)
    err = rel_l2(x.cpu().numpy(), x64)
    assert err < xtol, (err, xtol, [A.shape for A in As], lam)
    return err


def test_batched_matches_oracle(gpu_lib):
    """Sixteen uneven problems (N = 1..4, R_n 2..5, 1-3 right-hand sides, ridge and
    lambda = 0) with a fixed m each."""
    probs = _batch(16, seed=3)
    print("case batched 16 problems", [(len(p[0]), p[1].ndim, p[2]) for p in probs], flush=True)
    # fixed m per problem: run each problem's m through the batch one m at a time
    # is not possible (one opts per call), so the batch uses the largest m and the
    # oracle sketches with that same m
    m = max(p[3] for p in probs)
    probs = [(As, b, lam, m) for As, b, lam, _ in probs]
    g = _gpu(probs)
    xs, infos = gpu_lib.kron_ridge_batched([(tA, tb) for tA, tb in g], [p[2] for p in probs], eps=0.1, m=m, seed=5,
                                           stream=100, tol=1e-12, max_iter=400)
    worst = 0.0
    for i, (p, x, info) in enumerate(zip(probs, xs, infos)):
        assert info["status"] == "OK", (i, info)
        worst = max(worst, _check(p, x, info, 5, 100 + i))
    print("worst rel-L2 %.2e, iterations %s" % (worst, [inf["iters"] for inf in infos]), flush=True)


def test_batched_rlnr_rule_and_larger_problems(gpu_lib):
    """m = ceil(R ln R / eps) per problem; N = 2..4 with R up to 512."""
    import torch
    rng = np.random.default_rng(9)
    probs = []
    for i in range(6):
        N = 2 + i % 3
        I = tuple(int(v) for v in rng.integers(12, 30, size=N))
        hi = {2: 17, 3: 9, 4: 5}[N]
        R = tuple(int(min(v, i_)) for v, i_ in zip(rng.integers(3, hi, size=N), I))
        w = workloads.random_problem(I, R, seed=90 + i, nrhs=1 + i % 3, sigma=0.05)
        lam = float(10 ** rng.uniform(-4, 0))
        Rt = int(np.prod(R))
        m = max(1, int(np.ceil(Rt * np.log(Rt) / 0.1)))
        probs.append((w["As"], w["b"], lam, m))
    print("case batched R ln R", [int(np.prod([A.shape[1] for A in p[0]])) for p in probs], flush=True)
    g = _gpu(probs)
    xs, infos = gpu_lib.kron_ridge_batched([(tA, tb) for tA, tb in g], [p[2] for p in probs], eps=0.1,
                                           m_rule="rlnr", seed=1, stream=7, tol=1e-12, max_iter=400)
    torch.cuda.synchronize()
    print("gpu done", [inf["iters"] for inf in infos], flush=True)
    for i, (p, x, info) in enumerate(zip(probs, xs, infos)):
        assert info["m"] == p[3]
        assert info["status"] == "OK", (i, info)
        _check(p, x, info, 1, 7 + i)


def test_batched_mixes_large_and_small_problems(gpu_lib):
    """A problem with many sampled rows is iterated by the team, the small ones
    by the queue kernel; the large one alone through the single-problem entry
    point reaches the same minimiser."""
    import torch
    big = workloads.random_problem((300, 300), (8, 8), seed=41, nrhs=2, sigma=0.05)
    probs = [(big["As"], big["b"], 0.05, 0)]
    for i in range(5):
        w = workloads.random_problem((12 + i, 9, 7), (3, 4, 2), seed=50 + i, nrhs=1 + i % 2, sigma=0.05)
        probs.append((w["As"], w["b"], 0.0 if i == 2 else 0.01 * (i + 1), 0))
    m = 200000
    probs = [(As, b, lam, m) for As, b, lam, _ in probs]
    print("case batched big+small", flush=True)
    g = _gpu(probs)
    xs, infos = gpu_lib.kron_ridge_batched([(tA, tb) for tA, tb in g], [p[2] for p in probs], m=m, seed=4,
                                           stream=20, tol=1e-12, max_iter=400)
    torch.cuda.synchronize()
    print("gpu done", [inf["iters"] for inf in infos], flush=True)
    for i, (p, x, info) in enumerate(zip(probs, xs, infos)):
        assert info["status"] == "OK", (i, info)
        _check(p, x, info, 4, 20 + i)
    # the large problem alone, through the single-problem entry point, gives the
    # same minimiser (the two paths sum in different orders)
    x1, info1 = gpu_lib.kron_ridge(g[0][0], g[0][1], 0.05, m=m, seed=4, stream=20, tol=1e-12, max_iter=400)
    assert rel_l2(xs[0].cpu().numpy(), x1.cpu().numpy()) < 1e-11


def test_batched_team_problems_of_every_order(gpu_lib):
    """Large problems (iterated together by the launch's team of workgroups) with
    N = 2, 3, 4, lambda = 0 and lambda > 0, several right-hand sides, one with an
    implicit response; small ones on the queue beside them."""
    import torch
    from oracle.response import implicit_response
    specs = [((400, 300), (8, 6), 2, 0.0), ((60, 50, 40), (3, 4, 3), 2, 0.02), ((20, 18, 16, 15), (2, 3, 3, 2), 2, 0.0),
             ((60, 50, 40), (4, 3, 2), 3, 0.0), ((20, 18, 16, 15), (3, 2, 2, 3), 2, 0.3), ((9, 8), (3, 2), 1, 0.01)]
    m = 150000
    problems, dense, lams = [], [], []
    for i, (I, R, nrhs, lam) in enumerate(specs):
        rng = np.random.default_rng(600 + i)
        As = [rng.standard_normal((a, r)) for a, r in zip(I, R)]
        X = rng.standard_normal((int(np.prod(R)), nrhs))
        tA = [torch.tensor(A, device="cuda") for A in As]
        b = implicit_response(As, X, 0.05, 3, i)
        if i == 4:
            problems.append((tA, gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), 0.05, seed=3, stream=i)))
        else:
            problems.append((tA, torch.tensor(b, device="cuda")))
        dense.append((As, b))
        lams.append(lam)
    print("case batched team", [p[0] for p in specs], flush=True)
    xs, infos = gpu_lib.kron_ridge_batched(problems, lams, m=m, seed=6, stream=50, tol=1e-12, max_iter=600)
    torch.cuda.synchronize()
    print("gpu done", [inf["iters"] for inf in infos], flush=True)
    for i, ((As, b), x, info) in enumerate(zip(dense, xs, infos)):
        assert info["status"] == "OK", (i, info)
        sk = sketch(As, m, 6, 50 + i)
        assert info["distinct_rows"] == len(sk["rows"])
        x64 = sketched_solution(As, b, sk["rows"], sk["ridx"], sk["Omega"], lams[i])
        kappa2u = float(np.prod([np.linalg.cond(A) for A in As])) ** 2 * 2.2e-16
        err = rel_l2(x.cpu().numpy(), x64)
        print("problem", i, "rel-L2 %.2e" % err, flush=True)
        assert err < max(1e-10, 20 * kappa2u), (i, err)


def test_batched_isolates_a_failing_problem(gpu_lib):
    """A singular lambda = 0 problem fails with ESINGULAR; the others still solve."""
    probs = _batch(5, seed=11, lam_zero_every=100)
    As, b, lam, m = probs[2]
    As = [A.copy() for A in As]
    if As[0].shape[1] < 2:
        As[0] = np.hstack([As[0], As[0]])
    As[0][:, 1] = As[0][:, 0]
    Rt = int(np.prod([A.shape[1] for A in As]))
    b = np.random.default_rng(0).standard_normal(int(np.prod([A.shape[0] for A in As])))
    probs[2] = (As, b, 0.0, m)
    m = max(p[3] for p in probs)
    probs = [(A_, b_, l_, m) for A_, b_, l_, _ in probs]
    print("case batched failing problem", Rt, flush=True)
    g = _gpu(probs)
    xs, infos, st = gpu_lib.kron_ridge_batched([(tA, tb) for tA, tb in g], [p[2] for p in probs], m=m, seed=2,
                                               stream=0, raise_on_error=False)
    assert st == -4
    assert infos[2]["status"] == "ESINGULAR"
    for i in (0, 1, 3, 4):
        assert infos[i]["status"] == "OK", (i, infos[i])
        _check(probs[i], xs[i], infos[i], 2, i)


def test_batched_rejects_wide_modes_and_low_precision(gpu_lib):
    import torch
    w = workloads.random_problem((30, 20), (17, 3), seed=1)
    tA = [torch.tensor(A, device="cuda") for A in w["As"]]
    tb = torch.tensor(w["b"], device="cuda")
    print("case batched limits", flush=True)
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_ridge_batched([(tA, tb)], [0.1], m=100)
    assert e.value.status == -6
    assert gpu_lib.kron_ridge_batched([], [], m=100) == ([], [])


def _mixed_batch(gpu_lib, seed):
    import torch
    specs = [((60, 50, 40), (3, 4, 3), 2, 0.02), ((400, 300), (8, 6), 2, 0.1), ((9, 8), (3, 2), 1, 0.01),
             ((20, 18, 16, 15), (2, 3, 3, 2), 2, 0.05), ((12, 10, 9), (3, 2, 3), 3, 0.2)]
    probs, lams, dense = [], [], []
    for i, (I, R, nrhs, lam) in enumerate(specs):
        w = workloads.random_problem(I, R, seed=seed + i, nrhs=nrhs, sigma=0.05)
        probs.append(([torch.tensor(A, device="cuda") for A in w["As"]], torch.tensor(w["b"], device="cuda")))
        lams.append(lam)
        dense.append(w)
    return probs, lams, dense


def test_batched_graph_replays_match_eager(gpu_lib):
    """KR_OPT_GRAPH: the first call captures, later calls with the same buffers
    replay; every replay (with eager work and synchronisations between them, and
    new response values in the same buffers) equals the eager solve."""
    import torch
    probs, lams, _ = _mixed_batch(gpu_lib, 800)
    stream = torch.cuda.Stream()
    h = gpu_lib.Handle(stream=stream)
    he = gpu_lib.Handle(stream=stream)
    print("case batched graph", flush=True)
    kw = dict(m=60000, seed=3, stream=5, tol=1e-12, max_iter=400)
    with torch.cuda.stream(stream):
        xs = None
        for rep in range(4):
            if rep == 2:   # new data in the same buffers: the replay must see it
                for _, b in probs:
                    b.mul_(1.5).add_(0.25)
            xs, infos = gpu_lib.kron_ridge_batched(probs, lams, handle=h, graph=True, xs=xs, **kw)
            stream.synchronize()
            xe, _ = gpu_lib.kron_ridge_batched(probs, lams, handle=he, **kw)
            stream.synchronize()
            _ = torch.randn(1000, device="cuda").sum().item()   # unrelated eager work between replays
            for i, (a, b) in enumerate(zip(xs, xe)):
                assert infos[i]["status"] == "OK", (rep, i, infos[i])
                assert torch.equal(a, b), (rep, i, rel_l2(a.cpu().numpy(), b.cpu().numpy()))
    h.close()
    he.close()


def test_batched_autotune_keeps_results(gpu_lib):
    """KR_OPT_AUTOTUNE times the candidate configurations and returns the
    minimiser of every problem (checked against the oracle)."""
    import torch
    probs, lams, dense = _mixed_batch(gpu_lib, 900)
    h = gpu_lib.Handle()
    m = 60000
    print("case batched autotune", flush=True)
    xs, infos = gpu_lib.kron_ridge_batched(probs, lams, m=m, seed=4, stream=9, tol=1e-12, max_iter=400, handle=h,
                                           autotune=True)
    br, wg = gpu_lib.batched_config(handle=h)
    print("chosen", br, wg, flush=True)
    assert br in (2048.0, 8192.0, 32768.0) and wg in (0, 1)
    for i, (w, x, info) in enumerate(zip(dense, xs, infos)):
        assert info["status"] == "OK", (i, info)
        sk = sketch(w["As"], m, 4, 9 + i)
        x64 = sketched_solution(w["As"], w["b"], sk["rows"], sk["ridx"], sk["Omega"], lams[i])
        assert rel_l2(x.cpu().numpy(), x64) < 1e-10, i
    h.close()


def test_batched_edge_routes_and_statuses(gpu_lib):
    """A large single-factor problem (single-problem path), a singular lambda = 0
    problem large enough for the team (ESINGULAR, isolated), and the iteration
    limit (WMAXITER for every problem, positive return status)."""
    import torch
    rng = np.random.default_rng(77)
    A1 = rng.standard_normal((200000, 8))
    b1 = A1 @ rng.standard_normal(8) + 0.01 * rng.standard_normal(200000)
    w2 = workloads.random_problem((60, 50, 40), (3, 4, 3), seed=78, nrhs=2, sigma=0.05)
    As3 = [A.copy() for A in w2["As"]]
    As3[1][:, 1] = As3[1][:, 0]   # rank-deficient factor
    w4 = workloads.random_problem((30, 20), (4, 3), seed=79, sigma=0.05)
    probs = [([torch.tensor(A1, device="cuda")], torch.tensor(b1, device="cuda")),
             ([torch.tensor(A, device="cuda") for A in w2["As"]], torch.tensor(w2["b"], device="cuda")),
             ([torch.tensor(A, device="cuda") for A in As3], torch.tensor(w2["b"], device="cuda")),
             ([torch.tensor(A, device="cuda") for A in w4["As"]], torch.tensor(w4["b"], device="cuda"))]
    lams = [0.01, 0.02, 0.0, 0.1]
    m = 150000
    print("case batched edge routes", flush=True)
    xs, infos, st = gpu_lib.kron_ridge_batched(probs, lams, m=m, seed=3, stream=30, tol=1e-12, max_iter=400,
                                               raise_on_error=False)
    assert st == -4, (st, infos)
    assert infos[2]["status"] == "ESINGULAR"
    dense = [([A1], b1), (w2["As"], w2["b"]), None, (w4["As"], w4["b"])]
    for i in (0, 1, 3):
        assert infos[i]["status"] == "OK", (i, infos[i])
        As, b = dense[i]
        sk = sketch(As, m, 3, 30 + i)
        assert infos[i]["distinct_rows"] == len(sk["rows"])
        x64 = sketched_solution(As, b, sk["rows"], sk["ridx"], sk["Omega"], lams[i])
        assert rel_l2(xs[i].cpu().numpy(), x64) < 1e-10, i
    # the iteration limit: every problem stops after two iterations
    keep = [probs[1], probs[3]]
    xs2, infos2, st2 = gpu_lib.kron_ridge_batched(keep, [0.02, 0.1], m=m, seed=3, stream=30, tol=1e-14, max_iter=2,
                                                  raise_on_error=False)
    assert st2 == 1, st2
    assert [inf["status"] for inf in infos2] == ["WMAXITER", "WMAXITER"]
    assert [inf["iters"] for inf in infos2] == [2, 2]
