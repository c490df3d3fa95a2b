"""GPU parity of the implicit response b = K X_true + sigma E against the oracle.

The GPU forms b only at the sampled rows (sample-tree products of X_true plus
the row-indexed Philox normal); the oracle forms the dense b and solves the same
sketched problem directly."""

import numpy as np
import pytest

import workloads
from oracle.regression import sketch
from oracle.response import implicit_response
from parity import rel_l2, sketched_solution

pytestmark = pytest.mark.gpu

CASES = [((40,), (6,), 2, 0.0), ((30, 20), (5, 4), 3, 0.01), ((12, 10, 9), (3, 4, 3), 1, 0.0),
         ((8, 7, 6, 5), (2, 3, 2, 3), 2, 0.1)]


def _factors(I, R, seed):
    rng = np.random.default_rng(seed)
    As = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    return As, rng


@pytest.mark.parametrize("case", range(len(CASES)))
def test_implicit_response_matches_oracle(gpu_lib, case):
    import torch
    I, R, nrhs, lam = CASES[case]
    As, rng = _factors(I, R, 70 + case)
    X = rng.standard_normal((int(np.prod(R)), nrhs))
    sigma, m = 0.05, 3000
    print("case implicit response", I, R, nrhs, lam, flush=True)
    b = implicit_response(As, X, sigma, seed=7, stream=9 + case)
    tA = [torch.tensor(A, device="cuda") for A in As]
    gen = gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), sigma, seed=7, stream=9 + case)
    x, info = gpu_lib.kron_ridge(tA, gen, lam, m=m, seed=3, stream=case, tol=1e-13, max_iter=400)
    assert info["status"] == "OK", info
    sk = sketch(As, m, 3, case)
    assert info["distinct_rows"] == len(sk["rows"])
    x64 = sketched_solution(As, b, sk["rows"], sk["ridx"], sk["Omega"], lam)
    kappa2u = float(np.prod([np.linalg.cond(A) for A in As])) ** 2 * 2.2e-16
    err = rel_l2(x.cpu().numpy(), x64)
    assert err < max(1e-10, 20 * kappa2u), err
    # the same solve with the dense b agrees to rounding
    xd, _ = gpu_lib.kron_ridge(tA, torch.tensor(b, device="cuda"), lam, m=m, seed=3, stream=case, tol=1e-13,
                               max_iter=400)
    assert rel_l2(x.cpu().numpy(), xd.cpu().numpy()) < 1e-12


def test_implicit_response_in_a_batch(gpu_lib):
    import torch
    problems, lams, dense = [], [], []
    for i in range(6):
        N = 2 + i % 3
        I = tuple(12 + 3 * i + n for n in range(N))
        R = tuple(2 + (i + n) % 3 for n in range(N))
        As, rng = _factors(I, R, 300 + i)
        nrhs = 1 + i % 2
        X = rng.standard_normal((int(np.prod(R)), nrhs))
        tA = [torch.tensor(A, device="cuda") for A in As]
        problems.append((tA, gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), 0.02, seed=5, stream=i)))
        lams.append(0.01 * (i + 1))
        dense.append((As, implicit_response(As, X, 0.02, 5, i)))
    print("case implicit response batch", flush=True)
    m = 2500
    xs, infos = gpu_lib.kron_ridge_batched(problems, lams, m=m, seed=8, stream=40, tol=1e-12, max_iter=400)
    for i, ((As, b), x, info) in enumerate(zip(dense, xs, infos)):
        assert info["status"] == "OK", (i, info)
        sk = sketch(As, m, 8, 40 + i)
        x64 = sketched_solution(As, b, sk["rows"], sk["ridx"], sk["Omega"], lams[i])
        assert rel_l2(x.cpu().numpy(), x64) < 1e-10


def test_loss_opt_needs_an_implicit_response(gpu_lib):
    """kron_loss_opt is the implicit response's one-pass gate; with a dense b it
    refuses (kron_exact and kron_loss serve that case)."""
    import torch
    print("case loss_opt argument check", flush=True)
    As, rng = _factors((10, 9), (3, 2), 1)
    tA = [torch.tensor(A, device="cuda") for A in As]
    b = torch.tensor(rng.standard_normal(90), device="cuda")
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_loss_opt(tA, b, torch.zeros(6, dtype=torch.float64, device="cuda"))
    assert e.value.status == -1


LOSS_CASES = [((40,), (6,), 1, 0.0), ((30, 20), (5, 4), 3, 0.01), ((12, 10, 9), (3, 4, 3), 2, 0.0),
              ((8, 7, 6, 5), (2, 3, 2, 3), 1, 0.2), ((9, 300, 7), (2, 5, 3), 2, 0.05)]


@pytest.mark.parametrize("case", range(len(LOSS_CASES)))
def test_implicit_loss_and_exact(gpu_lib, case):
    """kron_loss and kron_exact with an implicit response (one pass over the
    generated noise for K^T E and ||E||^2, closed forms in R-space) against the
    oracle's loss and exact minimiser on the dense b; the loss also at a random x
    and at the exact minimiser (OPT)."""
    import torch
    from oracle.regression import exact_solution, loss
    I, R, nrhs, lam = LOSS_CASES[case]
    As, rng = _factors(I, R, 90 + case)
    Rt = int(np.prod(R))
    X = rng.standard_normal((Rt, nrhs))
    sigma = 0.3
    print("case implicit loss/exact", I, R, nrhs, lam, flush=True)
    b = implicit_response(As, X, sigma, seed=5, stream=40 + case)
    tA = [torch.tensor(A, device="cuda") for A in As]
    gen = gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), sigma, seed=5, stream=40 + case)
    xo = exact_solution(As, b, lam)
    xg = gpu_lib.kron_exact(tA, gen, lam).cpu().numpy()
    print("exact rel-L2 %.2e" % rel_l2(xg, xo), flush=True)
    assert rel_l2(xg, xo) < 1e-10
    for xt in (xo, X + 0.1 * rng.standard_normal(X.shape)):
        fg = gpu_lib.kron_loss(tA, gen, torch.tensor(np.ascontiguousarray(xt), device="cuda"), lam)
        for q in range(nrhs):
            fo = loss(As, b[:, q], xt[:, q], lam)
            print("q %d loss gpu %.12e oracle %.12e" % (q, fg[q], fo), flush=True)
            assert abs(fg[q] - fo) <= 1e-10 * fo
    # the gate in one pass: f(x) and OPT = f(x*)
    xt = X + 0.05 * rng.standard_normal(X.shape)
    f, opt = gpu_lib.kron_loss_opt(tA, gen, torch.tensor(np.ascontiguousarray(xt), device="cuda"), lam)
    for q in range(nrhs):
        fo, oo = loss(As, b[:, q], xt[:, q], lam), loss(As, b[:, q], xo[:, q], lam)
        assert abs(f[q] - fo) <= 1e-10 * fo and abs(opt[q] - oo) <= 1e-10 * oo, (f, opt, fo, oo)
