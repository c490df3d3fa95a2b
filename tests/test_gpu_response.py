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


def test_implicit_response_rejected_where_dense_data_is_needed(gpu_lib):
    import torch
    As, rng = _factors((10, 9), (3, 2), 1)
    tA = [torch.tensor(A, device="cuda") for A in As]
    gen = gpu_lib.ResponseGen(torch.tensor(rng.standard_normal(6), device="cuda"), 0.1)
    with pytest.raises(gpu_lib.KronRegressError):
        gpu_lib.kron_loss(tA, gen, torch.zeros(6, dtype=torch.float64, device="cuda"))
