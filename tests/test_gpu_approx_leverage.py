"""GPU parity of Algorithm 2 with approximate leverage scores (its first loop:
spectral approximation A~ by row-norm sampling, Lemma
block_sketch_is_spectral_approx; Johnson-Lindenstrauss scores, Lemma
fast-ls-comp) and of the many-workgroup setup passes that large factors take.

The GPU draws A~ and the projection from the same counter-based definitions as
the oracle, so its approximate scores equal the oracle's up to summation order
(relative 1e-11); the quantised tables then equal the oracle's (boundary
straddles reported), the sketch is bit-exact, and the solution is the oracle's
direct minimiser of that sketch (rel-L2 1e-10).  Large factors (I_n = 2^20, K
with 2^40 rows, implicit response) run both the exact and the approximate route."""

import numpy as np
import pytest

import workloads
from oracle.leverage import approximate_leverage_scores, leverage_scores
from oracle.regression import kron_rows, solve_sketched_direct
from oracle.response import noise
from parity import check_quantised_tables, check_sketch, rel_l2

pytestmark = pytest.mark.gpu


def _solve_and_check(gpu_lib, As, b_src, b_rows, lam, m, eps, seed, stream, approx, k=None, r=None):
    import torch
    I = [A.shape[0] for A in As]
    tA = [torch.tensor(A, device="cuda") for A in As]
    x, info = gpu_lib.kron_ridge(tA, b_src(torch), lam, eps=eps, m=m, seed=seed, stream=stream, tol=1e-13,
                                 max_iter=400, approx_leverage=(k, r) if approx else None)
    assert info["status"] == "OK", info
    lev = gpu_lib.export_leverage(I)
    if approx:
        ref = [approximate_leverage_scores(A, k, r, eps, seed, stream, n)[0] for n, A in enumerate(As)]
        tol = 1e-11
    else:
        ref = [leverage_scores(A) for A in As]
        tol = 1e-13
    for n in range(len(As)):
        d = float(np.max(np.abs(lev[n] - ref[n]) / np.maximum(ref[n], 1e-300)))
        ex = leverage_scores(As[n])
        p, pt = ex / ex.sum(), ref[n] / ref[n].sum()
        print("mode %d I=%d: max rel |l_gpu - l_oracle| %.2e; oracle p~/p in [%.3f, %.3f]" % (
            n, I[n], d, float(np.min(pt / p)), float(np.max(pt / p))), flush=True)
        if approx:
            assert d <= tol
        else:
            assert float(np.max(np.abs(lev[n] - ref[n]))) <= tol
    sk = gpu_lib.export_sketch(I)
    straddles = check_quantised_tables(As, sk["Q"], scores=ref)
    rows, ridx, counts, Omega = check_sketch(As, sk, m, seed=seed, stream=stream)
    assert counts.sum() == m
    xo = solve_sketched_direct(kron_rows(As, ridx), Omega, b_rows(rows, ridx), lam)
    err = rel_l2(x.cpu().numpy(), xo)
    print("straddles %d, D=%d, iters %d, rel-L2 vs direct %.2e" % (straddles, len(rows), info["iters"], err),
          flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_approx_leverage_small(gpu_lib, lam):
    print("case approximate leverage small lam=%g" % lam, flush=True)
    w = workloads.random_problem((300, 200, 40), (4, 3, 2), seed=17, heavy=3)
    As, b = w["As"], w["b"]
    _solve_and_check(gpu_lib, As, lambda torch: torch.tensor(b, device="cuda"), lambda rows, ridx: b[rows],
                     lam, 6000, 0.1, 3, 1, True, k=2000, r=24)


@pytest.mark.parametrize("approx", [False, True], ids=["exact", "approx"])
def test_large_factors(gpu_lib, approx):
    """Two factors of 2^20 x 8 (heavy rows), K of 2^40 x 64: b only at the sampled
    rows (K X_true + 0.01 E by the implicit response)."""
    I = 1 << 20
    print("case large factors I=%d approx=%s" % (I, approx), flush=True)
    rng = np.random.default_rng(23)
    As = []
    for _ in range(2):
        A = rng.standard_normal((I, 8))
        A[rng.choice(I, size=50, replace=False)] *= 30.0
        As.append(A)
    X = rng.standard_normal(64)
    sigma, key = 0.01, (4, 9)

    def gen(torch):
        return gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), sigma, seed=key[0], stream=key[1])

    def b_rows(rows, ridx):
        return kron_rows(As, ridx) @ X + sigma * noise(rows, 1, *key)[:, 0]

    m = workloads.m_rule(64, 0.1)
    _solve_and_check(gpu_lib, As, gen, b_rows, 0.0, m, 0.1, 5, 2, approx, k=4096, r=32)
