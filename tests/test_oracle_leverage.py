"""Pins leverage scores and the quantised distribution (Section 3; Lemma
kronecker_cross_leverage_scores)."""

import itertools

import numpy as np
import pytest

from oracle.kron import kron_explicit
from oracle.leverage import GRID, cdf, leverage_scores, quantize, ridge_leverage_scores


def _brute(A, lam):
    # definition: l_i = a_i (A^T A + lam I)^+ a_i^T
    P = np.linalg.pinv(A.T @ A + lam * np.eye(A.shape[1]))
    return np.einsum("ij,jk,ik->i", A, P, A)


@pytest.mark.parametrize("lam", [0.0, 0.3, 5.0])
def test_leverage_matches_definition(lam):
    A = np.random.default_rng(0).standard_normal((20, 4))
    np.testing.assert_allclose(ridge_leverage_scores(A, lam), _brute(A, lam), rtol=1e-12, atol=1e-14)


def test_leverage_sum_is_rank_and_bounded():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 5))
    lev = leverage_scores(A)
    assert abs(lev.sum() - 5) < 1e-12
    assert np.all(lev >= 0) and np.all(lev <= 1 + 1e-14)
    Ad = np.hstack([A, A[:, :1]])           # rank-deficient: duplicated column
    assert abs(leverage_scores(Ad).sum() - 5) < 1e-10
    Az = A.copy()
    Az[3] = 0.0
    assert leverage_scores(Az)[3] == 0.0


def test_kronecker_leverage_is_product():
    rng = np.random.default_rng(2)
    As = [rng.standard_normal((6, 2)), rng.standard_normal((5, 3)), rng.standard_normal((4, 2))]
    lK = leverage_scores(kron_explicit(As))
    prod = leverage_scores(As[0])
    for A in As[1:]:
        prod = np.multiply.outer(prod, leverage_scores(A)).reshape(-1)
    np.testing.assert_allclose(lK, prod, rtol=1e-11, atol=1e-14)
    assert abs(lK.sum() - 12) < 1e-10


def test_kronecker_ridge_leverage_formula():
    # ridge leverage of K = sum over t of prod sigma^2/(prod sigma^2 + lam) (prod u)^2
    rng = np.random.default_rng(3)
    As = [rng.standard_normal((5, 2)), rng.standard_normal((4, 3))]
    lam = 0.7
    svds = [np.linalg.svd(A, full_matrices=False) for A in As]
    ref = np.zeros((5, 4))
    for i1, i2 in itertools.product(range(5), range(4)):
        for t1, t2 in itertools.product(range(2), range(3)):
            s2 = (svds[0][1][t1] * svds[1][1][t2]) ** 2
            ref[i1, i2] += s2 / (s2 + lam) * (svds[0][0][i1, t1] * svds[1][0][i2, t2]) ** 2
    np.testing.assert_allclose(ridge_leverage_scores(kron_explicit(As), lam), ref.reshape(-1),
                               rtol=1e-11)


def test_quantize_grid():
    rng = np.random.default_rng(4)
    lev = rng.random(300) ** 4
    lev[7] = 0.0
    Q = quantize(lev)
    assert Q.dtype == np.uint64 and int(Q.sum()) == GRID and int(cdf(Q)[-1]) == GRID
    assert Q[7] == 0 and np.all(Q[lev > 0] >= 1)
    p = lev / lev.sum()
    err = np.abs(Q.astype(np.float64) - p * GRID)
    j = int(np.argmax(Q))
    bound = np.where(p * GRID < 0.5, 1.0, 0.5 + 1e-6)   # tiny p are lifted to Q = 1
    assert np.all(np.delete(err - bound, j) <= 0)
    assert err[j] <= 300.0


def test_quantize_uniform_power_of_two_is_exact():
    # uniform leverage over 2^k rows (square factors) lands exactly on the grid
    for k in (2, 3, 6):
        lev = np.ones(2**k) * (1 + 1e-15 * np.random.default_rng(k).standard_normal(2**k))
        Q = quantize(lev)
        assert np.all(Q == GRID // 2**k)


def test_quantize_rejects_bad_input():
    with pytest.raises(ValueError):
        quantize(np.zeros(4))
    with pytest.raises(ValueError):
        quantize(np.array([1.0, np.nan]))


def _heavy(rng, I, R, heavy=2, scale=30.0):
    A = rng.standard_normal((I, R))
    A[rng.choice(I, size=heavy, replace=False)] *= scale
    return A


def test_row_norm_distribution_is_a_beta_overestimate():
    # l_i <= ||a_i||^2 / sigma_min^2 gives the squared row norms beta1 = R
    # sigma_min^2 / ||A||_F^2, the uniform distribution has beta2 = R / (I max l);
    # their even mixture q satisfies q_i >= beta l_i / R with beta = max/2 (the
    # definition of beta-overestimate in Section 3), also with heavy rows
    from oracle.leverage import row_norm_weights
    rng = np.random.default_rng(3)
    for A in (rng.standard_normal((50, 4)), _heavy(rng, 60, 5)):
        lev = leverage_scores(A)
        I, R = A.shape
        q = row_norm_weights(A).astype(np.float64) / 2.0**32
        s = np.linalg.svd(A, compute_uv=False)
        beta = max(R * s[-1] ** 2 / np.sum(A * A), R / (I * lev.max())) / 2
        assert np.all(q >= beta * lev / R * (1 - 1e-6))
        assert 0 < beta <= 1
        np.testing.assert_allclose(q, (np.sum(A * A, axis=1) / np.sum(A * A) + 1.0 / I) / 2, rtol=1e-6)


def test_spectral_approximation_is_unbiased_and_lemma_bound():
    # E[A~^T A~] = A^T A (weights 1/sqrt(k q')), and Lemma
    # block_sketch_is_spectral_approx: with k > 144 R ln(2R/delta) / (beta e0^2)
    # rows the relative spectrum of A~^T A~ lies in [1 - e0, 1 + e0] with
    # probability >= 1 - delta (checked: >= 18 of 20 seeds at delta = 0.1)
    from oracle.leverage import spectral_approximation
    rng = np.random.default_rng(4)
    A = _heavy(rng, 40, 2)
    G = A.T @ A
    L = np.linalg.cholesky(G)
    Li = np.linalg.inv(L)
    acc = np.zeros_like(G)
    for s in range(400):
        At, rows = spectral_approximation(A, 64, s, 1, 0)
        acc += At.T @ At
    rel = Li @ (acc / 400) @ Li.T
    assert np.allclose(rel, np.eye(2), atol=0.05), rel
    s = np.linalg.svd(A, compute_uv=False)
    beta = 2 * s[-1] ** 2 / np.sum(A * A)
    e0, delta = 0.25, 0.1
    k = int(np.ceil(144 * 2 * np.log(4 / delta) / (beta * e0**2)))
    ok = 0
    for seed in range(20):
        At, _ = spectral_approximation(A, k, seed, 2, 1)
        ev = np.linalg.eigvalsh(Li @ (At.T @ At) @ Li.T)
        ok += int(ev.min() >= 1 - e0 and ev.max() <= 1 + e0)
    assert ok >= 18, (ok, k)


def test_jl_projection_entries_are_standard_normal():
    from oracle.leverage import jl_projection
    G = jl_projection(64, 4096, 5, 6, 2) * 8.0
    assert abs(G.mean()) < 0.01 and abs(G.var() - 1.0) < 0.02
    # entry (c, t) depends only on its own counter: a sub-block is the same block
    np.testing.assert_allclose(jl_projection(4, 10, 5, 6, 2) * 2.0, G[:4, :10], rtol=1e-15)
    np.testing.assert_allclose(jl_projection(4, 10, 5, 6, 2, t0=30) * 2.0, G[:4, 30:40], rtol=1e-15)


def test_fast_ls_comp_bound_with_a_known_spectral_approximation():
    # Lemma fast-ls-comp: given A~ with A^T A <= A~^T A~ <= (1 + eps/4) A^T A and a
    # Johnson-Lindenstrauss projection accurate to eps/20 (r = 4 ln(2I/delta) /
    # ((eps/20)^2 - (eps/20)^3) rows, Lemma random-projection), every score lies in
    # [l_i, (1 + eps/2) l_i].  A~ = sqrt(1 + eps/8) A meets the condition exactly.
    from oracle.leverage import jl_leverage_scores
    rng = np.random.default_rng(6)
    eps, I, delta = 0.25, 12, 0.05
    A = _heavy(rng, I, 3, heavy=1, scale=10.0)
    e = eps / 20
    r = int(np.ceil(4 * np.log(2 * I / delta) / (e**2 - e**3)))
    lt = jl_leverage_scores(A, np.sqrt(1 + eps / 8) * A, r, eps, 7, 8, 0)
    lev = leverage_scores(A)
    assert np.all(lt >= lev * (1 - 1e-12)) and np.all(lt <= (1 + eps / 2) * lev), (lt / lev, r)


def test_approximate_leverage_within_the_algorithm_factor():
    # Algorithm 2's first loop end to end on a small factor: with a spectral
    # approximation of many rows and a long projection, the normalised
    # approximate distribution is within the algorithm's per-mode factor
    # 1 + log(1 + eps/2)/N of the exact one (N = 1, eps = 0.25)
    from oracle.leverage import approximate_leverage_scores
    rng = np.random.default_rng(9)
    A = _heavy(rng, 30, 2, heavy=1, scale=5.0)
    eps, N = 0.25, 1
    lt, Nm = approximate_leverage_scores(A, 6000, 1500, eps, 1, 2, 0)
    p, pt = leverage_scores(A) / 2.0, lt / lt.sum()
    ratio = pt / p
    bound = 1 + np.log(1 + eps / 2) / N
    assert np.all(ratio <= bound) and np.all(ratio >= 1 / bound), (ratio.min(), ratio.max(), bound)
    np.testing.assert_allclose(Nm, A.T @ A, rtol=0.1)
