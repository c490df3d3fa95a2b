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
