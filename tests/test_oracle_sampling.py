"""Pins RowSampling on the product distribution (def:sample_rows_alg)."""

import numpy as np
from scipy import stats

from oracle.kron import kron_explicit
from oracle.leverage import GRID, cdf, leverage_scores, quantize, realised_probabilities
from oracle.regression import kron_rows
from oracle.sampling import linear_rows, merge, sample_product, sketch_matrix


def test_inverse_cdf_boundaries():
    # index i is chosen iff C_{i-1} <= u < C_i; zero-weight entries never chosen
    Q = np.array([0, 3, 0, 5, GRID - 8], dtype=np.uint64)
    C = cdf(Q)
    for u, want in [(0, 1), (2, 1), (3, 3), (7, 3), (8, 4), (GRID - 1, 4)]:
        assert int(np.searchsorted(C, np.uint64(u), side="right")) == want


def test_chi_square_product_distribution():
    rng = np.random.default_rng(0)
    As = [rng.standard_normal((5, 2)), rng.standard_normal((7, 3))]
    Qs = [quantize(leverage_scores(A)) for A in As]
    m = 200_000
    idx, _ = sample_product(Qs, m, seed=11, stream=0)
    p = np.multiply.outer(realised_probabilities(Qs[0]), realised_probabilities(Qs[1])).reshape(-1)
    counts = np.bincount(linear_rows(idx, [5, 7]), minlength=35)
    assert stats.chisquare(counts, m * p).pvalue > 1e-4


def test_five_modes_use_two_philox_groups():
    Qs = [quantize(np.ones(3)) for _ in range(5)]
    idx, _ = sample_product(Qs, 60_000, seed=1, stream=2)
    # all 5 coordinates marginally uniform and pairwise independent
    for n in range(5):
        assert stats.chisquare(np.bincount(idx[:, n], minlength=3)).pvalue > 1e-4
    joint = np.bincount(idx[:, 3] * 3 + idx[:, 4], minlength=9)
    assert stats.chisquare(joint).pvalue > 1e-4


def test_weights_and_merged_sketch():
    rng = np.random.default_rng(2)
    As = [rng.standard_normal((6, 2)), rng.standard_normal((5, 2))]
    Qs = [quantize(leverage_scores(A)) for A in As]
    m = 500
    idx, omega = sample_product(Qs, m, seed=3, stream=1)
    # omega = s_ij^2 with s_ij = 1/sqrt(p_j s) and p_j the product probability
    pj = np.prod([realised_probabilities(Q)[idx[:, n]] for n, Q in enumerate(Qs)], axis=0)
    np.testing.assert_allclose(omega, 1.0 / (pj * m), rtol=1e-14)
    S = sketch_matrix(idx, omega, [6, 5])
    rows, ridx, counts, Omega = merge(idx, omega, [6, 5])
    StS = S.T @ S
    np.testing.assert_allclose(np.diag(StS)[rows], Omega, rtol=1e-13)
    assert np.count_nonzero(StS - np.diag(np.diag(StS))) == 0
    assert counts.sum() == m and np.all(np.diff(rows) > 0)
    np.testing.assert_array_equal(kron_rows(As, ridx), kron_explicit(As)[rows])


def test_sampled_product_is_unbiased():
    # E[(SA)^T (SB)] = A^T B for the leverage sketch; here A = B = K
    rng = np.random.default_rng(4)
    As = [rng.standard_normal((6, 2)), rng.standard_normal((5, 2))]
    K = kron_explicit(As)
    Qs = [quantize(leverage_scores(A)) for A in As]
    acc = np.zeros((4, 4))
    trials = 3000
    for s in range(trials):
        idx, omega = sample_product(Qs, 20, seed=5, stream=s)
        KS = kron_rows(As, idx) * np.sqrt(omega)[:, None]
        acc += KS.T @ KS
    acc /= trials
    ref = K.T @ K
    assert np.linalg.norm(acc - ref) / np.linalg.norm(ref) < 0.03


def test_streams_and_rows_are_independent_draws():
    Qs = [quantize(np.ones(64)), quantize(np.ones(64))]
    a, _ = sample_product(Qs, 1000, seed=0, stream=0, row=0)
    b, _ = sample_product(Qs, 1000, seed=0, stream=1, row=0)
    c, _ = sample_product(Qs, 1000, seed=0, stream=0, row=1)
    d, _ = sample_product(Qs, 1000, seed=0, stream=0, row=0)
    np.testing.assert_array_equal(a, d)
    assert np.mean(a == b) < 0.1 and np.mean(a == c) < 0.1
