"""Leverage scores and the quantised sampling distribution (oracle, FP64).

Statistical and ridge leverage scores follow Section 3 (definition of the
lambda-ridge leverage score and its compact-SVD form).  The sampling
distribution p_i = l_i / sum(l) of each factor (Algorithm 2, product
distribution data structure) is quantised to the nearest integers on a 2^32 grid so that the
CPU and GPU samplers agree bit for bit; the realised probabilities p'_i = Q_i/2^32
are what the sketch weights use, which keeps the sketch unbiased for p' and makes
p' a beta-overestimate of p (Section 3, definition of beta-overestimate).

Pinned by tests/test_oracle_leverage.py: brute-force definition via pinv,
sum(l) = rank, 0 <= l <= 1, and the product form of Kronecker leverage scores
(Lemma kronecker_cross_leverage_scores) against an explicit K.
"""

import numpy as np

GRID_BITS = 32
GRID = 1 << GRID_BITS


def ridge_leverage_scores(A, lam=0.0, rank_tol=None):
    """lambda-ridge leverage scores via the compact SVD (Section 3).

    l_i = sum_{k<=r} sigma_k^2 / (sigma_k^2 + lam) * u_{ik}^2, r = rank(A).
    With lam = 0 these are the statistical leverage scores.  Rows that are
    exactly zero get exactly zero.
    """
    A = np.asarray(A, dtype=np.float64)
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    if rank_tol is None:
        rank_tol = max(A.shape) * np.finfo(np.float64).eps * (s[0] if s.size else 0.0)
    r = int(np.sum(s > rank_tol))
    U, s = U[:, :r], s[:r]
    wts = s**2 / (s**2 + lam)
    lev = (U**2) @ wts
    lev[~np.any(A != 0.0, axis=1)] = 0.0
    return lev


def leverage_scores(A):
    """Statistical leverage scores l_i = a_i (A^T A)^+ a_i^T (lambda = 0)."""
    return ridge_leverage_scores(A, 0.0)


def quantize(lev):
    """Integer weights Q on the 2^32 grid for p = lev / sum(lev).

    Q_i = max(1, floor(p_i * 2^32 + 1/2)) (nearest integer) where lev_i > 0, and 0
    where lev_i == 0.  Rounding to nearest keeps exactly representable
    probabilities (uniform leverage over 2^k rows, as for square factors) away
    from the quantisation boundaries, which sit at half-integers.
    The difference 2^32 - sum(Q) is added to the largest Q (lowest index on ties)
    so that sum(Q) == 2^32 exactly.  Returns uint64.
    """
    lev = np.asarray(lev, dtype=np.float64)
    if lev.ndim != 1 or lev.size == 0 or not np.all(np.isfinite(lev)) or np.any(lev < 0):
        raise ValueError("leverage scores must be a finite non-negative vector")
    total = float(np.sum(lev))
    if total <= 0.0:
        raise ValueError("all leverage scores are zero")
    p = lev / total
    q = np.floor(p * float(GRID) + 0.5).astype(np.int64)
    q = np.where(lev > 0.0, np.maximum(q, 1), 0)
    j = int(np.argmax(q))
    q[j] += GRID - int(np.sum(q))
    if q[j] < 1:
        raise ValueError("distribution cannot be quantised on the 2^32 grid")
    return q.astype(np.uint64)


def cdf(Q):
    """Inclusive integer CDF C_i = Q_0 + ... + Q_i (C_{I-1} = 2^32)."""
    return np.cumsum(np.asarray(Q, dtype=np.uint64), dtype=np.uint64)


def realised_probabilities(Q):
    """p'_i = Q_i / 2^32, the distribution the sampler actually draws from."""
    return np.asarray(Q, dtype=np.float64) / float(GRID)
