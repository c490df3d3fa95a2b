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


# ---------------------------------------------------------------------------
# Approximate leverage scores for large factors (Algorithm 2's first loop:
# a spectral approximation A~ by Lemma block_sketch_is_spectral_approx, then
# (1 + eps/2)-approximate scores by Lemma fast-ls-comp with a Johnson-Lindenstrauss
# projection, Lemma random-projection).
#
# Random bits (the build's layout, shared with the GPU by specification only):
# Philox4x64-10 with key (seed, stream);
#   row t of A~ for mode n: counter (t, n, 0, 1), word 0, top 32 bits u pick the
#     row i with C_{i-1} <= u < C_i on the inclusive CDF of the quantised
#     squared row norms;
#   entry (c, t) of the projection for mode n: counter (t, c, n, 2), words 0 and
#     1 through the Box-Muller transform of oracle/response.py, divided by sqrt(r).
# ---------------------------------------------------------------------------

def row_norm_weights(A):
    """The distribution that draws the rows of A~, quantised on the 2^32 grid (as
    quantize): the even mixture q_i = (||a_i||^2 / ||A||_F^2 + 1/I) / 2 of the
    squared row norms and the uniform distribution.  Each part is a
    beta-overestimate of the leverage distribution -- the row norms with
    beta = R sigma_min^2 / ||A||_F^2 >= 1/kappa(A)^2 (l_i <= ||a_i||^2 /
    sigma_min^2), the uniform one with beta = R / (I max_i l_i) -- so the mixture is
    one with beta >= max of the two / 2: the row norms find the coherent (heavy)
    rows, the uniform part keeps the directions that only light rows span."""
    A = np.asarray(A, dtype=np.float64)
    sq = np.sum(A * A, axis=1)
    return quantize(sq / np.sum(sq) + 1.0 / A.shape[0])


def spectral_approximation(A, k, seed, stream, mode):
    """A~ = S A for S = RowSampling(A, k, q') (Definition def:sample_rows_alg) with q'
    the realised distribution of row_norm_weights: k rows drawn i.i.d., row t equal to
    a_{i_t} / sqrt(k q'_{i_t}), so that E[A~^T A~] = A^T A.  By Lemma
    block_sketch_is_spectral_approx (second block empty), (1 - e0) A^T A <= A~^T A~
    <= (1 + e0) A^T A with probability 1 - delta once k > 144 R ln(2R/delta) /
    (beta e0^2).  Returns (A~, row indices)."""
    from .philox import philox4x64_10
    A = np.asarray(A, dtype=np.float64)
    Q = row_norm_weights(A)
    C = cdf(Q)
    t = np.arange(k, dtype=np.uint64)
    w = philox4x64_10([t, np.uint64(mode), np.uint64(0), np.uint64(1)], (seed, stream))[0]
    rows = np.searchsorted(C, w >> np.uint64(32), side="right")
    qp = Q[rows].astype(np.float64) / float(GRID)
    return A[rows] / np.sqrt(k * qp)[:, None], rows


def jl_projection(r, k, seed, stream, mode, t0=0):
    """G / sqrt(r): r x k with i.i.d. N(0, 1) entries G[c, t] (Lemma
    random-projection); columns t0 .. t0 + k - 1 of it."""
    from .philox import philox4x64_10
    from .response import box_muller
    t = np.arange(t0, t0 + k, dtype=np.uint64)[None, :]
    c = np.arange(r, dtype=np.uint64)[:, None]
    w = philox4x64_10([t, c, np.uint64(mode), np.uint64(2)], (seed, stream))
    return box_muller(w[0], w[1]) / np.sqrt(float(r))


def jl_apply(At, r, seed, stream, mode, chunk=1024):
    """(G / sqrt(r)) A~, with the projection's columns generated chunk at a time."""
    At = np.asarray(At, dtype=np.float64)
    out = np.zeros((r, At.shape[1]))
    for t0 in range(0, At.shape[0], chunk):
        blk = At[t0:t0 + chunk]
        out += jl_projection(r, blk.shape[0], seed, stream, mode, t0) @ blk
    return out


def gram_pinv(N, I=None):
    """N^+ through the symmetric eigen-decomposition, over the numerical rank
    (eigenvalues above (max(I, R) u)^2 lambda_max, the rule of the exact path)."""
    ev, V = np.linalg.eigh(N)
    R = N.shape[0]
    eps_r = max(I or R, R) * np.finfo(np.float64).eps
    keep = ev > eps_r * eps_r * max(ev.max(), 0.0)
    return (V[:, keep] / ev[keep]) @ V[:, keep].T


def jl_leverage_scores(A, At, r, eps, seed, stream, mode):
    """Lemma fast-ls-comp: with N = A~^T A~ and M = (1 + eps/4) N^+, the scores
    ||G A~ M a_i||^2 / ((1 + eps/4)(1 - eps/20)) for the projection G of
    jl_projection.  When A^T A <= A~^T A~ <= (1 + eps/4) A^T A and r is large
    enough for an eps/20 projection, each lies in [l_i, (1 + eps/2) l_i].  (A
    uniform factor cancels from the sampling distribution p = l~ / sum l~.)"""
    A = np.asarray(A, dtype=np.float64)
    At = np.asarray(At, dtype=np.float64)
    M = (1.0 + eps / 4.0) * gram_pinv(At.T @ At, A.shape[0])
    Z = jl_apply(At, r, seed, stream, mode) @ M
    return np.sum((A @ Z.T) ** 2, axis=1) / ((1.0 + eps / 4.0) * (1.0 - eps / 20.0))


def approximate_leverage_scores(A, k, r, eps, seed, stream, mode):
    """Algorithm 2's approximate scores of one factor: jl_leverage_scores on the
    spectral approximation of spectral_approximation.  Returns (scores, A~^T A~),
    the Gram whose eigen-decomposition gives the preconditioner's V and Sigma."""
    At, _ = spectral_approximation(A, k, seed, stream, mode)
    return jl_leverage_scores(A, At, r, eps, seed, stream, mode), At.T @ At
