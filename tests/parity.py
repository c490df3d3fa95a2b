"""Helpers shared by the GPU parity tests: compare the library's sketch and solution
with the oracle on the same seeded inputs."""

import numpy as np

from oracle.leverage import GRID, leverage_scores, quantize
from oracle.regression import kron_rows, solve_sketched_direct
from oracle.sampling import merge, sample_product


def check_quantised_tables(As, Q_gpu, scores=None):
    """The GPU's integer weights equal the oracle's, except entries whose exact
    value 2^32 p_i lies within rounding of an integer boundary (reported).
    scores: the oracle's scores per mode (default: exact leverage of As)."""
    straddles = 0
    for n, A in enumerate(As):
        lev = leverage_scores(A) if scores is None else np.asarray(scores[n], dtype=np.float64)
        Qo = quantize(lev)
        Qg = np.asarray(Q_gpu[n], dtype=np.uint64)
        assert int(Qg.sum()) == GRID
        diff = np.flatnonzero(Qg != Qo)
        if diff.size:
            p = lev / lev.sum() * GRID
            # distance of the exact value to the rounding boundary (a half-integer)
            dist = np.abs(p - np.floor(p) - 0.5)
            dq = np.abs(Qg[diff].astype(np.int64) - Qo[diff].astype(np.int64))
            jmax = int(np.argmax(Qo))
            near = dist[diff] < 1e-4
            # each straddle moves its entry by 1 and the deficit entry by 1
            nstr = int(np.sum(near))
            assert nstr >= 1 and diff.size <= nstr + 1, (n, diff, dist[diff])
            assert all((near[k] and dq[k] <= 1) or (diff[k] == jmax and dq[k] <= nstr)
                       for k in range(diff.size)), (n, diff, dq, dist[diff])
            straddles += nstr
    return straddles


def check_sketch(As, sk, m, seed, stream=0, row=0):
    """Samples drawn from the GPU's tables by the oracle sampler merge to exactly
    the GPU's distinct rows, multiplicities and weights.  Returns the oracle merge."""
    I = [A.shape[0] for A in As]
    idx, omega = sample_product(sk["Q"], m, seed, stream, row)
    rows, ridx, counts, Omega = merge(idx, omega, I)
    assert sk["rows"].shape == ridx.shape, (sk["rows"].shape, ridx.shape)
    np.testing.assert_array_equal(sk["rows"], ridx)
    np.testing.assert_array_equal(sk["counts"], counts)
    np.testing.assert_allclose(sk["Omega"], Omega, rtol=2e-16, atol=0)
    return rows, ridx, counts, Omega


def sketched_solution(As, b, rows, ridx, Omega, lam):
    """The oracle's minimiser of the merged sketched problem (direct QR)."""
    KD = kron_rows(As, ridx)
    return solve_sketched_direct(KD, Omega, np.asarray(b)[rows], lam)


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
