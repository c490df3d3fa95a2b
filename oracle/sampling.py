"""RowSampling on the Kronecker product distribution (oracle).

Definition def:sample_rows_alg: s rows are drawn i.i.d. with replacement, row j
with probability p_j, and given weight 1/sqrt(p_j s).  By Lemma
kronecker_cross_leverage_scores the leverage distribution of
K = A(1) kron ... kron A(N) is the product of the factor distributions, so each
coordinate i_n of a sample is drawn independently (Algorithm 2, product
distribution; the proof of Theorem fast_kronecker_regression samples each
coordinate from its own CDF).

Random bits (the build's fixed layout, shared with the GPU sampler by
specification only): Philox4x64-10 with key (seed, stream) and counter
(t, n // 4, row, 0) for sample t, mode n and sketch row `row` (the Tucker factor
row; 0 for a plain regression).  Mode n uses output word n % 4; its top 32 bits
u select the index i with C_{i-1} <= u < C_i on the inclusive integer CDF C.

The squared sketch weight of sample t is omega_t = 1 / (m * prod_n p'_{i_n}),
multiplied in mode order 1..N in float64.  Merging duplicates (the diagonal view
of S in Theorem kron_mat_mul_sqrt_decomp) gives distinct rows j with
Omega_j = count_j * omega_j, and S^T S = diag(Omega).

Pinned by tests/test_oracle_sampling.py: chi-square of counts, unbiasedness of
the sampled product E[(SA)^T SB] = A^T B, and the explicit s x I sketch matrix.
"""

import numpy as np

from .leverage import GRID, cdf
from .philox import philox4x64_10


CHUNK = 65536


def draw_uniform_words(m, n_modes, seed, stream, row=0):
    """The 64-bit Philox word of each (sample, mode): shape (m, n_modes) uint64.

    Each output depends on its own counter only, so the counters are taken in
    chunks of CHUNK samples (cache-sized arrays; the values do not depend on it)."""
    out = np.empty((m, n_modes), dtype=np.uint64)
    for c0 in range(0, m, CHUNK):
        t = np.arange(c0, min(m, c0 + CHUNK), dtype=np.uint64)
        for g in range((n_modes + 3) // 4):
            words = philox4x64_10([t, np.uint64(g), np.uint64(row), np.uint64(0)], (seed, stream))
            for w in range(4):
                n = 4 * g + w
                if n < n_modes:
                    out[c0:c0 + t.size, n] = words[w]
    return out


def sample_product(Qs, m, seed, stream, row=0):
    """Draw m samples (i_1..i_N) from the product of the quantised distributions.

    Qs: list of N uint64 weight vectors (each sums to 2^32).
    Returns (idx, omega): idx int64 (m, N), omega float64 (m,).
    Samples are independent of each other, so they are drawn CHUNK at a time
    (the result does not depend on it).
    """
    N = len(Qs)
    Cs = []
    for n, Q in enumerate(Qs):
        C = cdf(Q)
        if int(C[-1]) != GRID:
            raise ValueError("weights of mode %d do not sum to 2^32" % n)
        Cs.append(C)
    idx = np.empty((m, N), dtype=np.int64)
    omega = np.empty(m, dtype=np.float64)
    for c0 in range(0, m, CHUNK):
        c1 = min(m, c0 + CHUNK)
        t = np.arange(c0, c1, dtype=np.uint64)
        part = np.empty((c1 - c0, N), dtype=np.int64)
        for g in range((N + 3) // 4):
            words = philox4x64_10([t, np.uint64(g), np.uint64(row), np.uint64(0)], (seed, stream))
            for w in range(4):
                n = 4 * g + w
                if n < N:
                    part[:, n] = np.searchsorted(Cs[n], words[w] >> np.uint64(32), side="right")
        idx[c0:c1] = part
        omega[c0:c1] = sample_weights(Qs, part, m)
    return idx, omega


def sample_weights(Qs, idx, m):
    """omega_t = 1 / (m * prod_n p'_{i_n}) in float64, modes multiplied in order."""
    den = np.full(idx.shape[0], float(m), dtype=np.float64)
    for n, Q in enumerate(Qs):
        pn = np.asarray(Q, dtype=np.float64)[idx[:, n]] * (1.0 / float(GRID))
        den = den * pn
    return 1.0 / den


def linear_rows(idx, I):
    """Row-major linear row index sum_n i_n prod_{k>n} I_k of each sample."""
    lin = np.zeros(idx.shape[0], dtype=np.int64)
    for n in range(idx.shape[1]):
        lin = lin * int(I[n]) + idx[:, n]
    return lin


def merge(idx, omega, I):
    """Merge duplicate samples into distinct rows (sorted by linear index).

    Returns (rows, ridx, counts, Omega): linear indices (D,), per-mode indices
    (D, N), multiplicities (D,) and Omega_j = count_j * omega_j (D,).
    """
    lin = linear_rows(idx, I)
    rows, first, counts = np.unique(lin, return_index=True, return_counts=True)
    ridx = idx[first]
    Omega = counts.astype(np.float64) * omega[first]
    return rows, ridx, counts, Omega


def sketch_matrix(idx, omega, I):
    """The explicit s x I sketch of def:sample_rows_alg: S[t, row_t] = sqrt(omega_t)."""
    lin = linear_rows(idx, I)
    S = np.zeros((idx.shape[0], int(np.prod(I))), dtype=np.float64)
    S[np.arange(idx.shape[0]), lin] = np.sqrt(omega)
    return S
