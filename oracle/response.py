"""Implicit responses b = K X_true + sigma E for problems too large for a dense b.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's synthetic regressions take b as K times a planted solution plus
Gaussian noise.  When prod(I) x nrhs entries would not fit in memory, only the
sampled rows of b are ever needed, so the noise must be a function of the row
index rather than a stream of draws: E[i][q] is a standard normal made by the
Box-Muller transform from the first two words of Philox4x64-10 at counter
(i, q, 0, 0) with key (seed, stream), where i is K's row index
i = sum_n i_n prod_{k>n} I_k:

    u1 = ((w0 >> 11) + 1) 2^-53  in (0, 1]
    u2 = (w1 >> 11) 2^-53        in [0, 1)
    E  = sqrt(-2 ln u1) cos(2 pi u2)

Pinned by tests/test_oracle_response.py: the transform at words that give
u1 = 1, u2 = 0 and u2 = 1/2 and the smallest u1 (closed forms); the first two
moments and a Kolmogorov-Smirnov test of 2^18 draws against the standard normal;
K X_true against the explicit Kronecker product (np.kron) on tiny inputs.
"""

import numpy as np

from .kron import kron_matmul
from .philox import philox4x64_10

TWO_PI = 6.283185307179586


def box_muller(w0, w1):
    """Standard normals from two uint64 words (arrays), as defined above."""
    w0 = np.asarray(w0, dtype=np.uint64)
    w1 = np.asarray(w1, dtype=np.uint64)
    u1 = ((w0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (w1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(TWO_PI * u2)


def noise(rows, nrhs, seed, stream, chunk=16384):
    """E[rows][q] for q < nrhs: array of shape (len(rows), nrhs).  Each entry
    depends on its own counter only; rows are taken chunk at a time."""
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, 1)
    q = np.arange(nrhs, dtype=np.uint64).reshape(1, -1)
    out = np.empty((rows.shape[0], nrhs))
    for c0 in range(0, rows.shape[0], chunk):
        w = philox4x64_10([rows[c0:c0 + chunk], q, np.uint64(0), np.uint64(0)], (seed, stream))
        out[c0:c0 + chunk] = box_muller(w[0], w[1])
    return out


def implicit_response(As, X_true, sigma, seed, stream):
    """The dense b = K X_true + sigma E (prod(I) x nrhs, or a vector when X_true
    is one); for tests on problems small enough to hold it."""
    X = np.asarray(X_true, dtype=np.float64)
    vec = X.ndim == 1
    X2 = X[:, None] if vec else X
    KX = kron_matmul(As, X2)
    E = noise(np.arange(KX.shape[0]), X2.shape[1], seed, stream)
    b = KX + sigma * E
    return b[:, 0] if vec else b
