"""Kronecker products, mode-n products and KronMatMul (oracle, FP64).

Layout reading (the paper's vec is "lexicographic" but its matrix example stacks
columns, which only matches the reversed Kronecker order): everything here is
row-major with the last index fastest.  Row (i_1..i_N) of
K = A(1) kron ... kron A(N) is the linear index sum_n i_n prod_{k>n} I_k, column
(r_1..r_N) likewise, vec() flattens row-major, and the mode-n unfolding X_(n)
orders its columns row-major over the remaining indices.  With these, K vec(G) =
vec(G x_1 A(1) ... x_N A(N)).

Pinned by tests/test_oracle_kron.py (explicit np.kron on tiny inputs, the
column-stacking identity of Lemma mixed_kron_vec_mult, the Tucker identity above).
"""

from functools import reduce

import numpy as np


def vec(X):
    """Row-major vectorisation (last index fastest)."""
    return np.ascontiguousarray(X).reshape(-1)


def vec_col(C):
    """Column-stacking vectorisation used in Lemma mixed_kron_vec_mult."""
    return np.asarray(C).reshape(-1, order="F")


def kron_explicit(As):
    """A(1) kron A(2) kron ... kron A(N), formed densely (tiny inputs only)."""
    return reduce(np.kron, [np.asarray(A, dtype=np.float64) for A in As])


def mode_product(T, M, n):
    """n-mode product T x_n M with M of shape (J, I_n) (Section 2, Tensor Products).

    Each mode-n fibre of T is multiplied by M:
    (T x_n M)[.., j, ..] = sum_{i_n} T[.., i_n, ..] M[j, i_n].
    """
    T = np.asarray(T, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    out = np.tensordot(M, T, axes=([1], [n]))  # J first, remaining modes after
    return np.moveaxis(out, 0, n)


def kron_matmul(As, B):
    """(A(1) kron ... kron A(N)) B by successive mode products (Lemma kron_mat_mul).

    As[n] has shape (I_n, J_n); B has J_1*...*J_N rows (a vector is one column).
    Following the lemma's proof, the rightmost factor is applied first and the
    rest recursively; each column of B is the row-major vec of a J_1 x..x J_N
    tensor.
    """
    As = [np.asarray(A, dtype=np.float64) for A in As]
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    if squeeze:
        B = B[:, None]
    J = [A.shape[1] for A in As]
    I = [A.shape[0] for A in As]
    K = B.shape[1]
    if B.shape[0] != int(np.prod(J)):
        raise ValueError("B has %d rows, expected %d" % (B.shape[0], int(np.prod(J))))
    T = B.T.reshape([K] + J)  # column k of B as a tensor, batch axis first
    for n in reversed(range(len(As))):
        T = mode_product(T, As[n], n + 1)
    out = T.reshape(K, int(np.prod(I))).T
    return out[:, 0] if squeeze else out


def unfold(X, n):
    """Mode-n unfolding X_(n): rows i_n, columns row-major over the other modes."""
    X = np.asarray(X)
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def fold(Xn, n, shape):
    """Inverse of unfold() for a tensor of the given shape."""
    rest = [s for k, s in enumerate(shape) if k != n]
    return np.moveaxis(np.asarray(Xn).reshape([shape[n]] + rest), 0, n)


def tucker_reconstruct(G, As):
    """G x_1 A(1) x_2 ... x_N A(N) (reconstructed tensor, Tucker section)."""
    T = np.asarray(G, dtype=np.float64)
    for n, A in enumerate(As):
        T = mode_product(T, A, n)
    return T
