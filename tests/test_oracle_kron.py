"""Pins the oracle's layout conventions and KronMatMul against explicit Kronecker products."""

import itertools

import numpy as np
import pytest

from oracle.kron import (fold, kron_explicit, kron_matmul, mode_product, tucker_reconstruct,
                         unfold, vec, vec_col)


@pytest.mark.parametrize("shapes,K", [
    ([(3, 2)], 1), ([(4, 3), (2, 5)], 3), ([(3, 2), (4, 3), (2, 2)], 2),
    ([(2, 3), (3, 2), (2, 2), (3, 1)], 1)])
def test_kron_matmul_matches_explicit(shapes, K):
    rng = np.random.default_rng(0)
    As = [rng.standard_normal(s) for s in shapes]
    J = int(np.prod([s[1] for s in shapes]))
    B = rng.standard_normal((J, K))
    np.testing.assert_allclose(kron_matmul(As, B), kron_explicit(As) @ B, rtol=1e-13, atol=1e-13)


def test_column_stacking_identity():
    # Lemma mixed_kron_vec_mult: vec(B C A^T) = (A kron B) vec(C) with column-stacking vec
    rng = np.random.default_rng(1)
    A, B, C = rng.standard_normal((4, 3)), rng.standard_normal((5, 2)), rng.standard_normal((2, 3))
    np.testing.assert_allclose(vec_col(B @ C @ A.T), np.kron(A, B) @ vec_col(C), rtol=1e-13)


def test_row_major_tucker_identity():
    # (A1 kron A2 kron A3) vec(G) = vec(G x1 A1 x2 A2 x3 A3) with row-major vec
    rng = np.random.default_rng(2)
    As = [rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    G = rng.standard_normal((2, 3, 2))
    np.testing.assert_allclose(kron_explicit(As) @ vec(G), vec(tucker_reconstruct(G, As)),
                               rtol=1e-12, atol=1e-12)


def test_mode_product_elementwise():
    rng = np.random.default_rng(3)
    T = rng.standard_normal((3, 4, 2))
    M = rng.standard_normal((5, 4))
    Y = mode_product(T, M, 1)
    ref = np.zeros((3, 5, 2))
    for i, j, k, l in itertools.product(range(3), range(5), range(2), range(4)):
        ref[i, j, k] += T[i, l, k] * M[j, l]
    np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-14)


def test_unfolding_matches_kronecker_order():
    # X_(n) = A(n) G_(n) (kron_{m != n} A(m))^T for X = G x1 A1 .. xN AN
    rng = np.random.default_rng(4)
    As = [rng.standard_normal((4, 2)), rng.standard_normal((3, 3)), rng.standard_normal((5, 2))]
    G = rng.standard_normal((2, 3, 2))
    X = tucker_reconstruct(G, As)
    for n in range(3):
        Kn = kron_explicit([As[m] for m in range(3) if m != n])
        np.testing.assert_allclose(unfold(X, n), As[n] @ unfold(G, n) @ Kn.T, rtol=1e-12,
                                   atol=1e-12)
        np.testing.assert_array_equal(fold(unfold(X, n), n, X.shape), X)
