"""Pins Algorithm 3's oracle (Woodbury form, penalised row problem) and exact Tucker ALS."""

import math

import numpy as np
import pytest

from oracle.kron import kron_explicit, tucker_reconstruct, unfold
from oracle.regression import kron_rows
from oracle.tucker import (FactorUpdateSetup, exact_factor_update, fast_factor_matrix_update,
                           penalty_weight, rre, tucker_als, tucker_loss)


def _tiny(seed=0):
    rng = np.random.default_rng(seed)
    I, R = (7, 6, 5), (2, 3, 2)
    As = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    G = rng.standard_normal(R)
    X = tucker_reconstruct(G, As) + 0.1 * rng.standard_normal(I)
    return X, As, G


@pytest.mark.parametrize("n", [0, 1, 2])
def test_woodbury_inverse_matches_explicit(n):
    X, As, G = _tiny(1)
    S = FactorUpdateSetup(As, G, n, lam=0.2, eps=0.1)
    Minv = S.woodbury()
    M = S.M_explicit()
    H = np.random.default_rng(2).standard_normal((M.shape[0], 3))
    np.testing.assert_allclose(np.column_stack([Minv(h) for h in H.T]), np.linalg.solve(M, H),
                               rtol=1e-8, atol=1e-10)


def test_printed_woodbury_sign_is_not_the_inverse():
    X, As, G = _tiny(3)
    S = FactorUpdateSetup(As, G, 1, lam=0.2, eps=0.1)
    from oracle.regression import KronPreconditioner
    Ainv = KronPreconditioner(S.As_other, S.w)
    U, V = S.Gp, S.lam * S.GtP - S.w * S.Gn
    AinvU = Ainv.apply(U)
    C = np.eye(U.shape[1]) + V @ AinvU
    h = np.random.default_rng(4).standard_normal(U.shape[0])
    t = Ainv.apply(h)
    plus = t + AinvU @ np.linalg.solve(C, V @ t)
    ref = np.linalg.solve(S.M_explicit(), h)
    assert np.linalg.norm(plus - ref) > 1e-3 * np.linalg.norm(ref)


def test_penalty_weight_satisfies_constraint_lemma():
    X, As, G = _tiny(5)
    for n in range(3):
        S = FactorUpdateSetup(As, G, n, lam=0.3, eps=0.1)
        K = kron_explicit(S.As_other)
        blk = np.vstack([K, math.sqrt(S.lam) * S.GtP])
        bound = (1 + 12 / S.eps) * np.linalg.norm(blk @ np.linalg.pinv(S.Nmat, rcond=1e-10), 2) ** 2
        assert S.w >= bound * (1 - 1e-12)
        assert abs(penalty_weight(S.As_other, 0.1) - S.w) < 1e-12 * S.w


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_exact_factor_update_matches_lstsq(lam):
    X, As, G = _tiny(6)
    for n in range(3):
        K = kron_explicit([As[m] for m in range(3) if m != n])
        D = K @ unfold(G, n).T
        B = unfold(X, n)
        top = np.vstack([D, math.sqrt(lam) * np.eye(D.shape[1])])
        ref = np.linalg.lstsq(top, np.vstack([B.T, np.zeros((D.shape[1], B.shape[0]))]),
                              rcond=None)[0].T
        np.testing.assert_allclose(exact_factor_update(X, As, G, n, lam), ref, rtol=1e-9,
                                   atol=1e-10)


def test_penalised_row_problem_on_full_k_is_near_exact():
    # Lemma constraint-reg: the penalised (unsketched) problem is a (1+eps)-approximation of
    # the constrained one, which equals the original ridge row problem
    X, As, G = _tiny(7)
    lam = 0.3
    n = 0
    S = FactorUpdateSetup(As, G, n, lam=lam, eps=0.1)
    K = kron_explicit(S.As_other)
    B = unfold(X, n)
    exact = exact_factor_update(X, As, G, n, lam)
    D = K @ S.Gn.T
    for i in range(3):
        z = S.row_direct(K, np.ones(K.shape[0]), B[i])
        y = S.GtP @ z
        f = lambda yy: np.sum((D @ yy - B[i]) ** 2) + lam * yy @ yy
        assert f(y) <= (1 + 0.1) * f(exact[i]) + 1e-12


def test_row_richardson_converges_to_direct():
    X, As, G = _tiny(8)
    S = FactorUpdateSetup(As, G, 2, lam=0.1, eps=0.1)
    sk = S.row_sketch(400, seed=0, stream=9, row=3)
    KD = kron_rows(S.As_other, sk["ridx"])
    bD = unfold(X, 2)[3, sk["rows"]]
    zd = S.row_direct(KD, sk["Omega"], bD)
    rich = S.row_richardson(KD, sk["Omega"], bD, tol=1e-13, max_iter=2000)
    assert rich["status"] == "converged"
    assert np.linalg.norm(rich["z"] - zd) / np.linalg.norm(zd) < 1e-9


def test_fast_factor_update_close_to_exact():
    rng = np.random.default_rng(9)
    I, R = (30, 25, 20), (3, 3, 2)
    As = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    G = rng.standard_normal(R)
    X = tucker_reconstruct(G, As) + 0.05 * rng.standard_normal(I)
    lam, n = 0.01, 0
    A_fast, infos = fast_factor_matrix_update(X, As, G, n, lam, 0.1, m=600, seed=0, stream=1)
    A_ex = exact_factor_update(X, As, G, n, lam)
    K = kron_explicit([As[1], As[2]])
    D = K @ unfold(G, n).T
    B = unfold(X, n)
    for i in range(I[0]):
        f = lambda y: np.sum((D @ y - B[i]) ** 2) + lam * y @ y
        assert f(A_fast[i]) <= 1.1 * f(A_ex[i])
    assert all(inf["status"] == "converged" for inf in infos)


def test_exact_als_monotone_and_recovers_planted():
    rng = np.random.default_rng(10)
    I, R = (20, 18, 16), (3, 3, 3)
    Qs = [np.linalg.qr(rng.standard_normal((i, r)))[0] for i, r in zip(I, R)]
    G0 = rng.standard_normal(R)
    Xc = tucker_reconstruct(G0, Qs)
    E = rng.standard_normal(I)
    X = Xc + 0.01 * np.linalg.norm(Xc) / np.linalg.norm(E) * E
    As0 = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    lam = 1e-6
    G, As, trace = tucker_als(X, rng.standard_normal(R), As0, lam, sweeps=8)
    assert all(b <= a + 1e-12 for a, b in zip(trace, trace[1:]))
    assert trace[-1] < 2e-4
    assert abs(rre(X, G, As) - trace[-1]) < 1e-15


def test_tucker_loss_and_rre_brute_force():
    # both against the definition written out entry by entry (no mode products):
    # Xhat[i,j,k] = sum_{a,b,c} G[a,b,c] A1[i,a] A2[j,b] A3[k,c]
    rng = np.random.default_rng(12)
    I, R = (3, 4, 2), (2, 3, 2)
    As = [rng.standard_normal((i, r)) for i, r in zip(I, R)]
    G = rng.standard_normal(R)
    X = rng.standard_normal(I)
    lam = 0.37
    sq, xx = 0.0, 0.0
    for i in range(I[0]):
        for j in range(I[1]):
            for k in range(I[2]):
                xh = 0.0
                for a in range(R[0]):
                    for b in range(R[1]):
                        for c in range(R[2]):
                            xh += G[a, b, c] * As[0][i, a] * As[1][j, b] * As[2][k, c]
                sq += (X[i, j, k] - xh) ** 2
                xx += X[i, j, k] ** 2
    reg = sum(v * v for v in G.ravel()) + sum(v * v for A in As for v in A.ravel())
    assert abs(tucker_loss(X, G, As, lam) - (sq + lam * reg)) <= 1e-12 * (sq + lam * reg)
    assert abs(rre(X, G, As) - sq / xx) <= 1e-12 * (sq / xx)
