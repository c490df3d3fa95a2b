"""Algorithm 3 (FastFactorMatrixUpdate) and exact Tucker ALS (oracle, FP64).

Factor row update of Tucker ALS (Algorithm 1, factor loop): for row i of mode n,
y* = argmin_y ||K G_(n)^T y - b_i||^2 + lam ||y||^2 with K the Kronecker product of
the other factors in increasing mode order and b_i row i of X_(n).  Lemma
constrained_least_squares substitutes z = G_(n)^T y; Lemma constraint-reg replaces
the constraint N z = 0 (N = I - G_(n)^T (G_(n)^T)^+) by a penalty block sqrt(w) N.
Per row a fresh leverage sketch of K is drawn and the penalised sketched problem

    min_z sum_j Omega_j (k_j z - b_ij)^2 + lam ||(G^T)^+ z||^2 + w ||N z||^2

is solved; the row is a_i = (G^T)^+ z.

Readings:
  * the sampling distribution is the product over the other modes only (the
    algorithm's line listing all N factors contradicts its own K);
  * w = (1 + 12/eps) prod_{m != n} lambda_max(A(m)^T A(m)); since (G^T)^+ N = 0
    and N is an orthogonal projector, ||[K; sqrt(lam)(G^T)^+] N^+||^2 =
    ||K N||^2 <= ||K||^2, so this w satisfies Lemma constraint-reg's bound;
  * the Woodbury expression of Lemma fast_factor_richardson_step is used with a
    minus sign: (A + U V)^-1 = A^-1 - A^-1 U (I + V A^-1 U)^-1 V A^-1 (the printed
    plus sign does not give the inverse);
  * each row gets its own sketch: Philox counter word 2 is the row index.

Pinned by tests/test_oracle_tucker.py: explicit inv(M) for the Woodbury form,
the equivalence of the constrained and original row problems, Lemma
constraint-reg's inequality, the exact row update against lstsq on explicit
K G^T, monotone exact ALS, and rre / tucker_loss against the reconstruction
written out entry by entry.
"""

import math

import numpy as np

from .kron import fold, kron_matmul, mode_product, tucker_reconstruct, unfold, vec
from .leverage import leverage_scores, quantize
from .regression import KronPreconditioner, exact_solution, fast_kronecker_regression, kron_rows
from .sampling import merge, sample_product


def penalty_weight(As_other, eps):
    """w = (1 + 12/eps) * prod_{m != n} lambda_max(A(m)^T A(m))."""
    w = 1.0 + 12.0 / eps
    for A in As_other:
        A = np.asarray(A, dtype=np.float64)
        w *= float(np.linalg.eigvalsh(A.T @ A)[-1])
    return w


class FactorUpdateSetup:
    """Row-independent pieces of Algorithm 3 for mode n."""

    def __init__(self, As, G, n, lam, eps):
        self.n = n
        self.others = [m for m in range(len(As)) if m != n]
        self.As_other = [np.asarray(As[m], dtype=np.float64) for m in self.others]
        self.Gn = unfold(np.asarray(G, dtype=np.float64), n)          # R_n x R_{!=n}
        self.GtP = np.linalg.pinv(self.Gn.T)                           # (G_(n)^T)^+
        self.Gp = np.linalg.pinv(self.Gn)                              # G_(n)^+
        Rr = self.Gn.shape[1]
        self.Nmat = np.eye(Rr) - self.Gn.T @ self.GtP
        self.lam = lam
        self.eps = eps
        self.w = penalty_weight(self.As_other, eps)
        self.Q = [quantize(leverage_scores(A)) for A in self.As_other]
        self.I_other = [A.shape[0] for A in self.As_other]

    # ----- the operator M and its Woodbury inverse (Lemma fast_factor_richardson_step)
    def M_explicit(self):
        """M = K^T K + lam G^+ (G^T)^+ + w N^T N, formed densely (tiny inputs)."""
        G = [A.T @ A for A in self.As_other]
        KtK = G[0]
        for g in G[1:]:
            KtK = np.kron(KtK, g)
        return KtK + self.lam * self.Gp @ self.GtP + self.w * self.Nmat.T @ self.Nmat

    def woodbury(self):
        """Return a function h -> M^-1 h using (K^T K + w I)^-1 and a rank-R_n term."""
        Ainv = KronPreconditioner(self.As_other, self.w)
        U = self.Gp                                         # R_{!=n} x R_n
        V = self.lam * self.GtP - self.w * self.Gn          # R_n x R_{!=n}
        AinvU = Ainv.apply(U)
        C = np.eye(U.shape[1]) + V @ AinvU
        Cinv = np.linalg.inv(C)

        def apply(h):
            t = Ainv.apply(h)
            return t - AinvU @ (Cinv @ (V @ t))
        return apply

    # ----- one row
    def row_sketch(self, m, seed, stream, row):
        idx, omega = sample_product(self.Q, m, seed, stream, row)
        rows, ridx, counts, Omega = merge(idx, omega, self.I_other)
        return dict(idx=idx, omega=omega, rows=rows, ridx=ridx, counts=counts, Omega=Omega)

    def row_direct(self, KD, Omega, bD):
        """Minimiser of the penalised sketched row problem by Householder QR."""
        w = np.sqrt(Omega)
        top = np.vstack([KD * w[:, None], math.sqrt(self.lam) * self.GtP,
                         math.sqrt(self.w) * self.Nmat])
        rhs = np.concatenate([bD * w, np.zeros(self.GtP.shape[0] + self.Nmat.shape[0])])
        Qm, Rm = np.linalg.qr(top, mode="reduced")
        return np.linalg.solve(Rm, Qm.T @ rhs)

    def row_richardson(self, KD, Omega, bD, tol=1e-12, max_iter=400, Minv=None):
        """Algorithm 3's iteration for one row; returns dict(z, iters, status, dnorm)."""
        eta = 1.0 - math.sqrt(self.eps)
        Minv = self.woodbury() if Minv is None else Minv
        c = KD.T @ (Omega * bD)
        z = np.zeros(KD.shape[1])
        dn = []
        status = "maxiter"
        it = 0
        for it in range(1, max_iter + 1):
            grad = (KD.T @ (Omega * (KD @ z)) + self.w * z
                    + self.lam * (self.Gp @ (self.GtP @ z))
                    - self.w * (self.Gp @ (self.Gn @ z)) - c)
            d = Minv(grad)
            z = z - eta * d
            nd = float(np.linalg.norm(d))
            dn.append(nd)
            if not (np.isfinite(nd) and np.all(np.isfinite(z))):
                status = "diverged"
                break
            if eta * nd <= tol * float(np.linalg.norm(z)):
                status = "converged"
                break
        return {"z": z, "iters": it, "status": status, "dnorm": np.array(dn)}


def fast_factor_matrix_update(X, As, G, n, lam, eps, m, seed, stream, tol=1e-12,
                              max_iter=400, method="richardson", rows=None):
    """Algorithm 3 for mode n.  Returns (A_n_new, per-row info list).

    method 'richardson' replays the iteration; 'direct' solves each penalised
    sketched row problem by QR.  rows restricts the update to a subset (tests).
    """
    S = FactorUpdateSetup(As, G, n, lam, eps)
    B = unfold(np.asarray(X, dtype=np.float64), n)
    Anew = np.array(As[n], dtype=np.float64, copy=True)
    Minv = S.woodbury() if method == "richardson" else None
    infos = []
    for i in (range(B.shape[0]) if rows is None else rows):
        sk = S.row_sketch(m, seed, stream, i)
        KD = kron_rows(S.As_other, sk["ridx"])
        bD = B[i, sk["rows"]]
        if method == "direct":
            z = S.row_direct(KD, sk["Omega"], bD)
            info = {"iters": 0, "status": "direct"}
        else:
            info = S.row_richardson(KD, sk["Omega"], bD, tol, max_iter, Minv)
            z = info["z"]
        Anew[i] = S.GtP @ z
        info.update(sk)
        infos.append(info)
    return Anew, infos


def exact_factor_update(X, As, G, n, lam):
    """Exact Algorithm 1 factor update: every row's ridge problem solved exactly.

    K^T b_i for all rows is the TTM chain X x_{m != n} A(m)^T; K^T K is the
    Kronecker product of the other Gram matrices; each row solves
    (G_(n) K^T K G_(n)^T + lam I) y = G_(n) K^T b_i.
    """
    X = np.asarray(X, dtype=np.float64)
    T = X
    for m in range(X.ndim):
        if m != n:
            T = mode_product(T, np.asarray(As[m], dtype=np.float64).T, m)
    W = unfold(T, n)                                    # I_n x R_{!=n}
    Gn = unfold(np.asarray(G, dtype=np.float64), n)
    grams = [np.asarray(As[m], dtype=np.float64).T @ np.asarray(As[m], dtype=np.float64)
             for m in range(X.ndim) if m != n]
    KtK = grams[0]
    for g in grams[1:]:
        KtK = np.kron(KtK, g)
    H = Gn @ KtK @ Gn.T + lam * np.eye(Gn.shape[0])
    return np.linalg.solve(H, Gn @ W.T).T


def exact_core_update(X, As, lam):
    """Exact Algorithm 1 core update: argmin_g ||K g - vec X||^2 + lam ||g||^2."""
    R = [np.asarray(A).shape[1] for A in As]
    g = exact_solution(As, vec(np.asarray(X, dtype=np.float64)), lam)
    return np.asarray(g).reshape(R)


def rre(X, G, As):
    """Relative reconstruction error ||X^ - X||_F^2 / ||X||_F^2 (squared)."""
    X = np.asarray(X, dtype=np.float64)
    D = tucker_reconstruct(G, As) - X
    return float(np.sum(D * D) / np.sum(X * X))


def tucker_loss(X, G, As, lam):
    """||X - G x_1 A(1) .. x_N A(N)||_F^2 + lam (||G||_F^2 + sum_n ||A(n)||_F^2)."""
    X = np.asarray(X, dtype=np.float64)
    D = tucker_reconstruct(G, As) - X
    reg = np.sum(np.asarray(G, dtype=np.float64) ** 2) + sum(
        np.sum(np.asarray(A, dtype=np.float64) ** 2) for A in As)
    return float(np.sum(D * D) + lam * reg)


def als_stream(sweep, step):
    """Philox stream id of ALS step `step` (mode n, or N for the core) of a sweep."""
    return (int(sweep) << 8) | int(step)


def tucker_als(X, G0, As0, lam, sweeps, sketched=False, eps=0.1, m_factor=None,
               m_core=None, seed=0):
    """Algorithm 1 (TuckerALS): factor rows in mode order, then the core.

    sketched=False uses the exact updates; True uses Algorithm 3 for factors
    (direct per-row solve) and Algorithm 2 for the core.  Returns (G, As, rres).
    """
    X = np.asarray(X, dtype=np.float64)
    As = [np.array(A, dtype=np.float64, copy=True) for A in As0]
    G = np.array(G0, dtype=np.float64, copy=True)
    N = X.ndim
    trace = []
    for s in range(sweeps):
        for n in range(N):
            if sketched:
                As[n], _ = fast_factor_matrix_update(X, As, G, n, lam, eps, m_factor, seed,
                                                     als_stream(s, n), method="direct")
            else:
                As[n] = exact_factor_update(X, As, G, n, lam)
        if sketched:
            res = fast_kronecker_regression(As, vec(X), lam, eps, m_core, seed,
                                            stream=als_stream(s, N), direct=True)
            G = res["x_direct"].reshape([A.shape[1] for A in As])
        else:
            G = exact_core_update(X, As, lam)
        trace.append(rre(X, G, As))
    return G, As, trace


__all__ = ["FactorUpdateSetup", "fast_factor_matrix_update", "exact_factor_update",
           "exact_core_update", "rre", "tucker_loss", "tucker_als", "als_stream",
           "penalty_weight", "fold", "kron_matmul"]
