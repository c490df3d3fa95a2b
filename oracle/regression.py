"""Algorithm 2 (FastKroneckerRegression) and its exact baselines (oracle, FP64).

The result of the method is, by definition, the minimiser of the sketched ridge
problem  min_x sum_j Omega_j (k_j x - b_j)^2 + lam ||x||^2  (Corollary
approximate_ridge_regression); preconditioned Richardson (Lemma
richardson_iteration) only reaches that point.  So the oracle provides both:

  solve_sketched_direct   the sketched minimiser by Householder QR on the
                          stacked matrix [sqrt(Omega) K_D ; sqrt(lam) I];
  richardson              Algorithm 2's iteration x <- x - (1 - sqrt(eps)) M^+
                          (K~^T K~ x + lam x - K~^T b~) with the preconditioner
                          M^+ = (kron V) D (kron V)^T from the eigen-decomposition
                          of each factor Gram matrix, products taken with the
                          explicit sampled rows K_D.

Readings: the loop stops when eta ||d|| <= tol ||x|| (the paper says only "until
convergence"); the guarantee is read as f(x~) <= (1 + eps) min_x f(x) with
f(x) = ||Kx - b||^2 + lam ||x||^2.

exact_solution is the paper's exact KronMatMul baseline (the OPT column of its
Kronecker-regression tables) via the factor SVDs; loss evaluates f.

Pinned by tests/test_oracle_regression.py: explicit sketch-matrix normal
equations, lstsq on the explicit K, convergence to the direct solution at the
rate predicted from the spectrum, the (1 + eps) guarantee at the theory
sample count on a tiny problem (delta = 1/e, 0.1 and 0.5), and the theory count
itself against the rows-sampled percentages the paper prints in its Table 2
(eps = 0.1, delta = 0.01, scaled by alpha = 1e-5).
"""

import math

import numpy as np

from .kron import kron_matmul
from .leverage import leverage_scores, quantize
from .sampling import merge, sample_product


def theory_sample_count(R, eps, delta):
    """s = ceil(1680 R ln(40 R) ln(1/delta) / eps) (Algorithm 2, sample-count line).

    Pinned by the paper's Table 2 rows-sampled column (see the module header)."""
    return int(math.ceil(1680.0 * R * math.log(40.0 * R) * math.log(1.0 / delta) / eps))


def kron_rows(As, ridx):
    """Explicit rows k_j = a(1)_{i_1} kron ... kron a(N)_{i_N} of K: shape (D, R)."""
    As = [np.asarray(A, dtype=np.float64) for A in As]
    out = As[0][ridx[:, 0]]
    for n in range(1, len(As)):
        a = As[n][ridx[:, n]]
        out = (out[:, :, None] * a[:, None, :]).reshape(out.shape[0], -1)
    return out


def solve_sketched_direct(KD, Omega, bD, lam):
    """argmin_x sum_j Omega_j (k_j x - b_j)^2 + lam ||x||^2 by Householder QR.

    KD: (D, R) explicit distinct sampled rows; bD: (D,) or (D, nrhs).
    """
    KD = np.asarray(KD, dtype=np.float64)
    w = np.sqrt(np.asarray(Omega, dtype=np.float64))
    bD = np.asarray(bD, dtype=np.float64)
    squeeze = bD.ndim == 1
    if squeeze:
        bD = bD[:, None]
    R = KD.shape[1]
    top = KD * w[:, None]
    rhs = bD * w[:, None]
    if lam > 0.0:
        top = np.vstack([top, math.sqrt(lam) * np.eye(R)])
        rhs = np.vstack([rhs, np.zeros((R, bD.shape[1]))])
    Q, Rm = np.linalg.qr(top, mode="reduced")
    x = np.linalg.solve(Rm, Q.T @ rhs)
    return x[:, 0] if squeeze else x


class KronPreconditioner:
    """M^+ = (V(1) kron .. kron V(N)) D (V(1) kron .. kron V(N))^T, Algorithm 2.

    G_n = A(n)^T A(n) = V_n diag(lambda_n) V_n^T (numpy eigh), and
    D = (lambda_1 kron .. kron lambda_N + lam)^+ (zero where the sum vanishes).
    """

    def __init__(self, As, lam, shift_tol=None):
        self.V = []
        evals = []
        for A in As:
            A = np.asarray(A, dtype=np.float64)
            ev, V = np.linalg.eigh(A.T @ A)
            self.V.append(V)
            evals.append(ev)
        prod = evals[0]
        for ev in evals[1:]:
            prod = np.multiply.outer(prod, ev).reshape(-1)
        denom = prod + lam
        if shift_tol is None:
            shift_tol = denom.size * np.finfo(np.float64).eps * np.max(np.abs(denom))
        self.D = np.where(denom > shift_tol, 1.0 / np.where(denom > shift_tol, denom, 1.0), 0.0)
        self.singular = bool(np.any(denom <= shift_tol))

    def apply(self, h):
        t = kron_matmul([V.T for V in self.V], h)
        t = (t.T * self.D).T
        return kron_matmul(self.V, t)


def richardson(As, KD, Omega, bD, lam, eps, tol=1e-12, max_iter=200, x0=None):
    """Preconditioned Richardson of Algorithm 2 on the sketched problem.

    Returns dict(x, iters, status, dnorm) with status 'converged', 'maxiter' or
    'diverged' (non-finite iterate or update).  One right-hand side.
    """
    KD = np.asarray(KD, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    bD = np.asarray(bD, dtype=np.float64)
    eta = 1.0 - math.sqrt(eps)
    P = KronPreconditioner(As, lam)
    c = KD.T @ (Omega * bD)  # K~^T b~
    x = np.zeros(KD.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    dn = []
    status = "maxiter"
    it = 0
    for it in range(1, max_iter + 1):
        grad = KD.T @ (Omega * (KD @ x)) + lam * x - c
        d = P.apply(grad)
        x = x - eta * d
        nd = float(np.linalg.norm(d))
        dn.append(nd)
        if not (np.isfinite(nd) and np.all(np.isfinite(x))):
            status = "diverged"
            break
        if eta * nd <= tol * float(np.linalg.norm(x)):
            status = "converged"
            break
    return {"x": x, "iters": it, "status": status, "dnorm": np.array(dn)}


def exact_solution(As, b, lam=0.0):
    """argmin_x ||K x - b||^2 + lam ||x||^2 via the factor thin SVDs (KronMatMul).

    With A(n) = U_n S_n V_n^T: x* = (kron V) diag(kron s / (kron s^2 + lam))
    (kron U)^T b; for lam = 0 this is (kron A(n)^+) b.
    """
    Us, Ss, Vs = [], [], []
    for A in As:
        U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
        Us.append(U)
        Ss.append(s)
        Vs.append(Vt.T)
    sig = Ss[0]
    for s in Ss[1:]:
        sig = np.multiply.outer(sig, s).reshape(-1)
    den = sig**2 + lam
    scale = np.where(den > 0, sig / np.where(den > 0, den, 1.0), 0.0)
    t = kron_matmul([U.T for U in Us], b)
    t = (np.asarray(t).T * scale).T
    return kron_matmul(Vs, t)


def loss(As, b, x, lam=0.0):
    """f(x) = ||K x - b||^2 + lam ||x||^2, K x expanded by KronMatMul."""
    r = kron_matmul(As, x) - np.asarray(b, dtype=np.float64)
    return float(np.sum(r * r) + lam * np.sum(np.asarray(x, dtype=np.float64) ** 2))


def sketch(As, m, seed, stream=0, row=0):
    """Steps before the iteration: leverage, quantised weights, samples, merge.

    Returns dict(lev, Q, idx, omega, rows, ridx, counts, Omega).
    """
    lev = [leverage_scores(A) for A in As]
    Q = [quantize(l) for l in lev]
    idx, omega = sample_product(Q, m, seed, stream, row)
    I = [np.asarray(A).shape[0] for A in As]
    rows, ridx, counts, Omega = merge(idx, omega, I)
    return dict(lev=lev, Q=Q, idx=idx, omega=omega, rows=rows, ridx=ridx,
                counts=counts, Omega=Omega)


def fast_kronecker_regression(As, b, lam, eps, m, seed, stream=0, tol=1e-12,
                              max_iter=200, direct=True):
    """Algorithm 2 replayed step by step (exact leverage, explicit m).

    Returns the sketch() fields plus bD (gathered b), KD, x_direct (if direct),
    and the Richardson result (x, iters, status, dnorm).
    """
    out = sketch(As, m, seed, stream)
    b = np.asarray(b, dtype=np.float64)
    bD = b[out["rows"]]
    KD = kron_rows(As, out["ridx"])
    out["bD"] = bD
    out["KD"] = KD
    if direct:
        out["x_direct"] = solve_sketched_direct(KD, out["Omega"], bD, lam)
    out.update(richardson(As, KD, out["Omega"], bD, lam, eps, tol, max_iter))
    return out


def _split(As, ridx, t):
    """Common part of the split products: the distinct T^c-prefixes (first N - t
    modes) of the distinct rows, the explicit Kronecker rows of those prefixes
    (|S_2| x R_{T^c}), the row ranges [start_s, start_{s+1}) of each prefix (rows
    sorted by linear index keep each prefix's rows together), and R_T."""
    N = len(As)
    if not 1 <= t < N:
        raise ValueError("the split needs 1 <= t < N")
    I = [np.asarray(A).shape[0] for A in As]
    pre = np.zeros(ridx.shape[0], dtype=np.int64)
    for n in range(N - t):
        pre = pre * int(I[n]) + ridx[:, n]
    if np.any(np.diff(pre) < 0):
        raise ValueError("rows must be sorted by linear index (as merge returns them)")
    starts = np.concatenate([[0], np.flatnonzero(np.diff(pre)) + 1, [ridx.shape[0]]])
    Abar = kron_rows(As[:N - t], ridx[starts[:-1], :N - t])
    RT = int(np.prod([np.asarray(A).shape[1] for A in As[N - t:]]))
    return Abar, starts, RT


def _row_blocks(starts, rows_per_block):
    """Consecutive runs of prefixes [s0, s1) holding about rows_per_block rows."""
    s0 = 0
    ns = starts.size - 1
    while s0 < ns:
        s1 = int(np.searchsorted(starts, starts[s0] + rows_per_block, side="right")) - 1
        s1 = max(s1, s0 + 1)
        yield s0, min(s1, ns)
        s0 = min(s1, ns)


def sampled_forward_split(As, ridx, x, t, chunk=8192):
    """K_D x for the distinct sampled rows, by the split of Theorem
    kron_mat_mul_sqrt_decomp with T the last t modes: P = Abar_{S_2} X_mat (one
    matrix product over the distinct T^c-prefixes S_2, X_mat the iterate reshaped
    R_{T^c} x R_T), then the rows of each prefix s are the product of their T
    Kronecker rows with P[s] (R_T x nrhs).  x: (R,) or (R, nrhs); rows sorted.

    Pinned by tests/test_oracle_regression.py against the explicit rows kron_rows."""
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    X = x[:, None] if vec else x
    Abar, starts, RT = _split(As, ridx, t)
    q = X.shape[1]
    P = (Abar @ X.reshape(Abar.shape[1], RT * q)).reshape(-1, RT, q)
    N = len(As)
    out = np.empty((ridx.shape[0], q))
    for s0, s1 in _row_blocks(starts, chunk):
        r0, r1 = starts[s0], starts[s1]
        kT = kron_rows(As[N - t:], ridx[r0:r1, N - t:])
        for s in range(s0, s1):
            a, b = starts[s] - r0, starts[s + 1] - r0
            out[r0 + a:r0 + b] = kT[a:b] @ P[s]
    return out[:, 0] if vec else out


def sampled_adjoint_split(As, ridx, w, t, chunk=8192):
    """K_D^T w for weights w on the distinct sampled rows ((D,) or (D, nrhs)), by the
    same split: Q[s] = (T Kronecker rows of prefix s)^T w (R_T x nrhs per prefix),
    then Abar_{S_2}^T Q reshaped to R x nrhs.  Rows sorted.

    Pinned by tests/test_oracle_regression.py against the explicit rows kron_rows."""
    w = np.asarray(w, dtype=np.float64)
    vec = w.ndim == 1
    W = w[:, None] if vec else w
    Abar, starts, RT = _split(As, ridx, t)
    q = W.shape[1]
    N = len(As)
    Q = np.zeros((Abar.shape[0], RT, q))
    for s0, s1 in _row_blocks(starts, chunk):
        r0, r1 = starts[s0], starts[s1]
        kT = kron_rows(As[N - t:], ridx[r0:r1, N - t:])
        for s in range(s0, s1):
            a, b = starts[s] - r0, starts[s + 1] - r0
            Q[s] = kT[a:b].T @ W[r0 + a:r0 + b]
    out = (Abar.T @ Q.reshape(Abar.shape[0], RT * q)).reshape(-1, q)
    return out[:, 0] if vec else out


def sketched_gradient_split(As, ridx, Omega, bD, x, lam, t):
    """Gradient of the sketched ridge objective (halved), K_D^T diag(Omega)
    (K_D x - b_D) + lam x, by the split products above; zero exactly at the
    sketched minimiser (its normal equations)."""
    u = sampled_forward_split(As, ridx, x, t) - np.asarray(bD, dtype=np.float64)
    Om = np.asarray(Omega, dtype=np.float64)
    w = Om * u if u.ndim == 1 else Om[:, None] * u
    return sampled_adjoint_split(As, ridx, w, t) + lam * np.asarray(x, dtype=np.float64)


def split_point(As, ridx):
    """The t (number of trailing modes in T) that minimises the entries the split
    products touch, |S_2| R_{T^c} + D R_T (the balance the split theorem asks
    for; any t gives the same values)."""
    N = len(As)
    I = [np.asarray(A).shape[0] for A in As]
    R = [np.asarray(A).shape[1] for A in As]
    best, best_t = None, 1
    for t in range(1, N):
        pre = np.zeros(ridx.shape[0], dtype=np.int64)
        for n in range(N - t):
            pre = pre * int(I[n]) + ridx[:, n]
        cost = np.unique(pre).size * int(np.prod(R[:N - t])) + ridx.shape[0] * int(np.prod(R[N - t:]))
        if best is None or cost < best:
            best, best_t = cost, t
    return best_t
