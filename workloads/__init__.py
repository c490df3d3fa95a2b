"""Seeded synthetic inputs for the Kronecker-regression workloads.

This module only draws random inputs (NumPy PCG64, one data seed per workload)
and assembles the synthetic response b = K x_true + sigma * e; it holds none of
the method's steps (no leverage scores, sampling, sketching or solves).  The same
arrays feed the CPU oracle and the GPU library.

Workloads (sizes as named in the tests and the benchmark):
  small_regression  N=2, factors 64x8, m=2048 (K is 4096 x 64)
  skewed_regression N=3, factors 512x16 with 26 rows per mode scaled by 100,
                    K is 1.34e8 x 4096, m = ceil(R ln R / eps) = 340,696
  tucker_tensor     400^3 FP32 tensor = rank-(16,16,16) core times orthonormal
                    factors plus 1% Gaussian noise, with seeded initial factors
  paper_e1          the paper's synthetic Kronecker regression: two n x d factors
                    with entries N(1, 0.001^2), b = 1, lam = 1e-3
  random_problem    any shapes, for parity sweeps and edge cases
  batched_ridge     256 ridge problems of uneven shape: N ~ U{2,3,4},
                    I_n ~ U{32..256}, R_n ~ U{4..16}, 1-8 right-hand sides,
                    lambda = 10^U(-4,0), FP32 factors, implicit responses
"""

import math

import numpy as np


def _design_apply(As, x):
    """K x for K = A(1) kron ... kron A(N) (row-major vec), used only to synthesise b."""
    T = np.asarray(x, dtype=np.float64).reshape([A.shape[1] for A in As])
    for n, A in enumerate(As):
        T = np.moveaxis(np.tensordot(A, T, axes=([1], [n])), 0, n)
    return T.reshape(-1)


def m_rule(R, eps):
    """m = ceil(R ln R / eps), the explicit sample count of the large workloads."""
    return int(math.ceil(R * math.log(R) / eps))


def small_regression(seed=1):
    """N=2, A(n) 64x8 i.i.d. N(0,1), b = K x_true + 0.01 e, m = 2048, eps = 0.1."""
    rng = np.random.default_rng(seed)
    As = [rng.standard_normal((64, 8)) for _ in range(2)]
    x_true = rng.standard_normal(64)
    e = rng.standard_normal(64 * 64)
    b = _design_apply(As, x_true) + 0.01 * e
    return dict(name="small_regression N=2 I=64x64 R=8x8 m=2048", As=As, b=b,
                x_true=x_true, lam=0.0, eps=0.1, m=2048, seed=0)


def skewed_regression(seed=2, I=512, R=16, N=3, heavy_frac=0.05, scale=100.0, sigma=0.1):
    """N=3, A(n) 512x16 N(0,1) with 26 random rows per mode scaled x100.

    b = K x_true + 0.1 e (1.34e8 float64 entries, 1.07 GB); m = ceil(R ln R/eps).
    """
    rng = np.random.default_rng(seed)
    As = []
    nheavy = int(round(heavy_frac * I))
    for _ in range(N):
        A = rng.standard_normal((I, R))
        heavy = rng.choice(I, size=nheavy, replace=False)
        A[heavy] *= scale
        As.append(A)
    x_true = rng.standard_normal(R**N)
    b = _design_apply(As, x_true)
    b += sigma * rng.standard_normal(b.size)
    eps = 0.1
    return dict(name="skewed_regression N=%d I=%d^%d R=%d^%d" % (N, I, N, R, N), As=As, b=b,
                x_true=x_true, lam=0.0, eps=eps, m=m_rule(R**N, eps), seed=0)


def tucker_tensor(seed=3, I=400, R=16, N=3, noise=0.01):
    """Dense FP32 tensor = core x_n orthonormal factors + noise, and an initial guess.

    Noise is i.i.d. Gaussian scaled so that ||E||_F = noise * ||X_clean||_F.
    """
    rng = np.random.default_rng(seed)
    G0 = rng.standard_normal((R,) * N)
    Qs = [np.linalg.qr(rng.standard_normal((I, R)))[0] for _ in range(N)]
    X = G0
    for n, Q in enumerate(Qs):
        X = np.moveaxis(np.tensordot(Q, X, axes=([1], [n])), 0, n)
    E = rng.standard_normal(X.shape)
    E *= noise * np.linalg.norm(X) / np.linalg.norm(E)
    X = (X + E).astype(np.float32)
    G_init = rng.standard_normal((R,) * N)
    A_init = [rng.standard_normal((I, R)) for _ in range(N)]
    eps = 0.1
    return dict(name="tucker_tensor %d^%d rank %d^%d" % (I, N, R, N), X=X, G0=G0, Qs=Qs,
                G_init=G_init, A_init=A_init, lam=1e-3, eps=eps,
                m_core=m_rule(R**N, eps), m_factor=m_rule(R ** (N - 1), eps), sweeps=10,
                seed=0)


# The paper's Tucker experiments (its appendix on low-rank Tucker decomposition
# of image tensors) use three real image tensors that are not available here;
# planted synthetic tensors of the same shapes and multilinear ranks stand in.
TUCKER_PAPER_SHAPES = {
    "mri": ((256, 256, 14, 20), (8, 8, 4, 4)),             # cardiac MRI shape
    "hyperspectral": ((1024, 1344, 33), (16, 16, 4)),      # hyperspectral shape
    "coil": ((7200, 120, 120, 3), (16, 4, 4, 2)),          # COIL-100 shape
}


def tucker_paper_tensor(name, seed=7, noise=0.5, rank=None):
    """Planted stand-in for one of the paper's image tensors: X = G0 x_n Q_n + E in
    FP32, G0 ~ N(0,1) of the shape's multilinear rank, Q_n orthonormal (QR of
    Gaussian), E Gaussian with ||E||_F = noise * ||X_clean||_F (0.5: a
    reconstruction-error floor near 0.2, the range of the paper's image tensors),
    and the seeded start of ALS (core and factors N(0,1)) for a decomposition of
    multilinear rank `rank` (default: the planted one)."""
    I, R = TUCKER_PAPER_SHAPES[name]
    rng = np.random.default_rng(seed + sum(I))
    G0 = rng.standard_normal(R)
    Qs = [np.linalg.qr(rng.standard_normal((a, r)))[0] for a, r in zip(I, R)]
    X = G0
    for n in range(len(I) - 1, 0, -1):   # small modes first; mode 0 last, as one matrix product
        X = np.moveaxis(np.tensordot(Qs[n], X, axes=([1], [n])), 0, n)
    X = (Qs[0] @ X.reshape(R[0], -1)).astype(np.float32).reshape(I)
    nclean = float(np.linalg.norm(X))
    E = rng.standard_normal(X.shape, dtype=np.float32)
    E *= np.float32(noise * nclean / float(np.linalg.norm(E)))
    X += E
    del E
    Rd = tuple(rank) if rank is not None else R
    rs = np.random.default_rng([seed, *Rd])
    G_init = rs.standard_normal(Rd)
    A_init = [rs.standard_normal((a, r)) for a, r in zip(I, Rd)]
    return dict(name="%s-shaped planted tensor %s rank %s" % (name, "x".join(map(str, I)), ",".join(map(str, R))),
                X=X, G_init=G_init, A_init=A_init, I=I, R=R, rank=Rd, noise=noise)


def tucker_eps_samples(R, eps, alpha=0.001, delta=0.01):
    """The paper's epsilon-sensitivity sample count: Algorithm 2's count for R
    scaled by alpha, ceil(alpha 1680 R ln(40 R) ln(1/delta) / eps)."""
    return int(math.ceil(alpha * 1680 * R * math.log(40 * R) * math.log(1.0 / delta) / eps))


def paper_e1(n, d, seed=0):
    """The paper's synthetic workload: A(1), A(2) n x d with entries N(1, 0.001^2), b = 1."""
    rng = np.random.default_rng(seed)
    As = [1.0 + 0.001 * rng.standard_normal((n, d)) for _ in range(2)]
    return dict(name="paper_e1 n=%d d=%d" % (n, d), As=As, b=np.ones(n * n), lam=1e-3, eps=0.1)


def paper_e1_samples(d, alpha=1e-5, eps=0.1, delta=0.01):
    """The paper's sample count for its synthetic runs: its theory count for
    R = d^2 scaled by alpha, ceil(alpha 1680 R ln(40 R) ln(1/delta) / eps)."""
    R = d * d
    return int(math.ceil(alpha * 1680 * R * math.log(40 * R) * math.log(1.0 / delta) / eps))


def random_problem(I, R, seed=0, sigma=0.01, nrhs=1, heavy=0, scale=100.0):
    """Factors A(n) I_n x R_n i.i.d. N(0,1) (optionally `heavy` rows per mode scaled),
    x_true ~ N(0,1), b = K x_true + sigma e.  With nrhs > 1, b and x_true have
    nrhs columns (row-major: row index major, right-hand side minor)."""
    rng = np.random.default_rng(seed)
    As = []
    for In, Rn in zip(I, R):
        A = rng.standard_normal((In, Rn))
        if heavy:
            A[rng.choice(In, size=min(heavy, In), replace=False)] *= scale
        As.append(A)
    Rtot = int(np.prod(R))
    Itot = int(np.prod(I))
    x_true = rng.standard_normal((Rtot, nrhs))
    b = np.stack([_design_apply(As, x_true[:, k]) for k in range(nrhs)], axis=1)
    b += sigma * rng.standard_normal(b.shape)
    if nrhs == 1:
        x_true, b = x_true[:, 0], b[:, 0]
    assert b.shape[0] == Itot
    return dict(name="random I=%s R=%s" % (list(I), list(R)), As=As, b=b, x_true=x_true)


def batched_ridge_specs(seed=5, count=256, I_range=(32, 256), R_range=(4, 16), N_range=(2, 4), rhs_range=(1, 8)):
    """Shapes and parameters of the batched ridge workload (no arrays): one dict per
    problem with N, I, R, nrhs, lam, a factor seed, and the response's Philox key
    (b = K X_true + 0.01 e with e drawn by row, since prod(I) x nrhs entries would
    not fit in memory for N = 4).  m = ceil(R ln R / eps) per problem."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.integers(N_range[0], N_range[1] + 1))
        I = tuple(int(v) for v in rng.integers(I_range[0], I_range[1] + 1, size=N))
        R = tuple(int(v) for v in rng.integers(R_range[0], R_range[1] + 1, size=N))
        nrhs = int(rng.integers(rhs_range[0], rhs_range[1] + 1))
        lam = float(10.0 ** rng.uniform(-4.0, 0.0))
        out.append(dict(N=N, I=I, R=R, nrhs=nrhs, lam=lam, data_seed=int(seed) * 100000 + i, sigma=0.01,
                        noise_key=(int(seed), i)))
    return out


def batched_ridge_arrays(spec):
    """Factors (FP32, N(0,1)) and X_true (N(0,1)) of one batched_ridge problem."""
    rng = np.random.default_rng(spec["data_seed"])
    As = [rng.standard_normal((In, Rn)).astype(np.float32) for In, Rn in zip(spec["I"], spec["R"])]
    X = rng.standard_normal((int(np.prod(spec["R"])), spec["nrhs"]))
    return As, X
