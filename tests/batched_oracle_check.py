"""Oracle side of the full-size batched parity test, run as its own process.

The GPU test writes, per problem of the batched ridge workload, the library's
solution x and its quantised tables Q to an .npz file and starts this module as a
child process (which never touches the GPU).  Here a pool of worker processes
redoes every problem with the oracle only:

  - samples drawn by the oracle sampler from the given tables (Philox stream =
    problem index) and merged: digests (SHA-256) of the distinct rows, the
    multiplicities and the merged weights, which the parent compares with the
    digests of the GPU's exported sketch (bit-exact comparison);
  - b~ at the sampled rows: K X_true through the oracle's split products plus
    sigma E from its own Philox Box-Muller;
  - the gradient of the sketched objective at the GPU's x through the split
    products, and ||M^+ g|| / ||x|| with M = K^T K + lambda I (the oracle's
    eigen-decomposition preconditioner);
  - where the explicit sampled block D x R has at most DIRECT_MAX entries, the
    oracle's direct QR minimiser and rel-L2(x, x~).

Usage: python -m tests.batched_oracle_check IN.npz OUT.json [workers]
"""

import hashlib
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DIRECT_MAX = 4_000_000


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def sketch_digests(rows2d, counts, Omega):
    """Digests of a sketch in the exported dtypes (int32 rows, int32 counts, float64 weights)."""
    return {"rows": digest(np.asarray(rows2d, dtype=np.int32)), "counts": digest(np.asarray(counts, dtype=np.int32)),
            "Omega": digest(np.asarray(Omega, dtype=np.float64))}


def check_problem(args):
    i, spec, Q, x = args
    import workloads
    from oracle.regression import (KronPreconditioner, kron_rows, sampled_forward_split, sketched_gradient_split,
                                   solve_sketched_direct, split_point)
    from oracle.response import noise
    from oracle.sampling import merge, sample_product
    As32, X = workloads.batched_ridge_arrays(spec)
    As = [A.astype(np.float64) for A in As32]
    I = list(spec["I"])
    R = int(np.prod(spec["R"]))
    m = workloads.m_rule(R, 0.1)
    idx, omega = sample_product(Q, m, 0, i)
    rows, ridx, counts, Omega = merge(idx, omega, I)
    del idx, omega
    out = {"problem": i, "D": int(len(rows)), "m": int(m), "digests": sketch_digests(ridx, counts, Omega)}
    t = split_point(As, ridx)
    nrhs = spec["nrhs"]
    bD = sampled_forward_split(As, ridx, X, t) + spec["sigma"] * noise(rows, nrhs, *spec["noise_key"])
    xg = np.asarray(x, dtype=np.float64).reshape(R, nrhs)
    g = sketched_gradient_split(As, ridx, Omega, bD, xg, spec["lam"], t)
    d = KronPreconditioner(As, spec["lam"]).apply(g)
    out["precond_residual"] = float(np.linalg.norm(d) / np.linalg.norm(xg))
    if len(rows) * R <= DIRECT_MAX:
        xo = solve_sketched_direct(kron_rows(As, ridx), Omega, bD, spec["lam"])
        out["direct_rel_l2"] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    return out


def main(argv):
    src, dst = argv[0], argv[1]
    workers = int(argv[2]) if len(argv) > 2 else min(16, os.cpu_count() or 1)
    import workloads
    specs = workloads.batched_ridge_specs()
    data = np.load(src, allow_pickle=False)
    jobs = []
    for i, sp in enumerate(specs):
        Q = [data["Q_%d_%d" % (i, n)] for n in range(sp["N"])]
        jobs.append((i, sp, Q, data["x_%d" % i]))
    # largest problems first, so the pool's tail is short
    jobs.sort(key=lambda j: -int(np.prod(j[1]["R"])))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(check_problem, jobs))
    res.sort(key=lambda r: r["problem"])
    with open(dst, "w") as f:
        json.dump(res, f)


if __name__ == "__main__":
    main(sys.argv[1:])
