"""GPU parity of the full TuckerALS path (Algorithm 1) at the shapes of the paper's
Tucker experiments, on planted synthetic tensors (the paper's image tensors are
not available): 256x256x14x20 rank (8,8,4,4) and (4,4,2,2), 1024x1344x33 rank
(16,16,4), 7200x120x120x3 rank (16,4,4,2); FP32 tensors, lambda = 0 as in the
paper's experiments.

  - the exact factor update (tucker_factor_exact) against the oracle's on small
    tensors (N = 3, 4; FP64 and FP32 tensors; lambda = 0 and > 0): rel-L2 1e-10;
  - exact ALS at every paper shape: the relative reconstruction error after each
    of 5 sweeps against the oracle's exact-ALS trajectory on the same tensor
    (tests/golden/tucker_paper_als.txt, written by make_tucker_paper_als.py from
    the oracle only): relative difference <= 1e-8;
  - the paper's protocol (exact factor updates, core by Algorithm 2 with m
    samples): the core update's sketch bit-exact with the oracle sampler and its
    solution the oracle's direct sketched minimiser (rel-L2 1e-10) on the
    256x256x14x20 tensor.
"""

import os

import numpy as np
import pytest

import workloads
from oracle.kron import vec
from oracle.regression import kron_rows, solve_sketched_direct
from oracle.tucker import exact_factor_update
from parity import check_quantised_tables, check_sketch, rel_l2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tucker_paper_als.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, rank, sweep, v = line.split()
        out.setdefault((name, rank), []).append(float(v))
    return out


@pytest.mark.parametrize("I,R,lam,f32", [((9, 8, 7), (3, 2, 4), 0.0, False), ((9, 8, 7), (3, 2, 4), 0.1, True),
                                         ((8, 7, 6, 5), (2, 3, 2, 2), 0.0, True), ((8, 7, 6, 5), (3, 2, 2, 3), 0.3, False)])
def test_exact_factor_update(gpu_lib, I, R, lam, f32):
    import torch
    print("case exact factor update", I, R, lam, f32, flush=True)
    rng = np.random.default_rng(sum(I) + len(R))
    X = rng.standard_normal(I)
    if f32:
        X = X.astype(np.float32)
    G = rng.standard_normal(R)
    As = [rng.standard_normal((a, r)) for a, r in zip(I, R)]
    tX = torch.tensor(X, device="cuda")
    tG = torch.tensor(G, device="cuda")
    tA = [torch.tensor(A, device="cuda") for A in As]
    for n in range(len(I)):
        An = gpu_lib.tucker_factor_exact(tX, tA, tG, n, lam).cpu().numpy()
        ref = exact_factor_update(X.astype(np.float64), As, G, n, lam)
        assert rel_l2(An, ref) <= 1e-10, (n, rel_l2(An, ref))


RUNS = [("mri", None), ("mri", (4, 4, 2, 2)), ("hyperspectral", None), ("coil", None)]


@pytest.mark.parametrize("name,rank", RUNS, ids=["mri", "mri-4422", "hyperspectral", "coil"])
def test_exact_als_trajectory(gpu_lib, name, rank):
    import torch
    w = workloads.tucker_paper_tensor(name, rank=rank)
    key = (name, ",".join(map(str, w["rank"])))
    print("case exact ALS", w["name"], "rank", key[1], flush=True)
    ref = _golden()[key]
    X = torch.from_numpy(w["X"]).cuda()
    del w["X"]
    G0 = torch.tensor(w["G_init"], device="cuda")
    A0 = [torch.tensor(A, device="cuda") for A in w["A_init"]]
    G, As, trace = gpu_lib.tucker_als(X, G0, A0, 0.0, len(ref), factor_update="exact", core_update="exact")
    print("rre", ["%.6f" % v for v in trace], "oracle", ["%.6f" % v for v in ref], flush=True)
    for a, b in zip(trace, ref):
        assert abs(a - b) <= 1e-8 * b, (trace, ref)


def test_sketched_core_step_at_paper_shape(gpu_lib):
    """One sweep of the paper's protocol on the 256x256x14x20 tensor: exact factor
    updates, then the core by Algorithm 2 with m = 4096 samples (lambda = 0)."""
    import torch
    w = workloads.tucker_paper_tensor("mri")
    print("case sketched core update", w["name"], flush=True)
    Xn = w["X"]
    X = torch.from_numpy(Xn).cuda()
    G = torch.tensor(w["G_init"], device="cuda")
    As = [torch.tensor(A, device="cuda") for A in w["A_init"]]
    for n in range(4):
        As[n] = gpu_lib.tucker_factor_exact(X, As, G, n, 0.0)
    m = 4096
    g, info = gpu_lib.kron_ridge(As, X.reshape(-1), 0.0, eps=0.1, m=m, seed=0, stream=gpu_lib.als_stream(0, 4),
                                 tol=1e-13, max_iter=400)
    assert info["status"] == "OK", info
    Ah = [A.cpu().numpy() for A in As]
    I = list(Xn.shape)
    sk = gpu_lib.export_sketch(I)
    check_quantised_tables(Ah, sk["Q"])
    rows, ridx, counts, Omega = check_sketch(Ah, sk, m, seed=0, stream=gpu_lib.als_stream(0, 4))
    b = vec(Xn.astype(np.float64))
    xo = solve_sketched_direct(kron_rows(Ah, ridx), Omega, b[rows], 0.0)
    err = rel_l2(g.cpu().numpy(), xo)
    print("D=%d iters %d rel-L2 vs direct %.2e" % (len(rows), info["iters"], err), flush=True)
    assert err <= 1e-10
