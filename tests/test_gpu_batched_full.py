"""GPU parity of the batched ridge workload at its full size: 256 uneven problems
(N ~ U{2,3,4}, I_n ~ U{32..256}, R_n ~ U{4..16}, 1-8 right-hand sides, lambda =
10^U(-4,0), FP32 factors, implicit responses b = K X_true + 0.01 E, m = ceil(R ln R
/ 0.1) per problem), solved by one kron_ridge_batched call (autotuned launch
configuration, as the benchmark times it).

For every problem:
  - the leverage scores equal the oracle's within 1e-13 and the quantised tables
    equal the oracle's (boundary straddles reported);
  - the sketch (distinct rows, multiplicities, merged weights) equals the
    oracle sampler's bit for bit (digests; Philox stream = problem index);
  - the solution: the sketched normal equations through the oracle's split
    products, with the oracle's own b~ at the sampled rows (K X_true plus 0.01 E
    from its Philox Box-Muller), in the preconditioned norm ||M^+ g|| / ||x|| <=
    1e-10 (M = K^T K + lambda I; M^+ H = I + O(eps') for a subspace-embedding
    sketch, so this bounds rel-L2(x, x~) up to 1/(1 - eps')); and where the explicit
    sampled block D x R is small (<= 4e6 entries), rel-L2 <= 1e-10 against the
    oracle's direct QR minimiser.
The oracle side runs in a child process (tests/batched_oracle_check.py) with a
pool of worker processes; it reads only the tables and solutions written here.
"""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads
from batched_oracle_check import sketch_digests
from oracle.leverage import leverage_scores
from parity import check_quantised_tables

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_batched_full_workload(gpu_lib, tmp_path):
    import torch
    specs = workloads.batched_ridge_specs()
    print("case batched ridge full workload: %d problems" % len(specs), flush=True)
    probs, lams = [], []
    for sp in specs:
        As, X = workloads.batched_ridge_arrays(sp)
        tA = [torch.tensor(A, device="cuda") for A in As]
        gen = gpu_lib.ResponseGen(torch.tensor(X, device="cuda"), sp["sigma"], seed=sp["noise_key"][0],
                                  stream=sp["noise_key"][1])
        probs.append((tA, gen))
        lams.append(sp["lam"])
    xs, infos = gpu_lib.kron_ridge_batched(probs, lams, eps=0.1, m_rule="rlnr", seed=0, max_iter=400, autotune=True)
    torch.cuda.synchronize()
    print("GPU batch solved; exporting sketches", flush=True)
    arrays, gpu_digests = {}, []
    straddles, worst_lev = 0, 0.0
    for i, (sp, x, info) in enumerate(zip(specs, xs, infos)):
        assert info["status"] == "OK", (i, info)
        I = list(sp["I"])
        assert info["m"] == workloads.m_rule(int(np.prod(sp["R"])), 0.1)
        As = [A.cpu().numpy().astype(np.float64) for A in probs[i][0]]
        lev = gpu_lib.export_leverage(I, problem=i)
        for n, A in enumerate(As):
            worst_lev = max(worst_lev, float(np.max(np.abs(lev[n] - leverage_scores(A)))))
        sk = gpu_lib.export_batched_sketch(i, I)
        straddles += check_quantised_tables(As, sk["Q"])
        assert int(sk["counts"].sum()) == info["m"] and len(sk["rows"]) == info["distinct_rows"]
        gpu_digests.append(sketch_digests(sk["rows"], sk["counts"], sk["Omega"]))
        for n in range(sp["N"]):
            arrays["Q_%d_%d" % (i, n)] = np.asarray(sk["Q"][n], dtype=np.uint64)
        arrays["x_%d" % i] = x.cpu().numpy()
    print("max |l_gpu - l_oracle| %.2e, quantisation straddles %d" % (worst_lev, straddles), flush=True)
    assert worst_lev <= 1e-13
    src, dst = str(tmp_path / "gpu_results.npz"), str(tmp_path / "oracle.json")
    np.savez(src, **arrays)
    print("oracle check of every problem in a child process", flush=True)
    subprocess.run([sys.executable, os.path.join(ROOT, "tests", "batched_oracle_check.py"), src, dst],
                   check=True, cwd=ROOT, timeout=900)
    res = json.load(open(dst))
    assert len(res) == len(specs)
    worst_pre, worst_direct, ndirect = 0.0, 0.0, 0
    for r, dg, info in zip(res, gpu_digests, infos):
        i = r["problem"]
        assert r["D"] == info["distinct_rows"], (i, r["D"], info)
        assert r["digests"] == dg, (i, "sketch differs from the oracle sampler's")
        worst_pre = max(worst_pre, r["precond_residual"])
        assert r["precond_residual"] <= 1e-10, (i, specs[i], r)
        if "direct_rel_l2" in r:
            ndirect += 1
            worst_direct = max(worst_direct, r["direct_rel_l2"])
            assert r["direct_rel_l2"] <= 1e-10, (i, specs[i], r)
    print("256 problems: sketches bit-exact, max preconditioned residual %.2e, direct checks %d (max rel-L2 %.2e)"
          % (worst_pre, ndirect, worst_direct), flush=True)
