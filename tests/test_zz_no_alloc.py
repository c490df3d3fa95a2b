"""The allocation-free entry point kron_ridge_noalloc against kron_ridge, through
the C ABI: two calls in a row (the second on a smaller problem, so stale scratch
contents from the first would show), each compared bit for bit with the
allocating entry point on the same inputs, plus the size limit."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _inputs(w):
    import torch
    return ([torch.tensor(A, device="cuda") for A in w["As"]], torch.tensor(w["b"], device="cuda"))


def _case(gpu_lib, name, w, lam, m, nrhs_cols=None):
    import torch
    print("case no-alloc", name, "m", m, "lam", lam, flush=True)
    tA, tb = _inputs(w)
    R = int(np.prod([A.shape[1] for A in w["As"]]))
    shape = (R,) if tb.dim() == 1 else (R, tb.shape[1])
    x_ref, info_ref = gpu_lib.kron_ridge(tA, tb, lam, eps=0.1, m=m, seed=3, stream=1, tol=1e-13)
    x = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    x, info = gpu_lib.kron_ridge_noalloc(tA, tb, lam, x, eps=0.1, m=m, seed=3, stream=1, tol=1e-13)
    torch.cuda.synchronize()
    # every solver field equal; loss is NaN (not requested) and ms is each call's own clock
    keys = ("iters", "status", "m", "distinct_rows", "rel_update")
    assert {k: info[k] for k in keys} == {k: info_ref[k] for k in keys}, (info, info_ref)
    assert np.isnan(info["loss"]) and np.isnan(info_ref["loss"]) and info["ms"] > 0
    assert torch.equal(x, x_ref), float((x - x_ref).abs().max())
    return info


def test_noalloc_matches_kron_ridge_twice(gpu_lib):
    # first call: the small Kronecker regression workload (N = 2, 64 x 8 factors)
    w = workloads.small_regression()
    i1 = _case(gpu_lib, "small_regression", w, 0.0, w["m"])
    # second call: a smaller ridge problem with N = 3 and two right-hand sides
    w2 = workloads.random_problem((9, 7, 5), (2, 3, 2), seed=8, nrhs=2)
    i2 = _case(gpu_lib, "smaller N=3 nrhs=2 ridge", w2, 0.02, 300)
    assert i2["distinct_rows"] < i1["distinct_rows"]


def test_noalloc_rejects_problems_beyond_its_scratch(gpu_lib):
    import torch
    cap = gpu_lib.noalloc_capacity()
    assert cap == 64 << 20
    # m = 2^23 samples need 2 x 8 x 2^23 bytes of sort keys alone (128 MiB): the
    # size check fails on the host before anything is enqueued
    w = workloads.random_problem((40, 30), (3, 2), seed=2)
    tA, tb = _inputs(w)
    x = torch.empty(6, dtype=torch.float64, device="cuda")
    print("case no-alloc size limit", flush=True)
    with pytest.raises(gpu_lib.KronRegressError) as e:
        gpu_lib.kron_ridge_noalloc(tA, tb, 0.0, x, m=1 << 23)
    assert e.value.status == -6
    assert "scratch" in str(e.value)
