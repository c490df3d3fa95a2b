"""Writes tucker_400_als.txt: the oracle's exact Tucker ALS trajectory on the
400x400x400 tensor of workloads.tucker_tensor (rank-(16,16,16) core times
orthonormal factors plus 1% noise, FP32), the configuration the benchmark runs
with sketched updates.

Algorithm 1 with exact factor and core updates, lambda = 1e-3 (the ridge of the
benchmark's core update), 10 sweeps from the workload's seeded start; one line
per sweep:
    <sweep> <relative reconstruction error>
Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_tucker_400_als.py
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle.tucker import tucker_als  # noqa: E402


def main():
    w = workloads.tucker_tensor()
    G, As, trace = tucker_als(w["X"], w["G_init"], w["A_init"], w["lam"], w["sweeps"])
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tucker_400_als.txt")
    lines = ["# oracle exact Tucker ALS on the 400^3 tucker_tensor workload (lambda = 1e-3), "
             "written by make_tucker_400_als.py", "# sweep rre"]
    lines += ["%d %.15e" % (s + 1, v) for s, v in enumerate(trace)]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(trace, flush=True)


if __name__ == "__main__":
    main()
