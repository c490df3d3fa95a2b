"""Writes tucker_paper_als.txt: the oracle's exact Tucker ALS trajectories on the
planted tensors that stand in for the paper's image tensors (its appendix on
low-rank Tucker decomposition: cardiac MRI 256x256x14x20, hyperspectral
1024x1344x33, COIL-100 7200x120x120x3 shapes).

Algorithm 1 with exact factor and core updates and lambda = 0 (the paper's ALS
baseline runs without regularisation), 5 sweeps from the seeded start of
workloads.tucker_paper_tensor; one line per sweep:
    <shape> <rank> <sweep> <relative reconstruction error>
Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_tucker_paper_als.py
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle.tucker import tucker_als  # noqa: E402

RUNS = [("mri", None), ("mri", (4, 4, 2, 2)), ("hyperspectral", None), ("coil", None)]
SWEEPS = 5


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tucker_paper_als.txt")
    lines = ["# oracle exact Tucker ALS (lambda = 0), written by make_tucker_paper_als.py",
             "# shape rank sweep rre"]
    for name, rank in RUNS:
        w = workloads.tucker_paper_tensor(name, rank=rank)
        G, As, trace = tucker_als(w["X"], w["G_init"], w["A_init"], 0.0, SWEEPS)
        r = ",".join(map(str, w["rank"]))
        for s, v in enumerate(trace):
            lines.append("%s %s %d %.15e" % (name, r, s + 1, v))
        print(name, r, trace, flush=True)
        del w, G, As
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
