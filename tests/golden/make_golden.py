"""Write the stored expected values under tests/golden/ (calls only the oracle).

Run from the repository root:  python tests/golden/make_golden.py
The values are the FP64 oracle's (Tier B: implicit Householder nullspace and
ARPACK, FairSC variant 1) on seeded synthetic workloads that are too large to
re-solve on the CPU inside a GPU test.
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from sfairsc_inputs import workload  # noqa: E402


def write(name, header, rows):
    with open(os.path.join(HERE, name), "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for key, vals in rows:
            f.write(f"{key}: " + " ".join(repr(float(v)) for v in vals) + "\n")


def main():
    # n = 50,000 normalized workload, 12 smallest fair eigenvalues
    name = "msbm-50k-h5-normalized"
    g = workload(name)
    t = time.time()
    lam, H = oracle.fair_eigs_implicit(g.to_scipy(), g.groups, g.h, 12, True, tol=1e-14)
    res = oracle.residual_norms(g.to_scipy(), g.groups, g.h, True, lam, H)
    write(
        "msbm50k_normalized_eigs.txt",
        [
            f"Oracle (Tier B, FP64) eigenvalues of the {name} workload: the 12 smallest",
            "eigenvalues of V^T L_n V (FairSC variant 1, eq. lveig), V an orthonormal basis of null(C^T),",
            "C = D^{-1/2} F.  Written by tests/golden/make_golden.py (oracle only).",
            f"max residual {res.max():.3e}, {time.time() - t:.1f} s",
        ],
        [("eigenvalues", lam)],
    )


if __name__ == "__main__":
    main()
