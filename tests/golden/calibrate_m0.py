"""Pick a near-critical bare mass m0 for the 64x32^3 clover workload (c_sw = 1,
links exp(0.5 i H)): smallest |eigenvalue| of the oracle's Q on an 8^4 lattice
of the same link distribution, by Lanczos on Q^2 (scipy eigsh), over a grid of
m0.  Writes m0_critical.json next to this file.  Uses only the oracle and the
seeded input generator.

    OMP_NUM_THREADS=2 python tests/golden/calibrate_m0.py
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import clover, dense  # noqa: E402
from synth import random_links, seed_for  # noqa: E402


def lambda_min(U, C, m0):
    Q = dense.sparse_Q(U, m0, C)
    Q2 = sla.LinearOperator(Q.shape, matvec=lambda v: Q @ (Q @ v), dtype=np.complex128)
    w = sla.eigsh(Q2, k=1, which="SA", ncv=64, tol=1e-3, maxiter=20000, return_eigenvectors=False)
    return float(np.sqrt(abs(w[0])))


def main():
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.5, seed_for(5, "U"))
    C = clover.clover_term(U, 1.0)
    grid = [-0.8, -0.9, -0.95, -0.97, -1.0, -1.1]
    rows = []
    for m0 in grid:
        t = time.time()
        lm = lambda_min(U, C, m0)
        rows.append([m0, lm])
        print("m0 %.3f  lambda_min(|Q|) %.5f  (%.0f s)" % (m0, lm, time.time() - t), flush=True)
    target = 0.02
    heavy = [r for r in rows if r[0] > -1.0]     # stay on the heavy side of the minimum
    pick = min(heavy, key=lambda r: abs(r[1] - target))
    out = {"_about": "smallest |eigenvalue| of Q on 8^4, links exp(0.5 i H) seed config 5, c_sw = 1; "
                     "written by tests/golden/calibrate_m0.py (oracle only)",
           "dims": list(dims), "csw": 1.0, "eps": 0.5, "grid": rows, "target": target, "m0": pick[0],
           "lambda_min": pick[1]}
    with open(os.path.join(HERE, "m0_critical.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("chose m0 = %.3f" % pick[0])


if __name__ == "__main__":
    main()
