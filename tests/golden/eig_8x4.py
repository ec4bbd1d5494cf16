"""Reference eigenvalues for the GPU eigensolver on 8^4: the 60 eigenvalues of
smallest |lambda| of the oracle's Q (links exp(0.5 i H) with the config-10 seed,
m0 = -0.5, c_sw = 1), by the oracle's Lanczos route (oracle.eigen.
smallest_eigenpairs_sparse, pinned against the dense definition on 4^4).
Writes eig_8x4.json next to this file.  Uses only the oracle and the seeded
input generator.

    python tests/golden/eig_8x4.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import clover, dirac, eigen  # noqa: E402
from synth import random_links, seed_for  # noqa: E402


def main():
    dims, m0, csw, k = (8, 8, 8, 8), -0.5, 1.0, 60
    U = random_links(dims, 0.5, seed_for(10, "U"))
    C = clover.clover_term(U, csw)
    t = time.time()
    lam, X = eigen.smallest_eigenpairs_sparse(U, m0, C, k)
    res = [float(np.linalg.norm(dirac.apply_Q(U, X[i], m0, C) - lam[i] * X[i])) for i in range(k)]
    out = {"_about": "60 eigenvalues of Q of smallest |lambda| on 8^4, links exp(0.5 i H) seed config 10, "
                     "m0 = -0.5, c_sw = 1; written by tests/golden/eig_8x4.py (oracle only)",
           "dims": list(dims), "m0": m0, "csw": csw, "eps": 0.5, "seed_config": 10,
           "lambda": [float(v) for v in lam], "max_residual": max(res), "seconds": time.time() - t}
    with open(os.path.join(HERE, "eig_8x4.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("done in %.0f s, max residual %.2e" % (out["seconds"], out["max_residual"]))


if __name__ == "__main__":
    main()
