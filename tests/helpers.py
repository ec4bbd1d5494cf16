"""Shared test utilities: oracle evaluation at sampled sites, error norms."""
import os

import numpy as np

from oracle import clover as oclover
from oracle import dirac


def rel_err(a, b):
    """max |a - b| / max |b|; the value is also printed with the running test's
    name (visible with pytest -s), so the measured errors can be tabulated."""
    a = np.asarray(a)
    b = np.asarray(b)
    v = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    print("[rel_err] %s %.3e" % (os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0], v), flush=True)
    return v


def window(dims, x, radius=2):
    """Index arrays of the (2r+1)^4 periodic window centred at site x."""
    return np.ix_(*[(x[mu] + np.arange(-radius, radius + 1)) % dims[mu] for mu in range(4)])


def oracle_at_sites(U, psi, m0, csw, sites, tau=0.0, mode="Q"):
    """The oracle operator evaluated at individual sites of a large lattice.

    The oracle runs on a periodic 5^4 window around each site: hops reach
    distance 1 and clover leaves distance 2, so the window centre is exact.
    mode: "Q" -> (Q - tau) psi, "A" -> (D - tau Gamma5) psi.
    """
    dims = U.shape[:4]
    out = []
    for x in sites:
        idx = window(dims, x)
        Uw = U[idx]
        pw = psi[idx]
        Cw = oclover.clover_term(Uw, csw) if csw else None
        if mode == "Q":
            r = dirac.apply_Q_shifted(Uw, pw, m0, tau, Cw)
        else:
            r = dirac.apply_A(Uw, pw, m0, tau, Cw)
        out.append(r[2, 2, 2, 2])
    return np.array(out)


def sample_sites(dims, n, seed):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, d)) for d in dims) for _ in range(n)]
