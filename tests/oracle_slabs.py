"""Whole-lattice evaluation of the oracle's operator on large lattices.

The oracle is plain single-threaded NumPy; at 32^4 and 64x32^3 one clover
build takes minutes.  Here the lattice is cut into slabs along direction 0,
each slab padded with two periodic halo rows on both sides (hops reach one
site, the clover leaves one site in every direction), and the oracle runs
unchanged on every padded slab in its own process; the interior rows of each
slab are exactly the full-lattice result.  Nothing of the oracle's
arithmetic changes: it is evaluated piecewise.  Worker processes are started
fresh (spawn) and import only NumPy and the oracle.
"""
import multiprocessing as mp
import os

import numpy as np

HALO = 2


def _pad(a, t0, t1):
    n0 = a.shape[0]
    return np.take(a, np.arange(t0 - HALO, t1 + HALO) % n0, axis=0)


def _bounds(n0, nslab):
    nslab = max(1, min(nslab, n0))
    return [(n0 * i // nslab, n0 * (i + 1) // nslab) for i in range(nslab)]


def _residual_part(args):
    from oracle import clover, dirac
    Us, xs, bs, m0, csw, tau = args
    Cs = clover.clover_term(Us, csw) if csw else None
    n = bs.shape[1] if bs.ndim == 7 else bs.shape[0]
    out = []
    for k in range(xs.shape[0]):
        q = dirac.apply_Q_shifted(Us, xs[k], m0, tau[k], Cs)[HALO:HALO + n]
        out.append((float(np.sum(np.abs(bs[k] - q) ** 2)), float(np.sum(np.abs(bs[k]) ** 2))))
    return out


def _clover_part(args):
    from oracle import clover
    Us, csw, n = args
    return clover.clover_term(Us, csw)[HALO:HALO + n]


def default_procs():
    return max(1, min(16, os.cpu_count() or 1))


def full_residuals(U, xs, bs, m0, csw, taus, procs=None, nslab=None):
    """||b_k - (Q - tau_k) x_k|| / ||b_k|| for fields xs[k], bs[k] (canonical
    complex128 [N0, N1, N2, N3, 4, 3]) with the oracle's operator on the whole
    lattice."""
    procs = procs or default_procs()
    n0 = U.shape[0]
    jobs = []
    for t0, t1 in _bounds(n0, nslab or max(procs, 4)):
        jobs.append((_pad(U, t0, t1), np.stack([_pad(x, t0, t1) for x in xs]),
                     np.stack([b[t0:t1] for b in bs]), m0, csw, list(taus)))
    with mp.get_context("spawn").Pool(min(procs, len(jobs))) as pool:
        parts = pool.map(_residual_part, jobs)
    r2 = np.sum([[p[k][0] for k in range(len(xs))] for p in parts], axis=0)
    b2 = np.sum([[p[k][1] for k in range(len(xs))] for p in parts], axis=0)
    return list(np.sqrt(r2 / b2))


def full_clover(U, csw, procs=None, nslab=None):
    """The oracle's clover term C(x) on the whole lattice."""
    procs = procs or default_procs()
    jobs = [(_pad(U, t0, t1), csw, t1 - t0) for t0, t1 in _bounds(U.shape[0], nslab or max(procs, 4))]
    with mp.get_context("spawn").Pool(min(procs, len(jobs))) as pool:
        parts = pool.map(_clover_part, jobs)
    return np.concatenate(parts, axis=0)
