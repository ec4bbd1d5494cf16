"""Red-black Schwarz alternating procedure (SAP) with minimal-residual block solves.

eq. (2.10): one SAP step multiplies the block corrections
I - I_i A_i^{-1} I_i^H A over all blocks i, A_i = I_i^H A I_i the restriction
of the operator to block i (hops that leave the block are dropped); blocks of
one colour are independent and are treated together.  The operator here is
the Gamma5-preconditioned A_tau = D - tau Gamma5 of eq. (3.7).

Readings where the paper leaves the details open:
* block solves are n_mr steps of the minimal-residual method (GMRES(1))
  started from zero, with no tolerance: e = 0, rho = r; repeat
  q = A_i rho, alpha = (q^H rho)/(q^H q), e += alpha rho, rho -= alpha q;
  alpha = 0 when q = 0;
* colour 0 blocks first, then colour 1, in each sweep; the residual
  r = f - A_tau x is recomputed before each colour.

With ``qform`` the same procedure runs on Q - tau = Gamma5 A_tau itself (the
variant without Gamma5 preconditioning that Sec. 3.3 compares against): block
operator Gamma5 A_i, residual f - (Q - tau) x.
"""
import numpy as np

from . import blocks as bl
from .dirac import gamma5, hop_backward, hop_forward, site_diag


def block_operator(op, psi, tau, block, qform=False):
    """A_tau restricted to every block (Dirichlet: hops leaving a block dropped);
    with qform Gamma5 A_tau = Q - tau restricted to the blocks."""
    dims = op.dims
    out = site_diag(psi, op.m0, op.clover) - tau * gamma5(psi)
    for mu in range(4):
        mf = bl.inner_forward(dims, block, mu)[..., None, None]
        mb = bl.inner_backward(dims, block, mu)[..., None, None]
        out = out + mf * hop_forward(op.U, psi, mu) + mb * hop_backward(op.U, psi, mu)
    return gamma5(out) if qform else out


def block_mr(op, r, tau, block, n_mr, qform=False):
    """n_mr minimal-residual steps on every block at once, from e = 0."""
    dims = op.dims
    e = np.zeros_like(r)
    rho = r.copy()
    for _ in range(n_mr):
        q = block_operator(op, rho, tau, block, qform)
        num = bl.block_reduce(np.sum(np.conj(q) * rho, axis=(-2, -1)), dims, block)
        den = bl.block_reduce(np.sum(np.abs(q) ** 2, axis=(-2, -1)), dims, block)
        alpha = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        a = bl.block_expand(alpha, block)[..., None, None]
        e = e + a * rho
        rho = rho - a * q
    return e


def sap(op, f, x, tau, block, nsweep, n_mr, qform=False):
    """nsweep red-black SAP sweeps on A_tau x = f (qform: (Q - tau) x = f) from x."""
    bl.check_blocking(op.dims, block)
    colour = bl.site_colour(op.dims, block)
    x = x.copy()
    for _ in range(nsweep):
        for c in (0, 1):
            m = (colour == c)[..., None, None]
            ax = op.A(x, tau)
            r = (f - (gamma5(ax) if qform else ax)) * m
            x = x + block_mr(op, r, tau, block, n_mr, qform) * m
    return x


def sap_exact(op, f, x, tau, block, nsweep, qform=False):
    """SAP with exact block solves (dense block inverses); small lattices only."""
    bl.check_blocking(op.dims, block)
    dims = op.dims
    colour = bl.site_colour(op.dims, block)
    nb = bl.nblocks(dims, block)
    x = x.copy()
    # site lists per block
    xs = bl.coords(dims)
    bid = np.ravel_multi_index([xs[mu] // block[mu] for mu in range(4)], nb)
    flat_sites = [np.nonzero(bid.reshape(-1) == b)[0] for b in range(int(np.prod(nb)))]
    V = int(np.prod(dims))
    # dense A_tau columns (block-restricted) built by applying the operator
    for _ in range(nsweep):
        for c in (0, 1):
            ax = op.A(x, tau)
            r = f - (gamma5(ax) if qform else ax)
            rf = r.reshape(V, 12)
            xf = x.reshape(V, 12).copy()
            for b, sites in enumerate(flat_sites):
                if colour.reshape(-1)[sites[0]] != c:
                    continue
                n = 12 * len(sites)
                Ai = np.zeros((n, n), dtype=np.complex128)
                for k in range(n):
                    e = np.zeros((V, 12), dtype=np.complex128)
                    e[sites[k // 12], k % 12] = 1.0
                    col = block_operator(op, e.reshape(x.shape), tau, block, qform)
                    Ai[:, k] = col.reshape(V, 12)[sites].reshape(-1)
                xf[sites] += np.linalg.solve(Ai, rf[sites].reshape(-1)).reshape(-1, 12)
            x = xf.reshape(x.shape)
    return x
