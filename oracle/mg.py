"""Two-level aggregation multigrid pieces: P, R = P^H, D_c = P^H D P, V-cycle.

eq. (2.8): E_2g = (I - M A)^nu (I - P A_c^{-1} R A)(I - M A)^mu with R = P^H and
the Galerkin coarse operator D_c = P^H D P; P is block diagonal with one block
per aggregate, built from test vectors W (Sec. 3.1, local-coherence paragraph
and the figure on the construction of P).  Spin structure is kept
(Gamma5 P = P Gamma5^c, text before eq. (2.9)) by splitting every lattice block into two
aggregates: spins {0,1} (gamma5 = +1) and spins {2,3} (gamma5 = -1).

Readings where the paper is silent:
* orthonormalisation of each aggregate's columns: modified Gram-Schmidt in
  column order, run twice per column, then normalisation; a column whose norm
  falls below 1e-12 of its original norm is rejected as rank deficient;
* coarse component order per coarse site: [chirality +: j = 0..ntv-1,
  chirality -: j = 0..ntv-1], so Gamma5^c = diag(+I, -I);
* D_c is stored as the self block and the 8 neighbour blocks (+mu, -mu kept
  apart even when they are the same block);
* the V-cycle does no pre-smoothing (mu = 0): z = P y with y an approximate
  solution of A_c(tau) y = P^H r, then nu SAP sweeps on A_tau z = r from z.
  With P^H P = I, P^H (D - tau Gamma5) P = D_c - tau Gamma5^c.
"""
import numpy as np

from . import blocks as bl
from .dirac import gamma5, hop_backward, hop_forward
from .krylov import gmres
from .sap import block_operator, sap


def to_aggregates(psi, block):
    """Field [N0..N3, 4, 3] -> [nb, 2, bs*6], index (local site, spin in half, colour)."""
    dims = psi.shape[:4]
    nb = bl.nblocks(dims, block)
    shp = []
    for n, b in zip(nb, block):
        shp += [n, b]
    g = psi.reshape(tuple(shp) + (4, 3))
    g = g.transpose(0, 2, 4, 6, 1, 3, 5, 7, 8, 9)
    nbt = int(np.prod(nb))
    bs = int(np.prod(block))
    g = g.reshape(nbt, bs, 2, 2, 3).transpose(0, 2, 1, 3, 4)
    return g.reshape(nbt, 2, bs * 6)


def from_aggregates(a, dims, block):
    nb = bl.nblocks(dims, block)
    bs = int(np.prod(block))
    g = a.reshape(-1, 2, bs, 2, 3).transpose(0, 2, 1, 3, 4)
    g = g.reshape(tuple(nb) + tuple(block) + (4, 3))
    g = g.transpose(0, 4, 1, 5, 2, 6, 3, 7, 8, 9)
    return g.reshape(tuple(dims) + (4, 3))


def build_P(W, block):
    """P[nb, 2, bs*6, ntv]: per aggregate, the ntv test vectors orthonormalised."""
    cols = [to_aggregates(w, block) for w in W]
    ntv = len(cols)
    P = np.zeros(cols[0].shape + (ntv,), dtype=np.complex128)
    for j in range(ntv):
        v = cols[j].copy()
        n0 = np.linalg.norm(v, axis=-1)
        for _ in range(2):
            for i in range(j):
                p = P[..., i]
                v = v - np.sum(np.conj(p) * v, axis=-1)[..., None] * p
        n1 = np.linalg.norm(v, axis=-1)
        if np.any(n1 < 1e-12 * n0):
            raise np.linalg.LinAlgError("test vectors are locally rank deficient")
        P[..., j] = v / n1[..., None]
    return P


def restrict(P, psi, block):
    """y = P^H psi as coarse vector [nb, 2*ntv]."""
    a = to_aggregates(psi, block)
    y = np.einsum("bhkj,bhk->bhj", np.conj(P), a)
    return y.reshape(y.shape[0], -1)


def prolong(P, y, dims, block):
    """psi = P y for a coarse vector [nb, 2*ntv]."""
    ntv = P.shape[-1]
    yy = y.reshape(y.shape[0], 2, ntv)
    a = np.einsum("bhkj,bhj->bhk", P, yy)
    return from_aggregates(a, dims, block)


def local_coherence(P, psi, block):
    """lc(v) = ||Pi v|| / ||v|| with Pi = P P^H the orthogonal projection on the
    range of P (Sec. 3.1, local coherence measure); P's columns are
    orthonormal per aggregate, so Pi v = prolong(restrict(v))."""
    dims = psi.shape[:4]
    return np.linalg.norm(prolong(P, restrict(P, psi, block), dims, block)) / np.linalg.norm(psi)


def gamma5_coarse(y):
    ntv = y.shape[-1] // 2
    s = np.concatenate([np.ones(ntv), -np.ones(ntv)])
    return y * s


def coarse_operator(op, P, block):
    """Dc[nb, 9, 2 ntv, 2 ntv]: blocks of P^H D P (0 self, 1+2mu: +mu, 2+2mu: -mu)."""
    dims = op.dims
    nbt, _, _, ntv = P.shape
    nc = 2 * ntv
    Dc = np.zeros((nbt, 9, nc, nc), dtype=np.complex128)
    for c in range(nc):
        y = np.zeros((nbt, nc), dtype=np.complex128)
        y[:, c] = 1.0
        p = prolong(P, y, dims, block)
        Dc[:, 0, :, c] = restrict(P, block_operator(op, p, 0.0, block), block)
        for mu in range(4):
            leave_f = (~bl.inner_forward(dims, block, mu))[..., None, None]
            leave_b = (~bl.inner_backward(dims, block, mu))[..., None, None]
            Dc[:, 1 + 2 * mu, :, c] = restrict(P, leave_f * hop_forward(op.U, p, mu), block)
            Dc[:, 2 + 2 * mu, :, c] = restrict(P, leave_b * hop_backward(op.U, p, mu), block)
    return Dc


class Coarse:
    """Coarse operator A_c(tau) = D_c - tau Gamma5^c on the block lattice."""

    def __init__(self, Dc, nbr):
        self.Dc = Dc
        self.nbr = nbr

    def apply(self, y, tau, qform=False):
        """A_c(tau) y; with qform Gamma5^c A_c(tau) y = (Gamma5^c D_c - tau) y, the
        Galerkin projection P^H (Q - tau) P (Gamma5 P = P Gamma5^c)."""
        out = np.einsum("bij,bj->bi", self.Dc[:, 0], y)
        for d in range(1, 9):
            out = out + np.einsum("bij,bj->bi", self.Dc[:, d], y[self.nbr[:, d]])
        out = out - tau * gamma5_coarse(y)
        return gamma5_coarse(out) if qform else out


class TwoLevel:
    """The multigrid hierarchy (fine operator, P, coarse operator)."""

    def __init__(self, op, W, block):
        self.op = op
        self.block = tuple(block)
        bl.check_blocking(op.dims, block)
        self.P = build_P(W, block)
        self.coarse = Coarse(coarse_operator(op, self.P, block),
                             bl.neighbour_table(op.dims, block))

    def vcycle(self, r, tau, nu, n_mr, coarse_iters, coarse_tol=None, qform=False, smoother="sap"):
        """z = nu SAP sweeps on A_tau z = r started from P A_c^{-1}(approx) P^H r
        (qform: the same cycle for Q - tau, coarse operator Gamma5^c A_c).
        smoother="gmres" (Sec. 2's alternative to SAP): instead of the sweeps,
        nu steps of GMRES from zero on A e = r - A z, then z + e."""
        rc = restrict(self.P, r, self.block)
        yc = gmres(lambda v: self.coarse.apply(v, tau, qform), rc, coarse_iters, coarse_tol)[0]
        z = prolong(self.P, yc, self.op.dims, self.block)
        return self.post_smooth(r, z, tau, nu, n_mr, qform, smoother)

    def post_smooth(self, r, z, tau, nu, n_mr, qform=False, smoother="sap"):
        """nu post-smoothing steps on A_tau z = r from z (SAP sweeps, or GMRES
        steps on the residual equation)."""
        if nu > 0 and smoother == "gmres":
            def A(v):
                av = self.op.A(v, tau)
                return gamma5(av) if qform else av
            z = z + gmres(A, r - A(z), nu, None)[0]
        elif nu > 0:
            z = sap(self.op, r, z, tau, self.block, nu, n_mr, qform)
        return z


def setup_test_vectors(op, W0, block, setup_iters=6, smooth=4, n_mr=3,
                       coarse_iters=20, coarse_tol=0.5):
    """Adaptive-setup reading: smooth W0 on A_0 w = 0, then V-cycle inverse iterations."""
    zero = np.zeros_like(W0[0])
    W = [sap(op, zero, w, 0.0, block, smooth, n_mr) for w in W0]
    W = [w / np.linalg.norm(w) for w in W]
    for _ in range(setup_iters - 1):
        mg = TwoLevel(op, W, block)
        W = [mg.vcycle(w, 0.0, smooth, n_mr, coarse_iters, coarse_tol) for w in W]
        W = [w / np.linalg.norm(w) for w in W]
    return W
