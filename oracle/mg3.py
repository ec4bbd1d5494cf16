"""A third multigrid level: aggregation of the block lattice -- TEST INFRASTRUCTURE.

The paper's solver, DD-alpha-AMG, is a multilevel method; the paper's own
experiments run it with two levels (eq. (2.8), Sec. 4).  This module adds one
more level, built from the first coarse level exactly as that level is built
from the lattice (Sec. 2 on aggregation, Sec. 3.1 on P from test vectors):

* level-2 sites are the lattice blocks (the coarse sites of ``mg``); they are
  grouped into aggregates of B2 = (B2_0, .., B2_3) level-2 sites, numbered
  lexicographically by aggregate coordinate, sites inside an aggregate
  lexicographically as well;
* every aggregate is split by coarse chirality: components 0..ntv-1 of a
  level-2 site have Gamma5^c = +1, ntv..2ntv-1 have -1.  So
  Gamma5^c P2 = P2 Gamma5^cc and the level-3 components are ordered
  [chirality +: j < ntv2, chirality -: j < ntv2] like the level-2 ones;
* the columns of an (aggregate, chirality) are the ntv2 level-2 test vectors
  restricted to it, orthonormalised by modified Gram-Schmidt in column order,
  twice per column (the reading ``mg`` takes for P);
* the level-3 operator is the Galerkin D3 = P2^H D_c P2, stored as the self
  block and the 8 neighbour blocks (+mu and -mu kept apart).

Readings (the paper specifies nothing beyond two levels):

* the level-2 correction inside the level-1 V-cycle is k2 steps of FGMRES
  from zero on A_c(tau) y = r_c (a K-cycle: the level-2 preconditioner holds
  GMRES and is therefore not a fixed linear map, which is why the flexible
  method is needed, as on the fine level, Sec. 2);
* its preconditioner, the level-2 cycle M2: z = P2 y with y from k3 GMRES
  steps from zero on A3(tau) y = P2^H r, then s2 GMRES steps from zero on
  A_c e = r - A_c z, z + e (the GMRES smoother the paper settles on in
  Sec. 4, used on level 2, where no lattice block structure is left to
  smooth with SAP);
* the level-2 test vectors start as the restrictions P^H w_j of the first
  ntv2 level-1 test vectors (normalised) and are improved by setup_iters - 1
  rounds of inverse iteration w <- M2(tau = 0) w, each followed by
  normalisation and a rebuild of P2 and D3 (the level-1 setup's reading,
  one level down).
"""
import numpy as np

from . import blocks as bl
from . import mg
from .krylov import fgmres, gmres


def check_blocking3(dims2, block2):
    """Level-2 lattice dims2 split into aggregates of block2 level-2 sites; every
    direction needs >= 2 aggregates so +mu and -mu neighbours are other aggregates."""
    for n, b in zip(dims2, block2):
        if b < 1 or n % b:
            raise ValueError("level-2 aggregate does not divide the block lattice")
        if n // b < 2:
            raise ValueError("need >= 2 level-2 aggregates per direction")


def to_aggregates2(y, dims2, block2):
    """Level-2 vector [nb2, 2 ntv] -> [n3, 2, bs2 * ntv], element (q, i): q the
    site inside the aggregate, i the component inside the chirality half."""
    ntv = y.shape[-1] // 2
    nb3 = bl.nblocks(dims2, block2)
    shp = []
    for n, b in zip(nb3, block2):
        shp += [n, b]
    g = y.reshape(tuple(shp) + (2, ntv)).transpose(0, 2, 4, 6, 1, 3, 5, 7, 8, 9)
    n3, bs2 = int(np.prod(nb3)), int(np.prod(block2))
    g = g.reshape(n3, bs2, 2, ntv).transpose(0, 2, 1, 3)
    return g.reshape(n3, 2, bs2 * ntv)


def from_aggregates2(a, dims2, block2, ntv):
    nb3 = bl.nblocks(dims2, block2)
    bs2 = int(np.prod(block2))
    g = a.reshape(-1, 2, bs2, ntv).transpose(0, 2, 1, 3)
    g = g.reshape(tuple(nb3) + tuple(block2) + (2, ntv)).transpose(0, 4, 1, 5, 2, 6, 3, 7, 8, 9)
    return g.reshape(int(np.prod(dims2)), 2 * ntv)


def build_P2(W2, dims2, block2):
    """P2[n3, 2, bs2 * ntv, ntv2]: per (aggregate, chirality) the ntv2 level-2
    test vectors orthonormalised (MGS, two passes per column)."""
    cols = [to_aggregates2(w, dims2, block2) for w in W2]
    ntv2 = len(cols)
    P = np.zeros(cols[0].shape + (ntv2,), dtype=np.complex128)
    for j in range(ntv2):
        v = cols[j].copy()
        n0 = np.linalg.norm(v, axis=-1)
        for _ in range(2):
            for i in range(j):
                p = P[..., i]
                v = v - np.sum(np.conj(p) * v, axis=-1)[..., None] * p
        n1 = np.linalg.norm(v, axis=-1)
        if np.any(n1 < 1e-12 * n0):
            raise np.linalg.LinAlgError("level-2 test vectors are locally rank deficient")
        P[..., j] = v / n1[..., None]
    return P


def restrict2(P2, y, dims2, block2):
    """P2^H y for a level-2 vector y [nb2, 2 ntv] -> [n3, 2 ntv2]."""
    a = to_aggregates2(y, dims2, block2)
    out = np.einsum("ahkj,ahk->ahj", np.conj(P2), a)
    return out.reshape(out.shape[0], -1)


def prolong2(P2, y3, dims2, block2):
    """P2 y3 for a level-3 vector [n3, 2 ntv2] -> level-2 vector [nb2, 2 ntv]."""
    ntv2 = P2.shape[-1]
    ntv = P2.shape[2] // int(np.prod(block2))
    a = np.einsum("ahkj,ahj->ahk", P2, y3.reshape(y3.shape[0], 2, ntv2))
    return from_aggregates2(a, dims2, block2, ntv)


def _stays_inside(dims2, block2):
    """inside[b, d]: the stencil entry d of level-2 site b couples b to a site of
    its own aggregate (d = 0 always; 1 + 2mu forward, 2 + 2mu backward hops)."""
    x = np.array(list(np.ndindex(*dims2)))
    inside = np.zeros((len(x), 9), dtype=bool)
    inside[:, 0] = True
    for mu in range(4):
        inside[:, 1 + 2 * mu] = (x[:, mu] % block2[mu]) != block2[mu] - 1
        inside[:, 2 + 2 * mu] = (x[:, mu] % block2[mu]) != 0
    return inside


def level3_operator(coarse2, P2, dims2, block2):
    """D3[n3, 9, 2 ntv2, 2 ntv2] = blocks of P2^H D_c P2, column by column: prolong
    a unit level-3 vector, split D_c applied to it into the part that stays in
    each aggregate and the 8 parts that cross to a neighbouring aggregate, and
    restrict every part."""
    n3, _, _, ntv2 = P2.shape
    nc3 = 2 * ntv2
    inside = _stays_inside(dims2, block2)
    D3 = np.zeros((n3, 9, nc3, nc3), dtype=np.complex128)
    for c in range(nc3):
        e = np.zeros((n3, nc3), dtype=np.complex128)
        e[:, c] = 1.0
        p = prolong2(P2, e, dims2, block2)
        parts = [np.einsum("bij,bj->bi", coarse2.Dc[:, d], p[coarse2.nbr[:, d]]) for d in range(9)]
        own = sum(parts[d] * inside[:, d, None] for d in range(9))
        D3[:, 0, :, c] = restrict2(P2, own, dims2, block2)
        for d in range(1, 9):
            D3[:, d, :, c] = restrict2(P2, parts[d] * (~inside[:, d, None]), dims2, block2)
    return D3


class Level3:
    """Level-2 -> level-3 part of the hierarchy (P2, A3), given the level-2 operator."""

    def __init__(self, coarse2, dims2, W2, block2):
        check_blocking3(dims2, block2)
        self.coarse2 = coarse2
        self.dims2 = tuple(dims2)
        self.block2 = tuple(block2)
        self.P2 = build_P2(W2, dims2, block2)
        self.coarse3 = mg.Coarse(level3_operator(coarse2, self.P2, dims2, block2),
                                 bl.neighbour_table(dims2, block2))

    def restrict(self, y):
        return restrict2(self.P2, y, self.dims2, self.block2)

    def prolong(self, y3):
        return prolong2(self.P2, y3, self.dims2, self.block2)

    def cycle(self, r2, tau, k3, s2, qform=False):
        """M2 r2: level-3 correction (k3 GMRES steps from zero), then s2 GMRES
        smoothing steps on level 2."""
        y3 = gmres(lambda v: self.coarse3.apply(v, tau, qform), self.restrict(r2), k3)[0]
        z = self.prolong(y3)
        if s2 > 0:
            def A(v):
                return self.coarse2.apply(v, tau, qform)
            z = z + gmres(A, r2 - A(z), s2)[0]
        return z

    def solve(self, r2, tau, k2, k3, s2, qform=False):
        """k2 FGMRES steps from zero on A_c(tau) y = r2, preconditioned by M2."""
        x, _, _ = fgmres(lambda v: self.coarse2.apply(v, tau, qform),
                         lambda v: self.cycle(v, tau, k3, s2, qform), r2, 0.0, k2, k2)
        return x


class ThreeLevel:
    """Three-level hierarchy: the two-level one plus Level3 on its coarse lattice.
    vcycle() has TwoLevel.vcycle's signature (coarse_iters = k2, coarse_tol
    unused: the level-2 solve takes a fixed number of steps)."""

    def __init__(self, op, W, block, W2, block2, k3=20, s2=2):
        self.two = mg.TwoLevel(op, W, block)
        self.op = op
        self.block = tuple(block)
        self.dims2 = bl.nblocks(op.dims, block)
        self.l3 = Level3(self.two.coarse, self.dims2, W2, block2)
        self.k3 = k3
        self.s2 = s2

    def vcycle(self, r, tau, nu, n_mr, coarse_iters, coarse_tol=None, qform=False, smoother="sap"):
        two = self.two
        rc = mg.restrict(two.P, r, self.block)
        yc = self.l3.solve(rc, tau, coarse_iters, self.k3, self.s2, qform)
        z = mg.prolong(two.P, yc, self.op.dims, self.block)
        return two.post_smooth(r, z, tau, nu, n_mr, qform, smoother)


def initial_level2_vectors(P, W, block, ntv2):
    """Level-2 test vectors to start from: P^H w_j of the first ntv2 level-1 test
    vectors, normalised."""
    out = []
    for w in W[:ntv2]:
        y = mg.restrict(P, w, block)
        out.append(y / np.linalg.norm(y))
    return out


def setup_level3(coarse2, dims2, W2, block2, setup_iters=3, s2=2, k3=20):
    """Level-2 test vectors after setup_iters - 1 rounds of inverse iteration with M2."""
    W2 = [w / np.linalg.norm(w) for w in W2]
    for _ in range(setup_iters - 1):
        l3 = Level3(coarse2, dims2, W2, block2)
        W2 = [l3.cycle(w, 0.0, k3, s2) for w in W2]
        W2 = [w / np.linalg.norm(w) for w in W2]
    return W2
