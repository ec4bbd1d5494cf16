"""Pins of the oracle's Dirac operator against the paper and closed forms."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import clover, dense, dirac
from oracle.gamma import GAMMA, GAMMA5, I4, sigma_munu
from synth import (gauge_transform, kappa_to_m0, random_links, random_spinors,
                   seed_for, unit_links)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def test_gamma_basis():
    # eq. (2.3): Clifford algebra; Hermitian gammas; gamma5 = g0 g1 g2 g3 = diag(I2, -I2)
    for mu in range(4):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        for nu in range(4):
            ac = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * I4)
        # gamma5 anticommutes with every gamma_mu (eq. (2.4))
        assert np.allclose(GAMMA5 @ GAMMA[mu], -GAMMA[mu] @ GAMMA5)
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))
    # sigma_{mu nu} is block diagonal in chirality, so the clover term splits into 6x6 blocks
    for mu, nu in itertools.combinations(range(4), 2):
        s = sigma_munu(mu, nu)
        assert np.allclose(s @ GAMMA5, GAMMA5 @ s)


def test_kappa_m0_table():
    with open(GOLDEN) as f:
        rows = json.load(f)["kappa_m0"]["rows"]
    for kappa, m0 in rows:
        assert abs(kappa_to_m0(kappa) - m0) < 5e-5


def _free_eigen(dims, m0, n):
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    mp = m0 + sum(1 - np.cos(q) for q in p)
    s2 = sum(np.sin(q) ** 2 for q in p)
    qp = GAMMA5 @ (mp * I4 + 1j * sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4)))
    return p, qp, np.sqrt(mp * mp + s2)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 4, 8)])
def test_free_field_plane_waves(dims):
    """U = 1: e^{ip.x} chi (x) c is an eigenvector of Q with lambda = +-sqrt(m(p)^2 + sum sin^2 p)."""
    m0 = -0.5
    U = unit_links(dims)
    rng = np.random.default_rng(7)
    x = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    for _ in range(6):
        n = [int(rng.integers(0, d)) for d in dims]
        p, qp, lam = _free_eigen(dims, m0, n)
        w, v = np.linalg.eigh(qp)
        assert np.allclose(np.sort(np.abs(w)), lam)
        phase = np.exp(1j * sum(p[mu] * x[mu] for mu in range(4)))
        col = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        for k in range(4):
            psi = phase[..., None, None] * np.einsum("s,c->sc", v[:, k], col)
            out = dirac.apply_Q(U, psi, m0)
            assert np.abs(out - w[k] * psi).max() < 1e-12 * np.abs(psi).max()
            assert abs(abs(w[k]) - lam) < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_free_field_dense_spectrum(dims):
    m0 = -0.5
    U = unit_links(dims)
    Q = dense.dense_Q(U, m0)
    ev = np.sort(np.linalg.eigvalsh(Q))
    ref = []
    for n in np.ndindex(*dims):
        _, _, lam = _free_eigen(dims, m0, n)
        ref += [lam] * 6 + [-lam] * 6
    ref = np.sort(np.array(ref))
    assert np.abs(ev - ref).max() < 1e-12
    if dims == (4, 4, 4, 4):
        mags = np.unique(np.round(np.abs(ev), 10))
        assert abs(mags.min() - 0.5) < 1e-12 and abs(mags.max() - 7.5) < 1e-12
        assert len(mags) == 15


@pytest.mark.parametrize("dims,csw", [((2, 2, 2, 2), 0.0), ((2, 2, 2, 2), 1.0),
                                      ((4, 2, 2, 2), 1.3)])
def test_matrix_free_equals_dense(dims, csw):
    U = random_links(dims, 0.5, seed_for(1, "U"))
    C = clover.clover_term(U, csw) if csw else None
    psi = random_spinors(dims, 1, seed_for(1, "b"))[0]
    D = dense.dense_D(U, -0.7, C)
    ref = (D @ psi.reshape(-1)).reshape(psi.shape)
    assert np.abs(dirac.apply_D(U, psi, -0.7, C) - ref).max() < 1e-13 * np.abs(ref).max()


def test_dense_brute_force_2x4():
    """Dense eigendecomposition of Q on 2^4: Hermitian, real spectrum, bounded, indefinite."""
    dims = (2, 2, 2, 2)
    U = random_links(dims, 0.3, seed_for(1, "U"))
    m0 = -0.5
    Q = dense.dense_Q(U, m0)
    assert np.abs(Q - Q.conj().T).max() < 1e-15
    w, v = np.linalg.eigh(Q)
    # eigenvectors of the dense matrix are eigenvectors of the matrix-free Q
    for k in (0, 50, 191):
        psi = v[:, k].reshape(dims + (4, 3))
        assert np.abs(dirac.apply_Q(U, psi, m0) - w[k] * psi).max() < 1e-12
    assert np.abs(w).max() <= abs(m0 + 4) + 4 + 1e-12
    # maximally indefinite (Sec. 3.1): about as many positive as negative eigenvalues
    assert abs(int(np.sum(w > 0)) - int(np.sum(w < 0))) <= 24


def test_gamma5_hermiticity():
    """eq. (2.7): Gamma5 D = (Gamma5 D)^H, i.e. <phi, Q psi> = <Q phi, psi>."""
    dims = (4, 4, 4, 4)
    U = random_links(dims, 0.5, seed_for(2, "U"))
    C = clover.clover_term(U, 1.0)
    phi, psi = random_spinors(dims, 2, seed_for(2, "b"))
    a = np.vdot(phi, dirac.apply_Q(U, psi, -0.8, C))
    b = np.vdot(dirac.apply_Q(U, phi, -0.8, C), psi)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_gauge_covariance(csw):
    """Q[U^Omega] (Omega psi) = Omega (Q[U] psi), U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^H."""
    dims = (4, 4, 2, 4)
    U = random_links(dims, 0.5, seed_for(2, "U"))
    Om = gauge_transform(dims, seed_for(2, "Omega"))
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(
            np.swapaxes(dirac.fwd(Om, mu), -1, -2))
    psi = random_spinors(dims, 1, seed_for(2, "b"))[0]
    C = clover.clover_term(U, csw) if csw else None
    Cg = clover.clover_term(Ug, csw) if csw else None
    lhs = dirac.apply_Q(Ug, np.einsum("...ab,...sb->...sa", Om, psi), -0.8, Cg)
    rhs = np.einsum("...ab,...sb->...sa", Om, dirac.apply_Q(U, psi, -0.8, C))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


def test_clover_structure():
    dims = (4, 4, 4, 4)
    U = random_links(dims, 0.5, seed_for(2, "U"))
    C1 = clover.clover_term(U, 1.0)
    C2 = clover.clover_term(U, 2.5)
    assert np.abs(C2 - 2.5 * C1).max() < 1e-13
    # Hermitian, commutes with gamma5 -> two Hermitian 6x6 chirality blocks
    assert np.abs(C1 - np.conj(np.swapaxes(C1, -1, -2))).max() < 1e-14
    g5 = np.kron(GAMMA5, np.eye(3))
    assert np.abs(C1 @ g5 - g5 @ C1).max() < 1e-14
    assert np.abs(C1[..., 0:6, 6:12]).max() == 0.0
    # each 6x6 block traceless (traceless field strength, traceless sigma blocks)
    blk = clover.chirality_blocks(C1)
    assert np.abs(np.trace(blk, axis1=-2, axis2=-1)).max() < 1e-13
    assert np.abs(clover.clover_term(unit_links(dims), 1.0)).max() == 0.0
    assert np.abs(C1).max() > 0.1


def test_clover_abelian_flux():
    """Uniform abelian flux phi in the (0,1) plane: Fhat_01 = i sin(phi) lambda, so
    C = -(c_sw/2) sin(phi) sigma_01 (x) lambda, lambda = diag(1, -1, 0)."""
    dims = (6, 4, 2, 2)
    k = 1
    phi = 2 * np.pi * k / dims[0]
    lam = np.diag([1.0, -1.0, 0.0])
    U = unit_links(dims)
    x0 = np.arange(dims[0])
    for t in range(dims[0]):
        U[t, :, :, :, 1] = np.diag(np.exp(1j * phi * t * np.diag(lam)))
    C = clover.clover_term(U, 1.7)
    ref = -(1.7 / 2) * np.sin(phi) * np.kron(sigma_munu(0, 1), lam)
    assert x0.size == dims[0]
    assert np.abs(C - ref).max() < 1e-14


def _uniform_flux_links(L0, L1, n):
    """SU(3) links on L0 x L1 x 1 x 1 carrying n quanta of uniform abelian flux in the (0,1)
    plane, colour-diagonal diag(B, -B, 0): every (0,1) plaquette equals exp(i B lambda),
    B = 2 pi n / (L0 L1) (the twist on the last t-slice closes the torus)."""
    dims = (L0, L1, 1, 1)
    B = 2 * np.pi * n / (L0 * L1)
    lam = np.array([1.0, -1.0, 0.0])
    U = unit_links(dims)
    for t in range(L0):
        U[t, :, :, :, 1] = np.diag(np.exp(1j * B * t * lam))
    for y in range(L1):
        U[L0 - 1, y, :, :, 0] = np.diag(np.exp(-1j * B * L0 * y * lam))
    return U, B


def test_clover_tree_level_improvement():
    """Sign and normalisation of the clover term, from the property the paper gives it
    (Sec. 2, text after eq. (2.5); Sec. 4): it lowers the discretisation error from O(a)
    to O(a^2).  In a uniform field B the lowest Landau level is annihilated by the
    continuum gamma.D; expanding the Wilson term, -(1/2) Laplacian = -(1/2)(gamma.D)^2
    - (i/4) sigma_{mu nu} F_{mu nu}, shifts those modes by the O(a) Pauli term +|B|/2, and
    the clover term at c_sw = 1 cancels it.  So the near-zero eigenvalues of D (m0 = 0) are
    (1 - c_sw) |B| / 2 + O(B^2), for either colour of the field; at c_sw = 1 what is left
    falls as B^2 (4x smaller B, ~16x smaller eigenvalue), at c_sw = 0 only as B.  A flipped
    sign, another normalisation of Fhat or sigma, or clockwise leaves move them by O(B)."""
    left = {}
    for L in (8, 16):
        U, B = _uniform_flux_links(L, L, 1)
        V = L * L
        for csw in (0.0, 1.0, -1.0, 2.0):
            A = dense.sparse_D(U, 0.0, clover.clover_term(U, csw) if csw else None)
            for col in (0, 1):
                idx = np.array([12 * i + 3 * s + col for i in range(V) for s in range(4)])
                w = np.linalg.eigvals(A[idx][:, idx].toarray())
                w = w[np.argsort(np.abs(w))]
                # a degenerate real pair (the two spin states of the lowest level) ...
                assert np.abs(w[:2].imag).max() < 1e-9
                assert abs(w[0].real - w[1].real) < 1e-9
                # ... well separated from the next level (|lambda| ~ sqrt(2 B))
                assert np.abs(w[2]) > 4 * B
                assert abs(w[0].real - (1 - csw) * B / 2) < 0.1 * B * B, (L, csw, col, w[0])
                left[(L, csw, col)] = w[0].real
    for col in (0, 1):
        r1 = left[(8, 1.0, col)] / left[(16, 1.0, col)]
        r0 = left[(8, 0.0, col)] / left[(16, 0.0, col)]
        assert 12 < r1 < 20, r1
        assert 3.5 < r0 < 4.5, r0


def test_norm_bound_lambda_max():
    """|lambda| <= |m0 + 4| + 4 (+ ||C||); the paper's estimate lambda_max = 8 (Sec. 4)."""
    with open(GOLDEN) as f:
        lmax = json.load(f)["lambda_max_Q"]["value"]
    dims = (2, 2, 2, 2)
    U = random_links(dims, 0.5, seed_for(1, "U"))
    C = clover.clover_term(U, 1.0)
    m0 = kappa_to_m0(0.13632)
    Q = dense.dense_Q(U, m0, C)
    w = np.linalg.eigvalsh(Q)
    cn = max(np.linalg.norm(C[x], 2) for x in np.ndindex(*dims))
    assert np.abs(w).max() <= abs(m0 + 4) + 4 + cn + 1e-12
    assert abs(m0 + 4) + 4 <= lmax
