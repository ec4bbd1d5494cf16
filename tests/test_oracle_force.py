"""Pins of the oracle's gauge-force derivative d(phi^H Q x)/dU."""
import numpy as np

from oracle import dirac, force
from synth import gauge_transform, random_links, random_spinors, seed_for


def _L(U, phi, x, m0):
    return np.vdot(phi, dirac.apply_Q(U, x, m0))


def test_force_matches_central_differences():
    """L is affine in each single link entry, so central differences are exact up to rounding."""
    dims = (4, 4, 2, 4)
    m0 = -0.4
    U = random_links(dims, 0.5, seed_for(3, "U"))
    phi = random_spinors(dims, 1, seed_for(3, "phi"))[0]
    x = random_spinors(dims, 1, seed_for(3, "x"))[0]
    G, Gb = force.gauge_force(phi, x)
    rng = np.random.default_rng(0)
    h = 1e-6
    L0 = abs(_L(U, phi, x, m0))
    for _ in range(24):
        idx = tuple(int(rng.integers(0, n)) for n in dims) + (
            int(rng.integers(0, 4)), int(rng.integers(0, 3)), int(rng.integers(0, 3)))
        for direction, expect in ((1.0, G[idx] + Gb[idx]), (1j, 1j * (G[idx] - Gb[idx]))):
            Up = U.copy()
            Um = U.copy()
            Up[idx] += h * direction
            Um[idx] -= h * direction
            fd = (_L(Up, phi, x, m0) - _L(Um, phi, x, m0)) / (2 * h)
            assert abs(fd - expect) < 1e-8 * L0


def test_force_second_order_affine():
    """Perturbing one entry by a finite amount changes L exactly linearly (affine in U, Ubar)."""
    dims = (2, 2, 4, 2)
    U = random_links(dims, 0.5, seed_for(3, "U"))
    phi, x = random_spinors(dims, 2, 77)
    G, Gb = force.gauge_force(phi, x)
    idx = (1, 0, 3, 1, 2, 0, 2)      # site (1,0,3,1), mu = 2, entry (0, 2)
    dz = 0.7 - 0.4j
    Up = U.copy()
    Up[idx] += dz
    dL = _L(Up, phi, x, -0.3) - _L(U, phi, x, -0.3)
    assert abs(dL - (G[idx] * dz + Gb[idx] * np.conj(dz))) < 1e-12 * abs(dL)


def test_force_gauge_covariance():
    """Under U_mu(y) -> O(y) U_mu(y) O(y+mu)^H, phi -> O phi, x -> O x:
    G_mu(y) -> conj(O(y)) G_mu(y) O(y+mu)^T."""
    dims = (4, 2, 2, 4)
    U = random_links(dims, 0.5, seed_for(3, "U"))
    Om = gauge_transform(dims, seed_for(3, "Omega"))
    phi, x = random_spinors(dims, 2, 5)
    G, _ = force.gauge_force(phi, x)
    rot = lambda f: np.einsum("...ab,...sb->...sa", Om, f)
    Gg, _ = force.gauge_force(rot(phi), rot(x))
    for mu in range(4):
        ref = np.conj(Om) @ G[..., mu, :, :] @ np.swapaxes(dirac.fwd(Om, mu), -1, -2)
        assert np.abs(Gg[..., mu, :, :] - ref).max() < 1e-12
    assert U.shape[-3] == 4
