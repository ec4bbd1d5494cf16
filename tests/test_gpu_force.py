"""GPU gauge force d(phi^H Q x)/dU: parity with the oracle and autograd."""
import numpy as np
import pytest

from gpu_common import case, dev, host, need_gpu, torch
from helpers import rel_err
from oracle import dirac, force
from synth import random_links, random_spinors, seed_for

pytestmark = pytest.mark.gpu


def test_force_parity_16x4():
    """Config: 16^4, random SU(3) links eps = 0.5, Gaussian phi and x."""
    case("gauge force 16^4")
    qmg = need_gpu()
    dims = (16, 16, 16, 16)
    U = random_links(dims, 0.5, seed_for(3, "U"))
    phi = random_spinors(dims, 1, seed_for(3, "phi"))
    x = random_spinors(dims, 1, seed_for(3, "x"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), -0.8, 0.0)
    G, Gb = lat.gauge_force(lat.pack(dev(phi)), lat.pack(dev(x)))
    Gr, Gbr = force.gauge_force(phi[0], x[0])
    assert rel_err(host(G), Gr) < 1e-13
    assert rel_err(host(Gb), Gbr) < 1e-13


def test_force_autograd_and_finite_differences():
    """torch.autograd through the library vs central differences of L at h = 1e-6."""
    case("gauge force autograd 4x4x4x8")
    qmg = need_gpu()
    dims = (4, 4, 4, 8)
    m0 = -0.6
    U = random_links(dims, 0.5, seed_for(3, "U"))
    phi = random_spinors(dims, 1, seed_for(3, "phi"))
    x = random_spinors(dims, 1, seed_for(3, "x"))
    lat = qmg.Lattice(dims, (2, 2, 2, 2))
    Ut = dev(U).requires_grad_(True)
    pt = dev(phi)
    xt = dev(x)
    L = qmg.QuadraticForm.apply(lat, Ut, pt, xt, m0)
    Lref = np.vdot(phi[0], dirac.apply_Q(U, x[0], m0))
    assert abs(complex(L.item()) - Lref) < 1e-12 * abs(Lref)
    L.real.backward()
    gU = host(Ut.grad)
    G, Gb = force.gauge_force(phi[0], x[0])
    assert rel_err(gU, Gb + np.conj(G)) < 1e-13
    # d Re L / d Re U_e and d Re L / d Im U_e by central differences of the GPU forward
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(8):
        e = tuple(int(rng.integers(0, n)) for n in dims) + (int(rng.integers(0, 4)), int(rng.integers(0, 3)),
                                                             int(rng.integers(0, 3)))
        for dz, comp in ((1.0, gU[e].real), (1j, gU[e].imag)):
            Up = U.copy()
            Um = U.copy()
            Up[e] += h * dz
            Um[e] -= h * dz
            Lp = qmg.QuadraticForm.apply(lat, dev(Up), pt, xt, m0).item()
            Lm = qmg.QuadraticForm.apply(lat, dev(Um), pt, xt, m0).item()
            fd = (complex(Lp).real - complex(Lm).real) / (2 * h)
            assert abs(fd - comp) < 1e-8 * abs(Lref)


def test_force_rejects_clover():
    case("gauge force clover rejected")
    qmg = need_gpu()
    lat = qmg.Lattice((8, 8, 8, 8), (4, 4, 4, 4))
    lat.set_gauge(dev(random_links((8, 8, 8, 8), 0.5, 1)), -0.8, 1.0)
    with pytest.raises(qmg.QmgError) as e:
        lat.gauge_force(lat.field(1), lat.field(1))
    assert e.value.status == -2
