"""Seeded synthetic lattice fields in canonical order.

Canonical layout (shared by the oracle, the tests and the C interface):

* lattice ``dims = (N0, N1, N2, N3)``, ``N0`` the time extent; site index
  ``((x0*N1 + x1)*N2 + x2)*N3 + x3``;
* spinor field: ``complex128[N0, N1, N2, N3, 4, 3]`` (spin-major, then
  colour, so component ``3*s + c``); ``nrhs`` fields stack in front;
* gauge field: ``complex128[N0, N1, N2, N3, 4, 3, 3]``, ``U[x, mu, a, b]``
  is the link from ``x`` to ``x + mu`` acting as ``(U psi)_a = sum_b U_ab psi_b``.

Links are ``exp(i*eps*H)`` with ``H`` a traceless Hermitian 3x3 matrix built
from Gaussian entries, so every link lies in SU(3); ``eps`` sets how rough the
field is (``eps=pi`` is used for random gauge transformations).
"""
import numpy as np

_SEED_BASE = 20040814600
ROLES = {"U": 0, "b": 1, "phi": 2, "x": 3, "W": 4, "Omega": 5}


def seed_for(config, role):
    """Seed of input ``role`` (U, b, phi, x, W, Omega) of workload ``config``."""
    return _SEED_BASE + 100 * int(config) + ROLES[role]


def kappa_to_m0(kappa):
    """Bare mass from the hopping parameter: a*m0 = 1/(2 kappa) - 4."""
    return 1.0 / (2.0 * kappa) - 4.0


def _random_su3(rng, n, eps):
    g1 = rng.standard_normal((n, 3, 3))
    g2 = rng.standard_normal((n, 3, 3))
    a = g1 + 1j * g2
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[:, None, None] * np.eye(3)
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    return (v * ph[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def random_links(dims, eps, seed, chunk=1 << 20):
    """SU(3) links exp(i eps H), drawn in canonical [site][mu] order."""
    dims = tuple(int(d) for d in dims)
    nlink = int(np.prod(dims)) * 4
    rng = np.random.default_rng(seed)
    out = np.empty((nlink, 3, 3), dtype=np.complex128)
    for s in range(0, nlink, chunk):
        e = min(nlink, s + chunk)
        out[s:e] = _random_su3(rng, e - s, eps)
    return out.reshape(dims + (4, 3, 3))


def unit_links(dims):
    dims = tuple(int(d) for d in dims)
    u = np.zeros(dims + (4, 3, 3), dtype=np.complex128)
    u[..., :, :] = np.eye(3)
    return u


def random_spinors(dims, nrhs, seed):
    """``nrhs`` complex Gaussian spinor fields (Re, Im iid N(0,1))."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    shape = (int(nrhs),) + dims + (4, 3)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def gauge_transform(dims, seed):
    """Random SU(3) matrix per site (exp(i pi H)), for covariance checks."""
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    return _random_su3(rng, n, np.pi).reshape(dims + (3, 3))


def random_test_vectors(dims, ntv, seed):
    """``ntv`` complex Gaussian fields used as multigrid test vectors."""
    return random_spinors(dims, ntv, seed)


def device_gaussian_spinors(dims, nrhs, seed, device="cuda"):
    """Complex Gaussian spinor fields drawn on the GPU with torch's seeded
    generator (for large inputs only the GPU consumes, e.g. setup vectors)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    shape = (int(nrhs),) + tuple(int(d) for d in dims) + (4, 3)
    re = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=g, device=device, dtype=torch.float64)
    return torch.complex(re, im)
