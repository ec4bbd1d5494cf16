"""Sheikholeslami-Wohlert clover term.

The paper adds a site-diagonal clover term to D for its large configurations,
states that it has 6x6 diagonal blocks and keeps D Gamma5-Hermitian, and
cites Sheikholeslami-Wohlert for it (Sec. 4, text before the configuration
table), but prints no formula.  Reading (standard clover-leaf form):

  C(x)      = c_sw * (i/4) * sum_{mu,nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
  Fhat      = (1/8) (Q_{mu nu}(x) - Q_{mu nu}(x)^H), made traceless,
  Q_{mu nu} = sum of the four plaquettes in the (mu, nu) plane that start and
              end at x, each taken counter-clockwise.

The paper prints no clover values; sign and normalisation are pinned by the
property it states for the term (Sec. 2, text after eq. (2.5)): it lowers the
discretisation error from O(a) to O(a^2).  In a uniform abelian field the
near-zero eigenvalues of D at m0 = 0 are (1 - c_sw) |B| / 2 + O(B^2), the
Wilson term's O(a) Pauli shift cancelled at c_sw = 1 (tests/test_oracle_operator.py).
The structure is pinned as well: two Hermitian 6x6 chirality blocks,
[C, Gamma5] = 0, C = 0 at U = 1, linearity in c_sw, gauge covariance.
"""
import numpy as np

from .dirac import bwd, fwd
from .gamma import sigma_munu


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def leaves(U, mu, nu):
    """Q_{mu nu}(x): the four counter-clockwise plaquettes based at x."""
    umu = U[..., mu, :, :]
    unu = U[..., nu, :, :]
    # leaf 1: x -> x+mu -> x+mu+nu -> x+nu -> x
    l1 = umu @ fwd(unu, mu) @ _dag(fwd(umu, nu)) @ _dag(unu)
    # leaf 2: x -> x+nu -> x-mu+nu -> x-mu -> x
    l2 = unu @ _dag(bwd(fwd(umu, nu), mu)) @ _dag(bwd(unu, mu)) @ bwd(umu, mu)
    # leaf 3: x -> x-mu -> x-mu-nu -> x-nu -> x
    l3 = (_dag(bwd(umu, mu)) @ _dag(bwd(bwd(unu, mu), nu))
          @ bwd(bwd(umu, mu), nu) @ bwd(unu, nu))
    # leaf 4: x -> x-nu -> x-nu+mu -> x+mu -> x
    l4 = _dag(bwd(unu, nu)) @ bwd(umu, nu) @ fwd(bwd(unu, nu), mu) @ _dag(umu)
    return l1 + l2 + l3 + l4


def field_strength(U, mu, nu, traceless=True):
    """Fhat_{mu nu}(x) = (Q_{mu nu} - Q_{mu nu}^H) / 8 (anti-Hermitian)."""
    q = leaves(U, mu, nu)
    f = (q - _dag(q)) / 8.0
    if traceless:
        tr = np.trace(f, axis1=-2, axis2=-1) / 3.0
        f = f - tr[..., None, None] * np.eye(3)
    return f


def clover_term(U, csw, traceless=True):
    """C(x) as complex128[N0, N1, N2, N3, 12, 12] (component index 3*s + c)."""
    dims = U.shape[:4]
    c = np.zeros(dims + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            f = field_strength(U, mu, nu, traceless)
            s = sigma_munu(mu, nu)
            c += np.einsum("st,...ab->...satb", s, f)
    c *= csw * 0.25j
    return c.reshape(dims + (12, 12))


def chirality_blocks(clover):
    """The two 6x6 blocks of C (spins 0,1 and spins 2,3): [..., 2, 6, 6]."""
    return np.stack([clover[..., 0:6, 0:6], clover[..., 6:12, 6:12]], axis=-3)
