"""Gauge-field derivative of L = phi^H Q x (Wilson part).

Not part of the paper; follows from eq. (2.5).  L contains each link U_mu(y)
linearly through the forward hop at y and its conjugate through the backward
hop at y + mu, so the two Wirtinger derivatives per link are

  G[y,mu]_{ab}    = dL/dU_mu(y)_{ab}
                  = -1/2 sum_{s,t} conj(phi(y)_{s,a}) [g5 (I - g_mu)]_{st} x(y+mu)_{t,b},
  Gbar[y,mu]_{ab} = dL/d conj(U_mu(y)_{ab})
                  = -1/2 sum_{s,t} conj(phi(y+mu)_{s,b}) [g5 (I + g_mu)]_{st} x(y)_{t,a}.
"""
import numpy as np

from .dirac import fwd
from .gamma import GAMMA, GAMMA5, I4


def gauge_force(phi, x):
    """(G, Gbar), each complex128[N0, N1, N2, N3, 4, 3, 3]."""
    dims = phi.shape[:4]
    G = np.zeros(dims + (4, 3, 3), dtype=np.complex128)
    Gb = np.zeros_like(G)
    for mu in range(4):
        gm = GAMMA5 @ (I4 - GAMMA[mu])
        gp = GAMMA5 @ (I4 + GAMMA[mu])
        G[..., mu, :, :] = -0.5 * np.einsum("...sa,st,...tb->...ab",
                                            np.conj(phi), gm, fwd(x, mu))
        Gb[..., mu, :, :] = -0.5 * np.einsum("...sb,st,...ta->...ab",
                                             np.conj(fwd(phi, mu)), gp, x)
    return G, Gb
