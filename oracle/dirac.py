"""Wilson(-clover) Dirac operator D, Q = Gamma5 D and the shifted forms.

Follows eq. (2.5) (the action of D on a quark field) with lattice spacing
a = 1 and periodic boundaries in all four directions:

  (D psi)(x) = (m0 + 4) psi(x) + C(x) psi(x)
               - 1/2 sum_mu ((I - gamma_mu) (x) U_mu(x)) psi(x + mu)
               - 1/2 sum_mu ((I + gamma_mu) (x) U_mu(x - mu)^H) psi(x - mu),

C(x) the optional clover term (``oracle.clover``).  Q = Gamma5 D is the
Hermitian Wilson-Dirac operator (Sec. 2, definition after eq. (2.7));
the shifted system of eq. (1.1) is (Q - tau I) x = b, and its
Gamma5-preconditioned form, eq. (3.6) <=> eq. (3.7), is (D - tau Gamma5) x = Gamma5 b.

Fields are complex128 arrays ``psi[N0, N1, N2, N3, 4, 3]`` and
``U[N0, N1, N2, N3, 4, 3, 3]`` (see ``synth.fields``).
"""
import numpy as np

from .gamma import GAMMA, GAMMA5, I4


def fwd(f, mu):
    """f(x + mu) as a field of x (periodic)."""
    return np.roll(f, -1, axis=mu)


def bwd(f, mu):
    """f(x - mu) as a field of x (periodic)."""
    return np.roll(f, 1, axis=mu)


def colour_mul(u, psi):
    """(U psi)_{s,a} = sum_b U_{ab} psi_{s,b} at every site."""
    return np.einsum("...ab,...sb->...sa", u, psi)


def colour_mul_dag(u, psi):
    """(U^H psi)_{s,a} = sum_b conj(U_{ba}) psi_{s,b} at every site."""
    return np.einsum("...ba,...sb->...sa", np.conj(u), psi)


def spin_mul(g, psi):
    """(g psi)_{s,c} = sum_t g_{st} psi_{t,c} at every site."""
    return np.einsum("st,...tc->...sc", g, psi)


def hop_forward(U, psi, mu):
    """-1/2 ((I - gamma_mu) (x) U_mu(x)) psi(x + mu)."""
    return -0.5 * spin_mul(I4 - GAMMA[mu], colour_mul(U[..., mu, :, :], fwd(psi, mu)))


def hop_backward(U, psi, mu):
    """-1/2 ((I + gamma_mu) (x) U_mu(x - mu)^H) psi(x - mu)."""
    ub = bwd(U[..., mu, :, :], mu)
    return -0.5 * spin_mul(I4 + GAMMA[mu], colour_mul_dag(ub, bwd(psi, mu)))


def site_diag(psi, m0, clover=None):
    """(m0 + 4) psi(x) + C(x) psi(x); ``clover`` is complex128[..., 12, 12]."""
    out = (m0 + 4.0) * psi
    if clover is not None:
        shp = psi.shape
        out = out + np.einsum("...ij,...j->...i", clover,
                              psi.reshape(shp[:-2] + (12,))).reshape(shp)
    return out


def apply_D(U, psi, m0, clover=None):
    """D psi per eq. (2.5) (plus the clover term when given)."""
    out = site_diag(psi, m0, clover)
    for mu in range(4):
        out = out + hop_forward(U, psi, mu) + hop_backward(U, psi, mu)
    return out


def gamma5(psi):
    """Gamma5 = I_sites (x) gamma5 (x) I_3."""
    return spin_mul(GAMMA5, psi)


def apply_Q(U, psi, m0, clover=None):
    """Q psi = Gamma5 D psi."""
    return gamma5(apply_D(U, psi, m0, clover))


def apply_Q_shifted(U, psi, m0, tau, clover=None):
    """(Q - tau I) psi, the operator of eq. (1.1) / eq. (3.6)."""
    return apply_Q(U, psi, m0, clover) - tau * psi


def apply_A(U, psi, m0, tau, clover=None):
    """(D - tau Gamma5) psi, the Gamma5-preconditioned operator of eq. (3.7)."""
    return apply_D(U, psi, m0, clover) - tau * gamma5(psi)


class Operator:
    """Bundle of (U, m0, clover) with the shifted applies used by the solver."""

    def __init__(self, U, m0, clover=None):
        self.U = U
        self.m0 = float(m0)
        self.clover = clover
        self.dims = tuple(U.shape[:4])

    def D(self, psi):
        return apply_D(self.U, psi, self.m0, self.clover)

    def Q(self, psi):
        return apply_Q(self.U, psi, self.m0, self.clover)

    def Q_shifted(self, psi, tau):
        return apply_Q_shifted(self.U, psi, self.m0, tau, self.clover)

    def A(self, psi, tau):
        return apply_A(self.U, psi, self.m0, tau, self.clover)
