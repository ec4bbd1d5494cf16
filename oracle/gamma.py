"""Euclidean gamma matrices in a chiral basis with gamma5 = diag(I2, -I2).

The paper fixes only gamma5 = gamma0 gamma1 gamma2 gamma3 = diag(I2, -I2)
(Sec. 2, text before eq. (2.5), the Wilson-Dirac operator) and the Clifford relation
gamma_mu gamma_nu + gamma_nu gamma_mu = 2 delta_mu_nu (eq. (2.3)).  The
basis chosen here (reading: gamma0 = [[0,-I],[-I,0]],
gamma_k = [[0,-i sigma_k],[i sigma_k,0]]) satisfies both; any such basis gives
the same spectrum.
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
Z2 = np.zeros((2, 2), dtype=np.complex128)
SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)

GAMMA = (
    np.block([[Z2, -I2], [-I2, Z2]]),
    np.block([[Z2, -1j * SIGMA[0]], [1j * SIGMA[0], Z2]]),
    np.block([[Z2, -1j * SIGMA[1]], [1j * SIGMA[1], Z2]]),
    np.block([[Z2, -1j * SIGMA[2]], [1j * SIGMA[2], Z2]]),
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
I4 = np.eye(4, dtype=np.complex128)


def sigma_munu(mu, nu):
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])
