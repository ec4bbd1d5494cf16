"""Eigenpairs of Q = Gamma5 D of smallest modulus -- the object the GD-lambdaAMG
eigensolver computes (Alg. GD-lambdaAMG, Sec. 3.3; Q Hermitian, eq. (1.1)).

Test infrastructure.  The result has a plain definition, so the oracle writes
the definition out for lattices small enough to hold Q densely: assemble Q
from the site couplings (``oracle.dense``), take the full Hermitian
eigendecomposition, and order the pairs by |lambda|.  Eigenvectors are
returned as canonical fields; within a degenerate eigenspace they are one
valid basis, so comparisons use eigenvalues, residuals and subspaces.
"""
import numpy as np

from . import dense


def smallest_eigenpairs(U, m0, clover, k):
    """(lambda[k], X[k, *dims, 4, 3]): the k eigenpairs of Q of smallest |lambda|,
    in order of increasing |lambda|."""
    dims = U.shape[:4]
    w, v = np.linalg.eigh(dense.dense_Q(U, m0, clover))
    order = np.argsort(np.abs(w), kind="stable")[:k]
    X = v[:, order].T.reshape((k,) + tuple(dims) + (4, 3))
    return w[order], X


def free_spectrum(dims, m0):
    """Closed form of spec(Q) for U = 1: for each lattice momentum p (p_mu = 2 pi
    n_mu / N_mu) Q(p) = Gamma5 [M(p) + i sum_mu gamma_mu sin p_mu] with
    M(p) = m0 + sum_mu (1 - cos p_mu); Q(p)^2 = M^2 + sum sin^2, trace Q(p) = 0,
    so +-sqrt(M^2 + sum sin^2 p) each occur twice in spin and three times in
    colour."""
    vals = []
    for n in np.ndindex(*dims):
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
        M = m0 + sum(1 - np.cos(q) for q in p)
        e = np.sqrt(M * M + sum(np.sin(q) ** 2 for q in p))
        vals += [e] * 6 + [-e] * 6
    return np.sort(np.array(vals))


def smallest_eigenpairs_sparse(U, m0, clover, k, extra=12):
    """As smallest_eigenpairs, for lattices too large for a dense Q.

    The eigenpairs of Q of smallest |lambda| are those of Q^2 of smallest
    eigenvalue: Lanczos (scipy.sparse.linalg.eigsh) on Q^2, applied as two
    products with the sparse Q of the site couplings, gives an orthonormal
    basis of the span of the k + extra smallest; Q restricted to that span
    (Rayleigh-Ritz, exact for an invariant subspace) is diagonalised densely and
    the k pairs of smallest |lambda| are returned.  The margin of `extra`
    vectors keeps a +-lambda pair from being cut at the boundary."""
    import scipy.sparse.linalg as sla

    dims = U.shape[:4]
    Q = dense.sparse_Q(U, m0, clover)
    Q2 = sla.LinearOperator(Q.shape, matvec=lambda v: Q @ (Q @ v), dtype=np.complex128)
    m = k + extra
    _, B = sla.eigsh(Q2, k=m, which="SA", ncv=max(2 * m + 20, 100), tol=1e-14, maxiter=200000)
    B, _ = np.linalg.qr(B)
    H = B.conj().T @ (Q @ B)
    w, s = np.linalg.eigh(0.5 * (H + H.conj().T))
    order = np.argsort(np.abs(w), kind="stable")[:k]
    X = (B @ s[:, order]).T.reshape((k,) + tuple(dims) + (4, 3))
    return w[order], X
