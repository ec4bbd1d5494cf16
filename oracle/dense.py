"""Dense matrix of D assembled entry block by entry block (small lattices).

Independent of the matrix-free ``oracle.dirac`` code: it writes out the
site couplings of eq. (2.6),

  D_{x, x+mu} = -1/2 (I - gamma_mu) (x) U_mu(x),
  D_{x, x-mu} = -1/2 (I + gamma_mu) (x) U_mu(x - mu)^H,

plus the diagonal (m0 + 4) I + C(x), with a Python loop over sites.  Blocks
are accumulated, so lattices with extent 2 (where x + mu = x - mu) are right.
Row/column index = 12 * site + 3 * spin + colour.
"""
import numpy as np

from .gamma import GAMMA, GAMMA5, I4


def site_index(x, dims):
    return ((x[0] * dims[1] + x[1]) * dims[2] + x[2]) * dims[3] + x[3]


def dense_D(U, m0, clover=None):
    dims = U.shape[:4]
    V = int(np.prod(dims))
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for x in np.ndindex(*dims):
        i = site_index(x, dims)
        blk = (m0 + 4.0) * np.eye(12, dtype=np.complex128)
        if clover is not None:
            blk = blk + clover[x]
        D[12 * i:12 * i + 12, 12 * i:12 * i + 12] += blk
        for mu in range(4):
            xp = list(x)
            xp[mu] = (xp[mu] + 1) % dims[mu]
            xm = list(x)
            xm[mu] = (xm[mu] - 1) % dims[mu]
            j = site_index(xp, dims)
            k = site_index(xm, dims)
            D[12 * i:12 * i + 12, 12 * j:12 * j + 12] += \
                -0.5 * np.kron(I4 - GAMMA[mu], U[x][mu])
            D[12 * i:12 * i + 12, 12 * k:12 * k + 12] += \
                -0.5 * np.kron(I4 + GAMMA[mu], np.conj(U[tuple(xm)][mu]).T)
    return D


def dense_gamma5(V):
    return np.kron(np.eye(V), np.kron(GAMMA5, np.eye(3)))


def dense_Q(U, m0, clover=None):
    V = int(np.prod(U.shape[:4]))
    return dense_gamma5(V) @ dense_D(U, m0, clover)


def sparse_D(U, m0, clover=None):
    """D as a scipy.sparse CSR matrix, from the same site couplings (any size)."""
    import scipy.sparse as sp
    dims = U.shape[:4]
    V = int(np.prod(dims))
    rows, cols, vals = [], [], []
    base = np.arange(12)
    for x in np.ndindex(*dims):
        i = site_index(x, dims)
        blk = (m0 + 4.0) * np.eye(12, dtype=np.complex128)
        if clover is not None:
            blk = blk + clover[x]
        blocks = [(i, blk)]
        for mu in range(4):
            xp = list(x)
            xp[mu] = (xp[mu] + 1) % dims[mu]
            xm = list(x)
            xm[mu] = (xm[mu] - 1) % dims[mu]
            blocks.append((site_index(xp, dims), -0.5 * np.kron(I4 - GAMMA[mu], U[x][mu])))
            blocks.append((site_index(xm, dims),
                           -0.5 * np.kron(I4 + GAMMA[mu], np.conj(U[tuple(xm)][mu]).T)))
        for j, b in blocks:
            rows.append(np.repeat(12 * i + base, 12))
            cols.append(np.tile(12 * j + base, 12))
            vals.append(b.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(12 * V, 12 * V))
    return A.tocsr()   # duplicate (i, j) entries are summed


def sparse_Q(U, m0, clover=None):
    import scipy.sparse as sp
    V = int(np.prod(U.shape[:4]))
    g5 = sp.diags(np.tile(np.repeat([1.0, 1.0, -1.0, -1.0], 3), V))
    return (g5 @ sparse_D(U, m0, clover)).tocsr()
