"""Lattice blocks (Schwarz domains / aggregates) and their red-black colouring.

A block is a B0 x B1 x B2 x B3 sub-lattice; block coordinates are
X_mu = floor(x_mu / B_mu) and the colour of a block is (sum_mu X_mu) mod 2
(red-black ordering of the Schwarz domains, Sec. 2, text after eq. (2.10), the SAP error
propagator).  Blocks are numbered lexicographically,
b = ((X0*NB1 + X1)*NB2 + X2)*NB3 + X3, and sites inside a block likewise.
"""
import numpy as np


def check_blocking(dims, block):
    for n, b in zip(dims, block):
        if n % b:
            raise ValueError("block does not divide lattice")
        if (n // b) % 2 or n // b < 2:
            raise ValueError("need an even number (>= 2) of blocks per direction")


def nblocks(dims, block):
    return tuple(n // b for n, b in zip(dims, block))


def coords(dims):
    """Integer coordinate arrays x_mu[N0, N1, N2, N3]."""
    return np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")


def site_colour(dims, block):
    x = coords(dims)
    return sum(x[mu] // block[mu] for mu in range(4)) % 2


def inner_forward(dims, block, mu):
    """True where x + mu lies in the same block as x."""
    return (coords(dims)[mu] % block[mu]) != block[mu] - 1


def inner_backward(dims, block, mu):
    """True where x - mu lies in the same block as x."""
    return (coords(dims)[mu] % block[mu]) != 0


def block_reduce(f, dims, block):
    """Sum a per-site scalar (or [..., 4, 3] field) over each block -> [NB0..NB3]."""
    nb = nblocks(dims, block)
    shp = []
    for n, b in zip(nb, block):
        shp += [n, b]
    g = f.reshape(tuple(shp) + f.shape[4:])
    axes = (1, 3, 5, 7) + tuple(range(8, g.ndim))
    return g.sum(axis=axes)


def block_expand(a, block):
    """Per-block array [NB0..NB3] -> per-site array [N0..N3]."""
    out = a
    for mu in range(4):
        out = np.repeat(out, block[mu], axis=mu)
    return out


def neighbour_table(dims, block):
    """nbr[b, d]: d = 0 self, 1 + 2 mu block at X + mu, 2 + 2 mu block at X - mu."""
    nb = nblocks(dims, block)
    n = int(np.prod(nb))
    tab = np.zeros((n, 9), dtype=np.int64)
    for b, X in enumerate(np.ndindex(*nb)):
        tab[b, 0] = b
        for mu in range(4):
            for d, s in ((1 + 2 * mu, 1), (2 + 2 * mu, -1)):
                Y = list(X)
                Y[mu] = (Y[mu] + s) % nb[mu]
                tab[b, d] = np.ravel_multi_index(Y, nb)
    return tab
