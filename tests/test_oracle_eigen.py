"""Pins of the eigenpair oracle and of the library's host Hermitian eigensolver."""
import numpy as np
import pytest

from oracle import clover as oclover
from oracle import dirac
from oracle import eigen
from synth import random_links, seed_for, unit_links


def test_free_field_spectrum_closed_form():
    """U = 1 on 4^4: the dense spectrum equals the momentum-space closed form."""
    dims, m0 = (4, 4, 4, 4), -0.5
    U = unit_links(dims)
    lam, _ = eigen.smallest_eigenpairs(U, m0, None, 12 * 256)
    assert np.allclose(np.sort(lam), eigen.free_spectrum(dims, m0), atol=1e-12)


def test_smallest_pairs_are_eigenpairs_of_the_matrix_free_operator():
    """Random links with clover on 2^4 x 4: residuals through oracle.dirac (the
    matrix-free code, independent of the dense assembly), orthonormality, and
    ordering by modulus with nothing smaller left out."""
    dims = (2, 2, 2, 4)
    U = random_links(dims, 0.5, seed_for(8, "U"))
    C = oclover.clover_term(U, 1.0)
    lam, X = eigen.smallest_eigenpairs(U, -0.5, C, 10)
    for k in range(10):
        r = dirac.apply_Q(U, X[k], -0.5, C) - lam[k] * X[k]
        assert np.linalg.norm(r) < 1e-12
    G = X.reshape(10, -1).conj() @ X.reshape(10, -1).T
    assert np.allclose(G, np.eye(10), atol=1e-12)
    assert np.all(np.diff(np.abs(lam)) >= 0)
    allw = np.linalg.eigvalsh(eigen.dense.dense_Q(U, -0.5, C))
    assert np.abs(lam[-1]) <= np.sort(np.abs(allw))[10] + 1e-14


@pytest.mark.parametrize("m", [1, 2, 7, 33])
def test_host_hermitian_eig_matches_lapack(m):
    """The library's host Jacobi eigensolver (used for the harmonic Ritz pencil)
    against LAPACK on random Hermitian matrices and one with repeated
    eigenvalues; pure host code, no device."""
    from paper_2004_08146_amd import qmg
    rng = np.random.default_rng(m)
    a = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    a = a + a.conj().T
    w, z = qmg.hermitian_eig(a)
    assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-12 * max(1.0, np.abs(w).max()))
    assert np.linalg.norm(a @ z - z * w) < 1e-12 * np.linalg.norm(a)
    assert np.allclose(z.conj().T @ z, np.eye(m), atol=1e-12)
    if m >= 7:
        q, _ = np.linalg.qr(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)))
        d = np.repeat([1.0, -2.0, 3.0], [3, 2, m - 5]).astype(complex)
        b = (q * d) @ q.conj().T
        w, z = qmg.hermitian_eig(b)
        assert np.allclose(w, np.sort(d.real), atol=1e-12)
        assert np.linalg.norm(b @ z - z * w) < 1e-12


def test_sparse_lanczos_eigenpairs_match_dense():
    """The Lanczos route for large lattices (eigsh on Q^2, then Rayleigh-Ritz of Q on
    the span) against the dense definition on 4^4 with random links and clover:
    the same eigenvalues, and pairs that are eigenpairs of the matrix-free oracle
    operator, orthonormal."""
    dims, m0 = (4, 4, 4, 4), -0.5
    U = random_links(dims, 0.5, seed_for(9, "U"))
    C = oclover.clover_term(U, 1.0)
    ref, _ = eigen.smallest_eigenpairs(U, m0, C, 24)
    lam, X = eigen.smallest_eigenpairs_sparse(U, m0, C, 20)
    assert np.allclose(lam, ref[:20], atol=1e-11, rtol=0)
    for k in range(20):
        r = dirac.apply_Q(U, X[k], m0, C) - lam[k] * X[k]
        assert np.linalg.norm(r) < 1e-10
    G = X.reshape(20, -1).conj() @ X.reshape(20, -1).T
    assert np.allclose(G, np.eye(20), atol=1e-11)
