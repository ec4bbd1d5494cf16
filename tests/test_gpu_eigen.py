"""GD-lambdaAMG eigensolver on the GPU against the eigenpair oracle."""
import numpy as np
import pytest

from gpu_common import case, dev, host, need_gpu
from helpers import rel_err
from oracle import clover as oclover
from oracle import dirac, eigen
from synth import random_links, random_spinors, seed_for

pytestmark = pytest.mark.gpu


def _run(dims, block, m0, ntv, nev, mmin, mmax, cfg, update=1, seed=4, nblk=1, l3=None):
    qmg = need_gpu()
    U = random_links(dims, 0.5, seed_for(cfg, "U"))
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, 1.0)
    W = lat.pack(dev(random_spinors(dims, ntv, seed_for(cfg, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    solve = {}
    if l3 is not None:
        ntv2, block2 = l3
        W2 = lat.level2_vectors_from(W, ntv2)
        lat.setup_level3(W2, ntv2, block2, setup_iters=2, smooth=2, l3_iters=8)
        solve = {"levels": 3, "coarse_maxiter": 3, "l3_iters": 8, "l2_smooth": 2}
    t0 = lat.pack(dev(random_spinors(dims, 1, seed_for(cfg, "x") + seed)))
    X = lat.field(nev)
    prm = qmg.default_eig_params(m_min=mmin, m_max=mmax, maxiter=3000, update_interp=update, block=nblk,
                                 solve=solve)
    st, lam, stats = lat.eigensolve(nev, X, t0, V0=W, n0=ntv, params=prm)
    return qmg, lat, U, st, lam, host(lat.unpack(X, nev)), stats


def _check_pairs(U, m0, lam, X, tol):
    C = oclover.clover_term(U, 1.0)
    k = len(lam)
    for i in range(k):
        r = dirac.apply_Q(U, X[i], m0, C) - lam[i] * X[i]
        assert np.linalg.norm(r) <= tol, (i, lam[i], np.linalg.norm(r))
    G = X.reshape(k, -1).conj() @ X.reshape(k, -1).T
    assert np.allclose(G, np.eye(k), atol=1e-9)


@pytest.mark.parametrize("nblk", [1, 4])
def test_eigensolve_4x4_matches_dense_oracle(nblk):
    """4^4 lattice, 2^4 blocks, clover, 8 test vectors: the locked eigenvalues are
    the oracle's smallest-modulus ones, with restarts (m_max = 20) on the way;
    one target per step and four targets solved as one multi-shift batch."""
    case("eigensolve 4^4 vs dense oracle, block %d" % nblk)
    dims, m0 = (4, 4, 4, 4), -0.5
    U = random_links(dims, 0.5, seed_for(9, "U"))
    ref, _ = eigen.smallest_eigenpairs(U, m0, oclover.clover_term(U, 1.0), 40)
    # pick nev at a clear gap in |lambda| so "the nev smallest" is unambiguous
    gaps = np.diff(np.abs(ref))
    nev = 10 + int(np.argmax(gaps[9:20] > 1e-3))
    qmg, lat, U2, st, lam, X, stats = _run(dims, (2, 2, 2, 2), m0, 8, nev, 10, 20, 9, nblk=nblk)
    assert st == 0 and stats["converged"] == nev, stats
    assert np.allclose(np.sort(lam), np.sort(ref[:nev]), atol=1e-9, rtol=0)
    _check_pairs(U, m0, lam, X, 1.1e-8)
    assert stats["interp_updates"] >= 1


@pytest.mark.parametrize("nblk", [1, 8])
def test_eigensolve_8x4_pairs_valid(nblk):
    """8^4 lattice, 4^4 blocks (the 4^4-block kernels), 4 test vectors so the
    interpolation is rebuilt from eigenvectors: every locked pair has residual
    <= 1e-8 under the oracle's operator and the vectors are orthonormal."""
    case("eigensolve 8^4 pairs, block %d" % nblk)
    dims, m0 = (8, 8, 8, 8), -0.5
    qmg, lat, U, st, lam, X, stats = _run(dims, (4, 4, 4, 4), m0, 4, 8, 10, 20, 10, nblk=nblk)
    assert st == 0 and stats["converged"] == 8, stats
    _check_pairs(U, m0, lam, X, 1.1e-8)
    assert stats["interp_updates"] >= 1


def test_eigensolve_three_level_inner_solves():
    """Correction equations solved with three levels, the third level rebuilt after
    every interpolation update (single-site level-2 aggregates on 4^4): the locked
    eigenvalues are the dense oracle's; on 8^4 with 2^4 aggregates every pair is valid."""
    case("eigensolve with three levels")
    dims, m0 = (4, 4, 4, 4), -0.5
    U = random_links(dims, 0.5, seed_for(9, "U"))
    ref, _ = eigen.smallest_eigenpairs(U, m0, oclover.clover_term(U, 1.0), 40)
    gaps = np.diff(np.abs(ref))
    nev = 10 + int(np.argmax(gaps[9:20] > 1e-3))
    qmg, lat, U2, st, lam, X, stats = _run(dims, (2, 2, 2, 2), m0, 8, nev, 10, 20, 9, l3=(4, (1, 1, 1, 1)))
    assert st == 0 and stats["converged"] == nev, stats
    assert np.allclose(np.sort(lam), np.sort(ref[:nev]), atol=1e-9, rtol=0)
    _check_pairs(U, m0, lam, X, 1.1e-8)
    assert stats["interp_updates"] >= 1
    assert lat.level3_shape() == (16, 8)
    dims = (8, 8, 8, 8)
    qmg, lat, U, st, lam, X, stats = _run(dims, (2, 2, 2, 2), m0, 8, 10, 10, 20, 10, l3=(8, (2, 2, 2, 2)))
    assert st == 0 and stats["converged"] == 10, stats
    _check_pairs(U, m0, lam, X, 1.1e-8)
    assert stats["interp_updates"] >= 1


def test_eigensolve_bad_arguments():
    case("eigensolve argument errors")
    qmg = need_gpu()
    dims = (4, 4, 4, 4)
    lat = qmg.Lattice(dims, (2, 2, 2, 2))
    lat.set_gauge(dev(random_links(dims, 0.5, 1)), -0.5, 0.0)
    X = lat.field(2)
    t0 = lat.field(1)
    with pytest.raises(qmg.QmgError) as e:
        lat.eigensolve(2, X, t0, params=qmg.default_eig_params(m_min=10, m_max=10))
    assert e.value.status == -1
    with pytest.raises(qmg.QmgError) as e:
        lat.eigensolve(2, X, t0, params=qmg.default_eig_params(m_min=10, m_max=20, block=11))
    assert e.value.status == -1
    with pytest.raises(qmg.QmgError) as e:
        lat.eigensolve(0, X, t0)
    assert e.value.status == -1
