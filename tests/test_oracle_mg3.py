"""Pins of the oracle's third multigrid level (aggregation of the block lattice)."""
import numpy as np
import pytest

from oracle import blocks as bl
from oracle import clover, dirac, mg, mg3
from oracle.solve import solve_shifted
from synth import random_links, random_spinors, random_test_vectors, seed_for


def _two_level(dims, block, ntv, csw=1.0, m0=-0.8, cfg=2):
    U = random_links(dims, 0.5, seed_for(cfg, "U"))
    op = dirac.Operator(U, m0, clover.clover_term(U, csw) if csw else None)
    W = list(random_test_vectors(dims, ntv, seed_for(cfg, "W")))
    return op, W, mg.TwoLevel(op, W, block)


def _level3(dims, block, ntv, block2, ntv2):
    op, W, two = _two_level(dims, block, ntv)
    dims2 = bl.nblocks(dims, block)
    W2 = mg3.initial_level2_vectors(two.P, W, block, ntv2)
    return op, W, two, dims2, W2, mg3.Level3(two.coarse, dims2, W2, block2)


def _dense(apply, n_sites, nc, tau=0.0, qform=False):
    """Matrix of a level operator by applying it to every unit vector."""
    n = n_sites * nc
    M = np.zeros((n, n), dtype=np.complex128)
    for c in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[c] = 1.0
        M[:, c] = apply(e.reshape(n_sites, nc), tau, qform).reshape(-1)
    return M


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_aggregate_index_map_brute_force():
    """to_aggregates2 against an explicit loop over level-2 sites."""
    dims2, block2, ntv = (4, 2, 6, 2), (2, 1, 3, 1), 3
    rng = np.random.default_rng(1)
    y = _rand(rng, (int(np.prod(dims2)), 2 * ntv))
    a = mg3.to_aggregates2(y, dims2, block2)
    nb3 = bl.nblocks(dims2, block2)
    for b, x in enumerate(np.ndindex(*dims2)):
        A = np.ravel_multi_index([x[mu] // block2[mu] for mu in range(4)], nb3)
        q = np.ravel_multi_index([x[mu] % block2[mu] for mu in range(4)], block2)
        for h in range(2):
            for i in range(ntv):
                assert a[A, h, q * ntv + i] == y[b, h * ntv + i]
    assert np.array_equal(mg3.from_aggregates2(a, dims2, block2, ntv), y)


def test_blocking_checks():
    with pytest.raises(ValueError):
        mg3.check_blocking3((4, 2, 2, 2), (2, 2, 1, 1))   # one aggregate in direction 1
    with pytest.raises(ValueError):
        mg3.check_blocking3((4, 4, 4, 4), (3, 1, 1, 1))   # does not divide
    mg3.check_blocking3((4, 2, 2, 2), (2, 1, 1, 1))


def test_P2_orthonormal_and_spans_test_vectors():
    op, W, two, dims2, W2, l3 = _level3((8, 4, 4, 4), (2, 2, 2, 2), 8, (2, 1, 1, 1), 4)
    P2 = l3.P2
    G = np.einsum("ahki,ahkj->ahij", np.conj(P2), P2)
    assert np.abs(G - np.eye(P2.shape[-1])).max() < 1e-13
    for w in W2:
        assert np.linalg.norm(l3.prolong(l3.restrict(w)) - w) < 1e-13 * np.linalg.norm(w)


def test_P2_keeps_coarse_chirality():
    """Gamma5^c P2 = P2 Gamma5^cc: prolonging a level-3 vector of one chirality
    gives a level-2 vector of that chirality only."""
    op, W, two, dims2, W2, l3 = _level3((8, 4, 4, 4), (2, 2, 2, 2), 8, (2, 1, 1, 1), 4)
    rng = np.random.default_rng(2)
    y3 = _rand(rng, (16, 8))
    lhs = mg.gamma5_coarse(l3.prolong(y3))
    rhs = l3.prolong(mg.gamma5_coarse(y3))
    assert np.abs(lhs - rhs).max() < 1e-14 * np.abs(lhs).max()


@pytest.mark.parametrize("qform", [False, True])
def test_galerkin_identity_level3(qform):
    """A3(tau) y = P2^H A_c(tau) P2 y for random y: pins the split of D_c by
    aggregate and the neighbour-block indexing of the level-3 stencil."""
    op, W, two, dims2, W2, l3 = _level3((8, 8, 4, 4), (2, 2, 2, 2), 8, (2, 2, 1, 1), 6)
    rng = np.random.default_rng(3)
    n3 = l3.P2.shape[0]
    for tau in (0.0, 0.13):
        y = _rand(rng, (n3, 12))
        got = l3.coarse3.apply(y, tau, qform)
        ref = l3.restrict(two.coarse.apply(l3.prolong(y), tau, qform))
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_level3_dense_triple_product_and_hermiticity():
    """D3 equals the dense P2^H D_c P2 entry by entry; Gamma5^cc D3 is Hermitian."""
    op, W, two, dims2, W2, l3 = _level3((8, 4, 4, 4), (2, 2, 2, 2), 8, (2, 1, 1, 1), 4)
    n2, n3 = int(np.prod(dims2)), l3.P2.shape[0]
    D2 = _dense(two.coarse.apply, n2, 16)
    P2d = np.zeros((n2 * 16, n3 * 8), dtype=np.complex128)
    for c in range(n3 * 8):
        e = np.zeros(n3 * 8, dtype=np.complex128)
        e[c] = 1.0
        P2d[:, c] = l3.prolong(e.reshape(n3, 8)).reshape(-1)
    D3 = _dense(l3.coarse3.apply, n3, 8)
    assert np.abs(D3 - np.conj(P2d.T) @ D2 @ P2d).max() < 1e-13 * np.abs(D3).max()
    Q3 = _dense(l3.coarse3.apply, n3, 8, 0.0, True)
    assert np.abs(Q3 - np.conj(Q3.T)).max() < 1e-13 * np.abs(Q3).max()


def test_full_rank_single_site_aggregates_are_similar():
    """Aggregates of one level-2 site with ntv2 = ntv make P2 unitary per site and
    chirality, so D3 is unitarily similar to D_c: equal spectra."""
    op, W, two, dims2, W2, _ = _level3((4, 4, 4, 4), (2, 2, 2, 2), 4, (1, 1, 1, 1), 4)
    rng = np.random.default_rng(6)
    W2 = [_rand(rng, (16, 8)) for _ in range(4)]
    l3 = mg3.Level3(two.coarse, dims2, W2, (1, 1, 1, 1))
    D2 = _dense(two.coarse.apply, 16, 8, 0.05)
    D3 = _dense(l3.coarse3.apply, 16, 8, 0.05)
    e2 = list(np.linalg.eigvals(D2))
    e3 = np.linalg.eigvals(D3)
    # match each eigenvalue of D3 to the nearest unmatched one of D_c
    worst = 0.0
    for ev in e3:
        i = int(np.argmin([abs(ev - x) for x in e2]))
        worst = max(worst, abs(ev - e2.pop(i)))
    assert worst < 1e-11 * np.abs(e3).max()


def test_level2_cycle_with_exact_level3_solve():
    """k3 = level-3 dimension (GMRES exact) and no level-2 smoothing:
    M2 r = P2 A3^{-1} P2^H r."""
    op, W, two, dims2, W2, l3 = _level3((8, 4, 4, 4), (2, 2, 2, 2), 8, (2, 1, 1, 1), 4)
    n3 = l3.P2.shape[0]
    rng = np.random.default_rng(7)
    r2 = _rand(rng, (int(np.prod(dims2)), 16))
    tau = 0.02
    A3 = _dense(l3.coarse3.apply, n3, 8, tau)
    y3 = np.linalg.solve(A3, l3.restrict(r2).reshape(-1)).reshape(n3, 8)
    got = l3.cycle(r2, tau, n3 * 8, 0)
    ref = l3.prolong(y3)
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()


def test_level2_fgmres_reaches_dense_solution():
    """Enough K-cycle steps solve A_c(tau) y = r to the dense solution."""
    op, W, two, dims2, W2, l3 = _level3((8, 4, 4, 4), (2, 2, 2, 2), 4, (2, 1, 1, 1), 4)
    n2 = int(np.prod(dims2))
    rng = np.random.default_rng(8)
    r2 = _rand(rng, (n2, 8))
    tau = -0.03
    A2 = _dense(two.coarse.apply, n2, 8, tau)
    ref = np.linalg.solve(A2, r2.reshape(-1))
    y = l3.solve(r2, tau, 60, 10, 2)
    res = np.linalg.norm(A2 @ y.reshape(-1) - r2.reshape(-1)) / np.linalg.norm(r2)
    assert res < 1e-10
    assert np.linalg.norm(y.reshape(-1) - ref) < 1e-8 * np.linalg.norm(ref)


def test_three_level_solve_matches_two_level():
    """FGMRES with the three-level V-cycle reaches 1e-10 (true residual by the
    operator itself) and the same solution as the two-level solve."""
    dims, block = (8, 8, 8, 8), (2, 2, 2, 2)
    op, W, two = _two_level(dims, block, 8)
    dims2 = bl.nblocks(dims, block)
    W2 = mg3.initial_level2_vectors(two.P, W, block, 8)
    three = mg3.ThreeLevel(op, W, block, W2, (2, 2, 2, 2), k3=12, s2=2)
    b = random_spinors(dims, 1, seed_for(2, "b"))[0]
    tau = 0.01
    x3, it3, h3 = solve_shifted(op, b, tau, block, three, restart=8, maxiter=200, coarse_iters=4)
    x2, it2, h2 = solve_shifted(op, b, tau, block, two, restart=8, maxiter=200, coarse_iters=50)
    for x in (x3, x2):
        r = dirac.apply_Q_shifted(op.U, x, op.m0, tau, op.clover) - b
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x3 - x2) < 1e-7 * np.linalg.norm(x2)
    assert it3 < 60


def test_setup_improves_level2_vectors():
    """Inverse iteration with M2 at tau = 0 moves the level-2 test vectors towards
    the small singular vectors of A_c: their mean ||A_c w|| / ||w|| drops with
    every setup round, and stays above the smallest singular value."""
    op, W, two, dims2, W2, _ = _level3((8, 4, 4, 4), (2, 2, 2, 2), 8, (2, 1, 1, 1), 4)

    def rq(ws):
        return np.mean([np.linalg.norm(two.coarse.apply(w, 0.0)) / np.linalg.norm(w) for w in ws])

    smin = np.linalg.svd(_dense(two.coarse.apply, int(np.prod(dims2)), 16), compute_uv=False)[-1]
    prev = rq(W2)
    for iters in (2, 3, 4):
        W2s = mg3.setup_level3(two.coarse, dims2, W2, (2, 1, 1, 1), setup_iters=iters, s2=2, k3=10)
        assert all(abs(np.linalg.norm(w) - 1.0) < 1e-13 for w in W2s)
        cur = rq(W2s)
        assert smin <= cur < prev
        prev = cur
