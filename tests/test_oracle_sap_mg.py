"""Pins of the oracle's SAP smoother, multigrid pieces and Krylov solvers."""
import json
import os

import numpy as np
import pytest

from oracle import blocks as bl
from oracle import clover, dense, dirac, krylov, mg, sap
from oracle.solve import solve_shifted
from synth import random_links, random_spinors, random_test_vectors, seed_for

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _op(dims, eps=0.3, m0=-0.5, csw=0.0, cfg=1):
    U = random_links(dims, eps, seed_for(cfg, "U"))
    C = clover.clover_term(U, csw) if csw else None
    return dirac.Operator(U, m0, C)


def _block_index_sets(dims, block):
    nb = bl.nblocks(dims, block)
    x = bl.coords(dims)
    bid = np.ravel_multi_index([x[mu] // block[mu] for mu in range(4)], nb).reshape(-1)
    colour = bl.site_colour(dims, block).reshape(-1)
    sets = []
    for b in range(int(np.prod(nb))):
        sites = np.nonzero(bid == b)[0]
        dof = (12 * sites[:, None] + np.arange(12)[None, :]).reshape(-1)
        sets.append((int(colour[sites[0]]), dof))
    return sets


def _dense_sap(A, f, x, sets, nsweep):
    """Textbook multiplicative Schwarz on a dense matrix, colour 0 blocks first."""
    x = x.copy()
    for _ in range(nsweep):
        for c in (0, 1):
            r = f - A @ x
            for col, dof in sets:
                if col == c:
                    x[dof] += np.linalg.solve(A[np.ix_(dof, dof)], r[dof])
    return x


def test_block_operator_is_dense_block_restriction():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _op(dims, csw=1.0)
    tau = 0.07
    A = dense.dense_D(op.U, op.m0, op.clover) - tau * dense.dense_gamma5(256)
    psi = random_spinors(dims, 1, 5)[0]
    out = sap.block_operator(op, psi, tau, block).reshape(-1)
    ref = np.zeros_like(out)
    v = psi.reshape(-1)
    for _, dof in _block_index_sets(dims, block):
        ref[dof] = A[np.ix_(dof, dof)] @ v[dof]
    assert np.abs(out - ref).max() < 1e-13


def test_proposition1_sap_Q_equals_sap_D():
    """Proposition 1: with exact block solves, SAP on Q gives the same iterates as SAP on D."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _op(dims)
    f = random_spinors(dims, 1, 11)[0]
    x0 = random_spinors(dims, 1, 12)[0]
    xD = sap.sap_exact(op, f, x0, 0.0, block, 2)
    Qd = dense.dense_Q(op.U, op.m0)
    sets = _block_index_sets(dims, block)
    g5f = dirac.gamma5(f).reshape(-1)
    xQ = _dense_sap(Qd, g5f, x0.reshape(-1), sets, 2)
    assert np.abs(xD.reshape(-1) - xQ).max() < 1e-12 * np.abs(xQ).max()


def test_mr_sap_tends_to_exact_sap():
    """Many MR steps per block reproduce the exact block solves."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _op(dims, m0=0.5)
    f = random_spinors(dims, 1, 11)[0]
    x0 = np.zeros_like(f)
    xe = sap.sap_exact(op, f, x0, 0.1, block, 1)
    xm = sap.sap(op, f, x0, 0.1, block, 1, 60)
    assert np.abs(xm - xe).max() < 1e-10 * np.abs(xe).max()


def test_mr_residual_monotone():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _op(dims, csw=1.0)
    r = random_spinors(dims, 1, 13)[0]
    prev = None
    for n in range(0, 6):
        e = sap.block_mr(op, r, 0.05, block, n)
        res = r - sap.block_operator(op, e, 0.05, block)
        norms = bl.block_reduce(np.sum(np.abs(res) ** 2, axis=(-2, -1)), dims, block)
        if prev is not None:
            assert np.all(norms <= prev * (1 + 1e-12))
        prev = norms


def test_sap_as_stationary_solver():
    """For a well-conditioned operator, repeated SAP sweeps converge to A^{-1} f."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _op(dims, m0=1.0)
    tau = 0.2
    f = random_spinors(dims, 1, 14)[0]
    A = dense.dense_D(op.U, op.m0) - tau * dense.dense_gamma5(256)
    xs = np.linalg.solve(A, f.reshape(-1)).reshape(f.shape)
    x = sap.sap(op, f, np.zeros_like(f), tau, block, 25, 4)
    assert np.abs(x - xs).max() < 1e-8 * np.abs(xs).max()


def test_block_colouring_rejects_bad_blocking():
    with pytest.raises(ValueError):
        bl.check_blocking((4, 4, 4, 4), (4, 2, 2, 2))     # one block in direction 0
    with pytest.raises(ValueError):
        bl.check_blocking((6, 4, 4, 4), (2, 2, 2, 2))     # 3 blocks: odd
    bl.check_blocking((8, 4, 4, 4), (2, 2, 2, 2))


def test_aggregate_layout_roundtrip():
    dims, block = (4, 8, 4, 4), (2, 4, 2, 2)
    psi = random_spinors(dims, 1, 3)[0]
    a = mg.to_aggregates(psi, block)
    assert a.shape == (2 * 2 * 2 * 2, 2, 32 * 6)
    assert np.array_equal(mg.from_aggregates(a, dims, block), psi)
    # explicit element: site x = (3, 5, 0, 1) is in block X = (1, 1, 0, 0), local (1, 1, 0, 1)
    x, X, loc = (3, 5, 0, 1), (1, 1, 0, 0), (1, 1, 0, 1)
    b = ((X[0] * 2 + X[1]) * 2 + X[2]) * 2 + X[3]
    ls = ((loc[0] * 4 + loc[1]) * 2 + loc[2]) * 2 + loc[3]
    for s in range(4):
        for c in range(3):
            assert a[b, s // 2, ls * 6 + (s % 2) * 3 + c] == psi[x + (s, c)]


def test_paper_dimension_counts():
    with open(GOLDEN) as f:
        g = json.load(f)
    c = g["counts_4x4"]
    dims, block = tuple(c["dims"]), tuple(c["block"])
    W = random_test_vectors(dims, c["ntv"], 4)
    P = mg.build_P(list(W), block)
    nagg = P.shape[0] * P.shape[1]
    assert nagg * c["ntv"] == c["coarse_dim"]
    assert P.shape[0] * P.shape[1] * P.shape[2] == c["fine_dim"]
    assert abs(c["coarse_dim"] / c["fine_dim"] - c["expected_lc2"]) < 1e-15
    c = g["counts_64x32"]
    nb = bl.nblocks(c["dims"], c["block"])
    assert 2 * int(np.prod(nb)) == c["aggregates"]
    assert 12 * int(np.prod(c["dims"])) == c["fine_dim"]


def _small_mg(dims=(4, 4, 4, 4), block=(2, 2, 2, 2), ntv=6, csw=1.0, m0=-0.5):
    op = _op(dims, csw=csw, m0=m0)
    W = list(random_test_vectors(dims, ntv, seed_for(1, "W")))
    return op, W, mg.TwoLevel(op, W, block)


def _dense_P(P, dims, block):
    nbt, _, _, ntv = P.shape
    V = int(np.prod(dims))
    cols = []
    for c in range(2 * ntv):
        y = np.zeros((nbt, 2 * ntv), dtype=np.complex128)
        y[:, c] = 1.0
        cols.append(mg.prolong(P, y, dims, block).reshape(-1))
    # column (b, c) of the dense P = column c restricted to block b
    Pd = np.zeros((12 * V, nbt * 2 * ntv), dtype=np.complex128)
    nb = bl.nblocks(dims, block)
    x = bl.coords(dims)
    bid = np.ravel_multi_index([x[mu] // block[mu] for mu in range(4)], nb).reshape(-1)
    dof_block = np.repeat(bid, 12)
    for b in range(nbt):
        for c in range(2 * ntv):
            Pd[:, b * 2 * ntv + c] = np.where(dof_block == b, cols[c], 0.0)
    return Pd


def test_P_orthonormal_spin_preserving_and_spans_W():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op, W, h = _small_mg(dims, block)
    P = h.P
    G = np.einsum("bhki,bhkj->bhij", np.conj(P), P)
    assert np.abs(G - np.eye(P.shape[-1])).max() < 1e-14
    # Gamma5 P = P Gamma5^c (text before eq. (2.9))
    y = random_spinors((1, 1, 1, 1), 1, 9)[0].reshape(-1)[:1] * np.ones((P.shape[0], 2 * P.shape[-1]))
    y = y + 0.3j * np.arange(y.size).reshape(y.shape)
    lhs = dirac.gamma5(mg.prolong(P, y, dims, block))
    rhs = mg.prolong(P, mg.gamma5_coarse(y), dims, block)
    assert np.abs(lhs - rhs).max() < 1e-14
    # range(P) contains the test vectors: P P^H w = w
    for w in W:
        back = mg.prolong(P, mg.restrict(P, w, block), dims, block)
        assert np.abs(back - w).max() < 1e-13 * np.abs(w).max()
    # lc of a random vector ~ sqrt(coarse_dim / fine_dim) (footnote of Sec. 3.1)
    v = random_spinors(dims, 1, 17)[0]
    lc = np.linalg.norm(mg.prolong(P, mg.restrict(P, v, block), dims, block)) / np.linalg.norm(v)
    assert abs(lc ** 2 - 2 * 6 * 16 / 3072) < 0.02


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)),
                                        ((8, 4, 2, 2), (2, 2, 1, 1))])
def test_coarse_operator_equals_dense_galerkin(dims, block):
    op, W, h = _small_mg(dims, block, ntv=4)
    V = int(np.prod(dims))
    Pd = _dense_P(h.P, dims, block)
    Dd = dense.dense_D(op.U, op.m0, op.clover)
    Dcd = Pd.conj().T @ Dd @ Pd
    nc = 2 * h.P.shape[-1]
    Dc, nbr = h.coarse.Dc, h.coarse.nbr
    nbt = Dc.shape[0]
    ref = np.zeros_like(Dcd)
    for b in range(nbt):
        for d in range(9):
            bb = nbr[b, d]
            ref[b * nc:(b + 1) * nc, bb * nc:(bb + 1) * nc] += Dc[b, d]
    assert np.abs(ref - Dcd).max() < 1e-13 * np.abs(Dcd).max()
    assert V * 12 == Pd.shape[0]
    # Q_c = Gamma5^c D_c is Hermitian (text before eq. (2.9))
    g5c = np.kron(np.eye(nbt), np.diag([1.0] * (nc // 2) + [-1.0] * (nc // 2)))
    Qc = g5c @ ref
    assert np.abs(Qc - Qc.conj().T).max() < 1e-13


def test_coarse_grid_identity_eq29():
    """eq. (2.9): I - P Q_c^{-1} P^H Q = I - P D_c^{-1} P^H D."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op, W, h = _small_mg(dims, block, ntv=4)
    Pd = _dense_P(h.P, dims, block)
    Dd = dense.dense_D(op.U, op.m0, op.clover)
    g5 = dense.dense_gamma5(256)
    Dc = Pd.conj().T @ Dd @ Pd
    Qc = Pd.conj().T @ g5 @ Pd @ Dc
    lhs = Pd @ np.linalg.solve(Qc, Pd.conj().T @ g5 @ Dd)
    rhs = Pd @ np.linalg.solve(Dc, Pd.conj().T @ Dd)
    assert np.abs(lhs - rhs).max() < 1e-11


def test_coarse_shift_fold():
    """P^H (D - tau Gamma5) P y = (D_c - tau Gamma5^c) y when P^H P = I."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op, W, h = _small_mg(dims, block)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((16, 12)) + 1j * rng.standard_normal((16, 12))
    tau = 0.13
    fine = mg.restrict(h.P, op.A(mg.prolong(h.P, y, dims, block), tau), block)
    assert np.abs(h.coarse.apply(y, tau) - fine).max() < 1e-13 * np.abs(fine).max()


def test_gmres_small_dense():
    rng = np.random.default_rng(1)
    n = 30
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, k, est = krylov.gmres(lambda v: A @ v, b, n)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-11
    # residual estimate equals the true residual and decreases with k
    prev = np.inf
    for k in range(1, 12):
        x, _, est = krylov.gmres(lambda v: A @ v, b, k)
        true = np.linalg.norm(b - A @ x)
        assert abs(true - est) < 1e-10 * np.linalg.norm(b)
        assert true <= prev + 1e-12
        prev = true
    x, k, est = krylov.gmres(lambda v: A @ v, b, n, tol=0.5)
    assert est <= 0.5 * np.linalg.norm(b) and k < n


def test_fgmres_identity_preconditioner_is_gmres():
    rng = np.random.default_rng(2)
    n = 40
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x1, _, _ = krylov.fgmres(lambda v: A @ v, lambda v: v, b, 1e-14, 7, 7)
    x2, _, _ = krylov.gmres(lambda v: A @ v, b, 7)
    assert np.abs(x1 - x2).max() < 1e-12 * np.abs(x2).max()
    x, it, hist = krylov.fgmres(lambda v: A @ v, lambda v: v, b, 1e-10, 10, 400)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)


def test_vcycle_exact_coarse_no_smoothing():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op, W, h = _small_mg(dims, block, ntv=4)
    tau = 0.05
    r = random_spinors(dims, 1, 21)[0]
    z = h.vcycle(r, tau, 0, 3, 16 * 8)
    Pd = _dense_P(h.P, dims, block)
    A = dense.dense_D(op.U, op.m0, op.clover) - tau * dense.dense_gamma5(256)
    Ac = Pd.conj().T @ A @ Pd
    ref = Pd @ np.linalg.solve(Ac, Pd.conj().T @ r.reshape(-1))
    assert np.abs(z.reshape(-1) - ref).max() < 1e-9 * np.abs(ref).max()


def test_shifted_solve_matches_dense():
    """FGMRES + SAP and FGMRES + two-level MG both reach 1e-10 and agree with a dense solve;
    with near-null eigenvectors as test vectors the coarse level cuts the iteration count."""
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    op, _, _ = _small_mg(dims, block, ntv=6, m0=-0.3)
    tau = 0.05
    Qd = dense.dense_Q(op.U, op.m0, op.clover)
    w, v = np.linalg.eigh(Qd)
    W = [v[:, i].reshape(dims + (4, 3)) for i in np.argsort(np.abs(w))[:8]]
    h = mg.TwoLevel(op, W, block)
    b = random_spinors(dims, 1, seed_for(1, "b"))[0]
    Qs = Qd - tau * np.eye(3072)
    xs = np.linalg.solve(Qs, b.reshape(-1))
    kappa = np.linalg.cond(Qs)
    its = []
    for hier in (None, h):
        x, it, hist = solve_shifted(op, b, tau, block, mg=hier, tol=1e-10, restart=20,
                                    maxiter=400, coarse_iters=30)
        res = np.linalg.norm(b.reshape(-1) - Qs @ x.reshape(-1)) / np.linalg.norm(b)
        assert res <= 1e-10 * 1.0001 and hist[-1] <= 1e-10
        assert np.linalg.norm(x.reshape(-1) - xs) <= kappa * 1e-10 * np.linalg.norm(xs)
        its.append(it)
    assert its[1] < its[0] / 2


def test_local_coherence_pins():
    """lc(v) = ||Pi v|| / ||v|| (Sec. 3.1): 1 on the test vectors, <= 1 always, the
    dense projector P P^H gives the same values, and for Gaussian vectors the
    mean of lc^2 is rank(P) / N (0.25 for 4^4 with 2^4 aggregates and 24 test
    vectors, the no-coherence value the paper quotes)."""
    from oracle import mg
    from synth import random_spinors
    dims, block, ntv = (4, 4, 4, 4), (2, 2, 2, 2), 24
    W = random_spinors(dims, ntv, 3)
    P = mg.build_P(W, block)
    for w in W[:4]:
        assert abs(mg.local_coherence(P, w, block) - 1.0) < 1e-12
    V = random_spinors(dims, 64, 5)
    lc = np.array([mg.local_coherence(P, v, block) for v in V])
    assert np.all(lc <= 1.0 + 1e-12)
    N = V[0].size
    assert abs(np.mean(lc ** 2) - 768 / 3072) < 0.01
    # dense projector from the prolongations of the coarse unit vectors
    nb = np.prod([d // b for d, b in zip(dims, block)])
    cols = []
    for i in range(nb * 2 * ntv):
        y = np.zeros(nb * 2 * ntv, dtype=np.complex128)
        y[i] = 1.0
        cols.append(mg.prolong(P, y.reshape(nb, 2 * ntv), dims, block).ravel())
    Pd = np.array(cols).T
    assert np.allclose(Pd.conj().T @ Pd, np.eye(Pd.shape[1]), atol=1e-12)
    for v, l in zip(V[:8], lc[:8]):
        x = v.ravel()
        assert abs(np.linalg.norm(Pd @ (Pd.conj().T @ x)) / np.linalg.norm(x) - l) < 1e-12
    assert N == Pd.shape[0]


def test_qform_sap_exact_equals_gamma5_form():
    """Sec. 2: with exact block solves SAP for Q - tau and for D - tau Gamma5 have
    the same error propagation, so (Q - tau) x = f and (D - tau Gamma5) x =
    Gamma5 f give the same iterates."""
    from oracle.dirac import Operator, gamma5
    from oracle import sap as osap
    from oracle import clover as oclover
    from synth import random_links, random_spinors
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = random_links(dims, 0.5, 21)
    op = Operator(U, -0.5, oclover.clover_term(U, 1.0))
    f = random_spinors(dims, 1, 22)[0]
    x0 = random_spinors(dims, 1, 23)[0]
    xq = osap.sap_exact(op, f, x0, 0.13, block, 2, qform=True)
    xa = osap.sap_exact(op, gamma5(f), x0, 0.13, block, 2)
    assert np.linalg.norm(xq - xa) < 1e-12 * np.linalg.norm(xa)


def test_qform_coarse_is_galerkin_of_Q():
    """Gamma5^c (D_c - tau Gamma5^c) = P^H (Q - tau) P, with Q - tau applied
    matrix-free (the coarse matrix is assembled independently)."""
    from oracle.dirac import Operator, gamma5
    from oracle import mg
    from oracle import clover as oclover
    from synth import random_links, random_spinors
    dims, block, ntv = (4, 4, 4, 4), (2, 2, 2, 2), 6
    U = random_links(dims, 0.5, 24)
    op = Operator(U, -0.5, oclover.clover_term(U, 1.0))
    h = mg.TwoLevel(op, random_spinors(dims, ntv, 25), block)
    nb = h.P.shape[0]
    rng = np.random.default_rng(26)
    y = rng.standard_normal((nb, 2 * ntv)) + 1j * rng.standard_normal((nb, 2 * ntv))
    tau = -0.21
    got = h.coarse.apply(y, tau, qform=True)
    ref = mg.restrict(h.P, gamma5(op.A(mg.prolong(h.P, y, dims, block), tau)), block)
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_qform_solve_same_solution():
    """Both forms solve the same system: (Q - tau) x = b to 1e-10."""
    from oracle.dirac import Operator
    from oracle import mg, solve
    from oracle import clover as oclover
    from synth import random_links, random_spinors
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = random_links(dims, 0.5, 27)
    op = Operator(U, -0.5, oclover.clover_term(U, 1.0))
    h = mg.TwoLevel(op, random_spinors(dims, 8, 28), block)
    b = random_spinors(dims, 1, 29)[0]
    xa, ita, ha = solve.solve_shifted(op, b, 0.05, block, h, tol=1e-10, restart=10, maxiter=800)
    xq, itq, hq = solve.solve_shifted(op, b, 0.05, block, h, tol=1e-10, restart=10, maxiter=800, qform=True)
    assert ha[-1] <= 1e-10 and hq[-1] <= 1e-10
    assert np.linalg.norm(xq - xa) < 1e-7 * np.linalg.norm(xa)
    # Sec. 3.3: with approximate (MR) block solves multigrid for Q itself is far
    # slower than for the Gamma5-preconditioned form (here 10 vs 361 iterations)
    assert itq > 4 * ita, (ita, itq)


class _FineOnly:
    """Holds only the fine operator: the GMRES branch of TwoLevel.post_smooth
    uses nothing else of the hierarchy."""

    def __init__(self, op, block):
        self.op = op
        self.block = tuple(block)


def _dense_A(op, tau, qform):
    V = int(np.prod(op.dims))
    A = dense.dense_D(op.U, op.m0, op.clover) - tau * dense.dense_gamma5(V)
    return dense.dense_gamma5(V) @ A if qform else A


def test_gmres_smoother_full_dimension_is_exact():
    """GMRES smoothing (Sec. 2, the alternative to SAP) solves the residual equation
    A e = r - A z; with as many steps as unknowns that solve is exact, so the smoothed
    iterate is A^{-1} r whatever z it starts from (both operator forms).  A sign slip
    in the residual (A z - r) or in the update (z - e) fails this."""
    dims = (2, 2, 2, 2)
    op = _op(dims, m0=0.5, csw=1.0)
    tau = 0.1
    r = random_spinors(dims, 1, 31)[0]
    z0 = random_spinors(dims, 1, 32)[0]
    for qform in (False, True):
        xs = np.linalg.solve(_dense_A(op, tau, qform), r.reshape(-1))
        for z_start in (np.zeros_like(z0), z0):
            z = mg.TwoLevel.post_smooth(_FineOnly(op, (1, 1, 1, 1)), r, z_start, tau, 192, 3, qform,
                                        "gmres")
            assert np.abs(z.reshape(-1) - xs).max() < 1e-10 * np.abs(xs).max()


def test_gmres_smoother_minimises_over_krylov_space():
    """nu GMRES smoothing steps give z + e with e the element of the Krylov space
    K_nu(A, s), s = r - A z, that minimises ||s - A e||: the same as a dense
    least-squares solve over an explicitly built basis of that space."""
    dims = (4, 4, 4, 2)
    op = _op(dims, csw=1.0)
    tau = 0.05
    r = random_spinors(dims, 1, 33)[0]
    z0 = random_spinors(dims, 1, 34)[0]
    fine = _FineOnly(op, (2, 2, 2, 1))
    for qform in (False, True):
        A = _dense_A(op, tau, qform)
        s = r.reshape(-1) - A @ z0.reshape(-1)
        for nu in (1, 3, 6):
            K = [s]
            for _ in range(nu - 1):
                K.append(A @ K[-1])
            Qk, _ = np.linalg.qr(np.stack(K, axis=1))
            c = np.linalg.lstsq(A @ Qk, s, rcond=None)[0]
            ref = z0.reshape(-1) + Qk @ c
            z = mg.TwoLevel.post_smooth(fine, r, z0, tau, nu, 3, qform, "gmres")
            assert np.abs(z.reshape(-1) - ref).max() < 1e-10 * np.abs(ref).max()
            # and the residual really went down
            assert np.linalg.norm(r.reshape(-1) - A @ z.reshape(-1)) < np.linalg.norm(s)


def test_setup_test_vectors_inverse_iteration():
    """The adaptive-setup reading (Sec. 4 parameter table: test vectors, setup
    iterations, smoothing steps): W is smoothed on A_0 w = 0 and then improved by
    V-cycle inverse iteration at tau = 0.  The vectors come back normalised; their
    mean ||A_0 w|| / ||w|| falls with every setup round and stays above the smallest
    singular value of A_0; and the final interpolation represents the eigenvectors
    of Q of smallest |lambda| better than random test vectors do (local coherence,
    Sec. 3.1), which is what the setup is for."""
    dims, block = (4, 4, 4, 2), (2, 2, 2, 1)
    op = _op(dims, csw=1.0, m0=-0.5)
    ntv = 6
    W0 = [w / np.linalg.norm(w) for w in random_test_vectors(dims, ntv, seed_for(1, "W"))]
    V = int(np.prod(dims))
    smin = np.linalg.svd(_dense_A(op, 0.0, False), compute_uv=False)[-1]

    def rq(ws):
        return np.mean([np.linalg.norm(op.A(w, 0.0)) / np.linalg.norm(w) for w in ws])

    prev = rq(W0)
    W = W0
    for iters in (1, 2, 3, 4):
        W = mg.setup_test_vectors(op, W0, block, setup_iters=iters, smooth=2, n_mr=3, coarse_iters=20,
                                  coarse_tol=0.5)
        assert len(W) == ntv and all(abs(np.linalg.norm(w) - 1.0) < 1e-13 for w in W)
        cur = rq(W)
        assert smin <= cur < prev
        prev = cur
    lam, vec = np.linalg.eigh(dense.dense_Q(op.U, op.m0, op.clover))
    low = [vec[:, i].reshape(dims + (4, 3)) for i in np.argsort(np.abs(lam))[:2 * ntv]]
    P_setup = mg.build_P(W, block)
    P_rand = mg.build_P(W0, block)
    lc_setup = np.mean([mg.local_coherence(P_setup, v, block) for v in low])
    lc_rand = np.mean([mg.local_coherence(P_rand, v, block) for v in low])
    assert lc_setup > lc_rand + 0.1, (lc_setup, lc_rand)
    assert V == 128
