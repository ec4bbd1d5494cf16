"""GPU parity of the third multigrid level (P2, level-2 <-> level-3 transfers, D3,
the level-2 K-cycle, the three-level V-cycle, solve and setup) against the oracle."""
import numpy as np
import pytest

from gpu_common import case, coarse_to_lex, dev, host, lex_to_coarse, need_gpu, torch  # noqa: F401
from helpers import rel_err
from oracle import blocks as bl
from oracle import clover as oclover
from oracle import dirac, mg, mg3
from oracle.solve import solve_shifted
from synth import random_links, random_spinors, random_test_vectors, seed_for

pytestmark = pytest.mark.gpu


def _setup(dims, block, ntv, block2, ntv2, csw=1.0, m0=-0.8):
    qmg = need_gpu()
    U = random_links(dims, 0.5, seed_for(2, "U"))
    op = dirac.Operator(U, m0, oclover.clover_term(U, csw) if csw else None)
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    W = list(random_test_vectors(dims, ntv, seed_for(2, "W")))
    lat.set_test_vectors(lat.pack(dev(np.array(W))), ntv)
    two = mg.TwoLevel(op, W, block)
    order = lat.coarse_site_order()
    dims2 = bl.nblocks(dims, block)
    W2 = mg3.initial_level2_vectors(two.P, W, block, ntv2)
    lat.set_level3_vectors(dev(lex_to_coarse(np.array(W2), order).view(np.float64)), ntv2, block2)
    l3 = mg3.Level3(two.coarse, dims2, W2, block2)
    return qmg, lat, op, W, two, W2, l3, order


CASES = [((8, 8, 8, 8), (2, 2, 2, 2), 8, (2, 2, 2, 2), 8),
         ((16, 8, 8, 8), (4, 4, 4, 4), 24, (2, 1, 1, 1), 16)]


def _rand(rng, shape, dt=np.complex128):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dt)


@pytest.mark.parametrize("dims,block,ntv,block2,ntv2", CASES)
def test_l3_transfer_parity(dims, block, ntv, block2, ntv2):
    case("level-3 restrict/prolong %s block2 %s ntv2 %d" % (dims, block2, ntv2))
    qmg, lat, op, W, two, W2, l3, order = _setup(dims, block, ntv, block2, ntv2)
    n3, nc3 = lat.level3_shape()
    assert (n3, nc3) == (l3.P2.shape[0], 2 * ntv2)
    rng = np.random.default_rng(11)
    y2 = _rand(rng, (2, len(order), 2 * ntv))
    y3 = host(lat.restrict_l3(lat.l3_vec(2), dev(lex_to_coarse(y2, order).view(np.float64)), 2)).view(np.complex128)
    y3 = y3.reshape(2, n3, nc3)
    for k in range(2):
        assert rel_err(y3[k], l3.restrict(y2[k])) < 1e-13
    z3 = _rand(rng, (2, n3, nc3))
    z2 = host(lat.prolong_l3(lat.coarse(2), dev(z3.view(np.float64)), 2)).view(np.complex128)
    z2 = coarse_to_lex(z2, order, ntv)
    for k in range(2):
        assert rel_err(z2[k], l3.prolong(z3[k])) < 1e-13


@pytest.mark.parametrize("dims,block,ntv,block2,ntv2", CASES)
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_l3_apply_parity(dims, block, ntv, block2, ntv2, prec, tol):
    """D3 (assembled on the GPU by triple products) against the oracle's D3
    (assembled column by column), applied to ragged batches (1, 5 and 17 rhs:
    the generic and the MFMA kernels)."""
    case("level-3 apply %s ntv2 %d %s" % (dims, ntv2, prec))
    qmg, lat, op, W, two, W2, l3, order = _setup(dims, block, ntv, block2, ntv2)
    n3, nc3 = lat.level3_shape()
    rng = np.random.default_rng(12)
    cdt = np.complex128 if prec == "f64" else np.complex64
    rdt = np.float64 if prec == "f64" else np.float32
    for nrhs in (1, 5, 17):
        y = _rand(rng, (nrhs, n3, nc3), cdt)
        taus = [0.02 * (k - 2) for k in range(nrhs)]
        out = host(lat.apply_l3(lat.l3_vec(nrhs, prec), dev(y.view(rdt)), taus, nrhs, prec)).view(cdt)
        out = out.reshape(nrhs, n3, nc3)
        for k in range(nrhs):
            ref = l3.coarse3.apply(y[k].astype(np.complex128), taus[k])
            assert rel_err(out[k], ref) < tol, (nrhs, k)


def test_level2_kcycle_parity():
    """k2 FGMRES steps on A_c preconditioned by M2 (level-3 GMRES, level-2 GMRES
    smoothing), all scalars on the device, against the oracle's K-cycle."""
    case("level-2 K-cycle 8^4")
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    rng = np.random.default_rng(13)
    r = _rand(rng, (2, len(order), 16))
    taus = [0.01, -0.05]
    yg = lat.level2_solve(lat.coarse(2), dev(lex_to_coarse(r, order).view(np.float64)), taus, 2, k2=4, k3=10, s2=2)
    y = coarse_to_lex(host(yg).view(np.complex128), order, 8)
    for k in range(2):
        ref = l3.solve(r[k], taus[k], 4, 10, 2)
        assert rel_err(y[k], ref) < 1e-13


@pytest.mark.parametrize("prec,tol,graph", [("f64", 1e-13, 0), ("f32", 1e-6, 0), ("f32", 1e-6, 1)])
def test_vcycle3_parity(prec, tol, graph):
    """The three-level V-cycle (restrict, level-2 K-cycle, prolong, SAP) against
    the oracle's; in graph mode every replay matches."""
    case("three-level vcycle 8^4 %s graph=%d" % (prec, graph))
    dims, block, ntv, block2, ntv2 = CASES[0]
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    three = mg3.ThreeLevel(op, W, block, W2, block2, k3=10, s2=2)
    r = random_spinors(dims, 2, 47)
    taus = [0.02, -0.1]
    prm = qmg.default_params(levels=3, coarse_maxiter=3, l3_iters=10, l2_smooth=2, nu_post=2, n_mr=3,
                             mg_prec=prec, use_graph=graph)
    ref = [three.vcycle(r[k], taus[k], 2, 3, 3) for k in range(2)]
    rg = lat.pack(dev(r))
    z = lat.field(2)
    for rep in range(3 if graph else 1):
        lat.vcycle(z, rg, taus, 2, prm)
        got = host(lat.unpack(z, 2))
        for k in range(2):
            assert rel_err(got[k], ref[k]) < tol, (rep, k)
        lat.apply_Q(lat.field(1), rg, 1)
        torch.cuda.synchronize()
        z.zero_()


def test_three_level_solve():
    """FGMRES with the three-level V-cycle reaches 1e-10 (residual recomputed by
    the oracle's operator) in the oracle's number of iterations (within 1)."""
    case("three-level solve 8^4 2 rhs")
    dims, block, ntv, block2, ntv2 = CASES[0]
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    three = mg3.ThreeLevel(op, W, block, W2, block2, k3=10, s2=2)
    b = random_spinors(dims, 2, seed_for(2, "b"))
    taus = [0.01, -0.03]
    prm = qmg.default_params(levels=3, coarse_maxiter=3, l3_iters=10, l2_smooth=2, restart=8, maxiter=200)
    x = lat.field(2)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, 2, prm)
    assert st == 0
    xs = host(lat.unpack(x, 2))
    for k in range(2):
        r = dirac.apply_Q_shifted(op.U, xs[k], op.m0, taus[k], op.clover) - b[k]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[k])
        _, it_ref, _ = solve_shifted(op, b[k], taus[k], block, three, restart=8, maxiter=200, coarse_iters=3)
        assert abs(stats[k]["iters"] - it_ref) <= 1, (stats[k]["iters"], it_ref)


def test_setup_level3_parity():
    """Level-2 test vectors after two rounds of inverse iteration with M2 (FP64)."""
    case("level-3 setup 8^4")
    dims, block, ntv, block2, ntv2 = CASES[0]
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    W2g = dev(lex_to_coarse(np.array(W2), order).view(np.float64))
    lat.setup_level3(W2g, ntv2, block2, setup_iters=3, smooth=2, l3_iters=10)
    got = coarse_to_lex(host(W2g).view(np.complex128), order, ntv)
    ref = mg3.setup_level3(two.coarse, bl.nblocks(dims, block), W2, block2, setup_iters=3, s2=2, k3=10)
    for j in range(ntv2):
        assert rel_err(got[j], ref[j]) < 1e-13, j


def test_level3_arguments_and_state():
    case("level-3 argument checks")
    dims, block, ntv, block2, ntv2 = CASES[0]
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    W2g = dev(lex_to_coarse(np.array(W2), order).view(np.float64))
    for bad_block2, bad_ntv2 in (((4, 2, 2, 2), 8), ((3, 2, 2, 2), 8), ((2, 2, 2, 2), 25), ((2, 2, 2, 2), 0)):
        with pytest.raises(qmg.QmgError) as e:
            lat.set_level3_vectors(W2g, bad_ntv2, bad_block2)
        assert e.value.status == -1
    # rank-deficient level-2 vectors
    Wd = np.array(W2)
    Wd[3] = Wd[1] * (0.5 + 0.5j)
    with pytest.raises(qmg.QmgError) as e:
        lat.set_level3_vectors(dev(lex_to_coarse(Wd, order).view(np.float64)), ntv2, block2)
    assert e.value.status == -5
    # a rebuild of P / D_c drops the third level
    lat.set_level3_vectors(W2g, ntv2, block2)
    lat.set_test_vectors(lat.pack(dev(np.array(W))), ntv)
    prm = qmg.default_params(levels=3)
    with pytest.raises(qmg.QmgError) as e:
        lat.vcycle(lat.field(1), lat.pack(dev(random_spinors(dims, 1, 3))), [0.0], 1, prm)
    assert e.value.status == -2
    with pytest.raises(qmg.QmgError) as e:
        lat.vcycle(lat.field(1), lat.pack(dev(random_spinors(dims, 1, 3))), [0.0], 1, qmg.default_params(levels=4))
    assert e.value.status == -1


@pytest.mark.parametrize("prec,tol,qform", [("f64", 1e-13, 1), ("bf16", 5e-2, 0)])
def test_vcycle3_qform_and_bf16(prec, tol, qform):
    """Three-level V-cycle on Q - tau (every level in the Q form: Gamma5^cc D3 - tau on
    level 3) and with BF16 storage of the fine and level-2 data (level 3 in FP32)."""
    case("three-level vcycle 8^4 %s qform=%d" % (prec, qform))
    dims, block, ntv, block2, ntv2 = CASES[0]
    qmg, lat, op, W, two, W2, l3, order = _setup(*CASES[0])
    three = mg3.ThreeLevel(op, W, block, W2, block2, k3=10, s2=2)
    r = random_spinors(dims, 2, 53)
    taus = [0.03, -0.07]
    prm = qmg.default_params(levels=3, coarse_maxiter=3, l3_iters=10, l2_smooth=2, nu_post=2, n_mr=3,
                             mg_prec=prec, q_form=qform)
    z = host(lat.unpack(lat.vcycle(lat.field(2), lat.pack(dev(r)), taus, 2, prm), 2))
    for k in range(2):
        ref = three.vcycle(r[k], taus[k], 2, 3, 3, qform=bool(qform))
        assert rel_err(z[k], ref) < tol, k


def test_three_level_full_size():
    """64x32^3 near-critical clover field, 16 shifts, 24 + 24 test vectors, 2^4 level-2 aggregates
    (512 level-3 sites): the three-level graph-mode solve reaches 1e-10 for every shift; for the
    first and last shift Q x at sampled sites, recomputed by the oracle, reproduces b."""
    case("three-level solve 64x32^3 16 rhs")
    from gpu_common import big_inputs
    from helpers import oracle_at_sites, sample_sites
    from synth import device_gaussian_spinors
    import json
    import os
    qmg = need_gpu()
    dims, nrhs = (64, 32, 32, 32), 16
    with open(os.path.join(os.path.dirname(__file__), "golden", "m0_critical.json")) as fh:
        m0 = float(json.load(fh)["m0"])
    U, b = big_inputs(dims, 0.5, 5, nrhs)
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, 1.0)
    W = lat.pack(device_gaussian_spinors(dims, 24, seed_for(5, "W")))
    lat.setup_mg(W, 24, setup_iters=6, smooth=4)
    lat.setup_level3(lat.level2_vectors_from(W, 24), 24, (2, 2, 2, 2), setup_iters=3, smooth=2)
    assert lat.level3_shape() == (512, 48)
    del W
    taus = [0.001 * (2 * k - 15) for k in range(nrhs)]
    prm = qmg.default_params(mg_prec="f32", use_graph=1, levels=3, coarse_maxiter=4, l3_iters=8, l2_smooth=2,
                             restart=6, maxiter=300)
    x = lat.field(nrhs)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, nrhs, prm)
    assert st == 0
    assert max(s["true_relres"] for s in stats) <= 1e-10
    sites = sample_sites(dims, 12, 5)
    for k in (0, nrhs - 1):
        xk = host(lat.unpack(x[k * lat.field_bytes():(k + 1) * lat.field_bytes()], 1))[0]
        qx = oracle_at_sites(U, xk, m0, 1.0, sites, taus[k])
        assert np.abs(qx - b[k][tuple(np.array(sites).T)]).max() <= 1e-6 * np.abs(b[k]).max()
