"""GPU shifted solves: true residuals checked against the oracle's operator."""
import numpy as np
import pytest

from gpu_common import big_inputs, case, dev, host, need_gpu, torch
from helpers import oracle_at_sites, sample_sites
from oracle import clover as oclover
from oracle import dirac
from synth import random_links, random_spinors, random_test_vectors, seed_for

pytestmark = pytest.mark.gpu


def _true_relres_oracle(U, m0, C, x, b, tau):
    r = b - dirac.apply_Q_shifted(U, x, m0, tau, C)
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_solve_sap_only_16x4():
    """Config: 16^4, SAP (4^4 blocks, 3 MR steps) + shifted FGMRES, tau = 0.01, m0 = -0.8, c_sw = 1."""
    case("solve 16^4 SAP-only f64")
    qmg = need_gpu()
    dims = (16, 16, 16, 16)
    U = random_links(dims, 0.5, seed_for(2, "U"))
    m0, csw, tau = -0.8, 1.0, 0.01
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    b = random_spinors(dims, 1, seed_for(2, "b"))
    x = lat.field(1)
    prm = qmg.default_params(use_coarse=0, restart=16, maxiter=400)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), [tau], 1, prm)
    assert st == 0 and stats[0]["true_relres"] <= 1e-10
    C = oclover.clover_term(U, csw)
    assert _true_relres_oracle(U, m0, C, host(lat.unpack(x))[0], b[0], tau) <= 1.5e-10


@pytest.mark.parametrize("prec,graph", [("f64", 0), ("f32", 0), ("bf16", 0), ("f32", 1)])
def test_solve_two_level_multishift(prec, graph):
    """8^4 lattice, 4^4 aggregates, setup-built test vectors, 4 shifts, V-cycle in prec
    (optionally replayed as a HIP graph), FP64 FGMRES."""
    case("solve 8^4 two-level multishift %s graph=%d" % (prec, graph))
    qmg = need_gpu()
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.5, seed_for(4, "U"))
    m0, csw = -0.8, 1.0
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    ntv = 12
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(4, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    nrhs = 4
    taus = [0.005 * (2 * k - 3) for k in range(nrhs)]
    b = random_spinors(dims, nrhs, seed_for(4, "b"))
    x = lat.field(nrhs)
    prm = qmg.default_params(mg_prec=prec, restart=16, maxiter=300, use_graph=graph,
                             coarse_maxiter=8 if graph else 50)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, nrhs, prm)
    assert st == 0
    xs = host(lat.unpack(x, nrhs))
    C = oclover.clover_term(U, csw)
    for k in range(nrhs):
        assert stats[k]["true_relres"] <= 1e-10
        assert _true_relres_oracle(U, m0, C, xs[k], b[k], taus[k]) <= 1.5e-10
    print("iterations", [s["iters"] for s in stats], flush=True)


def test_solve_not_converged_status():
    case("solve maxiter too small")
    qmg = need_gpu()
    dims = (8, 8, 8, 8)
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(random_links(dims, 0.5, 1)), -0.8, 1.0)
    b = lat.pack(dev(random_spinors(dims, 1, 2)))
    st, stats = lat.solve_shifted(lat.field(1), b, [0.0], 1, qmg.default_params(use_coarse=0, maxiter=3,
                                                                                  restart=3))
    assert st == 1 and stats[0]["iters"] == 3 and stats[0]["true_relres"] > 1e-10


def test_state_and_argument_errors():
    case("error paths")
    qmg = need_gpu()
    with pytest.raises(qmg.QmgError):
        qmg.Lattice((6, 4, 4, 4), (4, 4, 4, 4))        # block does not divide
    lat = qmg.Lattice((8, 8, 8, 8), (4, 4, 4, 4))
    f = lat.field(1)
    with pytest.raises(qmg.QmgError) as e:
        lat.apply_Q(lat.field(1), f)
    assert e.value.status == -2                          # no gauge field yet
    lat.set_gauge(dev(random_links((8, 8, 8, 8), 0.5, 1)), -0.8, 0.0)
    with pytest.raises(qmg.QmgError) as e:
        lat.restrict(lat.coarse(1), f)
    assert e.value.status == -2                          # no multigrid yet
    with pytest.raises(qmg.QmgError) as e:
        lat.apply_Q(f, f)
    assert e.value.status == -1                          # aliasing
    lat1 = qmg.Lattice((8, 8, 8, 8), (8, 4, 4, 4))      # one block in direction 0
    lat1.set_gauge(dev(random_links((8, 8, 8, 8), 0.5, 1)), -0.8, 0.0)
    with pytest.raises(qmg.QmgError) as e:
        lat1.sap_smooth(lat1.field(1), lat1.field(1), [0.0])
    assert e.value.status == -1
    bad = random_spinors((8, 8, 8, 8), 1, 3)
    bad[0, 1, 2, 3, 4, 0, 0] = np.nan
    with pytest.raises(qmg.QmgError) as e:
        lat.solve_shifted(lat.field(1), lat.pack(dev(bad)), [0.0], 1, qmg.default_params(use_coarse=0))
    assert e.value.status == -5


def test_solve_full_size_sampled():
    """64x32^3, c_sw = 1, 2 shifts, SAP-preconditioned FP32 smoother; residual via the GPU FP64
    operator (parity-tested) and sampled sites of Q x against the oracle."""
    case("solve 64x32^3 sampled")
    qmg = need_gpu()
    dims = (64, 32, 32, 32)
    U, b = big_inputs(dims, 0.5, 5, 2)
    m0, csw = -0.8, 1.0
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    taus = [0.01, -0.02]
    bg = lat.pack(dev(b))
    x = lat.field(2)
    st, stats = lat.solve_shifted(x, bg, taus, 2, qmg.default_params(use_coarse=0, mg_prec="f32", restart=16,
                                                                    maxiter=400))
    assert st == 0
    qx = lat.apply_Q_shifted(lat.field(2), x, taus, 2)
    for k in range(2):
        assert stats[k]["true_relres"] <= 1e-10
    xs = lat.unpack(x, 2)
    sites = sample_sites(dims, 12, 3)
    qxs = lat.unpack(qx, 2)
    for k in range(2):
        ref = oracle_at_sites(U, host(xs[k]), m0, csw, sites, taus[k])
        got = np.array([host(qxs[k][s]) for s in sites])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        # at those sites Q x reproduces b up to the solve tolerance
        assert np.abs(got - b[k][tuple(np.array(sites).T)]).max() <= 1e-6


def test_solve_batch_compaction_writes_back_every_column():
    """FGMRES drops the columns that have converged when a restart cycle ends (later cycles
    run on the others only) and writes each column's x back to its own slot.  8 shifts
    with short restart cycles, so columns leave the batch at different restarts: every
    column meets the tolerance under the oracle's operator, and each takes the iterations
    it takes when solved alone (within one: the alone solve runs the single-rhs kernels)."""
    case("solve 8^4 batch compaction")
    qmg = need_gpu()
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.5, seed_for(4, "U"))
    m0, csw = -0.8, 1.0
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    ntv = 12
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(4, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    nrhs = 8
    taus = [0.03 * (k - 3.5) for k in range(nrhs)]
    b = random_spinors(dims, nrhs, seed_for(4, "b") + 7)
    prm = qmg.default_params(mg_prec="f32", restart=3, maxiter=300)
    x = lat.field(nrhs)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, nrhs, prm)
    assert st == 0
    its = [s["iters"] for s in stats]
    print("iterations", its, flush=True)
    assert len(set(its)) > 1          # the columns did converge at different times
    xs = host(lat.unpack(x, nrhs))
    C = oclover.clover_term(U, csw)
    for k in range(nrhs):
        assert _true_relres_oracle(U, m0, C, xs[k], b[k], taus[k]) <= 1.5e-10, k
    for k in (int(np.argmin(its)), int(np.argmax(its))):
        x1 = lat.field(1)
        st1, s1 = lat.solve_shifted(x1, lat.pack(dev(b[k:k + 1])), [taus[k]], 1, prm)
        assert st1 == 0 and abs(s1[0]["iters"] - its[k]) <= 1, (k, s1[0]["iters"], its[k])


def test_solve_statistics_history_and_phases():
    """The per-rhs statistics of a batched solve: the true relative residual at the start of
    every restart cycle (1 at x = 0, non-increasing up to rounding, the last entry the final
    residual, one entry more than restart cycles), and the phase times (V-cycles, FP64
    products, Gram-Schmidt) positive and within the wall time of the solve."""
    case("solve statistics")
    qmg = need_gpu()
    dims = (8, 8, 8, 8)
    U = random_links(dims, 0.5, seed_for(4, "U"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), -0.8, 1.0)
    ntv = 12
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(4, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    nrhs = 4
    taus = [0.03 * (k - 1.5) for k in range(nrhs)]
    b = random_spinors(dims, nrhs, seed_for(4, "b") + 11)
    prm = qmg.default_params(mg_prec="f32", restart=3, maxiter=300)
    x = lat.field(nrhs)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, nrhs, prm)
    assert st == 0
    for s in stats:
        h = s["relres_hist"]
        print("restarts", s["restarts"], "history", ["%.2e" % v for v in h], flush=True)
        assert s["n_hist"] == s["restarts"] + 1 == len(h)
        assert abs(h[0] - 1.0) < 1e-12
        assert h[-1] == s["true_relres"] <= 1e-10
        assert all(h[i + 1] <= h[i] * (1 + 1e-6) for i in range(len(h) - 1))
        ph = (s["vcycle_seconds"], s["apply_seconds"], s["orth_seconds"])
        assert all(p > 0 for p in ph) and sum(ph) <= s["seconds"], (ph, s["seconds"])


def test_solve_resumes_from_initial_guess():
    """qmg_params.x0 = 1: a solve cut off by maxiter resumes from its own x (its first
    residual is the one the stopped solve ended with) and converges in about the
    iterations a single solve takes; a converged x passed back needs no iteration."""
    case("solve resume from x0")
    qmg = need_gpu()
    dims, m0, csw = (8, 8, 8, 8), -0.8, 1.0
    U = random_links(dims, 0.5, seed_for(4, "U"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    ntv = 12
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(4, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    nrhs, taus = 2, [0.01, -0.02]
    b = random_spinors(dims, nrhs, seed_for(4, "b") + 13)
    bg = lat.pack(dev(b))
    x1 = lat.field(nrhs)
    st1, s1 = lat.solve_shifted(x1, bg, taus, nrhs, qmg.default_params(mg_prec="f32", restart=4, maxiter=300))
    assert st1 == 0
    x = lat.field(nrhs)
    st_a, sa = lat.solve_shifted(x, bg, taus, nrhs, qmg.default_params(mg_prec="f32", restart=4, maxiter=5))
    assert st_a == 1 and all(s["true_relres"] > 1e-10 for s in sa)
    st_b, sb = lat.solve_shifted(x, bg, taus, nrhs, qmg.default_params(mg_prec="f32", restart=4, maxiter=300, x0=1))
    assert st_b == 0
    for k in range(nrhs):
        print("single", s1[k]["iters"], "resumed", sa[k]["iters"], "+", sb[k]["iters"], flush=True)
        assert abs(sb[k]["relres_hist"][0] - sa[k]["true_relres"]) <= 1e-12 * sa[k]["true_relres"]
        assert abs(sa[k]["iters"] + sb[k]["iters"] - s1[k]["iters"]) <= 4
    xs = host(lat.unpack(x, nrhs))
    C = oclover.clover_term(U, csw)
    for k in range(nrhs):
        assert _true_relres_oracle(U, m0, C, xs[k], b[k], taus[k]) <= 1.5e-10
    st_c, sc = lat.solve_shifted(x, bg, taus, nrhs, qmg.default_params(mg_prec="f32", restart=4, x0=1))
    assert st_c == 0 and all(s["iters"] == 0 and s["true_relres"] <= 1e-10 for s in sc)
