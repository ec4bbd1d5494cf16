"""Edge cases of the batch: the largest batch the library takes (64 right-hand sides)
against the oracle, the limits of the batch size, and the independence of the columns
of a batch (identical columns come out bit for bit identical wherever they sit)."""
import numpy as np
import pytest

from gpu_common import case, dev, host, need_gpu
from helpers import rel_err
from oracle import clover as oclover
from oracle import dirac
from synth import random_links, random_spinors, random_test_vectors, seed_for

pytestmark = pytest.mark.gpu

MAXRHS = 64


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_apply_largest_batch(prec, tol):
    """(Q - tau_k) on 64 right-hand sides with 64 distinct shifts in one launch (four
    16-rhs groups of the stencil's work order), every column against the oracle."""
    case("apply 8^4 clover, 64 rhs, " + prec)
    qmg = need_gpu()
    dims, m0 = (8, 8, 8, 8), -0.8
    U = random_links(dims, 0.5, seed_for(6, "U"))
    psi = random_spinors(dims, MAXRHS, seed_for(6, "b"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, 1.0)
    C = oclover.clover_term(U, 1.0)
    taus = [0.01 * (k - 31.5) for k in range(MAXRHS)]
    fin = lat.pack(dev(psi), prec)
    out = host(lat.unpack(lat.apply_Q_shifted(lat.field(MAXRHS, prec), fin, taus, MAXRHS, prec), MAXRHS, prec))
    pin = host(lat.unpack(fin, MAXRHS, prec))
    errs = [rel_err(out[k], dirac.apply_Q_shifted(U, pin[k], m0, taus[k], C)) for k in range(MAXRHS)]
    assert max(errs) < tol, max(errs)


def test_batch_size_limits():
    """0 and 65 right-hand sides are rejected with QMG_E_ARG by the apply, SAP and solve
    entry points (the shift arrays and kernel arguments hold at most 64)."""
    case("batch size limits")
    qmg = need_gpu()
    dims = (8, 8, 8, 8)
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(random_links(dims, 0.5, 1)), -0.8, 1.0)
    x, f = lat.field(1), lat.field(1)
    for n in (0, MAXRHS + 1):
        taus = [0.0] * n
        with pytest.raises(qmg.QmgError) as e:
            lat.apply_Q_shifted(x, f, taus, n)
        assert e.value.status == -1
        with pytest.raises(qmg.QmgError) as e:
            lat.sap_smooth(x, f, taus, n)
        assert e.value.status == -1
        with pytest.raises(qmg.QmgError) as e:
            lat.solve_shifted(x, f, taus, n, qmg.default_params(use_coarse=0))
        assert e.value.status == -1


def test_solve_largest_batch_columns_independent():
    """A 64-rhs two-level solve (FP32 graph V-cycle in FP64 FGMRES) whose columns k and
    k + 32 are the same system: every pair comes out bit for bit identical, with the same
    iteration count, although the two sit in different 16-rhs tiles of every MFMA and
    stencil launch, in different SAP slots, and move when converged columns leave the
    batch; sampled columns meet the tolerance under the oracle's operator."""
    case("solve 8^4, 64 rhs, identical column pairs")
    qmg = need_gpu()
    dims, m0, csw = (8, 8, 8, 8), -0.8, 1.0
    U = random_links(dims, 0.5, seed_for(6, "U"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, csw)
    ntv = 12
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(6, "W"))))
    lat.setup_mg(W, ntv, setup_iters=3, smooth=3)
    half = MAXRHS // 2
    b = random_spinors(dims, half, seed_for(6, "b") + 1)
    b = np.concatenate([b, b])
    t = [0.002 * (2 * k - half + 1) for k in range(half)]
    taus = t + t
    prm = qmg.default_params(mg_prec="f32", restart=4, maxiter=300, use_graph=1, coarse_maxiter=12)
    x = lat.field(MAXRHS)
    st, stats = lat.solve_shifted(x, lat.pack(dev(b)), taus, MAXRHS, prm)
    assert st == 0
    its = [s["iters"] for s in stats]
    print("iterations", its[:half], flush=True)
    xs = host(lat.unpack(x, MAXRHS))
    for k in range(half):
        assert its[k] == its[k + half], k
        assert np.array_equal(xs[k], xs[k + half]), k
    C = oclover.clover_term(U, csw)
    for k in (0, half - 1):
        r = b[k] - dirac.apply_Q_shifted(U, xs[k], m0, taus[k], C)
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) <= 1.5e-10, k
