"""Bitwise reproducibility: every reduction in the library runs in a fixed order
(two-stage dot products, fixed wave butterflies, no atomics), so the same inputs give
the same bits run after run, and a HIP-graph replay of the V-cycle gives the same bits
as the eager sequence of the same kernels."""
import pytest

from gpu_common import case, dev, need_gpu, torch
from synth import random_links, random_spinors, random_test_vectors, seed_for

pytestmark = pytest.mark.gpu


def _lat(qmg, dims=(8, 8, 8, 8)):
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(random_links(dims, 0.5, seed_for(4, "U"))), -0.8, 1.0)
    ntv = 8
    W = lat.pack(dev(random_test_vectors(dims, ntv, seed_for(4, "W"))))
    lat.set_test_vectors(W, ntv)
    return lat


def test_bitwise_two_runs():
    case("bitwise: apply, SAP, solve twice")
    qmg = need_gpu()
    dims, nrhs = (8, 8, 8, 8), 16
    lat = _lat(qmg, dims)
    b = random_spinors(dims, nrhs, seed_for(4, "b"))
    taus = [0.004 * (2 * k - 15) for k in range(nrhs)]
    for prec in ("f64", "f32", "bf16"):
        bg = lat.pack(dev(b), prec)
        o1 = lat.apply_Q_shifted(lat.field(nrhs, prec), bg, taus, nrhs, prec)
        o2 = lat.apply_Q_shifted(lat.field(nrhs, prec), bg, taus, nrhs, prec)
        assert torch.equal(o1, o2), prec
        x1 = lat.sap_smooth(lat.field(nrhs, prec), bg, taus, nrhs, 3, 3, prec)
        x2 = lat.sap_smooth(lat.field(nrhs, prec), bg, taus, nrhs, 3, 3, prec)
        assert torch.equal(x1, x2), prec
    bg = lat.pack(dev(b[:4]))
    prm = qmg.default_params(mg_prec="f32", restart=8, maxiter=200)
    x1, x2 = lat.field(4), lat.field(4)
    st1, s1 = lat.solve_shifted(x1, bg, taus[:4], 4, prm)
    st2, s2 = lat.solve_shifted(x2, bg, taus[:4], 4, prm)
    assert st1 == st2 == 0
    assert torch.equal(x1, x2)
    assert [s["iters"] for s in s1] == [s["iters"] for s in s2]
    assert [s["true_relres"] for s in s1] == [s["true_relres"] for s in s2]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replay_bitwise_equals_eager(prec):
    """Fixed-step V-cycle (device-resident coarse GMRES): eager launch sequence vs the
    captured graph, replayed three times with eager work in between."""
    case("bitwise: graph replay vs eager V-cycle " + prec)
    qmg = need_gpu()
    dims, nrhs = (8, 8, 8, 8), 4
    lat = _lat(qmg, dims)
    r = lat.pack(dev(random_spinors(dims, nrhs, 43)))
    taus = [0.02, -0.1, 0.0, 0.05]
    kw = dict(coarse_maxiter=10, coarse_tol=0.0, nu_post=2, n_mr=3, mg_prec=prec)
    eager = lat.vcycle(lat.field(nrhs), r, taus, nrhs, qmg.default_params(use_graph=0, **kw))
    z = lat.field(nrhs)
    for rep in range(4):
        lat.vcycle(z, r, taus, nrhs, qmg.default_params(use_graph=1, **kw))
        torch.cuda.synchronize()
        assert torch.equal(z, eager), rep
        lat.apply_Q(lat.field(1), r, 1)
        z.zero_()
