"""GPU parity of the stencil (apply_Q, apply_Q_shifted, apply_A) against the oracle."""
import numpy as np
import pytest

from gpu_common import big_inputs, case, dev, host, need_gpu, torch
from helpers import oracle_at_sites, rel_err, sample_sites
from oracle import clover as oclover
from oracle import dirac
from oracle.gamma import GAMMA, GAMMA5, I4
from synth import random_links, random_spinors, seed_for, unit_links

pytestmark = pytest.mark.gpu


def _setup(dims, block, eps, m0, csw, cfg, nrhs):
    qmg = need_gpu()
    U = random_links(dims, eps, seed_for(cfg, "U"))
    psi = random_spinors(dims, nrhs, seed_for(cfg, "b"))
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    return qmg, lat, U, psi


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_pack_roundtrip(prec):
    case("pack roundtrip " + prec)
    qmg, lat, U, psi = _setup((4, 4, 4, 8), (2, 2, 2, 4), 0.3, -0.5, 0.0, 1, 3)
    back = host(lat.unpack(lat.pack(dev(psi), prec), 3, prec))
    if prec == "f64":
        assert np.array_equal(back, psi)
    elif prec == "f32":
        assert np.array_equal(back, psi.real.astype(np.float32) + 1j * psi.imag.astype(np.float32))
    else:
        assert rel_err(back, psi) < 2 ** -8


@pytest.mark.parametrize("nrhs", [1, 4])
def test_apply_Q_wilson_4x4(nrhs):
    """Config: 4^4, FP64 Q = gamma5 (D + m0), m0 = -0.5, no clover, eps = 0.3 links."""
    case("apply_Q 4^4 wilson nrhs=%d" % nrhs)
    qmg, lat, U, psi = _setup((4, 4, 4, 4), (2, 2, 2, 2), 0.3, -0.5, 0.0, 1, nrhs)
    out = host(lat.unpack(lat.apply_Q(lat.field(nrhs), lat.pack(dev(psi)), nrhs), nrhs))
    for k in range(nrhs):
        assert rel_err(out[k], dirac.apply_Q(U, psi[k], -0.5)) < 1e-13


def test_apply_Q_one_block_per_direction():
    """A single 4^4 block covering the lattice: hops wrap inside the block."""
    case("apply_Q 4^4 single block")
    qmg, lat, U, psi = _setup((4, 4, 4, 4), (4, 4, 4, 4), 0.3, -0.5, 0.0, 1, 1)
    out = host(lat.unpack(lat.apply_Q(lat.field(1), lat.pack(dev(psi)))))
    assert rel_err(out[0], dirac.apply_Q(U, psi[0], -0.5)) < 1e-13


def test_free_field_plane_wave():
    case("free field plane wave 8x4x4x4")
    qmg = need_gpu()
    dims, m0 = (8, 4, 4, 4), -0.5
    lat = qmg.Lattice(dims, (2, 2, 2, 2))
    lat.set_gauge(dev(unit_links(dims)), m0, 0.0)
    n = (3, 1, 0, 2)
    p = [2 * np.pi * n[mu] / dims[mu] for mu in range(4)]
    mp = m0 + sum(1 - np.cos(q) for q in p)
    qp = GAMMA5 @ (mp * I4 + 1j * sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4)))
    w, v = np.linalg.eigh(qp)
    x = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    phase = np.exp(1j * sum(p[mu] * x[mu] for mu in range(4)))
    psi = phase[..., None, None] * np.einsum("s,c->sc", v[:, 0], np.array([1.0, 0.5j, -0.25]))
    out = host(lat.unpack(lat.apply_Q(lat.field(1), lat.pack(dev(psi[None])))))
    assert rel_err(out[0], w[0] * psi) < 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6), ("bf16", 3e-2)])
def test_apply_clover_shifted_8x4(prec, tol):
    """Clover c_sw = 1, m0 = -0.8, eps = 0.5 links, per-rhs shifts, both operator forms."""
    case("apply clover 8^4 " + prec)
    dims = (8, 8, 8, 8)
    qmg, lat, U, psi = _setup(dims, (4, 4, 4, 4), 0.5, -0.8, 1.0, 2, 2)
    C = oclover.clover_term(U, 1.0)
    taus = [0.01, -0.37]
    fin = lat.pack(dev(psi), prec)
    outQ = host(lat.unpack(lat.apply_Q_shifted(lat.field(2, prec), fin, taus, 2, prec), 2, prec))
    outA = host(lat.unpack(lat.apply_A(lat.field(2, prec), fin, taus, 2, prec), 2, prec))
    for k in range(2):
        # the reference takes the same rounded input the GPU saw
        pin = host(lat.unpack(fin, 2, prec))[k]
        assert rel_err(outQ[k], dirac.apply_Q_shifted(U, pin, -0.8, taus[k], C)) < tol
        assert rel_err(outA[k], dirac.apply_A(U, pin, -0.8, taus[k], C)) < tol


def test_apply_Q_hermitian_and_dot():
    case("apply_Q hermiticity 8^4 via field_dot")
    qmg, lat, U, psi = _setup((8, 8, 8, 8), (4, 4, 4, 4), 0.5, -0.8, 1.0, 2, 2)
    a = lat.pack(dev(psi[:1]))
    b = lat.pack(dev(psi[1:]))
    qa = lat.apply_Q(lat.field(1), a)
    qb = lat.apply_Q(lat.field(1), b)
    d1 = lat.field_dot(a, qb)[0]
    d2 = lat.field_dot(qa, b)[0]
    assert abs(d1 - d2) < 1e-12 * abs(d1)
    assert abs(lat.field_dot(a, a)[0] - np.vdot(psi[0], psi[0])) < 1e-12 * np.vdot(psi[0], psi[0]).real


@pytest.mark.parametrize("prec,nrhs,tol", [("f64", 1, 1e-13), ("f32", 16, 1e-6)])
def test_apply_full_size_sampled(prec, nrhs, tol, tmp_path):
    """64x32^3, c_sw = 1, the bench configuration and the launch configuration the
    autotuner picks there (as in the bench): sampled sites against the oracle."""
    case("apply 64x32^3 sampled %s nrhs=%d" % (prec, nrhs))
    qmg = need_gpu()
    dims = (64, 32, 32, 32)
    U, psi = big_inputs(dims, 0.5, 5, nrhs)
    m0 = -0.8
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(dev(U), m0, 1.0)
    path = tmp_path / "tune.json"
    lat.autotune(str(path))
    cls = "|dslash|%s|%d\":" % (prec, 0 if nrhs == 1 else 1)
    print("tuned:", [ln.strip() for ln in path.read_text().splitlines() if cls in ln or "ds_order\":" in ln],
          flush=True)
    taus = [0.0025 * (2 * k - 15) for k in range(nrhs)]
    fin = lat.pack(dev(psi), prec)
    out = lat.unpack(lat.apply_Q_shifted(lat.field(nrhs, prec), fin, taus, nrhs, prec), nrhs, prec)
    pin = lat.unpack(fin, nrhs, prec)
    sites = sample_sites(dims, 24, 9)
    for k in sorted({0, nrhs - 1}):
        ref = oracle_at_sites(U, host(pin[k]), m0, 1.0, sites, taus[k])
        got = np.array([host(out[k][x]) for x in sites])
        assert rel_err(got, ref) < tol


def _force_variant(lat, tmp_path, dims, block, clover, v):
    key = "gfx950|%s|%s|clover=%d" % ("x".join(map(str, dims)), "x".join(map(str, block)), clover)
    entries = ['"%s|dslash|%s|%d": %d' % (key, p, c, v) for p in ("f64", "f32", "bf16") for c in (0, 1)]
    path = tmp_path / ("tune_%d.json" % v)
    path.write_text("{\n" + ",\n".join(entries) + "\n}\n")
    lat.autotune(str(path))


@pytest.mark.parametrize("order,variant", [(1, 1), (4, 1), (6, 5), (7, 2)])
def test_stencil_tile_orders(order, variant, tmp_path):
    """Work orders that visit tiles of blocks (each tile's rhs groups back to
    back) change only which work-group computes what: results equal the oracle's
    on a 16x8x8x8 lattice (4x2x2x2 blocks, so several tiles) with a ragged batch."""
    case("stencil tile order %d variant %d" % (order, variant))
    dims, block = (16, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, U, psi = _setup(dims, block, 0.5, -0.8, 1.0, 2, 3)
    key = "gfx950|%s|%s|clover=1" % ("x".join(map(str, dims)), "x".join(map(str, block)))
    entries = ['"%s|dslash|%s|%d": %d' % (key, p, c, variant) for p in ("f64", "f32", "bf16") for c in (0, 1)]
    entries.append('"%s|ds_order": %d' % (key, order))
    path = tmp_path / "tune_order.json"
    path.write_text("{\n" + ",\n".join(entries) + "\n}\n")
    lat.autotune(str(path))
    C = oclover.clover_term(U, 1.0)
    taus = [0.01, -0.2, 0.05]
    fin = lat.pack(dev(psi), "f64")
    pin = host(lat.unpack(fin, 3, "f64"))
    out = host(lat.unpack(lat.apply_Q_shifted(lat.field(3, "f64"), fin, taus, 3, "f64"), 3, "f64"))
    for k in range(3):
        assert rel_err(out[k], dirac.apply_Q_shifted(U, pin[k], -0.8, taus[k], C)) < 1e-13


@pytest.mark.parametrize("variant", range(12))
def test_stencil_variants(variant, tmp_path):
    """Every launch variant of the stencil (generic, 4^4 kernels with 1/2/4 rhs per
    thread and occupancy targets) against the oracle, with a ragged rhs batch."""
    case("stencil variant %d" % variant)
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, U, psi = _setup(dims, block, 0.5, -0.8, 1.0, 2, 3)
    _force_variant(lat, tmp_path, dims, block, 1, variant)
    C = oclover.clover_term(U, 1.0)
    taus = [0.01, -0.2, 0.05]
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6)):
        fin = lat.pack(dev(psi), prec)
        pin = host(lat.unpack(fin, 3, prec))
        for nrhs in (1, 3):
            outQ = host(lat.unpack(lat.apply_Q_shifted(lat.field(nrhs, prec), fin, taus[:nrhs], nrhs, prec),
                                   nrhs, prec))
            outA = host(lat.unpack(lat.apply_A(lat.field(nrhs, prec), fin, taus[:nrhs], nrhs, prec), nrhs, prec))
            for k in range(nrhs):
                assert rel_err(outQ[k], dirac.apply_Q_shifted(U, pin[k], -0.8, taus[k], C)) < tol
                assert rel_err(outA[k], dirac.apply_A(U, pin[k], -0.8, taus[k], C)) < tol
