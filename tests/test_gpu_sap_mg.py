"""GPU parity of SAP, P, restriction/prolongation, D_c and the V-cycle."""
import numpy as np
import pytest

from gpu_common import case, coarse_to_lex, dev, host, lex_to_coarse, need_gpu, torch  # noqa: F401
from helpers import rel_err
from oracle import clover as oclover
from oracle import dirac, krylov, mg, sap
from synth import random_links, random_spinors, random_test_vectors, seed_for

pytestmark = pytest.mark.gpu


def _op(dims, block, csw=1.0, m0=-0.8, cfg=2):
    qmg = need_gpu()
    U = random_links(dims, 0.5, seed_for(cfg, "U"))
    C = oclover.clover_term(U, csw) if csw else None
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    return qmg, lat, dirac.Operator(U, m0, C)


@pytest.mark.parametrize("dims,block", [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 4, 4, 4), (2, 2, 2, 2)),
                                        ((8, 4, 4, 8), (4, 2, 2, 4))])
def test_sap_parity(dims, block):
    case("sap %s %s" % (dims, block))
    qmg, lat, op = _op(dims, block)
    nrhs = 2
    f = random_spinors(dims, nrhs, seed_for(2, "b"))
    x0 = random_spinors(dims, nrhs, seed_for(2, "x"))
    taus = [0.01, 0.2]
    xg = lat.pack(dev(x0))
    lat.sap_smooth(xg, lat.pack(dev(f)), taus, nrhs, nsweep=2, n_mr=3)
    got = host(lat.unpack(xg, nrhs))
    for k in range(nrhs):
        ref = sap.sap(op, f[k], x0[k], taus[k], block, 2, 3)
        assert rel_err(got[k], ref) < 1e-13


def _force_sap(lat, tmp_path, dims, block, clover, v):
    key = "gfx950|%s|%s|clover=%d" % ("x".join(map(str, dims)), "x".join(map(str, block)), clover)
    entries = ['"%s|dslash|%s|%d": 1' % (key, p, c) for p in ("f64", "f32", "bf16") for c in (0, 1)]
    entries.append('"%s|sap": %d' % (key, v))
    path = tmp_path / ("tune_sap_%d.json" % v)
    path.write_text("{\n" + ",\n".join(entries) + "\n}\n")
    lat.autotune(str(path))


_SAP_REF = {}


@pytest.mark.parametrize("sapv,nrhs", [(0, 2), (1, 2), (1, 5), (1, 16), (2, 2), (2, 5), (2, 16)])
@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("bf16", 5e-2)])
def test_sap_reduced_precision(prec, tol, sapv, nrhs, tmp_path):
    """FP32 / BF16-storage SAP, all three kernels (generic; LDS-staged 4^4 with one or two
    rhs per work-group), on 2, 5 and 16 rhs with distinct shifts: 16 rhs is the solve's batch
    (eight passes of the two-slot kernel's rhs loop, alternating reduction buffers), 5 leaves
    the second slot idle on the last pass (the generic kernel takes one rhs per work-group, so
    its path does not depend on the batch).  Every rhs against the oracle."""
    case("sap 8^4 %s variant %d nrhs %d" % (prec, sapv, nrhs))
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op = _op(dims, block)
    _force_sap(lat, tmp_path, dims, block, 1, sapv)
    f = random_spinors(dims, nrhs, seed_for(2, "b") + nrhs)
    taus = [-0.15 + 0.3 * k / max(1, nrhs - 1) for k in range(nrhs)]
    xg = lat.field(nrhs, prec)
    fg = lat.pack(dev(f), prec)
    lat.sap_smooth(xg, fg, taus, nrhs, nsweep=3, n_mr=3, prec=prec)
    got = host(lat.unpack(xg, nrhs, prec))
    if (prec, nrhs) not in _SAP_REF:
        fin = host(lat.unpack(fg, nrhs, prec))
        _SAP_REF[(prec, nrhs)] = [sap.sap(op, fin[k], np.zeros_like(f[0]), taus[k], block, 3, 3)
                                  for k in range(nrhs)]
    errs = [rel_err(got[k], _SAP_REF[(prec, nrhs)][k]) for k in range(nrhs)]
    print("max rel err %.2e" % max(errs), flush=True)
    assert max(errs) < tol, errs


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_setup_parity(prec, tol):
    """qmg_setup_mg against the oracle's setup (smoothing on A_0 w = 0, then V-cycle inverse
    iterations with interpolation rebuilds): 8^4, 8 test vectors, 4 setup iterations, 3
    smoothing steps, coarse GMRES to 0.5 (at most 20 steps).  Both sides start from the same W.
    FP64 V-cycles: the iteration is nonlinear (minimal-residual steps, a coarse GMRES whose
    length depends on a tolerance test) and repeated four times; the rounding-order
    differences measure about 1e-15, held to the FP64 bar of 1e-13.  FP32 V-cycles: each
    round adds FP32 rounding of the smoother output; the result is renormalised, and the
    difference measures about 3e-7, held to the FP32 bar of 1e-6."""
    case("setup parity 8^4 " + prec)
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op = _op(dims, block)
    ntv = 8
    W0 = random_test_vectors(dims, ntv, seed_for(2, "W"))
    Wg = lat.pack(dev(W0))
    lat.setup_mg(Wg, ntv, setup_iters=4, smooth=3, n_mr=3, coarse_maxiter=20, coarse_tol=0.5, prec=prec)
    got = host(lat.unpack(Wg, ntv))
    ref = mg.setup_test_vectors(op, list(W0), block, setup_iters=4, smooth=3, n_mr=3, coarse_iters=20,
                                coarse_tol=0.5)
    errs = [rel_err(got[j], ref[j]) for j in range(ntv)]
    print("max rel err %.2e" % max(errs), flush=True)
    assert max(errs) < tol, errs


def _mg(dims, block, ntv=8, csw=1.0):
    qmg, lat, op = _op(dims, block, csw)
    W = random_test_vectors(dims, ntv, seed_for(2, "W"))
    lat.set_test_vectors(lat.pack(dev(W)), ntv)
    return qmg, lat, op, mg.TwoLevel(op, list(W), block), lat.coarse_site_order()


@pytest.mark.parametrize("dims,block", [((8, 8, 8, 8), (4, 4, 4, 4)), ((4, 4, 4, 4), (2, 2, 2, 2))])
def test_restrict_prolong_coarse_parity(dims, block):
    case("restrict/prolong/coarse %s" % (dims,))
    ntv = 8
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    v = random_spinors(dims, 2, 31)
    yc = host(lat.restrict(lat.coarse(2), lat.pack(dev(v)), 2)).view(np.complex128)
    y = coarse_to_lex(yc, order, ntv)
    for k in range(2):
        assert rel_err(y[k], mg.restrict(h.P, v[k], block)) < 1e-13
    rng = np.random.default_rng(4)
    ylex = rng.standard_normal((2, len(order), 2 * ntv)) + 1j * rng.standard_normal((2, len(order), 2 * ntv))
    yg = dev(lex_to_coarse(ylex, order).view(np.float64))
    pv = host(lat.unpack(lat.prolong(lat.field(2), yg, 2), 2))
    for k in range(2):
        assert rel_err(pv[k], mg.prolong(h.P, ylex[k], dims, block)) < 1e-13
    taus = [0.0, 0.3]
    out = coarse_to_lex(host(lat.apply_coarse(lat.coarse(2), yg, taus, 2)).view(np.complex128), order, ntv)
    for k in range(2):
        assert rel_err(out[k], h.coarse.apply(ylex[k], taus[k])) < 1e-13


def test_coarse_gmres_fixed_iterations():
    case("coarse gmres 8^4 fixed 12 iterations")
    ntv = 8
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((2, len(order), 2 * ntv)) + 1j * rng.standard_normal((2, len(order), 2 * ntv))
    taus = [0.01, -0.05]
    yg = lat.coarse_solve(lat.coarse(2), dev(lex_to_coarse(r, order).view(np.float64)), taus, 2, iters=12, tol=0.0)
    y = coarse_to_lex(host(yg).view(np.complex128), order, ntv)
    for k in range(2):
        ref, its, _ = krylov.gmres(lambda v: h.coarse.apply(v, taus[k]), r[k], 12)
        assert its == 12
        assert rel_err(y[k], ref) < 1e-13


def test_vcycle_parity():
    case("vcycle 8^4 f64 fixed coarse iterations")
    ntv = 8
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    r = random_spinors(dims, 1, 41)
    prm = qmg.default_params(coarse_maxiter=10, coarse_tol=0.0, nu_post=2, n_mr=3)
    z = host(lat.unpack(lat.vcycle(lat.field(1), lat.pack(dev(r)), [0.02], 1, prm)))
    ref = h.vcycle(r[0], 0.02, 2, 3, 10, None)
    assert rel_err(z[0], ref) < 1e-13


def test_rank_deficient_test_vectors_rejected():
    case("rank deficient W")
    qmg, lat, op = _op((8, 8, 8, 8), (4, 4, 4, 4))
    W = random_test_vectors((8, 8, 8, 8), 4, 3)
    W[3] = W[1] * (0.5 - 0.25j)
    with pytest.raises(qmg.QmgError) as e:
        lat.set_test_vectors(lat.pack(dev(W)), 4)
    assert e.value.status == -5


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_vcycle_graph_replays(prec, tol):
    """The HIP-graph V-cycle (device-resident coarse GMRES, fixed steps): every replay,
    with eager work and synchronisations in between, matches the oracle V-cycle."""
    case("vcycle graph replays " + prec)
    ntv = 8
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    r = random_spinors(dims, 2, 43)
    taus = [0.02, -0.1]
    rg = lat.pack(dev(r))
    prm = qmg.default_params(coarse_maxiter=10, coarse_tol=0.0, nu_post=2, n_mr=3, mg_prec=prec, use_graph=1)
    prm0 = qmg.default_params(coarse_maxiter=10, coarse_tol=0.0, nu_post=2, n_mr=3, mg_prec=prec, use_graph=0)
    ref = [h.vcycle(r[k], taus[k], 2, 3, 10, None) for k in range(2)]
    eager = host(lat.unpack(lat.vcycle(lat.field(2), rg, taus, 2, prm0), 2))
    z = lat.field(2)
    for rep in range(4):
        lat.vcycle(z, rg, taus, 2, prm)          # rep 0 runs eagerly and captures; later reps replay
        got = host(lat.unpack(z, 2))
        for k in range(2):
            assert rel_err(got[k], ref[k]) < tol, (rep, k)
            assert rel_err(got[k], eager[k]) < tol, (rep, k)
        # unrelated eager work between replays
        lat.apply_Q(lat.field(1), rg, 1)
        torch.cuda.synchronize()
        z.zero_()


@pytest.mark.parametrize("ntv", [8, 24])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5), ("bf16", 2e-2)])
def test_coarse_apply_many_rhs(ntv, prec, tol):
    """Coarse apply for ragged batches (5 and 17 rhs: the MFMA path, partial 16-rhs tiles).
    FP32: each output sums 9 * 2 ntv = 432 products; rounding ~ sqrt(432) * 6e-8 ~ 1e-6 of the
    largest entry, so 1e-5 bounds it with margin.  BF16 storage of D_c: 2^-8 per entry."""
    case("coarse apply many rhs ntv=%d %s" % (ntv, prec))
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    rng = np.random.default_rng(8)
    cdt = np.complex128 if prec == "f64" else np.complex64
    rdt = np.float64 if prec == "f64" else np.float32
    for nrhs in (5, 17):
        ylex = (rng.standard_normal((nrhs, len(order), 2 * ntv))
                + 1j * rng.standard_normal((nrhs, len(order), 2 * ntv))).astype(cdt)
        taus = [0.01 * (k - 3) for k in range(nrhs)]
        yg = dev(lex_to_coarse(ylex, order).view(rdt))
        og = lat.apply_coarse(lat.coarse(nrhs, prec), yg, taus, nrhs, prec)
        out = coarse_to_lex(host(og).view(cdt), order, ntv)
        for k in range(nrhs):
            ref = h.coarse.apply(ylex[k].astype(np.complex128), taus[k])
            assert rel_err(out[k], ref) < tol, (nrhs, k)


def _block_window(U, f, X, block, csw, nwin=4):
    """Periodic window of nwin blocks per direction holding block X of the big lattice at
    window position p (1 or 2 per direction, so its 8 neighbouring blocks are inside); the
    origin sits on an even block offset so window and lattice colours agree.  The clover term
    is computed on the window plus a one-site margin (its leaves reach one site out), so no
    value the sampled block depends on sees the window's own periodic wrap.
    Returns (U, clover, f, inner slice) of the window."""
    dims = U.shape[:4]
    idx, idx_m, inner = [], [], []
    for mu in range(4):
        p = 1 if X[mu] % 2 else 2
        start = (X[mu] - p) * block[mu]
        idx.append((start + np.arange(nwin * block[mu])) % dims[mu])
        idx_m.append((start - 1 + np.arange(nwin * block[mu] + 2)) % dims[mu])
        inner.append(slice(p * block[mu], (p + 1) * block[mu]))
    Cm = oclover.clover_term(U[np.ix_(*idx_m)], csw)
    C = Cm[1:-1, 1:-1, 1:-1, 1:-1]
    sl = np.ix_(*idx)
    return U[sl], C, f[sl], tuple(inner)


def test_full_size_sap_fp32_16rhs_tuned(tmp_path):
    """64x32^3, c_sw = 1, the bench's SAP launch configuration: FP32, 16 right-hand sides with
    their own shifts tau_k = 0.002 (2k - 15), the kernel the autotuner picks.  One sweep from
    x = 0; for a colour-1 block the result depends only on f in the block and its 8
    colour-0 neighbours, so the oracle's SAP on a 4^4-block window (FP64 links and clover, f
    as the GPU stored it) reproduces it up to the FP32 arithmetic.  rhs 0 and 15, two sampled
    blocks each."""
    from gpu_common import big_inputs, torch
    from synth import device_gaussian_spinors
    case("full-size SAP FP32 16 rhs, tuned")
    qmg = need_gpu()
    dims, block = (64, 32, 32, 32), (4, 4, 4, 4)
    U, _ = big_inputs(dims, 0.5, 5, 1)
    m0, csw = -0.95, 1.0
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    lat.autotune(str(tmp_path / "tune.json"))
    nrhs = 16
    taus = [0.002 * (2 * k - 15) for k in range(nrhs)]
    fg = lat.pack(device_gaussian_spinors(dims, nrhs, seed_for(5, "b")), "f32")
    xg = lat.field(nrhs, "f32")
    lat.sap_smooth(xg, fg, taus, nrhs, nsweep=1, n_mr=3, prec="f32")
    xs = lat.unpack(xg, nrhs, "f32")
    fs = lat.unpack(fg, nrhs, "f32")
    rng = np.random.default_rng(21)
    nbk = [d // b for d, b in zip(dims, block)]
    errs = []
    for k in (0, nrhs - 1):
        fk = host(fs[k])
        done = 0
        while done < 2:
            X = [int(rng.integers(0, n)) for n in nbk]
            if sum(X) % 2 != 1:
                continue
            Uw, C, fw, inner = _block_window(U, fk, X, block, csw)
            ref = sap.sap(dirac.Operator(Uw, m0, C), fw, np.zeros_like(fw), taus[k], block, 1, 3)[inner]
            sl = tuple(slice(X[mu] * block[mu], (X[mu] + 1) * block[mu]) for mu in range(4))
            errs.append(rel_err(host(xs[k][sl]), ref))
            done += 1
        del fk
    print("max rel err %.2e" % max(errs), flush=True)
    assert max(errs) < 1e-6, errs


def test_full_size_coarse_apply_fp32_16rhs_tuned(tmp_path):
    """64x32^3, c_sw = 1, 24 test vectors: the coarse apply (D_c - tau_k Gamma5^c), the restriction
    and the prolongation in the bench's launch configuration (FP32, 16 right-hand sides, the
    kernels the autotuner picks) on sampled coarse sites and blocks.  Reference: D_c = P^H D P, so at coarse site X it needs P y on block X and its
    8 neighbours only; the oracle prolongs there (P of each block from its own test vectors),
    applies D on a 3-block window around X (links and clover of the big lattice) and restricts
    on X.  The input is the FP32 vector the GPU read."""
    from gpu_common import big_inputs
    case("full-size coarse apply FP32 16 rhs, tuned")
    qmg = need_gpu()
    dims, block = (64, 32, 32, 32), (4, 4, 4, 4)
    U, _ = big_inputs(dims, 0.5, 5, 1)
    m0, csw, ntv = -0.95, 1.0, 24
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    W = random_test_vectors(dims, ntv, seed_for(5, "W"))
    lat.set_test_vectors(lat.pack(dev(W)), ntv)
    lat.autotune(str(tmp_path / "tune.json"))
    order = lat.coarse_site_order()
    nrhs = 16
    taus = [0.002 * (2 * k - 15) for k in range(nrhs)]
    rng = np.random.default_rng(8)
    ylex = (rng.standard_normal((nrhs, len(order), 2 * ntv))
            + 1j * rng.standard_normal((nrhs, len(order), 2 * ntv))).astype(np.complex64)
    yg = dev(lex_to_coarse(ylex, order).view(np.float32))
    out = coarse_to_lex(host(lat.apply_coarse(lat.coarse(nrhs, "f32"), yg, taus, nrhs, "f32")).view(np.complex64),
                        order, ntv)
    nbk = [d // b for d, b in zip(dims, block)]

    def lex(Y):
        return ((Y[0] * nbk[1] + Y[1]) * nbk[2] + Y[2]) * nbk[3] + Y[3]

    def gslice(Y):
        return tuple(slice(Y[mu] * block[mu], (Y[mu] + 1) * block[mu]) for mu in range(4))

    errs = []
    for _ in range(3):
        X = [int(rng.integers(0, n)) for n in nbk]
        idx = [((X[mu] - 1) * block[mu] + np.arange(3 * block[mu])) % dims[mu] for mu in range(4)]
        Uw = U[np.ix_(*idx)]
        Cw = oclover.clover_term(Uw, csw)
        nine = [(1, 1, 1, 1)] + [tuple(1 + (s if m == mu else 0) for m in range(4))
                                 for mu in range(4) for s in (1, -1)]
        Ps = {}
        for wpos in nine:
            Yg = [(X[mu] + wpos[mu] - 1) % nbk[mu] for mu in range(4)]
            Ps[wpos] = (mg.build_P([w[gslice(Yg)] for w in W], block), lex(Yg))
        PX, lX = Ps[(1, 1, 1, 1)]
        for k in (0, nrhs - 1):
            v = np.zeros(tuple(3 * b for b in block) + (4, 3), dtype=np.complex128)
            for wpos, (P, ly) in Ps.items():
                v[gslice(wpos)] = mg.prolong(P, ylex[k][ly][None, :].astype(np.complex128), block, block)
            Dv = dirac.apply_D(Uw, v, m0, Cw)[gslice((1, 1, 1, 1))]
            yX = ylex[k][lX].astype(np.complex128)
            ref = mg.restrict(PX, Dv, block)[0] - taus[k] * mg.gamma5_coarse(yX)
            errs.append(rel_err(out[k][lX], ref))
    print("max rel err %.2e" % max(errs), flush=True)
    assert max(errs) < 1e-5, errs
    # restriction and prolongation of 16 FP32 fields (the MFMA kernels), sampled blocks: the
    # aggregate of block b only sees P_b and the field on block b
    from synth import device_gaussian_spinors
    vg = lat.pack(device_gaussian_spinors(dims, nrhs, seed_for(5, "x")), "f32")
    vs = lat.unpack(vg, nrhs, "f32")
    yr = coarse_to_lex(host(lat.restrict(lat.coarse(nrhs, "f32"), vg, nrhs, "f32")).view(np.complex64), order, ntv)
    pv = lat.unpack(lat.prolong(lat.field(nrhs, "f32"), yg, nrhs, "f32"), nrhs, "f32")
    terr, perr = [], []
    for _ in range(3):
        Y = [int(rng.integers(0, n)) for n in nbk]
        P = mg.build_P([w[gslice(Y)] for w in W], block)
        for k in (0, nrhs - 1):
            terr.append(rel_err(yr[k][lex(Y)], mg.restrict(P, host(vs[k][gslice(Y)]), block)[0]))
            perr.append(rel_err(host(pv[k][gslice(Y)]),
                                mg.prolong(P, ylex[k][lex(Y)][None, :].astype(np.complex128), block, block)))
    print("restriction %.2e, prolongation %.2e" % (max(terr), max(perr)), flush=True)
    assert max(terr) < 2e-6 and max(perr) < 2e-6, (terr, perr)


def test_full_size_sap_and_restrict_sampled():
    """64x32^3, c_sw = 1, 16 rhs batch layout of the bench: one FP64 SAP sweep from x = 0 and the
    restriction, checked on sampled blocks.  For a colour-1 block the sweep depends only on f in the
    block and its 8 neighbouring colour-0 blocks, so a 4^4-block window reproduces it exactly."""
    from gpu_common import big_inputs
    case("full-size SAP / restrict sampled")
    qmg = need_gpu()
    dims, block = (64, 32, 32, 32), (4, 4, 4, 4)
    U, f = big_inputs(dims, 0.5, 5, 2)
    m0, csw, tau = -0.8, 1.0, 0.0125
    lat = qmg.Lattice(dims, block)
    lat.set_gauge(dev(U), m0, csw)
    fg = lat.pack(dev(f))
    xg = lat.field(2)
    lat.sap_smooth(xg, fg, [tau, tau], 2, nsweep=1, n_mr=3)
    xs = lat.unpack(xg, 2)
    rng = np.random.default_rng(12)
    nbk = [d // b for d, b in zip(dims, block)]
    done = 0
    while done < 2:
        X = [int(rng.integers(0, n)) for n in nbk]
        if sum(X) % 2 != 1:   # colour-1 block: its residual reads the colour-0 neighbours
            continue
        Uw, C, fw, inner = _block_window(U, f[0], X, block, csw)
        ref = sap.sap(dirac.Operator(Uw, m0, C), fw, np.zeros_like(fw), tau, block, 1, 3)[inner]
        sl = tuple(slice(X[mu] * block[mu], (X[mu] + 1) * block[mu]) for mu in range(4))
        got = host(xs[0][sl])
        assert rel_err(got, ref) < 1e-13
        done += 1
    # restriction: the aggregate of block b only sees P_b (built from W on block b) and v on block b
    ntv = 24
    W = random_test_vectors(dims, ntv, seed_for(5, "W"))
    lat.set_test_vectors(lat.pack(dev(W)), ntv)
    order = lat.coarse_site_order()
    yc = coarse_to_lex(host(lat.restrict(lat.coarse(2), fg, 2)).view(np.complex128), order, ntv)
    for _ in range(3):
        X = [int(rng.integers(0, n)) for n in nbk]
        sl = tuple(slice(X[mu] * block[mu], (X[mu] + 1) * block[mu]) for mu in range(4))
        Pb = mg.build_P([w[sl] for w in W], block)
        ref = mg.restrict(Pb, f[1][sl], block)[0]
        lex = ((X[0] * nbk[1] + X[1]) * nbk[2] + X[2]) * nbk[3] + X[3]
        assert rel_err(yc[1][lex], ref) < 1e-13
    # coarse operator, any size: Q_c = Gamma5^c D_c is Hermitian, <u, Q_c v> = <Q_c u, v>
    nc = 2 * ntv
    u = (rng.standard_normal((len(order), nc)) + 1j * rng.standard_normal((len(order), nc)))
    v = (rng.standard_normal((len(order), nc)) + 1j * rng.standard_normal((len(order), nc)))
    g5 = np.concatenate([np.ones(ntv), -np.ones(ntv)])
    Du = host(lat.apply_coarse(lat.coarse(1), dev(u.view(np.float64)), [0.0])).view(np.complex128).reshape(u.shape)
    Dv = host(lat.apply_coarse(lat.coarse(1), dev(v.view(np.float64)), [0.0])).view(np.complex128).reshape(v.shape)
    a = np.vdot(u, g5 * Dv)
    b = np.vdot(g5 * Du, v)
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_restrict_prolong_ragged_batches(prec, tol):
    """Restriction / prolongation kernels that share P loads across right-hand sides,
    on ragged batches (1, 5, 7 rhs) with 24 test vectors."""
    case("restrict/prolong ragged " + prec)
    ntv = 24
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    qmg, lat, op, h, order = _mg(dims, block, ntv)
    cdt = np.complex128 if prec == "f64" else np.complex64
    rdt = np.float64 if prec == "f64" else np.float32
    rng = np.random.default_rng(21)
    for nrhs in (1, 5, 7):
        v = random_spinors(dims, nrhs, 100 + nrhs)
        vg = lat.pack(dev(v), prec)
        vin = host(lat.unpack(vg, nrhs, prec))
        y = coarse_to_lex(host(lat.restrict(lat.coarse(nrhs, prec), vg, nrhs, prec)).view(cdt), order, ntv)
        for k in range(nrhs):
            assert rel_err(y[k], mg.restrict(h.P, vin[k], block)) < tol, (nrhs, k)
        ylex = (rng.standard_normal((nrhs, len(order), 2 * ntv))
                + 1j * rng.standard_normal((nrhs, len(order), 2 * ntv))).astype(cdt)
        pv = host(lat.unpack(lat.prolong(lat.field(nrhs, prec), dev(lex_to_coarse(ylex, order).view(rdt)), nrhs,
                                         prec), nrhs, prec))
        for k in range(nrhs):
            assert rel_err(pv[k], mg.prolong(h.P, ylex[k].astype(np.complex128), dims, block)) < tol, (nrhs, k)
