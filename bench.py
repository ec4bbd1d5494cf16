"""Benchmark of the shifted-solve hot path on one MI355X.

Workload (config 5): 64x32^3 lattice, clover c_sw = 1.0, synthetic links
exp(i*0.5*H), near-critical bare mass (m0 = -0.95 from tests/golden/
m0_critical.json), 16 right-hand sides with shifts tau_k = 0.002*(2k - 15),
two-level multigrid (4^4 aggregates, 24 test vectors, 6 setup iterations),
FP64 FGMRES(6) to a 1e-10 true relative residual.

A step is one batched shifted solve of the 16 right-hand sides with the
mixed-precision (FP32) V-cycle -- every kernel of the path (stencil, SAP,
restriction, coarse GMRES, prolongation, FP64 Gram-Schmidt) runs inside it.
`value` = right-hand sides solved per second.  Also reported: the FP64- and
BF16-preconditioned solve times, Q-apply GFLOP/s and GB/s, the roofline of
the dominant kernel and the oracle's CPU throughput on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FLOP_SITE = 1320
# published MI355X FP32 vector peak; the kernels are built without packed FP32
# arithmetic, whose issue ceiling is half of it (256 CU x 4 SIMD x 16 lanes x
# 2 flop x 2.4 GHz = 78.6 TFLOP/s)
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_NONPACKED_TFLOPS = 78.6
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_64x32x32x32_16rhs.json")
# sources that define each profiled kernel: a change to any of them voids its counters
KERNEL_SOURCES = {
    "sap_f32": ["paper_2004_08146_amd/csrc/sap.hip", "paper_2004_08146_amd/csrc/qmg_device.h"],
    "stencil_f32": ["paper_2004_08146_amd/csrc/dslash.hip", "paper_2004_08146_amd/csrc/qmg_device.h",
                    "paper_2004_08146_amd/csrc/tune.hip"],
}
KERNEL_NAMES = {"sap_f32": "k_sap44<float, true, 2, false>", "stencil_f32": "k_dslash"}


def sap_flops_per_site(n_mr):
    """Algorithmic flops of one SAP half-sweep per site of that colour and per
    rhs: the residual f - A x (8 hops at 1320, clover 552, diagonal and shift
    48, subtraction 24) and n_MR block minimal-residual steps, each a block
    operator (in-block hops only: 6 of 8 on a 4^4 block, 990; clover 552;
    diagonal 48) plus the MR inner products and updates (336)."""
    return (1320 + 552 + 48 + 24) + n_mr * (990 + 552 + 48 + 336)


def eigensolver_run(args, torch, qmg, random_links, seed_for, device_gaussian_spinors, m0):
    """GD-lambdaAMG (Alg. GD-lambdaAMG) on a second synthetic lattice: setup with
    24 test vectors, then nev eigenpairs of Q of smallest modulus to a 1e-8
    residual with the paper's default parameters (m_min 30, m_max 50, inner
    FGMRES to 0.1 or 5 iterations, coarse tolerance 0.5, interpolation
    updates), BF16-storage V-cycle by default (--eig-prec).  Residuals are
    recomputed with the library's operator."""
    dims = tuple(int(v) for v in args.eig_dims.split(","))
    t0 = time.time()
    U = random_links(dims, 0.5, seed_for(4, "U"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(U).cuda(), m0, 1.0)
    del U
    ntv = 24
    W = lat.pack(device_gaussian_spinors(dims, ntv, seed_for(4, "W")))
    lat.setup_mg(W, ntv, setup_iters=6, smooth=4)
    solve = {"mg_prec": args.eig_prec}
    if args.eig_levels == 3:
        # inner solves with a third level (2^4 aggregates of blocks, 24 level-2 vectors)
        k2, k3, s2 = (int(v) for v in (args.l3 or "4,8,2").split(","))
        W2 = lat.level2_vectors_from(W, ntv)
        lat.setup_level3(W2, ntv, (2, 2, 2, 2), setup_iters=3, smooth=s2, l3_iters=20)
        del W2
        solve.update(levels=3, coarse_maxiter=k2, l3_iters=k3, l2_smooth=s2)
    lat.autotune(None)
    t0v = lat.pack(device_gaussian_spinors(dims, 1, seed_for(4, "x")))
    X = lat.field(args.eig_nev)
    prm = qmg.default_eig_params(block=args.eig_block, solve=solve, both_signs=args.eig_both_signs)
    torch.cuda.synchronize()
    print("[bench] eigensolver inputs and setup %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    st, lam, stats = lat.eigensolve(args.eig_nev, X, t0v, V0=W, n0=ntv, params=prm)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t1
    fb = lat.field_bytes()
    res = []
    for k in range(len(lam)):
        x = X[k * fb:(k + 1) * fb]
        r = lat.apply_Q_shifted(lat.field(1), x, [float(lam[k])], 1)
        res.append(float(np.sqrt(max(0.0, lat.field_dot(r, r)[0].real))))
    print("[bench] eigensolver %.1f s: %d pairs, status %d" % (sec, len(lam), st), file=sys.stderr, flush=True)
    return {"workload": "%s clover (c_sw 1, m0 %.2f), %d eigenpairs of Q of smallest |lambda|, tol 1e-8, "
                        "%s V-cycle in the inner solves" % ("x".join(map(str, dims)), m0, args.eig_nev, args.eig_prec),
            "seconds": sec, "status": st, "eigenpairs_per_s": len(lam) / sec,
            "outer_iters": stats["iters"], "inner_fgmres_iters": stats["inner_iters"],
            "interp_updates": stats["interp_updates"], "block": args.eig_block, "levels": args.eig_levels,
            "both_signs": args.eig_both_signs, "negative_pairs": int(np.sum(np.asarray(lam) < 0)),
            "inner_prec": args.eig_prec,
            "max_residual": max(res) if res else None,
            "lambda_abs_range": [float(np.min(np.abs(lam))), float(np.max(np.abs(lam)))] if len(lam) else None}


def config4_run(args, torch, qmg, random_links, random_spinors, seed_for, device_gaussian_spinors, m0):
    """The 32^4 mixed-precision workload: c_sw = 1, near-critical m0, two-level
    multigrid (4^4 aggregates, 24 test vectors, 6 setup iterations), 8 shifts
    tau_k = 0.005 (2k - 7) in one batch, FGMRES(6) to 1e-10 with the V-cycle in
    FP32, BF16 storage or FP64 (graph mode, 20 coarse steps).  Each solve is run
    once to record its graph, then timed."""
    dims, nrhs = (32, 32, 32, 32), 8
    t0 = time.time()
    U = random_links(dims, 0.5, seed_for(4, "U"))
    b = random_spinors(dims, nrhs, seed_for(4, "b"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(U).cuda(), m0, 1.0)
    del U
    bg = lat.pack(torch.from_numpy(b).cuda())
    del b
    W = lat.pack(device_gaussian_spinors(dims, 24, seed_for(4, "W")))
    torch.cuda.synchronize()
    t1 = time.time()
    lat.setup_mg(W, 24, setup_iters=6, smooth=4, n_mr=3, coarse_maxiter=20, coarse_tol=0.5)
    torch.cuda.synchronize()
    setup_s = time.time() - t1
    del W
    lat.autotune(os.path.join("/tmp", "qmg_tune_c4_%d.json" % os.getpid()))
    taus = [0.005 * (2 * k - 7) for k in range(nrhs)]
    out = {"workload": "32^4 clover (c_sw 1, m0 %.2f), 8 shifts tau_k = 0.005(2k - 7) in one batch, two-level MG, "
                       "FGMRES(6) to 1e-10" % m0, "setup_s": setup_s, "solves": {}}
    for prec in ("f32", "bf16", "f64"):
        prm = qmg.default_params(mg_prec=prec, restart=6, maxiter=500, use_graph=1, coarse_maxiter=20)
        x = lat.field(nrhs)
        lat.solve_shifted(x, bg, taus, nrhs, prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, stats = lat.solve_shifted(x, bg, taus, nrhs, prm)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t1)
        out["solves"][prec] = {"ms": ms, "rhs_per_s": nrhs / (ms / 1000.0), "status": st,
                               "iters": [s_["iters"] for s_ in stats],
                               "max_true_relres": max(s_["true_relres"] for s_ in stats)}
        del x
    print("[bench] config-4 leg %.1f s: %s" % (time.time() - t0, json.dumps(out["solves"])), file=sys.stderr,
          flush=True)
    return out


def sources_hash(names):
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(key):
    """HBM bytes per launch of a profiled kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a 1 GiB copy), or
    None when the kernel's sources changed after the counters were taken."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get("kernels", {}).get(key)
    if not e or e.get("sources_sha256_16") != sources_hash(KERNEL_SOURCES[key]):
        return None
    return e["hbm_bytes_per_launch"]


def summarize_pmc(fetch_dir, write_dir, cmd):
    """Writes the traffic summary from two rocprofv3 --pmc runs of the kernels
    mode (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  The factors that map
    the counters to bytes come from the same runs' 1 GiB device copy."""
    import csv
    import glob

    def dispatches(d):
        rows = {}
        for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
            for r in csv.DictReader(open(f)):
                k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                rows[k] = rows.get(k, 0.0) + float(r["Counter_Value"])
        return [(i, n, v) for (i, n), v in sorted(rows.items())]

    def short(n):
        n = n.replace("(anonymous namespace)::", "")
        if n.startswith("void "):
            n = n[5:]
        return n.split("(")[0]

    fet, wri = dispatches(fetch_dir), dispatches(write_dir)
    cfet = [v for _, n, v in fet if "copyBuffer" in n and v > 1e5]
    cwri = [v for _, n, v in wri if "copyBuffer" in n and v > 1e5]
    cf = (1 << 30) / 1024.0 / np.mean(cfet)
    cw = (1 << 30) / 1024.0 / np.mean(cwri)
    out = {"command_fetch": cmd % ("FETCH_SIZE", "fetch"), "command_write": cmd % ("WRITE_SIZE", "write"),
           "calibration": {"kernel": "__amd_rocclr_copyBuffer (torch copy_ of 1 GiB)", "bytes_read": 1 << 30,
                           "bytes_written": 1 << 30, "fetch_factor": cf, "write_factor": cw},
           "note": "per-launch averages over the kernels mode's own timed launches (the last ones of that "
                   "kernel: after the autotuner), HBM bytes = 1024 * (FETCH_SIZE * fetch_factor + "
                   "WRITE_SIZE * write_factor)",
           "kernels": {}}
    # the kernels mode runs, after the autotuner: f64 1-rhs apply x4, f32 16-rhs apply x4, SAP sweep x3 (6 launches)
    picks = {"stencil_f32": (lambda n: short(n).startswith("k_dslash") and "float" in short(n)
                             and "double" not in short(n), 4),
             "sap_f32": (lambda n: short(n) == KERNEL_NAMES["sap_f32"], 6)}
    for key, (match, last) in picks.items():
        fsel = [(i, n, v) for i, n, v in fet if match(n)][-last:]
        wsel = [(i, n, v) for i, n, v in wri if match(n)][-last:]
        if not fsel or not wsel:
            continue
        f_kib, w_kib = float(np.mean([v for _, _, v in fsel])), float(np.mean([v for _, _, v in wsel]))
        out["kernels"][key] = {"kernel": short(fsel[-1][1]), "launches": len(fsel),
                               "fetch_kib": f_kib, "write_kib": w_kib,
                               "hbm_bytes_per_launch": 1024.0 * (f_kib * cf + w_kib * cw),
                               "sources_sha256_16": sources_hash(KERNEL_SOURCES[key])}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def spinor_bytes(prec):
    return 12 * {"f64": 16, "f32": 8, "bf16": 4}[prec]


def apply_bytes_per_site(prec, nrhs, clover):
    """Algorithmic HBM bytes per site of one Q apply on nrhs fields: read the
    input and write the output once per rhs, read 4 links (and the clover
    blocks) once for all rhs."""
    c = {"f64": 16, "f32": 8, "bf16": 4}[prec]
    per_rhs = 2 * spinor_bytes(prec)
    shared = 4 * 9 * c + (36 * c if clover else 0)
    return per_rhs * nrhs + shared


def sap_bytes_per_site(prec, nrhs, clover):
    """Algorithmic HBM bytes per lattice site of one SAP sweep (both colours):
    f read, x read, x write, neighbouring-block faces of x (8 faces x 1/4 of a
    4^4 block's sites), links and clover once per rhs-batch."""
    c = {"f64": 16, "f32": 8, "bf16": 4}[prec]
    per_rhs = (3 + 2) * spinor_bytes(prec)
    shared = (4 * 9 + 9) * c + (36 * c if clover else 0)
    return per_rhs * nrhs + shared


def roofline_entry(kernel, flops, alg_bytes, launch_ms, flop_peak_tf, traffic):
    """Roofline of one kernel launch, the bound chosen from the evidence: the
    algorithmic arithmetic intensity (flops / algorithmic bytes) against the
    ridge point of the published peaks (flop_peak_tf / 8 TB/s).  Below the ridge
    HBM binds and `achieved` is algorithmic GB/s; above it the arithmetic peak
    binds.  Both fractions are kept, plus the fraction of the issue ceiling
    without packed FP32 (half the published FP32 vector peak)."""
    ai = flops / alg_bytes
    ridge = flop_peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    gbs = alg_bytes / launch_ms / 1e6
    tfs = flops / launch_ms / 1e9
    out = {"kernel": kernel, "launch_ms": launch_ms, "flops_per_launch": flops, "alg_bytes_per_launch": alg_bytes,
           "arith_intensity_flop_per_byte": ai, "ridge_flop_per_byte": ridge,
           "hbm_gbps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "tflops": tfs, "alu_frac": tfs / flop_peak_tf,
           "frac_of_nonpacked_issue_peak": tfs / FP32_NONPACKED_TFLOPS,
           "traffic": traffic}
    if ai < ridge:
        out.update({"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS})
    else:
        out.update({"bound": "alu", "achieved": tfs, "peak": flop_peak_tf, "unit": "TFLOP/s",
                    "frac": tfs / flop_peak_tf})
    return out


class EventTimer:
    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, reps):
        t = self.torch
        fn()
        t.cuda.synchronize()
        s = t.cuda.Event(enable_timing=True)
        e = t.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        t.cuda.synchronize()
        return s.elapsed_time(e) / reps


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": os.cpu_count(), "cpus_available": avail, "model": model}


def cpu_baseline(U, b0, m0, csw, tau, applies_per_rhs):
    """The oracle (NumPy FP64) timed on this host.  The NumPy oracle is
    single-threaded (its elementwise and einsum kernels run on one core), so
    every figure is one core.

    * The workload's own (Q - tau) apply on the whole lattice (64x32^3, clover),
      one right-hand side, timed once after a warm-up apply on a 16^4 slice.
      The oracle's clover term is built beforehand (untimed) on t-slabs in
      worker processes (tests/oracle_slabs.py).  rhs/s = 1 / (apply time x the
      number of fine-operator applications the GPU solve made per right-hand side:
      an estimate; a full oracle solve at this size would take days).
    * The same apply on a 16^4 lattice: median of 5 after a warm-up.
    * A timed oracle solve: two-level multigrid FGMRES to 1e-10 on 8^4 (8 test
      vectors, 2 setup rounds), 1 right-hand side, with the 16^4 workload's
      m0 = -0.8 and tau = 0.01 -- at 16^4 the oracle needs minutes per V-cycle."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle import clover, dirac, mg
    from oracle.solve import solve_shifted
    from oracle_slabs import default_procs, full_clover
    from synth import random_links, random_spinors, random_test_vectors, seed_for

    out = {"unit": "rhs/s", "cores": 1, "kind": "oracle", "threads": "1 (the NumPy oracle is single-threaded)"}
    out.update(cpu_info())
    t0 = time.perf_counter()
    C = full_clover(U, csw)
    clover_s = time.perf_counter() - t0
    # warm-up on a 16^4 slice, then the whole lattice once
    Us, Cs, xs = (np.ascontiguousarray(a[:16, :16, :16, :16]) for a in (U, C, b0[0]))
    dirac.apply_Q_shifted(Us, xs, m0, tau, Cs)
    t0 = time.perf_counter()
    dirac.apply_Q_shifted(U, b0[0], m0, tau, C)
    t_full = time.perf_counter() - t0
    del C
    V = int(np.prod(U.shape[:4]))
    out["value"] = 1.0 / (t_full * applies_per_rhs)
    out["full_apply_s"] = t_full
    out["full_apply_gflops"] = FLOP_SITE * V / t_full / 1e9
    out["clover_build_s_untimed_slab_processes"] = clover_s
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        dirac.apply_Q_shifted(Us, xs, m0, tau, Cs)
        ts.append(time.perf_counter() - t0)
    out["apply_16x4_median_s"] = float(np.median(ts))
    out["apply_16x4_gflops"] = FLOP_SITE * 16 ** 4 / float(np.median(ts)) / 1e9
    dims8, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U8 = random_links(dims8, 0.5, seed_for(4, "U"))
    op = dirac.Operator(U8, -0.8, clover.clover_term(U8, csw))
    t0 = time.perf_counter()
    W = mg.setup_test_vectors(op, list(random_test_vectors(dims8, 8, seed_for(4, "W"))), block, setup_iters=2,
                              smooth=3, n_mr=3, coarse_iters=20, coarse_tol=0.5)
    h = mg.TwoLevel(op, W, block)
    t1 = time.perf_counter()
    b8 = random_spinors(dims8, 1, seed_for(4, "b"))[0]
    x, it, hist = solve_shifted(op, b8, 0.01, block, mg=h, tol=1e-10, restart=8, maxiter=100)
    t2 = time.perf_counter()
    out["solve_8x4"] = {"setup_s": t1 - t0, "solve_s": t2 - t1, "fgmres_iters": it, "true_relres": hist[-1],
                        "rhs_per_s": 1.0 / (t2 - t1)}
    out["sample"] = ("the workload's FP64 (Q - tau) apply on the whole 64x32^3 clover lattice, one rhs, one thread: "
                     "%.1f s (clover term built beforehand on t-slabs in %d processes, untimed); rhs/s = 1 / "
                     "(apply time x %.0f fine-operator applications per rhs of the GPU solve). Also: 16^4 apply "
                     "median of 5, and a whole oracle two-level solve on 8^4" % (t_full, default_procs(),
                                                                              applies_per_rhs))
    return out


MFMA_JSON = os.path.join(ROOT, "profiles", "mfma_64x32x32x32_16rhs.json")
MFMA_SOURCES = ["paper_2004_08146_amd/csrc/coarse.hip", "paper_2004_08146_amd/csrc/transfer.hip",
                "paper_2004_08146_amd/csrc/qmg_device.h"]


def mfma_util_for(kernel):
    """rocprof MFMA utilisation (percent) of a kernel from the committed summary,
    or None when the summary is missing or its sources have changed since."""
    try:
        with open(MFMA_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("sources_sha256_16") != sources_hash(MFMA_SOURCES):
        return None
    e = d.get("kernels", {}).get(kernel)
    return e["mfma_util_pct"] if e else None
MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}  # MI355X dense MFMA peaks (FP32, FP64)


def mfma_mode(args, dims, torch, qmg, device_gaussian_spinors, random_links, seed_for):
    """The multigrid's MFMA kernels at the solve's shape: coarse apply (FP32 and
    FP64, 16 rhs), restriction and prolongation (FP32, 16 rhs), each timed with
    HIP events; run under rocprofv3 --pmc MfmaUtil MfmaFlopsF32 MfmaFlopsF64 for
    the matrix units' utilisation.  P comes from random test vectors (the work
    does not depend on their values)."""
    V = int(np.prod(dims))
    nrhs = args.nrhs
    U = random_links(dims, 0.5, seed_for(5, "U"))
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(U).cuda(), args.m0, 1.0)
    del U
    ntv = 24
    W = lat.pack(device_gaussian_spinors(dims, ntv, seed_for(5, "W")))
    lat.set_test_vectors(W, ntv)
    del W
    lat.autotune(args.tune_cache or os.path.join("/tmp", "qmg_tune_m_%d.json" % os.getpid()))
    timer = EventTimer(torch)
    taus = [0.001 * (2 * k - (nrhs - 1)) for k in range(nrhs)]
    nb = V // 256
    nc = 2 * ntv
    out = {}
    for prec in ("f32", "f64"):
        yc = lat.coarse(nrhs, prec)
        oc = lat.coarse(nrhs, prec)
        ms = timer(lambda: lat.apply_coarse(oc, yc, taus, nrhs, prec), 10)
        # one complex multiply-add = 4 real MFMA products = 8 flop
        fl = 8.0 * 9 * nc * nc * nrhs * nb
        out["coarse_apply_%s" % prec] = {"ms": ms, "mfma_flop": fl, "tflops": fl / ms / 1e9,
                                         "frac_of_mfma_peak": fl / ms / 1e9 / MFMA_PEAK_TFLOPS[prec]}
        del yc, oc
    f = lat.field(nrhs, "f32")
    yc = lat.coarse(nrhs, "f32")
    fl = 8.0 * 12 * ntv * nrhs * V  # P^H v: 12 components x ntv columns per site and rhs
    ms = timer(lambda: lat.restrict(yc, f, nrhs, "f32"), 10)
    out["restrict_f32"] = {"ms": ms, "mfma_flop": fl, "tflops": fl / ms / 1e9,
                           "frac_of_mfma_peak": fl / ms / 1e9 / MFMA_PEAK_TFLOPS["f32"]}
    ms = timer(lambda: lat.prolong(f, yc, nrhs, "f32"), 10)
    out["prolong_f32"] = {"ms": ms, "mfma_flop": fl, "tflops": fl / ms / 1e9,
                          "frac_of_mfma_peak": fl / ms / 1e9 / MFMA_PEAK_TFLOPS["f32"]}
    print(json.dumps({"mode": "mfma", "dims": list(dims), "nrhs": nrhs, "ntv": ntv, "kernels": out}))


def summarize_mfma(pmc_dir, cmd):
    """MFMA utilisation per kernel from a rocprofv3 --pmc MfmaUtil MfmaFlopsF32
    MfmaFlopsF64 run of the mfma mode (the last 10 dispatches of each kernel:
    the timed ones)."""
    import csv
    import glob
    rows = {}
    for f in glob.glob(os.path.join(pmc_dir, "*counter_collection.csv")):
        for r in csv.DictReader(open(f)):
            k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            rows.setdefault(k, {})[r["Counter_Name"]] = rows.get(k, {}).get(r["Counter_Name"], 0.0) + \
                float(r["Counter_Value"])
    disp = sorted(rows.items())

    def short(n):
        n = n.replace("(anonymous namespace)::", "")
        if n.startswith("void "):
            n = n[5:]
        return n.split("(")[0]

    out = {"command": cmd, "note": "MfmaUtil = 100 * SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE * SIMDs); "
                                   "MfmaFlops = MFMA MOPS * 512; averages over the last 10 dispatches",
           "kernels": {}}
    for name in sorted({short(n) for (_, n), _ in disp}):
        if "mfma" not in name:
            continue
        sel = [v for (_, n), v in disp if short(n) == name][-10:]
        out["kernels"][name] = {
            "dispatches": len(sel),
            "mfma_util_pct": float(np.mean([v.get("MfmaUtil", 0.0) for v in sel])),
            "mfma_flops_f32": float(np.mean([v.get("MfmaFlopsF32", 0.0) for v in sel])),
            "mfma_flops_f64": float(np.mean([v.get("MfmaFlopsF64", 0.0) for v in sel]))}
    out["sources_sha256_16"] = sources_hash(MFMA_SOURCES)
    with open(MFMA_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def kernels_mode(args, dims, torch, qmg, unit_links):
    """A few launches of each hot kernel (memory traffic does not depend on the
    field values, so unit links are used) plus a plain 1 GiB device copy whose
    known size calibrates the HBM byte counters."""
    V = int(np.prod(dims))
    nrhs = args.nrhs
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(unit_links(dims)).cuda(), args.m0, 1.0)
    # the same launch choices as the solve bench: a fresh autotune unless told otherwise
    lat.autotune(args.tune_cache or os.path.join("/tmp", "qmg_tune_k_%d.json" % os.getpid()))
    if args.variant is not None:
        # pin one stencil variant (and the XCD remap) for counter runs
        key = "gfx950|%s|4x4x4x4|clover=1" % "x".join(map(str, dims))
        path = "/tmp/qmg_pin_%d.json" % os.getpid()
        with open(path, "w") as fh:
            ent = ['"%s|dslash|%s|%d": %d' % (key, p, c, args.variant) for p in ("f64", "f32", "bf16") for c in (0, 1)]
            ent.append('"%s|xcd_remap": %d' % (key, args.remap))
            fh.write("{\n" + ",\n".join(ent) + "\n}\n")
        lat.autotune(path)
    timer = EventTimer(torch)
    taus = [0.0] * nrhs
    out = {}
    for prec, n in (("f64", 1), ("f32", nrhs)):
        a = lat.field(n, prec)
        o = lat.field(n, prec)
        ms = timer(lambda: lat.apply_Q_shifted(o, a, taus[:n], n, prec), 3)
        byts = apply_bytes_per_site(prec, n, True) * V
        out["apply_%s_%d" % (prec, n)] = {"ms": ms, "alg_bytes": byts, "gbps": byts / ms / 1e6}
        del a, o
    xs = lat.field(nrhs, "f32")
    fs = lat.field(nrhs, "f32")
    ms = timer(lambda: lat.sap_smooth(xs, fs, taus, nrhs, 1, 3, "f32"), 2)
    out["sap_f32_%d" % nrhs] = {"ms": ms, "alg_bytes": sap_bytes_per_site("f32", nrhs, True) * V}
    del xs, fs
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    ms = timer(lambda: dst.copy_(src), 3)
    out["copy_1GiB"] = {"ms": ms, "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                        "gbps": 2 * (1 << 30) / ms / 1e6}
    # the library's own streaming kernels on 1 GiB fields: read-only (dot) and copy
    nf = (1 << 30) // lat.field_bytes("f64")
    fa = lat.field(nf, "f64")
    fb = lat.field(nf, "f64")
    ms = timer(lambda: lat.field_dot(fa, fa, nf, "f64"), 3)
    out["dot_1GiB_read"] = {"ms": ms, "gbps": nf * lat.field_bytes("f64") / ms / 1e6}
    del fa, fb
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=str, default="64,32,32,32")
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--m0", type=float, default=None,
                    help="bare mass (default: the near-critical value in tests/golden/m0_critical.json)")
    ap.add_argument("--setup-iters", type=int, default=6)
    ap.add_argument("--dtau", type=float, default=0.002, help="shift spacing: tau_k = dtau*(2k - nrhs + 1)")
    ap.add_argument("--maxiter", type=int, default=500)
    ap.add_argument("--restart", type=int, default=6)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-config4", action="store_true", help="skip the 32^4 8-shift mixed-precision leg")
    ap.add_argument("--quick", action="store_true", help="skip the extra FP64/BF16 solves")
    ap.add_argument("--tune-cache", type=str, default=None, help="autotuner JSON cache (default: fresh)")
    ap.add_argument("--graph", type=int, default=1, help="1: V-cycle replayed as a HIP graph (fixed coarse steps)")
    ap.add_argument("--coarse-iters", type=int, default=20, help="coarse GMRES steps in graph mode")
    ap.add_argument("--l3", type=str, default="4,8,2",
                    help="three-level leg: K-cycle steps k2, level-3 GMRES steps k3, level-2 smoothing steps s2 "
                         "('' to skip)")
    ap.add_argument("--variant", type=int, default=None, help="kernels mode: pin this stencil variant")
    ap.add_argument("--remap", type=int, default=1, help="kernels mode: XCD-aware work-group mapping (with --variant)")
    ap.add_argument("--mode", choices=["solve", "kernels", "mfma"], default="solve",
                    help="kernels: only a few launches of the hot kernels and a 1 GiB copy (for counter runs)")
    ap.add_argument("--eig-dims", type=str, default="32,32,32,32",
                    help="lattice of the GD-lambdaAMG eigensolver measurement ('' to skip)")
    ap.add_argument("--eig-nev", type=int, default=20, help="eigenpairs in the eigensolver measurement")
    ap.add_argument("--eig-block", type=int, default=1, help="targets per outer step of the eigensolver")
    ap.add_argument("--eig-both-signs", type=int, default=1, choices=[0, 1],
                    help="1: each outer step targets the smallest unlocked pair of each sign (finds both signs); "
                         "0: the single smallest |theta| target of the printed algorithm")
    ap.add_argument("--eig-levels", type=int, default=2, choices=[2, 3],
                    help="multigrid levels of the eigensolver's inner solves")
    ap.add_argument("--eig-prec", type=str, default="bf16", choices=["f64", "f32", "bf16"],
                    help="V-cycle precision of the eigensolver's inner solves (they stop at a 0.1 "
                         "reduction, so BF16 storage suffices; FP64 outer FGMRES either way)")
    ap.add_argument("--summarize-mfma", metavar="PMC_DIR", default=None,
                    help="write the MFMA utilisation summary from a --pmc MfmaUtil MfmaFlopsF32 MfmaFlopsF64 "
                         "run of --mode mfma")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="write the traffic summary from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of --mode kernels")
    args = ap.parse_args()
    if args.summarize_pmc:
        cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc %s --output-format csv -d "
               "$GRAFT_REPO_ROOT/gpurun_out/pk_%s -o k -- python -u $GRAFT_REPO_ROOT/bench.py --mode kernels")
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], cmd)
        return
    if args.summarize_mfma:
        cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc MfmaUtil MfmaFlopsF32 MfmaFlopsF64 "
               "--output-format csv -d $GRAFT_REPO_ROOT/gpurun_out/pm_mfma -o m -- python -u "
               "$GRAFT_REPO_ROOT/bench.py --mode mfma")
        summarize_mfma(args.summarize_mfma, cmd)
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_08146_amd import qmg
    from synth import device_gaussian_spinors, random_links, random_spinors, seed_for, unit_links

    dims = tuple(int(v) for v in args.dims.split(","))
    if args.m0 is None:
        with open(os.path.join(ROOT, "tests", "golden", "m0_critical.json")) as fh:
            args.m0 = float(json.load(fh)["m0"])
    if args.mode == "kernels":
        return kernels_mode(args, dims, torch, qmg, unit_links)
    if args.mode == "mfma":
        return mfma_mode(args, dims, torch, qmg, device_gaussian_spinors, random_links, seed_for)
    V = int(np.prod(dims))
    nrhs = args.nrhs
    csw, m0 = 1.0, args.m0
    taus = [args.dtau * (2 * k - (nrhs - 1)) for k in range(nrhs)]
    timer = EventTimer(torch)

    t0 = time.time()
    U = random_links(dims, 0.5, seed_for(5, "U"))
    b = random_spinors(dims, nrhs, seed_for(5, "b"))
    print("[bench] inputs generated in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(U).cuda(), m0, csw)
    bg = lat.pack(torch.from_numpy(b).cuda())
    ntv = 24
    W0 = lat.pack(device_gaussian_spinors(dims, ntv, seed_for(5, "W")))
    torch.cuda.synchronize()
    t0 = time.time()
    lat.setup_mg(W0, ntv, setup_iters=args.setup_iters, smooth=4, n_mr=3, coarse_maxiter=20, coarse_tol=0.5)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    # starting level-2 vectors of the three-level leg: P^H w_j of the level-1 test vectors
    W2 = lat.level2_vectors_from(W0, ntv) if args.l3 and not args.quick else None
    del W0
    print("[bench] setup %.2f s" % setup_s, file=sys.stderr, flush=True)
    tune_path = args.tune_cache or os.path.join("/tmp", "qmg_tune_%d.json" % os.getpid())
    t0 = time.time()
    lat.autotune(tune_path)
    tuning = json.load(open(tune_path))
    print("[bench] autotune %.1f s: %s" % (time.time() - t0, json.dumps(tuning)), file=sys.stderr, flush=True)

    def solve(prec, graph=args.graph):
        x = lat.field(nrhs)
        prm = qmg.default_params(mg_prec=prec, restart=args.restart, maxiter=args.maxiter, use_graph=graph,
                                 coarse_maxiter=args.coarse_iters if graph else 50)
        st, stats = lat.solve_shifted(x, bg, taus, nrhs, prm)
        return st, stats

    for _ in range(args.warmup):
        st, stats = solve("f32")
        print("[bench] warmup solve status %d iters %s" % (st, [s["iters"] for s in stats]),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for i in range(args.steps):
        st, stats = solve("f32")
        all_stats.append((st, stats))
        print("[bench] step %d done: status %d" % (i, st), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1000.0 * dt / args.steps
    ok = all(s == 0 for s, _ in all_stats)
    relres = max(s["true_relres"] for _, ss in all_stats for s in ss)
    iters = [s["iters"] for s in all_stats[-1][1]]
    print("[bench] timed %d steps: %.1f ms/step, converged=%s, max relres %.2e" % (args.steps, ms_step, ok, relres),
          file=sys.stderr, flush=True)

    extra = {}
    if not args.quick:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, stats = solve("f32", graph=1 - args.graph)
        torch.cuda.synchronize()
        extra["f32_graph%d" % (1 - args.graph)] = {
            "ms": 1000.0 * (time.perf_counter() - t1), "status": st,
            "max_true_relres": max(s["true_relres"] for s in stats), "iters": [s["iters"] for s in stats]}
        for prec in ("f64", "bf16"):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, stats = solve(prec)
            torch.cuda.synchronize()
            extra[prec] = {"ms": 1000.0 * (time.perf_counter() - t1), "status": st,
                           "max_true_relres": max(s["true_relres"] for s in stats),
                           "iters": [s["iters"] for s in stats]}
            print("[bench] %s solve %.1f ms" % (prec, extra[prec]["ms"]), file=sys.stderr, flush=True)

    if W2 is not None:
        # third level: aggregates of 2^4 blocks, 24 level-2 test vectors improved by two rounds of
        # inverse iteration; the coarse correction is a K-cycle on level 2
        k2, k3, s2 = (int(v) for v in args.l3.split(","))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat.setup_level3(W2, ntv, (2, 2, 2, 2), setup_iters=3, smooth=s2, l3_iters=20)
        torch.cuda.synchronize()
        l3_setup = time.perf_counter() - t1
        del W2
        prm3 = qmg.default_params(mg_prec="f32", restart=args.restart, maxiter=args.maxiter, use_graph=1,
                                  levels=3, coarse_maxiter=k2, l3_iters=k3, l2_smooth=s2)
        x3 = lat.field(nrhs)
        lat.solve_shifted(x3, bg, taus, nrhs, prm3)  # records the three-level V-cycle graph
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, stats = lat.solve_shifted(x3, bg, taus, nrhs, prm3)
        torch.cuda.synchronize()
        extra["f32_three_level"] = {"ms": 1000.0 * (time.perf_counter() - t1), "status": st,
                                    "max_true_relres": max(s["true_relres"] for s in stats),
                                    "iters": [s["iters"] for s in stats], "level3_setup_s": l3_setup,
                                    "k2": k2, "k3": k3, "s2": s2, "ntv2": ntv, "block2": [2, 2, 2, 2]}
        del x3
        print("[bench] three-level solve %.1f ms" % extra["f32_three_level"]["ms"], file=sys.stderr, flush=True)

    # Q-apply throughput (the stencil), timed with events on torch's stream
    qapply = {}
    for prec, n in (("f64", 1), ("f32", nrhs)):
        a = lat.field(n, prec)
        o = lat.field(n, prec)
        ms = timer(lambda: lat.apply_Q_shifted(o, a, taus[:n], n, prec), 20)
        byts = apply_bytes_per_site(prec, n, True) * V
        qapply["%s_%drhs" % (prec, n)] = {"ms": ms, "gflops": FLOP_SITE * V * n / ms / 1e6,
                                          "gbps": byts / ms / 1e6, "hbm_frac": byts / ms / 1e6 / HBM_PEAK_GBS}
    # SAP sweep (FP32, all rhs): the smoother inside every V-cycle and the
    # dominant kernel of the solve; one sweep = two launches (one per colour)
    xs = lat.field(nrhs, "f32")
    fs = lat.field(nrhs, "f32")
    sap_ms = timer(lambda: lat.sap_smooth(xs, fs, taus, nrhs, 1, 3, "f32"), 10)
    sap_bytes = sap_bytes_per_site("f32", nrhs, True) * V
    del xs, fs
    launch_ms = sap_ms / 2
    # the dominant kernel of the solve (about 40% of its kernel time): one colour's SAP half-sweep
    roofline = roofline_entry("k_sap44<float, clover, 2 rhs slots>: one colour's SAP half-sweep, 16 rhs",
                              sap_flops_per_site(3) * (V // 2) * nrhs, sap_bytes / 2, launch_ms,
                              FP32_VECTOR_PEAK_TFLOPS, traffic_for("sap_f32"))
    roofline["flop_per_site_rhs"] = sap_flops_per_site(3)
    st = qapply["f32_%drhs" % nrhs]
    roofline_stencil = roofline_entry("stencil (Q - tau), FP32, 16 rhs",
                                      (FLOP_SITE + 552 + 48) * V * nrhs, apply_bytes_per_site("f32", nrhs, True) * V,
                                      st["ms"], FP32_VECTOR_PEAK_TFLOPS, traffic_for("stencil_f32"))
    # measured streaming-copy bandwidth: the practical ceiling of any HBM-bound kernel here
    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    copy_ms = timer(lambda: qmg.stream_copy(dst, src), 10)
    stream_copy = {"bytes_moved": 2 * (1 << 30), "ms": copy_ms, "gbps": 2 * (1 << 30) / copy_ms / 1e6,
                   "frac_of_8TBs": 2 * (1 << 30) / copy_ms / 1e6 / HBM_PEAK_GBS,
                   "kernel": "qmg_stream_copy (1 GiB read + 1 GiB written, 16 B per lane)"}
    del src, dst
    for r in (roofline, roofline_stencil):
        r["frac_of_measured_copy"] = r["hbm_gbps"] / stream_copy["gbps"]

    # coarse apply on MFMA (FP32, 16 rhs): algorithmic MFMA rate against the FP32 MFMA peak,
    # with the matrix units' busy fraction from the committed rocprof summary
    ycs = lat.coarse(nrhs, "f32")
    ocs = lat.coarse(nrhs, "f32")
    cms = timer(lambda: lat.apply_coarse(ocs, ycs, taus, nrhs, "f32"), 10)
    del ycs, ocs
    cfl = 8.0 * 9 * (2 * ntv) ** 2 * nrhs * (V // 256)
    roofline_coarse = {"bound": "mfma", "kernel": "coarse apply (D_c - tau Gamma5^c), FP32 MFMA, 16 rhs",
                       "achieved": cfl / cms / 1e9, "peak": MFMA_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                       "frac": cfl / cms / 1e9 / MFMA_PEAK_TFLOPS["f32"], "launch_ms": cms,
                       "mfma_flop_per_launch": cfl,
                       "mfma_util_pct": mfma_util_for("k_coarse_mfma<float, float, 3>")}

    del lat
    torch.cuda.empty_cache()
    c4 = None
    if not args.no_config4:
        c4 = config4_run(args, torch, qmg, random_links, random_spinors, seed_for, device_gaussian_spinors, m0)
        torch.cuda.empty_cache()
    eig = None
    if args.eig_dims:
        eig = eigensolver_run(args, torch, qmg, random_links, seed_for, device_gaussian_spinors, -0.8)

    # fine-operator applications per rhs: FGMRES apply + nu * (1 residual + n_MR block applies)
    applies = float(np.mean([s["iters"] * (1 + 3 * 4) + s["restarts"] + 1 for s in all_stats[-1][1]]))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(U, b[:8], m0, csw, taus[0], applies)

    line = {
        "metric": "Q-apply GFLOP/s & HBM GB/s; shifted-solve time mixed vs FP64 at 1e-10 rel. residual",
        "value": nrhs / (ms_step / 1000.0),
        "unit": "rhs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer / f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": "64x32^3 clover shifted solve, 16 rhs, two-level MG, FGMRES to 1e-10",
                   "dims": list(dims), "csw": csw, "m0": m0, "nrhs": nrhs, "taus": [taus[0], taus[-1]],
                   "dtau": args.dtau,
                   "block": [4, 4, 4, 4], "ntv": ntv, "restart": args.restart, "setup_iters": args.setup_iters},
        "converged": ok, "max_true_relres": relres, "fgmres_iters": iters, "setup_s": setup_s,
        "solve_ms": {"mixed_f32": ms_step, **{"%s_precond" % k: v["ms"] for k, v in extra.items()}},
        "graph": args.graph, "coarse_iters_graph": args.coarse_iters,
        "solve_detail": extra,
        "q_apply": qapply,
        "sap_sweep_f32": {"ms": sap_ms, "gbps": sap_bytes / sap_ms / 1e6, "hbm_frac": sap_bytes / sap_ms / 1e6 / HBM_PEAK_GBS},
        "roofline": roofline,
        "roofline_stencil": roofline_stencil,
        "roofline_coarse": roofline_coarse,
        "stream_copy": stream_copy,
        "config4_32x32x32x32_8shifts": c4,
        "eigensolver": eig,
        "autotune": tuning,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
