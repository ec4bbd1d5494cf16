"""Benchmark of the shifted-solve hot path on one MI355X.

Workload (config 5): 64x32^3 lattice, clover c_sw = 1.0, synthetic links
exp(i*0.5*H), near-critical bare mass (m0 = -0.95 from tests/golden/
m0_critical.json), 16 right-hand sides with shifts tau_k = 0.001*(2k - 15),
two-level multigrid (4^4 aggregates, 24 test vectors, 6 setup iterations),
FP64 FGMRES(8) to a 1e-10 true relative residual.

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


def cpu_baseline(U, b0, m0, csw, tau, applies_per_rhs):
    """The oracle (NumPy FP64) timed on one Q apply of one right-hand side on a
    1/16 sub-volume of the workload's gauge field (32x16^3, same link
    distribution), scaled to the full volume (the oracle's cost is linear in
    the volume) and to right-hand sides per second with the number of
    fine-operator applications the GPU solve needed per right-hand side."""
    from oracle import clover, dirac
    sub = (slice(0, U.shape[0] // 2),) + (slice(0, U.shape[1] // 2),) * 3
    Us = np.ascontiguousarray(U[sub])
    bs = np.ascontiguousarray(b0[sub])
    scale = U[..., 0, 0, 0].size / Us[..., 0, 0, 0].size
    t0 = time.perf_counter()
    C = clover.clover_term(Us, csw)
    t1 = time.perf_counter()
    dirac.apply_Q_shifted(Us, bs, m0, tau, C)
    t2 = time.perf_counter()
    t_apply = (t2 - t1) * scale
    V = int(np.prod(U.shape[:4]))
    return {
        "value": 1.0 / (t_apply * applies_per_rhs),
        "unit": "rhs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": ("one FP64 (Q - tau) apply of 1 rhs on a 1/16 sub-volume (32x16^3) of the clover workload, "
                   "%.2f s scaled x%d to %.1f s per full apply (clover build not counted), times %.0f "
                   "fine-operator applications per rhs of the GPU solve" % (t2 - t1, scale, t_apply,
                                                                          applies_per_rhs)),
        "apply_gflops": FLOP_SITE * V / t_apply / 1e9,
    }


def kernels_mode(args, dims, torch, qmg, unit_links):
    """A few launches of each hot kernel (memory traffic does not depend on the
    field values, so unit links are used) plus a plain 1 GiB device copy whose
    known size calibrates the HBM byte counters."""
    V = int(np.prod(dims))
    nrhs = args.nrhs
    lat = qmg.Lattice(dims, (4, 4, 4, 4))
    lat.set_gauge(torch.from_numpy(unit_links(dims)).cuda(), args.m0, 1.0)
    if args.tune_cache:
        lat.autotune(args.tune_cache)
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
    ap.add_argument("--dtau", type=float, default=0.001, help="shift spacing: tau_k = dtau*(2k - nrhs + 1)")
    ap.add_argument("--maxiter", type=int, default=500)
    ap.add_argument("--restart", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the extra FP64/BF16 solves")
    ap.add_argument("--tune-cache", type=str, default=None, help="autotuner JSON cache (default: fresh)")
    ap.add_argument("--graph", type=int, default=1, help="1: V-cycle replayed as a HIP graph (fixed coarse steps)")
    ap.add_argument("--coarse-iters", type=int, default=16, help="coarse GMRES steps in graph mode")
    ap.add_argument("--variant", type=int, default=None, help="kernels mode: pin this stencil variant")
    ap.add_argument("--remap", type=int, default=1, help="kernels mode: XCD-aware work-group mapping (with --variant)")
    ap.add_argument("--mode", choices=["solve", "kernels"], default="solve",
                    help="kernels: only a few launches of the hot kernels and a 1 GiB copy (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
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

    # Q-apply throughput (the stencil), timed with events on torch's stream
    qapply = {}
    for prec, n in (("f64", 1), ("f32", nrhs)):
        a = lat.field(n, prec)
        o = lat.field(n, prec)
        ms = timer(lambda: lat.apply_Q_shifted(o, a, taus[:n], n, prec), 20)
        byts = apply_bytes_per_site(prec, n, True) * V
        qapply["%s_%drhs" % (prec, n)] = {"ms": ms, "gflops": FLOP_SITE * V * n / ms / 1e6,
                                          "gbps": byts / ms / 1e6, "hbm_frac": byts / ms / 1e6 / HBM_PEAK_GBS}
    # SAP sweep (FP32, all rhs): the smoother inside every V-cycle
    xs = lat.field(nrhs, "f32")
    fs = lat.field(nrhs, "f32")
    sap_ms = timer(lambda: lat.sap_smooth(xs, fs, taus, nrhs, 1, 3, "f32"), 5)
    sap_bytes = sap_bytes_per_site("f32", nrhs, True) * V
    del xs, fs

    dom = qapply["f32_%drhs" % nrhs]
    roofline = {"bound": "hbm", "kernel": "k_dslash<float, clover, Q-tau> (16 rhs)",
                "achieved": dom["gbps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["gbps"] / HBM_PEAK_GBS, "traffic": None}

    # fine-operator applications per rhs: FGMRES apply + nu * (1 residual + n_MR block applies)
    applies = float(np.mean([s["iters"] * (1 + 3 * 4) + s["restarts"] + 1 for s in all_stats[-1][1]]))
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(U, b[0], m0, csw, taus[0], applies)

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
        "autotune": tuning,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
