#!/usr/bin/env python3
"""Benchmark: lowest-|lambda| eigenpairs of the Hermitian Wilson-Dirac operator
on one MI355X (RQI + gamma5-aggregation multigrid), plus the Dirac-apply
bandwidth.

One step = mg_setup (adaptive setup from random test vectors) + rqi_lowmodes
(Alg. 1 to the target residual) on a synthetic SU(3) field of the workload's
shape, inputs already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 1] [--warmup 0] [--workload large|medium|small]
"""
import os

os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import argparse  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time for lowest-100 eigenpairs of Q at 32^3x64, tol 1e-10; Dirac-apply HBM GB/s"
DEFAULT_CLASS = "sap"          # the kernel class with the largest share of the step's device time
# HBM bytes per launch from rocprofv3 FETCH_SIZE + WRITE_SIZE passes (scaled by a
# plain copy of known size), by kernel class and workload, with the SHA-256 of
# the kernel's source at the time; reported only while the source is unchanged
TRAFFIC = {
    # profiles/hbm_traffic_16x4.md: k_sap_colour<float>, one colour, 16 right-hand sides
    ("sap", "medium"): {"bytes_per_launch": 278.68e6,
                        "source_sha256": "f0bb59517c4b540d91b95fafaa30216e14ebc7f4a23629f88098bc6a7de29de0"},
    # k_coarse_apply<float>, 16 right-hand sides, 256 coarse sites of 40 unknowns
    ("coarse", "medium"): {"bytes_per_launch": 16.17e6,
                           "source_sha256": "99ecebd727a242a9cdc02b7d7d6ee5ef944c55ba736c123e8d41bd057266d979"},
}
KSOURCES = {"wilson": ["wilson.hip", "lq_dslash.h"], "sap": ["sap.hip", "lq_dslash.h"],
            "restrict": ["transfer.hip"], "prolong": ["transfer.hip"], "coarse": ["coarse.hip"],
            "gram": ["gram.hip"], "combine": ["gram.hip"]}


def kernel_source_sha(cls):
    import hashlib
    h = hashlib.sha256()
    for f in KSOURCES[cls]:
        with open(os.path.join(ROOT, "paper_1509_06865_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(cls, workload):
    t = TRAFFIC.get((cls, workload))
    if t is None or t["source_sha256"] != kernel_source_sha(cls):
        return None
    return t["bytes_per_launch"]
HBM_PEAK_GBS = 8000.0

# Workloads: lattice, field, aggregation, Nv, N_eig, tolerance.  Masses come
# from tests/golden/m0.json (written by tests/golden/make_m0.py).
WORKLOADS = {
    # guard bands reach past the near-degenerate momentum shell that the
    # n_eig-th mode lies in (16^4: 12 + 96 modes; 32^3x64: 12 + 24 + 96)
    "large": dict(golden="large", agg=(4, 4, 4, 4), nv=32, n_eig=100, tol=1e-10, guard=32,
                  params=dict(rqi_block=8, fgmres_m=8, n_setup=4, coarse_m=40, coarse_restarts=1,
                              coarse_tol=0.15, rqi_start_passes=6, rqi_solve_restarts=0)),
    "medium": dict(golden="medium", agg=(4, 4, 4, 4), nv=20, n_eig=50, tol=1e-10, guard=70,
                   params=dict(rqi_block=16, fgmres_m=8, n_setup=4, coarse_m=40, coarse_restarts=1,
                               coarse_tol=0.3, rqi_start_passes=6, rqi_solve_restarts=0)),
    "small": dict(golden="tiny_periodic", agg=(2, 2, 2, 2), nv=8, n_eig=8, tol=1e-10, guard=4,
                  params=dict(rqi_block=4, fgmres_m=10, n_setup=4, coarse_m=128, coarse_restarts=2,
                              coarse_tol=1e-8)),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_golden(name):
    with open(os.path.join(ROOT, "tests", "golden", "m0.json")) as f:
        return json.load(f)[name]


def device_gaussian(n, dims, seed, torch):
    """Seeded complex Gaussian start vectors drawn on the device (input
    generation only; the large lattices make host generation slow)."""
    V = int(np.prod(dims))
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = torch.empty((n, 12, V), dtype=torch.complex128, device="cuda")
    view = torch.view_as_real(out)                    # [n, 12, V, 2] float64
    for k in range(n):                                # one field at a time: small temporaries
        view[k].normal_(generator=g)
    out /= np.sqrt(2.0)
    return out


def time_q_apply(ctx, U, m0, x, reps, torch):
    """Average device time of one q_apply launch (HIP events on the context's stream)."""
    st = ctx.stream
    for _ in range(3):
        ctx.q_apply(U, m0, x)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(st)
    for _ in range(reps):
        ctx.q_apply(U, m0, x)
    stop.record(st)
    stop.synchronize()
    return start.elapsed_time(stop) / reps / 1e3


def cpu_baseline(U_host, m0, dims, t_bc, x_host, n_outer):
    """The oracle's FP64 Q apply (definition route) timed on the host on the
    full lattice, scaled by the step's outer FGMRES iterations (each applies Q
    once): a lower bound on the oracle's time for the same eigensolve, which
    also needs the smoother, the coarse solves and the orthogonalisation."""
    from oracle.dirac import Lattice, apply_Q
    lat = Lattice(dims, t_bc)
    lat.tables()                                   # neighbour tables built outside the timing
    reps, t0 = 0, time.perf_counter()
    while True:
        apply_Q(U_host, m0, x_host, lat)
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps >= 3:
            break
    t = (time.perf_counter() - t0) / reps
    return {"value": round(t * n_outer, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} FP64 Q applies of the oracle's numpy definition on the full {dims} lattice, "
                      f"{t:.2f} s each, times the {n_outer} outer FGMRES iterations of the GPU step (one Q "
                      f"apply each): a lower bound for the oracle's eigensolve, whose smoother, coarse solves "
                      f"and orthogonalisation are not counted"}


# kernel classes of the library's timer (paper_1509_06865_amd.KT_*) and how
# their algorithmic bytes are counted
KCLASS = {"wilson": (0, "Wilson stencil k_wilson (links once + fields in/out)"),
          "sap": (1, "SAP colour pass k_sap_colour (the colour's links once + per field r, z on all sites "
                     "(own and halo), z out)"),
          "restrict": (2, "restriction k_restrict (P once + fields + coarse out)"),
          "prolong": (3, "prolongation k_prolong"),
          "coarse": (4, "coarse operator apply k_coarse_apply (< 1024 coarse sites) / k_coarse_apply_multi "
                        "(5 stored blocks per coarse site once + x in, y out per field)"),
          "gram": (5, "Gram products k_gram (E and W once)"),
          "combine": (6, "basis combination k_combine")}


def coarse_variants(args):
    """Time each coarse-apply kernel (0: one wave per (site, field); 1-3: LDS-staged
    blocks for 4, 8, 16 fields per pass; 4, 5: as 1, 2 per (site, chunk of
    fields)) with the FP32 coarse operator and with its bfloat16 copy, on the
    coarse grid of a 16^3 x 32 lattice with 2^4 aggregates and Nv = 24 (8192
    coarse sites, 48 x 48 blocks), 16 fields, through the library's kernel timer.
    Prints one JSON line per (storage, kernel)."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import (KT_COARSE, Context, MGParams, coarse_variant, kernel_timer_read,
                                      kernel_timer_start)
    dims, agg, nv, nf = (16, 16, 16, 32), (2, 2, 2, 2), 24, 16
    n_sites = int(np.prod([d // a for d, a in zip(dims, agg)]))
    U = torch.from_numpy(lqsynth.gauge_field(dims, 0.25, 31)).cuda()
    tv0 = device_gaussian(nv, dims, 32, torch)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    shape = (nf, n_sites, 2 * nv)
    x = torch.complex(torch.randn(shape, generator=g, device="cuda", dtype=torch.float64),
                      torch.randn(shape, generator=g, device="cuda", dtype=torch.float64))
    sig = [0.01 * k for k in range(nf)]
    for bf16 in (0, 1):
        ctx = Context(dims, 1)
        ctx.mg_setup(U, -0.15, agg, tv0, MGParams(precision=1, n_setup=0, n_init=1, coarse_bf16=bf16))
        for v in range(6):
            coarse_variant(v)
            ctx.coarse_apply(sig, x)
            torch.cuda.synchronize()
            kernel_timer_start(KT_COARSE)
            for _ in range(10):
                ctx.coarse_apply(sig, x)
            torch.cuda.synchronize()
            n, ms, by = kernel_timer_read()
            print(json.dumps({"coarse_storage": "bf16" if bf16 else "fp32", "kernel": v, "coarse_sites": n_sites,
                              "block": 2 * nv, "fields": nf, "avg_launch_ms": round(ms / n, 4),
                              "bytes_per_launch": by / n, "algorithmic_GBs": round(by / (ms * 1e-3) / 1e9, 1)}),
                  flush=True)
        coarse_variant(-1)
        del ctx


def kernel_only(args):
    """Launch only the kernels of one class on the workload's lattice, plus a
    plain device copy of known size (12 V complex128 read and written), for
    hardware-counter passes."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    wl = WORKLOADS[args.workload]
    gold = load_golden(wl["golden"])
    dims, t_bc, m0 = tuple(gold["dims"]), gold["t_bc"], gold["m0"]
    V = int(np.prod(dims))
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    ctx = Context(dims, t_bc)
    cls = args.roofline_class
    if cls == "all":
        x = device_gaussian(1, dims, gold["field_seed"] + 3, torch)
        t = time_q_apply(ctx, U, m0, x, 10, torch)
        log(f"kernel-only: q_apply FP64 {t * 1e3:.3f} ms")
    if cls == "wilson":
        x = device_gaussian(1, dims, gold["field_seed"] + 3, torch)
        t = time_q_apply(ctx, U, m0, x, 10, torch)
        log(f"kernel-only: q_apply FP64 {t * 1e3:.3f} ms ({960.0 * V / t / 1e9:.0f} GB/s algorithmic)")
    else:
        tv0 = device_gaussian(wl["nv"], dims, gold["field_seed"] + 1, torch)
        ctx.mg_setup(U, m0, wl["agg"], tv0, MGParams(precision=1, n_setup=0, n_init=1))
        del tv0
        nr = wl["params"]["rqi_block"]            # the solves' batch width
        r = device_gaussian(nr, dims, gold["field_seed"] + 4, torch)
        sig = [0.01 * k for k in range(nr)]
        for _ in range(3):
            if cls == "all":
                c = ctx.restrict(r)
                ctx.coarse_apply(sig, c)
                ctx.prolong(c)
                ctx.smooth(sig, r, 1)
                ctx.cycle(sig, r)
            elif cls == "sap":
                ctx.smooth(sig, r, 1)
            elif cls in ("restrict", "prolong", "coarse"):
                c = ctx.restrict(r)
                if cls == "coarse":
                    ctx.coarse_apply(sig, c)
                if cls == "prolong":
                    ctx.prolong(c)
            else:
                ctx.cycle(sig, r)
        torch.cuda.synchronize()
        log(f"kernel-only: class {cls}, 3 passes over {nr} fields")
    a = torch.empty(12 * V * 2, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"kernel-only: copy of {a.numel() * 8} bytes x10")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    # 16^4 / 50 pairs by default: the 32^3 x 64 / 100-pair case runs (--workload large) but does not
    # converge within one run's time budget yet (its interior shifts defeat the two-level solver)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true", help="skip the all-FP64 comparison solve")
    ap.add_argument("--n-eig", type=int, default=None, help="override the workload's eigenpair count")
    ap.add_argument("--guard", type=int, default=None)
    ap.add_argument("--nv", type=int, default=None)
    ap.add_argument("--max-sweeps", type=int, default=40)
    ap.add_argument("--param", action="append", default=[], help="MGParams override name=value")
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the roofline kernel class and a reference copy (for counter passes)")
    ap.add_argument("--coarse-variants", action="store_true",
                    help="time the six coarse-apply kernels with FP32 and bfloat16 storage (8192 coarse sites)")
    ap.add_argument("--roofline-class", default=DEFAULT_CLASS, choices=sorted(KCLASS) + ["all"],
                    help="kernel class timed live for the roofline object (default: the step's dominant one)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the solver over "
              f"several GPUs (by shift or by lattice) is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.coarse_variants:
        coarse_variants(args)
        return
    if args.kernel_only:
        kernel_only(args)
        return
    if args.roofline_class == "all":
        ap.error("--roofline-class all is for --kernel-only runs")

    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams

    wl = dict(WORKLOADS[args.workload])
    wl["params"] = dict(wl["params"])
    for key in ("n_eig", "guard", "nv"):
        if getattr(args, key) is not None:
            wl[key] = getattr(args, key)
    for kv in args.param:
        k, v = kv.split("=")
        wl["params"][k] = float(v) if ("." in v or "e" in v) else int(v)
    gold = load_golden(wl["golden"])
    dims, t_bc, eps, seed, m0 = tuple(gold["dims"]), gold["t_bc"], gold["eps"], gold["field_seed"], gold["m0"]
    V = int(np.prod(dims))
    log(f"workload {args.workload}: dims {dims} t_bc {t_bc} eps {eps} m0 {m0} Nv {wl['nv']} n_eig {wl['n_eig']}")
    t0 = time.time()
    U_host = lqsynth.gauge_field(dims, eps, seed)
    U = torch.from_numpy(U_host).cuda()
    log(f"gauge field ready ({time.time() - t0:.1f} s)")
    tv0 = device_gaussian(wl["nv"], dims, seed + 1, torch)
    n_work = wl["n_eig"] + wl["guard"]
    n_v0 = n_work - min(wl["nv"], n_work)
    V0 = device_gaussian(n_v0, dims, seed + 2, torch) if n_v0 > 0 else None
    prm = MGParams(precision=1, rqi_guard=wl["guard"], rayleigh_ritz=1, rqi_max_sweeps=args.max_sweeps,
                   **wl["params"])
    torch.cuda.empty_cache()          # hand torch's cached temporaries back before the library allocates
    ctx = Context(dims, t_bc)

    # Dirac apply bandwidth (FP64 and FP32), device time per launch
    x = device_gaussian(1, dims, seed + 3, torch)
    t64 = time_q_apply(ctx, U, m0, x, 20, torch)
    t32 = time_q_apply(ctx, U.to(torch.complex64), m0, x.to(torch.complex64), 20, torch)
    gbs64, gbs32 = 960.0 * V / t64 / 1e9, 480.0 * V / t32 / 1e9
    log(f"q_apply FP64 {t64 * 1e3:.3f} ms = {gbs64:.0f} GB/s ; FP32 {t32 * 1e3:.3f} ms = {gbs32:.0f} GB/s")

    def step():
        ctx.mg_setup(U, m0, wl["agg"], tv0, prm)
        t_setup = time.time()
        free, total = torch.cuda.mem_get_info()
        log(f"after setup: device free {free / 2**30:.1f} GiB, torch reserved "
            f"{torch.cuda.memory_reserved() / 2**30:.1f} GiB")
        lam, Vv, res, info = ctx.rqi_lowmodes(wl["n_eig"], wl["tol"], V0=V0)
        return lam, res, info, t_setup

    os.environ["LQMG_VERBOSE"] = "1"
    for w in range(args.warmup):
        step()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    from paper_1509_06865_amd import kernel_timer_read, kernel_timer_start
    kernel_timer_start(KCLASS[args.roofline_class][0])
    times, setups = [], []
    for s in range(args.steps):
        torch.cuda.synchronize()
        a = time.time()
        lam, res, info, t_setup = step()
        torch.cuda.synchronize()
        b = time.time()
        times.append(b - a)
        setups.append(t_setup - a)
        log(f"step {s + 1}/{args.steps}: {b - a:.2f} s (setup {t_setup - a:.2f} s), converged {info['converged']}, "
            f"sweeps {info['sweeps']}, solves {info['solves']}, fgmres its {info['fgmres_iters']}")
    T = max(times)
    k_launches, k_ms, k_bytes = kernel_timer_read()
    kernel_timer_start(-1)
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    log(f"roofline class {args.roofline_class}: {k_launches} launches, {k_ms / max(k_launches, 1):.4f} ms avg, "
        f"{k_gbs:.0f} GB/s algorithmic")
    out = {
        "metric": METRIC, "value": round(T, 3), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * T, 1), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 (RQI, FGMRES) + f32 (multigrid)", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} t_bc={t_bc} eps={eps} "
                               f"m0={m0}, 2-level MG {wl['agg']} aggregates Nv={wl['nv']}, lowest {wl['n_eig']} "
                               f"eigenpairs at residual {wl['tol']}",
                   "n_eig": wl["n_eig"], "tol": wl["tol"], "converged": info["converged"],
                   "smallest_abs_lambda": float(abs(lam[0])), "largest_abs_lambda": float(abs(lam[-1])),
                   "max_residual": float(max(res)), "setup_s": round(max(setups), 3),
                   "rqi_s": round(T - max(setups), 3), "sweeps": info["sweeps"], "solves": info["solves"],
                   "fgmres_iters": info["fgmres_iters"],
                   "phase_s": {k: round(info[k], 3) for k in ("t_solve", "t_ortho", "t_rebuild", "t_rq")},
                   "dirac_apply_gbs": {"fp64": round(gbs64, 1), "fp32": round(gbs32, 1)}},
        "roofline": {"bound": "hbm", "achieved": round(k_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(k_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.roofline_class, args.workload),
                     "kernel": KCLASS[args.roofline_class][1], "launches": k_launches,
                     "avg_launch_ms": round(k_ms / max(k_launches, 1), 4),
                     "bytes_per_launch": round(k_bytes / max(k_launches, 1))},
    }
    # the same solve on the all-FP64 GPU path (smoother and coarse solves in FP64
    # too), after the timed steps: time and agreement of the eigenvalues
    if not args.no_fp64_compare and args.workload != "large":
        prm64 = MGParams(precision=0, rqi_guard=wl["guard"], rayleigh_ritz=1, rqi_max_sweeps=args.max_sweeps,
                         **wl["params"])
        torch.cuda.synchronize()
        a = time.time()
        ctx.mg_setup(U, m0, wl["agg"], tv0, prm64)
        lam64, _, res64, info64 = ctx.rqi_lowmodes(wl["n_eig"], wl["tol"], V0=V0)
        torch.cuda.synchronize()
        t64p = time.time() - a
        lam_m, lam_d = np.array(lam), np.array(lam64)
        out["config"]["fp64_path"] = {"s": round(t64p, 3), "converged": info64["converged"],
                                      "sweeps": info64["sweeps"], "fgmres_iters": info64["fgmres_iters"],
                                      "max_residual": float(max(res64)),
                                      "max_rel_lambda_diff_vs_mixed": float(np.abs(lam_m - lam_d).max()
                                                                            / np.abs(lam_d).max())}
        log(f"all-FP64 path: {t64p:.2f} s, converged {info64['converged']}, sweeps {info64['sweeps']}, "
            f"max |dlambda|/|lambda| vs mixed {out['config']['fp64_path']['max_rel_lambda_diff_vs_mixed']:.2e}")
    # the metric's Dirac-apply bandwidth is quoted at 32^3 x 64: measure it there
    # (after the timed step) when the workload is another lattice
    if args.workload != "large":
        big = load_golden(WORKLOADS["large"]["golden"])
        bdims = tuple(big["dims"])
        bV = int(np.prod(bdims))
        bU = torch.from_numpy(lqsynth.gauge_field(bdims, big["eps"], big["field_seed"])).cuda()
        bctx = Context(bdims, big["t_bc"])
        bx = device_gaussian(1, bdims, big["field_seed"] + 3, torch)
        b64 = time_q_apply(bctx, bU, big["m0"], bx, 20, torch)
        b32 = time_q_apply(bctx, bU.to(torch.complex64), big["m0"], bx.to(torch.complex64), 20, torch)
        out["config"]["dirac_apply_gbs_32x32x32x64"] = {"fp64": round(960.0 * bV / b64 / 1e9, 1),
                                                         "fp32": round(480.0 * bV / b32 / 1e9, 1),
                                                         "fp64_ms": round(b64 * 1e3, 4), "fp32_ms": round(b32 * 1e3, 4)}
        log(f"q_apply at 32^3x64: FP64 {b64 * 1e3:.3f} ms, FP32 {b32 * 1e3:.3f} ms")
        del bU, bx, bctx
    else:
        out["config"]["dirac_apply_gbs_32x32x32x64"] = out["config"]["dirac_apply_gbs"]
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle Q apply on the host)")
        x_host = x[0].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(U_host, m0, dims, t_bc, x_host, info["fgmres_iters"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
