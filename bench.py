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
# HBM bytes per launch from rocprofv3 counter passes: reads from the L2's read
# requests by size (TCC_EA0_RDREQ_128B x 128 + TCC_EA0_RDREQ_64B x 64; the
# derived FETCH_SIZE counts every request as 64 B on this chip, half of what a
# plain copy of known size reads), writes from WRITE_SIZE (equal to the copy's
# written bytes), by kernel class and workload, with the SHA-256 of the kernel's
# source at the time; reported only while the source is unchanged
TRAFFIC = {
    # profiles/hbm_traffic_16x4.md: k_sap_colour<float, false>, one colour, 16 right-hand sides
    ("sap", "medium"): {"bytes_per_launch": 537.80e6,
                        "source_sha256": "ca9ccebdcf4b8bc964eeae88d8748d398ba0fe6dedc88b95f79ad98973007c2d"},
    # k_coarse_apply_mfma (the tuned kernel), 16 right-hand sides, 256 coarse sites of 40 unknowns
    ("coarse", "medium"): {"bytes_per_launch": 30.07e6,
                           "source_sha256": "2f797ceab98415869eb162ea6a2980e5d59e3dd56b6cc8ee92480f287417b69a"},
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
# FP32 vector issue rate the build can use: 256 CUs x 4 SIMDs x 16 lanes x 2 flop
# (FMA) x 2.4 GHz; the published 157.3 TFLOP/s needs packed FP32, which the
# build turns off
VALU_FP32_PEAK_TFLOPS = 78.6
# FP32 VALU work of one SAP colour pass per (site, field) with 4 MR steps on 4^4
# blocks: the residual (8 hops of 180 flop with the boundary sign, the site
# term 120, gamma5 r - D z 24), then per MR step the in-block hops (6 on
# average, 168 flop each), the site term 120, the three block sums 144 and the
# two updates 192, and z += e 24
SAP_FLOP_PER_SITE_FIELD = 8 * 180 + 120 + 24 + 4 * (6 * 168 + 120 + 144 + 192) + 24

# Workloads: lattice, field, aggregation, Nv, N_eig, tolerance.  Masses come
# from tests/golden/m0.json (written by tests/golden/make_m0.py).
WORKLOADS = {
    # guard bands reach past the near-degenerate momentum shell that the
    # n_eig-th mode lies in (16^4: 12 + 96 modes; 32^3x64: 12 + 24 + 96)
    "large": dict(golden="large", agg=(4, 4, 4, 4), nv=32, n_eig=100, tol=1e-10, guard=32,
                  params=dict(rqi_block=8, fgmres_m=8, n_setup=4, coarse_m=40, coarse_restarts=1,
                              coarse_tol=0.15, rqi_start_passes=6, rqi_solve_restarts=0)),
    # medium: FGMRES(7) and 8 start passes measured fastest in a sweep of the solver parameters
    "medium": dict(golden="medium", agg=(4, 4, 4, 4), nv=20, n_eig=50, tol=1e-10, guard=70,
                   params=dict(rqi_block=16, fgmres_m=7, n_setup=4, coarse_m=40, coarse_restarts=1,
                               coarse_tol=0.3, rqi_start_passes=8, rqi_solve_restarts=0)),
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


def host_cpu_info():
    """(logical CPUs, CPU model) of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


_ORACLE = {}


def _oracle_init(dims, t_bc, eps, seed, m0, agg, sweeps, n_mr, barrier):
    """Worker set-up: the oracle's operator on the benchmark field (generated
    again from its seed) and four seeded vectors."""
    import lqsynth
    from oracle import mg as M
    from oracle.dirac import Lattice, WilsonOp
    lat = Lattice(dims, t_bc)
    op = WilsonOp(lqsynth.gauge_field(dims, eps, seed), m0, lat)
    _ORACLE.update(op=op, ag=M.Aggregation(lat, agg), x=lqsynth.gaussian_spinors(4, dims, 11), sweeps=sweeps,
                   n_mr=n_mr, barrier=barrier)


def _oracle_iteration(k):
    """One worker's share of the sample: the fine-level work of one outer
    FGMRES iteration of the oracle's solver on its own right-hand side (the
    FP64 Q apply and the smoother's sweeps), timed in the worker."""
    from oracle import mg as M
    o = _ORACLE
    x = o["x"][k % len(o["x"])]
    o["barrier"].wait(timeout=900)        # every worker starts at once: all cores busy
    t0 = time.perf_counter()
    o["op"].Q(x)
    M.sap(o["op"], o["ag"], 0.01 * k, x, o["sweeps"], o["n_mr"])
    return time.perf_counter() - t0


def cpu_baseline(dims, t_bc, eps, seed, m0, agg, nv, prm, n_outer, n_rebuild, cores):
    """The oracle (numpy, FP64) timed on this host on a bounded sample of the
    benchmark step, scaled by the step's own counts:
      * `cores` worker processes run at once, each the fine-level work of one
        outer FGMRES iteration (a Q apply and the smoother's SAP sweeps) on its
        own vector: the wall time over `cores` is the cost per iteration with
        every core busy (the iterations of a block of shifted solves are
        independent);
      * the coarse operator of a 2-column interpolation (a tenth of one
        rebuild's columns at Nv = 20) times Nv, per rebuild.
    The coarse solves, the Gram-Schmidt and Rayleigh-Ritz products are not
    counted, so the figure is a lower bound of the oracle's time."""
    import multiprocessing as mp

    import lqsynth
    from oracle import mg as M
    from oracle.dirac import Lattice, WilsonOp
    # fresh interpreters (no state of this process, which holds the GPU)
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    with ctx.Pool(cores, initializer=_oracle_init,
                  initargs=(dims, t_bc, eps, seed, m0, agg, prm["post"], prm["sap_mr"], barrier)) as pool:
        # one task per worker: each waits at the barrier until all have started
        per_worker = pool.map(_oracle_iteration, range(cores), chunksize=1)
    wall = max(per_worker)
    t_iter = wall / cores
    lat = Lattice(dims, t_bc)
    op = WilsonOp(lqsynth.gauge_field(dims, eps, seed), m0, lat)
    ag = M.Aggregation(lat, agg)
    t0 = time.perf_counter()
    M.coarse_operator(op, ag, M.build_P(lqsynth.gaussian_spinors(1, dims, 12), ag))
    t_cols = time.perf_counter() - t0           # 2 of the 2 Nv columns
    t_rebuild = t_cols * nv
    value = n_outer * t_iter + n_rebuild * t_rebuild
    return {"value": round(value, 1), "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"oracle on this host ({host_cpu_info()[1]}, {host_cpu_info()[0]} logical CPUs): "
                      f"{cores} processes at once, each one outer FGMRES iteration's fine-level work (FP64 Q apply + "
                      f"{prm['post']} SAP sweeps of {prm['sap_mr']} MR steps on {agg} blocks) on the {dims} lattice: "
                      f"{min(per_worker):.1f}-{wall:.1f} s per process, {wall:.1f} s for all = "
                      f"{t_iter:.3f} s per iteration x {n_outer} outer iterations of the GPU step; plus the coarse "
                      f"operator of 2 interpolation columns ({t_cols:.1f} s, one core) x Nv = {nv} per rebuild x "
                      f"{n_rebuild} rebuilds.  Coarse solves, Gram-Schmidt and Rayleigh-Ritz are not counted: a lower "
                      f"bound",
            "per_iteration_s": round(t_iter, 4), "rebuild_s": round(t_rebuild, 1)}


def _tiny_oracle_solve(q):
    """The oracle's complete eigensolve on the tiny periodic lattice (4^4):
    adaptive setup and Alg. 1 with a Rayleigh-Ritz step per pass, the 8
    lowest pairs at 1e-10, one core.  Runs in a child process."""
    try:
        import lqsynth
        from oracle import mg as M
        from oracle import rqi as R
        from oracle.dirac import Lattice, WilsonOp
        g = load_golden("tiny_periodic")
        dims = tuple(g["dims"])
        U = lqsynth.gauge_field(dims, g["eps"], g["field_seed"])
        op = WilsonOp(U, g["m0"], Lattice(dims, g["t_bc"]))
        t0 = time.perf_counter()
        mg, W = M.setup(op, (2, 2, 2, 2), lqsynth.gaussian_spinors(8, dims, 102),
                        M.MGParams(coarse_m=128, coarse_tol=1e-8, coarse_restarts=2, n_setup=4))
        V0 = np.concatenate([W, lqsynth.gaussian_spinors(2, dims, 103)])
        lam, v, eps, info = R.rqi(mg, V0, 1e-10, W_pad=W, solve_tol=1e-6, max_sweeps=10, rayleigh_ritz=True,
                                  n_want=8)
        q.put({"s": round(time.perf_counter() - t0, 2), "converged": info["converged"], "sweeps": info["sweeps"],
               "lambda": [float(x) for x in lam[:8]]})
    except Exception as e:                      # reported, never fatal to the benchmark
        q.put({"error": repr(e)})


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
    fields); 6: matrix cores in FP32; 7: matrix cores on bfloat16 operands, bfloat16
    storage only) with the FP32 coarse operator and with its bfloat16 copy, on the
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
        for v in range(8 if bf16 else 7):
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


def learned_setup(args):
    """Train the learned setup's network on generated 16^4 fields (eps between
    0.2 and 0.4, bare mass m_c(eps) + 0.005 from tests/golden/mc_curve.json,
    the 24 lowest eigenvectors of each field as targets), then compare it with
    the plain adaptive setup on the 16^4 benchmark field (a field it was not
    trained on): setup time, eigensolver sweeps and time, final residuals and
    the projection loss of the test vectors each setup produces.  Prints one
    JSON line."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    from paper_1509_06865_amd import learned as L
    with open(os.path.join(ROOT, "tests", "golden", "mc_curve.json")) as f:
        mc = json.load(f)
    dims, agg, K = (16, 16, 16, 16), (4, 4, 4, 4), 24
    V = int(np.prod(dims))
    ctx = Context(dims, 1)
    net = L.init_network(seed=5000)
    phi_seed = 6000
    losses, t_targets, t_train = [], 0.0, 0.0
    n_fields = args.train_fields
    for j in range(n_fields):
        eps = 0.2 + 0.2 * j / max(n_fields - 1, 1)
        m0 = float(np.interp(eps, mc["eps"], mc["m_c"])) + mc["target"]
        U = torch.from_numpy(lqsynth.gauge_field(dims, eps, 1000 + j)).cuda()
        phi0 = L.gaussian_fields(K, V, phi_seed + j)
        a = time.time()
        tgt, info = L.eigen_targets(ctx, U, m0, agg, phi0[:20].contiguous(), K, 1e-6)
        torch.cuda.synchronize()
        t_targets += time.time() - a
        a = time.time()
        for _ in range(args.train_steps):
            losses.append(L.train_step(ctx, U, net, phi0, tgt, agg, args.train_lr, bf16=args.train_bf16))
        torch.cuda.synchronize()
        t_train += time.time() - a
        log(f"field {j + 1}/{n_fields}: eps {eps:.3f} m0 {m0:.4f} targets converged {info['converged']} "
            f"({info['sweeps']} sweeps), loss {losses[-args.train_steps]:.4f} -> {losses[-1]:.4f}")
        del U, phi0, tgt
    if args.learned_eval == "large":
        ctx.close()                                 # the 16^4 context's buffers go back first
        del ctx
        learned_eval_large(args, net, L, losses, t_targets, t_train, n_fields)
        return
    # evaluation on the benchmark field
    gold = load_golden("medium")
    m0 = gold["m0"]
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    phi0 = L.gaussian_fields(K, V, gold["field_seed"] + 1)
    ref_V, _ = L.eigen_targets(ctx, U, m0, agg, phi0[:20].contiguous(), K, 1e-6)
    wl = WORKLOADS["medium"]
    n_eig, guard, nv = wl["n_eig"], wl["guard"], 24
    base = dict(wl["params"], precision=1, rqi_guard=guard, rayleigh_ritz=1, rqi_max_sweeps=args.max_sweeps)
    plain = MGParams(**base)
    learned = MGParams(**dict(base, n_setup=args.learned_n_setup, n_init=0))
    V0 = device_gaussian(n_eig + guard - nv, dims, gold["field_seed"] + 2, torch)
    out = {"train": {"fields": n_fields, "steps_per_field": args.train_steps, "lr": args.train_lr,
                     "layers": "bf16_mfma" if args.train_bf16 else "fp64_direct",
                     "first_loss": losses[0], "last_loss": losses[-1],
                     "mean_loss_first_10": float(np.mean(losses[:10])), "mean_loss_last_10": float(np.mean(losses[-10:])),
                     "targets_s": round(t_targets, 1), "train_s": round(t_train, 1)}}
    # the test vectors' projection loss against the 24 lowest modes
    ctx.mg_setup(U, m0, agg, phi0[:nv].contiguous(), plain)
    P_plain = ctx.get_interp()
    X = L.propose(ctx, U, net, phi0)
    torch.cuda.synchronize()
    a = time.time()
    Xb = L.propose(ctx, U, net, phi0, bf16=True)        # the layers on the bfloat16 matrix cores
    torch.cuda.synchronize()
    t_bf16 = time.time() - a
    a = time.time()
    X = L.propose(ctx, U, net, phi0)
    torch.cuda.synchronize()
    t_fp64 = time.time() - a
    out["loss_vs_lowest24"] = {"network_outputs": L.loss_of(ctx, X, ref_V, agg),
                               "network_outputs_bf16_layers": L.loss_of(ctx, Xb, ref_V, agg),
                               "plain_setup_P": L.loss_of(ctx, P_plain, ref_V, agg),
                               "random_start_vectors": L.loss_of(ctx, phi0, ref_V, agg)}
    out["inference_s"] = {"fp64_direct": round(t_fp64, 3), "bf16_mfma": round(t_bf16, 3),
                          "rel_diff": float(torch.linalg.norm(Xb - X) / torch.linalg.norm(X))}
    del Xb
    del P_plain
    res = {}
    for name in ("plain", "learned"):
        if name == "plain":
            lam, Vv, r, info, ts, tr = L.setup_and_solve(ctx, U, m0, agg, phi0[:nv].contiguous(), plain, n_eig,
                                                         wl["tol"], V0)
            info = dict(info, setup_s=ts, rqi_s=tr)
        else:
            lam, Vv, r, info = L.learned_solve(ctx, U, m0, agg, net, phi0, learned, plain, n_eig, wl["tol"], V0, nv,
                                               bf16=args.train_bf16)
        res[name] = {"converged": info["converged"], "sweeps": info["sweeps"], "solves": info["solves"],
                     "fgmres_iters": info["fgmres_iters"], "setup_s": round(info["setup_s"], 3),
                     "rqi_s": round(info["rqi_s"], 3), "max_residual": float(max(r)),
                     "learned_hierarchy_used": info.get("learned", False),
                     "network_s": round(info.get("network_s", 0.0), 3)}
        log(f"{name}: {res[name]}")
        del Vv
    out["solve"] = res
    out["workload"] = f"16^4 eps={gold['eps']} m0={m0}, Nv={nv}, lowest {n_eig} at {wl['tol']}"
    print(json.dumps(out), flush=True)


def learned_eval_large(args, net, L, losses, t_targets, t_train, n_fields):
    """The network trained on 16^4 fields applied to the 32^3 x 64 field: its
    24 outputs against 24 random vectors as the test vectors of the large
    workload's setup (the learned one with --learned-n-setup passes and no
    initial ones), then the same capped number of eigensolver sweeps from the
    same start vectors; pairs converged, residuals, times.  Prints one JSON line."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    torch.cuda.empty_cache()
    gold = load_golden("large")
    wl = WORKLOADS["large"]
    dims, m0, agg = tuple(gold["dims"]), gold["m0"], wl["agg"]
    nv, n_eig, guard = 24, wl["n_eig"], wl["guard"]
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    ctx = Context(dims, gold["t_bc"])
    phi0 = device_gaussian(nv, dims, gold["field_seed"] + 1, torch)
    V0 = device_gaussian(n_eig + guard - nv, dims, gold["field_seed"] + 2, torch)
    base = dict(wl["params"], precision=1, rqi_guard=guard, rayleigh_ritz=1, rqi_max_sweeps=args.max_sweeps)
    plain = MGParams(**base)
    learned = MGParams(**dict(base, n_setup=args.learned_n_setup, n_init=0))
    torch.cuda.synchronize()
    a = time.time()
    X = L.propose(ctx, U, net, phi0, bf16=args.train_bf16)
    torch.cuda.synchronize()
    t_net = time.time() - a
    torch.cuda.empty_cache()                        # the layers' activations: back to the device for the solver
    log(f"network on 32^3x64: {t_net:.2f} s")
    out = {"train": {"fields": n_fields, "steps_per_field": args.train_steps, "lr": args.train_lr,
                     "layers": "bf16_mfma" if args.train_bf16 else "fp64_direct",
                     "first_loss": losses[0], "last_loss": losses[-1],
                     "targets_s": round(t_targets, 1), "train_s": round(t_train, 1)},
           "network_s": round(t_net, 3)}
    res = {}
    for name, tv, prm in (("plain", phi0, plain), ("learned", X, learned)):
        lam, Vv, r, info, ts, tr = L.setup_and_solve(ctx, U, m0, agg, tv[:nv].contiguous(), prm, n_eig, wl["tol"],
                                                     V0)
        r = np.asarray(r, dtype=float)
        res[name] = {"converged_pairs": int((r <= wl["tol"]).sum()), "sweeps": info["sweeps"],
                     "solves": info["solves"], "fgmres_iters": info["fgmres_iters"], "setup_s": round(ts, 2),
                     "rqi_s": round(tr, 2), "max_residual": float(r.max()), "median_residual": float(np.median(r))}
        log(f"{name}: {res[name]}")
        del Vv
    out["solve"] = res
    out["workload"] = (f"32^3x64 eps={gold['eps']} m0={m0}, Nv={nv}, lowest {n_eig} at {wl['tol']}, "
                       f"at most {args.max_sweeps} sweeps")
    print(json.dumps(out), flush=True)


def lma_mode(args):
    """Approximate low-mode averaging (sec. 3.2-3.3) on the 16^4 benchmark
    field: the loop L(t) = sum_x tr Q^-1_xx per timeslice estimated with Z2 +
    i Z2 noise (a) without low modes, (b) with exact low modes (residual
    1e-10), (c) with loose ones (1e-3), (d) with the setup's vectors after one
    more multigrid pass (sec. 3.3), each with the cutoff eps/|lambda| <= 0.75
    and the oblique projector; times of the eigenpairs and of the deflated
    solves, the low-mode connected correlator, and the spread of the estimates.
    Prints one JSON line."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    gold = load_golden("medium")
    dims, m0 = tuple(gold["dims"]), gold["m0"]
    T = dims[3]
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    ctx = Context(dims, gold["t_bc"])
    wl = WORKLOADS["medium"]
    nv, n_eig, cutoff = 20, args.lma_modes, 0.75
    tv0 = device_gaussian(nv, dims, gold["field_seed"] + 1, torch)
    eta = torch.from_numpy(lqsynth.z2_spinors(args.lma_noise, dims, 403)).cuda()
    out = {"workload": f"16^4 eps={gold['eps']} m0={m0}, {n_eig} modes, {args.lma_noise} Z2 noise vectors, "
                       f"cutoff {cutoff}", "cutoff": cutoff}
    variants = {"exact": dict(tol=1e-10, sweeps=40, passes=6), "loose": dict(tol=1e-3, sweeps=40, passes=6),
                "setup": dict(tol=1e-10, sweeps=0, passes=1)}
    for name, v in [("none", None)] + list(variants.items()):
        rec = {}
        if v is None:
            Vd, lam, eps = None, None, None
            ctx.mg_setup(U, m0, wl["agg"], tv0, MGParams(precision=1, **wl["params"]))
        else:
            prm = dict(wl["params"], rqi_start_passes=v["passes"], rqi_max_sweeps=v["sweeps"])
            guard = 30
            p = MGParams(precision=1, rqi_guard=guard, rayleigh_ritz=1, **prm)
            torch.cuda.synchronize()
            a = time.time()
            ctx.mg_setup(U, m0, wl["agg"], tv0, p)
            V0 = device_gaussian(n_eig + guard - nv, dims, gold["field_seed"] + 2, torch)
            lam, Vd, eps, info = ctx.rqi_lowmodes(n_eig, v["tol"], V0=V0)
            torch.cuda.synchronize()
            rec["eigen_s"] = round(time.time() - a, 3)
            rec["max_eps"] = float(max(eps))
            del V0
            low, conn, kept = ctx.lma_low(U, m0, Vd, lam, eps, cutoff)
            rec["kept"] = kept
            rec["loop_low_t0"] = [float(low[0].real), float(low[0].imag)]
            rec["conn_low"] = [float(x.real) for x in conn[: T // 2 + 1]]
        torch.cuda.synchronize()
        a = time.time()
        high = ctx.lma_high(U, m0, Vd, lam, eps, cutoff, eta, 1e-8)
        torch.cuda.synchronize()
        rec["high_s"] = round(time.time() - a, 3)
        base = 0 if v is None else low
        est = base + high.mean(axis=0)
        sem = high.std(axis=0) / np.sqrt(high.shape[0])
        rec["loop_t0"] = [float(est[0].real), float(est[0].imag)]
        rec["stderr_mean_over_t"] = float(np.mean(sem))
        out[name] = rec
        log(f"lma {name}: {rec}")
        del Vd
    print(json.dumps(out), flush=True)


def lanczos_mode(args):
    """The Krylov comparison of sec. 2.2 on the 16^4 benchmark field: the
    n_eig lowest eigenpairs of Q at 1e-10 by restarted Lanczos on Q^2 (no
    multigrid; a basis of n_kv vectors restarted from the lowest Ritz vectors)
    and by RQI with the multigrid (the benchmark's parameters), for each n_eig
    of --lanczos-neig, on the same GPU.  The eigenvalues of the two must agree.
    Prints one JSON line."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    gold = load_golden("medium")
    dims, m0 = tuple(gold["dims"]), gold["m0"]
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    ctx = Context(dims, gold["t_bc"])
    wl = WORKLOADS["medium"]
    out = {"workload": f"16^4 eps={gold['eps']} m0={m0}, tol 1e-10", "runs": []}
    for n_eig in [int(x) for x in args.lanczos_neig.split(",")]:
        n_kv = min(191, max(100, 2 * n_eig + 40))
        v0 = device_gaussian(1, dims, gold["field_seed"] + 7, torch)[0]
        torch.cuda.synchronize()
        a = time.time()
        lam_l, V_l, res_l, info_l = ctx.lanczos_lowmodes(U, m0, n_eig, v0, tol=1e-10, n_kv=n_kv, n_guard=4,
                                                         max_restarts=args.lanczos_max_restarts)
        torch.cuda.synchronize()
        t_l = time.time() - a
        del V_l
        log(f"lanczos n_eig {n_eig} n_kv {n_kv}: {t_l:.2f} s, {info_l}")
        # the guard band reaches past the momentum shell the n_eig-th mode lies in
        # (16^4: 12 + 96 modes), as for the benchmark's 50 pairs
        guard = max(wl["guard"], 120 - n_eig)
        p = MGParams(precision=1, rqi_guard=guard, rayleigh_ritz=1, **wl["params"])
        tv0 = device_gaussian(wl["nv"], dims, gold["field_seed"] + 1, torch)
        torch.cuda.synchronize()
        a = time.time()
        ctx.mg_setup(U, m0, wl["agg"], tv0, p)
        V0 = device_gaussian(n_eig + guard - wl["nv"], dims, gold["field_seed"] + 2, torch) \
            if n_eig + guard > wl["nv"] else None
        lam_r, V_r, res_r, info_r = ctx.rqi_lowmodes(n_eig, 1e-10, V0=V0)
        torch.cuda.synchronize()
        t_r = time.time() - a
        del V_r, V0, tv0
        log(f"rqi n_eig {n_eig}: {t_r:.2f} s, sweeps {info_r['sweeps']}")
        lr = np.sort(np.asarray(lam_r))
        ll = np.sort(np.asarray(lam_l))
        out["runs"].append({"n_eig": n_eig, "n_kv": n_kv,
                            "lanczos": {"s": round(t_l, 3), "q2_products": info_l["q2_products"],
                                        "restarts": info_l["restarts"], "converged": info_l["converged"],
                                        "max_residual": float(np.max(res_l))},
                            "rqi_mg": {"s": round(t_r, 3), "sweeps": info_r["sweeps"], "solves": info_r["solves"],
                                       "converged": info_r["converged"], "max_residual": float(np.max(res_r))},
                            "speedup": round(t_l / t_r, 2),
                            "max_rel_eigenvalue_diff": float(np.max(np.abs(lr - ll) / np.abs(lr)))})
    print(json.dumps(out), flush=True)


def ptc_layer_mode(args):
    """One 16 -> 16 parallel-transport layer of the learned setup on the 16^4
    field: the direct FP64 kernel against the bfloat16 matrix-core form, mean
    time of a few launches (HIP events through torch on the context's stream),
    the work as a complex product (8 flop per complex multiply-add:
    81 x (4 c_in) x (4 c_out) x 3 V) and the agreement of the two outputs.
    Prints one JSON line."""
    import torch
    import lqsynth
    from paper_1509_06865_amd import Context
    gold = load_golden("medium")
    dims = tuple(gold["dims"])
    V = int(np.prod(dims))
    cin = cout = 16
    U = torch.from_numpy(lqsynth.gauge_field(dims, gold["eps"], gold["field_seed"])).cuda()
    phi = device_gaussian(cin, dims, 501, torch)
    rng = np.random.default_rng(502)
    W = torch.from_numpy((rng.standard_normal((cout, cin, 81, 4, 4)) +
                          1j * rng.standard_normal((cout, cin, 81, 4, 4))) / 60).cuda()
    ctx = Context(dims, gold["t_bc"])
    flop = 8.0 * 81 * (4 * cin) * (4 * cout) * 3 * V
    out = {"workload": f"16^4, {cin} -> {cout} channels, 81 offsets", "flop_per_layer": flop}
    res = {}
    for name, fn, reps in (("fp64_direct", ctx.ptc_forward, 2), ("bf16_mfma", ctx.ptc_forward_bf16, 10)):
        y = fn(U, phi, W)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            y = fn(U, phi, W)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = y
        out[name] = {"ms": round(ms, 3), "TFLOPs": round(flop / (ms * 1e-3) / 1e12, 2)}
        log(f"ptc layer {name}: {ms:.3f} ms")
    a, b = res["bf16_mfma"].cpu().numpy(), res["fp64_direct"].cpu().numpy()
    out["rel_diff"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out["bf16_frac_of_2500_TFLOPs"] = round(out["bf16_mfma"]["TFLOPs"] / 2500.0, 4)
    # the backward: input and weight gradients, twice the forward's products
    G = device_gaussian(cout, dims, 503, torch)
    bwd = {}
    for name, fn, reps in (("fp64_direct", ctx.ptc_backward, 1), ("bf16_mfma", ctx.ptc_backward_bf16, 5)):
        g = fn(U, phi, W, G)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g = fn(U, phi, W, G)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        bwd[name] = g
        out["backward_" + name] = {"ms": round(ms, 3), "TFLOPs": round(2 * flop / (ms * 1e-3) / 1e12, 2)}
        log(f"ptc layer backward {name}: {ms:.3f} ms")
    for k, part in enumerate(("g_in", "g_W")):
        a, b = bwd["bf16_mfma"][k].cpu().numpy(), bwd["fp64_direct"][k].cpu().numpy()
        out[f"backward_rel_diff_{part}"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(json.dumps(out), flush=True)


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
    ap.add_argument("--no-large-solve", action="store_true",
                    help="skip the 20-pair solve on the 32^3 x 64 lattice after the timed step")
    ap.add_argument("--n-eig", type=int, default=None, help="override the workload's eigenpair count")
    ap.add_argument("--guard", type=int, default=None)
    ap.add_argument("--nv", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None, choices=(2, 3),
                    help="2 = drop the workload's third level; 3 = add one (aggregates 2^4 of the coarse lattice)")
    ap.add_argument("--nv2", type=int, default=None)
    ap.add_argument("--max-sweeps", type=int, default=40)
    ap.add_argument("--param", action="append", default=[], help="MGParams override name=value")
    ap.add_argument("--learned", action="store_true",
                    help="train the learned setup's network on generated 16^4 fields and compare it with the plain "
                         "setup on the benchmark field")
    ap.add_argument("--train-fields", type=int, default=200)
    ap.add_argument("--train-steps", type=int, default=1)
    ap.add_argument("--train-lr", type=float, default=1e-3)
    ap.add_argument("--learned-n-setup", type=int, default=1)
    ap.add_argument("--learned-eval", default="medium", choices=["medium", "large"],
                    help="field the trained network is evaluated on: the 16^4 benchmark field, or 32^3 x 64 with "
                         "--max-sweeps sweeps for both setups")
    ap.add_argument("--train-bf16", action="store_true",
                    help="train (and propose the learned setup's vectors) with the layers on the bfloat16 matrix cores")
    ap.add_argument("--lma", action="store_true", help="approximate low-mode averaging on the 16^4 field")
    ap.add_argument("--lma-modes", type=int, default=20)
    ap.add_argument("--lma-noise", type=int, default=32)
    ap.add_argument("--ptc-layer", action="store_true",
                    help="time one 16 -> 16 layer of the learned setup: direct FP64 against bfloat16 matrix cores")
    ap.add_argument("--lanczos", action="store_true",
                    help="restarted Lanczos on Q^2 against RQI with the multigrid on the 16^4 field (sec. 2.2)")
    ap.add_argument("--lanczos-neig", default="20,50")
    ap.add_argument("--lanczos-max-restarts", type=int, default=2000)
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the roofline kernel class and a reference copy (for counter passes)")
    ap.add_argument("--coarse-variants", action="store_true",
                    help="time the coarse-apply kernels with FP32 and bfloat16 storage (8192 coarse sites)")
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
    if args.learned:
        learned_setup(args)
        return
    if args.lma:
        lma_mode(args)
        return
    if args.lanczos:
        lanczos_mode(args)
        return
    if args.ptc_layer:
        ptc_layer_mode(args)
        return
    if args.kernel_only:
        kernel_only(args)
        return
    if args.roofline_class == "all":
        ap.error("--roofline-class all is for --kernel-only runs")

    # the oracle's complete tiny solve runs on one host core beside the GPU work
    tiny_proc = tiny_q = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        sctx = mp.get_context("spawn")
        tiny_q = sctx.Queue()
        tiny_proc = sctx.Process(target=_tiny_oracle_solve, args=(tiny_q,), daemon=True)
        tiny_proc.start()

    import torch
    import lqsynth
    from paper_1509_06865_amd import Context, MGParams
    from paper_1509_06865_amd import load as load_lib

    wl = dict(WORKLOADS[args.workload])
    wl["params"] = dict(wl["params"])
    for key in ("n_eig", "guard", "nv", "nv2"):
        if getattr(args, key) is not None:
            wl[key] = getattr(args, key)
    if args.levels == 2:
        wl.pop("agg2", None)
        wl.pop("nv2", None)
    elif args.levels == 3 and not wl.get("agg2"):
        wl["agg2"] = (2, 2, 2, 2)
        wl.setdefault("nv2", min(24, wl["nv"]))
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
        ctx.mg_setup(U, m0, wl["agg"], tv0, prm, agg2=wl.get("agg2"), nv2=wl.get("nv2"))
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
                               f"m0={m0}, " + (f"3-level MG {wl['agg']} / {wl['agg2']} aggregates "
                                               f"Nv={wl['nv']}/{wl['nv2']}" if wl.get("agg2") else
                                               f"2-level MG {wl['agg']} aggregates Nv={wl['nv']}") +
                               f", lowest {wl['n_eig']} eigenpairs at residual {wl['tol']}",
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
    if args.roofline_class == "sap" and k_ms > 0 and wl["params"].get("sap_mr", 4) == 4:
        # the pass's arithmetic intensity (about 19 flop per algorithmic byte) is
        # above the FP32 VALU ridge (9.8): report the ALU fraction beside the HBM one.
        # Site-field pairs from the bytes: (36 + 48 nf) complex FP32 per site of the colour
        site_fields = (k_bytes / 8.0 - 36.0 * (V / 2) * k_launches) / 48.0
        flops = SAP_FLOP_PER_SITE_FIELD * site_fields
        tf = flops / (k_ms * 1e-3) / 1e12
        out["roofline"]["alu"] = {"achieved": round(tf, 2), "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": round(tf / VALU_FP32_PEAK_TFLOPS, 4),
                                  "flop_per_launch": round(flops / max(k_launches, 1))}
    # the same solve on the all-FP64 GPU path (smoother and coarse solves in FP64
    # too), after the timed steps: time and agreement of the eigenvalues
    if not args.no_fp64_compare and args.workload != "large":
        prm64 = MGParams(precision=0, rqi_guard=wl["guard"], rayleigh_ritz=1, rqi_max_sweeps=args.max_sweeps,
                         **wl["params"])
        torch.cuda.synchronize()
        a = time.time()
        ctx.mg_setup(U, m0, wl["agg"], tv0, prm64, agg2=wl.get("agg2"), nv2=wl.get("nv2"))
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
        del bx
        if not args.no_large_solve:
            # time to solution on the same lattice for the 20 lowest pairs (the eigenpair count of
            # the paper's comparisons; guard 20 covers the momentum shell the 20th mode lies in),
            # the large workload's solver parameters
            lw = WORKLOADS["large"]
            ne, gd = 20, 20
            tv0_l = device_gaussian(lw["nv"], bdims, big["field_seed"] + 1, torch)
            V0_l = device_gaussian(ne + gd - lw["nv"], bdims, big["field_seed"] + 2, torch)
            prm_l = MGParams(precision=1, rqi_guard=gd, rayleigh_ritz=1, rqi_max_sweeps=30, **lw["params"])
            torch.cuda.empty_cache()
            torch.cuda.synchronize()
            a = time.time()
            bctx.mg_setup(bU, big["m0"], lw["agg"], tv0_l, prm_l)
            torch.cuda.synchronize()
            t_set = time.time() - a
            lam_l, V_l, res_l, info_l = bctx.rqi_lowmodes(ne, lw["tol"], V0=V0_l)
            torch.cuda.synchronize()
            t_l = time.time() - a
            out["config"]["lowest20_32x32x32x64"] = {
                "s": round(t_l, 3), "setup_s": round(t_set, 3), "converged": bool(info_l["converged"]),
                "sweeps": info_l["sweeps"], "solves": info_l["solves"], "fgmres_iters": info_l["fgmres_iters"],
                "max_residual": float(max(res_l)), "smallest_abs_lambda": float(min(abs(v) for v in lam_l)),
                "largest_abs_lambda": float(max(abs(v) for v in lam_l)), "nv": lw["nv"], "guard": gd}
            log(f"32^3x64, 20 lowest at {lw['tol']}: {t_l:.2f} s (setup {t_set:.2f} s), converged "
                f"{info_l['converged']}, sweeps {info_l['sweeps']}")
            del tv0_l, V0_l, V_l
        del bU, bctx
    else:
        out["config"]["dirac_apply_gbs_32x32x32x64"] = out["config"]["dirac_apply_gbs"]
    gpu_tiny = None
    if not args.no_cpu_baseline:
        # the GPU's time for the oracle's tiny solve (same lattice, field, start vectors, 8 lowest pairs)
        tw = WORKLOADS["small"]
        tg = load_golden(tw["golden"])
        tdims = tuple(tg["dims"])
        tU = torch.from_numpy(lqsynth.gauge_field(tdims, tg["eps"], tg["field_seed"])).cuda()
        ttv = torch.from_numpy(lqsynth.gaussian_spinors(tw["nv"], tdims, 102)).cuda()
        tV0 = torch.from_numpy(lqsynth.gaussian_spinors(tw["guard"], tdims, 103)).cuda()
        tctx = Context(tdims, tg["t_bc"])
        tprm = MGParams(precision=1, rqi_guard=tw["guard"], rayleigh_ritz=1, **tw["params"])
        torch.cuda.synchronize()
        a = time.time()
        tctx.mg_setup(tU, tg["m0"], tw["agg"], ttv, tprm)
        _, _, _, tinfo = tctx.rqi_lowmodes(tw["n_eig"], tw["tol"], V0=tV0)
        torch.cuda.synchronize()
        gpu_tiny = round(time.time() - a, 3)
        log(f"tiny workload on the GPU: {gpu_tiny} s, converged {tinfo['converged']}")
        del tctx
    if not args.no_cpu_baseline:
        cores = min(16, host_cpu_info()[0])
        log(f"cpu baseline: the oracle on {cores} host processes")
        eff = prm.to_c(load_lib())
        out["cpu_baseline"] = cpu_baseline(dims, t_bc, eps, seed, m0, wl["agg"], wl["nv"],
                                           {"post": eff.post, "sap_mr": eff.sap_mr}, info["fgmres_iters"],
                                           info["p_rebuilds"], cores)
        if tiny_proc is not None:
            import queue
            try:
                tiny = tiny_q.get(timeout=600)
            except queue.Empty:
                tiny = {"error": "no result within 600 s"}
            tiny_proc.join(timeout=30)
            out["cpu_baseline"]["tiny_full_solve"] = dict(
                tiny, what="the oracle's complete setup + Alg. 1 (Rayleigh-Ritz per pass, 8 lowest pairs at 1e-10, "
                           "4^4 periodic) on one core, run beside the GPU steps")
            if gpu_tiny is not None:
                out["cpu_baseline"]["tiny_full_solve"]["gpu_s"] = gpu_tiny
        log(f"cpu baseline: {out['cpu_baseline']['value']} s (lower bound for the step)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
