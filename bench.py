"""Benchmark of the lattice GaBP hot path on one MI355X.

One step = one check interval of the solver (`gabp_solve` with a 10-iteration
chunk): 10 flooding iterations (once the precision messages froze, five
two-iteration launches replayed from a recorded graph), then the FP64
posterior mean, the FP64 residual reduction and its read-back (the unit of
work the convergence driver repeats).  Default workload: the 8192 x 4096 global-scale lattice (periodic
in x, zero-flux in y, 13-point prior, kappa 0.02, 60 satellite-like tracks,
~5 % coverage, FP32 messages, FP64 residual).

Prints one JSON line with whole-job edge-message updates/s, the dominant
kernel's roofline figures and the oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge-message updates/s + HBM GB/s; time to 1e-6 rel. residual, warm vs cold"
ITERS_PER_STEP = 10
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_iter_global8192_traffic.md")
PHASE_KERNEL = {"full": "k_iter_direct", "theta": "k_iter_theta", "theta2": "k_iter_theta2",
                "theta2w": "k_iter_theta2w"}


def edge_count(nx, ny, alpha, bcx, bcy):
    """Directed edges of the lattice graph (pairs with Q_ij != 0)."""
    from paper_2404_12968_amd.inputs import BC_PERIODIC
    offs = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    if alpha == 2:
        offs += [(2, 0), (-2, 0), (0, 2), (0, -2), (1, 1), (-1, -1), (1, -1), (-1, 1)]
    total = 0
    for dx, dy in offs:
        cx = nx if bcx == BC_PERIODIC else max(0, nx - abs(dx))
        cy = ny if bcy == BC_PERIODIC else max(0, ny - abs(dy))
        total += cx * cy
    return total


ITER_SOURCES = ("iter.hip", "iter_node.h", "pair_tile.h", "walk_strip.h", "numerics.h", "lattice.h")
ST_SOURCES = ("st_iter.h", "numerics.h", "lattice.h")
ST_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "spacetime512x512x64_traffic.md")


def kernel_source_digest(files=ITER_SOURCES):
    """Digest of the iteration kernels' source with // comments, trailing
    blanks and empty lines removed (a comment edit leaves it unchanged; the
    files hold no block comments and no // inside literals)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2404_12968_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def _summary_value(path, digest, key):
    """A per-launch figure from a committed PMC summary, if that summary was
    taken on the current kernel source (its digest line matches)."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    t = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != digest:
        return None
    return float(t.group(1))


def measured_traffic(phase, rpt, workload="global8192"):
    """HBM bytes per launch of the timed kernel (its tile shape) from the
    committed PMC summary of the 8192 x 4096 workload, if that was taken on
    the current kernel source."""
    if workload != "global8192":
        return None
    shape = {"theta2": f"pair{rpt}", "theta2w": f"walk{-rpt}"}.get(phase, f"rpt{rpt}")
    key = f"{PHASE_KERNEL[phase]}_{shape}_traffic_bytes_per_launch"
    return _summary_value(TRAFFIC_SUMMARY, kernel_source_digest(), key)


def rel_err(a, b):
    """||a - b||_2 / ||b||_2 of two device FP64 arrays (a reported figure)."""
    import torch
    a = a.reshape(-1).to(torch.float64)
    b = b.reshape(-1).to(torch.float64)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def progress(msg):
    """One progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def fp64_reference(prob, tol=None):
    """The posterior mean an FP32 result is compared with: the same problem
    solved with FP64 messages (the path pinned to the oracle at 1e-12) by
    multigrid to the same stopping rule (the problem's relative residual, or
    tol).  Tighter FP64 references are out of reach on these workloads: the
    smoothest error modes of the 13-point prior decay so slowly that FP64
    iterations from a 1e-6 solution of the 8192 x 4096 lattice stay above 4e-8
    after 400 000 iterations.  Returns (mean on the device, description)."""
    import dataclasses

    from paper_2404_12968_amd import gabp as G
    from paper_2404_12968_amd import multigrid as MG
    tol = prob.rel_tol if tol is None else tol
    progress(f"FP64 reference of {prob.name} to {tol:g}")
    p64 = dataclasses.replace(prob, dtype="f64", rel_tol=tol)
    r = MG.multigrid_solve(p64, keep_context=True)
    mu = G.gabp_posterior(r["ctx"], want_var=False)[0]
    G.gabp_destroy(r["ctx"])
    progress(f"FP64 reference done in {r['seconds']:.1f} s")
    return mu, {"reference": "FP64 messages, multigrid to the residual below (the FP32 runs' "
                             "stopping rule)",
                "rel_residual": r["rel"], "status": G.gabp_status_string(r["status"]),
                "fine_iterations": r["iterations"], "seconds": r["seconds"]}


def _oracle_iter_seconds(O, graph_prob, eta, reps, threads=None):
    """Median wall time of one oracle iteration (after two warm-up
    iterations) and the directed edges of its graph."""
    if threads is not None:
        O.set_threads(threads)
    og = O.OracleGaBP.from_problem(graph_prob)
    og.iterate(2, eta)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        og.iterate(1, eta)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), og.g.nnz


def _crop(I, prob, w, h):
    """The centre w x h crop of a problem (same prior, coverage and noise;
    zero-flux edges), FP64."""
    w, h = min(w, prob.nx), min(h, prob.ny)
    x0, y0 = (prob.nx - w) // 2, (prob.ny - h) // 2
    cx, cy = prob.cells % prob.nx, prob.cells // prob.nx
    ins = (cx >= x0) & (cx < x0 + w) & (cy >= y0) & (cy < y0 + h)
    return I.Problem("crop", w, h, I.BC_NEUMANN, I.BC_NEUMANN, prob.alpha, prob.kappa, prob.tau,
                     prob.c, prob.sigma, (cy[ins] - y0) * w + (cx[ins] - x0), prob.y[ins],
                     dtype="f64")


def cpu_baseline(prob, seconds=10.0, gpu_iters=None):
    """The FP64 oracle, as it is, on the GPU machine's host cores (rank 0, one
    GPU).  Headline: per-iteration throughput on a 2048 x 2048 crop of the
    workload (same prior, coverage pattern and noise) with all host threads;
    beside it the same on one thread, the 64 x 64 parity workload solved to
    1e-10 (measured end to end), and per-iteration times of the 2048 x 2048
    track workload, the 1024 x 1024 warm-start workload and the crop, each
    multiplied by the iteration count its GPU run needed (labelled
    extrapolated: the full runs would take minutes to hours of host time)."""
    from oracle import oracle as O
    from paper_2404_12968_amd import inputs as I
    cores = O.max_threads()
    sub = _crop(I, prob, 2048, 2048)
    og = O.OracleGaBP.from_problem(sub)
    og.iterate(2, prob.damping)
    its = 0
    t0 = time.perf_counter()
    while True:
        og.iterate(2, prob.damping)
        its += 2
        el = time.perf_counter() - t0
        if el >= seconds and its >= 6:
            break
    value = og.g.nnz * its / el
    nnz = og.g.nnz
    del og
    one_s, _ = _oracle_iter_seconds(O, sub, prob.damping, 5, threads=1)
    O.set_threads(cores)
    out = {"value": value, "unit": "edge-message updates/s", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle, {sub.nx}x{sub.ny} crop of the workload ({nnz} directed "
                     f"edges), {its} iterations after 2 warm-up, {el:.1f} s, {cores} threads",
           "one_core": {"value": nnz / one_s, "unit": "edge-message updates/s",
                        "iteration_seconds": one_s,
                        "sample": "same crop, one thread, median of 5 iterations"}}
    # the 64 x 64 parity workload, to 1e-10, measured end to end
    p64 = I.parity64()
    t0 = time.perf_counter()
    og = O.OracleGaBP.from_problem(p64)
    st, rel = og.solve(200000, p64.damping, p64.rel_tol, p64.check_every)
    out["parity64_to_1e-10"] = {"seconds": time.perf_counter() - t0, "iterations": og.t,
                                "rel_residual": rel, "measured": True}
    ext = {}
    it_s, e = _oracle_iter_seconds(O, I.tracks2048(), 0.5, 5)
    ext["tracks2048_1000_iterations"] = {"iteration_seconds": it_s, "iterations": 1000,
                                         "seconds": 1000 * it_s, "directed_edges": e}
    w = I.warm1024(instance=300000)
    it_s, e = _oracle_iter_seconds(O, w, 0.5, 5)
    ext["warm1024_to_1e-6_cold"] = {"iteration_seconds": it_s, "directed_edges": e,
                                    "iterations": None, "seconds": None}
    if gpu_iters:
        for k, v in gpu_iters.items():
            if k in ext and v:
                ext[k]["iterations"] = int(v)
                ext[k]["seconds"] = int(v) * ext[k]["iteration_seconds"]
    # the workload itself: the crop's per-iteration time scaled by the edge
    # count, times the GPU cold solve's iterations
    E = edge_count(prob.nx, prob.ny, prob.alpha, prob.bc_x, prob.bc_y)
    it_full = nnz / value * E / nnz
    g_it = (gpu_iters or {}).get(prob.name)
    ext[f"{prob.name}_to_tol"] = {"iteration_seconds": it_full, "directed_edges": E,
                                  "iterations": g_it,
                                  "seconds": g_it * it_full if g_it else None,
                                  "scaled_from": f"{sub.nx}x{sub.ny} crop"}
    out["extrapolated"] = ext
    out["extrapolated_note"] = ("measured per-iteration time (median of 5 after 2 warm-up, all "
                                "threads) times the iteration count of the GPU run of the same "
                                "workload; not a measured time to tolerance")
    return out


def copy_ceiling_gbps(torch, dev, reps=10):
    """Device-to-device copy of 1 GiB timed with events: bytes read plus
    written per second (the HBM rate a plain stream reaches on this machine)."""
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def st_edge_count(prob):
    """Directed edges of the space-time graph (38 directions, include/gabp_st.h)."""
    from paper_2404_12968_amd.inputs import BC_PERIODIC
    lat = [(1, 0), (-1, 0), (0, 1), (0, -1), (2, 0), (-2, 0), (0, 2), (0, -2),
           (1, 1), (-1, -1), (1, -1), (-1, 1)]
    dirs = [(dx, dy, 0) for dx, dy in lat]
    for ox, oy in [(0, 0)] + lat:
        dirs += [(ox, oy, 1), (-ox, -oy, -1)]
    total = 0
    for dx, dy, dt in dirs:
        cx = prob.nx if prob.bc_x == BC_PERIODIC else max(0, prob.nx - abs(dx))
        cy = prob.ny if prob.bc_y == BC_PERIODIC else max(0, prob.ny - abs(dy))
        total += cx * cy * max(0, prob.nt - abs(dt))
    return total


def bench_spacetime(G, I, torch, args):
    """The space-time solver (heat-equation GMRF of the paper's
    spatio-temporal extension) on 64 slices of a 512 x 512 zero-flux grid,
    drifting satellite tracks (~2.3 % of the space-time cells), FP32
    messages.  The full iteration is timed first; the solver then runs with
    residual checks until the precision messages freeze (freeze tolerance
    --st-freeze-slots messages of at most 1e-6 relative change), and the
    timed steps are check intervals of the information-only iteration:
    ITERS_PER_STEP iterations (HIP events on the context's stream) plus the
    FP64 residual.  Algorithmic bytes per iteration: full kernel, both
    components of every directed message read and written once (16 B per
    edge) and the two node terms (8 B per node); information-only kernel,
    the information message read and written and the gain read (12 B per
    edge) and b (4 B per node).  CPU baseline: the FP64 oracle iterating on a
    128 x 128 x 16 problem of the same generator."""
    prob = I.spacetime(nx=args.st_nx, ny=args.st_ny, nt=args.st_nt)
    E = st_edge_count(prob)
    N = prob.n
    alg_full = 16 * E + 8 * N
    alg_theta = 12 * E + 4 * N
    progress(f"space-time {prob.nx}x{prob.ny}x{prob.nt}: {E} directed edges")
    ctx = G.gabp_st_create_problem(prob)
    if args.st_freeze_slots > 0:
        G.gabp_st_set_freeze_tolerance(ctx, args.st_freeze_slots, 1e-6)
    stream = ctx.stream

    def event_ms(fn, reps):
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in ev], time.perf_counter() - t0

    iterate = lambda: G.gabp_st_iterate(ctx, ITERS_PER_STEP, prob.damping)  # noqa: E731
    iterate()
    ms, _ = event_ms(iterate, 3)
    full_ms = sum(ms) / (3 * ITERS_PER_STEP)
    kernels = {"full": {"iter_ms": full_ms, "algorithmic_bytes": alg_full,
                        "gbps": alg_full / (full_ms * 1e-3) / 1e9}}
    # run on with checks until the precision messages freeze (bounded)
    while G.gabp_st_precision_frozen(ctx) < 0 and G.gabp_st_iteration_count(ctx)[0] < 3000:
        iterate()
        G.gabp_st_residual(ctx)
    frozen_at = G.gabp_st_precision_frozen(ctx)
    progress(f"space-time precision messages frozen at iteration {frozen_at}")
    best = None
    if frozen_at >= 0:
        # launch shape of the information-only kernel: slices per workgroup
        for sl in (1, 2, 4):
            G.gabp_st_set_theta_slices(ctx, sl)
            iterate()
            ms, _ = event_ms(iterate, 3)
            t_ms = sum(ms) / (3 * ITERS_PER_STEP)
            kernels[f"theta_slices{sl}"] = {"iter_ms": t_ms, "algorithmic_bytes": alg_theta,
                                            "gbps": alg_theta / (t_ms * 1e-3) / 1e9}
            if best is None or t_ms < kernels[f"theta_slices{best}"]["iter_ms"]:
                best = sl
        G.gabp_st_set_theta_slices(ctx, best)
    for _ in range(args.warmup):
        iterate()
        G.gabp_st_residual(ctx)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    rel = None
    for a, b in ev:
        a.record(stream)
        iterate()
        b.record(stream)
        rel, _ = G.gabp_st_residual(ctx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iter_ms = sum(a.elapsed_time(b) for a, b in ev) / (args.steps * ITERS_PER_STEP)
    its = G.gabp_st_iteration_count(ctx)[0]
    value = E * args.steps * ITERS_PER_STEP / wall
    phase = "theta" if frozen_at >= 0 else "full"
    alg = alg_theta if phase == "theta" else alg_full
    kname = "k_iter information-only (space-time)" if phase == "theta" else "k_iter full (space-time)"
    kernels[phase + "_timed"] = {"iter_ms": iter_ms, "algorithmic_bytes": alg,
                                 "gbps": alg / (iter_ms * 1e-3) / 1e9}
    achieved = alg / (iter_ms * 1e-3) / 1e9
    out = {"metric": "edge-message updates/s (space-time GMRF)", "value": value,
           "unit": "edge-message updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"{prob.name}: heat-equation prior (Crank-Nicolson, "
                                  f"nu dt/h^2 = {prob.nu * prob.dt / prob.h ** 2:g}), "
                                  f"{prob.nx}x{prob.ny} zero-flux grid x {prob.nt} slices, "
                                  f"38-neighbour stencil, {prob.coverage * 100:.2f}% observed, "
                                  f"c={prob.c}, damping={prob.damping}, FP32 messages, "
                                  f"FP64 residual",
                      "nodes": N, "directed_edges": E, "iters_per_step": ITERS_PER_STEP,
                      "parallelism": "single GPU"},
           "iterations_run": its, "rel_residual_after": rel,
           "timed_phase": {"kernel": kname, "precision_frozen_at_iteration": frozen_at,
                           "freeze_tolerance_slots": args.st_freeze_slots,
                           "theta_slices_per_workgroup": best},
           "kernels": kernels,
           "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "iter_ms": iter_ms, "algorithmic_bytes_per_launch": alg,
                        "traffic": (_summary_value(ST_TRAFFIC_SUMMARY,
                                                   kernel_source_digest(ST_SOURCES),
                                                   f"st_k_iter_{phase}"
                                                   + (f"_s{best}" if phase == "theta" else "")
                                                   + "_traffic_bytes_per_launch")
                                    if (prob.nx, prob.ny, prob.nt) == (512, 512, 64) else None)}}
    if args.st_solve_tol > 0:
        progress(f"space-time solve to {args.st_solve_tol:g}")
        ctx2 = G.gabp_st_create_problem(prob)
        if args.st_freeze_slots > 0:
            G.gabp_st_set_freeze_tolerance(ctx2, args.st_freeze_slots, 1e-6)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, it, r = G.gabp_st_solve(ctx2, args.solve_max_iters, prob.damping, args.st_solve_tol,
                                    100)
        torch.cuda.synchronize()
        out["time_to_tol"] = {"tol": args.st_solve_tol, "status": G.gabp_status_string(st),
                              "iterations": it, "seconds": time.perf_counter() - t1,
                              "rel_residual": r,
                              "precision_frozen_at": G.gabp_st_precision_frozen(ctx2)}
        del ctx2
        progress(f"space-time multigrid to {args.st_solve_tol:g}")
        from paper_2404_12968_amd import multigrid as MG
        import dataclasses
        pm = dataclasses.replace(prob, rel_tol=args.st_solve_tol)
        ft = (args.st_freeze_slots, 1e-6) if args.st_freeze_slots > 0 else None
        r = MG.st_multigrid_solve(pm, max_iters=args.solve_max_iters, freeze_tolerance=ft,
                                  check_every=100)
        out["multigrid"] = {"tol": args.st_solve_tol, "status": G.gabp_status_string(r["status"]),
                            "seconds": r["seconds"], "fine_iterations": r["iterations"],
                            "rel_residual": r["rel"],
                            "levels": [{k: lv[k] for k in ("level", "nx", "ny", "nt",
                                                           "iterations", "rel")}
                                       for lv in r["levels"]]}
    del ctx
    if not args.no_cpu_baseline:
        progress("space-time CPU baseline")
        from oracle import oracle as O
        from oracle import spacetime as S
        small = I.spacetime(nx=128, ny=128, nt=16, dtype="f64")
        A, b = S.posterior_system(small)
        og = O.OracleGaBP(O.FactorGraph(A, b), small.c)
        og.iterate(2, small.damping)
        n_it = 0
        t0 = time.perf_counter()
        while True:
            og.iterate(2, small.damping)
            n_it += 2
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds and n_it >= 6:
                break
        out["cpu_baseline"] = {"value": og.g.nnz * n_it / el, "unit": "edge-message updates/s",
                               "cores": O.max_threads(), "kind": "oracle",
                               "sample": f"FP64 oracle on 128x128x16 of the same generator "
                                         f"({og.g.nnz} directed edges), {n_it} iterations "
                                         f"after 2 warm-up, {el:.1f} s"}
    progress(f"space-time done: {value:.3e} edge-message updates/s, {achieved:.0f} GB/s")
    return out


def bench_warm(I, n, freeze=None, fp64_ref=True, tol=None):
    """Time to 1e-6 on held-out 1024^2 warm-start problems, cold vs the trained
    network's warm start (inference and the fallback probe included) vs
    multigrid; each FP32 mean's relative L2 error against the FP64 reference."""
    from paper_2404_12968_amd import gabp as G
    from paper_2404_12968_amd import multigrid as MG
    from paper_2404_12968_amd import warm as Wm
    path = os.path.join(ROOT, "paper_2404_12968_amd", "weights", "warm1024.npz")
    net = Wm.WarmNet.load(path)
    rows = []
    for k in range(n):
        p = I.warm1024(instance=300000 + k)
        c = Wm.cold_solve(p, freeze_tolerance=freeze, keep_mean=fp64_ref)
        w = Wm.warm_solve(net, p, freeze_tolerance=freeze, keep_mean=fp64_ref)
        rows.append({"instance": 300000 + k, "kappa": round(p.kappa, 4),
                     "cold_iters": c["iterations"], "cold_s": c["seconds"],
                     "warm_iters": w["iterations"], "warm_s": w["seconds"], "start": w["start"],
                     "cold_frozen_at": c["frozen_at"], "warm_frozen_at": w["frozen_at"]})
        m = MG.multigrid_solve(p, keep_context=fp64_ref, freeze_tolerance=freeze)
        rows[-1]["multigrid_iters"], rows[-1]["multigrid_s"] = m["iterations"], m["seconds"]
        if fp64_ref:
            mm = G.gabp_posterior(m["ctx"], want_var=False)[0]
            G.gabp_destroy(m["ctx"])
            ref, info = fp64_reference(p, tol)
            rows[-1]["error_vs_fp64"] = {"cold": rel_err(c["mean"], ref),
                                         "warm": rel_err(w["mean"], ref),
                                         "multigrid": rel_err(mm, ref),
                                         "reference_rel_residual": info["rel_residual"]}
            del ref, mm
    cs = sum(r["cold_s"] for r in rows)
    ws = sum(r["warm_s"] for r in rows)
    ms = sum(r["multigrid_s"] for r in rows)
    return {"workload": "warm1024: 1024x1024, alpha=2, kappa ~ U[0.02,0.3], 16 tracks (~6%), "
                        "sigma 0.05, FP32 to 1e-6; held-out seeds",
            "freeze_tolerance": {"max_slots": freeze[0], "max_rel": freeze[1]} if freeze
            else "bitwise",
            "error_vs_fp64_note": "relative L2 of each FP32 mean against the same problem solved "
                                  "with FP64 messages by multigrid to the same residual",
            "cold_seconds": cs, "warm_seconds": ws, "speedup": cs / ws if ws > 0 else None,
            "multigrid_seconds": ms, "multigrid_speedup": cs / ms if ms > 0 else None,
            "instances": rows}


def bench_multigrid(G, prob, ref=None):
    """Time to the problem's tolerance by coarse-to-fine multigrid (all levels
    and transfers included); with ref, the mean's error against it."""
    from paper_2404_12968_amd import multigrid as MG
    r = MG.multigrid_solve(prob, keep_context=True)
    out = {"tol": prob.rel_tol, "status": G.gabp_status_string(r["status"]),
           "seconds": r["seconds"], "fine_iterations": r["iterations"],
           "rel_residual": r["rel"],
           "levels": [{"nx": lv["nx"], "ny": lv["ny"], "iterations": lv["iterations"],
                       "observations": lv["observations"]} for lv in r["levels"]]}
    if ref is not None:
        out["error_vs_fp64"] = rel_err(G.gabp_posterior(r["ctx"], want_var=False)[0], ref)
    G.gabp_destroy(r["ctx"])
    return out


def bench_batch(G, I, torch, dev, args):
    """The 256-instance uneven batch: every instance solved to 1e-6 by the
    batched path (persistent work-list launches, per-instance retirement,
    captured chunk graphs)."""
    import numpy as np
    probs = I.batch256()
    Es = np.array([edge_count(p.nx, p.ny, p.alpha, p.bc_x, p.bc_y) for p in probs], dtype=np.int64)
    Ns = np.array([p.n for p in probs], dtype=np.int64)
    a2 = np.array([p.alpha == 2 for p in probs])

    def run(slots):
        b = G.gabp_batch_create(probs, device=dev)
        if slots > 0:
            G.gabp_batch_set_freeze_tolerance(b, slots, args.freeze_rel)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, its, rels, sts = G.gabp_batch_solve(b, max(args.solve_max_iters, 300000), 0.5, 1e-6,
                                                -10)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        frozen = [G.gabp_batch_info(b, i)[1] for i in range(len(probs))]
        del b
        return wall, st, its, rels, sts, frozen

    def summary(wall, st, its, rels, sts, frozen):
        return {"seconds_to_all_converged": wall, "status": G.gabp_status_string(st),
                "edge_updates_per_s": float((Es * its).sum()) / wall,
                "converged": int((sts == G.GABP_OK).sum()),
                "diverged": int((sts == G.GABP_E_DIVERGED).sum()),
                "iterations_alpha1": [int(its[~a2].min()), int(np.median(its[~a2])), int(its[~a2].max())],
                "iterations_alpha2": [int(its[a2].min()), int(np.median(its[a2])), int(its[a2].max())],
                "frozen_at_median": float(np.median([f for f in frozen if f >= 0])) if any(f >= 0 for f in frozen) else None,
                "frozen_instances": int(sum(f >= 0 for f in frozen)),
                "max_rel_residual": float(rels.max()),
                "not_converged": [{"instance": int(i), "side": probs[i].nx, "alpha": probs[i].alpha,
                                   "kappa": probs[i].kappa, "sigma": probs[i].sigma,
                                   "coverage": probs[i].coverage, "rel": float(rels[i]),
                                   "iterations": int(its[i])}
                                  for i in np.nonzero(sts != G.GABP_OK)[0]]}

    # headline: precision messages frozen only when bitwise stationary (every
    # result bitwise that of the unfrozen iteration); beside it the run with
    # the freeze tolerance
    progress("batch256, bitwise freeze")
    r0 = run(0)
    wall, st, its, rels, sts, frozen = r0
    updates = float((Es * its).sum())
    tol_run = None
    if args.freeze_slots > 0:
        progress(f"batch256, freeze tolerance {args.freeze_slots} messages / {args.freeze_rel:g}")
        tol_run = summary(*run(args.freeze_slots))
        tol_run["freeze_tolerance"] = {"max_slots": args.freeze_slots, "max_rel": args.freeze_rel}
    mg = None
    if not args.no_multigrid:
        from paper_2404_12968_amd import multigrid as MG
        ft = (args.freeze_slots, args.freeze_rel) if args.freeze_slots > 0 else None
        r = MG.multigrid_batch_solve(probs, max_iters=max(args.solve_max_iters, 300000),
                                     freeze_tolerance=ft)
        fi = np.asarray(r["iterations"])
        mg = {"seconds": r["seconds"], "status": G.gabp_status_string(r["status"]),
              "converged": int((np.asarray(r["statuses"]) == G.GABP_OK).sum()),
              "speedup_vs_bitwise_run": wall / r["seconds"],
              "speedup_vs_freeze_tolerance_run": (tol_run["seconds_to_all_converged"] / r["seconds"]
                                                  if tol_run else None),
              "fine_iterations_alpha1": [int(fi[~a2].min()), int(np.median(fi[~a2])), int(fi[~a2].max())],
              "fine_iterations_alpha2": [int(fi[a2].min()), int(np.median(fi[a2])), int(fi[a2].max())],
              "max_rel_residual": float(np.max(r["rel"])),
              "levels": [{"level": lv["level"], "instances": lv["instances"],
                          "max_iterations": max(lv["iterations"])} for lv in r["levels"]],
              "note": "every level's batch set-up (inputs to device) and the transfers are "
                      "inside the time; the one-level time above excludes its set-up"}
    return {
        "metric": METRIC, "value": updates / wall, "unit": "edge-message updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch256: 256 instances, side ~ U{64..1024}, alpha ~ U{1,2}, "
                               "kappa ~ U[0.02,0.3], 1-20% observed, sigma ~ U[0.02,0.2], "
                               "each to 1e-6, checks adaptive (every 10 until all running instances "
                               "froze, then growing with the slowest one's residual decay)",
                   "freeze_tolerance": {"max_slots": 0, "max_rel": 0.0,
                                        "note": "headline run: bitwise freeze only"},
                   "nodes": int(Ns.sum()), "directed_edges": int(Es.sum()),
                   "parallelism": "single GPU"},
        "batch": summary(*r0),
        "batch_freeze_tolerance": tol_run,
        "multigrid": mg,
    }


def bench_table1(G, I, torch, args):
    """The paper's synthetic experiment (Table 1): 256^2, 512^2 and 1024^2
    grids at 1, 5 and 10 % observed, three truths each, message passing as the
    paper runs it: multigrid from 32^2 (precision messages carried between
    levels), c = 10, learning rate 0.6, every level stopped by the early-stop
    rule at 1e-3 or after T = 10 000 iterations.  Times are end to end from
    host-resident observations (level set-up, transfers and read-backs
    included); truth sampling is not timed."""
    import math

    import numpy as np
    from paper_2404_12968_amd import multigrid as MG

    ft = (args.freeze_slots, args.freeze_rel) if args.freeze_slots > 0 else None

    def run(p, transfer="messages", stop="message_change", max_iters=10000):
        r = MG.multigrid_solve(p, coarse_stop=stop, final_stop=stop, max_iters=max_iters,
                               keep_context=True, freeze_tolerance=ft, transfer=transfer)
        mu = G.gabp_posterior(r["ctx"], want_var=False)[0].cpu().numpy().ravel()
        G.gabp_destroy(r["ctx"])
        return r, float(np.sqrt(np.mean((mu - p.truth.ravel()) ** 2)))

    run(I.table1(256, 0.05, 99))     # module load and first launches, untimed
    with open(os.path.join(ROOT, "tests", "golden", "table1.json")) as f:
        gold = json.load(f)
    rows = []
    total = 0.0
    for n in I.TABLE1_SIZES:
        for k, frac in enumerate(I.TABLE1_FRACS):
            v = []
            for inst in range(args.table1_truths):
                p = I.table1(n, frac, inst)
                r, e = run(p)
                v.append((r["seconds"], r["iterations"], e, G.gabp_status_string(r["status"]),
                          [lv["iterations"] for lv in r["levels"]]))
            secs = float(np.mean([x[0] for x in v]))
            rm = float(np.mean([x[2] for x in v]))
            row = {"grid": n, "observed": frac, "seconds": secs,
                   "rmse": rm if math.isfinite(rm) else None,
                   "fine_iterations": float(np.mean([x[1] for x in v])),
                   "level_iterations": [x[4] for x in v], "status": [x[3] for x in v],
                   "paper_mp_seconds_rtx3090": gold["seconds_mp_rtx3090"][str(n)][k],
                   "paper_mp_rmse": gold["rmse_mp"][str(n)][k],
                   "paper_exact_rmse": gold["rmse_exact"][str(n)][k]}
            total += secs
            rows.append(row)
            print(f"[table1] {n}^2 {frac:.0%}: {secs:.3f} s rmse {rm:.4f} "
                  f"(paper MP {row['paper_mp_rmse']}, exact {row['paper_exact_rmse']}) "
                  f"{[x[3] for x in v]}", file=sys.stderr, flush=True)
    diagnosis = None
    if args.table1_diagnose:
        # the 1 % rows, where every level runs into the T cap: the paper's
        # Upscale Messages read literally (edge values copied unchanged), and
        # the same runs with no cap, each level solved to a 1e-6 residual
        diagnosis = []
        for n in I.TABLE1_SIZES:
            k = I.TABLE1_FRACS.index(0.01)
            rec = {"grid": n, "observed": 0.01,
                   "paper_mp_rmse": gold["rmse_mp"][str(n)][k],
                   "paper_exact_rmse": gold["rmse_exact"][str(n)][k]}
            for name, kw in (("messages_T10000", {}),
                             ("literal_T10000", {"transfer": "literal"}),
                             ("messages_to_1e-6", {"stop": "residual", "max_iters": 300000})):
                out_v = []
                for inst in range(args.table1_truths):
                    r, e = run(I.table1(n, 0.01, inst), **kw)
                    out_v.append((e, r["seconds"], [lv["iterations"] for lv in r["levels"]],
                                  G.gabp_status_string(r["status"])))
                rec[name] = {"rmse": float(np.mean([x[0] for x in out_v])),
                             "seconds": float(np.mean([x[1] for x in out_v])),
                             "level_iterations": [x[2] for x in out_v],
                             "status": [x[3] for x in out_v]}
                print(f"[table1 1%] {n}^2 {name}: rmse {rec[name]['rmse']:.4f} "
                      f"{rec[name]['seconds']:.2f} s", file=sys.stderr, flush=True)
            diagnosis.append(rec)
    paper_total = sum(sum(v) for v in gold["seconds_mp_rtx3090"].values())
    return {"metric": "wall time of the paper's synthetic experiments (Table 1: 9 grids x "
                      "densities, mean over truths), message passing as the paper runs it",
            "value": total, "unit": "s", "n_gpus": 1, "steps": len(rows),
            "warmup": 1, "ms_per_step": total / len(rows) * 1e3, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": total / paper_total, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "table1: unit square, zero boundary values, alpha=2, nu=1, "
                                   "length scale 0.15, sigma_f 1.1, sigma_y 0.01, uniform "
                                   "random observations; multigrid from 32^2, c=10, eta=0.6, "
                                   "early stop 1e-3, T=10000 per level",
                       "truths_per_config": args.table1_truths, "parallelism": "single GPU",
                       "freeze_tolerance": {"max_slots": ft[0] if ft else 0,
                                            "max_rel": ft[1] if ft else 0.0}},
            "baseline_note": f"paper: {paper_total:.1f} s on one RTX 3090 (Table 1 MP column)",
            "rows": rows, "one_percent_diagnosis": diagnosis}


def net_flops_per_pixel():
    """FLOPs of one forward pass of the warm-start network per pixel: each
    layer is a 3x3 convolution computed over all its stored channels (the
    kernels pad the input to 16 or 32 channels), 2 FLOPs per multiply-add."""
    from paper_2404_12968_amd import warm as Wm
    return sum(2 * 9 * ci * co for ci, co in zip(Wm.CIN, Wm.COUT))


def bench_warmnet(G, I, torch, args):
    """The learned warm start's network kernels (BF16 operands, FP32
    accumulation on the matrix cores): inference on one 1024^2 problem and
    training steps (forward, both gradients, loss, Adam) on batches of eight
    256^2 crops, timed with HIP events on the stream the kernels run on."""
    from paper_2404_12968_amd import warm as Wm
    net = Wm.WarmNet.load(os.path.join(ROOT, "paper_2404_12968_amd", "weights", "warm1024.npz"))
    probs = [I.warm1024(instance=310000 + k) for k in range(2)]
    feats = [G.gabp_warm_features(p.cells, p.y, p.nx, p.ny, p.kappa) for p in probs]
    stream = torch.cuda.current_stream()
    fpp = net_flops_per_pixel()

    def events(fn, reps):
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]

    x1 = feats[0].unsqueeze(0).contiguous()
    for _ in range(3):
        net.forward(x1)
    inf_ms = events(lambda: net.forward(x1), max(5, args.steps))
    inf_flops = fpp * x1.shape[1] * x1.shape[2]
    # a training batch: 8 crops of 256^2 with synthetic targets of the real shape
    B, crop = 8, 256
    rng = np.random.default_rng(0)
    xs = []
    for k in range(B):
        f = feats[k % 2]
        cy, cx = int(rng.integers(0, 1024 - crop)), int(rng.integers(0, 1024 - crop))
        xs.append(f[cy:cy + crop, cx:cx + crop])
    xb = torch.stack(xs).contiguous()
    P = B * crop * crop
    mu = torch.zeros(P, dtype=torch.float32, device=xb.device)
    lam = torch.zeros((Wm.NDIR, P), dtype=torch.float32, device=xb.device)
    val = torch.ones_like(lam)

    def train_step():
        acts, pred = net.forward(xb)
        _, grad = G.gabp_warm_loss(pred, mu, lam, val, Wm.NDIR, 0.1)
        dws, dbs = net.backward(acts, grad)
        net.adam(dws, dbs, 0.0)

    for _ in range(3):
        train_step()
    step_ms = events(train_step, max(5, args.steps))
    # backward: the data gradient of layers 2..6 and the weight gradient of
    # every layer, each as many FLOPs as that layer's forward pass
    per_layer = [2 * 9 * ci * co for ci, co in zip(Wm.CIN, Wm.COUT)]
    train_flops = P * (sum(per_layer) + sum(per_layer[1:]) + sum(per_layer))
    peak = 2.5e15
    return {"metric": "warm-start network: inference and training step time, TFLOP/s",
            "value": train_flops / (step_ms * 1e-3) / 1e12, "unit": "TFLOP/s",
            "n_gpus": 1, "steps": max(5, args.steps), "warmup": 3, "ms_per_step": step_ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic",
            "config": {"workload": "warmnet: 6 layers of 3x3 convolutions, 32 channels, "
                                   "dilations 1,3,9,27,9,1; inference on 1024^2, training "
                                   "steps on 8 crops of 256^2", "parallelism": "single GPU"},
            "inference": {"ms": inf_ms, "pixels": int(x1.shape[1] * x1.shape[2]),
                          "gflop": inf_flops / 1e9,
                          "tflops": inf_flops / (inf_ms * 1e-3) / 1e12},
            "training_step": {"ms": step_ms, "pixels": P, "gflop": train_flops / 1e9,
                              "tflops": train_flops / (step_ms * 1e-3) / 1e12},
            "roofline": {"bound": "mfma", "kernel": "network forward (inference)",
                         "achieved": inf_flops / (inf_ms * 1e-3) / 1e12, "peak": peak / 1e12,
                         "unit": "TFLOP/s",
                         "frac": inf_flops / (inf_ms * 1e-3) / peak, "traffic": None}}


def bench_table2(G, I, torch, args):
    """The paper's grid search (Table 2): plain message passing (one grid,
    cold start) on the Table 1 generator's 128^2, 256^2 and 512^2 problems at
    5 % observed, for every re-weighting constant c and learning rate eta of
    the table, 4000 iterations (FP64 residual checks every 50: a flagged
    cavity precision or non-finite value, or a residual 1e3 times the first
    check's, is a divergence); RMSE against the truth divided by the exact
    posterior's RMSE (stored by tests/golden/make_table2_exact.py), mean over
    three truths, beside the paper's printed ratios."""
    import dataclasses
    gdir = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gdir, "table2_ratios.json")) as f:
        paper = json.load(f)
    with open(os.path.join(gdir, "table2_exact_rmse.json")) as f:
        exact = json.load(f)["rmse_exact"]
    cs = paper["c_values"]
    etas = ("0.6", "0.7", "0.8")
    rows = []
    pattern_ok = True
    t0 = time.perf_counter()
    for n in (128, 256, 512):
        probs = [I.table1(n, 0.05, inst) for inst in range(len(exact[str(n)]))]
        for eta_s in etas:
            ours = []
            for ci, c in enumerate(cs):
                ratios, div = [], False
                for k, p in enumerate(probs):
                    q = dataclasses.replace(p, c=float(c), damping=float(eta_s))
                    ctx = G.gabp_create_problem(q)
                    st, it, rel = G.gabp_solve(ctx, paper["iterations"], float(eta_s), 0.0, 50)
                    if st == G.GABP_E_DIVERGED:
                        div = True
                        G.gabp_destroy(ctx)
                        break
                    mu = G.gabp_posterior(ctx, want_var=False)[0].cpu().numpy().ravel()
                    G.gabp_destroy(ctx)
                    ratios.append(float(np.sqrt(np.mean((mu - p.truth.ravel()) ** 2))
                                        / exact[str(n)][k]))
                want = paper["ratio"][str(n)][eta_s][ci]
                pattern_ok &= div == (want is None)
                ours.append(None if div else float(np.mean(ratios)))
            rows.append({"grid": n, "eta": float(eta_s), "c": cs, "ratio": ours,
                         "paper_ratio": paper["ratio"][str(n)][eta_s]})
            progress(f"table2 {n}^2 eta {eta_s}: {ours}")
    sec = time.perf_counter() - t0
    best = {}
    for r in rows:
        if r["eta"] == 0.6:
            ok = [(v, c) for v, c in zip(r["ratio"], r["c"]) if v is not None]
            best[str(r["grid"])] = min(ok)[1] if ok else None
    return {"metric": "Table 2 grid search: RMSE(message passing after 4000 iterations) / "
                      "RMSE(exact posterior), 5% observed",
            "value": sec, "unit": "s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
            "ms_per_step": sec / len(rows) * 1e3, "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "table2: Table 1 generator (unit square, zero boundary "
                                   "values, alpha=2, length scale 0.15, sigma_f 1.1, "
                                   "sigma_y 0.01), 5% uniform random observations, one grid, "
                                   "cold start, 4000 iterations, FP32 messages",
                       "truths_per_config": len(exact["128"]), "parallelism": "single GPU"},
            "divergence_pattern_matches_paper": bool(pattern_ok),
            "best_c_at_eta_0.6": best, "rows": rows}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="global8192",
                    choices=["global8192", "tracks2048", "batch256", "table1", "table2",
                             "global32k", "warmnet", "spacetime"])
    ap.add_argument("--st-nx", type=int, default=512)
    ap.add_argument("--st-ny", type=int, default=512)
    ap.add_argument("--st-nt", type=int, default=64)
    ap.add_argument("--st-freeze-slots", type=int, default=64,
                    help="spacetime: freeze tolerance (messages changed by at most 1e-6)")
    ap.add_argument("--st-solve-tol", type=float, default=0.0,
                    help="spacetime: also solve a fresh context to this relative residual")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the cold solve to the workload's tolerance")
    ap.add_argument("--solve-max-iters", type=int, default=200000)
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the warm-vs-cold time-to-1e-6 leg (1024^2 workload)")
    ap.add_argument("--warm-instances", type=int, default=8)
    ap.add_argument("--warm-freeze-slots", type=int, default=64,
                    help="warm-start leg: freeze tolerance (messages) of the cold, warm and "
                         "multigrid solves alike (0: bitwise freeze only)")
    ap.add_argument("--fp64-ref-tol", type=float, default=None,
                    help="residual of the FP64 reference solves (default: each problem's own)")
    ap.add_argument("--no-fp64-ref", action="store_true",
                    help="skip the FP64 reference solves that the FP32 results' errors are "
                         "measured against")
    ap.add_argument("--freeze-slots", type=int, default=64,
                    help="batch256 and table1: freeze the precision messages when at most this "
                         "many changed in the last iteration (0: only when none did)")
    ap.add_argument("--freeze-rel", type=float, default=1e-6,
                    help="batch256 and table1: ... each by at most this relative change")
    ap.add_argument("--table1-truths", type=int, default=3,
                    help="ground truths per Table 1 configuration")
    ap.add_argument("--table1-diagnose", action="store_true",
                    help="table1: rerun the 1 %% rows with the literal message copy between "
                         "levels and with every level solved to a 1e-6 residual")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the paper's Table 1 leg (nine grid/density configurations)")
    ap.add_argument("--no-multigrid", action="store_true",
                    help="skip the multigrid time-to-tolerance leg")
    ap.add_argument("--print-digest", action="store_true",
                    help="print the iteration kernels' source digest and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain device copy of known size (PMC byte calibration) and exit")
    args = ap.parse_args(argv)

    if args.print_digest:
        print("lattice iteration kernels:", kernel_source_digest())
        print("space-time kernels:", kernel_source_digest(ST_SOURCES))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the lattice would shard into row strips with a halo exchange; not built).",
              file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))
        return 0

    from paper_2404_12968_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_2404_12968_amd import gabp as G
    from paper_2404_12968_amd import inputs as I

    if args.workload == "batch256":
        print(json.dumps(bench_batch(G, I, torch, dev, args)), flush=True)
        return 0
    if args.workload == "table1":
        print(json.dumps(bench_table1(G, I, torch, args)), flush=True)
        return 0
    if args.workload == "table2":
        print(json.dumps(bench_table2(G, I, torch, args)), flush=True)
        return 0
    if args.workload == "warmnet":
        print(json.dumps(bench_warmnet(G, I, torch, args)), flush=True)
        return 0
    if args.workload == "spacetime":
        print(json.dumps(bench_spacetime(G, I, torch, args)), flush=True)
        return 0

    prob = I.workload(args.workload)
    E = edge_count(prob.nx, prob.ny, prob.alpha, prob.bc_x, prob.bc_y)
    N = prob.n
    esize = 4 if prob.dtype == "f32" else 8
    # algorithmic bytes of one iteration.  Full kernel: read + write both
    # components of every directed message once, read the two node terms.
    # Information-only kernel (precision messages frozen): read the edge gain
    # and the information message, write the information message, read b.
    alg_full = 4 * esize * E + 2 * esize * N
    alg_theta = 3 * esize * E + esize * N

    ctx = G.gabp_create_problem(prob, device=dev)
    stream = ctx.stream

    def step(ev0=None, ev1=None):
        # one check interval of the solver: ITERS_PER_STEP iterations (a
        # recorded chunk graph), FP64 marginals and residual, read-back
        if ev0 is not None:
            ev0.record(stream)
        _, _, rel = G.gabp_solve(ctx, ITERS_PER_STEP, prob.damping, 0.0, ITERS_PER_STEP)
        if ev1 is not None:
            ev1.record(stream)
        return rel

    def timed(nsteps):
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(nsteps)]
        t0 = time.perf_counter()
        r = None
        for k in range(nsteps):
            r = step(*evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        it_ms = sum(a.elapsed_time(b) for a, b in evs) / (nsteps * ITERS_PER_STEP)
        return wall, it_ms, r

    kernels = {}
    # phase 1: full iteration kernel.  Freezing is only detected by residual
    # checks, so iterations without them stay on the full kernel.
    rpt_full = G.gabp_autotune(ctx, 3, prob.damping)
    torch.cuda.synchronize()
    evf = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(3)]
    for a, b in evf:
        a.record(stream)
        G.gabp_iterate(ctx, ITERS_PER_STEP, prob.damping)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evf) / (3 * ITERS_PER_STEP)
    kernels["full"] = {"iter_ms": ms, "algorithmic_bytes": alg_full,
                       "gbps": alg_full / (ms * 1e-3) / 1e9, "rows_per_thread": rpt_full}
    step()
    # run on until the precision messages freeze (bounded)
    while G.gabp_precision_frozen(ctx) < 0 and G.gabp_iteration_count(ctx)[0] < 2000:
        step()
    frozen_at = G.gabp_precision_frozen(ctx)
    phase = "theta" if frozen_at >= 0 else "full"
    rpt = G.gabp_autotune(ctx, 3, prob.damping) if phase == "theta" else rpt_full
    pair = G.gabp_get_tile(ctx)[1] if phase == "theta" else 0

    def event_ms(fn, reps):
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b_ in ev:
            a.record(stream)
            fn()
            b_.record(stream)
        torch.cuda.synchronize()
        return sum(a.elapsed_time(b_) for a, b_ in ev) / reps

    if phase == "theta":
        # single-iteration information kernel, then the two-iteration kernel:
        # a call of 2m+1 iterations is m pair launches and one single launch
        G.gabp_set_tile(ctx, rpt, 0)
        ms1 = event_ms(lambda: G.gabp_iterate(ctx, ITERS_PER_STEP, prob.damping), 3) / ITERS_PER_STEP
        kernels["theta"] = {"iter_ms": ms1, "algorithmic_bytes": alg_theta,
                            "gbps": alg_theta / (ms1 * 1e-3) / 1e9, "rows_per_thread": rpt}
        # tile heights, then the column-strip walker's bands (negative)
        for p2 in ((4, 8, 12, 16, 32, -2, -4, -8) if prob.dtype == "f32" else (4, -2)):
            G.gabp_set_tile(ctx, rpt, p2)
            m = 10
            ms_call = event_ms(lambda: G.gabp_iterate(ctx, 2 * m + 1, prob.damping), 3)
            ms2 = (ms_call - ms1) / m
            kernels[f"theta_pair{p2}" if p2 > 0 else f"theta_walk{-p2}"] = {
                "launch_ms": ms2, "iters_per_launch": 2, "iter_ms": ms2 / 2,
                "algorithmic_bytes": alg_theta,
                "gbps": alg_theta / (ms2 * 1e-3) / 1e9,
                "single_pass_equivalent_gbps": 2 * alg_theta / (ms2 * 1e-3) / 1e9,
                "pair_rows": p2}
        G.gabp_set_tile(ctx, rpt, pair)
    for _ in range(args.warmup):
        step()
    wall, iter_ms, rel = timed(args.steps)
    if phase == "full":
        kernels["full_timed"] = {"iter_ms": iter_ms}
    total_iters = args.steps * ITERS_PER_STEP
    value = E * total_iters / wall
    if phase == "theta" and pair != 0:
        # two iterations per launch with the intermediate one kept on chip:
        # the launch must read its inputs and write its outputs once, the
        # bytes of one single-iteration pass
        kname = "k_iter_theta2" if pair > 0 else "k_iter_theta2w"
        launch_ms = kernels[f"theta_pair{pair}" if pair > 0 else f"theta_walk{-pair}"]["launch_ms"]
        alg_launch = alg_theta
        traffic = measured_traffic("theta2" if pair > 0 else "theta2w", pair, prob.name)
    elif phase == "theta":
        kname = "k_iter_theta"
        launch_ms = kernels["theta"]["iter_ms"]
        alg_launch = alg_theta
        traffic = measured_traffic("theta", rpt, prob.name)
    else:
        kname = "k_iter_direct"
        launch_ms = kernels["full"]["iter_ms"]
        alg_launch = alg_full
        traffic = measured_traffic("full", rpt, prob.name)
    achieved = alg_launch / (launch_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edge-message updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prob.dtype,
        "data": "synthetic",
        "config": {"workload": f"{prob.name}: {prob.nx}x{prob.ny} lattice, alpha={prob.alpha} "
                               f"({'13' if prob.alpha == 2 else '5'}-point), kappa={prob.kappa}, "
                               f"{prob.coverage * 100:.2f}% observed, c={prob.c}, "
                               f"damping={prob.damping}, {prob.dtype} messages, FP64 residual",
                   "nodes": N, "directed_edges": E, "iters_per_step": ITERS_PER_STEP,
                   "parallelism": "single GPU"},
        "hbm_gbps_algorithmic": achieved,
        "step_ms_per_iteration": iter_ms,
        "rel_residual_after": rel,
        "timed_phase": {"kernel": kname, "precision_frozen_at_iteration": frozen_at,
                        "rows_per_thread": rpt, "pair_rows": pair,
                        "iterations_before_timing": G.gabp_iteration_count(ctx)[0] - total_iters},
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "measured_copy_ceiling": copy_ceiling_gbps(torch, dev),
                     "launch_ms": launch_ms, "algorithmic_bytes_per_launch": alg_launch,
                     "iterations_per_launch": 2 if kname.startswith("k_iter_theta2") else 1,
                     "single_pass_equivalent_gbps": (
                         (2 if kname.startswith("k_iter_theta2") else 1) * alg_launch
                         / (launch_ms * 1e-3) / 1e9),
                     "traffic": traffic},
    }
    del ctx
    progress(f"timed steps done: {value:.3e} edge-message updates/s")
    ref = None
    if not args.no_fp64_ref and (not args.no_solve or not args.no_multigrid):
        ref, info = fp64_reference(prob, args.fp64_ref_tol)
        out["fp64_reference"] = info
    if not args.no_solve:
        progress("cold solve to the tolerance")
        ctx2 = G.gabp_create_problem(prob, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, it, r = G.gabp_solve(ctx2, args.solve_max_iters, prob.damping, prob.rel_tol, -10)
        torch.cuda.synchronize()
        out["time_to_tol"] = {"tol": prob.rel_tol, "status": G.gabp_status_string(st),
                              "iterations": it, "seconds": time.perf_counter() - t1,
                              "rel_residual": r, "start": "cold"}
        if ref is not None:
            out["time_to_tol"]["error_vs_fp64"] = rel_err(
                G.gabp_posterior(ctx2, want_var=False)[0], ref)
        del ctx2
    if not args.no_multigrid:
        progress("multigrid solve to the tolerance")
        out["multigrid"] = bench_multigrid(G, prob, ref)
        if "time_to_tol" in out:
            out["multigrid"]["speedup_vs_cold"] = (out["time_to_tol"]["seconds"] /
                                                   out["multigrid"]["seconds"])
    del ref
    if not args.no_warm:
        progress("warm-start leg")
        wf = (args.warm_freeze_slots, args.freeze_rel) if args.warm_freeze_slots > 0 else None
        out["warm_start"] = bench_warm(I, args.warm_instances, wf, not args.no_fp64_ref,
                                       args.fp64_ref_tol)
    if not args.no_table1:
        progress("Table 1 leg")
        t1 = bench_table1(G, I, torch, args)
        out["table1"] = {"seconds": t1["value"], "paper_seconds_rtx3090": t1["value"] / t1["vs_baseline"],
                         "config": t1["config"]["workload"], "truths_per_config": args.table1_truths,
                         "rows": [{k: r[k] for k in ("grid", "observed", "seconds", "rmse",
                                                      "paper_mp_seconds_rtx3090", "paper_mp_rmse",
                                                      "paper_exact_rmse")} for r in t1["rows"]]}
    if not args.no_cpu_baseline:
        progress("CPU baseline")
        gi = {}
        if "time_to_tol" in out:
            gi[prob.name] = out["time_to_tol"]["iterations"]
        if "warm_start" in out:
            gi["warm1024_to_1e-6_cold"] = out["warm_start"]["instances"][0]["cold_iters"]
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds, gi)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
