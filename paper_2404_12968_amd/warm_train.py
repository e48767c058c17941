"""Train the warm-start network on solver solutions and evaluate it.

    python -m paper_2404_12968_amd.warm_train --n-train 128 --steps 3000 \\
        --out paper_2404_12968_amd/weights/warm1024.npz --eval 6

1. Draws `n-train` problems of the 1024 x 1024 warm-start workload (seeds
   seed-base .. seed-base + n-1) and solves them to 1e-6: with the batched
   solver (cold, or --multigrid), or (--warm-gen) one by one from the warm
   start of the network given by --init (the fixed points do not depend on
   the start).  The solutions stay on the GPU in compact form (observations
   and FP32 means; precision targets for the first --lam-targets).
2. Trains the network (Adam, cosine schedule) on random 256 x 256 crops of
   those solutions.
3. Solves `eval` held-out problems (seeds 100000 + k) cold and warm (network
   inference included in the warm time, cold fallback active, the same
   freeze tolerance for both) and prints one JSON summary line.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np
import torch

from . import inputs as I
from . import warm as Wm


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-train", type=int, default=128)
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lam-weight", type=float, default=0.1)
    ap.add_argument("--eval", type=int, default=6)
    ap.add_argument("--seed-base", type=int, default=0,
                    help="training problems are seeds seed_base .. seed_base + n_train - 1")
    ap.add_argument("--init", default=None,
                    help="continue from these weights (npz) instead of a fresh network")
    ap.add_argument("--multigrid", action="store_true",
                    help="solve the training problems by batched multigrid")
    ap.add_argument("--warm-gen", action="store_true",
                    help="solve the training problems from the --init network's warm start")
    ap.add_argument("--stream-multigrid", action="store_true",
                    help="solve the training problems one by one by multigrid while host "
                         "threads draw the next ones")
    ap.add_argument("--lam-targets", type=int, default=1024,
                    help="solutions that keep their precision targets")
    ap.add_argument("--max-gen-seconds", type=float, default=None,
                    help="stop generating training solutions after this long")
    ap.add_argument("--out", default=None)
    ap.add_argument("--summary", default=None)
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, flush=True)

    torch.cuda.set_device(0)
    seeds = range(args.seed_base, args.seed_base + args.n_train)

    def make(k):
        p = I.warm1024(instance=k, n=args.side)
        p.truth = None          # the solver's solution is the target
        return p

    ts = Wm.TrainingSet()
    deadline = time.time() + args.max_gen_seconds if args.max_gen_seconds else None
    t_gen = time.time()
    if args.stream_multigrid:
        ex = cf.ThreadPoolExecutor(max_workers=4)
        try:
            Wm.solve_training_set_multigrid(ex.map(make, seeds), log=log,
                                            lam_targets=args.lam_targets, ts=ts,
                                            deadline=deadline)
        finally:
            ex.shutdown(wait=False, cancel_futures=True)
    elif args.warm_gen:
        if not args.init:
            raise SystemExit("--warm-gen needs --init")
        gen_net = Wm.WarmNet.load(args.init)
        # problems are drawn on host threads while the GPU solves earlier ones
        ex = cf.ThreadPoolExecutor(max_workers=4)
        try:
            Wm.solve_training_set_warm(gen_net, ex.map(make, seeds), log=log,
                                       lam_targets=args.lam_targets, ts=ts, deadline=deadline)
        finally:
            ex.shutdown(wait=False, cancel_futures=True)
        del gen_net
    else:
        chunk = 64
        for c0 in range(0, len(seeds), chunk):
            if deadline is not None and time.time() >= deadline:
                log(f"[warm] generation deadline reached after {c0} problems")
                break
            Wm.solve_training_set([make(k) for k in seeds[c0:c0 + chunk]], log=log,
                                  multigrid=args.multigrid,
                                  lam_targets=len(ts) < args.lam_targets, ts=ts)
    gen_s = time.time() - t_gen
    log(f"[warm] training set: {len(ts)} solutions in {gen_s:.1f}s, iterations median "
        f"{int(np.median(ts.iters))}, {sum(l is not None for l in ts.lam)} with precision targets")
    net = Wm.WarmNet.load(args.init) if args.init else Wm.WarmNet(seed=0)
    t1 = time.time()
    hist = Wm.train(net, ts, args.steps, batch=args.batch, crop=args.crop, lr=args.lr,
                    lam_weight=args.lam_weight, log=log, log_every=200)
    train_s = time.time() - t1
    n_solutions = len(ts)
    del ts
    torch.cuda.empty_cache()
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        net.save(args.out, meta={"n_train": n_solutions, "steps": args.steps,
                                 "batch": args.batch, "crop": args.crop, "lr": args.lr,
                                 "side": args.side, "seed_base": args.seed_base,
                                 "init": args.init or "", "final_loss": hist[-1]})
        log(f"[warm] saved {args.out}")
    evals = []
    ft = (64, 1e-6)
    for k in range(args.eval):
        p = I.warm1024(instance=100000 + k, n=args.side)
        c = Wm.cold_solve(p, freeze_tolerance=ft)
        w = Wm.warm_solve(net, p, freeze_tolerance=ft)
        wm = Wm.warm_solve(net, p, use_precisions=False, freeze_tolerance=ft)
        evals.append({"instance": 100000 + k, "kappa": p.kappa, "coverage": p.coverage,
                      "cold_iters": c["iterations"], "cold_s": c["seconds"],
                      "warm_iters": w["iterations"], "warm_s": w["seconds"],
                      "warm_mean_only_iters": wm["iterations"], "warm_mean_only_s": wm["seconds"],
                      "start": w["start"], "cold_status": c["status"],
                      "warm_status": w["status"]})
        log(f"[warm] eval {k}: kappa {p.kappa:.3f} cold {c['iterations']} it {c['seconds']:.2f}s"
            f" | warm {w['iterations']} it {w['seconds']:.2f}s ({w['start']})"
            f" | mean-only {wm['iterations']} it")
    cold_t = sum(e["cold_s"] for e in evals)
    warm_t = sum(e["warm_s"] for e in evals)
    summary = {"n_train": n_solutions, "seed_base": args.seed_base, "init": args.init,
               "generation": ("multigrid" if args.stream_multigrid or args.multigrid else
                              "warm start" if args.warm_gen else "batched cold"),
               "generation_seconds": gen_s,
               "steps": args.steps, "train_seconds": train_s,
               "loss_first": hist[0], "loss_last": hist[-1], "eval": evals,
               "cold_seconds_total": cold_t, "warm_seconds_total": warm_t,
               "speedup": cold_t / warm_t if warm_t > 0 else None}
    line = json.dumps(summary)
    print(line, flush=True)
    if args.summary:
        with open(args.summary, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
