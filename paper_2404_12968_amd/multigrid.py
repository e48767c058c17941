"""Multigrid warm start (the paper's Algorithm 2, outer procedure).

Levels double the grid from coarse to fine.  Level l (0 = the target grid)
keeps every 2^l-th node of each axis, so a coarse node coincides with a fine
one; its spacing is 2^l h and its prior scale 4^l tau (the discretised SPDE
scales the precision with the cell area), and it sees only the observations
whose locations coincide with its nodes (Section "Multigrid").  Each level is
iterated until its FP64 relative residual reaches a tolerance; the next finer
level starts from the coarse posterior mean, upsampled bilinearly
(`gabp_upsample_mean`) and installed with `gabp_warm_init` -- the paper's
"Upscale Messages", read as initialising the finer grid's marginals to the
coarser grid's, which it states the message copy is equivalent to.  With
`transfer="messages"` (the default) the precision messages are carried over
too, from the covering coarse node in the same direction, scaled by
4^(alpha-1) (`gabp_upscale_precisions`: the prior's off-diagonal entries
shrink by that factor per level); with `transfer="mean"` they start cold on
every level; with `transfer="literal"` every edge value (both components)
is copied unchanged from the covering coarse node, the paper's description
read word for word (`gabp_copy_coarse_messages`).  A coarse level stops either at an FP64 relative residual
(`coarse_stop="residual"`) or by the paper's early-stop rule of Appendix A
(`"message_change"`: mean |m^t - m^(t-1)| below `coarse_tol` times the
level's mean |m^2 - m^1|; the paper takes 1e-3).  The last level is solved to
the problem's own residual tolerance, so the answer is the ordinary fixed
point.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import gabp as G
from . import inputs as I


def level_problem(prob: I.Problem, level: int) -> I.Problem:
    """The problem on the grid of level `level` (every 2^level-th node)."""
    if level == 0:
        return prob
    f = 1 << level
    nx, ny = (prob.nx + f - 1) // f, (prob.ny + f - 1) // f
    if (prob.bc_x == I.BC_PERIODIC and prob.nx % f) or (prob.bc_y == I.BC_PERIODIC and prob.ny % f):
        raise ValueError("periodic axes must be divisible by 2^level")
    cx, cy = prob.cells % prob.nx, prob.cells // prob.nx
    sel = (cx % f == 0) & (cy % f == 0)
    cells = (cy[sel] // f) * nx + cx[sel] // f
    return I.Problem(f"{prob.name}@L{level}", nx, ny, prob.bc_x, prob.bc_y, prob.alpha, prob.kappa,
                     prob.tau * f * f, prob.c, prob.sigma, cells.astype(np.int64), prob.y[sel],
                     hx=prob.hx * f, hy=prob.hy * f,
                     var=None if prob.var is None else prob.var[sel], dtype=prob.dtype,
                     damping=prob.damping, rel_tol=prob.rel_tol, check_every=prob.check_every)


def max_levels(prob: I.Problem, coarsest: int = 32) -> int:
    """Levels until the coarsest side would drop below `coarsest` nodes."""
    L = 1
    while True:
        f = 1 << L
        if min(prob.nx, prob.ny) // f < coarsest:
            return L
        if (prob.bc_x == I.BC_PERIODIC and prob.nx % f) or \
           (prob.bc_y == I.BC_PERIODIC and prob.ny % f):
            return L
        L += 1


def multigrid_solve(prob: I.Problem, levels: Optional[int] = None,
                    coarse_tol: Optional[float] = None, max_iters: int = 300000,
                    check_every: int = -10, device="cuda", keep_context: bool = False,
                    coarse_stop: str = "residual", final_stop: str = "residual",
                    final_tol: Optional[float] = None, transfer: str = "messages",
                    freeze_tolerance: Optional[tuple] = None):
    """Solve coarse-to-fine.  `levels` defaults to halving down to a 32-node
    short side (the paper's base grid); `coarse_tol` defaults to the problem's
    own residual tolerance (1e-3 for the message-change rule).  The target
    level stops at the problem's residual tolerance, or with
    `final_stop="message_change"` by the early-stop rule at `final_tol`
    (default 1e-3), the paper's own setting.  Returns a dict
    with the final status, the iterations and the iteration at which the
    precision messages froze (-1: never) per level (coarsest first), the
    fine-level iterations, the total seconds, and (keep_context) the fine
    context.  freeze_tolerance = (max_slots, max_rel) is passed to every
    level's gabp_set_freeze_tolerance."""
    if coarse_stop not in ("residual", "message_change") or \
            final_stop not in ("residual", "message_change"):
        raise ValueError("coarse_stop and final_stop are 'residual' or 'message_change'")
    if transfer not in ("messages", "mean", "literal"):
        raise ValueError("transfer is 'messages', 'mean' or 'literal'")
    if levels is None:
        levels = max_levels(prob, coarsest=32)
    if coarse_tol is None:
        coarse_tol = prob.rel_tol if coarse_stop == "residual" else 1e-3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred: Optional[torch.Tensor] = None
    per_level: List[dict] = []
    ctx = None
    coarse = None
    st = G.GABP_E_NOT_CONVERGED
    rel = float("inf")
    for lev in reversed(range(levels)):
        p = level_problem(prob, lev)
        ctx = G.gabp_create_problem(p, device=device)
        if freeze_tolerance is not None:
            G.gabp_set_freeze_tolerance(ctx, *freeze_tolerance)
        if coarse is not None:
            G.gabp_copy_coarse_messages(coarse, ctx)
            G.gabp_destroy(coarse)
            coarse = None
        if pred is not None:
            G.gabp_warm_init(ctx, pred, keep_precisions=(transfer == "mean"))
        if lev == 0 and final_stop == "message_change":
            st, it, rel = G.gabp_solve_early_stop(ctx, max_iters, p.damping,
                                                  1e-3 if final_tol is None else final_tol,
                                                  check_every)
        elif lev == 0:
            st, it, rel = G.gabp_solve(ctx, max_iters, p.damping,
                                       prob.rel_tol if final_tol is None else final_tol,
                                       check_every)
        elif coarse_stop == "residual":
            st, it, rel = G.gabp_solve(ctx, max_iters, p.damping, max(coarse_tol, prob.rel_tol),
                                       check_every)
        else:
            st, it, rel = G.gabp_solve_early_stop(ctx, max_iters, p.damping, coarse_tol,
                                                  check_every)
        per_level.append({"level": lev, "nx": p.nx, "ny": p.ny, "iterations": it,
                          "status": st, "rel": rel, "observations": int(p.cells.size),
                          "frozen_at": G.gabp_precision_frozen(ctx)})
        if st == G.GABP_E_DIVERGED:
            break
        if lev > 0 and transfer == "literal":
            coarse = ctx          # its messages are copied into the next level's context
        elif lev > 0:
            mean, _ = G.gabp_posterior(ctx, want_var=False)
            fine = level_problem(prob, lev - 1)
            pred = G.gabp_upsample_mean(mean, p.bc_x, p.bc_y, fine.nx, fine.ny)
            if transfer == "messages":
                G.gabp_upscale_precisions(ctx, pred, 4.0 ** (prob.alpha - 1))
            G.gabp_destroy(ctx)
    torch.cuda.synchronize()
    out = {"status": st, "levels": per_level, "iterations": per_level[-1]["iterations"],
           "seconds": time.perf_counter() - t0, "rel": rel}
    if keep_context:
        out["ctx"] = ctx
    return out


def multigrid_batch_solve(probs: List[I.Problem], levels: Optional[int] = None,
                          max_iters: int = 300000, check_every: int = -10, device="cuda",
                          freeze_tolerance: Optional[tuple] = None, keep_batch: bool = False):
    """Every instance solved coarse to fine as multigrid_solve does (every
    level to the instances' residual tolerance, precision messages carried
    over), one batch per level: the batch of level l holds the instances that
    have a level l (each has max_levels(p) levels, at most `levels`), and each
    of them starts from its own level-(l+1) solution.  The instances must
    share damping and tolerance.  Returns a dict with the final statuses,
    iterations and residuals (input order), per-level instance counts and
    iterations, the total seconds (level set-up and transfers included) and
    (keep_batch) the final batch."""
    n = len(probs)
    damping, rel_tol = probs[0].damping, probs[0].rel_tol
    if any(p.damping != damping or p.rel_tol != rel_tol for p in probs):
        raise ValueError("batch instances must share damping and rel_tol")
    nlev = [max_levels(p, coarsest=32) for p in probs]
    if levels is not None:
        nlev = [min(levels, k) for k in nlev]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    preds: List[Optional[torch.Tensor]] = [None] * n
    per_level: List[dict] = []
    out = None
    for lev in reversed(range(max(nlev))):
        members = [i for i in range(n) if nlev[i] > lev]
        lp = [level_problem(probs[i], lev) for i in members]
        b = G.gabp_batch_create(lp, device=device)
        if freeze_tolerance is not None:
            G.gabp_batch_set_freeze_tolerance(b, *freeze_tolerance)
        for k, i in enumerate(members):
            if preds[i] is not None:
                G.gabp_batch_warm_init(b, k, preds[i], keep_precisions=False)
                preds[i] = None
        st, its, rels, sts = G.gabp_batch_solve(b, max_iters, damping, rel_tol, check_every)
        per_level.append({"level": lev, "instances": len(members),
                          "iterations": [int(v) for v in its],
                          "status": [int(v) for v in sts]})
        if lev > 0:
            for k, i in enumerate(members):
                if sts[k] == G.GABP_E_DIVERGED:
                    continue             # the next level starts cold
                mean, _ = G.gabp_batch_posterior(b, k, want_var=False)
                fine = level_problem(probs[i], lev - 1)
                pred = G.gabp_upsample_mean(mean, lp[k].bc_x, lp[k].bc_y, fine.nx, fine.ny)
                G.gabp_batch_upscale_precisions(b, k, pred, 4.0 ** (probs[i].alpha - 1))
                preds[i] = pred
            torch.cuda.synchronize()
            G.gabp_batch_destroy(b)
        else:
            out = {"status": st, "statuses": sts, "iterations": its, "rel": rels, "batch": b}
    torch.cuda.synchronize()
    res = {"status": out["status"], "statuses": out["statuses"], "iterations": out["iterations"],
           "rel": out["rel"], "levels": per_level, "seconds": time.perf_counter() - t0}
    if keep_batch:
        res["batch"] = out["batch"]
    else:
        G.gabp_batch_destroy(out["batch"])
    return res


# --------------------------------------------------------------------------
# space-time lattice (the heat-equation GMRF of include/gabp_st.h)
# --------------------------------------------------------------------------

def st_level_problem(prob: I.SpaceTimeProblem, level: int) -> I.SpaceTimeProblem:
    """Level l keeps every 2^l-th node of x, y and t: the same heat equation
    discretised with spacing 2^l h and time step 2^l dt, and the
    observations whose space-time cell coincides with a level node.  The
    initial condition's factor is scaled by 2^(-l/2): the initial slice's
    precision (dt h^2 / sigma_u^2) (a0 L)^2 carries the time step, and this
    keeps the initial field's distribution the same on every level (a CPU
    test checks that a smooth field's prior energy agrees across levels)."""
    if level == 0:
        return prob
    f = 2 ** level
    if (prob.bc_x == I.BC_PERIODIC and prob.nx % f) or (prob.bc_y == I.BC_PERIODIC and prob.ny % f):
        raise ValueError("a periodic axis must be divisible by 2^level")
    nx, ny, nt = (prob.nx + f - 1) // f, (prob.ny + f - 1) // f, (prob.nt + f - 1) // f
    t, r = np.divmod(prob.cells, prob.nx * prob.ny)
    y, x = np.divmod(r, prob.nx)
    keep = (x % f == 0) & (y % f == 0) & (t % f == 0)
    cells = (t[keep] // f) * (nx * ny) + (y[keep] // f) * nx + x[keep] // f
    return dataclasses.replace(
        prob, name=f"{prob.name}/level{level}", nx=nx, ny=ny, nt=nt, dt=prob.dt * f,
        h=prob.h * f, a0=prob.a0 / np.sqrt(f), cells=cells, y=prob.y[keep],
        var=None if prob.var is None else np.asarray(prob.var)[keep], truth=None)


def st_max_levels(prob: I.SpaceTimeProblem, coarsest: int = 32) -> int:
    """Levels halving x, y and t while the short spatial side stays >= coarsest,
    every slice count >= 2, and periodic axes divide evenly."""
    L = 1
    while True:
        f = 2 ** L
        if min(prob.nx, prob.ny) // f < coarsest or (prob.nt + f - 1) // f < 2:
            return L
        if (prob.bc_x == I.BC_PERIODIC and prob.nx % f) or (prob.bc_y == I.BC_PERIODIC and prob.ny % f):
            return L
        L += 1


def st_multigrid_solve(prob: I.SpaceTimeProblem, levels: Optional[int] = None,
                       max_iters: int = 300000, check_every: int = 50, device="cuda",
                       keep_context: bool = False, freeze_tolerance: Optional[tuple] = (64, 1e-6),
                       coarse_tol: Optional[float] = None) -> dict:
    """Coarse-to-fine on the space-time lattice: each level solved to its
    FP64 relative residual (coarse_tol on the coarse levels, default the
    problem's own), then its mean upsampled trilinearly
    (`gabp_st_upsample_mean`) and installed in the next finer level with
    `gabp_st_warm_init`.  Returns the status, per-level iterations, the fine
    iterations, the seconds and (keep_context) the fine context."""
    if levels is None:
        levels = st_max_levels(prob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = None
    per_level: List[dict] = []
    ctx = None
    st, rel = G.GABP_E_NOT_CONVERGED, float("inf")
    for lev in reversed(range(levels)):
        p = st_level_problem(prob, lev)
        ctx = G.gabp_st_create_problem(p, device=device)
        if freeze_tolerance is not None:
            G.gabp_st_set_freeze_tolerance(ctx, *freeze_tolerance)
        if pred is not None:
            G.gabp_st_warm_init(ctx, pred)
        tol = prob.rel_tol if lev == 0 or coarse_tol is None else max(coarse_tol, prob.rel_tol)
        st, it, rel = G.gabp_st_solve(ctx, max_iters, p.damping, tol, check_every)
        per_level.append({"level": lev, "nx": p.nx, "ny": p.ny, "nt": p.nt, "iterations": it,
                          "status": st, "rel": rel, "observations": int(p.cells.size)})
        if st == G.GABP_E_DIVERGED:
            break
        if lev > 0:
            mean, _ = G.gabp_st_posterior(ctx, want_var=False)
            fine = st_level_problem(prob, lev - 1)
            pred = G.gabp_st_upsample_mean(mean, p.bc_x, p.bc_y, fine.nx, fine.ny, fine.nt)
            G.gabp_st_destroy(ctx)
    torch.cuda.synchronize()
    out = {"status": st, "levels": per_level, "iterations": per_level[-1]["iterations"],
           "seconds": time.perf_counter() - t0, "rel": rel}
    if keep_context:
        out["ctx"] = ctx
    return out
