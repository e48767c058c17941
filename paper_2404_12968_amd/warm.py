"""Learned warm start for the lattice solver.

A 6-layer 3x3 convolutional network with 32 hidden channels maps the
observation features of a problem (mask, observed values, log kappa) to a
prediction of the posterior mean and of the log(-precision) of every
sender-indexed message; ``gabp_warm_init`` turns the prediction into a
starting state and the ordinary solver iterates from there, so the FP64
residual test still decides convergence and cold start remains the fallback.

The network is trained on solutions the solver itself computed (batched
solves of seeded problems of the warm-start workload).  Every numeric step
-- convolutions forward and backward (BF16 matrix-core kernels, FP32
accumulation), loss, Adam -- runs in the library's kernels; this module only
orchestrates them and slices tensors.

Layers: dilations 1, 3, 9, 27, 9, 1 (with 3x3 kernels the first four cover
every offset up to +-40 cells exactly once; the whole stack sees +-50 cells),
channels 16 (3 used) -> 32 x 5 -> 16 (13 used), ReLU on all but the last.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import gabp as G
from . import inputs as I

DILATIONS = (1, 3, 9, 27, 9, 1)
CIN = (16, 32, 32, 32, 32, 32)
COUT = (32, 32, 32, 32, 32, 16)
RELU = (1, 1, 1, 1, 1, 0)
NDIR = 12
DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (2, 0), (-2, 0), (0, 2), (0, -2),
        (1, 1), (-1, -1), (1, -1), (-1, 1)]


class WarmNet:
    """Weights (FP32 masters + BF16 copies) and Adam state of the network."""

    def __init__(self, device="cuda", seed: int = 0):
        self.device = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        self.w: List[torch.Tensor] = []
        self.b: List[torch.Tensor] = []
        for l in range(len(DILATIONS)):
            fan_in = 9 * CIN[l]
            std = math.sqrt(2.0 / fan_in) if RELU[l] else math.sqrt(1.0 / fan_in)
            w = torch.zeros(32, 9 * CIN[l])
            w[: COUT[l]] = torch.randn(COUT[l], 9 * CIN[l], generator=g) * std
            self.w.append(w.to(self.device))
            self.b.append(torch.zeros(32, device=self.device))
        self.wb = [w.to(torch.bfloat16) for w in self.w]
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.step = 0
        self._ws = None

    # -- inference ---------------------------------------------------------
    def forward(self, x: torch.Tensor):
        """x: bf16 [B,H,W,16] -> (activations, pred FP32 [B,H,W,16])."""
        acts = [x]
        pred = None
        for l in range(len(DILATIONS)):
            last = l == len(DILATIONS) - 1
            yb, yf = G.gabp_conv3x3_fwd(acts[-1], self.wb[l], self.b[l], COUT[l], DILATIONS[l],
                                        bool(RELU[l]), want_bf16=True, want_f32=last)
            acts.append(yb)
            if last:
                pred = yf
        return acts, pred

    # -- training ----------------------------------------------------------
    def backward(self, acts, grad):
        """Gradients (dw, db) of every layer from the loss gradient (FP32)."""
        dws, dbs = [None] * len(DILATIONS), [None] * len(DILATIONS)
        dy = grad
        for l in reversed(range(len(DILATIONS))):
            dw, db, dx, self._ws = G.gabp_conv3x3_bwd(acts[l], acts[l + 1], dy, self.wb[l],
                                                      COUT[l], DILATIONS[l], bool(RELU[l]),
                                                      need_dx=l > 0, workspace=self._ws)
            dws[l], dbs[l] = dw, db
            dy = dx
        return dws, dbs

    def adam(self, dws, dbs, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        L = len(DILATIONS)
        for l in range(L):
            G.gabp_adam_step(self.w[l], dws[l], self.m[l], self.v[l], self.wb[l], lr, beta1, beta2,
                             eps, self.step)
            G.gabp_adam_step(self.b[l], dbs[l], self.m[L + l], self.v[L + l], None, lr, beta1,
                             beta2, eps, self.step)

    # -- persistence -------------------------------------------------------
    def save(self, path: str, meta: Optional[Dict] = None) -> None:
        arrs = {f"w{l}": self.w[l].cpu().numpy() for l in range(len(DILATIONS))}
        arrs.update({f"b{l}": self.b[l].cpu().numpy() for l in range(len(DILATIONS))})
        arrs["dilations"] = np.array(DILATIONS)
        if meta:
            arrs["meta"] = np.array(repr(meta))
        np.savez(path, **arrs)

    @classmethod
    def load(cls, path: str, device="cuda") -> "WarmNet":
        net = cls(device)
        with np.load(path, allow_pickle=False) as z:
            if tuple(z["dilations"]) != DILATIONS:
                raise ValueError("weights are for another architecture")
            for l in range(len(DILATIONS)):
                net.w[l] = torch.tensor(z[f"w{l}"], device=net.device)
                net.b[l] = torch.tensor(z[f"b{l}"], device=net.device)
        net.wb = [w.to(torch.bfloat16) for w in net.w]
        return net


# --------------------------------------------------------------------------
# training data: the solver's own solutions
# --------------------------------------------------------------------------

class TrainingSet:
    """Solutions of many problems, resident on the GPU in compact form: each
    problem's observations (cells, values, kappa: the network input is
    rebuilt from them by gabp_warm_features when a batch is drawn) and its
    FP32 posterior mean; for some problems also the log(-Lam) targets of the
    precision outputs (gabp_log_precisions), whose edge masks are shared by
    problems of one grid."""

    def __init__(self):
        self.cells: List[torch.Tensor] = []    # int64 device
        self.y: List[torch.Tensor] = []        # float64 device
        self.kappa: List[float] = []
        self.shape: List[tuple] = []           # (ny, nx)
        self.mu: List[torch.Tensor] = []       # fp32 [ny, nx]
        self.lam: List[Optional[torch.Tensor]] = []   # fp32 [12, ny, nx] or None
        self.valid: Dict[tuple, torch.Tensor] = {}    # (ny, nx, bc_x, bc_y) -> [12, ny, nx]
        self.key: List[tuple] = []
        self.iters: List[int] = []

    def __len__(self):
        return len(self.mu)

    def add(self, p: I.Problem, mu: torch.Tensor, lam: Optional[torch.Tensor],
            valid: Optional[torch.Tensor], iters: int, device) -> None:
        key = (p.ny, p.nx, p.bc_x, p.bc_y)
        if valid is not None and key not in self.valid:
            self.valid[key] = valid
        self.cells.append(torch.as_tensor(np.asarray(p.cells), dtype=torch.int64).to(device))
        self.y.append(torch.as_tensor(np.asarray(p.y), dtype=torch.float64).to(device))
        self.kappa.append(float(p.kappa))
        self.shape.append((p.ny, p.nx))
        self.mu.append(mu.to(torch.float32).reshape(p.ny, p.nx))
        self.lam.append(lam)
        self.key.append(key)
        self.iters.append(int(iters))

    def features(self, k: int) -> torch.Tensor:
        ny, nx = self.shape[k]
        return G.gabp_warm_features(self.cells[k], self.y[k], nx, ny, self.kappa[k],
                                    device=self.mu[k].device)


def solve_training_set(problems: Sequence[I.Problem], max_iters: int = 300000,
                       rel_tol: float = 1e-6, device="cuda", log=print,
                       multigrid: bool = False, lam_targets: bool = True,
                       ts: Optional[TrainingSet] = None) -> TrainingSet:
    """Solve the problems with the batched solver (multigrid: batched
    coarse-to-fine, the same fixed points at the same residual tolerance) and
    keep the solutions."""
    ts = TrainingSet() if ts is None else ts
    t0 = time.time()
    if multigrid:
        from . import multigrid as MG
        probs = list(problems)
        for p in probs:
            p.rel_tol = rel_tol
        res = MG.multigrid_batch_solve(probs, max_iters=max_iters, device=device,
                                       keep_batch=True)
        b, its, sts = res["batch"], np.asarray(res["iterations"]), np.asarray(res["statuses"])
    else:
        b = G.gabp_batch_create(list(problems), device=device)
        st, its, rels, sts = G.gabp_batch_solve(b, max_iters, 0.5, rel_tol, -10)
    torch.cuda.synchronize()
    log(f"[warm] solved {len(problems)} problems in {time.time() - t0:.1f}s: "
        f"{int((sts == G.GABP_OK).sum())} converged, iterations median {int(np.median(its))}")
    for i, p in enumerate(problems):
        if sts[i] != G.GABP_OK:
            continue
        mean, _ = G.gabp_batch_posterior(b, i, want_var=False)
        lam, valid = G.gabp_batch_log_precisions(b, i) if lam_targets else (None, None)
        ts.add(p, mean, lam, valid, its[i], device)
    del b
    torch.cuda.synchronize()
    return ts


def solve_training_set_warm(net: "WarmNet", problems: Sequence[I.Problem],
                            max_iters: int = 300000, rel_tol: float = 1e-6, device="cuda",
                            log=print, lam_targets: int = 0,
                            freeze_tolerance: Optional[tuple] = (64, 1e-6),
                            ts: Optional[TrainingSet] = None, deadline: Optional[float] = None,
                            log_every: int = 256) -> TrainingSet:
    """Solve each problem from the network's warm start (cold where that
    start diverges) to the residual tolerance and keep the solutions: the
    fixed point does not depend on the start, so a network can generate the
    data its successor trains on.  The first `lam_targets` solutions keep
    their precision targets.  Stops early at time.time() >= deadline."""
    ts = TrainingSet() if ts is None else ts
    t0 = time.time()
    its_all = []
    for k, p in enumerate(problems):
        if deadline is not None and time.time() >= deadline:
            log(f"[warm] generation deadline reached after {k} problems")
            break
        p.rel_tol = rel_tol
        pred = predict(net, p, device)
        ctx = G.gabp_create_problem(p, device=device)
        G.gabp_warm_init(ctx, pred)
        if freeze_tolerance is not None:
            G.gabp_set_freeze_tolerance(ctx, *freeze_tolerance)
        st, it, rel = G.gabp_solve(ctx, max_iters, p.damping, rel_tol, -10)
        if st == G.GABP_E_DIVERGED:
            G.gabp_destroy(ctx)
            ctx = G.gabp_create_problem(p, device=device)
            if freeze_tolerance is not None:
                G.gabp_set_freeze_tolerance(ctx, *freeze_tolerance)
            st, it, rel = G.gabp_solve(ctx, max_iters, p.damping, rel_tol, -10)
        if st == G.GABP_OK:
            mean, _ = G.gabp_posterior(ctx, want_var=False)
            want = len(ts) < lam_targets
            lam, valid = G.gabp_log_precisions(ctx) if want else (None, None)
            if not want and (p.ny, p.nx, p.bc_x, p.bc_y) not in ts.valid:
                _, valid = G.gabp_log_precisions(ctx)
            ts.add(p, mean, lam, valid, it, device)
            its_all.append(it)
        G.gabp_destroy(ctx)
        if (k + 1) % log_every == 0:
            log(f"[warm] {k + 1} problems in {time.time() - t0:.1f}s, iterations median "
                f"{int(np.median(its_all)) if its_all else -1}")
    torch.cuda.synchronize()
    return ts


def solve_training_set_multigrid(problems, rel_tol: float = 1e-6, device="cuda", log=print,
                                 lam_targets: int = 0,
                                 freeze_tolerance: Optional[tuple] = (64, 1e-6),
                                 ts: Optional[TrainingSet] = None,
                                 deadline: Optional[float] = None,
                                 log_every: int = 128) -> TrainingSet:
    """Solve each problem by multigrid (coarse levels carry the smooth modes
    that single-grid iterations leave far from converged at a given
    residual) and keep the solutions; problems may be an iterator.  The first
    `lam_targets` solutions keep their precision targets.  Stops early at
    time.time() >= deadline."""
    from . import multigrid as MG
    ts = TrainingSet() if ts is None else ts
    t0 = time.time()
    its_all = []
    for k, p in enumerate(problems):
        if deadline is not None and time.time() >= deadline:
            log(f"[warm] generation deadline reached after {k} problems")
            break
        p.rel_tol = rel_tol
        r = MG.multigrid_solve(p, keep_context=True, freeze_tolerance=freeze_tolerance,
                               device=device)
        ctx = r["ctx"]
        if r["status"] == G.GABP_OK:
            mean, _ = G.gabp_posterior(ctx, want_var=False)
            want = len(ts) < lam_targets
            lam, valid = G.gabp_log_precisions(ctx) if want else (None, None)
            if not want and (p.ny, p.nx, p.bc_x, p.bc_y) not in ts.valid:
                _, valid = G.gabp_log_precisions(ctx)
            ts.add(p, mean, lam, valid, r["iterations"], device)
            its_all.append(r["iterations"])
        G.gabp_destroy(ctx)
        if (k + 1) % log_every == 0:
            log(f"[warm] {k + 1} problems in {time.time() - t0:.1f}s, fine iterations median "
                f"{int(np.median(its_all)) if its_all else -1}")
    torch.cuda.synchronize()
    return ts


def train(net: WarmNet, ts: TrainingSet, steps: int, batch: int = 8, crop: int = 256,
          lr: float = 2e-3, lam_weight: float = 0.1, seed: int = 0, log=print,
          log_every: int = 100) -> List[float]:
    """Adam on random crops of the training set; returns the loss history.
    Crops of problems without precision targets carry no precision loss."""
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.time()
    zeros = {}
    for s in range(steps):
        xs, mus, lams, vals = [], [], [], []
        for _ in range(batch):
            k = int(rng.integers(0, len(ts)))
            ny, nx = ts.shape[k]
            cy = int(rng.integers(0, ny - crop + 1)) if ny > crop else 0
            cx = int(rng.integers(0, nx - crop + 1)) if nx > crop else 0
            h, w = min(crop, ny), min(crop, nx)
            xs.append(ts.features(k)[cy:cy + h, cx:cx + w])
            mus.append(ts.mu[k][cy:cy + h, cx:cx + w])
            if ts.lam[k] is not None:
                lams.append(ts.lam[k][:, cy:cy + h, cx:cx + w])
                vals.append(ts.valid[ts.key[k]][:, cy:cy + h, cx:cx + w])
            else:
                z = zeros.get((h, w))
                if z is None:
                    z = zeros[(h, w)] = torch.zeros((NDIR, h, w), dtype=torch.float32,
                                                    device=ts.mu[k].device)
                lams.append(z)
                vals.append(z)
        x = torch.stack(xs).contiguous()
        mu = torch.stack(mus).contiguous()
        # direction-major targets [12, B*h*w] to match the kernel's layout
        lam = torch.stack(lams, dim=1).reshape(NDIR, -1).contiguous()
        val = torch.stack(vals, dim=1).reshape(NDIR, -1).contiguous()
        acts, pred = net.forward(x)
        loss, grad = G.gabp_warm_loss(pred, mu.reshape(-1), lam, val, NDIR, lam_weight)
        dws, dbs = net.backward(acts, grad)
        cur = lr * 0.5 * (1 + math.cos(math.pi * s / max(1, steps)))
        net.adam(dws, dbs, cur)
        if s % log_every == 0 or s == steps - 1:
            lv = float(loss)
            hist.append(lv)
            log(f"[warm] step {s} loss {lv:.5f} lr {cur:.2e} ({time.time() - t0:.1f}s)")
    return hist


def predict(net: WarmNet, prob: I.Problem, device="cuda") -> torch.Tensor:
    """Prediction [ny, nx, 16] FP32 for one problem."""
    x = G.gabp_warm_features(prob.cells, prob.y, prob.nx, prob.ny, prob.kappa, device=device)
    _, pred = net.forward(x.unsqueeze(0).contiguous())
    return pred[0].contiguous()


def warm_solve(net: WarmNet, prob: I.Problem, max_iters: int = 300000, probe: int = 100,
               device="cuda", use_precisions: bool = True,
               freeze_tolerance: Optional[tuple] = None, keep_mean: bool = False):
    """Solve from the network's warm start; cold start is the fallback: after
    `probe` iterations the warm run's residual is compared with a cold run's
    at the same iteration, and the worse of the two is dropped.  Returns a
    dict with status, iterations, seconds (including inference) and which
    start won (keep_mean: and the FP64 posterior mean).  freeze_tolerance =
    (max_slots, max_rel) is given to both contexts' gabp_set_freeze_tolerance
    (a warm start's precision messages may settle into last-bit flips that the
    bitwise freeze never accepts)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = predict(net, prob, device)
    warm = G.gabp_create_problem(prob, device=device)
    G.gabp_warm_init(warm, pred, keep_precisions=not use_precisions)
    cold = G.gabp_create_problem(prob, device=device)
    if freeze_tolerance is not None:
        G.gabp_set_freeze_tolerance(warm, *freeze_tolerance)
        G.gabp_set_freeze_tolerance(cold, *freeze_tolerance)
    G.gabp_iterate(cold, probe, prob.damping)
    rc, _ = G.gabp_residual(cold)
    try:
        G.gabp_iterate(warm, probe, prob.damping)
        rw, _ = G.gabp_residual(warm)
    except G.GabpError as e:
        # a prediction that makes a cavity precision non-positive diverges at
        # once: the cold start takes over
        if e.status != G.GABP_E_DIVERGED:
            raise
        rw = math.inf
    if rw <= rc:
        ctx, which = warm, "warm"
        G.gabp_destroy(cold)
    else:
        ctx, which = cold, "cold"
        G.gabp_destroy(warm)
    st, it, rel = G.gabp_solve(ctx, max_iters - probe, prob.damping, prob.rel_tol,
                               prob.check_every)
    torch.cuda.synchronize()
    out = {"status": st, "iterations": it, "seconds": time.perf_counter() - t0,
           "rel": rel, "start": which, "probe_residual_warm": rw, "probe_residual_cold": rc,
           "frozen_at": G.gabp_precision_frozen(ctx)}
    if keep_mean:
        out["mean"] = G.gabp_posterior(ctx, want_var=False)[0]
    G.gabp_destroy(ctx)
    return out


def cold_solve(prob: I.Problem, max_iters: int = 300000, device="cuda",
               freeze_tolerance: Optional[tuple] = None, keep_mean: bool = False):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = G.gabp_create_problem(prob, device=device)
    if freeze_tolerance is not None:
        G.gabp_set_freeze_tolerance(ctx, *freeze_tolerance)
    st, it, rel = G.gabp_solve(ctx, max_iters, prob.damping, prob.rel_tol, prob.check_every)
    torch.cuda.synchronize()
    out = {"status": st, "iterations": it, "seconds": time.perf_counter() - t0, "rel": rel,
           "frozen_at": G.gabp_precision_frozen(ctx)}
    if keep_mean:
        out["mean"] = G.gabp_posterior(ctx, want_var=False)[0]
    G.gabp_destroy(ctx)
    return out
