"""Thin Python binding of the gfx950 library ``libgabp.so`` (C ABI in include/gabp.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  PyTorch provides device memory (workspace, outputs,
observation arrays) and the stream.  There is no CPU fallback: importing
this module without the built library raises ImportError.

The functions carry the C names.  Non-OK statuses raise ``GabpError``, except
that ``gabp_solve`` returns DIVERGED / NOT_CONVERGED as its first result.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgabp.so")

GABP_OK, GABP_E_INVALID, GABP_E_NOMEM, GABP_E_DEVICE, GABP_E_DIVERGED, GABP_E_NOT_CONVERGED = range(6)
GABP_BC_NEUMANN, GABP_BC_PERIODIC, GABP_BC_DIRICHLET = 0, 1, 2
GABP_F32, GABP_F64 = 0, 1
DTYPES = {"f32": GABP_F32, "f64": GABP_F64}
TORCH_DTYPES = {GABP_F32: torch.float32, GABP_F64: torch.float64}


class gabp_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("hx", ctypes.c_double),
                ("hy", ctypes.c_double), ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class gabp_stencil(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int32), ("kappa", ctypes.c_double), ("tau", ctypes.c_double),
                ("c", ctypes.c_double)]


class gabp_obs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cell", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("on_device", ctypes.c_int32)]


class gabp_noise(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("var", ctypes.c_void_p)]


class gabp_opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("prior_mean", ctypes.c_void_p)]


class gabp_st_model(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("dt", ctypes.c_double),
                ("h", ctypes.c_double), ("nu", ctypes.c_double), ("kappa", ctypes.c_double),
                ("a0", ctypes.c_double), ("sigma_u", ctypes.c_double), ("c", ctypes.c_double)]


class gabp_instance(ctypes.Structure):
    _fields_ = [("grid", gabp_grid), ("stencil", gabp_stencil), ("obs", gabp_obs),
                ("noise", gabp_noise)]


# name -> (argtypes, restype), mirroring include/gabp.h
_P = ctypes.c_void_p
_SIGS = {
    "gabp_workspace_size": ([_P, _P, ctypes.c_int32, _P], ctypes.c_int),
    "gabp_create": ([_P, _P, _P, _P, _P, _P], ctypes.c_int),
    "gabp_iterate": ([_P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "gabp_solve": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P, _P],
                   ctypes.c_int),
    "gabp_residual": ([_P, _P, _P], ctypes.c_int),
    "gabp_posterior": ([_P, _P, _P], ctypes.c_int),
    "gabp_message_change": ([_P, _P], ctypes.c_int),
    "gabp_get_messages": ([_P, _P, _P], ctypes.c_int),
    "gabp_set_messages": ([_P, _P, _P], ctypes.c_int),
    "gabp_iteration_count": ([_P, _P], ctypes.c_int),
    "gabp_autotune": ([_P, ctypes.c_int32, ctypes.c_double, _P], ctypes.c_int),
    "gabp_precision_frozen": ([_P, _P], ctypes.c_int),
    "gabp_num_directions": ([_P], ctypes.c_int32),
    "gabp_destroy": ([_P], None),
    "gabp_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "gabp_last_error": ([_P], ctypes.c_char_p),
    "gabp_batch_workspace_size": ([ctypes.c_int32, _P, ctypes.c_int32, _P], ctypes.c_int),
    "gabp_batch_create": ([ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "gabp_batch_iterate": ([_P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "gabp_batch_solve": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                          _P, _P, _P], ctypes.c_int),
    "gabp_batch_posterior": ([_P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gabp_batch_get_messages": ([_P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gabp_batch_autotune": ([_P, ctypes.c_int32, ctypes.c_double, _P], ctypes.c_int),
    "gabp_batch_info": ([_P, ctypes.c_int32, _P, _P, _P], ctypes.c_int),
    "gabp_batch_destroy": ([_P], None),
    "gabp_batch_last_error": ([_P], ctypes.c_char_p),
    "gabp_warm_init": ([_P, _P, ctypes.c_int32], ctypes.c_int),
    "gabp_solve_early_stop": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32, _P, _P], ctypes.c_int),
    "gabp_set_graph": ([_P, ctypes.c_int32], ctypes.c_int),
    "gabp_set_tile": ([_P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
    "gabp_launch_counts": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "gabp_log_precisions": ([_P, _P, _P], ctypes.c_int),
    "gabp_batch_log_precisions": ([_P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gabp_set_freeze_tolerance": ([_P, ctypes.c_int64, ctypes.c_double], ctypes.c_int),
    "gabp_batch_set_freeze_tolerance": ([_P, ctypes.c_int64, ctypes.c_double], ctypes.c_int),
    "gabp_batch_warm_init": ([_P, ctypes.c_int32, _P, ctypes.c_int32], ctypes.c_int),
    "gabp_batch_upscale_precisions": ([_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_double], ctypes.c_int),
    "gabp_get_tile": ([_P, _P, _P], ctypes.c_int),
    "gabp_copy_coarse_messages": ([_P, _P], ctypes.c_int),
    "gabp_upscale_precisions": ([_P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_double],
                                ctypes.c_int),
    "gabp_upsample_mean": ([_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                            _P, ctypes.c_int64, ctypes.c_int64, _P], ctypes.c_int),
    "gabp_conv3x3_fwd": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                          _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P, _P],
                         ctypes.c_int),
    "gabp_conv3x3_bwd_workspace": ([ctypes.c_int32] * 5, ctypes.c_size_t),
    "gabp_conv3x3_bwd": ([_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "gabp_adam_step": ([_P, _P, _P, _P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                        ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P], ctypes.c_int),
    "gabp_warm_loss": ([_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _P, _P,
                        _P, _P], ctypes.c_int),
    "gabp_warm_features_noalloc": ([ctypes.c_int64, _P, _P, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_double, _P, _P], ctypes.c_int),
    "gabp_warm_features": ([ctypes.c_int64, _P, _P, ctypes.c_int64, ctypes.c_int64,
                            ctypes.c_double, _P, _P, _P], ctypes.c_int),
    "gabp_net_last_error": ([], ctypes.c_char_p),
    # space-time solver, include/gabp_st.h
    "gabp_st_workspace_size": ([_P, ctypes.c_int32, _P], ctypes.c_int),
    "gabp_st_create": ([_P, _P, _P, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "gabp_st_create_error": ([], ctypes.c_char_p),
    "gabp_st_iterate": ([_P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "gabp_st_residual": ([_P, _P, _P], ctypes.c_int),
    "gabp_st_solve": ([_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                       _P, _P], ctypes.c_int),
    "gabp_st_posterior": ([_P, _P, _P], ctypes.c_int),
    "gabp_st_get_messages": ([_P, _P, _P], ctypes.c_int),
    "gabp_st_iteration_count": ([_P, _P, _P], ctypes.c_int),
    "gabp_st_set_freeze_tolerance": ([_P, ctypes.c_int64, ctypes.c_double], ctypes.c_int),
    "gabp_st_precision_frozen": ([_P, _P], ctypes.c_int),
    "gabp_st_set_theta_slices": ([_P, ctypes.c_int32], ctypes.c_int),
    "gabp_st_upsample_mean": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_int32, _P], ctypes.c_int),
    "gabp_st_warm_init": ([_P, _P], ctypes.c_int),
    "gabp_st_last_error": ([_P], ctypes.c_char_p),
    "gabp_st_destroy": ([_P], None),
}

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built: run `python -m paper_2404_12968_amd.build`")
_lib = ctypes.CDLL(_LIB_PATH)
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

LIBRARY_PATH = _LIB_PATH
EXPORTED = tuple(_SIGS)


class GabpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{gabp_status_string(status)}: {message}")
        self.status = status


class Context:
    """A live gabp_ctx plus the torch buffers it uses (kept alive here)."""

    def __init__(self, handle, workspace, stream, nx, ny, dtype, device):
        self.handle = handle
        self.workspace = workspace
        self.stream = stream
        self.nx, self.ny = nx, ny
        self.dtype = dtype
        self.device = device

    @property
    def deg(self) -> int:
        return int(_lib.gabp_num_directions(self.handle))

    def __del__(self):
        try:
            gabp_destroy(self)
        except Exception:
            pass


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(st: int, ctx: Optional[Context] = None):
    if st != GABP_OK:
        raise GabpError(st, gabp_last_error(ctx))


def gabp_status_string(status: int) -> str:
    return _lib.gabp_status_string(int(status)).decode()


def gabp_last_error(ctx: Optional[Context] = None) -> str:
    h = ctx.handle if ctx is not None else None
    return _lib.gabp_last_error(h).decode()


def _grid(nx, ny, hx=1.0, hy=1.0, bc_x=0, bc_y=0):
    return gabp_grid(int(nx), int(ny), float(hx), float(hy), int(bc_x), int(bc_y))


def _stencil(alpha, kappa, tau, c):
    return gabp_stencil(int(alpha), float(kappa), float(tau), float(c))


def gabp_workspace_size(grid: gabp_grid, stencil: gabp_stencil, dtype: int) -> int:
    n = ctypes.c_size_t(0)
    _check(_lib.gabp_workspace_size(ctypes.byref(grid), ctypes.byref(stencil), int(dtype),
                                    ctypes.byref(n)))
    return int(n.value)


def gabp_create(grid: gabp_grid, stencil: gabp_stencil, cells: torch.Tensor, y: torch.Tensor,
                sigma: float, var: Optional[torch.Tensor] = None, dtype: int = GABP_F32,
                prior_mean: Optional[torch.Tensor] = None, stream=None,
                device: Optional[torch.device] = None) -> Context:
    """Create a context.  cells (int64) and y (float64) are CUDA tensors (or
    numpy arrays, copied to the device here); workspace comes from torch."""
    device = torch.device(device or "cuda")
    cells = torch.as_tensor(np.asarray(cells) if not torch.is_tensor(cells) else cells,
                            dtype=torch.int64).to(device).contiguous()
    y = torch.as_tensor(np.asarray(y) if not torch.is_tensor(y) else y,
                        dtype=torch.float64).to(device).contiguous()
    if var is not None:
        var = torch.as_tensor(var, dtype=torch.float64).to(device).contiguous()
    if prior_mean is not None:
        prior_mean = torch.as_tensor(prior_mean, dtype=torch.float64).to(device).contiguous()
    nbytes = gabp_workspace_size(grid, stencil, dtype)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    obs = gabp_obs(int(cells.numel()), cells.data_ptr() if cells.numel() else None,
                   y.data_ptr() if y.numel() else None, 1)
    noise = gabp_noise(float(sigma), None if var is None else var.data_ptr())
    opts = gabp_opts(int(dtype), stream.cuda_stream, ws.data_ptr(), nbytes,
                     None if prior_mean is None else prior_mean.data_ptr())
    h = ctypes.c_void_p()
    _check(_lib.gabp_create(ctypes.byref(grid), ctypes.byref(stencil), ctypes.byref(obs),
                            ctypes.byref(noise), ctypes.byref(opts), ctypes.byref(h)))
    return Context(h, ws, stream, grid.nx, grid.ny, int(dtype), device)


def gabp_create_problem(prob, dtype: Optional[str] = None, stream=None, device=None,
                        prior_mean=None) -> Context:
    """gabp_create with the arguments taken from an ``inputs.Problem``."""
    dt = DTYPES[dtype or prob.dtype]
    return gabp_create(_grid(prob.nx, prob.ny, prob.hx, prob.hy, prob.bc_x, prob.bc_y),
                       _stencil(prob.alpha, prob.kappa, prob.tau, prob.c),
                       prob.cells, prob.y, prob.sigma, var=prob.var, dtype=dt,
                       prior_mean=prior_mean, stream=stream, device=device)


def gabp_iterate(ctx: Context, n_iters: int, damping: float) -> None:
    _check(_lib.gabp_iterate(ctx.handle, int(n_iters), float(damping)), ctx)


def gabp_solve(ctx: Context, max_iters: int, damping: float, rel_tol: float,
               check_every: int = 10) -> Tuple[int, int, float]:
    """Returns (status, total iterations, last relative residual)."""
    it = ctypes.c_int64(0)
    rel = ctypes.c_double(0.0)
    st = _lib.gabp_solve(ctx.handle, int(max_iters), float(damping), float(rel_tol),
                         int(check_every), ctypes.byref(it), ctypes.byref(rel))
    if st not in (GABP_OK, GABP_E_DIVERGED, GABP_E_NOT_CONVERGED):
        _check(st, ctx)
    return int(st), int(it.value), float(rel.value)


def gabp_solve_early_stop(ctx: Context, max_iters: int, damping: float, tau: float = 1e-3,
                          check_every: int = -10) -> Tuple[int, int, float]:
    """The paper's early-stop rule; returns (status, total iterations, last
    message-change ratio)."""
    it = ctypes.c_int64(0)
    r = ctypes.c_double(0.0)
    st = _lib.gabp_solve_early_stop(ctx.handle, int(max_iters), float(damping), float(tau),
                                    int(check_every), ctypes.byref(it), ctypes.byref(r))
    if st not in (GABP_OK, GABP_E_DIVERGED, GABP_E_NOT_CONVERGED):
        _check(st, ctx)
    return int(st), int(it.value), float(r.value)


def gabp_residual(ctx: Context) -> Tuple[float, float]:
    rel = ctypes.c_double(0.0)
    ab = ctypes.c_double(0.0)
    _check(_lib.gabp_residual(ctx.handle, ctypes.byref(rel), ctypes.byref(ab)), ctx)
    return float(rel.value), float(ab.value)


def gabp_posterior(ctx: Context, mean: Optional[torch.Tensor] = None,
                   var: Optional[torch.Tensor] = None, want_var: bool = True):
    """Posterior mean and variance as (ny, nx) float64 device tensors."""
    if mean is None:
        mean = torch.empty((ctx.ny, ctx.nx), dtype=torch.float64, device=ctx.device)
    if var is None and want_var:
        var = torch.empty((ctx.ny, ctx.nx), dtype=torch.float64, device=ctx.device)
    _check(_lib.gabp_posterior(ctx.handle, _ptr(mean), _ptr(var)), ctx)
    return mean, var


def gabp_message_change(ctx: Context) -> float:
    r = ctypes.c_double(0.0)
    _check(_lib.gabp_message_change(ctx.handle, ctypes.byref(r)), ctx)
    return float(r.value)


def gabp_get_messages(ctx: Context):
    """(prec, info) device tensors of shape (deg, ny, nx) in the context's dtype."""
    shape = (ctx.deg, ctx.ny, ctx.nx)
    prec = torch.empty(shape, dtype=TORCH_DTYPES[ctx.dtype], device=ctx.device)
    info = torch.empty(shape, dtype=TORCH_DTYPES[ctx.dtype], device=ctx.device)
    _check(_lib.gabp_get_messages(ctx.handle, _ptr(prec), _ptr(info)), ctx)
    return prec, info


def gabp_set_messages(ctx: Context, prec: torch.Tensor, info: torch.Tensor) -> None:
    shape = (ctx.deg, ctx.ny, ctx.nx)
    td = TORCH_DTYPES[ctx.dtype]
    prec = prec.to(device=ctx.device, dtype=td).contiguous()
    info = info.to(device=ctx.device, dtype=td).contiguous()
    if tuple(prec.shape) != shape or tuple(info.shape) != shape:
        raise ValueError(f"messages must have shape {shape}")
    _check(_lib.gabp_set_messages(ctx.handle, _ptr(prec), _ptr(info)), ctx)
    ctx._keep = (prec, info)   # alive until the stream has consumed them


def gabp_iteration_count(ctx: Context) -> Tuple[int, int]:
    """(iterations, status): status is GABP_E_DIVERGED after a divergence."""
    it = ctypes.c_int64(0)
    st = _lib.gabp_iteration_count(ctx.handle, ctypes.byref(it))
    if st not in (GABP_OK, GABP_E_DIVERGED):
        _check(st, ctx)
    return int(it.value), int(st)


def gabp_autotune(ctx: Context, trials: int, damping: float) -> int:
    """Time every tile shape on `trials` real iterations each; returns the chosen one."""
    ch = ctypes.c_int32(0)
    _check(_lib.gabp_autotune(ctx.handle, int(trials), float(damping), ctypes.byref(ch)), ctx)
    return int(ch.value)


def gabp_precision_frozen(ctx: Context) -> int:
    """Iteration at which the precision messages froze (-1 if not yet)."""
    at = ctypes.c_int64(-1)
    _check(_lib.gabp_precision_frozen(ctx.handle, ctypes.byref(at)), ctx)
    return int(at.value)


def gabp_num_directions(ctx: Context) -> int:
    return ctx.deg


def gabp_copy_coarse_messages(coarse: Context, fine: Context) -> None:
    """The paper's Upscale Messages literally: fine messages = coarse ones."""
    _check(_lib.gabp_copy_coarse_messages(coarse.handle, fine.handle), coarse)


def gabp_destroy(ctx: Context) -> None:
    if ctx.handle:
        _lib.gabp_destroy(ctx.handle)
        ctx.handle = None


# --------------------------------------------------------------------------
# batched instances
# --------------------------------------------------------------------------

class Batch:
    """A live gabp_batch plus its torch workspace."""

    def __init__(self, handle, workspace, shapes, dtype, device, stream):
        self.handle = handle
        self.workspace = workspace
        self.shapes = shapes          # (nx, ny, deg) per instance
        self.dtype = dtype
        self.device = device
        self.stream = stream
        self._keep = {}               # predictions read by queued warm starts

    @property
    def n(self) -> int:
        return len(self.shapes)

    def __del__(self):
        try:
            gabp_batch_destroy(self)
        except Exception:
            pass


def _bcheck(st: int, b: Optional[Batch] = None):
    if st != GABP_OK:
        h = b.handle if b is not None else None
        raise GabpError(st, _lib.gabp_batch_last_error(h).decode())


def gabp_batch_create(problems, dtype: Optional[str] = None, stream=None, device=None) -> Batch:
    """Create a batch from a list of ``inputs.Problem`` (observations are
    staged as device tensors, kept alive until the create call returns)."""
    device = torch.device(device or "cuda")
    dt = DTYPES[dtype or problems[0].dtype]
    if stream is None:
        stream = torch.cuda.current_stream(device)
    n = len(problems)
    arr = (gabp_instance * n)()
    keep = []
    shapes = []
    for k, p in enumerate(problems):
        cells = torch.as_tensor(np.asarray(p.cells), dtype=torch.int64).to(device).contiguous()
        y = torch.as_tensor(np.asarray(p.y), dtype=torch.float64).to(device).contiguous()
        var = None if p.var is None else \
            torch.as_tensor(np.asarray(p.var), dtype=torch.float64).to(device).contiguous()
        keep += [cells, y, var]
        arr[k].grid = _grid(p.nx, p.ny, p.hx, p.hy, p.bc_x, p.bc_y)
        arr[k].stencil = _stencil(p.alpha, p.kappa, p.tau, p.c)
        arr[k].obs = gabp_obs(int(cells.numel()), cells.data_ptr() if cells.numel() else None,
                              y.data_ptr() if y.numel() else None, 1)
        arr[k].noise = gabp_noise(float(p.sigma), None if var is None else var.data_ptr())
        shapes.append((p.nx, p.ny, 4 if p.alpha == 1 else 12))
    nbytes = ctypes.c_size_t(0)
    _bcheck(_lib.gabp_batch_workspace_size(n, arr, dt, ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    opts = gabp_opts(dt, stream.cuda_stream, ws.data_ptr(), int(nbytes.value), None)
    h = ctypes.c_void_p()
    _bcheck(_lib.gabp_batch_create(n, arr, ctypes.byref(opts), ctypes.byref(h)))
    del keep
    return Batch(h, ws, shapes, dt, device, stream)


def gabp_batch_iterate(b: Batch, n_iters: int, damping: float) -> None:
    _bcheck(_lib.gabp_batch_iterate(b.handle, int(n_iters), float(damping)), b)


def gabp_batch_solve(b: Batch, max_iters: int, damping: float, rel_tol: float,
                     check_every: int = 10):
    """Returns (status, iters[n], rel[n], status[n]) as numpy arrays."""
    it = np.zeros(b.n, dtype=np.int64)
    rel = np.zeros(b.n, dtype=np.float64)
    sts = np.zeros(b.n, dtype=np.int32)
    st = _lib.gabp_batch_solve(b.handle, int(max_iters), float(damping), float(rel_tol),
                               int(check_every), it.ctypes.data_as(_P), rel.ctypes.data_as(_P),
                               sts.ctypes.data_as(_P))
    if st not in (GABP_OK, GABP_E_NOT_CONVERGED):
        _bcheck(st, b)
    return int(st), it, rel, sts


def gabp_batch_posterior(b: Batch, i: int, want_var: bool = True):
    nx, ny, _ = b.shapes[i]
    mean = torch.empty((ny, nx), dtype=torch.float64, device=b.device)
    var = torch.empty((ny, nx), dtype=torch.float64, device=b.device) if want_var else None
    _bcheck(_lib.gabp_batch_posterior(b.handle, int(i), _ptr(mean), _ptr(var)), b)
    return mean, var


def gabp_batch_warm_init(b: Batch, i: int, pred: torch.Tensor,
                         keep_precisions: bool = False) -> None:
    """gabp_warm_init for instance i: pred FP32 [ny, nx, 16] of that instance."""
    nx, ny, _ = b.shapes[i]
    if pred.dtype != torch.float32 or tuple(pred.shape) != (ny, nx, 16) or not pred.is_cuda:
        raise ValueError("pred must be a CUDA float32 tensor of shape (ny, nx, 16)")
    pred = pred.contiguous()
    _bcheck(_lib.gabp_batch_warm_init(b.handle, int(i), _ptr(pred), int(bool(keep_precisions))), b)
    b._keep[int(i)] = pred


def gabp_batch_upscale_precisions(b: Batch, i: int, pred: torch.Tensor, scale: float) -> None:
    """gabp_upscale_precisions with instance i as the coarse lattice."""
    if pred.dtype != torch.float32 or pred.dim() != 3 or pred.shape[2] != 16 or \
            not pred.is_contiguous():
        raise ValueError("pred must be a contiguous float32 [nyf, nxf, 16] tensor")
    nyf, nxf, _ = pred.shape
    _bcheck(_lib.gabp_batch_upscale_precisions(b.handle, int(i), _ptr(pred), int(nxf), int(nyf),
                                               float(scale)), b)


def gabp_batch_log_precisions(b: Batch, i: int, want_valid: bool = True):
    """gabp_log_precisions of instance i: (lam, valid or None) [12, ny, nx]."""
    nx, ny, _ = b.shapes[i]
    lam = torch.empty((12, ny, nx), dtype=torch.float32, device=b.device)
    valid = torch.empty_like(lam) if want_valid else None
    _bcheck(_lib.gabp_batch_log_precisions(b.handle, int(i), _ptr(lam), _ptr(valid)), b)
    return lam, valid


def gabp_batch_get_messages(b: Batch, i: int):
    nx, ny, deg = b.shapes[i]
    td = TORCH_DTYPES[b.dtype]
    prec = torch.empty((deg, ny, nx), dtype=td, device=b.device)
    info = torch.empty((deg, ny, nx), dtype=td, device=b.device)
    _bcheck(_lib.gabp_batch_get_messages(b.handle, int(i), _ptr(prec), _ptr(info)), b)
    return prec, info


def gabp_batch_autotune(b: Batch, trials: int, damping: float) -> int:
    ch = ctypes.c_int32(0)
    _bcheck(_lib.gabp_batch_autotune(b.handle, int(trials), float(damping), ctypes.byref(ch)), b)
    return int(ch.value)


def gabp_batch_info(b: Batch, i: int):
    """(iterations, frozen_at, running) of instance i."""
    it = ctypes.c_int64(0)
    fz = ctypes.c_int64(0)
    run = ctypes.c_int32(0)
    _bcheck(_lib.gabp_batch_info(b.handle, int(i), ctypes.byref(it), ctypes.byref(fz),
                                 ctypes.byref(run)), b)
    return int(it.value), int(fz.value), bool(run.value)


def gabp_batch_destroy(b: Batch) -> None:
    if b.handle:
        _lib.gabp_batch_destroy(b.handle)
        b.handle = None


# --------------------------------------------------------------------------
# learned warm start: network primitives and message initialisation
# --------------------------------------------------------------------------

def _ncheck(st: int):
    if st != GABP_OK:
        raise GabpError(st, _lib.gabp_net_last_error().decode())


def _stream_handle(stream):
    return (stream or torch.cuda.current_stream()).cuda_stream


def gabp_warm_init(ctx: Context, pred: torch.Tensor, keep_precisions: bool = False) -> None:
    """pred: FP32 device tensor [ny, nx, 16] (mean, log(-Lam) per sender-indexed direction)."""
    if pred.dtype != torch.float32 or tuple(pred.shape) != (ctx.ny, ctx.nx, 16) or not pred.is_cuda:
        raise ValueError("pred must be a CUDA float32 tensor of shape (ny, nx, 16)")
    pred = pred.contiguous()
    _check(_lib.gabp_warm_init(ctx.handle, _ptr(pred), int(bool(keep_precisions))), ctx)
    ctx._keep_pred = pred


def gabp_conv3x3_fwd(x: torch.Tensor, w: torch.Tensor, bias: Optional[torch.Tensor], cout: int,
                     dil: int, relu: bool, want_bf16: bool = True, want_f32: bool = False,
                     stream=None):
    """x: bf16 [B,H,W,cin]; w: bf16 [32, 9*cin]; bias fp32 [32] -> (y_bf16, y_f32)."""
    B, H, W, cin = x.shape
    yb = torch.empty((B, H, W, cout), dtype=torch.bfloat16, device=x.device) if want_bf16 else None
    yf = torch.empty((B, H, W, cout), dtype=torch.float32, device=x.device) if want_f32 else None
    _ncheck(_lib.gabp_conv3x3_fwd(_ptr(x), B, H, W, cin, _ptr(w), _ptr(bias), int(cout), int(dil),
                                  int(bool(relu)), _ptr(yb), _ptr(yf), _stream_handle(stream)))
    return yb, yf


def gabp_conv3x3_bwd(x, y, dy, w, cout, dil, relu, need_dx=True, workspace=None, stream=None):
    """Returns (dw [32, 9*cin], db [32], dx [B,H,W,cin] or None), all FP32."""
    B, H, W, cin = x.shape
    nbytes = int(_lib.gabp_conv3x3_bwd_workspace(B, H, W, cin, int(cout)))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    dw = torch.empty((32, 9 * cin), dtype=torch.float32, device=x.device)
    db = torch.empty(32, dtype=torch.float32, device=x.device)
    dx = torch.empty((B, H, W, cin), dtype=torch.float32, device=x.device) if need_dx else None
    _ncheck(_lib.gabp_conv3x3_bwd(_ptr(x), _ptr(y), _ptr(dy), B, H, W, cin, _ptr(w), int(cout),
                                  int(dil), int(bool(relu)), _ptr(dw), _ptr(db), _ptr(dx),
                                  _ptr(workspace), nbytes, _stream_handle(stream)))
    return dw, db, dx, workspace


def gabp_adam_step(w, g, m, v, w_bf16, lr, beta1, beta2, eps, step, stream=None) -> None:
    _ncheck(_lib.gabp_adam_step(_ptr(w), _ptr(g), _ptr(m), _ptr(v), _ptr(w_bf16), int(w.numel()),
                                float(lr), float(beta1), float(beta2), float(eps), int(step),
                                _stream_handle(stream)))


def gabp_warm_loss(pred, mu_t, lam_t, valid, ndir, lam_weight, stream=None):
    """Returns (loss as a 0-d FP64 device tensor, grad [P,16])."""
    P = pred.numel() // 16
    grad = torch.empty_like(pred)
    parts = torch.empty((P + 255) // 256, dtype=torch.float64, device=pred.device)
    nparts = ctypes.c_int32(0)
    _ncheck(_lib.gabp_warm_loss(_ptr(pred), _ptr(mu_t), _ptr(lam_t), _ptr(valid), int(P), int(ndir),
                                float(lam_weight), _ptr(grad), _ptr(parts), ctypes.byref(nparts),
                                _stream_handle(stream)))
    return parts[: nparts.value].sum(), grad


def gabp_warm_features(cells, y, nx, ny, kappa, device=None, stream=None):
    """[ny, nx, 16] bf16 input features of one problem."""
    device = torch.device(device or "cuda")
    if not isinstance(cells, torch.Tensor):
        cells = torch.as_tensor(np.asarray(cells), dtype=torch.int64)
    if not isinstance(y, torch.Tensor):
        y = torch.as_tensor(np.asarray(y), dtype=torch.float64)
    cells = cells.to(device=device, dtype=torch.int64).contiguous()
    y = y.to(device=device, dtype=torch.float64).contiguous()
    scratch = torch.empty(2 * nx * ny, dtype=torch.float32, device=device)
    x = torch.empty((ny, nx, 16), dtype=torch.bfloat16, device=device)
    _ncheck(_lib.gabp_warm_features(int(cells.numel()), _ptr(cells) if cells.numel() else None,
                                    _ptr(y) if y.numel() else None, int(nx), int(ny), float(kappa),
                                    _ptr(scratch), _ptr(x), _stream_handle(stream)))
    return x


def gabp_warm_features_noalloc(cells: torch.Tensor, y: torch.Tensor, nx: int, ny: int,
                               kappa: float, out: torch.Tensor, stream=None) -> None:
    """gabp_warm_features_noalloc into a caller-owned [ny, nx, 16] bf16 tensor
    (cells int64 and y float64 device tensors; nothing is allocated)."""
    _ncheck(_lib.gabp_warm_features_noalloc(int(cells.numel()),
                                            _ptr(cells) if cells.numel() else None,
                                            _ptr(y) if y.numel() else None, int(nx), int(ny),
                                            float(kappa), _ptr(out), _stream_handle(stream)))


def gabp_set_graph(ctx: Context, enable: bool) -> None:
    """Record and replay solver chunks as hipGraphs (default) or launch directly."""
    _check(_lib.gabp_set_graph(ctx.handle, 1 if enable else 0), ctx)


def gabp_set_tile(ctx: Context, rows_per_thread: int, pair_rows: int) -> None:
    """Tile configuration of the iteration kernels (results never depend on it)."""
    _check(_lib.gabp_set_tile(ctx.handle, int(rows_per_thread), int(pair_rows)), ctx)


def gabp_set_freeze_tolerance(ctx: Context, max_slots: int, max_rel: float) -> None:
    """Freeze the precision messages also when at most max_slots of them
    changed in the last iteration, each by at most max_rel (0: bitwise)."""
    _check(_lib.gabp_set_freeze_tolerance(ctx.handle, int(max_slots), float(max_rel)), ctx)


def gabp_batch_set_freeze_tolerance(b: Batch, max_slots: int, max_rel: float) -> None:
    """gabp_set_freeze_tolerance for every instance of a batch."""
    _bcheck(_lib.gabp_batch_set_freeze_tolerance(b.handle, int(max_slots), float(max_rel)), b)


def gabp_log_precisions(ctx: Context, want_valid: bool = True):
    """(lam [12, ny, nx], valid [12, ny, nx] or None) FP32 device tensors."""
    lam = torch.empty((12, ctx.ny, ctx.nx), dtype=torch.float32, device=ctx.device)
    valid = torch.empty_like(lam) if want_valid else None
    _check(_lib.gabp_log_precisions(ctx.handle, _ptr(lam), _ptr(valid)), ctx)
    return lam, valid


def gabp_launch_counts(ctx: Context) -> dict:
    """Iteration-kernel launches issued by a context, by kind."""
    v = [ctypes.c_int64(0) for _ in range(4)]
    _check(_lib.gabp_launch_counts(ctx.handle, *[ctypes.byref(x) for x in v]), ctx)
    return {"full": v[0].value, "theta": v[1].value, "pair_tiles": v[2].value,
            "pair_walk": v[3].value}


def gabp_get_tile(ctx: Context) -> Tuple[int, int]:
    """(rows_per_thread, pair_rows) of a context."""
    r = ctypes.c_int32(0)
    p = ctypes.c_int32(0)
    _check(_lib.gabp_get_tile(ctx.handle, ctypes.byref(r), ctypes.byref(p)), ctx)
    return int(r.value), int(p.value)


def gabp_upscale_precisions(coarse_ctx: Context, pred: torch.Tensor, scale: float) -> None:
    """Write channels 1..deg of a fine prediction [nyf, nxf, 16] (FP32) from
    the coarse context's precision messages, multiplied by `scale`."""
    if pred.dtype != torch.float32 or pred.dim() != 3 or pred.shape[2] != 16 or \
            not pred.is_contiguous():
        raise ValueError("pred must be a contiguous float32 [nyf, nxf, 16] tensor")
    nyf, nxf, _ = pred.shape
    _check(_lib.gabp_upscale_precisions(coarse_ctx.handle, _ptr(pred), int(nxf), int(nyf),
                                        float(scale)), coarse_ctx)


def gabp_upsample_mean(coarse: torch.Tensor, bc_x: int, bc_y: int, nxf: int, nyf: int,
                       stream=None) -> torch.Tensor:
    """Prediction [nyf, nxf, 16] FP32 whose channel 0 is the bilinear
    upsampling of the coarse FP64 mean [nyc, nxc]."""
    coarse = coarse.to(torch.float64).contiguous()
    nyc, nxc = coarse.shape
    pred = torch.empty((nyf, nxf, 16), dtype=torch.float32, device=coarse.device)
    _check(_lib.gabp_upsample_mean(_ptr(coarse), int(nxc), int(nyc), int(bc_x), int(bc_y),
                                   _ptr(pred), int(nxf), int(nyf), _stream_handle(stream)))
    return pred


# --------------------------------------------------------------------------
# space-time solver (include/gabp_st.h)
# --------------------------------------------------------------------------

ST_DIRECTIONS = 38


class STContext:
    """A live gabp_st_ctx (the library owns its device memory)."""

    def __init__(self, handle, stream, nx, ny, nt, dtype, device):
        self.handle = handle
        self.stream = stream
        self.nx, self.ny, self.nt = nx, ny, nt
        self.dtype = dtype
        self.device = device

    def __del__(self):
        try:
            gabp_st_destroy(self)
        except Exception:
            pass


def _st_check(st: int, ctx: Optional[STContext] = None):
    if st != GABP_OK:
        raise GabpError(st, gabp_st_last_error(ctx) if ctx is not None else gabp_st_create_error())


def gabp_st_create_error() -> str:
    return _lib.gabp_st_create_error().decode()


def gabp_st_last_error(ctx: Optional[STContext]) -> str:
    return _lib.gabp_st_last_error(ctx.handle if ctx is not None else None).decode()


def st_model(prob) -> gabp_st_model:
    """gabp_st_model of an ``inputs.SpaceTimeProblem``."""
    return gabp_st_model(int(prob.nx), int(prob.ny), int(prob.nt), int(prob.bc_x),
                         int(prob.bc_y), float(prob.dt), float(prob.h), float(prob.nu),
                         float(prob.kappa), float(prob.a0), float(prob.sigma_u), float(prob.c))


def gabp_st_workspace_size(model: gabp_st_model, dtype: int) -> int:
    n = ctypes.c_size_t(0)
    _st_check(_lib.gabp_st_workspace_size(ctypes.byref(model), int(dtype), ctypes.byref(n)))
    return int(n.value)


def gabp_st_create(model: gabp_st_model, cells, y, sigma: float, var=None, prior_mean=None,
                   dtype: int = GABP_F32, stream=None, device=None) -> STContext:
    """Create a space-time context; cells (int64) and y (float64) go to the
    device first (torch tensors or numpy arrays)."""
    device = torch.device(device or "cuda")
    cells = torch.as_tensor(np.asarray(cells) if not torch.is_tensor(cells) else cells,
                            dtype=torch.int64).to(device).contiguous()
    y = torch.as_tensor(np.asarray(y) if not torch.is_tensor(y) else y,
                        dtype=torch.float64).to(device).contiguous()
    if var is not None:
        var = torch.as_tensor(var, dtype=torch.float64).to(device).contiguous()
    if prior_mean is not None:
        prior_mean = torch.as_tensor(prior_mean, dtype=torch.float64).to(device).contiguous()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    obs = gabp_obs(int(cells.numel()), cells.data_ptr() if cells.numel() else None,
                   y.data_ptr() if y.numel() else None, 1)
    noise = gabp_noise(float(sigma), None if var is None else var.data_ptr())
    h = ctypes.c_void_p()
    _st_check(_lib.gabp_st_create(ctypes.byref(model), ctypes.byref(obs), ctypes.byref(noise),
                                  _ptr(prior_mean), int(dtype), stream.cuda_stream,
                                  ctypes.byref(h)))
    return STContext(h, stream, model.nx, model.ny, model.nt, int(dtype), device)


def gabp_st_create_problem(prob, dtype: Optional[str] = None, prior_mean=None, stream=None,
                           device=None) -> STContext:
    """gabp_st_create with the arguments of an ``inputs.SpaceTimeProblem``."""
    return gabp_st_create(st_model(prob), prob.cells, prob.y, prob.sigma, var=prob.var,
                          prior_mean=prior_mean, dtype=DTYPES[dtype or prob.dtype],
                          stream=stream, device=device)


def gabp_st_iterate(ctx: STContext, n_iters: int, damping: float) -> None:
    _st_check(_lib.gabp_st_iterate(ctx.handle, int(n_iters), float(damping)), ctx)


def gabp_st_residual(ctx: STContext) -> Tuple[float, float]:
    rel = ctypes.c_double(0.0)
    ab = ctypes.c_double(0.0)
    _st_check(_lib.gabp_st_residual(ctx.handle, ctypes.byref(rel), ctypes.byref(ab)), ctx)
    return float(rel.value), float(ab.value)


def gabp_st_solve(ctx: STContext, max_iters: int, damping: float, rel_tol: float,
                  check_every: int = 50) -> Tuple[int, int, float]:
    """Returns (status, total iterations, last relative residual)."""
    it = ctypes.c_int64(0)
    rel = ctypes.c_double(0.0)
    st = _lib.gabp_st_solve(ctx.handle, int(max_iters), float(damping), float(rel_tol),
                            int(check_every), ctypes.byref(it), ctypes.byref(rel))
    if st not in (GABP_OK, GABP_E_DIVERGED, GABP_E_NOT_CONVERGED):
        _st_check(st, ctx)
    return int(st), int(it.value), float(rel.value)


def gabp_st_posterior(ctx: STContext, want_var: bool = True):
    """Posterior mean and variance as (nt, ny, nx) float64 device tensors."""
    shape = (ctx.nt, ctx.ny, ctx.nx)
    mean = torch.empty(shape, dtype=torch.float64, device=ctx.device)
    var = torch.empty(shape, dtype=torch.float64, device=ctx.device) if want_var else None
    _st_check(_lib.gabp_st_posterior(ctx.handle, _ptr(mean), _ptr(var)), ctx)
    return mean, var


def gabp_st_get_messages(ctx: STContext):
    """Receiver-indexed (prec, info) of shape (38, nt, ny, nx), message dtype."""
    shape = (ST_DIRECTIONS, ctx.nt, ctx.ny, ctx.nx)
    prec = torch.empty(shape, dtype=TORCH_DTYPES[ctx.dtype], device=ctx.device)
    info = torch.empty(shape, dtype=TORCH_DTYPES[ctx.dtype], device=ctx.device)
    _st_check(_lib.gabp_st_get_messages(ctx.handle, _ptr(prec), _ptr(info)), ctx)
    return prec, info


def gabp_st_iteration_count(ctx: STContext) -> Tuple[int, int]:
    it = ctypes.c_int64(0)
    dv = ctypes.c_int64(0)
    _st_check(_lib.gabp_st_iteration_count(ctx.handle, ctypes.byref(it), ctypes.byref(dv)), ctx)
    return int(it.value), int(dv.value)


def gabp_st_set_freeze_tolerance(ctx: STContext, max_slots: int, max_rel: float) -> None:
    _st_check(_lib.gabp_st_set_freeze_tolerance(ctx.handle, int(max_slots), float(max_rel)), ctx)


def gabp_st_upsample_mean(coarse: torch.Tensor, bc_x: int, bc_y: int, nx: int, ny: int,
                          nt: int, stream=None) -> torch.Tensor:
    """Trilinear upsampling of a coarse (ntc, nyc, nxc) FP64 mean onto the
    fine (nt, ny, nx) grid; returns a new device tensor."""
    ntc, nyc, nxc = coarse.shape
    coarse = coarse.contiguous()
    fine = torch.empty((nt, ny, nx), dtype=torch.float64, device=coarse.device)
    if stream is None:
        stream = torch.cuda.current_stream(coarse.device)
    _st_check(_lib.gabp_st_upsample_mean(_ptr(coarse), nxc, nyc, ntc, int(bc_x), int(bc_y),
                                         _ptr(fine), int(nx), int(ny), int(nt),
                                         stream.cuda_stream))
    return fine


def gabp_st_warm_init(ctx: STContext, mean: torch.Tensor) -> None:
    mean = mean.to(torch.float64).contiguous()
    _st_check(_lib.gabp_st_warm_init(ctx.handle, _ptr(mean)), ctx)
    ctx._keep = mean        # alive until the stream has used it


def gabp_st_set_theta_slices(ctx: STContext, slices: int) -> None:
    _st_check(_lib.gabp_st_set_theta_slices(ctx.handle, int(slices)), ctx)


def gabp_st_precision_frozen(ctx: STContext) -> int:
    """Iteration at which the precision messages froze, or -1."""
    v = ctypes.c_int64(0)
    _st_check(_lib.gabp_st_precision_frozen(ctx.handle, ctypes.byref(v)), ctx)
    return int(v.value)


def gabp_st_destroy(ctx: STContext) -> None:
    if getattr(ctx, "handle", None) is not None and ctx.handle.value:
        _lib.gabp_st_destroy(ctx.handle)
        ctx.handle = ctypes.c_void_p()
