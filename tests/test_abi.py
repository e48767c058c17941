"""The C ABI library: it loads, exports every function include/*.h
declares, and validates arguments on the host before touching a device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def G():
    from paper_2404_12968_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2404_12968_amd import gabp
    return gabp


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(gabp_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_declared_function_is_exported(G):
    lib = ctypes.CDLL(G.LIBRARY_PATH)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(G.EXPORTED)


def test_status_strings(G):
    assert G.gabp_status_string(G.GABP_OK) == "ok"
    assert G.gabp_status_string(G.GABP_E_DIVERGED) == "diverged"


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=0), "nx"), (dict(alpha=3), "alpha"), (dict(kappa=0.0), "kappa"),
    (dict(kappa=float("nan")), "kappa"), (dict(tau=-1.0), "tau"), (dict(c=0.0), "c must"),
    (dict(bc_x=1, nx=4), "periodic"), (dict(hx=0.0), "hx"), (dict(dtype=7), "dtype"),
    (dict(bc_y=5), "boundary"),
])
def test_workspace_size_rejects_invalid(G, kw, msg):
    a = dict(nx=16, ny=16, hx=1.0, hy=1.0, bc_x=0, bc_y=0, alpha=2, kappa=0.1, tau=1.0, c=10.0,
             dtype=0)
    a.update(kw)
    grid = G.gabp_grid(a["nx"], a["ny"], a["hx"], a["hy"], a["bc_x"], a["bc_y"])
    st = G.gabp_stencil(a["alpha"], a["kappa"], a["tau"], a["c"])
    with pytest.raises(G.GabpError) as ei:
        G.gabp_workspace_size(grid, st, a["dtype"])
    assert ei.value.status == G.GABP_E_INVALID
    assert msg in G.gabp_last_error()


def test_workspace_size_of_the_global_grid(G):
    grid = G.gabp_grid(8192, 4096, 1.0, 1.0, G.GABP_BC_PERIODIC, G.GABP_BC_NEUMANN)
    st = G.gabp_stencil(2, 0.02, 1.0, 10.0)
    n = G.gabp_workspace_size(grid, st, G.GABP_F32)
    planes = 8192 * 4096 * 4
    # two buffers of 24 FP32 planes, 12 gain planes, four FP64 and two FP32
    # node planes
    assert 60 * planes + 10 * planes <= n <= 70 * planes + (64 << 20)


def test_create_rejects_host_observations_before_any_device_call(G):
    grid = G.gabp_grid(8, 8, 1.0, 1.0, 0, 0)
    st = G.gabp_stencil(1, 0.2, 1.0, 1.0)
    cells = (ctypes.c_int64 * 2)(3, 64)
    ys = (ctypes.c_double * 2)(1.0, 2.0)
    obs = G.gabp_obs(2, ctypes.cast(cells, ctypes.c_void_p), ctypes.cast(ys, ctypes.c_void_p), 0)
    noise = G.gabp_noise(0.1, None)
    opts = G.gabp_opts(0, None, None, 0, None)
    h = ctypes.c_void_p()
    rc = G._lib.gabp_create(ctypes.byref(grid), ctypes.byref(st), ctypes.byref(obs),
                            ctypes.byref(noise), ctypes.byref(opts), ctypes.byref(h))
    assert rc == G.GABP_E_INVALID and not h.value
    assert "out of range" in G.gabp_last_error()
    noise = G.gabp_noise(-1.0, None)
    rc = G._lib.gabp_create(ctypes.byref(grid), ctypes.byref(st), ctypes.byref(obs),
                            ctypes.byref(noise), ctypes.byref(opts), ctypes.byref(h))
    assert rc == G.GABP_E_INVALID and "sigma" in G.gabp_last_error()


def test_null_context_calls_are_invalid(G):
    assert G._lib.gabp_iterate(None, 1, 0.5) == G.GABP_E_INVALID
    assert G._lib.gabp_residual(None, None, None) == G.GABP_E_INVALID
    G._lib.gabp_destroy(None)


def _st_model(G, **kw):
    a = dict(nx=32, ny=24, nt=6, bc_x=0, bc_y=0, dt=1.0, h=1.0, nu=0.25, kappa=0.1, a0=1.0,
             sigma_u=0.1, c=3.0)
    a.update(kw)
    return G.gabp_st_model(*[a[f] for f, _ in G.gabp_st_model._fields_])


@pytest.mark.parametrize("kw,msg", [
    (dict(nt=0), "nt"), (dict(bc_x=2), "boundary"), (dict(bc_y=1, ny=4), "periodic"),
    (dict(kappa=0.0), "kappa"), (dict(dt=float("inf")), "dt"), (dict(nu=-1.0), "nu"),
    (dict(c=0.0), "c must"), (dict(nx=4096, ny=4096, nt=128), "too large"),
])
def test_st_workspace_size_rejects_invalid(G, kw, msg):
    with pytest.raises(G.GabpError) as ei:
        G.gabp_st_workspace_size(_st_model(G, **kw), G.GABP_F32)
    assert ei.value.status == G.GABP_E_INVALID
    assert msg in G.gabp_st_create_error()


def test_st_workspace_size_of_the_space_time_workload(G):
    n = G.gabp_st_workspace_size(_st_model(G, nx=512, ny=512, nt=64), G.GABP_F32)
    nodes = 512 * 512 * 64
    # two buffers of 76 FP32 planes, 38 gain planes, three FP64 and two FP32
    # node planes
    assert 190 * 4 * nodes + 32 * nodes <= n <= 190 * 4 * nodes + 32 * nodes + (1 << 20) + 190 * 256


def test_st_create_rejects_host_observations_before_any_device_call(G):
    model = _st_model(G, nx=8, ny=8, nt=3)
    cells = (ctypes.c_int64 * 2)(3, 8 * 8 * 3)
    ys = (ctypes.c_double * 2)(1.0, 2.0)
    obs = G.gabp_obs(2, ctypes.cast(cells, ctypes.c_void_p), ctypes.cast(ys, ctypes.c_void_p), 0)
    noise = G.gabp_noise(0.1, None)
    h = ctypes.c_void_p()
    rc = G._lib.gabp_st_create(ctypes.byref(model), ctypes.byref(obs), ctypes.byref(noise), None,
                               0, None, ctypes.byref(h))
    assert rc == G.GABP_E_INVALID and not h.value
    assert "out of range" in G.gabp_st_create_error()
    assert G._lib.gabp_st_iterate(None, 1, 0.5) == G.GABP_E_INVALID
    G._lib.gabp_st_destroy(None)
