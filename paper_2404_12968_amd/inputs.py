"""Seeded synthetic workloads for lattice data assimilation.

This module only draws inputs: truth fields, observation masks and noisy
observations.  It holds none of the message-passing arithmetic and none of the
prior-precision assembly, so both the GPU path and the CPU oracle can take
their inputs from it without sharing any of the method's code.

Workload shapes follow the paper's experiments: square synthetic grids with
uniformly random observed cells (Section "Effect of Domain Size and
Observation Density") and a large global grid observed along satellite ground
tracks, periodic in longitude (Section "Large-scale Example").  The paper's
own data (Met Office model output, ERA5 climatology, satellite ephemerides) is
not public; the track generator below stands in for it.

Random stream: ``numpy.random.default_rng(1000 * k + instance)`` for workload
number k.  Within one problem the draw order is: truth, observation mask,
observation noise.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BC_NEUMANN = 0
BC_PERIODIC = 1
BC_DIRICHLET = 2

BC_NAMES = {BC_NEUMANN: "neumann", BC_PERIODIC: "periodic", BC_DIRICHLET: "dirichlet"}


@dataclasses.dataclass
class Problem:
    """One assimilation instance: grid, prior parameters, observations.

    Cells are row-major, ``cell = y * nx + x``.  ``sigma`` is the observation
    noise standard deviation; ``var`` (optional) overrides it per observation.
    ``c`` is the re-weighting constant and ``damping`` the learning rate of
    the damped update; ``dtype`` is the message-plane precision ("f32"/"f64").
    """

    name: str
    nx: int
    ny: int
    bc_x: int
    bc_y: int
    alpha: int
    kappa: float
    tau: float
    c: float
    sigma: float
    cells: np.ndarray
    y: np.ndarray
    hx: float = 1.0
    hy: float = 1.0
    var: Optional[np.ndarray] = None
    truth: Optional[np.ndarray] = None
    dtype: str = "f32"
    damping: float = 0.5
    rel_tol: float = 1e-6
    max_iters: int = 100000
    fixed_iters: Optional[int] = None
    check_every: int = 10
    seed: int = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def coverage(self) -> float:
        return np.unique(self.cells).size / float(self.n)


# --------------------------------------------------------------------------
# truth fields
# --------------------------------------------------------------------------

def fourier_modes_field(nx: int, ny: int, rng: np.random.Generator,
                        n_modes: int = 16, max_freq: int = 6) -> np.ndarray:
    """Sum of ``n_modes`` random plane waves on the grid (shape (ny, nx)).

    Amplitudes a_k ~ N(0, 1/n_modes), integer wave numbers (u_k, v_k) uniform
    on [-max_freq, max_freq]^2 without (0, 0), phases uniform on [0, 2 pi).
    Evaluated separably: cos(a + b) = cos a cos b - sin a sin b.
    """
    amp = rng.normal(0.0, np.sqrt(1.0 / n_modes), size=n_modes)
    uv = np.zeros((n_modes, 2), dtype=np.int64)
    for k in range(n_modes):
        while True:
            cand = rng.integers(-max_freq, max_freq + 1, size=2)
            if cand[0] != 0 or cand[1] != 0:
                uv[k] = cand
                break
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    xs = np.arange(nx, dtype=np.float64)[:, None]
    ys = np.arange(ny, dtype=np.float64)[:, None]
    ax = 2.0 * np.pi * xs * uv[None, :, 0] / nx          # (nx, K)
    ay = 2.0 * np.pi * ys * uv[None, :, 1] / ny + phase  # (ny, K)
    f = (np.cos(ay) * amp) @ np.cos(ax).T - (np.sin(ay) * amp) @ np.sin(ax).T
    return np.ascontiguousarray(f)


def spectral_field(nx: int, ny: int, kappa: float, alpha: int,
                   rng: np.random.Generator) -> np.ndarray:
    """Periodic Gaussian random field with a Matern-type spectrum, unit variance.

    Spectral synthesis: white complex noise on the discrete Fourier grid,
    shaped by the continuous Matern spectral density
    (kappa^2 + |omega|^2)^(-alpha), omega in radians per cell, then an inverse
    real FFT.  This stands in for the paper's prior samples of the truth; it
    does not use the discrete precision operator of the solver.
    """
    wx = 2.0 * np.pi * np.fft.rfftfreq(nx)
    wy = 2.0 * np.pi * np.fft.fftfreq(ny)
    spec = (kappa * kappa + wy[:, None] ** 2 + wx[None, :] ** 2) ** (-0.5 * alpha)
    noise = rng.standard_normal((ny, wx.size, 2))
    coef = (noise[..., 0] + 1j * noise[..., 1]) * spec
    del noise
    f = np.fft.irfft2(coef, s=(ny, nx))
    f -= f.mean()
    sd = f.std()
    if sd > 0:
        f /= sd
    return np.ascontiguousarray(f)


def spde_tau(kappa: float, h: float, sigma_f: float) -> float:
    """Precision scale of the discretised SPDE with alpha = 2 in two
    dimensions (nu = 1): tau = h^2 / (sigma_f^2 q), q = 4 pi kappa^2, so that
    the marginal variance is about sigma_f^2 away from the boundary
    (Appendix "White Noise Discretisation", the constant q)."""
    return h * h / (sigma_f * sigma_f * 4.0 * np.pi * kappa * kappa)


def spde_field_dirichlet(nx: int, ny: int, kappa: float, h: float, sigma_f: float,
                         z: np.ndarray) -> np.ndarray:
    """Map white noise z (ny, nx) to a sample of the discretised Matern SPDE
    with alpha = 2: (kappa^2 I - Delta_h) f = sqrt(sigma_f^2 q / h^2) z on the
    nx x ny interior nodes of a grid with zero boundary values (Appendix
    "White Noise Discretisation"), i.e. f ~ N(0, (tau (kappa^2 I - Delta_h)^2)^-1)
    with tau = spde_tau(kappa, h, sigma_f).

    The orthonormal type-I sine transform diagonalises the Dirichlet operator
    (eigenvalues kappa^2 + (4/h^2)(sin^2(pi j / (2(nx+1))) + sin^2(pi k / (2(ny+1))))),
    so the solve is two transforms.  This draws the truth of the synthetic
    experiments; neither solver calls it.
    """
    import scipy.fft as sf
    jx = np.arange(1, nx + 1)
    jy = np.arange(1, ny + 1)
    ex = 4.0 / (h * h) * np.sin(np.pi * jx / (2.0 * (nx + 1))) ** 2
    ey = 4.0 / (h * h) * np.sin(np.pi * jy / (2.0 * (ny + 1))) ** 2
    lam = kappa * kappa + ey[:, None] + ex[None, :]
    scale = 1.0 / np.sqrt(spde_tau(kappa, h, sigma_f))
    zh = sf.dstn(np.asarray(z, dtype=np.float64), type=1, norm="ortho")
    return np.ascontiguousarray(scale * sf.dstn(zh / lam, type=1, norm="ortho"))


# --------------------------------------------------------------------------
# observation masks
# --------------------------------------------------------------------------

def uniform_cells(n: int, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Distinct cells drawn uniformly at random, ``round(frac * n)`` of them, sorted."""
    m = int(round(frac * n))
    m = max(0, min(n, m))
    cells = rng.choice(n, size=m, replace=False)
    return np.sort(cells.astype(np.int64))


def track_cells(nx: int, ny: int, n_tracks: int, run: int,
                rng: np.random.Generator) -> np.ndarray:
    """Union of diagonal satellite-like ground tracks, sorted distinct cells.

    Track j has slope s_j = +-1 and x-offset x0_j uniform on {0..nx-1}; in row
    y it covers the ``run`` cells starting at (x0_j + s_j*y - run//2) mod nx,
    wrapping in x like a ground track.
    """
    ys = np.arange(ny, dtype=np.int64)
    out = []
    for _ in range(n_tracks):
        s = 1 if rng.integers(0, 2) == 1 else -1
        x0 = int(rng.integers(0, nx))
        start = x0 + s * ys - run // 2
        xs = (start[:, None] + np.arange(run, dtype=np.int64)[None, :]) % nx
        out.append((ys[:, None] * nx + xs).ravel())
    if not out:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(out))


def observe(truth: np.ndarray, cells: np.ndarray, sigma: float,
            rng: np.random.Generator) -> np.ndarray:
    """Noisy point observations y = f(cell) + sigma * eps, eps ~ N(0, 1)."""
    flat = truth.reshape(-1)
    return flat[cells] + sigma * rng.standard_normal(cells.size)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

WORKLOADS = ("parity64", "tracks2048", "global8192", "batch256", "warm1024", "table1",
             "global32k")
_WORKLOAD_K = {name: k + 1 for k, name in enumerate(WORKLOADS)}

# re-weighting constant by prior order: plain GaBP for the 5-point prior, the
# paper's selected c = 10 for the 13-point prior (it diverges at c = 1).
DEFAULT_C = {1: 1.0, 2: 10.0}


def parity64(instance: int = 0) -> Problem:
    """64x64 Neumann lattice, 5-point prior (kappa 0.2), 5 % random cells, FP64."""
    rng = np.random.default_rng(1000 * 1 + instance)
    nx = ny = 64
    truth = fourier_modes_field(nx, ny, rng)
    cells = uniform_cells(nx * ny, 0.05, rng)
    sigma = 0.1
    y = observe(truth, cells, sigma, rng)
    return Problem("parity64", nx, ny, BC_NEUMANN, BC_NEUMANN, alpha=1, kappa=0.2,
                   tau=1.0, c=DEFAULT_C[1], sigma=sigma, cells=cells, y=y, truth=truth,
                   dtype="f64", damping=0.5, rel_tol=1e-10, seed=1000 + instance)


def tracks2048(instance: int = 0, n: int = 2048) -> Problem:
    """2048^2 Neumann lattice, 13-point prior (kappa 0.05), 40 tracks of 4 cells, FP32."""
    rng = np.random.default_rng(1000 * 2 + instance)
    truth = spectral_field(n, n, 0.05, 2, rng)
    cells = track_cells(n, n, 40, 4, rng)
    sigma = 0.05
    y = observe(truth, cells, sigma, rng)
    return Problem("tracks2048", n, n, BC_NEUMANN, BC_NEUMANN, alpha=2, kappa=0.05,
                   tau=1.0, c=DEFAULT_C[2], sigma=sigma, cells=cells, y=y, truth=truth,
                   dtype="f32", damping=0.5, fixed_iters=1000, seed=2000 + instance)


def global8192(instance: int = 0, nx: int = 8192, ny: int = 4096,
               keep_truth: bool = False) -> Problem:
    """8192x4096 global-scale lattice, periodic in x, Neumann in y, 13-point prior
    (kappa 0.02), 60 tracks of 7 cells (~5 %), FP32 messages, to 1e-6."""
    rng = np.random.default_rng(1000 * 3 + instance)
    truth = spectral_field(nx, ny, 0.02, 2, rng)
    cells = track_cells(nx, ny, 60, 7, rng)
    sigma = 0.05
    y = observe(truth, cells, sigma, rng)
    return Problem("global8192", nx, ny, BC_PERIODIC, BC_NEUMANN, alpha=2, kappa=0.02,
                   tau=1.0, c=DEFAULT_C[2], sigma=sigma, cells=cells, y=y,
                   truth=truth if keep_truth else None,
                   dtype="f32", damping=0.5, rel_tol=1e-6, check_every=10,
                   seed=3000 + instance)


def global32k(instance: int = 0, nx: int = 32768, ny: int = 24576) -> Problem:
    """The global-scale workload at 32768 x 24576 (805 M nodes, 9.7 G directed
    edges, about 225 GB of solver state in FP32): periodic in x, zero-flux in
    y, 13-point prior, kappa 0.02, 240 tracks of 7 cells (~5 %), sigma 0.05.
    The truth is a sum of 64 random plane waves (a spectral synthesis would
    need an FFT of the whole grid on the host); only throughput is measured
    on it."""
    rng = np.random.default_rng(1000 * 7 + instance)
    truth = fourier_modes_field(nx, ny, rng, n_modes=64, max_freq=48)
    cells = track_cells(nx, ny, 240, 7, rng)
    sigma = 0.05
    y = observe(truth, cells, sigma, rng)
    del truth
    return Problem("global32k", nx, ny, BC_PERIODIC, BC_NEUMANN, alpha=2, kappa=0.02,
                   tau=1.0, c=DEFAULT_C[2], sigma=sigma, cells=cells, y=y, truth=None,
                   dtype="f32", damping=0.5, rel_tol=1e-6, check_every=10,
                   seed=7000 + instance)


def batch256_instance(inst: int, side_lo: int = 64, side_hi: int = 1024) -> Problem:
    """Instance `inst` of the uneven batch: square side ~ U{64..1024}, alpha ~
    U{1,2}, kappa ~ U[0.02,0.3], observed fraction ~ U[1 %, 20 %] (uniform
    cells), sigma ~ U[0.02, 0.2]."""
    rng = np.random.default_rng(1000 * 4 + inst)
    side = int(rng.integers(side_lo, side_hi + 1))
    alpha = int(rng.integers(1, 3))
    kappa = float(rng.uniform(0.02, 0.3))
    frac = float(rng.uniform(0.01, 0.20))
    sigma = float(rng.uniform(0.02, 0.2))
    truth = spectral_field(side, side, kappa, alpha, rng)
    cells = uniform_cells(side * side, frac, rng)
    y = observe(truth, cells, sigma, rng)
    return Problem(f"batch256[{inst}]", side, side, BC_NEUMANN, BC_NEUMANN,
                   alpha=alpha, kappa=kappa, tau=1.0, c=DEFAULT_C[alpha],
                   sigma=sigma, cells=cells, y=y, truth=None, dtype="f32",
                   damping=0.5, rel_tol=1e-6, seed=4000 + inst)


def batch256(count: int = 256, side_lo: int = 64, side_hi: int = 1024) -> List[Problem]:
    """The uneven batch: `count` instances of batch256_instance."""
    return [batch256_instance(inst, side_lo, side_hi) for inst in range(count)]


def warm1024(instance: int = 0, n: int = 1024, kappa: Optional[float] = None) -> Problem:
    """1024^2 Neumann lattice, 13-point prior, kappa ~ U[0.02, 0.3] unless given,
    16 tracks of 4 cells (~6 %), sigma 0.05, FP32 to 1e-6."""
    rng = np.random.default_rng(1000 * 5 + instance)
    k = float(rng.uniform(0.02, 0.3)) if kappa is None else float(kappa)
    truth = spectral_field(n, n, k, 2, rng)
    cells = track_cells(n, n, 16, 4, rng)
    sigma = 0.05
    y = observe(truth, cells, sigma, rng)
    return Problem(f"warm1024[{instance}]", n, n, BC_NEUMANN, BC_NEUMANN, alpha=2,
                   kappa=k, tau=1.0, c=DEFAULT_C[2], sigma=sigma, cells=cells, y=y,
                   truth=truth, dtype="f32", damping=0.5, rel_tol=1e-6,
                   seed=5000 + instance)


TABLE1_SIZES = (256, 512, 1024)
TABLE1_FRACS = (0.01, 0.05, 0.10)


def table1(n: int = 256, frac: float = 0.05, instance: int = 0) -> Problem:
    """The paper's synthetic experiment (Table 1; Appendix "Experiment
    Details", synthetic data): an n x n grid of interior nodes of the unit
    square with zero boundary values (h = 1/(n+1)), truth drawn from the
    alpha = 2 SPDE prior with nu = 1, length scale 0.15 (kappa = sqrt(2)/0.15)
    and sigma_f = 1.1, a fraction `frac` of the nodes observed uniformly at
    random, and the same prior for inference; c = 10, learning rate 0.6.
    The observation noise is not given in the paper; 0.01 is the reading
    under which the exact posterior reproduces the table's R-INLA column."""
    rng = np.random.default_rng([1000 * 6 + instance, n, int(round(frac * 1000))])
    kappa = np.sqrt(2.0) / 0.15
    sigma_f = 1.1
    h = 1.0 / (n + 1)
    truth = spde_field_dirichlet(n, n, kappa, h, sigma_f, rng.standard_normal((n, n)))
    cells = uniform_cells(n * n, frac, rng)
    sigma = 0.01
    y = observe(truth, cells, sigma, rng)
    return Problem(f"table1[{n},{frac:g},{instance}]", n, n, BC_DIRICHLET, BC_DIRICHLET,
                   alpha=2, kappa=float(kappa), tau=spde_tau(kappa, h, sigma_f), c=10.0,
                   sigma=sigma, cells=cells, y=y, hx=h, hy=h, truth=truth, dtype="f32",
                   damping=0.6, rel_tol=1e-6, seed=6000 + instance)


def small_lattice(nx: int, ny: int, alpha: int, *, bc_x: int = BC_NEUMANN,
                  bc_y: int = BC_NEUMANN, kappa: float = 0.2, tau: float = 1.0,
                  c: Optional[float] = None, frac: float = 0.05, sigma: float = 0.1,
                  seed: int = 0, dtype: str = "f64", damping: float = 0.5,
                  hx: float = 1.0, hy: float = 1.0, tracks: int = 0,
                  run: int = 3) -> Problem:
    """Generic small problem for tests: random (or track) cells on any grid/BC."""
    rng = np.random.default_rng(seed)
    truth = fourier_modes_field(nx, ny, rng, n_modes=8, max_freq=3)
    if tracks > 0:
        cells = track_cells(nx, ny, tracks, run, rng)
    else:
        cells = uniform_cells(nx * ny, frac, rng)
    y = observe(truth, cells, sigma, rng)
    return Problem(f"small{nx}x{ny}a{alpha}", nx, ny, bc_x, bc_y, alpha=alpha,
                   kappa=kappa, tau=tau, c=DEFAULT_C[alpha] if c is None else c,
                   sigma=sigma, cells=cells, y=y, truth=truth, dtype=dtype,
                   damping=damping, hx=hx, hy=hy, seed=seed)


def workload(name: str, instance: int = 0):
    """Named workload by its name (see WORKLOADS)."""
    fn = {"parity64": parity64, "tracks2048": tracks2048, "global8192": global8192,
          "batch256": lambda instance=0: batch256(), "warm1024": warm1024,
          "table1": lambda instance=0: table1(instance=instance), "global32k": global32k}[name]
    return fn(instance)


# --------------------------------------------------------------------------
# space-time workloads (the paper's spatio-temporal extension, Appendix
# "Extension to Spatiotemporal Systems")
# --------------------------------------------------------------------------

@dataclasses.dataclass
class SpaceTimeProblem:
    """One space-time assimilation instance: nt slices of an nx x ny grid.

    Prior: the stochastic heat equation du/dt = nu Lap u + sigma_u W on a grid
    of spacing h, Crank-Nicolson steps of length dt, initial condition with
    precision (dt h^2 / sigma_u^2) (a0 (kappa^2 I - Lap_h))^2 and zero mean.
    Cells are ``n * nx * ny + y * nx + x`` for slice n; ``sigma`` is the
    observation noise standard deviation, ``var`` (optional) overrides it.
    """

    name: str
    nx: int
    ny: int
    nt: int
    bc_x: int
    bc_y: int
    dt: float
    h: float
    nu: float
    kappa: float
    a0: float
    sigma_u: float
    c: float
    sigma: float
    cells: np.ndarray
    y: np.ndarray
    var: Optional[np.ndarray] = None
    truth: Optional[np.ndarray] = None
    dtype: str = "f32"
    damping: float = 0.5
    rel_tol: float = 1e-6
    max_iters: int = 100000
    check_every: int = 10
    seed: int = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nt

    @property
    def coverage(self) -> float:
        return np.unique(self.cells).size / float(self.n)


def heat_field_neumann(nx: int, ny: int, nt: int, dt: float, h: float, nu: float,
                       kappa: float, a0: float, sigma_u: float,
                       rng: np.random.Generator) -> np.ndarray:
    """A sample of the discretised stochastic heat equation on a zero-flux
    grid, shape (nt, ny, nx): u^0 solves a0 (kappa^2 I - Lap_h) u^0 = s z^0 and
    (I/dt - nu/2 Lap_h) u^{n+1} = (I/dt + nu/2 Lap_h) u^n + s z^{n+1} with
    s = sigma_u / sqrt(dt h^2) and z white noise.  The orthonormal DCT-II
    diagonalises the zero-flux Laplacian (eigenvalues -(4/h^2)(sin^2(pi j /
    (2 nx)) + sin^2(pi k / (2 ny)))) and maps white noise to white noise, so
    every step is a division per mode.  Draws the truth only; neither solver
    calls it."""
    import scipy.fft as sf
    ex = 4.0 / (h * h) * np.sin(np.pi * np.arange(nx) / (2.0 * nx)) ** 2
    ey = 4.0 / (h * h) * np.sin(np.pi * np.arange(ny) / (2.0 * ny)) ** 2
    g = ey[:, None] + ex[None, :]                      # eigenvalues of -Lap_h
    s = sigma_u / np.sqrt(dt * h * h)
    ua = s * rng.standard_normal((ny, nx)) / (a0 * (kappa * kappa + g))
    a = 1.0 / dt + 0.5 * nu * g
    b = 1.0 / dt - 0.5 * nu * g
    out = np.empty((nt, ny, nx))
    for k in range(nt):
        if k > 0:
            ua = (b * ua + s * rng.standard_normal((ny, nx))) / a
        out[k] = sf.idctn(ua, type=2, norm="ortho")
    return out


def spacetime_track_cells(nx: int, ny: int, nt: int, n_tracks: int, run: int,
                          drift: int, rng: np.random.Generator) -> np.ndarray:
    """Ground tracks that move between slices: track j (slope +-1, offset x0_j)
    sits at offset x0_j + drift_j * n in slice n, drift_j uniform on
    {-drift..drift}; each slice's cells as in ``track_cells``.  Sorted,
    distinct space-time cells."""
    ys = np.arange(ny, dtype=np.int64)
    out = []
    for _ in range(n_tracks):
        s = 1 if rng.integers(0, 2) == 1 else -1
        x0 = int(rng.integers(0, nx))
        v = int(rng.integers(-drift, drift + 1))
        for k in range(nt):
            start = x0 + v * k + s * ys - run // 2
            xs = (start[:, None] + np.arange(run, dtype=np.int64)[None, :]) % nx
            out.append(k * nx * ny + (ys[:, None] * nx + xs).ravel())
    if not out:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(out))


# heat-equation prior of the space-time workloads: one grid unit, unit time
# step, diffusion number nu dt / h^2 = 1/4, Matern-type initial field (kappa
# 0.1), process noise 0.1; re-weighting and damping chosen by the oracle's
# c x eta sweep on small grids.
SPACETIME_PRIOR = dict(dt=1.0, h=1.0, nu=0.25, kappa=0.1, a0=1.0, sigma_u=0.1)
SPACETIME_C = 3.0
SPACETIME_ETA = 0.4


def spacetime(instance: int = 0, nx: int = 512, ny: int = 512, nt: int = 64,
              n_tracks: int = 4, run: int = 3, sigma: float = 0.05,
              dtype: str = "f32", **prior) -> SpaceTimeProblem:
    """nt slices of an nx x ny zero-flux grid under the heat-equation prior,
    observed along ``n_tracks`` drifting ground tracks of ``run`` cells per
    slice (about 2 % of the space-time cells at 512^2 x 64), noise sigma."""
    pr = dict(SPACETIME_PRIOR)
    pr.update(prior)
    rng = np.random.default_rng([1000 * 8 + instance, nx, ny, nt])
    truth = heat_field_neumann(nx, ny, nt, pr["dt"], pr["h"], pr["nu"], pr["kappa"], pr["a0"],
                               pr["sigma_u"], rng)
    cells = spacetime_track_cells(nx, ny, nt, n_tracks, run, 3, rng)
    y = observe(truth, cells, sigma, rng)
    return SpaceTimeProblem(f"spacetime{nx}x{ny}x{nt}[{instance}]", nx, ny, nt, BC_NEUMANN,
                            BC_NEUMANN, c=SPACETIME_C, sigma=sigma, cells=cells, y=y,
                            truth=truth, dtype=dtype, damping=SPACETIME_ETA,
                            seed=8000 + instance, **pr)


def small_spacetime(nx: int, ny: int, nt: int, *, bc_x: int = BC_NEUMANN,
                    bc_y: int = BC_NEUMANN, frac: float = 0.05, sigma: float = 0.1,
                    seed: int = 0, dtype: str = "f64", c: float = SPACETIME_C,
                    damping: float = SPACETIME_ETA, **prior) -> SpaceTimeProblem:
    """Generic small space-time problem for tests: a plane-wave truth per slice,
    uniformly random observed space-time cells."""
    pr = dict(SPACETIME_PRIOR)
    pr.update(prior)
    rng = np.random.default_rng([seed, nx, ny, nt])
    truth = np.stack([fourier_modes_field(nx, ny, rng, n_modes=8, max_freq=3)
                      for _ in range(nt)])
    cells = uniform_cells(nx * ny * nt, frac, rng)
    y = observe(truth, cells, sigma, rng)
    return SpaceTimeProblem(f"small_st{nx}x{ny}x{nt}", nx, ny, nt, bc_x, bc_y, c=c,
                            sigma=sigma, cells=cells, y=y, truth=truth, dtype=dtype,
                            damping=damping, seed=seed, **pr)
