"""CPU oracle of the spatio-temporal extension (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the test suite, never by the GPU library
or its binding; shares no code with the GPU path.

The paper's appendix "Extension to Spatiotemporal Systems" turns a linear
SPDE discretised first-order in time,

    A u^{n+1} = B u^n + s z^{n+1},   u^0 = m + s L^{-1} z^0,   z ~ N(0, I),

into one GMRF over the space-time field (u^0, ..., u^N): stacking the
equations gives M u = [L m; 0; ...; 0] + s z with the block lower-bidiagonal
M (blocks L, then A on the diagonal and -B below it), so the prior precision
is Q = M^T M / s^2 and its shift vector b = [P m; 0; ...; 0] with
P = L^T L / s^2 the precision of the initial condition.

Here, as in the appendix's example, the SPDE is the stochastic heat equation
du/dt = nu Lap u + sigma W with the Crank-Nicolson scheme, A = I/dt -
(nu/2) Lap_h and B = I/dt + (nu/2) Lap_h, on a 2-D grid of spacing h
(5-point Laplacian; zero-flux or periodic axes, the readings of the spatial
path), and s^2 = sigma^2 / (dt h^2) (the appendix's dt dx with the cell area
h^2 of a 2-D grid).  Reading for the initial condition's factor, which the
appendix leaves open: L = a0 (kappa^2 I - Lap_h), a Matern-type field.

Functions:
* ``dynamics_matrix``: M by sparse blocks; ``prior``: Q and b by sparse
  products; ``posterior_system``: A = Q + H^T R^-1 H, b + H^T R^-1 y for
  point observations of (x, y, n) cells (cell index n nx ny + y nx + x).
* ``kalman_smoother``: the posterior mean of the same linear-Gaussian model
  by a forward Kalman filter and the Rauch-Tung-Striebel backward pass
  (dense covariances; tiny grids only) -- a computation that never forms Q.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import oracle as O


def laplacian_2d(nx: int, ny: int, h: float, bc_x: int, bc_y: int) -> sp.csr_matrix:
    """The 5-point Laplacian Lap_h = -(G_x + G_y) / h^2 (G: 1-D graph
    Laplacians of the oracle's spatial operator)."""
    gx = O.laplacian_1d(nx, bc_x)
    gy = O.laplacian_1d(ny, bc_y)
    G = sp.kron(sp.identity(ny), gx) + sp.kron(gy, sp.identity(nx))
    return sp.csr_matrix(-G / (h * h))


def dynamics_matrix(nx: int, ny: int, nt: int, dt: float, h: float, nu: float, kappa: float,
                    a0: float = 1.0, bc_x: int = O.BC_NEUMANN,
                    bc_y: int = O.BC_NEUMANN) -> sp.csr_matrix:
    """M for nt time slices (u^0 .. u^{nt-1}): block (0, 0) = L, blocks
    (n, n) = A and (n, n-1) = -B for n >= 1."""
    n = nx * ny
    lap = laplacian_2d(nx, ny, h, bc_x, bc_y)
    eye = sp.identity(n, format="csr")
    L0 = a0 * (kappa * kappa * eye - lap)
    A = eye / dt - 0.5 * nu * lap
    B = eye / dt + 0.5 * nu * lap
    rows = []
    for k in range(nt):
        row = [None] * nt
        if k == 0:
            row[0] = L0
        else:
            row[k - 1] = -B
            row[k] = A
        rows.append(row)
    return sp.csr_matrix(sp.bmat(rows, format="csr"))


def initial_factor(nx, ny, h, kappa, a0=1.0, bc_x=O.BC_NEUMANN, bc_y=O.BC_NEUMANN):
    lap = laplacian_2d(nx, ny, h, bc_x, bc_y)
    return sp.csr_matrix(a0 * (kappa * kappa * sp.identity(nx * ny) - lap))


def prior(nx, ny, nt, dt, h, nu, kappa, sigma, a0=1.0, bc_x=O.BC_NEUMANN, bc_y=O.BC_NEUMANN,
          m: Optional[np.ndarray] = None):
    """(Q, b): Q = M^T M / s^2 with s^2 = sigma^2 / (dt h^2), b = [P m; 0 ...]
    with P = L^T L / s^2 (zero when m is None)."""
    M = dynamics_matrix(nx, ny, nt, dt, h, nu, kappa, a0, bc_x, bc_y)
    inv_s2 = dt * h * h / (sigma * sigma)
    Q = sp.csr_matrix(inv_s2 * (M.T @ M))
    Q.sum_duplicates()
    Q.eliminate_zeros()
    Q.sort_indices()
    b = np.zeros(nx * ny * nt)
    if m is not None:
        L0 = initial_factor(nx, ny, h, kappa, a0, bc_x, bc_y)
        b[: nx * ny] = inv_s2 * (L0.T @ (L0 @ np.asarray(m, float).ravel()))
    return Q, b


def posterior_system(prob, m: Optional[np.ndarray] = None):
    """(A, b) of a space-time problem: prior plus point observations."""
    Q, b = prior(prob.nx, prob.ny, prob.nt, prob.dt, prob.h, prob.nu, prob.kappa, prob.sigma_u,
                 prob.a0, prob.bc_x, prob.bc_y, m)
    p, hh = O.observation_terms(prob.nx * prob.ny * prob.nt, prob.cells, prob.y, prob.sigma,
                                prob.var)
    A = sp.csr_matrix(Q + sp.diags(p))
    A.sort_indices()
    return A, b + hh


def kalman_smoother(prob, m: Optional[np.ndarray] = None) -> np.ndarray:
    """Posterior mean of the linear-Gaussian state-space model behind the
    space-time prior: state u^n, u^0 ~ N(m, P^-1), u^{n+1} = F u^n + w with
    F = A^-1 B and w ~ N(0, s^2 A^-1 A^-T), observations y = u^n[cell] +
    N(0, sigma_y^2) at slice n.  Forward Kalman filter, then the
    Rauch-Tung-Striebel smoother (dense algebra: tiny grids)."""
    nx, ny, nt = prob.nx, prob.ny, prob.nt
    n = nx * ny
    lap = laplacian_2d(nx, ny, prob.h, prob.bc_x, prob.bc_y).toarray()
    eye = np.eye(n)
    A = eye / prob.dt - 0.5 * prob.nu * lap
    B = eye / prob.dt + 0.5 * prob.nu * lap
    s2 = prob.sigma_u ** 2 / (prob.dt * prob.h ** 2)
    Ainv = np.linalg.inv(A)
    F = Ainv @ B
    Qw = s2 * Ainv @ Ainv.T
    L0 = prob.a0 * (prob.kappa ** 2 * eye - lap)
    P0 = (L0.T @ L0) / s2
    mean = np.zeros(n) if m is None else np.asarray(m, float).ravel()
    cov = np.linalg.inv(P0)
    var = np.full(prob.cells.size, prob.sigma ** 2) if prob.var is None else np.asarray(prob.var)
    slice_of = prob.cells // n
    means_f, covs_f, means_p, covs_p = [], [], [], []
    for k in range(nt):
        if k > 0:
            mean = F @ mean
            cov = F @ cov @ F.T + Qw
        means_p.append(mean.copy())
        covs_p.append(cov.copy())
        # update with this slice's observations, one at a time
        for j in np.nonzero(slice_of == k)[0]:
            c = int(prob.cells[j] % n)
            S = cov[c, c] + var[j]
            K = cov[:, c] / S
            mean = mean + K * (prob.y[j] - mean[c])
            cov = cov - np.outer(K, cov[c, :])
        means_f.append(mean.copy())
        covs_f.append(cov.copy())
    smooth = [None] * nt
    smooth[-1] = means_f[-1]
    for k in range(nt - 2, -1, -1):
        G = covs_f[k] @ F.T @ np.linalg.inv(covs_p[k + 1])
        smooth[k] = means_f[k] + G @ (smooth[k + 1] - means_p[k + 1])
    return np.concatenate(smooth)
