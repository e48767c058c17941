/*
 * gabp_st.h -- C ABI of the space-time solver: Gaussian belief propagation on
 * the Gaussian Markov random field of a linear stochastic PDE discretised in
 * space and time (paper: Appendix "Extension to Spatiotemporal Systems").
 *
 * Model.  The stochastic heat equation du/dt = nu Lap u + sigma_u W on an
 * nx x ny grid of spacing h (5-point Laplacian Lap_h, zero-flux or periodic
 * axes), Crank-Nicolson steps of length dt (the appendix's example):
 *     A u^{n+1} = B u^n + s z^{n+1},  A = I/dt - (nu/2) Lap_h,
 *                                     B = I/dt + (nu/2) Lap_h,
 * s^2 = sigma_u^2 / (dt h^2), and an initial condition u^0 ~ N(m, P^-1) with
 * P = L^T L / s^2, L = a0 (kappa^2 I - Lap_h).  Stacking the nt slices
 * u^0 .. u^{nt-1} gives M u = [L m; 0; ...] + s z with M block lower
 * bidiagonal (L, then A on the diagonal, -B below it), hence the prior
 * precision Q = M^T M / s^2 and shift b = [P m; 0; ...] (same appendix).
 * Point observations y_k ~ N(u[cell_k], s_k^2) give the posterior precision
 * Q + H^T R^-1 H and information b + H^T R^-1 y.
 *
 * Q couples each node with 38 others: 12 in its own slice (the 13-point
 * stencil of Lap_h^2) and 13 in each neighbouring slice.  Directions
 * d = 0 .. 37, offset (dx, dy, dt):
 *     0 .. 11   (dx, dy, 0) in the order of gabp.h's 12 lattice directions;
 *     12 + 2k   (ox_k, oy_k, +1),  13 + 2k  (-ox_k, -oy_k, -1),  k = 0 .. 12,
 *               with o_0 = (0, 0) and o_k for k >= 1 gabp.h's direction k - 1.
 * The opposite direction of d is d ^ 1.  Space-time cells are
 * n * nx * ny + y * nx + x for slice n.
 *
 * The solver is the same damped, re-weighted flooding GaBP as gabp.h's
 * (Algorithm 2's inner loop; Appendix "Re-weighted message updates"; Section
 * "Update Damping"), on this graph.  The precisions are not stored: kernels
 * evaluate every Q_ij from (dt, h, nu, kappa, a0, sigma_u), the position and
 * the slice.  Conventions (status codes, device memory, streams, error text,
 * no exceptions, one device and stream per context) are gabp.h's.
 */
#ifndef GABP_ST_H
#define GABP_ST_H

#include <stddef.h>
#include <stdint.h>

#include "gabp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gabp_st_ctx gabp_st_ctx;

/* Space-time grid and heat-equation prior.  nx, ny >= 1 (>= 5 on a periodic
 * axis, where the 13-point stencil would alias), nt >= 1, nx*ny*nt < 2^31;
 * bc_x, bc_y GABP_BC_NEUMANN or GABP_BC_PERIODIC; dt, h, sigma_u > 0,
 * nu >= 0, a0 > 0 and kappa > 0 (L must be invertible: the Laplacian of
 * zero-flux and periodic axes has the constant mode); c != 0 and finite, the
 * re-weighting constant. */
typedef struct {
    int32_t nx, ny, nt;
    int32_t bc_x, bc_y;
    double dt, h, nu, kappa, a0, sigma_u;
    double c;
} gabp_st_model;

/* Create a context: fold the observations (gabp_obs / gabp_noise as in
 * gabp.h, cells indexing the space-time grid; several observations of one
 * cell add in the order given, so the result does not depend on thread
 * timing), the prior mean m of the first slice (device, nx*ny FP64 values,
 * or NULL for zero) and the prior diagonal into FP64 node terms, and set
 * every message to zero.  dtype: message precision (GABP_F32 / GABP_F64).
 * stream: the hipStream_t of every call (NULL = default stream).  The library
 * allocates its device memory (two message buffers of 76 planes, 38 gain
 * planes, node terms, reduction scratch: gabp_st_workspace_size bytes).  INVALID on the first
 * bad argument (text in gabp_st_create_error). */
gabp_status gabp_st_create(const gabp_st_model *model, const gabp_obs *obs,
                           const gabp_noise *noise, const double *prior_mean,
                           int32_t dtype, void *stream, gabp_st_ctx **out);

/* Device bytes a context of this model and dtype allocates. */
gabp_status gabp_st_workspace_size(const gabp_st_model *model, int32_t dtype, size_t *bytes);

/* Text of the last failed gabp_st_create on this thread. */
const char *gabp_st_create_error(void);

/* n_iters flooding iterations with damping in (0, 1] (as gabp_iterate).
 * A cavity precision <= 0 or a non-finite value records the iteration on the
 * device; later launches write nothing and the next synchronising call
 * returns DIVERGED.  Asynchronous. */
gabp_status gabp_st_iterate(gabp_st_ctx *ctx, int32_t n_iters, double damping);

/* FP64 residual ||A mu - b||_2 of the posterior mean (rel: divided by
 * ||b||_2).  Either pointer may be NULL.  Synchronises.  Also runs the freeze
 * test of the precision messages (gabp_st_set_freeze_tolerance). */
gabp_status gabp_st_residual(gabp_st_ctx *ctx, double *rel_residual, double *abs_residual);

/* Iterate until the relative residual is <= rel_tol (OK), max_iters
 * iterations were run by this call (NOT_CONVERGED) or the run diverged
 * (DIVERGED), checking every check_every > 0 iterations. */
gabp_status gabp_st_solve(gabp_st_ctx *ctx, int64_t max_iters, double damping, double rel_tol,
                          int32_t check_every, int64_t *iters_done, double *rel_residual);

/* Posterior mean and approximate marginal variance of every space-time cell
 * (Compute Marginal): mean = th / Lam and var = 1 / Lam of the beliefs
 * Lam = A_ii + c sum Lam_{k->i}, th = b_i + c sum th_{k->i}.  Device FP64
 * arrays of nx*ny*nt values, either may be NULL.  Asynchronous. */
gabp_status gabp_st_posterior(gabp_st_ctx *ctx, double *mean, double *var);

/* Current messages, receiver-indexed: prec[d][n][y][x] and info[d][n][y][x]
 * hold the message INTO (x, y, n) FROM (x, y, n) + off_d; slots without a
 * sender are zero.  Device arrays of 38*nx*ny*nt values of the message
 * dtype.  Asynchronous. */
gabp_status gabp_st_get_messages(gabp_st_ctx *ctx, void *prec, void *info);

/* Freeze tolerance of the precision messages (as gabp_set_freeze_tolerance):
 * the precision recursion involves neither the information messages nor the
 * data, so once an iteration leaves every precision message unchanged (tested
 * at each gabp_st_residual after the first iteration), later iterations store
 * the edge gains once and update only the information messages -- bitwise
 * the same results, 12 instead of 16 bytes per FP32 edge.  With max_slots > 0
 * the precisions also freeze when at most max_slots of them changed, each by
 * at most max_rel relative to the larger value (both buffers then keep the
 * current precisions).  INVALID for max_slots < 0 or a negative or
 * non-finite max_rel. */
gabp_status gabp_st_set_freeze_tolerance(gabp_st_ctx *ctx, int64_t max_slots, double max_rel);

/* Multigrid transfer on the space-time lattice (Alg. 2, Upscale Messages,
 * read as in gabp.h's gabp_upsample_mean: the finer level starts from the
 * coarser level's marginals).  A coarse level keeps every second node of x, y
 * and t: coarse node (X, Y, N) sits on fine node (2X, 2Y, 2N), so
 * nxc = ceil(nx/2), nyc = ceil(ny/2), ntc = ceil(nt/2).  Writes fine
 * [nt][ny][nx] (FP64, device) with the trilinear interpolation of coarse
 * [ntc][nyc][nxc] (FP64, device): a fine coordinate between two coarse nodes
 * takes their average, one past the last coarse node of a zero-flux axis or
 * of t takes that node's value, a periodic axis wraps (and needs an even fine
 * size).  Async on `stream`; INVALID on a size or boundary mismatch (text in
 * gabp_st_create_error). */
gabp_status gabp_st_upsample_mean(const double *coarse, int32_t nxc, int32_t nyc, int32_t ntc,
                                  int32_t bc_x, int32_t bc_y, double *fine, int32_t nx,
                                  int32_t ny, int32_t nt, void *stream);

/* Warm start from a predicted posterior mean mu (device, FP64 [nt][ny][nx]):
 * every precision message is set to zero and every information message to
 * th_{i->j} = -(Q_ij/c) mu_i, so that the beliefs start at
 * mu + (b - A mu) / diag(A) -- mu itself when it is the posterior mean.  The
 * freeze test starts afresh.  DIVERGED after a divergence.  Async. */
gabp_status gabp_st_warm_init(gabp_st_ctx *ctx, const double *mean);

/* Launch shape of the information-only iteration: a workgroup covers one
 * 64 x 4 tile on `slices` consecutive slices (1, 2 or 4; default 1), so the
 * messages passing between those slices are read twice inside one
 * workgroup.  Results do not depend on it.  INVALID for other values. */
gabp_status gabp_st_set_theta_slices(gabp_st_ctx *ctx, int32_t slices);

/* Iteration at which the precision messages froze, or -1. */
gabp_status gabp_st_precision_frozen(gabp_st_ctx *ctx, int64_t *frozen_at);

/* Iterations run so far and the first invalid iteration (0: none).
 * Synchronises. */
gabp_status gabp_st_iteration_count(gabp_st_ctx *ctx, int64_t *iters, int64_t *diverged_at);

/* Text of the context's last error. */
const char *gabp_st_last_error(gabp_st_ctx *ctx);

/* Release the context (NULL is ignored). */
void gabp_st_destroy(gabp_st_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GABP_ST_H */
