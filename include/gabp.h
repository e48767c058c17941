/*
 * gabp.h -- C ABI of the MI355X (gfx950) lattice Gaussian belief propagation
 * library for data assimilation on a Gaussian Markov random field.
 *
 * Model (paper: Section "Derivation of the Factor Graph", Section "Including
 * Observations", Appendix "Details on the Finite Difference Discretisation"):
 *   prior      f ~ N(0, Q^-1),  Q = tau * (kappa^2 I - Delta_h)^alpha, alpha in {1, 2},
 *              Delta_h the 5-point finite-difference Laplacian on an nx x ny grid
 *              (alpha = 1 gives a 5-point, alpha = 2 a 13-point precision stencil);
 *   likelihood y_k ~ N(f[cell_k], s_k^2) at observed grid cells;
 *   posterior  precision A = Q + H^T R^-1 H, information b = H^T R^-1 y (+ Q f_b).
 * The library runs damped, re-weighted Gaussian belief propagation with a
 * flooding schedule (Algorithms 1 and 2, inner procedure; Appendix sections
 * "Gaussian Setting" and "Re-weighted message updates"; Section "Update
 * Damping") and returns the posterior mean and approximate marginal variances
 * (Compute Marginal).
 *
 * Conventions
 *   - Grid cells are row-major, cell = y * nx + x, 0 <= x < nx, 0 <= y < ny.
 *   - All arrays named "device" live in device memory of the context's GPU.
 *   - Messages are in information form: a message into node i is the pair
 *     (Lam, th) standing for exp(-1/2 Lam x^2 + th x).
 *   - Stencil directions (deg = 4 for alpha = 1, 12 for alpha = 2), offset (dx, dy):
 *       0 (+1, 0)   1 (-1, 0)   2 (0, +1)   3 (0, -1)
 *       4 (+2, 0)   5 (-2, 0)   6 (0, +2)   7 (0, -2)
 *       8 (+1, +1)  9 (-1, -1) 10 (+1, -1) 11 (-1, +1)
 *     Plane d at cell (x, y) holds the message INTO (x, y) FROM
 *     (x + dx, y + dy); the opposite direction of d is d ^ 1.  Slots whose
 *     sender lies outside the grid (non-periodic axes) are always zero.
 *   - Every call returns a gabp_status; the library never aborts and never
 *     throws across this interface.  gabp_last_error() gives a text.
 *   - A context is bound to one device and one stream and is not thread-safe.
 */
#ifndef GABP_H
#define GABP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gabp_ctx gabp_ctx;

typedef enum {
    GABP_OK = 0,
    GABP_E_INVALID = 1,       /* an argument is out of its documented range */
    GABP_E_NOMEM = 2,         /* device or host allocation failed, or workspace too small */
    GABP_E_DEVICE = 3,        /* a HIP runtime call failed */
    GABP_E_DIVERGED = 4,      /* non-positive cavity precision, non-finite values, or residual blow-up */
    GABP_E_NOT_CONVERGED = 5  /* max_iters reached before rel_tol */
} gabp_status;

typedef enum {
    GABP_BC_NEUMANN = 0,   /* zero flux: graph Laplacian of the path (not in the paper; see reading) */
    GABP_BC_PERIODIC = 1,  /* ghost points wrap (Appendix, discretisation) */
    GABP_BC_DIRICHLET = 2  /* boundary values zero and removed (Appendix, discretisation) */
} gabp_bc;

typedef enum { GABP_F32 = 0, GABP_F64 = 1 } gabp_dtype;  /* message-plane precision */

/* Grid: nx x ny cells with spacings hx, hy > 0 and one boundary type per axis. */
typedef struct {
    int64_t nx, ny;
    double hx, hy;
    int32_t bc_x, bc_y;   /* gabp_bc */
} gabp_grid;

/* Prior Q = tau (kappa^2 I - Delta_h)^alpha (Section "Derivation of the Factor
 * Graph", the discretised SPDE) and the re-weighting constant c of the
 * message updates (Appendix, "Re-weighted message updates"); c = 1 is plain
 * Gaussian belief propagation. */
typedef struct {
    int32_t alpha;        /* 1 or 2 */
    double kappa;         /* > 0 unless an axis is Dirichlet (then >= 0) */
    double tau;           /* > 0 */
    double c;             /* != 0, finite */
} gabp_stencil;

/* Point observations (Section "Including Observations"): y[k] observes cell
 * cell[k].  Several observations of one cell multiply their likelihoods.
 * cell and y are device pointers when on_device != 0, else host pointers.
 * Copied (folded into node terms) at create; the caller keeps ownership. */
typedef struct {
    int64_t n;
    const int64_t *cell;
    const double *y;
    int32_t on_device;
} gabp_obs;

/* Observation noise: variance sigma^2 for every observation, or var[k] when
 * var != NULL (same memory space as the observations). */
typedef struct {
    double sigma;
    const double *var;
} gabp_noise;

/* Options.  stream: the hipStream_t every call of the context is ordered on
 * (NULL = the device's default stream).  workspace: device memory of at least
 * gabp_workspace_size() bytes, owned by the caller and not freed by the
 * library (NULL = the library allocates and frees its own).  prior_mean: a
 * device array of nx*ny FP64 values f_b, or NULL for a zero prior mean. */
typedef struct {
    int32_t dtype;        /* gabp_dtype */
    void *stream;
    void *workspace;
    size_t workspace_bytes;
    const double *prior_mean;
} gabp_opts;

/* Bytes of device workspace a context needs for this grid, prior order and
 * message precision: two message buffers (ping-pong) of 2*deg planes, the
 * node planes and reduction scratch.  INVALID for bad grid/stencil/dtype. */
gabp_status gabp_workspace_size(const gabp_grid *grid, const gabp_stencil *stencil,
                                int32_t dtype, size_t *bytes);

/* Build the factor graph of the posterior (Section "Derivation of the Factor
 * Graph": one node per cell, an edge wherever Q_ij != 0, node factor from
 * Q_ii and the observations) and set every message to zero (iteration 0).
 * The off-diagonal precisions are not stored: kernels evaluate them from
 * (alpha, kappa, tau, h, boundary, position).  Validates every argument
 * (sizes >= 1; a periodic axis needs >= 3 cells for alpha = 1 and >= 5 for
 * alpha = 2, where the stencil would alias; finite y and positive noise;
 * cells in range) and returns INVALID on the first violation.  On success
 * *out receives a context to be released with gabp_destroy. */
gabp_status gabp_create(const gabp_grid *grid, const gabp_stencil *stencil,
                        const gabp_obs *obs, const gabp_noise *noise,
                        const gabp_opts *opts, gabp_ctx **out);

/* Run n_iters flooding iterations (Algorithm 2, inner loop): every new
 * message is computed from the previous iteration's messages, then damped,
 * m^t = (1 - damping) m^{t-1} + damping * m~ (Section "Update Damping"),
 * damping in (0, 1].  Asynchronous on the context's stream.  n then m
 * iterations give bitwise the same state as n + m.  A divergence is recorded
 * on the device at the first invalid iteration; later launches write nothing,
 * so the messages kept are those of the launch that produced it (the
 * iteration itself, or the second iteration of a two-iteration launch; see
 * gabp_set_tile), and the next synchronising call reports GABP_E_DIVERGED
 * and names both iterations in gabp_last_error. */
gabp_status gabp_iterate(gabp_ctx *ctx, int32_t n_iters, double damping);

/* Iterate in chunks until the FP64 relative residual ||A mu - b||_2 / ||b||_2
 * of the posterior mean is <= rel_tol (returns OK), max_iters iterations
 * were run by this call (NOT_CONVERGED), or the run diverged (DIVERGED:
 * invalid cavity precision, non-finite values, or a residual more than 1e3
 * times the first check's).  check_every > 0 checks every check_every
 * iterations; check_every < 0 checks adaptively: every |check_every|
 * iterations until the precision messages froze, then after half the
 * iterations the observed geometric rate predicts to rel_tol (at least
 * |check_every|, at most 2000; with graphs on, rounded down to
 * |check_every| * 2^j).  Each chunk of iterations is recorded once as a
 * hipGraph (per chunk length, starting buffer, phase, tile shape and
 * damping) and replayed (see gabp_set_graph).  Once the precision messages
 * froze, a chunk may end on a two-iteration launch, so that afterwards the
 * two buffers need not hold consecutive iterations: gabp_message_change then
 * returns INVALID until gabp_iterate has run.  iters_done (total iterations
 * of the context) and rel_residual (last residual) may be NULL.
 * Synchronises the stream at every check. */
gabp_status gabp_solve(gabp_ctx *ctx, int64_t max_iters, double damping, double rel_tol,
                       int32_t check_every, int64_t *iters_done, double *rel_residual);

/* FP64 residual of the posterior mean of the current messages: abs = ||A mu - b||_2
 * and rel = abs / ||b||_2 (rel = abs when b = 0).  Either pointer may be NULL.
 * Synchronises the stream.  Returns DIVERGED if the run has diverged.
 * Also tests whether the last iteration left every precision message bitwise
 * unchanged; the precision recursion involves neither the information
 * messages nor the data, so they then stay fixed for ever and later
 * iterations update only the information messages, with precomputed edge
 * gains (bitwise the same results, 12 instead of 16 bytes per FP32 edge).
 * See gabp_set_freeze_tolerance for a relaxed form of that test. */
gabp_status gabp_residual(gabp_ctx *ctx, double *rel_residual, double *abs_residual);

/* Freeze tolerance of the precision messages.  In FP32 the precision
 * recursion can settle to a state where a few messages keep changing in
 * their last bits for ever, and then never freezes under the bitwise test
 * of gabp_residual.  With max_slots > 0, the precision messages also freeze
 * when the last iteration changed at most max_slots of them, each by at most
 * max_rel relative to the larger of its two values; the edge gains are then
 * taken from the current messages (which both message buffers keep from
 * then on, as after a bitwise freeze), and later results differ from those of
 * the unfrozen iteration by amounts of the order of those last-bit changes
 * (convergence is still decided by the FP64 residual).  max_slots = 0 (the
 * default) keeps the bitwise test.  INVALID for max_slots < 0 or a max_rel
 * that is negative or not finite.  Applies from the next residual check;
 * an already frozen context stays frozen. */
gabp_status gabp_set_freeze_tolerance(gabp_ctx *ctx, int64_t max_slots, double max_rel);

/* The paper's stopping rule (Alg. 2, Iterate MP Until Convergence, with the
 * Early Stop of Appendix A): iterate until mean|m^t - m^{t-1}| <
 * tau * mean|m^2 - m^1| (both components of every directed message, m^1 and
 * m^2 the context's first two iterations; the paper takes tau = 1e-3), with
 * at most max_iters iterations in this call (the paper's T; NOT_CONVERGED
 * when reached, which the paper treats as a normal end), or until the run
 * diverges (DIVERGED).  check_every > 0: the statistic every check_every
 * iterations; < 0: adaptively, every |check_every| iterations until the
 * precision messages froze (with a residual check, which detects the
 * freeze), then after half the iterations the ratio's observed geometric
 * decay predicts to tau (at least |check_every|, at most 2000).  iters_done
 * and ratio (the last statistic) may be NULL.  Synchronises at every check. */
gabp_status gabp_solve_early_stop(gabp_ctx *ctx, int64_t max_iters, double damping, double tau,
                                  int32_t check_every, int64_t *iters_done, double *ratio);

/* Marginals of the current messages (Compute Marginal): belief precision
 * Lam_i = A_ii + c sum Lam_{k->i}, information th_i = b_i + c sum th_{k->i}
 * accumulated in FP64; mean[i] = th_i / Lam_i, var[i] = 1 / Lam_i.  mean and
 * var are caller-owned device arrays of nx*ny FP64 (row-major); either may be
 * NULL.  Asynchronous on the context's stream. */
gabp_status gabp_posterior(gabp_ctx *ctx, double *mean, double *var);

/* The paper's early-stopping statistic (Appendix, Early Stop):
 * mean|m^t - m^{t-1}| / mean|m^2 - m^1| over both components of every
 * directed message.  Needs t >= 2 reached by gabp_iterate/gabp_solve since
 * create (else INVALID).  Synchronises the stream. */
gabp_status gabp_message_change(gabp_ctx *ctx, double *ratio);

/* Copy the current messages out to (get) or in from (set) caller-owned device
 * arrays prec and info, each deg*ny*nx values of the context's dtype, layout
 * [deg][ny][nx] (receiver-indexed, see the conventions above).  get writes 0
 * in slots without a sender; set ignores them and keeps the iteration
 * counter.  Used for checkpoint/resume and warm starts.  Async. */
gabp_status gabp_get_messages(gabp_ctx *ctx, void *prec, void *info);
gabp_status gabp_set_messages(gabp_ctx *ctx, const void *prec, const void *info);

/* Autotuner: after one untimed iteration, run `trials` iterations with each
 * tile shape of the active iteration kernel (rows per thread 1, 2, 4, 8),
 * twice over, time them with HIP events on the context's stream, and keep
 * the fastest for this context and for later contexts of the same prior
 * order, dtype and size class in this process.  Once the precision messages
 * have frozen, the two-iteration tile kernel (tile heights 4, 8, 12, 16 and
 * 32 in FP32, 4 in FP64; see gabp_set_tile) is timed against the best of those,
 * twice over, and the fastest kept (the column-strip walker is not timed).
 * Every shape computes bitwise-identical messages, so these are ordinary
 * iterations: the counter advances by 1 + 8 * trials, plus 10 * trials (FP32)
 * or 2 * trials (FP64) when frozen.  *chosen (may be NULL) receives the rows
 * per thread.  Synchronises. */
gabp_status gabp_autotune(gabp_ctx *ctx, int32_t trials, double damping, int32_t *chosen);

/* Chunk graphs of gabp_solve and gabp_solve_early_stop (Alg. 2, Iterate MP
 * Until Convergence: chunks of iterations between checks): enable != 0
 * (default) records each chunk of at least 2 iterations, once the context has
 * run 2 iterations, as a hipGraph on an internal stream and replays it on the
 * context's stream (iteration numbers come from a device counter the graph
 * advances); 0 launches every kernel directly and drops recorded graphs.
 * Results are bitwise identical either way.  gabp_iterate always launches
 * directly. */
gabp_status gabp_set_graph(gabp_ctx *ctx, int32_t enable);

/* Tile configuration of a context's iteration kernels, a tuning knob that
 * never changes results.  rows_per_thread (1, 2, 4 or 8): rows each thread
 * of a 64-wide, 256-thread tile walks, for the single-iteration kernels.
 * pair_rows: once the precision messages have frozen, gabp_iterate runs
 * two information-only iterations per launch (one HBM pass per two
 * iterations) and the last one or two iterations of each call singly.
 * pair_rows > 0 (4, or 8, 12, 16 and 32 for FP32 only): on independent
 * 64 x pair_rows tiles (iteration t+1 of the tile and a halo of the stencil
 * radius kept in LDS, iteration t+2 written out; tiles whose halo crosses
 * the grid's edge take the general code path, in the same launch); pair_rows < 0 (-2, or -4
 * and -8 for FP32 only): persistent workgroups walk 64-column strips
 * downwards in bands of -pair_rows rows, keeping iteration t+1 of the rows
 * the next band needs in LDS; 0 = always one iteration per launch.
 * Default: rows 4, pair 8 (FP32) or 4 (FP64), or what the autotuner chose
 * for this problem class.  INVALID for other values. */
gabp_status gabp_set_tile(gabp_ctx *ctx, int32_t rows_per_thread, int32_t pair_rows);
gabp_status gabp_get_tile(const gabp_ctx *ctx, int32_t *rows_per_thread, int32_t *pair_rows);

/* Learned warm start: set the current messages from a prediction pred, a
 * device array [ny][nx][16] of FP32 (channel 0 the posterior mean mu^,
 * channels 1..deg the log(-Lam^) of the precision message from the cell to
 * its neighbour in direction d-1).  Lam_{i->j} = -exp(pred), and
 * th_{i->j} = Lam_{i->j} mu^_j - (Q_ij / c) mu^_i, the information message
 * that makes every edge consistent with mu^ (with exact means and converged
 * precisions this is the fixed point; otherwise the beliefs start at
 * mu^_i + (b - A mu^)_i / Lam_i).  keep_precisions != 0 keeps the current
 * precision messages.  The iteration counter is kept.  Async. */
gabp_status gabp_warm_init(gabp_ctx *ctx, const float *pred, int32_t keep_precisions);

/* Training targets of the learned warm start's precision outputs from the
 * current messages: lam [12][ny][nx] (FP32, device) receives log(-Lam) of the
 * message from each cell to its neighbour in direction d (-Lam floored at
 * 1e-30), and valid [12][ny][nx] (FP32, device, may be NULL) 1 where that
 * neighbour exists; both 0 elsewhere and for d >= deg.  These are the
 * channels 1..12 gabp_warm_init reads.  Async. */
gabp_status gabp_log_precisions(gabp_ctx *ctx, float *lam, float *valid);

/* Multigrid transfer (Alg. 2, Upscale Messages, read as initialising the
 * finer grid's marginals to the coarser grid's): writes into channel 0 of a
 * prediction pred [nyf][nxf][16] (FP32, other channels 0) the bilinear
 * interpolation of a coarse mean coarse [nyc][nxc] (FP64) whose node (i, j)
 * sits on fine node (2i, 2j); nxc = ceil(nxf/2), nyc = ceil(nyf/2); periodic
 * axes wrap (and need even fine sizes).  Feed pred to gabp_warm_init with
 * keep_precisions = 1.  Device arrays; async on `stream`; errors via
 * gabp_last_error(NULL). */
gabp_status gabp_upsample_mean(const double *coarse, int64_t nxc, int64_t nyc, int32_t bc_x,
                               int32_t bc_y, float *pred, int64_t nxf, int64_t nyf, void *stream);

/* Multigrid transfer of the precision messages (Alg. 2, Upscale Messages:
 * the finer grid's edge values start from the coarser grid's).  For every
 * node (x, y) of a fine grid nxf x nyf with ceil(nxf/2) x ceil(nyf/2) = the
 * coarse context's grid, writes channels 1..deg of pred [nyf][nxf][16]
 * (FP32, device) with log(scale * -Lam) of the coarse context's current
 * precision message from node (x/2, y/2) in the same direction (the opposite
 * direction where the coarse node has none in that direction; -inf, a zero
 * message, where it has neither).  Channel 0 and the channels past deg are
 * not written: fill channel 0 with gabp_upsample_mean first, then pass pred
 * to the fine context's gabp_warm_init with keep_precisions = 0.  The paper
 * gives no rescaling between levels; halving h with tau scaled by 4 scales
 * the prior's off-diagonal entries by 4^(1-alpha), so scale = 4^(alpha-1)
 * brings the coarse messages to the fine scale.  Async on the coarse
 * context's stream; INVALID on a size mismatch, a NULL pred or a scale that
 * is not finite and positive. */
gabp_status gabp_upscale_precisions(gabp_ctx *coarse, float *pred, int64_t nxf, int64_t nyf,
                                    double scale);

/* Multigrid transfer, the paper's Upscale Messages taken literally (Alg. 2):
 * every message of the fine context (both components), for each fine node
 * (x, y) and direction d whose fine neighbour exists, is set to the coarse
 * context's current message from node (x/2, y/2) in direction d (the
 * opposite direction where the coarse node has none in d, zero where it has
 * neither), unscaled; the fine context's other slots stay zero.  The
 * contexts must share device, dtype, alpha and boundary types, with
 * ceil(nx_fine/2) = nx_coarse and ceil(ny_fine/2) = ny_coarse (INVALID
 * otherwise).  Synchronises the coarse stream, then runs on the fine
 * context's stream; the fine context starts its freeze test afresh. */
gabp_status gabp_copy_coarse_messages(gabp_ctx *coarse, gabp_ctx *fine);

/* Iteration kernels launched by this context so far (graph replays
 * included): one-iteration launches of the full update (full) and of the
 * information-only update once the precision messages froze (theta), and
 * two-iteration launches on independent tiles (pair_tiles) and by the
 * column-strip walker (pair_walk); see gabp_set_tile.  Any pointer may be
 * NULL.  Does not synchronise; counts launches issued, not completed. */
gabp_status gabp_launch_counts(const gabp_ctx *ctx, int64_t *full, int64_t *theta,
                               int64_t *pair_tiles, int64_t *pair_walk);

/* Iteration at which the precision messages were found frozen, or -1. */
gabp_status gabp_precision_frozen(const gabp_ctx *ctx, int64_t *at);

/* Iterations applied so far (synchronises).  After a divergence: returns
 * DIVERGED and the iteration of the kept messages (see gabp_iterate). */
gabp_status gabp_iteration_count(gabp_ctx *ctx, int64_t *iters);

/* Number of stencil directions (4 or 12) of a context. */
int32_t gabp_num_directions(const gabp_ctx *ctx);

/* Release a context (frees only what the library allocated). NULL is a no-op. */
void gabp_destroy(gabp_ctx *ctx);

const char *gabp_status_string(gabp_status status);

/* ------------------------------------------------------------------------
 * Batched solving of many independent lattice problems of uneven sizes in
 * one workspace.  One iteration of the whole batch is one launch of a
 * persistent-grid kernel over a work list of (instance, tile) items of the
 * instances still running; instances that converge or diverge retire from
 * the list; each instance switches to the information-only iteration when
 * its precision messages freeze.  A chunk of check_every iterations plus the
 * per-instance FP64 check is captured in a hipGraph and replayed while the
 * running set is unchanged.  Every instance computes bitwise what a lone
 * context with the same arguments computes.  The same damping applies to
 * every instance; c and the prior are per instance.  The batch orders its
 * work on an internal stream joined to opts->stream (NULL: the default
 * stream) at every call, so calls are stream-ordered with the caller's work.
 * ------------------------------------------------------------------------ */
typedef struct gabp_batch gabp_batch;

typedef struct {
    gabp_grid grid;
    gabp_stencil stencil;
    gabp_obs obs;
    gabp_noise noise;
} gabp_instance;

/* Workspace bytes for n instances (INVALID names the first bad instance). */
gabp_status gabp_batch_workspace_size(int32_t n, const gabp_instance *inst, int32_t dtype,
                                      size_t *bytes);

/* Create a batch: validates every instance as gabp_create does, folds the
 * observations into node terms, zeroes all messages.  opts->prior_mean must
 * be NULL.  Synchronises. */
gabp_status gabp_batch_create(int32_t n, const gabp_instance *inst, const gabp_opts *opts,
                              gabp_batch **out);

/* n_iters iterations of every running instance (asynchronous). */
gabp_status gabp_batch_iterate(gabp_batch *b, int32_t n_iters, double damping);

/* Iterate every running instance in chunks of check_every and check each
 * one's FP64 relative residual after every chunk; an instance retires when
 * it reaches rel_tol (status OK), diverges (DIVERGED, same rules as
 * gabp_solve), or the call has run max_iters iterations (NOT_CONVERGED).
 * check_every < 0 sizes chunks adaptively: |check_every| until every running
 * instance's precision messages froze, then the largest |check_every| * 2^j
 * (at most 1280) not above half the iterations the slowest running
 * instance's observed residual decay predicts to rel_tol.
 * Per-instance results go to the caller's host arrays of n entries (each
 * may be NULL).  Returns OK when every instance converged, else
 * NOT_CONVERGED.  Synchronises at every check. */
gabp_status gabp_batch_solve(gabp_batch *b, int64_t max_iters, double damping, double rel_tol,
                             int32_t check_every, int64_t *iters_done, double *rel_residual,
                             int32_t *status);

/* Marginals / checkpoint copy of instance i, as gabp_posterior and
 * gabp_get_messages (device arrays of that instance's size). */
gabp_status gabp_batch_posterior(gabp_batch *b, int32_t i, double *mean, double *var);
gabp_status gabp_batch_get_messages(gabp_batch *b, int32_t i, void *prec, void *info);

/* Tile-shape autotuner of the batched iteration, as gabp_autotune (advances
 * every running instance by 1 + 8 * trials iterations). */
gabp_status gabp_batch_autotune(gabp_batch *b, int32_t trials, double damping, int32_t *chosen);

/* gabp_warm_init for instance i of a batch (its current messages; the
 * prediction has the instance's own nx, ny): the instance's freeze state is
 * reset.  Asynchronous on the batch's stream.  INVALID for an index out of
 * range or a NULL pred, DIVERGED for an instance that diverged. */
gabp_status gabp_batch_warm_init(gabp_batch *b, int32_t i, const float *pred,
                                 int32_t keep_precisions);

/* gabp_log_precisions for instance i of a batch (arrays of its own size).
 * Asynchronous on the batch's stream; INVALID for an index out of range or a
 * NULL lam. */
gabp_status gabp_batch_log_precisions(gabp_batch *b, int32_t i, float *lam, float *valid);

/* gabp_upscale_precisions from instance i of a batch (as the coarse
 * context) into a finer prediction pred[nyf][nxf][16].  Asynchronous on the
 * batch's stream; INVALID as gabp_upscale_precisions. */
gabp_status gabp_batch_upscale_precisions(gabp_batch *b, int32_t i, float *pred, int64_t nxf,
                                          int64_t nyf, double scale);

/* The batch's freeze tolerance, as gabp_set_freeze_tolerance's, for every
 * instance (default max_slots = 0: bitwise test); INVALID for the same
 * arguments.  Applies from the next check of gabp_batch_solve. */
gabp_status gabp_batch_set_freeze_tolerance(gabp_batch *b, int64_t max_slots, double max_rel);

/* Iterations applied to instance i, the iteration its precision messages
 * froze at (-1 if not), and whether it is still running. */
gabp_status gabp_batch_info(const gabp_batch *b, int32_t i, int64_t *iters, int64_t *frozen_at,
                            int32_t *running);

void gabp_batch_destroy(gabp_batch *b);

/* Text of the last error of b, or of the last failed batch create (b NULL). */
const char *gabp_batch_last_error(const gabp_batch *b);

/* ------------------------------------------------------------------------
 * Network primitives of the learned warm start: a small 3x3 convolutional
 * network (BF16 operands, FP32 accumulation on the matrix cores) that maps
 * observation features to mu^ and log(-Lam^) (see gabp_warm_init), trained
 * on solutions of this solver.  Tensors are device arrays: activations NHWC
 * BF16 [B][H][W][C] (C = 16 or 32; BF16 passed as 16-bit words), weights
 * BF16 [32][9*cin] with k = tap*cin + ci, tap = 3*(dy+1) + (dx+1) (rows
 * beyond cout zero), FP32 biases [32].  All calls are asynchronous on
 * `stream` (a hipStream_t, NULL = default stream) and deterministic.
 * ------------------------------------------------------------------------ */

/* y = act(conv3x3(x, w; dilation dil, zero padding) + bias), act = ReLU when
 * relu != 0.  Writes y_bf16 and/or y_f32 (NHWC, cout channels). */
gabp_status gabp_conv3x3_fwd(const void *x, int32_t B, int32_t H, int32_t W, int32_t cin,
                             const void *w, const float *bias, int32_t cout, int32_t dil,
                             int32_t relu, void *y_bf16, float *y_f32, void *stream);

/* Bytes of scratch gabp_conv3x3_bwd needs for these shapes. */
size_t gabp_conv3x3_bwd_workspace(int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout);

/* Backward of y = act(conv3x3(x, w) + b) given dy (FP32 NHWC): weight and
 * bias gradients dw [32][9*cin], db [32] (FP32) and, when dx != NULL, the
 * input gradient dx (FP32 NHWC, cin channels).  x and y are the layer's BF16
 * input and output. */
gabp_status gabp_conv3x3_bwd(const void *x, const void *y, const float *dy, int32_t B, int32_t H,
                             int32_t W, int32_t cin, const void *w, int32_t cout, int32_t dil,
                             int32_t relu, float *dw, float *db, float *dx, void *workspace,
                             size_t workspace_bytes, void *stream);

/* One Adam step (bias-corrected, step >= 1) on n FP32 master weights w with
 * gradient g and moments m, v; refreshes the BF16 copy w_bf16 (may be NULL). */
gabp_status gabp_adam_step(float *w, const float *g, float *m, float *v, void *w_bf16, int64_t n,
                           double lr, double beta1, double beta2, double eps, int32_t step,
                           void *stream);

/* Warm-start loss on P pixels: mean of (pred[.,0] - mu_t)^2 plus lam_weight
 * times the mean over existing edges (valid[d][p] > 0) of
 * (pred[.,1+d] - lam_t[d][p])^2, d < ndir.  Writes the gradient grad
 * [P][16] and per-workgroup partial sums partials[*nparts] (FP64; the loss is
 * their sum). */
gabp_status gabp_warm_loss(const float *pred, const float *mu_t, const float *lam_t,
                           const float *valid, int64_t P, int32_t ndir, double lam_weight,
                           float *grad, double *partials, int32_t *nparts, void *stream);

/* Network input features [ny][nx][16] BF16 from observations (device arrays):
 * channel 0 mask, 1 mean observed value, 2 log(kappa) + 2.5, others 0.
 * scratch: 2*nx*ny FP32. */
gabp_status gabp_warm_features(int64_t nobs, const int64_t *cell, const double *y, int64_t nx,
                               int64_t ny, double kappa, float *scratch, void *x_bf16,
                               void *stream);

/* gabp_warm_features without the scratch argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops that
 * forbid allocation): the two scratch planes live in a static device array
 * of 2 x 2^21 FP32 values (16 MiB per GPU, held until the process ends), so
 * nx * ny may be at most 2^21 (INVALID beyond).  The call allocates nothing;
 * the scratch is cleared by a kernel on every call.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (different streams
 * or threads without ordering) race.  Same arguments and results otherwise. */
gabp_status gabp_warm_features_noalloc(int64_t nobs, const int64_t *cell, const double *y,
                                       int64_t nx, int64_t ny, double kappa, void *x_bf16,
                                       void *stream);

/* Text of the last error of a network primitive. */
const char *gabp_net_last_error(void);

/* Text of the last error of ctx, or of the last failed create when ctx is NULL. */
const char *gabp_last_error(const gabp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GABP_H */
