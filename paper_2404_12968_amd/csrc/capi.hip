// C ABI of the lattice Gaussian belief propagation library (include/gabp.h):
// argument validation, workspace layout, context state and the host-side
// drivers (iterate, solve with FP64 residual checks, posterior, checkpoint).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "gabp.h"
#include "host_common.h"
#include "internal.h"

using gabp::Lattice;
using namespace gabp::host;

namespace {

thread_local std::string g_create_error;

struct HostMirror {
    double red[8];
    uint32_t flags[8];
};

std::string fmt(const char *f, double a = 0, double b = 0) {
    char buf[256];
    snprintf(buf, sizeof buf, f, a, b);
    return buf;
}

}  // namespace

struct gabp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Lattice L{};
    int dtype = 0;
    size_t esize = 4;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    Layout lay;
    void *msg[2] = {nullptr, nullptr};
    void *gain = nullptr;          // edge gains once the precision messages froze
    double *adiag64 = nullptr, *b64 = nullptr, *mu64 = nullptr;
    double *bel64 = nullptr;       // FP64 belief precisions once frozen
    void *adiag_w = nullptr, *b_w = nullptr;
    double *partials = nullptr, *red = nullptr;
    uint32_t *flags = nullptr;     // [0] diverged-at iteration, [1] input error,
                                   // [3] iteration counter of the launches, [4, 5] precision
                                   // messages changed by the last iteration (64-bit) and
                                   // [6] their largest relative change (float bits)
    HostMirror *host = nullptr;    // pinned
    int rpt = 4;                   // rows per thread of the iteration kernel's tile
    int pair = 0;                  // tile height of the two-iteration kernel, 0 = unused
    int cur = 0;                   // buffer holding the current messages m^iter
    // launches since the last flag read-back, one record per gabp_iterate
    // call: it started at iteration `start` with buffer `buf`, ran `pairs`
    // two-iteration launches, then `singles` one-iteration launches (each
    // launch writes the other buffer).  A divergence found at the next
    // read-back selects the buffer its launch wrote.
    struct LaunchRun {
        int64_t start;
        int buf, pairs, singles;
    };
    std::vector<LaunchRun> runs;
    // captured chunks: iterations are numbered from the device counter
    // flags[3] (host copy tbase); graphs are recorded on a side stream and
    // replayed on the context's stream
    uint32_t tbase = 0;
    bool graphs = true;
    hipStream_t side = nullptr;
    struct Chunk {
        int32_t k;
        int cur, frozen, rpt, pair, tail;
        double eta;
        hipGraphExec_t exec;
        int pairs, singles;
        bool last_single;
    };
    std::vector<Chunk> chunks;
    // launches issued so far: one-iteration full and information-only
    // kernels, two-iteration tile and walker kernels (graph replays included)
    int64_t launches[4] = {0, 0, 0, 0};
    int64_t iter = 0;
    int64_t diverged_at = 0;       // first invalid iteration (0: none)
    bool diverged = false;
    bool prev_valid = false;       // the other buffer holds m^{iter-1}
    bool have_ref = false;         // sum |m^2 - m^1| recorded in red[4]
    bool frozen = false;           // precision messages frozen (gains stored)
    int64_t frozen_at = -1;
    int64_t freeze_slots = 0;      // freeze tolerance: at most this many precision
    double freeze_rel = 0.0;       // messages changed, each by at most this (relative)
    std::string err;
};

namespace {

gabp_status fail(gabp_ctx *ctx, gabp_status st, const std::string &msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_create_error = msg;
    return st;
}

#define GABP_HIP(ctx, call)                                                               \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((ctx), GABP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

gabp_status ctx_ok(gabp_ctx *ctx) {
    if (!ctx) return GABP_E_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return fail(ctx, GABP_E_DEVICE, "hipSetDevice failed");
    return GABP_OK;
}

// Copy the device flags (and reduction results) to the pinned mirror, wait,
// and fold a recorded divergence into the host state.
gabp_status sync_flags(gabp_ctx *ctx, bool with_red) {
    GABP_HIP(ctx, hipMemcpyAsync(ctx->host->flags, ctx->flags, 8 * sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, ctx->stream));
    if (with_red)
        GABP_HIP(ctx, hipMemcpyAsync(ctx->host->red, ctx->red, 8 * sizeof(double),
                                     hipMemcpyDeviceToHost, ctx->stream));
    GABP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const uint32_t t = ctx->host->flags[0];
    if (t != 0u && !ctx->diverged) {
        ctx->diverged = true;
        ctx->diverged_at = (int64_t)t;
        ctx->iter = (int64_t)t;
        // later launches returned without writing: the messages kept are
        // those of the launch that diverged (for a two-iteration launch, its
        // second iteration), in the buffer it wrote
        for (const auto &r : ctx->runs) {
            const int64_t rel = (int64_t)t - r.start;
            if (rel < 1 || rel > 2 * (int64_t)r.pairs + r.singles) continue;
            const HeldState h = held_after_run(r.start, r.buf, r.pairs, (int64_t)t);
            ctx->iter = h.iter;
            ctx->cur = h.buf;
            break;
        }
    }
    ctx->runs.clear();
    if (ctx->diverged)
        return fail(ctx, GABP_E_DIVERGED,
                    fmt("diverged at iteration %.0f (non-positive cavity precision or non-finite "
                        "message); messages kept at iteration %.0f",
                        (double)ctx->diverged_at, (double)ctx->iter));
    return GABP_OK;
}

const void *cur_msgs(const gabp_ctx *ctx) { return ctx->msg[ctx->cur]; }

void drop_chunks(gabp_ctx *ctx) {
    for (auto &c : ctx->chunks) (void)hipGraphExecDestroy(c.exec);
    ctx->chunks.clear();
}

// Autotuner results (rows per thread, pair tile height), process-wide,
// keyed by (alpha, dtype, size class).
std::mutex g_tune_mu;
std::map<long long, std::pair<int, int>> g_tune;

// pair > 0: tile height of the two-iteration tile kernel; pair < 0: the
// column-strip walker with -pair rows per band; 0: one iteration per launch.
bool pair_ok(int dtype, int pair) {
    if (pair < 0) return pair == -2 || ((pair == -4 || pair == -8) && dtype == GABP_F32);
    return pair == 0 || pair == 4 ||
           ((pair == 8 || pair == 12 || pair == 16 || pair == 32) && dtype == GABP_F32);
}

long long tune_key(const gabp_ctx *ctx) {
    const long long n = (long long)ctx->L.nx * ctx->L.ny;
    int cls = 0;
    while (cls < 40 && (1LL << (cls + 1)) <= n) ++cls;   // log2 of the node count
    return ((long long)ctx->L.alpha * 4 + ctx->dtype) * 64 + cls;
}

}  // namespace

extern "C" {

const char *gabp_status_string(gabp_status st) {
    switch (st) {
        case GABP_OK: return "ok";
        case GABP_E_INVALID: return "invalid argument";
        case GABP_E_NOMEM: return "out of memory";
        case GABP_E_DEVICE: return "device error";
        case GABP_E_DIVERGED: return "diverged";
        case GABP_E_NOT_CONVERGED: return "not converged";
    }
    return "unknown status";
}

const char *gabp_last_error(const gabp_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

gabp_status gabp_workspace_size(const gabp_grid *grid, const gabp_stencil *stencil,
                                int32_t dtype, size_t *bytes) {
    std::string why;
    gabp_status st = check_grid_stencil(grid, stencil, dtype, why);
    if (st != GABP_OK) return fail(nullptr, st, why);
    if (!bytes) return fail(nullptr, GABP_E_INVALID, "bytes is NULL");
    const int deg = stencil->alpha == 1 ? 4 : 12;
    const size_t es = dtype == GABP_F32 ? 4 : 8;
    *bytes = make_layout(grid->nx, grid->ny, deg, es, dtype == GABP_F32).total;
    return GABP_OK;
}

int32_t gabp_num_directions(const gabp_ctx *ctx) { return ctx ? ctx->L.deg : 0; }

gabp_status gabp_create(const gabp_grid *grid, const gabp_stencil *stencil, const gabp_obs *obs,
                        const gabp_noise *noise, const gabp_opts *opts, gabp_ctx **out) {
    if (!out) return fail(nullptr, GABP_E_INVALID, "out is NULL");
    *out = nullptr;
    const int32_t dtype = opts ? opts->dtype : GABP_F32;
    std::string why;
    gabp_status st = check_grid_stencil(grid, stencil, dtype, why);
    if (st != GABP_OK) return fail(nullptr, st, why);
    if (!noise) return fail(nullptr, GABP_E_INVALID, "noise is required");
    if (!noise->var && (!(noise->sigma > 0) || !std::isfinite(noise->sigma)))
        return fail(nullptr, GABP_E_INVALID, "sigma must be positive and finite");
    const int64_t nobs = obs ? obs->n : 0;
    if (nobs < 0) return fail(nullptr, GABP_E_INVALID, "negative observation count");
    if (nobs > 0 && (!obs->cell || !obs->y))
        return fail(nullptr, GABP_E_INVALID, "observation arrays are NULL");
    const int64_t N = grid->nx * grid->ny;
    const bool obs_dev = obs && obs->on_device;
    if (nobs > 0 && !obs_dev) {
        for (int64_t k = 0; k < nobs; ++k) {
            if (obs->cell[k] < 0 || obs->cell[k] >= N)
                return fail(nullptr, GABP_E_INVALID, fmt("observation %.0f: cell out of range", (double)k));
            if (!std::isfinite(obs->y[k]))
                return fail(nullptr, GABP_E_INVALID, fmt("observation %.0f: y not finite", (double)k));
            if (noise->var && (!(noise->var[k] > 0) || !std::isfinite(noise->var[k])))
                return fail(nullptr, GABP_E_INVALID, fmt("observation %.0f: variance not positive", (double)k));
        }
    }

    gabp_ctx *ctx = new (std::nothrow) gabp_ctx();
    if (!ctx) return fail(nullptr, GABP_E_NOMEM, "host allocation failed");
    auto bail = [&](gabp_status s2) {
        g_create_error = ctx->err;
        gabp_destroy(ctx);
        return s2;
    };
    ctx->dtype = dtype;
    ctx->esize = dtype == GABP_F32 ? 4 : 8;
    const int deg = stencil->alpha == 1 ? 4 : 12;
    ctx->lay = make_layout(grid->nx, grid->ny, deg, ctx->esize, dtype == GABP_F32);
    ctx->L = make_lattice(grid, stencil, ctx->lay);
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        ctx->err = "no HIP device";
        return bail(GABP_E_DEVICE);
    }
    // NULL selects the device's default (null) stream, which is also what
    // PyTorch's default stream is.
    ctx->stream = opts ? (hipStream_t)opts->stream : nullptr;
    if (opts && opts->workspace) {
        if (opts->workspace_bytes < ctx->lay.total) {
            ctx->err = fmt("workspace too small: %.0f bytes needed", (double)ctx->lay.total);
            return bail(GABP_E_NOMEM);
        }
        if (((uintptr_t)opts->workspace) % kAlign != 0) {
            ctx->err = "workspace must be 256-byte aligned";
            return bail(GABP_E_INVALID);
        }
        ctx->ws = (char *)opts->workspace;
        ctx->ws_bytes = opts->workspace_bytes;
    } else {
        if (hipMalloc((void **)&ctx->ws, ctx->lay.total) != hipSuccess) {
            ctx->ws = nullptr;
            ctx->err = fmt("hipMalloc of %.0f bytes failed", (double)ctx->lay.total);
            return bail(GABP_E_NOMEM);
        }
        ctx->own_ws = true;
        ctx->ws_bytes = ctx->lay.total;
    }
    if (hipHostMalloc((void **)&ctx->host, sizeof(HostMirror), hipHostMallocDefault) != hipSuccess) {
        ctx->host = nullptr;
        ctx->err = "pinned host allocation failed";
        return bail(GABP_E_NOMEM);
    }
    const Layout &lay = ctx->lay;
    ctx->msg[0] = ctx->ws + lay.msg[0];
    ctx->msg[1] = ctx->ws + lay.msg[1];
    ctx->gain = ctx->ws + lay.gain;
    ctx->adiag64 = (double *)(ctx->ws + lay.adiag64);
    ctx->b64 = (double *)(ctx->ws + lay.b64);
    ctx->mu64 = (double *)(ctx->ws + lay.mu64);
    ctx->bel64 = (double *)(ctx->ws + lay.bel64);
    if (dtype == GABP_F32) {
        ctx->adiag_w = ctx->ws + lay.adiag_w;
        ctx->b_w = ctx->ws + lay.b_w;
    } else {
        ctx->adiag_w = ctx->adiag64;
        ctx->b_w = ctx->b64;
    }
    ctx->partials = (double *)(ctx->ws + lay.partials);
    ctx->red = (double *)(ctx->ws + lay.red);
    ctx->flags = (uint32_t *)(ctx->ws + lay.flags);

    // Zero everything: both message buffers (slots without a sender stay 0
    // for ever), the node accumulators and the flags.
    if (hipMemsetAsync(ctx->ws, 0, lay.total, ctx->stream) != hipSuccess) {
        ctx->err = "hipMemsetAsync failed";
        return bail(GABP_E_DEVICE);
    }
    int64_t *tmp_cell = nullptr;
    double *tmp_y = nullptr, *tmp_var = nullptr;
    const int64_t *d_cell = nullptr;
    const double *d_y = nullptr, *d_var = nullptr;
    if (nobs > 0) {
        if (obs_dev) {
            d_cell = obs->cell;
            d_y = obs->y;
            d_var = noise->var;
        } else {
            bool ok = hipMalloc((void **)&tmp_cell, nobs * sizeof(int64_t)) == hipSuccess &&
                      hipMalloc((void **)&tmp_y, nobs * sizeof(double)) == hipSuccess &&
                      (!noise->var || hipMalloc((void **)&tmp_var, nobs * sizeof(double)) == hipSuccess);
            ok = ok &&
                 hipMemcpyAsync(tmp_cell, obs->cell, nobs * sizeof(int64_t), hipMemcpyHostToDevice,
                                ctx->stream) == hipSuccess &&
                 hipMemcpyAsync(tmp_y, obs->y, nobs * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream) == hipSuccess &&
                 (!noise->var || hipMemcpyAsync(tmp_var, noise->var, nobs * sizeof(double),
                                                hipMemcpyHostToDevice, ctx->stream) == hipSuccess);
            if (!ok) {
                (void)hipStreamSynchronize(ctx->stream);
                (void)hipFree(tmp_cell);
                (void)hipFree(tmp_y);
                (void)hipFree(tmp_var);
                ctx->err = "staging observations on the device failed";
                return bail(GABP_E_NOMEM);
            }
            d_cell = tmp_cell;
            d_y = tmp_y;
            d_var = tmp_var;
        }
    }
    const double s2 = noise->var ? 0.0 : noise->sigma * noise->sigma;
    hipError_t e = gabp::launch_setup(dtype == GABP_F32 ? 0 : 1, ctx->L, nobs, d_cell, d_y, d_var,
                                      s2, ctx->adiag64, ctx->b64, opts ? opts->prior_mean : nullptr,
                                      dtype == GABP_F32 ? ctx->adiag_w : nullptr,
                                      dtype == GABP_F32 ? ctx->b_w : nullptr, ctx->flags + 1,
                                      ctx->stream);
    hipError_t e2 = hipMemcpyAsync(ctx->host->flags, ctx->flags, 4 * sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, ctx->stream);
    hipError_t e3 = hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp_cell);
    (void)hipFree(tmp_y);
    (void)hipFree(tmp_var);
    if (e != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        ctx->err = std::string("setup failed: ") +
                   hipGetErrorString(e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3));
        return bail(GABP_E_DEVICE);
    }
    if (ctx->host->flags[1] != 0u) {
        ctx->err = "invalid observation (cell out of range, non-finite value or non-positive "
                   "variance) or non-finite prior mean";
        return bail(GABP_E_INVALID);
    }
    ctx->iter = 0;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(tune_key(ctx));
        if (it != g_tune.end()) {
            ctx->rpt = it->second.first;
            ctx->pair = it->second.second;
        } else {
            ctx->pair = dtype == GABP_F32 ? 8 : 4;
        }
    }
    *out = ctx;
    return GABP_OK;
}

void gabp_destroy(gabp_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_chunks(ctx);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->own_ws && ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->host) (void)hipHostFree(ctx->host);
    delete ctx;
}

namespace {

// Issue n iterations on stream s, starting from iteration iter0 held in
// buffer cur0, with iteration numbers relative to the device counter's value
// tbase when they run.  Frozen contexts run two iterations per launch; with
// tail_single the last one or two run singly, so that the two buffers end on
// m^{t-1} and m^t (the message-change statistic and the freeze probe need
// that), else pairs run while two iterations remain.  Touches no context
// state; reports the launch counts, whether the last launch was single and
// whether the t = 2 reference change was taken.
gabp_status enqueue_iters(gabp_ctx *ctx, int32_t n, double damping, hipStream_t s, int64_t iter0,
                          int cur0, uint32_t tbase, bool tail_single, int &pairs, int &singles,
                          bool &last_single, bool &ref) {
    const int dt = ctx->dtype == GABP_F32 ? 0 : 1;
    int64_t it = iter0;
    int cur = cur0;
    pairs = singles = 0;
    ref = false;
    last_single = true;
    const int32_t min_left = tail_single ? 3 : 2;
    int32_t k = 0;
    while (k < n) {
        const void *src = ctx->msg[cur];
        void *dst = ctx->msg[cur ^ 1];
        if (ctx->frozen && ctx->pair != 0 && it >= 2 && n - k >= min_left) {
            if (ctx->pair < 0)
                GABP_HIP(ctx, gabp::launch_iter_theta2w(dt, -ctx->pair, ctx->L, src, dst,
                                                        ctx->gain, ctx->b_w, damping, ctx->flags,
                                                        ctx->flags + 3, (uint32_t)(it - tbase), s));
            else
                GABP_HIP(ctx, gabp::launch_iter_theta2(dt, ctx->pair, ctx->L, src, dst, ctx->gain,
                                                       ctx->b_w, damping, ctx->flags, ctx->flags + 3,
                                                       (uint32_t)(it - tbase), s));
            it += 2;
            k += 2;
            ++pairs;
            last_single = false;
        } else {
            const int64_t t = it + 1;
            if (ctx->frozen)
                GABP_HIP(ctx, gabp::launch_iter_theta(dt, ctx->rpt, ctx->L, src, dst, ctx->gain,
                                                      ctx->b_w, damping, ctx->flags,
                                                      ctx->flags + 3, (uint32_t)(t - tbase), s));
            else
                GABP_HIP(ctx, gabp::launch_iter(dt, ctx->rpt, ctx->L, src, dst, ctx->adiag_w,
                                                ctx->b_w, damping, ctx->flags, ctx->flags + 3,
                                                (uint32_t)(t - tbase), s));
            it = t;
            ++k;
            ++singles;
            last_single = true;
            if (t == 2) {
                const int64_t m = (int64_t)(2 * ctx->L.deg) * ctx->L.plane;
                GABP_HIP(ctx, gabp::launch_abs_change(dt, ctx->msg[0], ctx->msg[1], m,
                                                      ctx->partials, kNumPartials, ctx->red + 4,
                                                      s));
                ref = true;
            }
        }
        cur ^= 1;
    }
    return GABP_OK;
}

// Adaptive chunk lengths as kmin * 2^j, so that few chunk graphs are recorded.
int64_t quantize_chunk(int64_t next, int64_t kmin) {
    int64_t q = kmin;
    while (q * 2 <= next) q *= 2;
    return q;
}

// Context state after n iterations issued by enqueue_iters (runs of pairs
// then singles; a chunk that ends on a pair leaves m^{t-2} in the other
// buffer).
void advance_state(gabp_ctx *ctx, int32_t n, int pairs, int singles, bool last_single, bool ref) {
    ctx->runs.push_back({ctx->iter, ctx->cur, pairs, singles});
    ctx->launches[ctx->frozen ? 1 : 0] += singles;
    ctx->launches[ctx->pair > 0 ? 2 : 3] += pairs;
    ctx->iter += n;
    ctx->cur ^= (pairs + singles) & 1;
    if (ref) ctx->have_ref = true;
    if (n > 0) ctx->prev_valid = last_single;
}

gabp_status check_iterate_args(gabp_ctx *ctx, int32_t n_iters, double damping) {
    if (n_iters < 0) return fail(ctx, GABP_E_INVALID, "n_iters must be >= 0");
    if (!(damping > 0.0) || !(damping <= 1.0))
        return fail(ctx, GABP_E_INVALID, "damping must be in (0, 1]");
    if (ctx->diverged) return fail(ctx, GABP_E_DIVERGED, "run has diverged");
    if (ctx->iter + n_iters >= (int64_t)UINT32_MAX)
        return fail(ctx, GABP_E_INVALID, "iteration counter overflow");
    return GABP_OK;
}

// k iterations as one captured graph (recorded once per chunk length,
// starting buffer, phase, tile shape and damping; replayed after), else
// eagerly.  The graph ends by advancing the device iteration counter.
gabp_status run_chunk(gabp_ctx *ctx, int32_t k, double damping, bool tail_single) {
    gabp_status st = check_iterate_args(ctx, k, damping);
    if (st != GABP_OK) return st;
    if (!ctx->graphs || k < 2 || ctx->iter < 2) {
        int pairs = 0, singles = 0;
        bool last = true, ref = false;
        st = enqueue_iters(ctx, k, damping, ctx->stream, ctx->iter, ctx->cur, ctx->tbase,
                           tail_single, pairs, singles, last, ref);
        if (st != GABP_OK) return st;
        advance_state(ctx, k, pairs, singles, last, ref);
        return GABP_OK;
    }
    if (ctx->tbase != (uint32_t)ctx->iter) {
        GABP_HIP(ctx, gabp::launch_set_u32(ctx->flags + 3, (uint32_t)ctx->iter, ctx->stream));
        ctx->tbase = (uint32_t)ctx->iter;
    }
    gabp_ctx::Chunk *c = nullptr;
    for (auto &e : ctx->chunks)
        if (e.k == k && e.cur == ctx->cur && e.frozen == (int)ctx->frozen && e.rpt == ctx->rpt &&
            e.pair == ctx->pair && e.tail == (int)tail_single && e.eta == damping)
            c = &e;
    if (!c) {
        if (ctx->chunks.size() >= 16) {
            // replays of the recorded graphs may still be in flight
            GABP_HIP(ctx, hipStreamSynchronize(ctx->stream));
            drop_chunks(ctx);
        }
        if (!ctx->side)
            GABP_HIP(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        gabp_ctx::Chunk e{k,       ctx->cur, (int)ctx->frozen, ctx->rpt, ctx->pair,
                          (int)tail_single, damping, nullptr, 0, 0, true};
        bool ref = false;
        GABP_HIP(ctx, hipStreamBeginCapture(ctx->side, hipStreamCaptureModeThreadLocal));
        // relative numbering: the counter holds the chunk's first iteration
        st = enqueue_iters(ctx, k, damping, ctx->side, ctx->iter, ctx->cur, (uint32_t)ctx->iter,
                           tail_single, e.pairs, e.singles, e.last_single, ref);
        if (st == GABP_OK && gabp::launch_add_u32(ctx->flags + 3, (uint32_t)k, ctx->side) != hipSuccess)
            st = fail(ctx, GABP_E_DEVICE, "capturing the counter advance failed");
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->side, &g);
        if (st != GABP_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ec != hipSuccess || !g) return fail(ctx, GABP_E_DEVICE, "hipStreamEndCapture failed");
        const hipError_t ei = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return fail(ctx, GABP_E_DEVICE, "hipGraphInstantiate failed");
        ctx->chunks.push_back(e);
        c = &ctx->chunks.back();
    }
    GABP_HIP(ctx, hipGraphLaunch(c->exec, ctx->stream));
    ctx->tbase += (uint32_t)k;
    advance_state(ctx, k, c->pairs, c->singles, c->last_single, false);
    return GABP_OK;
}

}  // namespace

gabp_status gabp_iterate(gabp_ctx *ctx, int32_t n_iters, double damping) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    st = check_iterate_args(ctx, n_iters, damping);
    if (st != GABP_OK) return st;
    int pairs = 0, singles = 0;
    bool last = true, ref = false;
    st = enqueue_iters(ctx, n_iters, damping, ctx->stream, ctx->iter, ctx->cur, ctx->tbase, true,
                       pairs, singles, last, ref);
    if (st != GABP_OK) return st;
    advance_state(ctx, n_iters, pairs, singles, last, ref);
    return GABP_OK;
}

gabp_status gabp_set_graph(gabp_ctx *ctx, int32_t enable) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    ctx->graphs = enable != 0;
    if (!ctx->graphs && !ctx->chunks.empty()) {
        GABP_HIP(ctx, hipStreamSynchronize(ctx->stream));
        drop_chunks(ctx);
    }
    return GABP_OK;
}

gabp_status gabp_residual(gabp_ctx *ctx, double *rel_residual, double *abs_residual) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (ctx->diverged) return fail(ctx, GABP_E_DIVERGED, "run has diverged");
    const int dt = ctx->dtype == GABP_F32 ? 0 : 1;
    // How many precision messages did the last iteration change, and by how
    // much at most?
    const bool probe = !ctx->frozen && ctx->prev_valid && ctx->iter >= 2;
    if (probe) {
        GABP_HIP(ctx, hipMemsetAsync(ctx->flags + 4, 0, 3 * sizeof(uint32_t), ctx->stream));
        GABP_HIP(ctx, gabp::launch_prec_change(dt, ctx->msg[ctx->cur], ctx->msg[ctx->cur ^ 1],
                                               (int64_t)ctx->L.deg * ctx->L.plane,
                                               (unsigned long long *)(ctx->flags + 4),
                                               ctx->flags + 6, ctx->stream));
    }
    GABP_HIP(ctx, gabp::launch_post(dt, ctx->L, cur_msgs(ctx), ctx->adiag64, ctx->b64,
                                    ctx->frozen ? ctx->bel64 : nullptr, ctx->mu64, nullptr,
                                    nullptr, probe ? ctx->bel64 : nullptr, ctx->stream));
    GABP_HIP(ctx, gabp::launch_resid(ctx->L, ctx->mu64, ctx->adiag64, ctx->b64, ctx->partials,
                                     kNumPartials, ctx->red, ctx->stream));
    st = sync_flags(ctx, true);
    if (st != GABP_OK) return st;
    uint64_t changed = 0;
    std::memcpy(&changed, ctx->host->flags + 4, sizeof changed);
    if (probe && freeze_now(changed, ctx->host->flags[6], ctx->freeze_slots, ctx->freeze_rel)) {
        // frozen: from now on only the information messages change
        GABP_HIP(ctx, gabp::launch_gain(dt, ctx->L, cur_msgs(ctx), ctx->adiag_w, ctx->gain,
                                        ctx->stream));
        // frozen within the tolerance: the other buffer's precision messages
        // still differ in a few places; make both buffers hold the ones the
        // gains come from
        if (changed != 0u)
            GABP_HIP(ctx, hipMemcpyAsync(ctx->msg[ctx->cur ^ 1], ctx->msg[ctx->cur],
                                         (size_t)ctx->L.deg * (size_t)ctx->L.plane * ctx->esize,
                                         hipMemcpyDeviceToDevice, ctx->stream));
        ctx->frozen = true;
        ctx->frozen_at = ctx->iter;
    }
    const double a = std::sqrt(ctx->host->red[0]), b = std::sqrt(ctx->host->red[1]);
    if (abs_residual) *abs_residual = a;
    if (rel_residual) *rel_residual = b > 0 ? a / b : a;
    return GABP_OK;
}

gabp_status gabp_solve(gabp_ctx *ctx, int64_t max_iters, double damping, double rel_tol,
                       int32_t check_every, int64_t *iters_done, double *rel_residual) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (max_iters < 0 || check_every == 0 || !(rel_tol >= 0))
        return fail(ctx, GABP_E_INVALID, "need max_iters >= 0, check_every != 0, rel_tol >= 0");
    // check_every > 0: fixed interval.  check_every < 0: adaptive, at least
    // |check_every| iterations apart; fixed until the precision messages
    // froze, then half the iterations the observed geometric rate predicts
    // to rel_tol, at most kMaxInterval.
    constexpr int64_t kMaxInterval = 2000;
    const bool adaptive = check_every < 0;
    const int64_t kmin = adaptive ? -(int64_t)check_every : (int64_t)check_every;
    double rel = INFINITY, first = -1.0, prev_rel = -1.0;
    int64_t run = 0, prev_t = 0, next = kmin;
    st = GABP_E_NOT_CONVERGED;
    while (run < max_iters) {
        const int32_t k = (int32_t)std::min<int64_t>(next, max_iters - run);
        gabp_status s1 = run_chunk(ctx, k, damping, false);
        if (s1 != GABP_OK) {
            st = s1;
            break;
        }
        run += k;
        s1 = gabp_residual(ctx, &rel, nullptr);
        if (s1 != GABP_OK) {
            st = s1;
            break;
        }
        if (!std::isfinite(rel) || (first > 0 && rel > 1e3 * first)) {
            st = fail(ctx, GABP_E_DIVERGED, fmt("residual blew up to %g at iteration %.0f", rel,
                                                (double)ctx->iter));
            break;
        }
        if (first < 0) first = rel;
        if (rel <= rel_tol) {
            st = GABP_OK;
            break;
        }
        next = kmin;
        if (adaptive && ctx->frozen && prev_rel > 0 && rel < prev_rel && rel > 0) {
            const double rate = std::log(rel / prev_rel) / (double)(ctx->iter - prev_t);
            const double need = std::log(rel_tol / rel) / rate;   // iterations to rel_tol
            next = std::max<int64_t>(kmin, std::min<int64_t>(kMaxInterval, (int64_t)(0.5 * need)));
            if (ctx->graphs) next = quantize_chunk(next, kmin);
        }
        prev_rel = rel;
        prev_t = ctx->iter;
    }
    if (st == GABP_E_NOT_CONVERGED) {
        if (max_iters == 0) {
            gabp_status s1 = gabp_residual(ctx, &rel, nullptr);
            if (s1 != GABP_OK) st = s1;
            else if (rel <= rel_tol) st = GABP_OK;
        }
        if (st == GABP_E_NOT_CONVERGED)
            fail(ctx, st, fmt("relative residual %g after %.0f iterations", rel, (double)ctx->iter));
    }
    if (iters_done) *iters_done = ctx->iter;
    if (rel_residual) *rel_residual = rel;
    return st;
}

gabp_status gabp_solve_early_stop(gabp_ctx *ctx, int64_t max_iters, double damping, double tau,
                                  int32_t check_every, int64_t *iters_done, double *ratio_out) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (max_iters < 0 || check_every == 0 || !(tau >= 0))
        return fail(ctx, GABP_E_INVALID, "need max_iters >= 0, check_every != 0, tau >= 0");
    // same check schedule as gabp_solve, on the message-change ratio
    constexpr int64_t kMaxInterval = 2000;
    const bool adaptive = check_every < 0;
    const int64_t kmin = adaptive ? -(int64_t)check_every : (int64_t)check_every;
    double ratio = INFINITY, prev = -1.0;
    int64_t run = 0, prev_t = 0;
    int64_t next = std::max<int64_t>(kmin, ctx->iter < 3 ? 3 - ctx->iter : 0);
    st = GABP_E_NOT_CONVERGED;
    while (run < max_iters) {
        const int32_t k = (int32_t)std::min<int64_t>(next, max_iters - run);
        gabp_status s1 = run_chunk(ctx, k, damping, true);
        if (s1 != GABP_OK) {
            st = s1;
            break;
        }
        run += k;
        if (ctx->iter < 3) {
            next = 3 - ctx->iter;
            continue;
        }
        s1 = gabp_message_change(ctx, &ratio);
        if (s1 != GABP_OK) {
            st = s1;
            break;
        }
        if (ratio < tau) {
            st = GABP_OK;
            break;
        }
        next = kmin;
        if (adaptive && ctx->frozen && prev > 0 && ratio < prev && ratio > 0 && tau > 0) {
            const double rate = std::log(ratio / prev) / (double)(ctx->iter - prev_t);
            const double need = std::log(tau / ratio) / rate;
            next = std::max<int64_t>(kmin, std::min<int64_t>(kMaxInterval, (int64_t)(0.5 * need)));
            if (ctx->graphs) next = quantize_chunk(next, kmin);
        }
        if (!ctx->frozen && adaptive) {
            // a residual check is what detects frozen precision messages
            double rel;
            s1 = gabp_residual(ctx, &rel, nullptr);
            if (s1 != GABP_OK) {
                st = s1;
                break;
            }
        }
        prev = ratio;
        prev_t = ctx->iter;
    }
    if (st == GABP_E_NOT_CONVERGED)
        fail(ctx, st, fmt("message change ratio %g after %.0f iterations", ratio, (double)ctx->iter));
    if (iters_done) *iters_done = ctx->iter;
    if (ratio_out) *ratio_out = ratio;
    return st;
}

gabp_status gabp_posterior(gabp_ctx *ctx, double *mean, double *var) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    const int dt = ctx->dtype == GABP_F32 ? 0 : 1;
    GABP_HIP(ctx, gabp::launch_post(dt, ctx->L, cur_msgs(ctx), ctx->adiag64, ctx->b64,
                                    ctx->frozen ? ctx->bel64 : nullptr, nullptr, mean, var,
                                    nullptr, ctx->stream));
    return GABP_OK;
}

gabp_status gabp_message_change(gabp_ctx *ctx, double *ratio) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (!ratio) return fail(ctx, GABP_E_INVALID, "ratio is NULL");
    if (!ctx->have_ref || !ctx->prev_valid || ctx->iter < 2)
        return fail(ctx, GABP_E_INVALID, "needs two consecutive iterations past t = 2");
    const int dt = ctx->dtype == GABP_F32 ? 0 : 1;
    const int64_t n = (int64_t)(2 * ctx->L.deg) * ctx->L.plane;
    GABP_HIP(ctx, gabp::launch_abs_change(dt, ctx->msg[ctx->cur], ctx->msg[ctx->cur ^ 1],
                                          n, ctx->partials, kNumPartials, ctx->red + 2, ctx->stream));
    st = sync_flags(ctx, true);
    if (st != GABP_OK) return st;
    const double num = ctx->host->red[2], den = ctx->host->red[4];
    *ratio = den > 0 ? num / den : (num > 0 ? INFINITY : 0.0);
    return GABP_OK;
}

gabp_status gabp_get_messages(gabp_ctx *ctx, void *prec, void *info) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    GABP_HIP(ctx, gabp::launch_msgs_get(ctx->dtype == GABP_F32 ? 0 : 1, ctx->L, cur_msgs(ctx),
                                        prec, info, ctx->stream));
    return GABP_OK;
}

gabp_status gabp_set_messages(gabp_ctx *ctx, const void *prec, const void *info) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (ctx->diverged) return fail(ctx, GABP_E_DIVERGED, "run has diverged");
    GABP_HIP(ctx, gabp::launch_msgs_set(ctx->dtype == GABP_F32 ? 0 : 1, ctx->L,
                                        ctx->msg[ctx->cur], prec, info, ctx->stream));
    ctx->prev_valid = false;
    ctx->frozen = false;
    ctx->frozen_at = -1;
    return GABP_OK;
}

gabp_status gabp_autotune(gabp_ctx *ctx, int32_t trials, double damping, int32_t *chosen) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (trials < 1) return fail(ctx, GABP_E_INVALID, "trials must be >= 1");
    hipEvent_t ev[2];
    GABP_HIP(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(ctx, GABP_E_DEVICE, "hipEventCreate failed");
    }
    const int saved_rpt = ctx->rpt, saved_pair = ctx->pair;
    auto finish = [&](gabp_status s1) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        return s1;
    };
    // time `trials` iterations with one tile configuration
    auto timed = [&](int rpt, int pair, float &ms) {
        ctx->rpt = rpt;
        ctx->pair = pair;
        gabp_status s1 = GABP_OK;
        if (hipEventRecord(ev[0], ctx->stream) != hipSuccess) s1 = GABP_E_DEVICE;
        if (s1 == GABP_OK) s1 = gabp_iterate(ctx, trials, damping);
        if (s1 == GABP_OK && hipEventRecord(ev[1], ctx->stream) != hipSuccess) s1 = GABP_E_DEVICE;
        if (s1 == GABP_OK && hipEventSynchronize(ev[1]) != hipSuccess) s1 = GABP_E_DEVICE;
        ms = 0.f;
        if (s1 == GABP_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            s1 = GABP_E_DEVICE;
        if (s1 != GABP_OK) {
            ctx->rpt = saved_rpt;
            ctx->pair = saved_pair;
            if (s1 == GABP_E_DEVICE) fail(ctx, s1, "autotune timing failed");
        }
        return s1;
    };
    // one untimed iteration first, then two timed passes over the shapes;
    // the best time of a shape over both passes counts
    st = gabp_iterate(ctx, 1, damping);
    if (st != GABP_OK) return finish(st);
    float best_ms = INFINITY;
    int best_rpt = ctx->rpt, best_pair = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int rpt : gabp::kRptChoices) {
            float ms;
            if ((st = timed(rpt, 0, ms)) != GABP_OK) return finish(st);
            if (ms < best_ms) {
                best_ms = ms;
                best_rpt = rpt;
            }
        }
    if (ctx->frozen) {
        // the two-iteration tile kernel against the best single-iteration
        // shape (the column-strip walker is selectable with gabp_set_tile but
        // not timed here: it measured slower on every lattice tried)
        for (int pass = 0; pass < 2; ++pass)
            for (int pair : gabp::kPairChoicesF32) {
                if (!pair_ok(ctx->dtype, pair)) continue;
                float ms;
                if ((st = timed(best_rpt, pair, ms)) != GABP_OK) return finish(st);
                if (ms < best_ms) {
                    best_ms = ms;
                    best_pair = pair;
                }
            }
    } else {
        best_pair = saved_pair;
    }
    ctx->rpt = best_rpt;
    ctx->pair = best_pair;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[tune_key(ctx)] = {best_rpt, best_pair};
    }
    if (chosen) *chosen = best_rpt;
    return finish(sync_flags(ctx, false));
}

gabp_status gabp_set_tile(gabp_ctx *ctx, int32_t rows_per_thread, int32_t pair_rows) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    bool rpt_ok = false;
    for (int r : gabp::kRptChoices) rpt_ok |= r == rows_per_thread;
    if (!rpt_ok) return fail(ctx, GABP_E_INVALID, "rows_per_thread must be 1, 2, 4 or 8");
    if (!pair_ok(ctx->dtype, pair_rows))
        return fail(ctx, GABP_E_INVALID,
                    "pair_rows must be 0, 4, -2 or (FP32 only) 8, 12, 16, 32, -4 or -8");
    ctx->rpt = rows_per_thread;
    ctx->pair = pair_rows;
    return GABP_OK;
}

gabp_status gabp_get_tile(const gabp_ctx *ctx, int32_t *rows_per_thread, int32_t *pair_rows) {
    if (!ctx) return GABP_E_INVALID;
    if (rows_per_thread) *rows_per_thread = ctx->rpt;
    if (pair_rows) *pair_rows = ctx->pair;
    return GABP_OK;
}

gabp_status gabp_set_freeze_tolerance(gabp_ctx *ctx, int64_t max_slots, double max_rel) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (max_slots < 0 || !(max_rel >= 0.0) || !std::isfinite(max_rel))
        return fail(ctx, GABP_E_INVALID, "need max_slots >= 0 and a finite max_rel >= 0");
    ctx->freeze_slots = max_slots;
    ctx->freeze_rel = max_rel;
    return GABP_OK;
}

gabp_status gabp_launch_counts(const gabp_ctx *ctx, int64_t *full, int64_t *theta,
                               int64_t *pair_tiles, int64_t *pair_walk) {
    if (!ctx) return GABP_E_INVALID;
    if (full) *full = ctx->launches[0];
    if (theta) *theta = ctx->launches[1];
    if (pair_tiles) *pair_tiles = ctx->launches[2];
    if (pair_walk) *pair_walk = ctx->launches[3];
    return GABP_OK;
}

gabp_status gabp_precision_frozen(const gabp_ctx *ctx, int64_t *at) {
    if (!ctx || !at) return GABP_E_INVALID;
    *at = ctx->frozen ? ctx->frozen_at : -1;
    return GABP_OK;
}

gabp_status gabp_upsample_mean(const double *coarse, int64_t nxc, int64_t nyc, int32_t bc_x,
                               int32_t bc_y, float *pred, int64_t nxf, int64_t nyf, void *stream) {
    if (!coarse || !pred || nxc < 1 || nyc < 1 || nxf < 1 || nyf < 1 ||
        (nxf + 1) / 2 != nxc || (nyf + 1) / 2 != nyc)
        return fail(nullptr, GABP_E_INVALID,
                    "upsample_mean: need nxc = ceil(nxf / 2) and nyc = ceil(nyf / 2)");
    if ((bc_x == GABP_BC_PERIODIC && nxf != 2 * nxc) || (bc_y == GABP_BC_PERIODIC && nyf != 2 * nyc))
        return fail(nullptr, GABP_E_INVALID, "upsample_mean: periodic axes need even fine sizes");
    hipError_t e = gabp::launch_upsample_mean(coarse, (int)nxc, (int)nyc, bc_x == GABP_BC_PERIODIC,
                                              bc_y == GABP_BC_PERIODIC, pred, (int)nxf, (int)nyf,
                                              (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, GABP_E_DEVICE, hipGetErrorString(e));
    return GABP_OK;
}

gabp_status gabp_upscale_precisions(gabp_ctx *coarse, float *pred, int64_t nxf, int64_t nyf,
                                    double scale) {
    gabp_status st = ctx_ok(coarse);
    if (st != GABP_OK) return st;
    if (!pred) return fail(coarse, GABP_E_INVALID, "pred is NULL");
    if (nxf < 1 || nyf < 1 || (nxf + 1) / 2 != coarse->L.nx || (nyf + 1) / 2 != coarse->L.ny)
        return fail(coarse, GABP_E_INVALID,
                    "upscale_precisions: need ceil(nxf / 2) = nx and ceil(nyf / 2) = ny of the "
                    "coarse context");
    if (!(scale > 0.0) || !std::isfinite(scale))
        return fail(coarse, GABP_E_INVALID, "upscale_precisions: scale must be finite and > 0");
    GABP_HIP(coarse, gabp::launch_upscale_prec(coarse->dtype == GABP_F32 ? 0 : 1, coarse->L,
                                               cur_msgs(coarse), (float)scale, pred, (int)nxf,
                                               (int)nyf, coarse->stream));
    return GABP_OK;
}

gabp_status gabp_copy_coarse_messages(gabp_ctx *coarse, gabp_ctx *fine) {
    gabp_status st = ctx_ok(coarse);
    if (st != GABP_OK) return st;
    if (!fine) return fail(coarse, GABP_E_INVALID, "fine is NULL");
    if (fine->device != coarse->device || fine->dtype != coarse->dtype ||
        fine->L.alpha != coarse->L.alpha || fine->L.bcx != coarse->L.bcx ||
        fine->L.bcy != coarse->L.bcy)
        return fail(coarse, GABP_E_INVALID,
                    "copy_coarse_messages: contexts differ in device, dtype, alpha or boundary");
    if ((fine->L.nx + 1) / 2 != coarse->L.nx || (fine->L.ny + 1) / 2 != coarse->L.ny)
        return fail(coarse, GABP_E_INVALID,
                    "copy_coarse_messages: need ceil(nx_fine / 2) = nx and ceil(ny_fine / 2) = ny "
                    "of the coarse context");
    if (fine->diverged) return fail(coarse, GABP_E_DIVERGED, "the fine run has diverged");
    // the fine context's stream waits for the coarse messages
    GABP_HIP(coarse, hipStreamSynchronize(coarse->stream));
    GABP_HIP(coarse, gabp::launch_copy_coarse(coarse->dtype == GABP_F32 ? 0 : 1, coarse->L,
                                              cur_msgs(coarse), fine->L, fine->msg[fine->cur],
                                              fine->stream));
    fine->prev_valid = false;
    fine->frozen = false;
    fine->frozen_at = -1;
    return GABP_OK;
}

gabp_status gabp_warm_init(gabp_ctx *ctx, const float *pred, int32_t keep_precisions) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (!pred) return fail(ctx, GABP_E_INVALID, "pred is NULL");
    if (ctx->diverged) return fail(ctx, GABP_E_DIVERGED, "run has diverged");
    GABP_HIP(ctx, gabp::launch_warm_init(ctx->dtype == GABP_F32 ? 0 : 1, ctx->L, pred,
                                         keep_precisions ? 1 : 0, ctx->msg[ctx->cur],
                                         ctx->stream));
    ctx->prev_valid = false;
    ctx->frozen = false;
    ctx->frozen_at = -1;
    return GABP_OK;
}

gabp_status gabp_log_precisions(gabp_ctx *ctx, float *lam, float *valid) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    if (!lam) return fail(ctx, GABP_E_INVALID, "lam is NULL");
    GABP_HIP(ctx, gabp::launch_log_prec(ctx->dtype == GABP_F32 ? 0 : 1, ctx->L, cur_msgs(ctx), lam,
                                        valid, ctx->stream));
    return GABP_OK;
}

gabp_status gabp_iteration_count(gabp_ctx *ctx, int64_t *iters) {
    gabp_status st = ctx_ok(ctx);
    if (st != GABP_OK) return st;
    st = sync_flags(ctx, false);
    if (iters) *iters = ctx->iter;
    return st;
}

}  // extern "C"
