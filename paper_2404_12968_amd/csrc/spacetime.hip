// Space-time Gaussian belief propagation (include/gabp_st.h): set-up,
// marginals, FP64 residual, message read-back, multigrid transfers and the
// C ABI.  The iteration kernels and the closed forms of the precision live
// in st_iter.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "gabp_st.h"
#include "host_common.h"
#include "internal.h"
#include "lattice.h"
#include "numerics.h"
#include "st_iter.h"

#pragma clang fp contract(off)

namespace gabp {
namespace st {

constexpr int kPartials = 2048;     // workgroups of the residual reduction

// --------------------------------------------------------------------------
// Set-up: A_ii = Q_ii + p_i (p_i already folded into adiag64 by the
// observation fold), b_i = h_i + (P m)_i on slice 0 with P = S L^2, the
// message-precision copies of both.  Thread per node.
// --------------------------------------------------------------------------
__device__ __forceinline__ double q_diag(const Grid &G, int x, int y, int t) {
    const double gi = (double)(axis_g(x, G.nx, G.bcx) + axis_g(y, G.ny, G.bcy));
    return coef<double>(G.blk[slice_kind(G, t)], 0, gi, 0.0);
}

template <typename T>
__global__ __launch_bounds__(256) void k_node_init(Grid G, double *__restrict__ adiag64,
                                                   double *__restrict__ b64,
                                                   const double *__restrict__ pm,
                                                   T *__restrict__ aw, T *__restrict__ bw,
                                                   uint32_t *__restrict__ err_flag) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nodes = (int64_t)G.nx * G.ny * G.nt;
    if (k >= nodes) return;
    const int x = (int)(k % G.nx);
    const int y = (int)((k / G.nx) % G.ny);
    const int t = (int)(k / ((int64_t)G.nx * G.ny));
    const int64_t i = (int64_t)t * G.slice + (int64_t)y * G.pitch + x;
    const double a = q_diag(G, x, y, t) + adiag64[i];
    double b = b64[i];
    if (pm && t == 0) {
        // (S L^2 m)_i over the 13-point stencil of S L^2
        const double *lsq = G.lsq;
        const double gi = (double)(axis_g(x, G.nx, G.bcx) + axis_g(y, G.ny, G.bcy));
        double s = coef<double>(lsq, 0, gi, 0.0) * pm[(int64_t)y * G.nx + x];
        for (int d = 0; d < 12; ++d) {
            int xn, yn, tn;
            if (!nbr(G, x, y, 0, d, xn, yn, tn)) continue;
            const double gj = (double)(axis_g(xn, G.nx, G.bcx) + axis_g(yn, G.ny, G.bcy));
            s += coef<double>(lsq, scls(d), gi, gj) * pm[(int64_t)yn * G.nx + xn];
        }
        if (!isfinite(s)) *err_flag = 1u;
        b += s;
    }
    adiag64[i] = a;
    b64[i] = b;
    aw[i] = (T)a;
    bw[i] = (T)b;
}

// --------------------------------------------------------------------------
// Marginals (Compute Marginal) in FP64: Lam = A_ii + c sum Lam_{k->i},
// th = b_i + c sum th_{k->i}, mu = th / Lam, var = 1 / Lam.  Writes the
// pitched mean plane read by the residual and, when given, dense outputs.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_post(Grid G, const T *__restrict__ m,
                                              const double *__restrict__ adiag64,
                                              const double *__restrict__ b64,
                                              double *__restrict__ mu_plane,
                                              double *__restrict__ mean,
                                              double *__restrict__ var) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nodes = (int64_t)G.nx * G.ny * G.nt;
    if (k >= nodes) return;
    const int x = (int)(k % G.nx);
    const int y = (int)((k / G.nx) % G.ny);
    const int t = (int)(k / ((int64_t)G.nx * G.ny));
    const int64_t i = (int64_t)t * G.slice + (int64_t)y * G.pitch + x;
    double sl = 0.0, st = 0.0;
    for (int d = 0; d < kDeg; ++d) {
        int xn, yn, tn;
        if (!nbr(G, x, y, t, d, xn, yn, tn)) continue;
        const int64_t j = (int64_t)tn * G.slice + (int64_t)yn * G.pitch + xn;
        sl += (double)(m + (size_t)(d ^ 1) * G.plane)[j];
        st += (double)(m + (size_t)(kDeg + (d ^ 1)) * G.plane)[j];
    }
    const double bl = adiag64[i] + G.c * sl;
    const double bt = b64[i] + G.c * st;
    const double mu = bt / bl;
    mu_plane[i] = mu;
    if (mean) mean[k] = mu;
    if (var) var[k] = 1.0 / bl;
}

// FP64 residual partials: workgroup g sums (A mu - b)_i^2 and b_i^2 over the
// nodes g*256 + l + k*256*gridDim (fixed order), wave64 butterfly then LDS.
__global__ __launch_bounds__(256) void k_resid(Grid G, const double *__restrict__ mu,
                                               const double *__restrict__ adiag64,
                                               const double *__restrict__ b64,
                                               double *__restrict__ partials) {
    __shared__ double sh[2][4];
    const int64_t nodes = (int64_t)G.nx * G.ny * G.nt;
    double rr = 0.0, bb = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < nodes;
         k += (int64_t)gridDim.x * 256) {
        const int x = (int)(k % G.nx);
        const int y = (int)((k / G.nx) % G.ny);
        const int t = (int)(k / ((int64_t)G.nx * G.ny));
        const int64_t i = (int64_t)t * G.slice + (int64_t)y * G.pitch + x;
        const int kind = slice_kind(G, t);
        const double gi = (double)(axis_g(x, G.nx, G.bcx) + axis_g(y, G.ny, G.bcy));
        double r = adiag64[i] * mu[i];
        for (int d = 0; d < kDeg; ++d) {
            int xn, yn, tn;
            if (!nbr(G, x, y, t, d, xn, yn, tn)) continue;
            const int64_t j = (int64_t)tn * G.slice + (int64_t)yn * G.pitch + xn;
            const double gj = (double)(axis_g(xn, G.nx, G.bcx) + axis_g(yn, G.ny, G.bcy));
            r += coef<double>(d < 12 ? G.blk[kind] : G.blk[3], scls(d), gi, gj) * mu[j];
        }
        r -= b64[i];
        rr += r * r;
        bb += b64[i] * b64[i];
    }
    rr = wave_sum(rr);
    bb = wave_sum(bb);
    const int w = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0u) {
        sh[0][w] = rr;
        sh[1][w] = bb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        partials[2 * blockIdx.x + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

__global__ __launch_bounds__(256) void k_reduce(const double *__restrict__ partials, int npart,
                                                double *__restrict__ out) {
    __shared__ double sh[2][4];
    double a = 0.0, b = 0.0;
    for (int k = (int)threadIdx.x; k < npart; k += 256) {
        a += partials[2 * k];
        b += partials[2 * k + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63u) == 0u) {
        sh[0][w] = a;
        sh[1][w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        out[1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// Receiver-indexed copy: out[d][node] = message into node from node + off_d
// (sender plane d ^ 1 at the sender), 0 where the sender does not exist.
template <typename T>
__global__ __launch_bounds__(256) void k_msgs_get(Grid G, const T *__restrict__ m,
                                                  T *__restrict__ prec, T *__restrict__ info) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nodes = (int64_t)G.nx * G.ny * G.nt;
    if (k >= nodes) return;
    const int x = (int)(k % G.nx);
    const int y = (int)((k / G.nx) % G.ny);
    const int t = (int)(k / ((int64_t)G.nx * G.ny));
    for (int d = 0; d < kDeg; ++d) {
        int xn, yn, tn;
        T l = (T)0, th = (T)0;
        if (nbr(G, x, y, t, d, xn, yn, tn)) {
            const int64_t j = (int64_t)tn * G.slice + (int64_t)yn * G.pitch + xn;
            l = (m + (size_t)(d ^ 1) * G.plane)[j];
            th = (m + (size_t)(kDeg + (d ^ 1)) * G.plane)[j];
        }
        prec[(size_t)d * nodes + k] = l;
        info[(size_t)d * nodes + k] = th;
    }
}

// --------------------------------------------------------------------------
// Multigrid transfers (the paper's Algorithm 2, outer procedure, on the
// space-time lattice).  A coarse level keeps every second node of each of
// x, y and t, so coarse node (X, Y, N) sits on fine node (2X, 2Y, 2N).
// k_upsample: trilinear interpolation of a coarse FP64 mean onto the fine
// grid (dense [nt][ny][nx]); a fine coordinate between two coarse nodes takes
// their average, one past the last coarse node of a zero-flux axis takes that
// node's value, a periodic axis wraps.
// --------------------------------------------------------------------------
__device__ __forceinline__ void lerp_axis(int v, int nc, bool periodic, int &a, int &b) {
    a = v >> 1;
    b = (v & 1) ? a + 1 : a;
    if (b >= nc) b = periodic ? b - nc : nc - 1;
}

__global__ __launch_bounds__(256) void k_upsample(const double *__restrict__ coarse, int nxc,
                                                  int nyc, int ntc, int px, int py,
                                                  double *__restrict__ fine, int nx, int ny,
                                                  int nt) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)nx * ny * nt) return;
    const int x = (int)(k % nx);
    const int y = (int)((k / nx) % ny);
    const int t = (int)(k / ((int64_t)nx * ny));
    int xa, xb, ya, yb, ta, tb;
    lerp_axis(x, nxc, px != 0, xa, xb);
    lerp_axis(y, nyc, py != 0, ya, yb);
    lerp_axis(t, ntc, false, ta, tb);
    auto at = [&](int X, int Y, int N) {
        return coarse[((int64_t)N * nyc + Y) * nxc + X];
    };
    const double v = 0.125 * (at(xa, ya, ta) + at(xb, ya, ta) + at(xa, yb, ta) + at(xb, yb, ta) +
                              at(xa, ya, tb) + at(xb, ya, tb) + at(xa, yb, tb) + at(xb, yb, tb));
    fine[k] = v;
}

// Warm start from a predicted mean mu (dense FP64 [nt][ny][nx]): precision
// messages zero, information messages th_{i->j} = -(Q_ij/c) mu_i, so the
// beliefs start at mu + (b - A mu) / diag(A) (the fixed point when mu is the
// posterior mean).  The entries Q_ij/c are those the iteration uses.
template <typename T, bool PX, bool PY>
__global__ __launch_bounds__(256) void k_warm_init(Grid G, const double *__restrict__ mu,
                                                   T *__restrict__ m) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)G.nx * G.ny * G.nt) return;
    const int x = (int)(k % G.nx);
    const int y = (int)((k / G.nx) % G.ny);
    const int t = (int)(k / ((int64_t)G.nx * G.ny));
    const uint32_t i = (uint32_t)t * (uint32_t)G.slice + (uint32_t)(y * G.pitch + x);
    const int kind = slice_kind(G, t);
    const T pq_same[3] = {(T)G.blk[kind][0], (T)G.blk[kind][1], (T)G.blk[kind][2]};
    const T pq_cross[3] = {(T)G.blk[3][0], (T)G.blk[3][1], (T)G.blk[3][2]};
    const T gi = (T)g_at<PX, PY>(G, x, y);
    const T mi = (T)mu[k];
    for (int d = 0; d < kDeg; ++d) {
        int xn, yn, tn;
        const bool ok = nbr_at<PX, PY>(G, d, x, y, t, xn, yn, tn);
        T th = (T)0;
        if (ok) th = -(q_dir<T, false, PX, PY>(G, d, x, y, t, gi, pq_same, pq_cross) * mi);
        (m + (size_t)d * G.plane)[i] = (T)0;
        (m + (size_t)(kDeg + d) * G.plane)[i] = th;
    }
}

__global__ void k_zero_u32(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

}  // namespace st
}  // namespace gabp

// ==========================================================================
// Host side
// ==========================================================================
using gabp::st::Grid;

namespace {

thread_local std::string g_st_create_error;

struct Layout {
    int32_t pitch = 0;
    int64_t slice = 0, plane = 0, node_elems = 0;
    size_t msg[2] = {0, 0};
    size_t gain = 0, adiag64 = 0, b64 = 0, mu64 = 0, aw = 0, bw = 0;
    size_t partials = 0, red = 0, flags = 0, total = 0;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Layout make_layout(const gabp_st_model &m, size_t esize) {
    Layout l;
    const size_t row = 256 / esize;
    l.pitch = (int32_t)round_up((size_t)m.nx, row);
    l.slice = (int64_t)l.pitch * m.ny;
    l.node_elems = l.slice * m.nt;
    l.plane = (int64_t)(round_up((size_t)l.node_elems, row) + row);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = round_up(off + bytes, 256);
        return o;
    };
    const size_t buf = (size_t)(2 * gabp::st::kDeg) * (size_t)l.plane * esize;
    l.msg[0] = take(buf);
    l.msg[1] = take(buf);
    l.gain = take(buf / 2);
    const size_t n8 = (size_t)l.node_elems * 8;
    l.adiag64 = take(n8);
    l.b64 = take(n8);
    l.mu64 = take(n8);
    if (esize == 4) {
        l.aw = take((size_t)l.node_elems * 4);
        l.bw = take((size_t)l.node_elems * 4);
    }
    l.partials = take((size_t)gabp::st::kPartials * 2 * sizeof(double));
    l.red = take(8 * sizeof(double));
    l.flags = take(8 * sizeof(uint32_t));
    l.total = off;
    return l;
}

std::string check_model(const gabp_st_model *m, int32_t dtype) {
    if (!m) return "model is NULL";
    if (dtype != GABP_F32 && dtype != GABP_F64) return "dtype must be GABP_F32 or GABP_F64";
    if (m->nx < 1 || m->ny < 1 || m->nt < 1) return "nx, ny and nt must be >= 1";
    for (int32_t bc : {m->bc_x, m->bc_y})
        if (bc != GABP_BC_NEUMANN && bc != GABP_BC_PERIODIC)
            return "boundary must be GABP_BC_NEUMANN or GABP_BC_PERIODIC";
    if ((m->bc_x == GABP_BC_PERIODIC && m->nx < 5) || (m->bc_y == GABP_BC_PERIODIC && m->ny < 5))
        return "a periodic axis needs at least 5 cells";
    const int64_t pitch = (m->nx + 63) / 64 * 64;
    if (pitch * (int64_t)m->ny * (int64_t)m->nt >= ((int64_t)1 << 31))
        return "grid too large (nx*ny*nt, rows padded to 64, must stay below 2^31)";
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(m->dt) || !pos(m->h) || !pos(m->sigma_u) || !pos(m->a0) || !pos(m->kappa))
        return "dt, h, sigma_u, a0 and kappa must be finite and > 0";
    if (!std::isfinite(m->nu) || m->nu < 0.0) return "nu must be finite and >= 0";
    if (!std::isfinite(m->c) || m->c == 0.0) return "c must be finite and non-zero";
    return "";
}

// (p, q, r) of the four blocks and of L^2, times S (see the file comment).
void block_coefficients(const gabp_st_model &m, double blk[4][3], double lsq[3]) {
    const double S = m.dt * m.h * m.h / (m.sigma_u * m.sigma_u);
    const double a1 = 1.0 / m.dt, a2 = m.nu / (2.0 * m.h * m.h);
    const double l1 = m.a0 * m.kappa * m.kappa, l2 = m.a0 / (m.h * m.h);
    const double AA[3] = {a1 * a1, 2.0 * a1 * a2, a2 * a2};
    const double BB[3] = {a1 * a1, -2.0 * a1 * a2, a2 * a2};
    const double LL[3] = {l1 * l1, 2.0 * l1 * l2, l2 * l2};
    const double AB[3] = {a1 * a1, 0.0, -a2 * a2};
    for (int k = 0; k < 3; ++k) {
        blk[0][k] = S * (m.nt > 1 ? LL[k] + BB[k] : LL[k]);
        blk[1][k] = S * (AA[k] + BB[k]);
        blk[2][k] = S * AA[k];
        blk[3][k] = -S * AB[k];
        lsq[k] = S * LL[k];
    }
}

}  // namespace

struct gabp_st_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Grid G{};
    int dtype = 0;
    char *ws = nullptr;
    Layout lay;
    void *msg[2] = {nullptr, nullptr};
    double *adiag64 = nullptr, *b64 = nullptr, *mu64 = nullptr;
    void *aw = nullptr, *bw = nullptr;
    void *gain = nullptr;         // edge gains once the precision messages froze
    double *partials = nullptr, *red = nullptr;
    uint32_t *flags = nullptr;    // [0] diverged-at iteration, [1] input error,
                                  // [4, 5] precision messages changed by the last
                                  // iteration (64-bit), [6] their largest relative change
    uint32_t *host_flags = nullptr;   // pinned mirrors
    double *host_red = nullptr;
    int cur = 0;
    int64_t iter = 0;
    int64_t diverged_at = 0;
    bool frozen = false;
    int64_t frozen_at = -1;
    int64_t freeze_slots = 0;     // freeze tolerance (0: bitwise only)
    double freeze_rel = 0.0;
    int theta_slices = 1;         // slices per workgroup of the information-only kernel
    std::string err;
};

namespace {

gabp_status st_fail(gabp_st_ctx *ctx, gabp_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    else g_st_create_error = msg;
    return s;
}

#define ST_HIP(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return st_fail((ctx), GABP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

gabp_status st_ok(gabp_st_ctx *ctx) {
    if (!ctx) return GABP_E_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess)
        return st_fail(ctx, GABP_E_DEVICE, "hipSetDevice failed");
    return GABP_OK;
}

// Read the device flags back and fold a recorded divergence into the host state.
gabp_status st_sync(gabp_st_ctx *ctx) {
    ST_HIP(ctx, hipMemcpyAsync(ctx->host_flags, ctx->flags, 8 * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, ctx->stream));
    ST_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->host_flags[0] != 0u && ctx->diverged_at == 0) {
        ctx->diverged_at = ctx->host_flags[0];
        // the launch of that iteration completed; later ones wrote nothing
        ctx->cur = (int)(ctx->diverged_at & 1);
        ctx->iter = ctx->diverged_at;
    }
    if (ctx->diverged_at != 0)
        return st_fail(ctx, GABP_E_DIVERGED,
                       "non-positive cavity precision or non-finite message at iteration " +
                           std::to_string(ctx->diverged_at));
    return GABP_OK;
}

// One iteration of a mode: the information-only iteration in one launch
// over every tile; the others as the interior launch (tiles of the hole on
// slices 1 .. nt - 2), then the boundary launch.
template <typename T, int MODE, int SL, bool PX, bool PY>
void launch_parts(const Grid &G, const void *in, void *out, void *gain, const void *aw,
                  const void *bw, T eta, uint32_t *flags, uint32_t it, hipStream_t s) {
    using namespace gabp::st;
    if constexpr (MODE == MODE_THETA) {
        const unsigned n = (unsigned)(G.tiles_x * G.tiles_y * ((G.nt + SL - 1) / SL));
        hipLaunchKernelGGL((k_iter<T, MODE, PX, PY, SL, PART_ALL>), dim3(n), dim3(256 * SL), 0, s,
                           G, (const T *)in, (T *)out, (T *)gain, (const T *)aw, (const T *)bw,
                           eta, flags, it);
        return;
    } else {
        const gabp::TileRange h = st_hole(G);
        if (!h.empty() && G.nt >= 3) {
            const unsigned n = (unsigned)(h.hole_count() * ((G.nt - 2 + SL - 1) / SL));
            hipLaunchKernelGGL((k_iter<T, MODE, PX, PY, SL, PART_INTERIOR>), dim3(n), dim3(256 * SL),
                               0, s, G, (const T *)in, (T *)out, (T *)gain, (const T *)aw,
                               (const T *)bw, eta, flags, it);
        }
        const unsigned nb = (unsigned)st_boundary_count(G);
        if (nb > 0)
            hipLaunchKernelGGL((k_iter<T, MODE, PX, PY, 1, PART_BOUNDARY>), dim3(nb), dim3(256), 0, s,
                               G, (const T *)in, (T *)out, (T *)gain, (const T *)aw, (const T *)bw,
                               eta, flags, it);
    }
}

template <typename T, int MODE, int SL>
void launch_mode(const Grid &G, const void *in, void *out, void *gain, const void *aw,
                 const void *bw, T eta, uint32_t *flags, uint32_t it, hipStream_t s) {
    const bool px = G.bcx == GABP_BC_PERIODIC, py = G.bcy == GABP_BC_PERIODIC;
    if (px && py) launch_parts<T, MODE, SL, true, true>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else if (px) launch_parts<T, MODE, SL, true, false>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else if (py) launch_parts<T, MODE, SL, false, true>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else launch_parts<T, MODE, SL, false, false>(G, in, out, gain, aw, bw, eta, flags, it, s);
}

// mode's kernel; the information-only one covers theta_slices slices per
// workgroup (1, 2 or 4), the others one
template <typename T>
void launch_any(int mode, int theta_slices, const Grid &G, const void *in, void *out, void *gain,
                const void *aw, const void *bw, T eta, uint32_t *flags, uint32_t it,
                hipStream_t s) {
    using namespace gabp::st;
    if (mode == MODE_FULL)
        launch_mode<T, MODE_FULL, 1>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else if (mode == MODE_GAIN)
        launch_mode<T, MODE_GAIN, 1>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else if (theta_slices == 4)
        launch_mode<T, MODE_THETA, 4>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else if (theta_slices == 2)
        launch_mode<T, MODE_THETA, 2>(G, in, out, gain, aw, bw, eta, flags, it, s);
    else
        launch_mode<T, MODE_THETA, 1>(G, in, out, gain, aw, bw, eta, flags, it, s);
}

unsigned node_blocks(const Grid &G) {
    return (unsigned)(((int64_t)G.nx * G.ny * G.nt + 255) / 256);
}

}  // namespace

extern "C" {

const char *gabp_st_create_error(void) { return g_st_create_error.c_str(); }

gabp_status gabp_st_workspace_size(const gabp_st_model *model, int32_t dtype, size_t *bytes) {
    const std::string e = check_model(model, dtype);
    if (!e.empty()) return st_fail(nullptr, GABP_E_INVALID, e);
    if (!bytes) return st_fail(nullptr, GABP_E_INVALID, "bytes is NULL");
    *bytes = make_layout(*model, dtype == GABP_F32 ? 4 : 8).total;
    return GABP_OK;
}

gabp_status gabp_st_create(const gabp_st_model *model, const gabp_obs *obs,
                           const gabp_noise *noise, const double *prior_mean, int32_t dtype,
                           void *stream, gabp_st_ctx **out) {
    g_st_create_error.clear();
    if (!out) return st_fail(nullptr, GABP_E_INVALID, "out is NULL");
    *out = nullptr;
    const std::string me = check_model(model, dtype);
    if (!me.empty()) return st_fail(nullptr, GABP_E_INVALID, me);
    if (!obs || !noise) return st_fail(nullptr, GABP_E_INVALID, "obs and noise are required");
    if (obs->n < 0 || (obs->n > 0 && (!obs->cell || !obs->y)))
        return st_fail(nullptr, GABP_E_INVALID, "observation arrays missing");
    if (!noise->var && !(std::isfinite(noise->sigma) && noise->sigma > 0.0))
        return st_fail(nullptr, GABP_E_INVALID, "sigma must be finite and > 0");
    if (obs->n > 0 && !obs->on_device) {
        // host observations are checked before any device call
        const int64_t ncells = (int64_t)model->nx * model->ny * model->nt;
        for (int64_t k = 0; k < obs->n; ++k) {
            const double v = noise->var ? noise->var[k] : noise->sigma * noise->sigma;
            if (obs->cell[k] < 0 || obs->cell[k] >= ncells)
                return st_fail(nullptr, GABP_E_INVALID, "observation cell out of range");
            if (!std::isfinite(obs->y[k]) || !std::isfinite(v) || !(v > 0.0))
                return st_fail(nullptr, GABP_E_INVALID,
                               "non-finite observation or non-positive variance");
        }
    }
    gabp_st_ctx *ctx = new (std::nothrow) gabp_st_ctx();
    if (!ctx) return st_fail(nullptr, GABP_E_NOMEM, "host allocation failed");
    auto bail = [&](gabp_status s) {
        g_st_create_error = ctx->err;
        gabp_st_destroy(ctx);
        return s;
    };
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        ctx->err = "hipGetDevice failed";
        return bail(GABP_E_DEVICE);
    }
    ctx->stream = (hipStream_t)stream;
    ctx->dtype = dtype;
    const size_t esize = dtype == GABP_F32 ? 4 : 8;
    ctx->lay = make_layout(*model, esize);
    const Layout &l = ctx->lay;
    Grid &G = ctx->G;
    G.nx = model->nx;
    G.ny = model->ny;
    G.nt = model->nt;
    G.pitch = l.pitch;
    G.bcx = model->bc_x;
    G.bcy = model->bc_y;
    G.tiles_x = (model->nx + 63) / 64;
    G.tiles_y = (model->ny + 3) / 4;
    G.slice = l.slice;
    G.plane = l.plane;
    block_coefficients(*model, G.blk, G.lsq);
    G.c = model->c;
    G.inv_c = 1.0 / model->c;
    if ((int64_t)G.tiles_x * G.tiles_y * G.nt >= INT32_MAX) {
        ctx->err = "grid too large for one launch";
        return bail(GABP_E_INVALID);
    }
    if (hipMalloc((void **)&ctx->ws, l.total) != hipSuccess) {
        ctx->err = "device allocation of " + std::to_string(l.total) + " bytes failed";
        return bail(GABP_E_NOMEM);
    }
    if (hipHostMalloc((void **)&ctx->host_flags, 8 * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->host_red, 8 * sizeof(double)) != hipSuccess) {
        ctx->err = "pinned host allocation failed";
        return bail(GABP_E_NOMEM);
    }
    ctx->msg[0] = ctx->ws + l.msg[0];
    ctx->msg[1] = ctx->ws + l.msg[1];
    ctx->adiag64 = (double *)(ctx->ws + l.adiag64);
    ctx->b64 = (double *)(ctx->ws + l.b64);
    ctx->mu64 = (double *)(ctx->ws + l.mu64);
    ctx->aw = esize == 4 ? (void *)(ctx->ws + l.aw) : (void *)ctx->adiag64;
    ctx->bw = esize == 4 ? (void *)(ctx->ws + l.bw) : (void *)ctx->b64;
    ctx->gain = ctx->ws + l.gain;
    ctx->partials = (double *)(ctx->ws + l.partials);
    ctx->red = (double *)(ctx->ws + l.red);
    ctx->flags = (uint32_t *)(ctx->ws + l.flags);
    if (hipMemsetAsync(ctx->ws, 0, l.total, ctx->stream) != hipSuccess) {
        ctx->err = "hipMemsetAsync failed";
        return bail(GABP_E_DEVICE);
    }
    // observations on the device (staged when given on the host)
    const int64_t nobs = obs->n;
    int64_t *tc = nullptr;
    double *ty = nullptr, *tv = nullptr;
    const int64_t *dc = obs->cell;
    const double *dy = obs->y, *dv = noise->var;
    if (nobs > 0 && !obs->on_device) {
        bool ok = hipMalloc((void **)&tc, nobs * sizeof(int64_t)) == hipSuccess &&
                  hipMalloc((void **)&ty, nobs * sizeof(double)) == hipSuccess &&
                  (!noise->var || hipMalloc((void **)&tv, nobs * sizeof(double)) == hipSuccess) &&
                  hipMemcpyAsync(tc, obs->cell, nobs * sizeof(int64_t), hipMemcpyHostToDevice,
                                 ctx->stream) == hipSuccess &&
                  hipMemcpyAsync(ty, obs->y, nobs * sizeof(double), hipMemcpyHostToDevice,
                                 ctx->stream) == hipSuccess &&
                  (!noise->var || hipMemcpyAsync(tv, noise->var, nobs * sizeof(double),
                                                 hipMemcpyHostToDevice, ctx->stream) == hipSuccess);
        if (!ok) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(tc);
            (void)hipFree(ty);
            (void)hipFree(tv);
            ctx->err = "staging observations on the device failed";
            return bail(GABP_E_NOMEM);
        }
        dc = tc;
        dy = ty;
        dv = tv;
    }
    const double s2 = noise->var ? 0.0 : noise->sigma * noise->sigma;
    hipError_t e = gabp::launch_obs_fold(nobs, dc, dy, dv, s2,
                                         (int64_t)G.nx * G.ny * G.nt, G.nx, G.pitch, ctx->adiag64,
                                         ctx->b64, ctx->flags + 1, ctx->stream);
    (void)hipFree(tc);
    (void)hipFree(ty);
    (void)hipFree(tv);
    if (e == hipSuccess) {
        if (esize == 4)
            hipLaunchKernelGGL((gabp::st::k_node_init<float>), dim3(node_blocks(G)), dim3(256), 0,
                               ctx->stream, G, ctx->adiag64, ctx->b64, prior_mean, (float *)ctx->aw, (float *)ctx->bw,
                               ctx->flags + 1);
        else
            hipLaunchKernelGGL((gabp::st::k_node_init<double>), dim3(node_blocks(G)), dim3(256), 0,
                               ctx->stream, G, ctx->adiag64, ctx->b64, prior_mean, (double *)ctx->aw, (double *)ctx->bw,
                               ctx->flags + 1);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->host_flags, ctx->flags, 8 * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, ctx->stream);
    const hipError_t es = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) {
        ctx->err = std::string("set-up failed: ") + hipGetErrorString(e);
        return bail(GABP_E_DEVICE);
    }
    if (ctx->host_flags[1] != 0u) {
        ctx->err = "invalid observation (cell out of range, non-finite value or non-positive "
                   "variance) or non-finite prior mean";
        return bail(GABP_E_INVALID);
    }
    *out = ctx;
    return GABP_OK;
}

gabp_status gabp_st_iterate(gabp_st_ctx *ctx, int32_t n_iters, double damping) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (n_iters < 0) return st_fail(ctx, GABP_E_INVALID, "n_iters must be >= 0");
    if (!(damping > 0.0 && damping <= 1.0))
        return st_fail(ctx, GABP_E_INVALID, "damping must lie in (0, 1]");
    if (ctx->diverged_at != 0) return st_sync(ctx);
    if (ctx->iter + n_iters >= (int64_t)UINT32_MAX)
        return st_fail(ctx, GABP_E_INVALID, "iteration count would exceed 2^32 - 1");
    const Grid &G = ctx->G;
    const int mode = ctx->frozen ? gabp::st::MODE_THETA : gabp::st::MODE_FULL;
    for (int32_t k = 0; k < n_iters; ++k) {
        const uint32_t it = (uint32_t)(ctx->iter + 1);
        void *in = ctx->msg[ctx->cur], *out = ctx->msg[ctx->cur ^ 1];
        if (ctx->dtype == GABP_F32)
            launch_any<float>(mode, ctx->theta_slices, G, in, out, ctx->gain, ctx->aw, ctx->bw,
                              (float)damping, ctx->flags, it, ctx->stream);
        else
            launch_any<double>(mode, ctx->theta_slices, G, in, out, ctx->gain, ctx->aw, ctx->bw,
                               damping, ctx->flags, it, ctx->stream);
        ST_HIP(ctx, hipGetLastError());
        ctx->cur ^= 1;
        ctx->iter += 1;
    }
    return GABP_OK;
}

gabp_status gabp_st_posterior(gabp_st_ctx *ctx, double *mean, double *var) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    const Grid &G = ctx->G;
    if (ctx->dtype == GABP_F32)
        hipLaunchKernelGGL((gabp::st::k_post<float>), dim3(node_blocks(G)), dim3(256), 0,
                           ctx->stream, G, (const float *)ctx->msg[ctx->cur], ctx->adiag64,
                           ctx->b64, ctx->mu64, mean, var);
    else
        hipLaunchKernelGGL((gabp::st::k_post<double>), dim3(node_blocks(G)), dim3(256), 0,
                           ctx->stream, G, (const double *)ctx->msg[ctx->cur], ctx->adiag64,
                           ctx->b64, ctx->mu64, mean, var);
    ST_HIP(ctx, hipGetLastError());
    return GABP_OK;
}

gabp_status gabp_st_residual(gabp_st_ctx *ctx, double *rel_residual, double *abs_residual) {
    gabp_status s = st_sync(ctx);
    if (s != GABP_OK) return s;
    s = gabp_st_posterior(ctx, nullptr, nullptr);
    if (s != GABP_OK) return s;
    const Grid &G = ctx->G;
    const int64_t want = ((int64_t)G.nx * G.ny * G.nt + 255) / 256;
    const int nb = (int)std::min<int64_t>(want, gabp::st::kPartials);
    hipLaunchKernelGGL(gabp::st::k_resid, dim3(nb), dim3(256), 0, ctx->stream, G,
                       (const double *)ctx->mu64, (const double *)ctx->adiag64,
                       (const double *)ctx->b64, ctx->partials);
    hipLaunchKernelGGL(gabp::st::k_reduce, dim3(1), dim3(256), 0, ctx->stream,
                       (const double *)ctx->partials, nb, ctx->red);
    // freeze probe: did the last iteration change any precision message?
    // (the other buffer holds the previous iteration once one has run)
    const bool probe = !ctx->frozen && ctx->iter >= 1;
    if (probe) {
        const int64_t n = (int64_t)gabp::st::kDeg * G.plane;
        hipLaunchKernelGGL(gabp::st::k_zero_u32, dim3(1), dim3(64), 0, ctx->stream,
                           ctx->flags + 4, 3);
        const int pb = (int)std::min<int64_t>((n + 255) / 256, 4096);
        if (ctx->dtype == GABP_F32)
            hipLaunchKernelGGL(gabp::st::k_prec_change<float>, dim3(pb), dim3(256), 0,
                               ctx->stream, (const float *)ctx->msg[ctx->cur],
                               (const float *)ctx->msg[ctx->cur ^ 1], n,
                               (unsigned long long *)(ctx->flags + 4), ctx->flags + 6);
        else
            hipLaunchKernelGGL(gabp::st::k_prec_change<double>, dim3(pb), dim3(256), 0,
                               ctx->stream, (const double *)ctx->msg[ctx->cur],
                               (const double *)ctx->msg[ctx->cur ^ 1], n,
                               (unsigned long long *)(ctx->flags + 4), ctx->flags + 6);
        ST_HIP(ctx, hipMemcpyAsync(ctx->host_flags, ctx->flags, 8 * sizeof(uint32_t),
                                   hipMemcpyDeviceToHost, ctx->stream));
    }
    ST_HIP(ctx, hipGetLastError());
    ST_HIP(ctx, hipMemcpyAsync(ctx->host_red, ctx->red, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    ST_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double a = std::sqrt(ctx->host_red[0]), nb2 = std::sqrt(ctx->host_red[1]);
    if (!std::isfinite(a))
        return st_fail(ctx, GABP_E_DIVERGED, "non-finite residual");
    if (probe) {
        uint64_t changed;
        std::memcpy(&changed, ctx->host_flags + 4, sizeof changed);
        if (gabp::host::freeze_now(changed, ctx->host_flags[6], ctx->freeze_slots,
                                   ctx->freeze_rel)) {
            // gains from the current precisions; both buffers keep them
            if (ctx->dtype == GABP_F32)
                launch_any<float>(gabp::st::MODE_GAIN, 1, G, ctx->msg[ctx->cur], nullptr,
                                  ctx->gain, ctx->aw, ctx->bw, 0.0f, ctx->flags, 0u, ctx->stream);
            else
                launch_any<double>(gabp::st::MODE_GAIN, 1, G, ctx->msg[ctx->cur], nullptr,
                                   ctx->gain, ctx->aw, ctx->bw, 0.0, ctx->flags, 0u, ctx->stream);
            ST_HIP(ctx, hipGetLastError());
            const size_t esize = ctx->dtype == GABP_F32 ? 4 : 8;
            ST_HIP(ctx, hipMemcpyAsync(ctx->msg[ctx->cur ^ 1], ctx->msg[ctx->cur],
                                       (size_t)gabp::st::kDeg * (size_t)G.plane * esize,
                                       hipMemcpyDeviceToDevice, ctx->stream));
            ctx->frozen = true;
            ctx->frozen_at = ctx->iter;
        }
    }
    if (abs_residual) *abs_residual = a;
    if (rel_residual) *rel_residual = nb2 > 0.0 ? a / nb2 : a;
    return GABP_OK;
}

gabp_status gabp_st_set_freeze_tolerance(gabp_st_ctx *ctx, int64_t max_slots, double max_rel) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (max_slots < 0 || !std::isfinite(max_rel) || max_rel < 0.0)
        return st_fail(ctx, GABP_E_INVALID, "max_slots must be >= 0 and max_rel finite, >= 0");
    ctx->freeze_slots = max_slots;
    ctx->freeze_rel = max_rel;
    return GABP_OK;
}

gabp_status gabp_st_upsample_mean(const double *coarse, int32_t nxc, int32_t nyc, int32_t ntc,
                                  int32_t bc_x, int32_t bc_y, double *fine, int32_t nx,
                                  int32_t ny, int32_t nt, void *stream) {
    g_st_create_error.clear();
    if (!coarse || !fine) return st_fail(nullptr, GABP_E_INVALID, "upsample: NULL array");
    if (nx < 1 || ny < 1 || nt < 1 || (nx + 1) / 2 != nxc || (ny + 1) / 2 != nyc ||
        (nt + 1) / 2 != ntc)
        return st_fail(nullptr, GABP_E_INVALID,
                       "upsample: need ceil(n/2) coarse nodes on every axis");
    for (int32_t bc : {bc_x, bc_y})
        if (bc != GABP_BC_NEUMANN && bc != GABP_BC_PERIODIC)
            return st_fail(nullptr, GABP_E_INVALID, "upsample: boundary must be zero-flux or periodic");
    if ((bc_x == GABP_BC_PERIODIC && nx % 2) || (bc_y == GABP_BC_PERIODIC && ny % 2))
        return st_fail(nullptr, GABP_E_INVALID, "upsample: a periodic axis needs an even fine size");
    const int64_t n = (int64_t)nx * ny * nt;
    hipLaunchKernelGGL(gabp::st::k_upsample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, coarse, nxc, nyc, ntc,
                       (int)(bc_x == GABP_BC_PERIODIC), (int)(bc_y == GABP_BC_PERIODIC), fine, nx,
                       ny, nt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return st_fail(nullptr, GABP_E_DEVICE, std::string("upsample: ") + hipGetErrorString(e));
    return GABP_OK;
}

gabp_status gabp_st_warm_init(gabp_st_ctx *ctx, const double *mean) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (!mean) return st_fail(ctx, GABP_E_INVALID, "mean is NULL");
    if (ctx->diverged_at != 0) return st_fail(ctx, GABP_E_DIVERGED, "the run has diverged");
    const Grid &G = ctx->G;
    const bool px = G.bcx == GABP_BC_PERIODIC, py = G.bcy == GABP_BC_PERIODIC;
    const dim3 grid(node_blocks(G)), block(256);
    auto go = [&](auto kern, auto *buf) {
        hipLaunchKernelGGL(kern, grid, block, 0, ctx->stream, G, mean, buf);
    };
    if (ctx->dtype == GABP_F32) {
        float *m = (float *)ctx->msg[ctx->cur];
        if (px && py) go(gabp::st::k_warm_init<float, true, true>, m);
        else if (px) go(gabp::st::k_warm_init<float, true, false>, m);
        else if (py) go(gabp::st::k_warm_init<float, false, true>, m);
        else go(gabp::st::k_warm_init<float, false, false>, m);
    } else {
        double *m = (double *)ctx->msg[ctx->cur];
        if (px && py) go(gabp::st::k_warm_init<double, true, true>, m);
        else if (px) go(gabp::st::k_warm_init<double, true, false>, m);
        else if (py) go(gabp::st::k_warm_init<double, false, true>, m);
        else go(gabp::st::k_warm_init<double, false, false>, m);
    }
    ST_HIP(ctx, hipGetLastError());
    ctx->frozen = false;
    ctx->frozen_at = -1;
    return GABP_OK;
}

gabp_status gabp_st_set_theta_slices(gabp_st_ctx *ctx, int32_t slices) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (slices != 1 && slices != 2 && slices != 4)
        return st_fail(ctx, GABP_E_INVALID, "slices must be 1, 2 or 4");
    ctx->theta_slices = slices;
    return GABP_OK;
}

gabp_status gabp_st_precision_frozen(gabp_st_ctx *ctx, int64_t *frozen_at) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (!frozen_at) return st_fail(ctx, GABP_E_INVALID, "frozen_at is NULL");
    *frozen_at = ctx->frozen_at;
    return GABP_OK;
}

gabp_status gabp_st_solve(gabp_st_ctx *ctx, int64_t max_iters, double damping, double rel_tol,
                          int32_t check_every, int64_t *iters_done, double *rel_residual) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (max_iters < 0 || check_every <= 0 || !(rel_tol >= 0.0))
        return st_fail(ctx, GABP_E_INVALID,
                       "max_iters must be >= 0, check_every > 0 and rel_tol >= 0");
    int64_t done = 0;
    double rel = INFINITY, first = -1.0;
    s = gabp_st_residual(ctx, &rel, nullptr);
    while (s == GABP_OK && rel > rel_tol && done < max_iters) {
        const int32_t k = (int32_t)std::min<int64_t>(check_every, max_iters - done);
        s = gabp_st_iterate(ctx, k, damping);
        if (s != GABP_OK) break;
        done += k;
        s = gabp_st_residual(ctx, &rel, nullptr);
        if (s != GABP_OK) break;
        if (first < 0.0) first = rel;
        else if (rel > 1e3 * first) {
            s = st_fail(ctx, GABP_E_DIVERGED, "residual grew more than 1e3 times");
            break;
        }
    }
    if (iters_done) *iters_done = ctx->iter;
    if (rel_residual) *rel_residual = rel;
    if (s != GABP_OK) return s;
    return rel <= rel_tol ? GABP_OK : GABP_E_NOT_CONVERGED;
}

gabp_status gabp_st_get_messages(gabp_st_ctx *ctx, void *prec, void *info) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    if (!prec || !info) return st_fail(ctx, GABP_E_INVALID, "prec and info are required");
    const Grid &G = ctx->G;
    if (ctx->dtype == GABP_F32)
        hipLaunchKernelGGL((gabp::st::k_msgs_get<float>), dim3(node_blocks(G)), dim3(256), 0,
                           ctx->stream, G, (const float *)ctx->msg[ctx->cur], (float *)prec,
                           (float *)info);
    else
        hipLaunchKernelGGL((gabp::st::k_msgs_get<double>), dim3(node_blocks(G)), dim3(256), 0,
                           ctx->stream, G, (const double *)ctx->msg[ctx->cur], (double *)prec,
                           (double *)info);
    ST_HIP(ctx, hipGetLastError());
    return GABP_OK;
}

gabp_status gabp_st_iteration_count(gabp_st_ctx *ctx, int64_t *iters, int64_t *diverged_at) {
    gabp_status s = st_ok(ctx);
    if (s != GABP_OK) return s;
    s = st_sync(ctx);
    if (iters) *iters = ctx->iter;
    if (diverged_at) *diverged_at = ctx->diverged_at;
    return s == GABP_E_DIVERGED ? GABP_OK : s;
}

const char *gabp_st_last_error(gabp_st_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

void gabp_st_destroy(gabp_st_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    (void)hipFree(ctx->ws);
    (void)hipHostFree(ctx->host_flags);
    (void)hipHostFree(ctx->host_red);
    delete ctx;
}

}  // extern "C"
