// gfx950 auxiliary kernels of the lattice Gaussian belief propagation
// library: marginals, the FP64 residual and its deterministic reductions,
// problem set-up, checkpoint copies and the bitwise-change test.  The
// iteration kernels live in iter.hip.
//
// Message storage is SENDER indexed: plane d at (x, y) is the message FROM
// (x, y) TO (x, y) + off_d, so the incoming messages of a node are plane d^1
// at its neighbours.  The C ABI's checkpoint layout is receiver-indexed;
// k_msgs_get/k_msgs_set convert.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <atomic>

#include "internal.h"
#include "lattice.h"
#include "numerics.h"
#include "check_node.h"

// Rounding is spelled out: no implicit multiply-add contraction in this file,
// explicit fused multiply-adds where wanted.  The full iteration and the
// information-only iteration (after the precision messages have frozen) must
// round identically to stay bitwise equal.
#pragma clang fp contract(off)

namespace gabp {

// --------------------------------------------------------------------------
// Marginals (Compute Marginal) in FP64 from messages of precision T:
// Lam_i = A_ii + c sum Lam_{k->i}, th_i = b_i + c sum th_{k->i}; mu = th/Lam,
// var = 1/Lam.  Writes the pitched FP64 mean plane used by the residual and,
// when given, contiguous mean/var arrays.  Once the precision messages have
// frozen, Lam_i is a constant read from bel64 (FROZEN) and only the
// information messages are read; bel_out records Lam_i for that phase.
// --------------------------------------------------------------------------
template <typename T, int ALPHA, bool FROZEN>
__global__ __launch_bounds__(256) void k_post(Lattice L, const T *__restrict__ m,
                                              const double *__restrict__ adiag64,
                                              const double *__restrict__ b64,
                                              const double *__restrict__ bel64,
                                              double *__restrict__ mu_plane,
                                              double *__restrict__ mean,
                                              double *__restrict__ var,
                                              double *__restrict__ bel_out) {
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    post_node<T, ALPHA, FROZEN>(L, m, adiag64, b64, bel64, mu_plane, mean, var, bel_out, x, y);
}

// --------------------------------------------------------------------------
// FP64 residual r = A mu - b of the posterior-mean equations, A = Q + diag(p).
// Workgroup g (after XCD remapping) owns the g-th contiguous run of 64 x 4
// tiles in strip-major order, so the mean rows a tile shares with the tiles
// above, below and beside it are read once into its XCD's L2.  It takes its
// tiles kResidUnroll at a time: every thread first loads its share of each
// tile's (64 + 2R) x (4 + 2R) window of the mean (wrapped on periodic axes,
// zero outside the lattice) and its own node's diagonal and data term, then
// the windows go to LDS and every node reads its stencil from there.  Each
// node's arithmetic (resid_accum) and the order of the sums (tile by tile)
// are those of resid_node, so the r^2 and b^2 partials (wave64 butterfly,
// then LDS across the four waves, into partials[g]) are deterministic and do
// not depend on the staging.
// --------------------------------------------------------------------------
constexpr int kResidUnroll = 4;

template <int ALPHA>
__global__ __launch_bounds__(256) void k_resid(Lattice L, const double *__restrict__ mu,
                                               const double *__restrict__ adiag64,
                                               const double *__restrict__ b64,
                                               double *__restrict__ partials, int ntiles) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    constexpr int R = ALPHA == 1 ? 1 : 2;
    constexpr int WX = 64 + 2 * R, WY = 4 + 2 * R, WN = WX * WY;
    constexpr int LPT = (WN + 255) / 256;          // window loads per thread and tile
    constexpr int U = kResidUnroll;
    __shared__ double win[U][WY][WX];
    __shared__ double sh[2][4];
    double rr = 0.0, bb = 0.0;
    const int nb = (int)gridDim.x, g = xcd_remap((int)blockIdx.x, nb);
    const int per = ntiles / nb, extra = ntiles % nb;
    const int t0 = g * per + min(g, extra), t1 = t0 + per + (g < extra ? 1 : 0);
    const int rows = (L.ny + 3) / 4;
    const int lane = (int)(threadIdx.x & 63u), wrow = (int)(threadIdx.x >> 6);
    const bool px = L.bcx == BC_PERIODIC, py = L.bcy == BC_PERIODIC;
    // A tile is interior when its stencil never leaves the lattice.  Every
    // node of such a tile and its +-1 neighbours lie off the boundary rows
    // and columns, where ell takes one value, so the off-diagonal entries of
    // its rows depend on the direction only: q_in[d], evaluated as q_off does
    // at an interior position.
    auto interior_tile = [&](int tx0, int ty0) {
        return tx0 >= 2 * R && tx0 + 64 + 2 * R <= L.nx && ty0 >= 2 * R && ty0 + 4 + 2 * R <= L.ny;
    };
    double q_in[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d)
        q_in[d] = q_off<double>(L, d, 2 * R, 2 * R, 2 * R + dir_dx(d), 2 * R + dir_dy(d));
    for (int base = t0; base < t1; base += U) {
        const int n = min(U, t1 - base);
        int x0[U], y0[U];
        double wv[U][LPT], a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = 0.0;
            b[u] = 0.0;
#pragma unroll
            for (int q = 0; q < LPT; ++q) wv[u][q] = 0.0;
            if (u >= n) continue;
            int tx, ty;
            strip_order(base + u, L.tiles_x, rows, tx, ty);
            x0[u] = tx * 64;
            y0[u] = ty * 4;
#pragma unroll
            for (int q = 0; q < LPT; ++q) {
                const int e = (int)threadIdx.x + 256 * q;
                if (e >= WN) continue;
                int gx = x0[u] + e % WX - R, gy = y0[u] + e / WX - R;
                bool in = true;
                if (gx < 0 || gx >= L.nx) {
                    if (px) gx = (gx % L.nx + L.nx) % L.nx;   // the window may be wider
                    else in = false;                            // than the lattice
                }
                if (gy < 0 || gy >= L.ny) {
                    if (py) gy = (gy % L.ny + L.ny) % L.ny;
                    else in = false;
                }
                if (in) wv[u][q] = mu[(uint32_t)(gy * L.pitch + gx)];
            }
            const int x = x0[u] + lane, y = y0[u] + wrow;
            if (x < L.nx && y < L.ny) {
                const uint32_t i = (uint32_t)(y * L.pitch + x);
                a[u] = adiag64[i];
                b[u] = b64[i];
            }
        }
        __syncthreads();   // the previous round's readers are done with win
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < LPT; ++q) {
                const int e = (int)threadIdx.x + 256 * q;
                if (e < WN) win[u][e / WX][e % WX] = wv[u][q];
            }
        }
        __syncthreads();
        for (int u = 0; u < n; ++u) {
            const int x = x0[u] + lane, y = y0[u] + wrow;
            if (x >= L.nx || y >= L.ny) continue;
            if (interior_tile(x0[u], y0[u])) {
                // the arithmetic of resid_accum with every neighbour present
                double s = a[u] * win[u][wrow + R][lane + R];
#pragma unroll
                for (int d = 0; d < DEG; ++d)
                    s += q_in[d] * win[u][wrow + R + dir_dy(d)][lane + R + dir_dx(d)];
                const double r = s - b[u];
                rr += r * r;
                bb += b[u] * b[u];
                continue;
            }
            ResidIn<ALPHA> in;
            uint32_t j[DEG];
            node_nbrs<DEG, false>(L, x, y, j, in.xs, in.ys, in.ok);
#pragma unroll
            for (int d = 0; d < DEG; ++d)
                in.v[d] = win[u][wrow + R + dir_dy(d)][lane + R + dir_dx(d)];
            in.a = a[u];
            in.m0 = win[u][wrow + R][lane + R];
            in.b = b[u];
            resid_accum<ALPHA>(L, x, y, in, rr, bb);
        }
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
        partials[2 * g] = (sh[0][0] + sh[0][1]) + (sh[0][2] + sh[0][3]);
        partials[2 * g + 1] = (sh[1][0] + sh[1][1]) + (sh[1][2] + sh[1][3]);
    }
}

// Sum of |a - b| over a flat range of message slots (the paper's early-stop
// statistic); zero slots contribute nothing.  Deterministic partials.
template <typename T>
__global__ __launch_bounds__(256) void k_abs_change(const T *__restrict__ a,
                                                    const T *__restrict__ b, int64_t n,
                                                    double *__restrict__ partials) {
    __shared__ double sh[4];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride)
        s += fabs((double)a[k] - (double)b[k]);
    s = wave_sum(s);
    if ((threadIdx.x & 63u) == 0u) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// Fixed-order reduction of npart (pairs of) partials into out[0..1].
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

// --------------------------------------------------------------------------
// Problem setup (Section "Including Observations"): launch_obs_fold
// (obs.hip, deterministic) folds the observations into adiag64 (p_i) and b64
// (h_i); then k_node_init forms A_ii = Q_ii + p_i in FP64, b_i (+ (Q f_b)_i
// for a prior mean f_b), and the copies in message precision that the
// iteration reads.
template <typename T>
__global__ __launch_bounds__(256) void k_node_init(Lattice L, double *__restrict__ adiag64,
                                                   double *__restrict__ b64,
                                                   const double *__restrict__ prior_mean,
                                                   T *__restrict__ adiag_w, T *__restrict__ b_w,
                                                   uint32_t *__restrict__ err_flag) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t i = (int64_t)y * L.pitch + x;
    const double a = q_diag<double>(L, x, y) + adiag64[i];
    double b = b64[i];
    if (prior_mean) {
        double s = q_diag<double>(L, x, y) * prior_mean[(int64_t)y * L.nx + x];
        for (int d = 0; d < L.deg; ++d) {
            int xn, yn;
            if (!neighbour(L, x, y, d, xn, yn)) continue;
            s += q_off<double>(L, d, x, y, xn, yn) * prior_mean[(int64_t)yn * L.nx + xn];
        }
        if (!isfinite(s)) *err_flag = 1u;
        b += s;
    }
    adiag64[i] = a;
    b64[i] = b;
    if (adiag_w) adiag_w[i] = (T)a;
    if (b_w) b_w[i] = (T)b;
}

// Checkpoint copies between the sender-indexed message planes and the C ABI's
// dense receiver-indexed [deg][ny][nx] layout: receiver slot d of (x, y) is
// the message from s = (x, y) + off_d, i.e. sender plane d^1 at s.  Slots
// without a sender read as 0; set ignores them.
template <typename T>
__global__ __launch_bounds__(256) void k_msgs_get(Lattice L, const T *__restrict__ m,
                                                  T *__restrict__ prec, T *__restrict__ info) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t n = (int64_t)L.nx * L.ny, o = (int64_t)y * L.nx + x;
    for (int d = 0; d < L.deg; ++d) {
        int xn, yn;
        const bool ok = neighbour(L, x, y, d, xn, yn);
        const int64_t s = (int64_t)yn * L.pitch + xn;
        if (prec) prec[d * n + o] = ok ? m[(d ^ 1) * L.plane + s] : (T)0;
        if (info) info[d * n + o] = ok ? m[(L.deg + (d ^ 1)) * L.plane + s] : (T)0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_msgs_set(Lattice L, T *__restrict__ m,
                                                  const T *__restrict__ prec,
                                                  const T *__restrict__ info) {
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const int64_t n = (int64_t)L.nx * L.ny, o = (int64_t)y * L.nx + x;
    for (int d = 0; d < L.deg; ++d) {
        int xn, yn;
        if (!neighbour(L, x, y, d, xn, yn)) continue;
        const int64_t s = (int64_t)yn * L.pitch + xn;
        if (prec) m[(d ^ 1) * L.plane + s] = prec[d * n + o];
        if (info) m[(L.deg + (d ^ 1)) * L.plane + s] = info[d * n + o];
    }
}

// Change of the precision messages between two buffers: *count += the
// number of the n elements whose bits differ (64-bit: n may exceed 2^32),
// *maxrel = max of the relative
// changes |a - b| / max(|a|, |b|) over them, as the bits of a non-negative
// float (+inf for a non-finite element), so that unsigned comparison orders
// them.  Both are independent of the order of the atomics.
template <typename T>
__global__ __launch_bounds__(256) void k_prec_change(const T *__restrict__ a,
                                                     const T *__restrict__ b, int64_t n,
                                                     unsigned long long *__restrict__ count,
                                                     uint32_t *__restrict__ maxrel) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint32_t c = 0u;   // per thread: at most n / stride + 1 elements
    float mr = 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += stride) {
        const T x = a[k], y = b[k];
        const bool diff = sizeof(T) == 4
                              ? __float_as_uint((float)x) != __float_as_uint((float)y)
                              : __double_as_longlong((double)x) != __double_as_longlong((double)y);
        if (!diff) continue;
        ++c;
        const double dx = (double)x, dy = (double)y, d = fabs(dx - dy);
        const double m = fmax(fabs(dx), fabs(dy));
        const float rel = !isfinite(d) || !isfinite(m) ? INFINITY : d == 0.0 ? 0.0f : (float)(d / m);
        mr = fmaxf(mr, rel);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        c += (uint32_t)__shfl_xor((int)c, o, 64);
        mr = fmaxf(mr, __shfl_xor(mr, o, 64));
    }
    if ((threadIdx.x & 63u) == 0u && c != 0u) {
        atomicAdd(count, (unsigned long long)c);
        atomicMax(maxrel, __float_as_uint(mr));
    }
}

// Multigrid transfer: coarse node (i, j) sits on fine node (2i, 2j); every
// fine node takes the bilinear interpolation of the coarse mean (wrapping on
// periodic axes, clamped at the end of others) into channel 0 of a
// prediction [nyf][nxf][16] (other channels zero).
__global__ __launch_bounds__(256) void k_upsample_mean(const double *__restrict__ coarse,
                                                       int nxc, int nyc, int perx, int pery,
                                                       float *__restrict__ pred, int nxf,
                                                       int nyf) {
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long)nxf * nyf) return;
    const int x = (int)(p % nxf), y = (int)(p / nxf);
    const int i0 = x >> 1, j0 = y >> 1;
    int i1 = i0 + (x & 1), j1 = j0 + (y & 1);
    if (i1 >= nxc) i1 = perx ? i1 - nxc : nxc - 1;
    if (j1 >= nyc) j1 = pery ? j1 - nyc : nyc - 1;
    const int ia = min(i0, nxc - 1), ja = min(j0, nyc - 1);
    const double v = 0.25 * (coarse[(long)ja * nxc + ia] + coarse[(long)ja * nxc + i1] +
                             coarse[(long)j1 * nxc + ia] + coarse[(long)j1 * nxc + i1]);
    float *o = pred + p * 16;
    o[0] = (float)v;
#pragma unroll
    for (int k = 1; k < 16; ++k) o[k] = 0.0f;
}

// Multigrid transfer of the precision messages: fine node (x, y) is covered
// by coarse node (x/2, y/2) (clamped at the end of an axis); channel 1 + d of
// the prediction gets log(scale * -Lam) of the coarse sender-indexed precision
// message in direction d, or in the opposite direction where the coarse node
// has no neighbour in direction d, or -inf (a zero message) where it has
// neither.  Channel 0 and channels past the stencil are left untouched.
template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_upscale_prec(Lattice Lc, const T *__restrict__ m,
                                                      float scale, float *__restrict__ pred,
                                                      int nxf, int nyf) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long)nxf * nyf) return;
    const int x = (int)(p % nxf), y = (int)(p / nxf);
    const int xc = min(x >> 1, Lc.nx - 1), yc = min(y >> 1, Lc.ny - 1);
    const size_t ic = (size_t)yc * Lc.pitch + xc;
    float *o = pred + p * 16 + 1;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        int xn, yn;
        int src = -1;
        if (neighbour(Lc, xc, yc, d, xn, yn)) src = d;
        else if (neighbour(Lc, xc, yc, d ^ 1, xn, yn)) src = d ^ 1;
        float v = -INFINITY;
        if (src >= 0) {
            const float lam = -(float)(m + (size_t)src * Lc.plane)[ic];
            if (lam > 0.0f) v = logf(scale * lam);
        }
        o[d] = v;
    }
}

// The paper's Upscale Messages taken literally: every message of the fine
// grid (both components, sender-indexed plane d at fine node (x, y)) starts
// as the coarse grid's message from the covering node (x/2, y/2) in the same
// direction (the opposite one where the coarse node has none in that
// direction, zero where it has neither), unscaled.  Slots whose fine
// neighbour does not exist stay zero.
template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_copy_coarse(Lattice Lc, const T *__restrict__ mc,
                                                     Lattice Lf, T *__restrict__ mf) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const long p = (long)blockIdx.x * 256 + threadIdx.x;
    if (p >= (long)Lf.nx * Lf.ny) return;
    const int x = (int)(p % Lf.nx), y = (int)(p / Lf.nx);
    const int xc = min(x >> 1, Lc.nx - 1), yc = min(y >> 1, Lc.ny - 1);
    const size_t ic = (size_t)yc * Lc.pitch + xc;
    const size_t i = (size_t)y * Lf.pitch + x;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        int xn, yn;
        T l = (T)0, th = (T)0;
        if (neighbour(Lf, x, y, d, xn, yn)) {
            int src = -1;
            if (neighbour(Lc, xc, yc, d, xn, yn)) src = d;
            else if (neighbour(Lc, xc, yc, d ^ 1, xn, yn)) src = d ^ 1;
            if (src >= 0) {
                l = (mc + (size_t)src * Lc.plane)[ic];
                th = (mc + (size_t)(DEG + src) * Lc.plane)[ic];
            }
        }
        (mf + (size_t)d * Lf.plane)[i] = l;
        (mf + (size_t)(DEG + d) * Lf.plane)[i] = th;
    }
}

__global__ void k_set_u32(uint32_t *p, uint32_t v) {
    if (threadIdx.x == 0) *p = v;
}

__global__ void k_add_u32(uint32_t *p, uint32_t k) {
    if (threadIdx.x == 0) *p += k;
}

// --------------------------------------------------------------------------
// host launchers
// --------------------------------------------------------------------------
static inline int tiles_of(const Lattice &L) {
    return L.tiles_x * ((L.ny + 3) / 4);
}

hipError_t launch_prec_change(int dtype, const void *a, const void *b, int64_t n,
                              unsigned long long *count, uint32_t *maxrel, hipStream_t s) {
    int64_t want = (n + 255) / 256;
    const int nb = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
    if (dtype == 0)
        hipLaunchKernelGGL((k_prec_change<float>), dim3(nb), dim3(256), 0, s, (const float *)a,
                           (const float *)b, n, count, maxrel);
    else
        hipLaunchKernelGGL((k_prec_change<double>), dim3(nb), dim3(256), 0, s, (const double *)a,
                           (const double *)b, n, count, maxrel);
    return hipGetLastError();
}

template <typename T, int ALPHA>
static void launch_post_a(bool frozen, const Lattice &L, const void *m, const double *adiag64,
                          const double *b64, const double *bel64, double *mu_plane,
                          double *mean, double *var, double *bel_out, hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (frozen)
        hipLaunchKernelGGL((k_post<T, ALPHA, true>), grid, block, 0, s, L, (const T *)m, adiag64,
                           b64, bel64, mu_plane, mean, var, (double *)nullptr);
    else
        hipLaunchKernelGGL((k_post<T, ALPHA, false>), grid, block, 0, s, L, (const T *)m, adiag64,
                           b64, bel64, mu_plane, mean, var, bel_out);
}

hipError_t launch_post(int dtype, const Lattice &L, const void *m, const double *adiag64,
                       const double *b64, const double *bel64, double *mu_plane, double *mean,
                       double *var, double *bel_out, hipStream_t s) {
    const bool fr = bel64 != nullptr;
    if (dtype == 0) {
        if (L.alpha == 1) launch_post_a<float, 1>(fr, L, m, adiag64, b64, bel64, mu_plane, mean, var, bel_out, s);
        else launch_post_a<float, 2>(fr, L, m, adiag64, b64, bel64, mu_plane, mean, var, bel_out, s);
    } else {
        if (L.alpha == 1) launch_post_a<double, 1>(fr, L, m, adiag64, b64, bel64, mu_plane, mean, var, bel_out, s);
        else launch_post_a<double, 2>(fr, L, m, adiag64, b64, bel64, mu_plane, mean, var, bel_out, s);
    }
    return hipGetLastError();
}

// Workgroups of the residual kernel that are resident at once on the current
// device (its occupancy times the CU count), so that its one wave of
// workgroups has no tail; cached per device and stencil.
static int resident_resid_blocks(int alpha) {
    static std::atomic<int> cache[16][2];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
    const int a = alpha == 1 ? 0 : 1;
    int v = cache[dev][a].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int per_cu = 0, cus = 0;
    const hipError_t e1 =
        alpha == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_resid<1>, 256, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_resid<2>, 256, 0);
    const hipError_t e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e1 != hipSuccess || e2 != hipSuccess || per_cu <= 0 || cus <= 0) return 0;
    v = per_cu * cus;
    cache[dev][a].store(v, std::memory_order_relaxed);
    return v;
}

hipError_t launch_resid(const Lattice &L, const double *mu, const double *adiag64,
                        const double *b64, double *partials, int npart, double *out,
                        hipStream_t s) {
    const int nt = tiles_of(L);
    int nb = nt < npart ? nt : npart;
    const int resident = resident_resid_blocks(L.alpha);
    if (resident > 0 && resident < nb) nb = resident;
    if (L.alpha == 1)
        hipLaunchKernelGGL((k_resid<1>), dim3(nb), dim3(256), 0, s, L, mu, adiag64, b64, partials,
                           nt);
    else
        hipLaunchKernelGGL((k_resid<2>), dim3(nb), dim3(256), 0, s, L, mu, adiag64, b64, partials,
                           nt);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, (const double *)partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_abs_change(int dtype, const void *a, const void *b, int64_t n,
                             double *partials, int npart, double *out, hipStream_t s) {
    int64_t want = (n + 255) / 256;
    const int nb = (int)(want < npart ? (want > 0 ? want : 1) : npart);
    if (dtype == 0)
        hipLaunchKernelGGL((k_abs_change<float>), dim3(nb), dim3(256), 0, s, (const float *)a,
                           (const float *)b, n, partials);
    else
        hipLaunchKernelGGL((k_abs_change<double>), dim3(nb), dim3(256), 0, s, (const double *)a,
                           (const double *)b, n, partials);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, (const double *)partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_setup(int dtype, const Lattice &L, int64_t nobs, const int64_t *cell,
                        const double *y, const double *var, double sigma2, double *adiag64,
                        double *b64, const double *prior_mean, void *adiag_w, void *b_w,
                        uint32_t *err_flag, hipStream_t s) {
    if (nobs > 0) {
        const hipError_t e = launch_obs_fold(nobs, cell, y, var, sigma2, (int64_t)L.nx * L.ny, L.nx,
                                             L.pitch, adiag64, b64, err_flag, s);
        if (e != hipSuccess) return e;
    }
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_node_init<float>), grid, block, 0, s, L, adiag64, b64, prior_mean,
                           (float *)adiag_w, (float *)b_w, err_flag);
    else
        hipLaunchKernelGGL((k_node_init<double>), grid, block, 0, s, L, adiag64, b64, prior_mean,
                           (double *)nullptr, (double *)nullptr, err_flag);
    return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t *p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_add_u32(uint32_t *p, uint32_t k, hipStream_t s) {
    hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(64), 0, s, p, k);
    return hipGetLastError();
}

hipError_t launch_upsample_mean(const double *coarse, int nxc, int nyc, int perx, int pery,
                                float *pred, int nxf, int nyf, hipStream_t s) {
    const long n = (long)nxf * nyf;
    hipLaunchKernelGGL(k_upsample_mean, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, coarse,
                       nxc, nyc, perx, pery, pred, nxf, nyf);
    return hipGetLastError();
}

hipError_t launch_upscale_prec(int dtype, const Lattice &Lc, const void *m, float scale,
                               float *pred, int nxf, int nyf, hipStream_t s) {
    const long n = (long)nxf * nyf;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dtype == 0) {
        if (Lc.alpha == 1)
            hipLaunchKernelGGL((k_upscale_prec<float, 1>), grid, block, 0, s, Lc, (const float *)m, scale, pred, nxf, nyf);
        else
            hipLaunchKernelGGL((k_upscale_prec<float, 2>), grid, block, 0, s, Lc, (const float *)m, scale, pred, nxf, nyf);
    } else {
        if (Lc.alpha == 1)
            hipLaunchKernelGGL((k_upscale_prec<double, 1>), grid, block, 0, s, Lc, (const double *)m, scale, pred, nxf, nyf);
        else
            hipLaunchKernelGGL((k_upscale_prec<double, 2>), grid, block, 0, s, Lc, (const double *)m, scale, pred, nxf, nyf);
    }
    return hipGetLastError();
}

hipError_t launch_copy_coarse(int dtype, const Lattice &Lc, const void *mc, const Lattice &Lf,
                              void *mf, hipStream_t s) {
    const long n = (long)Lf.nx * Lf.ny;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dtype == 0) {
        if (Lc.alpha == 1)
            hipLaunchKernelGGL((k_copy_coarse<float, 1>), grid, block, 0, s, Lc, (const float *)mc, Lf, (float *)mf);
        else
            hipLaunchKernelGGL((k_copy_coarse<float, 2>), grid, block, 0, s, Lc, (const float *)mc, Lf, (float *)mf);
    } else {
        if (Lc.alpha == 1)
            hipLaunchKernelGGL((k_copy_coarse<double, 1>), grid, block, 0, s, Lc, (const double *)mc, Lf, (double *)mf);
        else
            hipLaunchKernelGGL((k_copy_coarse<double, 2>), grid, block, 0, s, Lc, (const double *)mc, Lf, (double *)mf);
    }
    return hipGetLastError();
}

hipError_t launch_msgs_get(int dtype, const Lattice &L, const void *m, void *prec, void *info,
                           hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_msgs_get<float>), grid, block, 0, s, L, (const float *)m,
                           (float *)prec, (float *)info);
    else
        hipLaunchKernelGGL((k_msgs_get<double>), grid, block, 0, s, L, (const double *)m,
                           (double *)prec, (double *)info);
    return hipGetLastError();
}

hipError_t launch_msgs_set(int dtype, const Lattice &L, void *m, const void *prec,
                           const void *info, hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL((k_msgs_set<float>), grid, block, 0, s, L, (float *)m,
                           (const float *)prec, (const float *)info);
    else
        hipLaunchKernelGGL((k_msgs_set<double>), grid, block, 0, s, L, (double *)m,
                           (const double *)prec, (const double *)info);
    return hipGetLastError();
}

}  // namespace gabp
