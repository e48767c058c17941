// gfx950 iteration kernels of the lattice Gaussian belief propagation
// library: the full flooding iteration, the edge-gain set-up and the
// information-only iteration used once the precision messages have frozen.
//
// Message storage: two ping-pong buffers, each 2*deg planes (deg precision
// planes, then deg information planes) of the message precision T, SENDER
// indexed: plane d at (x, y) is the message FROM (x, y) TO (x, y) + off_d.
// A sender therefore reads its old outgoing messages (for damping) and
// writes the new ones at its own, aligned, position; only the incoming
// messages of a node are read at shifted positions (plane d^1 at the
// neighbour).  Iteration t reads buffer (t-1)&1 and writes buffer t&1
// (flooding schedule: every new message depends only on the previous
// iteration's messages).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "internal.h"
#include "lattice.h"
#include "numerics.h"
#include "iter_node.h"
#include "pair_tile.h"
#include "walk_strip.h"

// Rounding is spelled out: no implicit multiply-add contraction in this file,
// explicit fused multiply-adds where wanted.  The full iteration and the
// information-only iteration must round identically to stay bitwise equal.
#pragma clang fp contract(off)

namespace gabp {

// One workgroup = 256 threads on a 64 x (4*RPT) tile: lane -> column, wave ->
// row, each thread walks RPT rows 4 apart.  The tile shape is a tuning knob
// (gabp_autotune); results do not depend on it.
template <typename T, int ALPHA, int RPT>
__global__ __launch_bounds__(256) void k_iter_direct(Lattice L, const T *__restrict__ m_in,
                                                     T *__restrict__ m_out,
                                                     const T *__restrict__ adiag,
                                                     const T *__restrict__ bw, T eta,
                                                     uint32_t *__restrict__ diverged_at,
                                                     const uint32_t *__restrict__ t_base, uint32_t t_off) {
    if (*diverged_at != 0u) return;
    const uint32_t t = *t_base + t_off;   // this iteration's number
    constexpr int TH = 4 * RPT;
    int tx, ty;
    strip_order(xcd_remap((int)blockIdx.x, (int)gridDim.x), L.tiles_x, (L.ny + TH - 1) / TH, tx,
                ty);
    const int x = tx * 64 + (int)(threadIdx.x & 63u);
    const int y0 = ty * TH + (int)(threadIdx.x >> 6);
    const bool interior = tx * 64 >= 2 && tx * 64 + 66 <= L.nx && ty * TH >= 2 &&
                          ty * TH + TH + 2 <= L.ny;
    bool bad = false;
    if (interior) {
#pragma unroll 1
        for (int k = 0; k < RPT; ++k)
            iter_node<T, ALPHA, true>(L, m_in, m_out, adiag, bw, eta, bad, x, y0 + 4 * k);
    } else if (x < L.nx) {
#pragma unroll 1
        for (int k = 0; k < RPT; ++k)
            if (y0 + 4 * k < L.ny)
                iter_node<T, ALPHA, false>(L, m_in, m_out, adiag, bw, eta, bad, x, y0 + 4 * k);
    }
    if (bad) *diverged_at = t;
}

// --------------------------------------------------------------------------
// Frozen precision messages.  The precision recursion involves neither the
// information messages nor the data, so once one iteration leaves every
// precision message bitwise unchanged, all later iterations do too.  From
// then on the gains g_{i->j} are constants: k_gain stores them once
// (sender-indexed, plane d at i) and k_iter_theta updates only the
// information messages, reading 12 bytes per edge instead of 16 (FP32)
// with results bitwise equal to the full iteration's.
// --------------------------------------------------------------------------
template <typename T, int ALPHA>
__global__ __launch_bounds__(256) void k_gain(Lattice L, const T *__restrict__ m,
                                              const T *__restrict__ adiag,
                                              T *__restrict__ gain) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const int tile = (int)blockIdx.x;
    const int x = (tile % L.tiles_x) * 64 + (int)(threadIdx.x & 63u);
    const int y = (tile / L.tiles_x) * 4 + (int)(threadIdx.x >> 6);
    if (x >= L.nx || y >= L.ny) return;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    node_nbrs<DEG, false>(L, x, y, j, xs, ys, ok);
    T lin[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const T v = (m + (size_t)(d ^ 1) * L.plane)[j[d]];
        lin[d] = ok[d] ? v : (T)0;
    }
    T sl = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) sl += lin[d];
    const T bl = fmadd((T)L.c, sl, adiag[i]);
    const T li = ALPHA == 2 ? ell<T>(L, x, y) : (T)0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        if (!ok[d]) continue;
        const T q = q_over_c<T, ALPHA>(L, d, li, xs[d], ys[d]);
        (gain + (size_t)d * L.plane)[i] = edge_gain(q, bl - lin[d]);
    }
}

template <typename T, int ALPHA, int RPT>
__global__ __launch_bounds__(256) void k_iter_theta(Lattice L, const T *__restrict__ m_in,
                                                    T *__restrict__ m_out,
                                                    const T *__restrict__ gain,
                                                    const T *__restrict__ bw, T eta,
                                                    uint32_t *__restrict__ diverged_at,
                                                    const uint32_t *__restrict__ t_base, uint32_t t_off) {
    if (*diverged_at != 0u) return;
    const uint32_t t = *t_base + t_off;   // this iteration's number
    constexpr int TH = 4 * RPT;
    int tx, ty;
    strip_order(xcd_remap((int)blockIdx.x, (int)gridDim.x), L.tiles_x, (L.ny + TH - 1) / TH, tx,
                ty);
    const int x = tx * 64 + (int)(threadIdx.x & 63u);
    const int y0 = ty * TH + (int)(threadIdx.x >> 6);
    const bool interior = tx * 64 >= 2 && tx * 64 + 66 <= L.nx && ty * TH >= 2 &&
                          ty * TH + TH + 2 <= L.ny;
    bool bad = false;
    if (interior) {
#pragma unroll 1
        for (int k = 0; k < RPT; ++k)
            iter_theta_node<T, ALPHA, true>(L, m_in, m_out, gain, bw, eta, bad, x, y0 + 4 * k);
    } else if (x < L.nx) {
#pragma unroll 1
        for (int k = 0; k < RPT; ++k)
            if (y0 + 4 * k < L.ny)
                iter_theta_node<T, ALPHA, false>(L, m_in, m_out, gain, bw, eta, bad, x,
                                                 y0 + 4 * k);
    }
    if (bad) *diverged_at = t;
}

// A two-iteration pass is one launch over two sets of 64 x TH tiles (on any
// lattice; a small one may have no interior tiles): the first nring
// workgroups take the ring (the
// tiles whose halo reaches a boundary, TileRange::ring order) on the
// boundary code path; the others walk the tile grid in strip order and take
// the interior tiles (a ring tile there returns at once) on a path compiled
// without boundary code, with the halo bands' direction sets fixed at compile
// time.  The ring runs alongside the first interior tiles instead of as a
// second launch after them.  The interior path of an FP32 16-row tile takes
// 97 VGPRs and the ring path 110, both four waves per SIMD (two 8-wave
// workgroups per CU); 12-row tiles take 74 (two 12-wave workgroups).  Both
// paths return only for a divergence recorded by an earlier pass (an
// iteration <= t), so the pass that diverges is written whole.
template <typename T, int ALPHA, int TH, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_iter_theta2(Lattice L, TileRange in, int nring,
                                                            const T *__restrict__ m_in,
                                                            T *__restrict__ m_out,
                                                            const T *__restrict__ gain,
                                                            const T *__restrict__ bw, T eta,
                                                            uint32_t *__restrict__ diverged_at,
                                                            const uint32_t *__restrict__ t_base,
                                                            uint32_t t_off) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    __shared__ T lds[DEG * TH * 64];
    const uint32_t t = *t_base + t_off;           // the iteration the launch starts from
    const uint32_t seen = *diverged_at;
    if (seen != 0u && seen <= t) return;          // uniform across the workgroup
    bool bad1 = false, bad2 = false;
    int tx, ty;
    const int b = (int)blockIdx.x;
    if (b < nring) {
        if ((int64_t)b >= in.ring_count()) return;   // nring is rounded up to the XCD count
        in.ring(b, tx, ty);
        pair_tile<T, ALPHA, TH, WAVES, false>(L, m_in, m_out, gain, bw, eta, tx, ty, lds, bad1,
                                              bad2);
    } else {
        // strip-major tile order: tiles above and below share their halo
        // rows in one XCD's L2
        strip_order(xcd_remap(b - nring, (int)gridDim.x - nring), L.tiles_x, in.rows, tx, ty);
        if (!in.interior(tx, ty)) return;
        pair_tile<T, ALPHA, TH, WAVES, true>(L, m_in, m_out, gain, bw, eta, tx, ty, lds, bad1,
                                             bad2);
    }
    if (bad1 || bad2) record_divergence(diverged_at, bad1 ? t + 1u : t + 2u);
}

// Column-strip walker (walk_strip.h): one workgroup per (strip, segment)
// pair, segment-major so that each XCD's contiguous range of workgroups
// covers neighbouring strips of the same rows (their overlap columns then
// meet in one L2).
template <typename T, int ALPHA, int RB>
__global__ __launch_bounds__(64 * RB) void k_iter_theta2w(Lattice L, const T *__restrict__ m_in,
                                                          T *__restrict__ m_out,
                                                          const T *__restrict__ gain,
                                                          const T *__restrict__ bw, T eta,
                                                          uint32_t *__restrict__ diverged_at,
                                                          const uint32_t *__restrict__ t_base,
                                                          uint32_t t_off, int seglen) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    constexpr int R = ALPHA == 1 ? 1 : 2;
    __shared__ T lds[WalkRing<RB>::kRows * DEG * (64 + 2 * R)];
    if (*diverged_at != 0u) return;               // uniform across the workgroup
    const uint32_t t = *t_base + t_off;           // the iteration the launch starts from
    const int g = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int seg = g / L.tiles_x, strip = g - seg * L.tiles_x;
    const int Y0 = seg * seglen;
    if (Y0 >= L.ny) return;
    const int Y1 = min(L.ny, Y0 + seglen);
    bool bad1 = false, bad2 = false;
    walk_strip<T, ALPHA, RB>(L, m_in, m_out, gain, bw, eta, strip * 64, Y0, Y1, lds, bad1, bad2);
    if (bad1 || bad2) record_divergence(diverged_at, bad1 ? t + 1u : t + 2u);
}

static inline int tiles_of(const Lattice &L) {
    return L.tiles_x * ((L.ny + 3) / 4);
}

template <typename T, int ALPHA, int RPT>
static void launch_iter_k(const Lattice &L, const void *m_in, void *m_out, const void *adiag,
                          const void *bw, double eta, uint32_t *flag, const uint32_t *t_base,
                          uint32_t t_off, hipStream_t s) {
    const int tiles = L.tiles_x * ((L.ny + 4 * RPT - 1) / (4 * RPT));
    hipLaunchKernelGGL((k_iter_direct<T, ALPHA, RPT>), dim3(tiles), dim3(256), 0, s, L,
                       (const T *)m_in, (T *)m_out, (const T *)adiag, (const T *)bw, (T)eta, flag,
                       t_base, t_off);
}

template <typename T, int ALPHA>
static void launch_iter_a(int rpt, const Lattice &L, const void *m_in, void *m_out,
                          const void *adiag, const void *bw, double eta, uint32_t *flag,
                          const uint32_t *t_base, uint32_t t_off, hipStream_t s) {
    switch (rpt) {
        case 1: launch_iter_k<T, ALPHA, 1>(L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s); break;
        case 2: launch_iter_k<T, ALPHA, 2>(L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s); break;
        case 4: launch_iter_k<T, ALPHA, 4>(L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s); break;
        default: launch_iter_k<T, ALPHA, 8>(L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s); break;
    }
}

hipError_t launch_iter(int dtype, int rpt, const Lattice &L, const void *m_in, void *m_out,
                       const void *adiag, const void *bw, double eta, uint32_t *flag,
                       const uint32_t *t_base, uint32_t t_off, hipStream_t s) {
    if (dtype == 0) {
        if (L.alpha == 1) launch_iter_a<float, 1>(rpt, L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s);
        else launch_iter_a<float, 2>(rpt, L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s);
    } else {
        if (L.alpha == 1) launch_iter_a<double, 1>(rpt, L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s);
        else launch_iter_a<double, 2>(rpt, L, m_in, m_out, adiag, bw, eta, flag, t_base, t_off, s);
    }
    return hipGetLastError();
}

template <typename T, int ALPHA, int RPT>
static void launch_theta_k(const Lattice &L, const void *m_in, void *m_out, const void *gain,
                           const void *bw, double eta, uint32_t *flag, const uint32_t *t_base,
                           uint32_t t_off, hipStream_t s) {
    const int tiles = L.tiles_x * ((L.ny + 4 * RPT - 1) / (4 * RPT));
    hipLaunchKernelGGL((k_iter_theta<T, ALPHA, RPT>), dim3(tiles), dim3(256), 0, s, L,
                       (const T *)m_in, (T *)m_out, (const T *)gain, (const T *)bw, (T)eta, flag,
                       t_base, t_off);
}

template <typename T, int ALPHA>
static void launch_theta_a(int rpt, const Lattice &L, const void *m_in, void *m_out,
                           const void *gain, const void *bw, double eta, uint32_t *flag,
                           const uint32_t *t_base, uint32_t t_off, hipStream_t s) {
    switch (rpt) {
        case 1: launch_theta_k<T, ALPHA, 1>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s); break;
        case 2: launch_theta_k<T, ALPHA, 2>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s); break;
        case 4: launch_theta_k<T, ALPHA, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s); break;
        default: launch_theta_k<T, ALPHA, 8>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s); break;
    }
}

hipError_t launch_iter_theta(int dtype, int rpt, const Lattice &L, const void *m_in,
                             void *m_out, const void *gain, const void *bw, double eta,
                             uint32_t *flag, const uint32_t *t_base, uint32_t t_off, hipStream_t s) {
    if (dtype == 0) {
        if (L.alpha == 1) launch_theta_a<float, 1>(rpt, L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        else launch_theta_a<float, 2>(rpt, L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
    } else {
        if (L.alpha == 1) launch_theta_a<double, 1>(rpt, L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        else launch_theta_a<double, 2>(rpt, L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
    }
    return hipGetLastError();
}

// tile height -> waves per workgroup: 4 rows on 4 waves, 8 and 16 rows on 8,
// 12 rows on 12, 32 rows on 16
template <typename T, int ALPHA, int TH>
static void launch_theta2_k(const Lattice &L, const void *m_in, void *m_out, const void *gain,
                            const void *bw, double eta, uint32_t *flag, const uint32_t *t_base,
                            uint32_t t_off, hipStream_t s) {
    constexpr int WAVES = TH == 4 ? 4 : TH == 12 ? 12 : TH == 32 ? 16 : 8;
    constexpr int R = ALPHA == 1 ? 1 : 2;
    const TileRange in = interior_tiles(L.nx, L.ny, R, TH);
    // the ring's workgroups first, their count rounded up to a multiple of
    // the 8 XCDs so that the interior tiles keep xcd_remap's mapping
    const int nring = (int)((in.ring_count() + 7) / 8 * 8);
    const int ninner = in.hole_count() > 0 ? L.tiles_x * in.rows : 0;
    hipLaunchKernelGGL((k_iter_theta2<T, ALPHA, TH, WAVES>),
                       dim3((unsigned)(nring + ninner)), dim3(64 * WAVES), 0, s, L,
                       in, nring, (const T *)m_in, (T *)m_out, (const T *)gain, (const T *)bw,
                       (T)eta, flag, t_base, t_off);
}

hipError_t launch_iter_theta2(int dtype, int th, const Lattice &L, const void *m_in, void *m_out,
                              const void *gain, const void *bw, double eta, uint32_t *flag,
                              const uint32_t *t_base, uint32_t t_off, hipStream_t s) {
    if (dtype == 0) {
        if (L.alpha == 1) {
            if (th == 32) launch_theta2_k<float, 1, 32>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 16) launch_theta2_k<float, 1, 16>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 12) launch_theta2_k<float, 1, 12>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 8) launch_theta2_k<float, 1, 8>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else launch_theta2_k<float, 1, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        } else {
            if (th == 32) launch_theta2_k<float, 2, 32>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 16) launch_theta2_k<float, 2, 16>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 12) launch_theta2_k<float, 2, 12>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (th == 8) launch_theta2_k<float, 2, 8>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else launch_theta2_k<float, 2, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        }
    } else {
        if (L.alpha == 1) launch_theta2_k<double, 1, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        else launch_theta2_k<double, 2, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
    }
    return hipGetLastError();
}

// Segments per strip: enough workgroups to fill every compute unit at the
// kernel's occupancy (a persistent grid), each segment at least 4 bands.
template <typename T, int ALPHA, int RB>
static void launch_walk_k(const Lattice &L, const void *m_in, void *m_out, const void *gain,
                          const void *bw, double eta, uint32_t *flag, const uint32_t *t_base,
                          uint32_t t_off, hipStream_t s) {
    static int resident = 0;   // workgroups resident on the device at once
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, (const void *)k_iter_theta2w<T, ALPHA, RB>, 64 * RB, 0) == hipSuccess &&
            cus > 0 && per_cu > 0)
            resident = cus * per_cu;
        else
            resident = 512;
    }
    const int max_seg = std::max(1, L.ny / (4 * RB));
    const int nseg = std::min(max_seg, std::max(1, (resident + L.tiles_x / 2) / L.tiles_x));
    const int seglen = (L.ny + nseg - 1) / nseg;
    const int blocks = L.tiles_x * ((L.ny + seglen - 1) / seglen);
    hipLaunchKernelGGL((k_iter_theta2w<T, ALPHA, RB>), dim3(blocks), dim3(64 * RB), 0, s, L,
                       (const T *)m_in, (T *)m_out, (const T *)gain, (const T *)bw, (T)eta, flag,
                       t_base, t_off, seglen);
}

hipError_t launch_iter_theta2w(int dtype, int rb, const Lattice &L, const void *m_in,
                               void *m_out, const void *gain, const void *bw, double eta,
                               uint32_t *flag, const uint32_t *t_base, uint32_t t_off,
                               hipStream_t s) {
    if (dtype == 0) {
        if (L.alpha == 1) {
            if (rb == 8) launch_walk_k<float, 1, 8>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (rb == 4) launch_walk_k<float, 1, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else launch_walk_k<float, 1, 2>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        } else {
            if (rb == 8) launch_walk_k<float, 2, 8>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else if (rb == 4) launch_walk_k<float, 2, 4>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
            else launch_walk_k<float, 2, 2>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        }
    } else {
        if (L.alpha == 1) launch_walk_k<double, 1, 2>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
        else launch_walk_k<double, 2, 2>(L, m_in, m_out, gain, bw, eta, flag, t_base, t_off, s);
    }
    return hipGetLastError();
}

hipError_t launch_gain(int dtype, const Lattice &L, const void *m, const void *adiag, void *gain,
                       hipStream_t s) {
    dim3 grid(tiles_of(L)), block(256);
    if (dtype == 0) {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_gain<float, 1>), grid, block, 0, s, L, (const float *)m,
                               (const float *)adiag, (float *)gain);
        else
            hipLaunchKernelGGL((k_gain<float, 2>), grid, block, 0, s, L, (const float *)m,
                               (const float *)adiag, (float *)gain);
    } else {
        if (L.alpha == 1)
            hipLaunchKernelGGL((k_gain<double, 1>), grid, block, 0, s, L, (const double *)m,
                               (const double *)adiag, (double *)gain);
        else
            hipLaunchKernelGGL((k_gain<double, 2>), grid, block, 0, s, L, (const double *)m,
                               (const double *)adiag, (double *)gain);
    }
    return hipGetLastError();
}

}  // namespace gabp
