// Iteration kernels of the space-time solver (include/gabp_st.h): the GMRF of
// the stochastic heat equation discretised by Crank-Nicolson steps (paper:
// Appendix "Extension to Spatiotemporal Systems"), solved by the damped,
// re-weighted flooding iteration on its 38-neighbour graph.
//
// Precision closed form.  With G the graph Laplacian of the grid (unit
// spacing; G_ii = g_i, the number of in-grid axis neighbours of i, G_ij = -1
// for grid neighbours), Lap_h = -G/h^2 and every block of M is a polynomial
// in G: A = a1 I + a2 G, B = a1 I - a2 G, L = l1 I + l2 G with a1 = 1/dt,
// a2 = nu/(2 h^2), l1 = a0 kappa^2, l2 = a0/h^2.  The blocks of
// Q = S M^T M (S = dt h^2 / sigma_u^2) are then polynomials p I + q G + r G^2:
//     slice 0:        S (L^2 + B^2)      (S L^2 when there is one slice)
//     slices 1..N-2:  S (A^2 + B^2)
//     slice N-1:      S A^2
//     between n, n+1: -S A B = -S (a1^2 I - a2^2 G^2)
// and the entries of p I + q G + r G^2 follow from those of G and G^2 (the
// grid graph is bipartite, so grid neighbours share no neighbour):
//     (i, i):               p + q g_i + r (g_i^2 + g_i)
//     one step:             -q - r (g_i + g_j)
//     two steps on an axis: r
//     diagonal:             2 r
// The host folds the three products of each block into one (p, q, r) in
// FP64; kernels evaluate the entries from it, the position and the slice.
//
// Storage.  Sender-indexed SoA planes as in the lattice kernels: plane d at
// node i holds the message from i to i + off_d (d = 0..37, opposite d ^ 1),
// precisions in planes 0..37 and information in planes 38..75.  A node's
// plane index is n * slice + y * pitch + x with slice = pitch * ny.
//
// Launch shape.  A workgroup of 64 x 4 threads per slice owns one 64 x 4 tile
// of one slice (or of SL consecutive slices); the workgroup order (wg_tile)
// keeps the tiles that share halo rows and slices on one XCD at nearly the
// same time.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "lattice.h"
#include "numerics.h"

#pragma clang fp contract(off)

namespace gabp {
namespace st {


constexpr int kDeg = 38;

// Direction tables: d < 12 lie in the slice (the lattice directions of
// lattice.h); d = 12 + 2k is (o_k, +1), d = 13 + 2k is (-o_k, -1), with
// o_0 = (0, 0) and o_k the lattice direction k - 1.
__host__ __device__ constexpr int cross_k(int d) { return (d - 12) >> 1; }
__host__ __device__ constexpr int sdx(int d) {
    return d < 12 ? dir_dx(d)
                  : cross_k(d) == 0 ? 0 : ((d & 1) ? -dir_dx(cross_k(d) - 1) : dir_dx(cross_k(d) - 1));
}
__host__ __device__ constexpr int sdy(int d) {
    return d < 12 ? dir_dy(d)
                  : cross_k(d) == 0 ? 0 : ((d & 1) ? -dir_dy(cross_k(d) - 1) : dir_dy(cross_k(d) - 1));
}
__host__ __device__ constexpr int sdt(int d) { return d < 12 ? 0 : ((d & 1) ? -1 : 1); }
// spatial relation of direction d: 0 same position, 1 one step, 2 two steps
// along an axis, 3 diagonal
__host__ __device__ constexpr int scls(int d) {
    return d < 12 ? (d < 4 ? 1 : d < 8 ? 2 : 3)
                  : cross_k(d) == 0 ? 0 : (cross_k(d) - 1 < 4 ? 1 : cross_k(d) - 1 < 8 ? 2 : 3);
}

struct Grid {
    int32_t nx, ny, nt, pitch;
    int32_t bcx, bcy, tiles_x, tiles_y;
    int64_t slice;              // elements between slices (pitch * ny)
    int64_t plane;              // elements between planes
    double blk[4][3];           // (p, q, r) of blocks: slice 0, middle, last, coupling
    double lsq[3];              // (p, q, r) of S L^2, the initial condition's precision
    double c, inv_c;
};

__device__ __forceinline__ int axis_g(int v, int n, int bc) {
    return bc == BC_PERIODIC ? 2 : (int)(v > 0) + (int)(v < n - 1);
}

__device__ __forceinline__ int slice_kind(const Grid &G, int t) {
    return t == 0 ? 0 : (t == G.nt - 1 ? 2 : 1);
}

// Entry of p I + q G + r G^2 for a relation class (g_j only for one step).
template <typename T>
__device__ __forceinline__ T coef(const double *pqr, int cls, T gi, T gj) {
    const T p = (T)pqr[0], q = (T)pqr[1], r = (T)pqr[2];
    if (cls == 0) return p + q * gi + r * (gi * gi + gi);
    if (cls == 1) return -q - r * (gi + gj);
    if (cls == 2) return r;
    return r + r;
}

// Neighbour of (x, y, t) in direction d: wraps periodic axes; false when it
// lies outside the grid.
__device__ __forceinline__ bool nbr(const Grid &G, int x, int y, int t, int d, int &xn, int &yn,
                                    int &tn) {
    xn = x + sdx(d);
    yn = y + sdy(d);
    tn = t + sdt(d);
    if ((unsigned)tn >= (unsigned)G.nt) return false;
    if (G.bcx == BC_PERIODIC) {
        xn = xn < 0 ? xn + G.nx : (xn >= G.nx ? xn - G.nx : xn);
    } else if ((unsigned)xn >= (unsigned)G.nx) {
        return false;
    }
    if (G.bcy == BC_PERIODIC) {
        yn = yn < 0 ? yn + G.ny : (yn >= G.ny ? yn - G.ny : yn);
    } else if ((unsigned)yn >= (unsigned)G.ny) {
        return false;
    }
    return true;
}

// Q_ij / c for direction d of node (x, y, t) whose neighbour (xn, yn) exists.
template <typename T>
__device__ __forceinline__ T q_over_c(const Grid &G, int d, int kind, T gi, int xn, int yn) {
    const double *pqr = d < 12 ? G.blk[kind] : G.blk[3];
    const int cls = scls(d);
    T gj = (T)0;
    if (cls == 1) gj = (T)(axis_g(xn, G.nx, G.bcx) + axis_g(yn, G.ny, G.bcy));
    return coef<T>(pqr, cls, gi, gj) * (T)G.inv_c;
}

// --------------------------------------------------------------------------
// One flooding iteration of node (x, y, t) (as the lattice kernels):
//   Lam_i = A_ii + c sum_k Lam_{k->i},  th_i = b_i + c sum_k th_{k->i}
//   for each neighbour j: Lam_c = Lam_i - Lam_{j->i}, th_c = th_i - th_{j->i},
//   g = -(Q_ij/c)/Lam_c, new (g Q_ij/c, g th_c), damped with the previous
//   outgoing message (Appendix "Re-weighted message updates"; Section
//   "Update Damping").
// INTERIOR: every neighbour exists (radius-2 spatial halo inside the grid, a
// slice on either side) and needs no test.  Otherwise the code stays
// branch-free: a missing neighbour's address is clamped to the node itself,
// its message is read as zero, and its outgoing slot is written as zero.
// --------------------------------------------------------------------------
// v in [-2, n + 1] wrapped onto [0, n) without branches
__device__ __forceinline__ int wrap(int v, int n) {
    return v + n * ((int)(v < 0) - (int)(v >= n));
}

// Boundary handling is compile-time: PX / PY say whether an axis is periodic.
template <bool PX, bool PY>
__device__ __forceinline__ bool nbr_at(const Grid &G, int d, int x, int y, int t, int &xn,
                                       int &yn, int &tn) {
    xn = x + sdx(d);
    yn = y + sdy(d);
    tn = t + sdt(d);
    if (PX && sdx(d) != 0) xn = wrap(xn, G.nx);
    if (PY && sdy(d) != 0) yn = wrap(yn, G.ny);
    bool ok = (unsigned)tn < (unsigned)G.nt;
    if (!PX) ok = ok && (unsigned)xn < (unsigned)G.nx;
    if (!PY) ok = ok && (unsigned)yn < (unsigned)G.ny;
    return ok;
}

template <bool PX, bool PY>
__device__ __forceinline__ int g_at(const Grid &G, int x, int y) {
    return (PX ? 2 : (int)(x > 0) + (int)(x < G.nx - 1)) + (PY ? 2 : (int)(y > 0) + (int)(y < G.ny - 1));
}

// Plane index of neighbour d of (x, y, t) and whether it exists (a missing
// neighbour's index is the node's own, so every load stays in bounds).
template <bool INTERIOR, bool PX, bool PY>
__device__ __forceinline__ uint32_t nbr_index(const Grid &G, int d, int x, int y, int t,
                                              bool &ok) {
    int xn, yn, tn;
    if (INTERIOR) {
        xn = x + sdx(d);
        yn = y + sdy(d);
        tn = t + sdt(d);
        ok = true;
    } else {
        ok = nbr_at<PX, PY>(G, d, x, y, t, xn, yn, tn);
        xn = ok ? xn : x;
        yn = ok ? yn : y;
        tn = ok ? tn : t;
    }
    return (uint32_t)tn * (uint32_t)G.slice + (uint32_t)(yn * G.pitch + xn);
}

// Incoming messages of one component (0: precisions, 1: information), zero
// where the sender does not exist; bit d of okm says whether it does.
template <typename T, bool INTERIOR, bool PX, bool PY>
__device__ __forceinline__ void gather_in(const Grid &G, const T *__restrict__ m, int comp, int x,
                                          int y, int t, T *v, uint64_t &okm) {
    okm = 0;
#pragma unroll
    for (int d = 0; d < kDeg; ++d) {
        bool ok;
        const uint32_t j = nbr_index<INTERIOR, PX, PY>(G, d, x, y, t, ok);
        const T val = (m + (size_t)(comp * kDeg + (d ^ 1)) * G.plane)[j];
        v[d] = ok ? val : (T)0;
        okm |= (uint64_t)ok << d;
    }
}

// Both components at once (the full iteration): same values as two
// gather_in calls.
template <typename T, bool INTERIOR, bool PX, bool PY>
__device__ __forceinline__ void gather_both(const Grid &G, const T *__restrict__ m, int x, int y,
                                            int t, T *lv, T *tv, uint64_t &okm) {
    okm = 0;
#pragma unroll
    for (int d = 0; d < kDeg; ++d) {
        bool ok;
        const uint32_t j = nbr_index<INTERIOR, PX, PY>(G, d, x, y, t, ok);
        const T l = (m + (size_t)(d ^ 1) * G.plane)[j];
        const T th = (m + (size_t)(kDeg + (d ^ 1)) * G.plane)[j];
        lv[d] = ok ? l : (T)0;
        tv[d] = ok ? th : (T)0;
        okm |= (uint64_t)ok << d;
    }
}

// Belief parameter: a + c * sum_d v[d], summed in direction order.
template <typename T>
__device__ __forceinline__ T belief(T a, const T *v, T c) {
    T s = 0;
#pragma unroll
    for (int d = 0; d < kDeg; ++d) s += v[d];
    return fmadd(c, s, a);
}

// Q_ij / c for direction d (closed forms at the top of this file); gi is
// the node's neighbour count, pq_same / pq_cross the slice's blocks.
template <typename T, bool INTERIOR, bool PX, bool PY>
__device__ __forceinline__ T q_dir(const Grid &G, int d, int x, int y, int t, T gi,
                                   const T *pq_same, const T *pq_cross) {
    T gj = (T)4;
    if (!INTERIOR && scls(d) == 1) {
        int xn, yn, tn;
        (void)nbr_at<PX, PY>(G, d, x, y, t, xn, yn, tn);
        gj = (T)g_at<PX, PY>(G, xn, yn);
    }
    const T *pqr = d < 12 ? pq_same : pq_cross;
    T q;
    if (scls(d) == 0) q = pqr[0] + pqr[1] * gi + pqr[2] * (gi * gi + gi);
    else if (scls(d) == 1) q = -pqr[1] - pqr[2] * (gi + gj);
    else if (scls(d) == 2) q = pqr[2];
    else q = pqr[2] + pqr[2];
    return q * (T)G.inv_c;
}

// --------------------------------------------------------------------------
// Frozen precision messages.  The precision recursion involves neither the
// information messages nor the data, so once one iteration leaves every
// precision message unchanged, all later ones do too.  The edge gains
// g = -(Q_ij/c)/Lam_c are then stored once (MODE_GAIN) and the iteration
// updates only the information messages (MODE_THETA):
//   th_i = b_i + c sum_d th_{k->i},  out_d = (1 - eta) out_d + eta g_d (th_i - th_{j->i}).
// All three modes share gather_in, belief and q_dir, so the information-only
// iteration is bitwise the full one's.  New messages are written with
// non-temporal stores (nothing reads them in the same launch; 4-5 % faster)
// and the gains, read once per iteration, are loaded non-temporally (4 %
// more on the information-only kernel; on the lattice's two-iteration tiles
// the same hint costs 4 %, so it is used here only).
// --------------------------------------------------------------------------
enum { MODE_FULL = 0, MODE_GAIN = 1, MODE_THETA = 2 };

template <typename T, int MODE, bool INTERIOR, bool PX, bool PY>
__device__ __forceinline__ void st_node(const Grid &G, const T *__restrict__ m_in,
                                        T *__restrict__ m_out, T *__restrict__ gain,
                                        const T *__restrict__ aw, const T *__restrict__ bw,
                                        T eta, const T *pq_same, const T *pq_cross, bool &bad,
                                        int x, int y, int t) {
    const uint32_t i = (uint32_t)t * (uint32_t)G.slice + (uint32_t)(y * G.pitch + x);
    const T c = (T)G.c, keep = (T)1 - eta;
    const T gi = INTERIOR ? (T)4 : (T)g_at<PX, PY>(G, x, y);
    uint64_t okm;
    if constexpr (MODE == MODE_FULL) {
        T lin[kDeg], tin[kDeg];
        // the gather at a raised wave priority (as the lattice kernels):
        // full iteration 2.78 -> 2.63 ms at 512 x 512 x 64; the
        // information-only iteration does not gain from it
        __builtin_amdgcn_s_setprio(2);
        gather_both<T, INTERIOR, PX, PY>(G, m_in, x, y, t, lin, tin, okm);
        __builtin_amdgcn_s_setprio(0);
        const T bl = belief(aw[i], lin, c);
        const T bt = belief(bw[i], tin, c);
#pragma unroll
        for (int d = 0; d < kDeg; ++d) {
            const T q = q_dir<T, INTERIOR, PX, PY>(G, d, x, y, t, gi, pq_same, pq_cross);
            const T lc = bl - lin[d];
            const T tc = bt - tin[d];
            const T g = edge_gain(q, lc);
            const T ol = (m_in + (size_t)d * G.plane)[i];
            const T ot = (m_in + (size_t)(kDeg + d) * G.plane)[i];
            T dl = fmadd(eta, g * q, keep * ol);
            T dt = fmadd(eta, g * tc, keep * ot);
            const bool ok = INTERIOR || ((okm >> d) & 1u);
            bad |= ok && (!(lc > (T)0) || !isfinite(dl) || !isfinite(dt));
            dl = ok ? dl : (T)0;
            dt = ok ? dt : (T)0;
            __builtin_nontemporal_store(dl, &(m_out + (size_t)d * G.plane)[i]);
            __builtin_nontemporal_store(dt, &(m_out + (size_t)(kDeg + d) * G.plane)[i]);
        }
    } else if constexpr (MODE == MODE_GAIN) {
        T lin[kDeg];
        gather_in<T, INTERIOR, PX, PY>(G, m_in, 0, x, y, t, lin, okm);
        const T bl = belief(aw[i], lin, c);
#pragma unroll
        for (int d = 0; d < kDeg; ++d) {
            const T q = q_dir<T, INTERIOR, PX, PY>(G, d, x, y, t, gi, pq_same, pq_cross);
            const T g = edge_gain(q, bl - lin[d]);
            const bool ok = INTERIOR || ((okm >> d) & 1u);
            (gain + (size_t)d * G.plane)[i] = ok ? g : (T)0;
        }
    } else {
        T tin[kDeg];
        gather_in<T, INTERIOR, PX, PY>(G, m_in, 1, x, y, t, tin, okm);
        const T bt = belief(bw[i], tin, c);
#pragma unroll
        for (int d = 0; d < kDeg; ++d) {
            const T g = __builtin_nontemporal_load(&(gain + (size_t)d * G.plane)[i]);
            const T ot = (m_in + (size_t)(kDeg + d) * G.plane)[i];
            T dt = fmadd(eta, g * (bt - tin[d]), keep * ot);
            const bool ok = INTERIOR || ((okm >> d) & 1u);
            bad |= ok && !isfinite(dt);
            dt = ok ? dt : (T)0;
            __builtin_nontemporal_store(dt, &(m_out + (size_t)(kDeg + d) * G.plane)[i]);
        }
    }
}

// Workgroup -> (tile x, tile y, first slice).  A workgroup covers one 64 x 4
// tile on SL consecutive slices (4 waves per slice): the messages that pass
// between those slices are read twice inside one workgroup.  Tiles are
// grouped in bands of kGroupRows tile rows; within a band the order is slice
// group by slice group, each row by row.  With the XCD remap each XCD runs a
// contiguous range of this order, so a tile's vertical neighbours (same
// slices) are at most a few tile rows away and its slice neighbours one
// band-slice (tiles_x * kGroupRows workgroups) away: both halos are read
// while still in L2.
// Band height, measured on 512 x 512 x 64 (information-only iteration, ms):
// 2 rows 1.540, 4 rows 1.473, 8 rows 1.443, 16 rows 1.424, 32 rows 1.486,
// 128 rows (one band) 1.700.
constexpr int kGroupRows = 16;

// Band and slice-group order over a box of tiles_x x tiles_y tiles and nt
// slices: workgroup b -> (tx, ty, first slice) relative to the box.
template <int SL>
__device__ __forceinline__ void wg_tile(int b, int tiles_x, int tiles_y, int nt, int &tx, int &ty,
                                        int &t0) {
    const int groups = (nt + SL - 1) / SL;
    const int full = kGroupRows * tiles_x * groups;         // workgroups of a full band
    const int g = b / full;
    const int r = b - g * full;
    const int hg = min(kGroupRows, tiles_y - g * kGroupRows);   // tile rows of this band
    const int per_slice = hg * tiles_x;
    const int sg = r / per_slice;
    const int r2 = r - sg * per_slice;
    const int tyi = r2 / tiles_x;
    tx = r2 - tyi * tiles_x;
    ty = g * kGroupRows + tyi;
    t0 = sg * SL;
}

// Interior tiles of a slice grid (a halo of 2 inside the slice: every
// in-slice and cross-slice neighbour exists and none wraps); with the first
// and last slice excluded they are the tiles the interior kernel runs.
__host__ __device__ inline TileRange st_hole(const Grid &G) {
    return interior_tiles(G.nx, G.ny, 1, 4);
}

// Boundary tiles: every tile of the first and last slice, then the ring of
// each slice between (all tiles when the hole is empty or nt < 3).
__host__ __device__ inline int64_t st_boundary_count(const Grid &G) {
    const TileRange h = st_hole(G);
    const int64_t all = (int64_t)G.tiles_x * G.tiles_y;
    if (h.empty() || G.nt < 3) return all * G.nt;
    return 2 * all + (int64_t)(G.nt - 2) * h.ring_count();
}

__device__ __forceinline__ void st_boundary_tile(const Grid &G, int b, int &tx, int &ty, int &t) {
    const TileRange h = st_hole(G);
    const int all = G.tiles_x * G.tiles_y;
    int tile;
    if (h.empty() || G.nt < 3) {
        t = b / all;
        tile = b - t * all;
    } else if (b < 2 * all) {
        t = b < all ? 0 : G.nt - 1;
        tile = b < all ? b : b - all;
    } else {
        const int ring = (int)h.ring_count();
        const int q = (b - 2 * all) / ring;
        t = 1 + q;
        h.ring(b - 2 * all - q * ring, tx, ty);
        return;
    }
    ty = tile / G.tiles_x;
    tx = tile - ty * G.tiles_x;
}

// One launch of a mode over the grid or part of it: PART_ALL every tile
// (interior tiles through the interior path, in one kernel), PART_INTERIOR
// the interior tiles of slices 1 .. nt - 2 (compiled without the boundary
// paths: fewer registers, more waves per SIMD), PART_BOUNDARY the other tiles
// (one slice per workgroup); an iteration is then the two launches.  The
// full iteration runs split (3.07 -> 2.78 ms per iteration at 512 x 512 x 64:
// 96 instead of 121 VGPRs); the information-only one, already streaming
// near the copy rate, runs whole (split, its boundary sweep costs more than
// the occupancy gains: 1.47 -> 1.53 ms).  diverged_at[0] records the first
// iteration whose launches met an invalid value; launches of later
// iterations return at once (the launches of the iteration that met it
// complete, so its output buffer holds that iteration).  MODE_GAIN passes
// it = 0.
enum { PART_ALL = 0, PART_INTERIOR = 1, PART_BOUNDARY = 2 };

template <typename T, int MODE, bool PX, bool PY, int SL, int PART>
__global__ __launch_bounds__(256 * SL) void k_iter(Grid G, const T *__restrict__ m_in,
                                                   T *__restrict__ m_out, T *__restrict__ gain,
                                                   const T *__restrict__ aw,
                                                   const T *__restrict__ bw, T eta,
                                                   uint32_t *__restrict__ diverged_at,
                                                   uint32_t it) {
    const uint32_t seen = *diverged_at;
    if (MODE != MODE_GAIN && seen != 0u && seen < it) return;
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    int tx, ty, t;
    if (PART == PART_ALL) {
        int t0;
        wg_tile<SL>(b, G.tiles_x, G.tiles_y, G.nt, tx, ty, t0);
        t = t0 + (int)(threadIdx.x >> 8);          // one slice per four waves
        if (t >= G.nt) return;
    } else if (PART == PART_INTERIOR) {
        const TileRange h = st_hole(G);
        int t0;
        wg_tile<SL>(b, h.txb - h.txa + 1, h.tyb - h.tya + 1, G.nt - 2, tx, ty, t0);
        tx += h.txa;
        ty += h.tya;
        t = 1 + t0 + (int)(threadIdx.x >> 8);      // one slice per four waves
        if (t > G.nt - 2) return;
    } else {
        st_boundary_tile(G, b, tx, ty, t);
    }
    const int x = tx * 64 + (int)(threadIdx.x & 63u);
    const int y = ty * 4 + (int)((threadIdx.x >> 6) & 3u);
    // the slice's blocks (uniform over the wave) in message precision
    const int kind = slice_kind(G, t);
    const T pq_same[3] = {(T)G.blk[kind][0], (T)G.blk[kind][1], (T)G.blk[kind][2]};
    const T pq_cross[3] = {(T)G.blk[3][0], (T)G.blk[3][1], (T)G.blk[3][2]};
    const bool inner = PART == PART_INTERIOR ||
                       (PART == PART_ALL && tx * 64 >= 2 && tx * 64 + 66 <= G.nx && ty * 4 >= 2 &&
                        ty * 4 + 6 <= G.ny && t > 0 && t < G.nt - 1);
    bool bad = false;
    if (inner)
        st_node<T, MODE, true, PX, PY>(G, m_in, m_out, gain, aw, bw, eta, pq_same, pq_cross, bad,
                                       x, y, t);
    else if (x < G.nx && y < G.ny)
        st_node<T, MODE, false, PX, PY>(G, m_in, m_out, gain, aw, bw, eta, pq_same, pq_cross,
                                        bad, x, y, t);
    if (MODE != MODE_GAIN && bad) atomicCAS(diverged_at, 0u, it);
}

// Precision messages changed between two buffers: count of bitwise
// differences (64-bit) and the largest relative change |a - b| / max(|a|,
// |b|) as float bits (non-negative floats order like their bit patterns).
template <typename T>
__global__ __launch_bounds__(256) void k_prec_change(const T *__restrict__ a,
                                                     const T *__restrict__ b, int64_t n,
                                                     unsigned long long *__restrict__ count,
                                                     uint32_t *__restrict__ maxrel_bits) {
    uint32_t cnt = 0;
    float mx = 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * 256) {
        const T u = a[k], v = b[k];
        using U = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
        U ub, vb;
        __builtin_memcpy(&ub, &u, sizeof(T));
        __builtin_memcpy(&vb, &v, sizeof(T));
        if (ub != vb) {
            ++cnt;
            const double den = fmax(fabs((double)u), fabs((double)v));
            const float r = den > 0.0 ? (float)(fabs((double)u - (double)v) / den) : INFINITY;
            mx = fmaxf(mx, isnan(r) ? INFINITY : r);
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if ((threadIdx.x & 63u) == 0u && cnt != 0u) {
        atomicAdd(count, (unsigned long long)cnt);
        atomicMax(maxrel_bits, __float_as_uint(mx));
    }
}

}  // namespace st
}  // namespace gabp
