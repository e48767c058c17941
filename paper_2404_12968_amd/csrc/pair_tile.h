// One 64 x TH tile of two information-only iterations (temporal blocking),
// shared by the single-lattice and the batched two-iteration kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "iter_node.h"
#include "lattice.h"
#include "numerics.h"

#pragma clang fp contract(off)

namespace gabp {

// --------------------------------------------------------------------------
// Two information-only iterations per pass (temporal blocking).  A
// workgroup owns a 64 x TH tile (the caller passes LDS for deg x TH x 64
// values and synchronises before reusing it).  Step 1 computes iteration
// t+1 for the tile and for a halo of R = stencil radius nodes around it
// (inputs from HBM/L2; the halo runs as band jobs, each node computing only
// the messages it sends into the tile), and leaves in LDS, for every tile
// node and direction d, its incoming message from the node at + off_d
// (receiver-indexed, 64 x TH x deg values; the tile nodes' own new messages
// stay in registers with their gains).  Step 2
// computes iteration t+2 for the tile from LDS and writes it out.  HBM then
// sees one read of the inputs and one write of the outputs per two
// iterations.  Every node goes through theta_update, so the result is bitwise
// what two single-iteration launches give.  Local position (lx, ly) in
// [-R, 64 + R) x [-R, TH + R) is global (x0 + lx, y0 + ly), wrapped on
// periodic axes; positions outside a non-periodic axis are skipped (their
// edges do not exist), and tile positions past the end of a periodic axis
// repeat wrapped nodes without being written back.
// --------------------------------------------------------------------------
__device__ __forceinline__ void record_divergence(uint32_t *p, uint32_t v) {
    uint32_t old = atomicCAS(p, 0u, v);
    while (old != 0u && old > v) {   // keep the earliest iteration
        const uint32_t prev = atomicCAS(p, old, v);
        if (prev == old) break;
        old = prev;
    }
}

__device__ __forceinline__ int wrap_coord(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// --------------------------------------------------------------------------
// Halo jobs.  A band of halo nodes sends into the tile along a fixed set of
// directions (bit d of a mask), so its gather loads the previous outgoing
// messages and gains of those directions only and its update computes only
// those messages (same arithmetic, in the same order, as theta_update):
//   5-point:  row -1 {2}, row TH {3}, column -1 {0}, column 64 {1};
//   13-point: row -2 {6}, row -1 {2, 6, 8, 11}, row TH {3, 7, 9, 10},
//             row TH+1 {7}, columns -1 and -2 with the corners (-1, -1),
//             (-1, TH) {0, 4, 8, 10}, columns 64 and 65 with the corners
//             (64, -1), (64, TH) {1, 5, 9, 11}.
// A lane whose receiver in one of its directions lies outside the tile
// computes that message but does not store it.
// --------------------------------------------------------------------------
template <int ALPHA>
struct HaloMasks;
template <>
struct HaloMasks<1> {
    static constexpr int kRows = 2;
    static constexpr unsigned row(int j) { return j == 0 ? 1u << 2 : 1u << 3; }
    static constexpr unsigned kLeft = 1u << 0, kRight = 1u << 1;
};
template <>
struct HaloMasks<2> {
    static constexpr int kRows = 4;
    static constexpr unsigned row(int j) {
        return j == 0 ? 1u << 6
             : j == 1 ? (1u << 2) | (1u << 6) | (1u << 8) | (1u << 11)
             : j == 2 ? (1u << 3) | (1u << 7) | (1u << 9) | (1u << 10)
                      : 1u << 7;
    }
    static constexpr unsigned kLeft = (1u << 0) | (1u << 4) | (1u << 8) | (1u << 10);
    static constexpr unsigned kRight = (1u << 1) | (1u << 5) | (1u << 9) | (1u << 11);
};

// Halo node (lx, ly) of the tile at (x0, y0): its messages of MASK at t+1,
// stored into the receivers' LDS slots.
template <typename T, int ALPHA, int TH, unsigned MASK, bool IO>
__device__ __forceinline__ void halo_node(const Lattice &L, const T *__restrict__ m_in,
                                          const T *__restrict__ gain, const T *__restrict__ bw,
                                          T c, T eta, T keep, int x0, int y0, int lx, int ly,
                                          bool interior, T *lds, bool &bad1) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    int gx = x0 + lx, gy = y0 + ly;
    if (!IO && !interior) {
        if (gx < 0 || gx >= L.nx) {
            if (L.bcx != BC_PERIODIC) return;
            gx = wrap_coord(gx, L.nx);
        }
        if (gy < 0 || gy >= L.ny) {
            if (L.bcy != BC_PERIODIC) return;
            gy = wrap_coord(gy, L.ny);
        }
    }
    const uint32_t i = (uint32_t)(gy * L.pitch + gx);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    T tin[DEG], ot[DEG], g[DEG];
    if (IO || interior)
        node_nbrs<DEG, true>(L, gx, gy, j, xs, ys, ok);
    else
        node_nbrs<DEG, false>(L, gx, gy, j, xs, ys, ok);
#pragma unroll
    for (int d = 0; d < DEG; ++d) tin[d] = (m_in + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        if (!(MASK & (1u << d))) continue;
        ot[d] = (m_in + (size_t)(DEG + d) * L.plane)[i];
        g[d] = (gain + (size_t)d * L.plane)[i];
    }
    const T b = bw[i];
    if (!IO && !interior) {
#pragma unroll
        for (int d = 0; d < DEG; ++d) tin[d] = ok[d] ? tin[d] : (T)0;
    }
    T st = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) st += tin[d];
    const T bt = fmadd(c, st, b);
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        if (!(MASK & (1u << d))) continue;
        const int rx = lx + dir_dx(d), ry = ly + dir_dy(d);
        if (rx < 0 || rx >= 64 || ry < 0 || ry >= TH) continue;
        const T out = fmadd(eta, g[d] * (bt - tin[d]), keep * ot[d]);
        lds[((d ^ 1) * TH + ry) * 64 + rx] = out;
        if (ok[d]) bad1 |= !isfinite(out);
    }
}

// IO: the caller guarantees an interior tile; the boundary code paths are
// compiled out.
template <typename T, int ALPHA, int TH, int WAVES, bool IO = false>
__device__ __forceinline__ void pair_tile(const Lattice &L, const T *__restrict__ m_in,
                                          T *__restrict__ m_out, const T *__restrict__ gain,
                                          const T *__restrict__ bw, T eta, int tx, int ty,
                                          T *lds, bool &bad1, bool &bad2) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    constexpr int R = ALPHA == 1 ? 1 : 2;
    constexpr int RPT = TH / WAVES;
    static_assert(TH % WAVES == 0, "tile rows must be a multiple of the wave count");
    // lds[(d * TH + y) * 64 + x]: incoming message of tile node (x, y) from
    // direction d at t+1 (receiver-indexed)
    const int x0 = tx * 64, y0 = ty * TH;
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const bool px = L.bcx == BC_PERIODIC, py = L.bcy == BC_PERIODIC;
    const bool interior = IO || (x0 >= 2 * R && x0 + 64 + 2 * R <= L.nx && y0 >= 2 * R &&
                                 y0 + TH + 2 * R <= L.ny);
    const T c = (T)L.c, keep = (T)1 - eta;
    T th1[RPT][DEG], gk[RPT][DEG], bk[RPT];

    // store message (lx, ly) -> (lx, ly) + off_e if its receiver is in the tile
    auto deliver = [&](int lx, int ly, int e, T v) {
        const int rx = lx + dir_dx(e), ry = ly + dir_dy(e);
        if (rx >= 0 && rx < 64 && ry >= 0 && ry < TH) lds[((e ^ 1) * TH + ry) * 64 + rx] = v;
    };

    // The tile rows' loads go out at a raised wave priority, so that a
    // workgroup starting its step 1 gets its loads in flight ahead of the
    // step-2 work (LDS reads, updates, stores) of the other workgroups on the
    // CU; the priority drops again before the halo jobs.  Measured on the
    // 8192 x 4096 pass: 16-row tiles 1.122 -> 1.004 ms, 12-row 1.058 ->
    // 1.030 ms (raising it for the halo as well, or in step 2, is slower).
    __builtin_amdgcn_s_setprio(2);
    // step 1: tile positions (one column per lane, rows w, w + WAVES, ...)
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = w + WAVES * k;
        int gx = x0 + lane, gy = y0 + ly;
        T tin[DEG], ot[DEG];
        bool ok[DEG];
        bool here = true;
        if (interior) {
            theta_gather<T, ALPHA, true>(L, m_in, gain, bw, gx, gy, tin, ot, gk[k], bk[k], ok);
        } else {
            if (gx >= L.nx) { if (px) gx = wrap_coord(gx, L.nx); else here = false; }
            if (gy >= L.ny) { if (py) gy = wrap_coord(gy, L.ny); else here = false; }
            if (here)
                theta_gather<T, ALPHA, false>(L, m_in, gain, bw, gx, gy, tin, ot, gk[k], bk[k],
                                              ok);
        }
        if (here) {
            theta_update<T, DEG>(tin, ot, gk[k], bk[k], c, eta, keep, th1[k]);
#pragma unroll
            for (int d = 0; d < DEG; ++d) {
                deliver(lane, ly, d, th1[k][d]);
                if (ok[d]) bad1 |= !isfinite(th1[k][d]);
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    // step 1: halo jobs (row bands, then left and right column chunks of
    // 64 positions), one wave each
    {
        using HM = HaloMasks<ALPHA>;
        constexpr int NL = R * TH + (R == 2 ? 2 : 0);   // positions of one side
        constexpr int NC = (NL + 63) / 64;
        constexpr int NJOBS = HM::kRows + 2 * NC;
#pragma unroll 1
        for (int jb = w; jb < NJOBS; jb += WAVES) {
            if (jb < HM::kRows) {
                const int ly = jb < HM::kRows / 2 ? jb - HM::kRows / 2 : TH + jb - HM::kRows / 2;
                switch (jb) {
                    case 0: halo_node<T, ALPHA, TH, HM::row(0), IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lane, ly, interior, lds, bad1); break;
                    case 1: halo_node<T, ALPHA, TH, HM::row(1), IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lane, ly, interior, lds, bad1); break;
                    case 2: halo_node<T, ALPHA, TH, HM::row(2), IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lane, ly, interior, lds, bad1); break;
                    default: halo_node<T, ALPHA, TH, HM::row(3), IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lane, ly, interior, lds, bad1); break;
                }
            } else {
                const int cj = jb - HM::kRows;
                const bool right = cj >= NC;
                const int p = (right ? cj - NC : cj) * 64 + lane;
                if (p < NL) {
                    // p < TH: column -1 (64); p < 2 TH: column -2 (65); then
                    // the corners of row -1 and row TH
                    int lx, ly;
                    if (p < TH) {
                        lx = -1;
                        ly = p;
                    } else if (p < R * TH) {
                        lx = -2;
                        ly = p - TH;
                    } else {
                        lx = -1;
                        ly = p == R * TH ? -1 : TH;
                    }
                    if (right) lx = 63 - lx;
                    if (right)
                        halo_node<T, ALPHA, TH, HM::kRight, IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lx, ly, interior, lds, bad1);
                    else
                        halo_node<T, ALPHA, TH, HM::kLeft, IO>(L, m_in, gain, bw, c, eta, keep, x0, y0, lx, ly, interior, lds, bad1);
                }
            }
        }
    }
    __syncthreads();
    // step 2: the tile's own nodes, from LDS
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = w + WAVES * k;
        const int x = x0 + lane, y = y0 + ly;
        if (x >= L.nx || y >= L.ny) continue;
        const uint32_t i = (uint32_t)(y * L.pitch + x);
        T tin[DEG], out[DEG];
        bool ok[DEG];
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
            int xn, yn;
            ok[d] = interior || neighbour(L, x, y, d, xn, yn);
            tin[d] = ok[d] ? lds[(d * TH + ly) * 64 + lane] : (T)0;
        }
        theta_update<T, DEG>(tin, th1[k], gk[k], bk[k], c, eta, keep, out);
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
            if (ok[d]) {
                bad2 |= !isfinite(out[d]);
                __builtin_nontemporal_store(out[d], &(m_out + (size_t)(DEG + d) * L.plane)[i]);
            }
        }
    }
}

}  // namespace gabp
