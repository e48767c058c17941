// Two information-only iterations per launch by a column-strip walker: a
// persistent workgroup owns one 64-column strip of the lattice and one
// segment of its rows, and marches down the segment in bands of RB rows.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "iter_node.h"
#include "lattice.h"
#include "numerics.h"
#include "pair_tile.h"

#pragma clang fp contract(off)

namespace gabp {

// --------------------------------------------------------------------------
// Once the precision messages froze, the information recursion is a fixed
// linear stencil of radius R (2 for the 13-point prior, 1 for the 5-point
// one), so iteration t+2 of a node follows from iteration t+1 of the nodes
// within R, which follows from iteration t within 2R.
//
// Workgroup = RB waves, strip columns [x0, x0 + 64) (lane = column), rows
// [Y0, Y1).  Band j holds rows Y0 + j RB + w (wave w).  Iteration j of the
// march:
//   stage 1: iteration t+1 of band j's rows, for the strip's columns and for
//            the R columns on either side (those halo nodes compute only the
//            messages they send into the strip), read from HBM and written,
//            sender-indexed, into an LDS ring of rows;
//   barrier;
//   stage 2: iteration t+2 of band j-1's rows from the ring (their stencil
//            reaches R rows into band j, which is now complete) and written
//            to HBM.
// The same thread computes both stages of a node, so the node's gains, data
// term and own t+1 messages stay in registers for one band.  A prologue
// computes stage 1 for the R rows above the segment; the bands run on until
// stage 1 covered the R rows below it.  Every value is read from HBM once per
// launch except the R-row overlap of neighbouring segments and the 2R-column
// overlap of neighbouring strips (shared in L2), and no vertical halo row is
// recomputed.  Every node goes through theta_update, so the result is bitwise
// that of two single-iteration launches.
//
// LDS ring: S = 3 RB + 2 rows (so that one barrier per band orders the ring's
// reads and writes: the rows a band's stage 1 overwrites were last read two
// stages earlier), each DEG planes x (64 + 2R) columns; slot of unwrapped row
// r: (r - Y0 + R) mod S.  Positions past the end of a periodic axis hold the
// wrapped node (never written back); positions outside a non-periodic axis
// are skipped and never read.
// --------------------------------------------------------------------------
template <int RB>
struct WalkRing {
    static constexpr int kRows = 3 * RB + 2;
};

template <typename T, int ALPHA, int RB>
__device__ __forceinline__ void walk_strip(const Lattice &L, const T *__restrict__ m_in,
                                           T *__restrict__ m_out, const T *__restrict__ gain,
                                           const T *__restrict__ bw, T eta, int x0, int Y0,
                                           int Y1, T *lds, bool &bad1, bool &bad2) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    constexpr int R = ALPHA == 1 ? 1 : 2;
    constexpr int LW = 64 + 2 * R;              // ring row width (columns x0-R .. x0+63+R)
    constexpr int S = WalkRing<RB>::kRows;
    static_assert(RB >= R, "the prologue needs R waves");
    const int lane = (int)(threadIdx.x & 63u), w = (int)(threadIdx.x >> 6);
    const bool px = L.bcx == BC_PERIODIC, py = L.bcy == BC_PERIODIC;
    const T c = (T)L.c, keep = (T)1 - eta;
    const bool xin = x0 >= 2 * R && x0 + 64 + 2 * R <= L.nx;
    const int x = x0 + lane;

    // ring element (unwrapped row r, direction d, local column lx in [-R, 64+R))
    auto ring = [&](int r, int d, int lx) -> T & {
        const int slot = (r - Y0 + R) % S;
        return lds[(slot * DEG + d) * LW + lx + R];
    };

    // stage 1 of one node at local column lx, unwrapped row r; need == nullptr:
    // every direction (tile columns), else only the directions whose receiver
    // is a strip column.  Returns false where the node does not exist.
    auto stage1 = [&](int lx, int r, bool interior, const bool *need, T *g, T &b, T *out) {
        int gx = x0 + lx, gy = r;
        T tin[DEG], ot[DEG];
        bool ok[DEG];
        if (interior) {
            if (need) theta_gather_some<T, ALPHA, true>(L, m_in, gain, bw, gx, gy, need, tin, ot, g, b, ok);
            else theta_gather<T, ALPHA, true>(L, m_in, gain, bw, gx, gy, tin, ot, g, b, ok);
        } else {
            if (gx < 0 || gx >= L.nx) { if (px) gx = wrap_coord(gx, L.nx); else return false; }
            if (gy < 0 || gy >= L.ny) { if (py) gy = wrap_coord(gy, L.ny); else return false; }
            if (need) theta_gather_some<T, ALPHA, false>(L, m_in, gain, bw, gx, gy, need, tin, ot, g, b, ok);
            else theta_gather<T, ALPHA, false>(L, m_in, gain, bw, gx, gy, tin, ot, g, b, ok);
        }
        theta_update<T, DEG>(tin, ot, g, b, c, eta, keep, out);
#pragma unroll
        for (int d = 0; d < DEG; ++d)
            if (ok[d] && (!need || need[d])) bad1 |= !isfinite(out[d]);
        return true;
    };

    // the 2R halo nodes of row r (lanes 0 .. 2R-1 of the calling wave)
    auto halo_row = [&](int r, bool interior) {
        if (lane >= 2 * R) return;
        const int lx = lane < R ? lane - R : 64 + lane - R;
        bool need[DEG];
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
            const int rx = lx + dir_dx(d);
            need[d] = rx >= 0 && rx < 64;
        }
        T g[DEG], b, out[DEG];
        if (stage1(lx, r, interior, need, g, b, out)) {
#pragma unroll
            for (int d = 0; d < DEG; ++d)
                if (need[d]) ring(r, d, lx) = out[d];
        }
    };

    // rows of a band lie inside the lattice with a 2R margin: no wrapping,
    // no missing neighbour, for stage 1 and for stage 2
    auto band_interior = [&](int rs) { return xin && rs >= 2 * R && rs + RB + 2 * R <= L.ny; };

    // prologue: stage 1 of the R rows above the segment
    if (w < R) {
        const int r = Y0 - R + w;
        const bool in = xin && r >= 2 * R && r + 2 * R <= L.ny;
        T g[DEG], b, out[DEG];
        if (stage1(lane, r, in, nullptr, g, b, out)) {
#pragma unroll
            for (int d = 0; d < DEG; ++d) ring(r, d, lane) = out[d];
        }
        halo_row(r, in);
    }

    const int nb1 = (Y1 - Y0 + R + RB - 1) / RB;   // bands of stage 1
    const int nb2 = (Y1 - Y0 + RB - 1) / RB;       // bands of stage 2
    const int nbands = nb1 > nb2 + 1 ? nb1 : nb2 + 1;
    T gp[DEG], thp[DEG], bp = (T)0;                // this thread's node of the previous band
    bool hp = false;
#pragma unroll
    for (int d = 0; d < DEG; ++d) gp[d] = thp[d] = (T)0;

#pragma unroll 1
    for (int j = 0; j < nbands; ++j) {
        const int rs = Y0 + j * RB;
        const int r1 = rs + w;
        T gc[DEG], thc[DEG], bc = (T)0;
        bool hc = false;
        if (j < nb1) {
            const bool in = band_interior(rs);
            hc = stage1(lane, r1, in, nullptr, gc, bc, thc);
            if (hc) {
#pragma unroll
                for (int d = 0; d < DEG; ++d) ring(r1, d, lane) = thc[d];
            }
            halo_row(r1, in);
        }
        __syncthreads();
        if (j >= 1) {
            const int r2 = r1 - RB;
            if (hp && r2 < Y1 && x < L.nx && r2 < L.ny) {
                const bool in = band_interior(rs - RB);
                const uint32_t i = (uint32_t)(r2 * L.pitch + x);
                T tin[DEG], out[DEG];
                bool ok[DEG];
#pragma unroll
                for (int d = 0; d < DEG; ++d) {
                    int xn, yn;
                    ok[d] = in || neighbour(L, x, r2, d, xn, yn);
                    tin[d] = ok[d] ? ring(r2 + dir_dy(d), d ^ 1, lane + dir_dx(d)) : (T)0;
                }
                theta_update<T, DEG>(tin, thp, gp, bp, c, eta, keep, out);
#pragma unroll
                for (int d = 0; d < DEG; ++d) {
                    if (ok[d]) {
                        bad2 |= !isfinite(out[d]);
                        __builtin_nontemporal_store(out[d], &(m_out + (size_t)(DEG + d) * L.plane)[i]);
                    }
                }
            }
        }
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
            gp[d] = gc[d];
            thp[d] = thc[d];
        }
        bp = bc;
        hp = hc;
    }
}

}  // namespace gabp
