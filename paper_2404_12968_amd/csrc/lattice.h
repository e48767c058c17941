// Lattice geometry, stencil coefficients and launch helpers shared by the
// gfx950 kernels of the library.
//
// Prior precision Q = tau * L^alpha with L = kappa^2 I - Delta_h, the
// finite-difference operator of the paper's discretised SPDE (Section
// "Derivation of the Factor Graph"; Appendix "Details on the Finite Difference
// Discretisation").  No matrix is stored: every coefficient is evaluated
// in-kernel from the position.  Closed forms used here (derived from L = kappa^2
// I + G_x/hx^2 + G_y/hy^2 with G the 1-D second-difference matrices):
//   l_i        = kappa^2 + cx(i)/hx^2 + cy(i)/hy^2
//                cx = number of in-grid x-neighbours for a zero-flux axis,
//                     2 for periodic and Dirichlet axes (likewise cy)
//   alpha = 1: Q_ii = tau l_i, Q_{i,i+-x} = -tau/hx^2, Q_{i,i+-y} = -tau/hy^2
//   alpha = 2 (the grid graph is bipartite, so neighbours share no neighbour):
//              Q_ii        = tau (l_i^2 + nx(i)/hx^4 + ny(i)/hy^4)
//              Q_{i,i+-x}  = -tau (l_i + l_j)/hx^2        (likewise y)
//              Q_{i,i+-2x} = tau/hx^4                     (likewise y)
//              Q_{i,i+-x+-y} = 2 tau/(hx^2 hy^2)
//   with nx(i), ny(i) the numbers of in-grid neighbours along each axis.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gabp {

enum { BC_NEUMANN = 0, BC_PERIODIC = 1, BC_DIRICHLET = 2 };

// Stencil directions d with offsets off_d = (dir_dx(d), dir_dy(d)); the
// opposite direction is d ^ 1.  Directions 0..3 are the 5-point stencil,
// 4..11 complete the 13-point stencil.  The message planes are
// sender-indexed: plane d at (x, y) holds the message FROM (x, y) TO
// (x, y) + off_d.  (The C ABI's checkpoint layout is receiver-indexed: slot d
// of (x, y) is the message INTO (x, y) FROM (x, y) + off_d.)
__host__ __device__ constexpr int dir_dx(int d) {
    return d == 0 ? 1 : d == 1 ? -1 : d == 4 ? 2 : d == 5 ? -2 :
           d == 8 ? 1 : d == 9 ? -1 : d == 10 ? 1 : d == 11 ? -1 : 0;
}
__host__ __device__ constexpr int dir_dy(int d) {
    return d == 2 ? 1 : d == 3 ? -1 : d == 6 ? 2 : d == 7 ? -2 :
           d == 8 ? 1 : d == 9 ? -1 : d == 10 ? -1 : d == 11 ? 1 : 0;
}

// Everything a kernel needs to know about one lattice problem.  Passed by
// value as a kernel argument.
struct Lattice {
    int32_t nx, ny;        // grid
    int32_t pitch;         // row pitch of every plane, in elements
    int32_t bcx, bcy;      // boundary types
    int32_t alpha, deg;    // prior order, number of stencil directions
    int32_t tiles_x;       // 64-wide column tiles
    int64_t plane;         // stride between planes, in elements
    double kappa2, tau, ihx2, ihy2;   // kappa^2, tau, 1/hx^2, 1/hy^2
    double c, inv_c;       // re-weighting constant and its reciprocal
};

// Number of in-grid neighbours along one axis and the diagonal count of L.
__device__ __forceinline__ int axis_nb(int v, int n, int bc) {
    return bc == BC_PERIODIC ? 2 : (int)(v > 0) + (int)(v < n - 1);
}
__device__ __forceinline__ int axis_cdiag(int v, int n, int bc) {
    return bc == BC_NEUMANN ? (int)(v > 0) + (int)(v < n - 1) : 2;
}

template <typename T>
__device__ __forceinline__ T ell(const Lattice &L, int x, int y) {
    return (T)L.kappa2 + (T)axis_cdiag(x, L.nx, L.bcx) * (T)L.ihx2 +
           (T)axis_cdiag(y, L.ny, L.bcy) * (T)L.ihy2;
}

// Neighbour of (x, y) in direction d, with periodic wrapping; false when it
// falls outside a non-periodic axis.
__device__ __forceinline__ bool neighbour(const Lattice &L, int x, int y, int d, int &xn,
                                          int &yn) {
    xn = x + dir_dx(d);
    yn = y + dir_dy(d);
    if (L.bcx == BC_PERIODIC) {
        xn = xn < 0 ? xn + L.nx : (xn >= L.nx ? xn - L.nx : xn);
    } else if ((unsigned)xn >= (unsigned)L.nx) {
        return false;
    }
    if (L.bcy == BC_PERIODIC) {
        yn = yn < 0 ? yn + L.ny : (yn >= L.ny ? yn - L.ny : yn);
    } else if ((unsigned)yn >= (unsigned)L.ny) {
        return false;
    }
    return true;
}

// Diagonal prior precision Q_ii.
template <typename T>
__device__ __forceinline__ T q_diag(const Lattice &L, int x, int y) {
    T l = ell<T>(L, x, y);
    if (L.alpha == 1) return (T)L.tau * l;
    T ihx4 = (T)(L.ihx2 * L.ihx2), ihy4 = (T)(L.ihy2 * L.ihy2);
    return (T)L.tau * (l * l + (T)axis_nb(x, L.nx, L.bcx) * ihx4 +
                       (T)axis_nb(y, L.ny, L.bcy) * ihy4);
}

// Off-diagonal prior precision Q_ij between (x, y) and its neighbour
// (xn, yn) in direction d (d < deg, neighbour inside the grid).
template <typename T>
__device__ __forceinline__ T q_off(const Lattice &L, int d, int x, int y, int xn, int yn) {
    if (L.alpha == 1) return -(T)L.tau * (d < 2 ? (T)L.ihx2 : (T)L.ihy2);
    if (d < 4) {
        T h = d < 2 ? (T)L.ihx2 : (T)L.ihy2;
        return -(T)L.tau * (ell<T>(L, x, y) + ell<T>(L, xn, yn)) * h;
    }
    if (d < 8) return d < 6 ? (T)(L.tau * L.ihx2 * L.ihx2) : (T)(L.tau * L.ihy2 * L.ihy2);
    return (T)(2.0 * L.tau * L.ihx2 * L.ihy2);
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2.  Remap the dispatch index so that XCD k walks a contiguous
// band of logical tiles: vertically and horizontally adjacent tiles then
// share an L2.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int nx = 8;
    int q = nblocks / nx, r = nblocks % nx;
    int xcd = b % nx, local = b / nx;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Strip-major tile order: strips of kStrip tile columns (the last one
// narrower), each walked row by row.  Logical index t of a grid of
// tiles_x x rows tiles -> (tx, ty); with xcd_remap, each XCD then walks a
// contiguous run of whole rows of strips, so tiles above and below a tile
// run close together on the same L2.  On the 8192-wide lattice a strip is
// exactly one XCD's share.
constexpr int kStrip = 16;

__device__ __forceinline__ void strip_order(int t, int tiles_x, int rows, int &tx, int &ty) {
    const int strip = t / (kStrip * rows), r = t - strip * kStrip * rows;
    const int width = min(kStrip, tiles_x - strip * kStrip);
    ty = r / width;
    tx = strip * kStrip + r % width;
}

// --------------------------------------------------------------------------
// Interior tiles and the ring of a tiling by 64 x TH tiles.  A tile is
// interior when it and a halo of 2R lie inside the grid: no coordinate wraps
// or leaves it (R: the stencil radius for a two-iteration pass, whose halo
// nodes need their own neighbours; 2R = 2 covers a single iteration of a
// radius-2 stencil).  Interior tiles form the index range [txa, txb] x
// [tya, tyb] (empty when a > b).  They run on code paths compiled without
// the boundary handling, whose registers would otherwise cost occupancy.
// The other tiles, the ring, are enumerated band by band (top rows, bottom
// rows, then the left and right columns of the rows between).
// --------------------------------------------------------------------------
struct TileRange {
    int txa, txb, tya, tyb;   // interior (hole) range, inclusive
    int cols, rows;           // tile grid
    __host__ __device__ bool empty() const { return txa > txb || tya > tyb; }
    __host__ __device__ int64_t hole_count() const {
        return empty() ? 0 : (int64_t)(txb - txa + 1) * (tyb - tya + 1);
    }
    __host__ __device__ int64_t ring_count() const {
        return (int64_t)cols * rows - hole_count();
    }
    __host__ __device__ bool interior(int tx, int ty) const {
        return tx >= txa && tx <= txb && ty >= tya && ty <= tyb;
    }
    // b-th tile outside the hole, b in [0, ring_count())
    __host__ __device__ void ring(int b, int &tx, int &ty) const {
        if (empty()) {
            ty = b / cols;
            tx = b - ty * cols;
            return;
        }
        const int top = tya * cols, bottom = (rows - 1 - tyb) * cols;
        if (b < top) {
            ty = b / cols;
            tx = b - ty * cols;
            return;
        }
        b -= top;
        if (b < bottom) {
            ty = tyb + 1 + b / cols;
            tx = b - (ty - tyb - 1) * cols;
            return;
        }
        b -= bottom;
        const int side = txa + (cols - 1 - txb);
        ty = tya + b / side;
        const int c = b - (ty - tya) * side;
        tx = c < txa ? c : txb + 1 + (c - txa);
    }
};

// Interior range of the 64 x TH tile grid of an nx x ny lattice.
__host__ __device__ inline TileRange interior_tiles(int nx, int ny, int R, int TH) {
    TileRange r;
    r.cols = (nx + 63) / 64;
    r.rows = (ny + TH - 1) / TH;
    r.txa = (2 * R + 63) / 64;
    r.txb = nx - 64 - 2 * R >= 0 ? (nx - 64 - 2 * R) / 64 : -1;
    r.tya = (2 * R + TH - 1) / TH;
    r.tyb = ny - TH - 2 * R >= 0 ? (ny - TH - 2 * R) / TH : -1;
    return r;
}

// Wave64 sum in a fixed order (butterfly over lane masks 32..1).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

}  // namespace gabp
