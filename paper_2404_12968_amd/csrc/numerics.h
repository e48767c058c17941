// Device numerics and per-node neighbour helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

// No implicit multiply-add contraction in code that includes this header:
// kernels that must round identically spell their fused multiply-adds out.
#pragma clang fp contract(off)

namespace gabp {

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T>
__device__ __forceinline__ T recip(T v);
template <>
__device__ __forceinline__ float recip<float>(float v) {
    return __builtin_amdgcn_rcpf(v);  // 1 ulp; FP32 messages are checked at 1e-5
}
template <>
__device__ __forceinline__ double recip<double>(double v) {
    return 1.0 / v;  // correctly rounded: FP64 parity is checked at 1e-12
}

// --------------------------------------------------------------------------
// Neighbour table of one node: shifted offsets j[d] of (x, y) + off_d and
// whether that neighbour exists.  INTERIOR nodes (radius-2 halo inside the
// grid) need no tests; others wrap periodic axes and clamp addresses so
// that every load stays in bounds (the value is then masked).
// --------------------------------------------------------------------------
template <int DEG, bool INTERIOR>
__device__ __forceinline__ void node_nbrs(const Lattice &L, int x, int y, uint32_t *j, int *xs,
                                          int *ys, bool *ok) {
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        int xn, yn;
        if (INTERIOR) {
            xn = x + dir_dx(d);
            yn = y + dir_dy(d);
            ok[d] = true;
        } else {
            ok[d] = neighbour(L, x, y, d, xn, yn);
            xn = min(max(xn, 0), L.nx - 1);
            yn = min(max(yn, 0), L.ny - 1);
        }
        xs[d] = xn;
        ys[d] = yn;
        j[d] = (uint32_t)(yn * L.pitch + xn);
    }
}

// Off-diagonal prior precision divided by c for direction d of node (x, y)
// with l_i = ell(x, y) precomputed (closed forms in lattice.h).
template <typename T, int ALPHA>
__device__ __forceinline__ T q_over_c(const Lattice &L, int d, T li, int xn, int yn) {
    T q;
    if (ALPHA == 1) {
        q = -(T)L.tau * (d < 2 ? (T)L.ihx2 : (T)L.ihy2);
    } else if (d < 4) {
        q = -(T)L.tau * (li + ell<T>(L, xn, yn)) * (d < 2 ? (T)L.ihx2 : (T)L.ihy2);
    } else if (d < 8) {
        q = d < 6 ? (T)(L.tau * L.ihx2 * L.ihx2) : (T)(L.tau * L.ihy2 * L.ihy2);
    } else {
        q = (T)(2.0 * L.tau * L.ihx2 * L.ihy2);
    }
    return q * (T)L.inv_c;
}

// Gain of edge i -> j: g = -(Q_ij/c) / Lam_c.  The new message is
// (g (Q_ij/c), g th_c).  Shared by the full and the information-only
// iterations so that both round identically.
template <typename T>
__device__ __forceinline__ T edge_gain(T q, T lc) {
    return -(q * recip<T>(lc));
}

}  // namespace gabp
