// Per-node bodies of the convergence check (FP64 marginals and residual),
// shared by the single-lattice and the batched kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lattice.h"
#include "numerics.h"

namespace gabp {

// Marginal of node (x, y) (Compute Marginal) in FP64 from sender-indexed
// messages of precision T: incoming messages are plane d^1 at the neighbour.
// FROZEN reads the constant belief precision from bel64; otherwise bel_out
// (may be NULL) records it.
template <typename T, int ALPHA, bool FROZEN>
__device__ __forceinline__ void post_node(const Lattice &L, const T *__restrict__ m,
                                          const double *__restrict__ adiag64,
                                          const double *__restrict__ b64,
                                          const double *__restrict__ bel64,
                                          double *__restrict__ mu_plane,
                                          double *__restrict__ mean, double *__restrict__ var,
                                          double *__restrict__ bel_out, int x, int y) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    node_nbrs<DEG, false>(L, x, y, j, xs, ys, ok);
    T lin[DEG], tin[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        if (!FROZEN) lin[d] = (m + (size_t)(d ^ 1) * L.plane)[j[d]];
        tin[d] = (m + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
    }
    double bl;
    if (FROZEN) {
        bl = bel64[i];
    } else {
        double sl = 0.0;
#pragma unroll
        for (int d = 0; d < DEG; ++d) sl += ok[d] ? (double)lin[d] : 0.0;
        bl = adiag64[i] + L.c * sl;
        if (bel_out) bel_out[i] = bl;
    }
    double st = 0.0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) st += ok[d] ? (double)tin[d] : 0.0;
    const double bt = b64[i] + L.c * st;
    const double mu = bt / bl;
    if (mu_plane) mu_plane[i] = mu;
    const int64_t o = (int64_t)y * L.nx + x;
    if (mean) mean[o] = mu;
    if (var) var[o] = 1.0 / bl;
}

// Residual contribution of node (x, y): r = (A mu - b)_i with A = Q + diag(p),
// the 13- or 5-point FP64 stencil of the prior plus the diagonal.
template <int ALPHA, bool INTERIOR>
__device__ __forceinline__ void resid_node(const Lattice &L, const double *__restrict__ mu,
                                           const double *__restrict__ adiag64,
                                           const double *__restrict__ b64, int x, int y,
                                           double &rr, double &bb) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, xs, ys, ok);
    double v[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) v[d] = mu[j[d]];
    const double a = adiag64[i], m0 = mu[i], b = b64[i];
    double s = a * m0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const double q = q_off<double>(L, d, x, y, xs[d], ys[d]);
        s += ok[d] ? q * v[d] : 0.0;
    }
    const double r = s - b;
    rr += r * r;
    bb += b * b;
}

}  // namespace gabp
