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
// the 13- or 5-point FP64 stencil of the prior plus the diagonal.  Split into
// the loads (resid_load) and the arithmetic (resid_accum) so that a caller
// can issue the loads of several nodes before the first use; resid_node is
// the two in sequence.
template <int ALPHA>
struct ResidIn {
    static constexpr int DEG = ALPHA == 1 ? 4 : 12;
    double v[DEG], a, m0, b;
    int xs[DEG], ys[DEG];
    bool ok[DEG];
};

template <int ALPHA, bool INTERIOR>
__device__ __forceinline__ void resid_load(const Lattice &L, const double *__restrict__ mu,
                                           const double *__restrict__ adiag64,
                                           const double *__restrict__ b64, int x, int y,
                                           ResidIn<ALPHA> &in) {
    constexpr int DEG = ResidIn<ALPHA>::DEG;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, in.xs, in.ys, in.ok);
#pragma unroll
    for (int d = 0; d < DEG; ++d) in.v[d] = mu[j[d]];
    in.a = adiag64[i];
    in.m0 = mu[i];
    in.b = b64[i];
}

template <int ALPHA>
__device__ __forceinline__ void resid_accum(const Lattice &L, int x, int y,
                                            const ResidIn<ALPHA> &in, double &rr, double &bb) {
    constexpr int DEG = ResidIn<ALPHA>::DEG;
    double s = in.a * in.m0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const double q = q_off<double>(L, d, x, y, in.xs[d], in.ys[d]);
        s += in.ok[d] ? q * in.v[d] : 0.0;
    }
    const double r = s - in.b;
    rr += r * r;
    bb += in.b * in.b;
}

template <int ALPHA, bool INTERIOR>
__device__ __forceinline__ void resid_node(const Lattice &L, const double *__restrict__ mu,
                                           const double *__restrict__ adiag64,
                                           const double *__restrict__ b64, int x, int y,
                                           double &rr, double &bb) {
    ResidIn<ALPHA> in;
    resid_load<ALPHA, INTERIOR>(L, mu, adiag64, b64, x, y, in);
    resid_accum<ALPHA>(L, x, y, in, rr, bb);
}

}  // namespace gabp
