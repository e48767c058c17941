// Per-node bodies of the flooding iteration, shared by the single-lattice
// and the batched kernels so that both compute bitwise-identical messages.
// Message planes are sender-indexed (plane d at i: message from i to
// i + off_d); see iter.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lattice.h"
#include "numerics.h"

namespace gabp {

// --------------------------------------------------------------------------
// One flooding iteration, thread per node.
//
// Node i = (x, y) with incoming messages m_{k->i} (plane d^1 at k = i + off_d):
//   belief  Lam_i = A_ii + c sum_k Lam_{k->i},   th_i = b_i + c sum_k th_{k->i}
// and for every neighbour j = i + off_d (outgoing i -> j, plane d at i):
//   cavity  Lam_c = Lam_i - Lam_{j->i},  th_c = th_i - th_{j->i}
//   gain    g = -(Q_ij/c) / Lam_c
//   new     Lam~ = g (Q_ij/c) = -(Q_ij/c)^2 / Lam_c,  th~ = g th_c
//   damped  m^t = (1 - eta) m^{t-1} + eta m~
// (Appendix "Re-weighted message updates" in information form; Section
// "Update Damping".)  A cavity precision <= 0 or a non-finite value records t
// in diverged_at; later launches then return at once, keeping that state.
// Every load of a node is issued before the first use (~50 in flight per
// lane).
// --------------------------------------------------------------------------
template <typename T, int ALPHA, bool INTERIOR>
__device__ __forceinline__ void iter_node(const Lattice &L, const T *__restrict__ m_in,
                                          T *__restrict__ m_out, const T *__restrict__ adiag,
                                          const T *__restrict__ bw, T eta, bool &bad, int x,
                                          int y) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    const T c = (T)L.c, keep = (T)1 - eta;
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, xs, ys, ok);

    // plane bases are wave-uniform; per-lane offsets stay 32-bit
    T lin[DEG], tin[DEG], ol[DEG], ot[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        lin[d] = (m_in + (size_t)(d ^ 1) * L.plane)[j[d]];
        tin[d] = (m_in + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
    }
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        ol[d] = (m_in + (size_t)d * L.plane)[i];
        ot[d] = (m_in + (size_t)(DEG + d) * L.plane)[i];
    }
    const T a = adiag[i];
    const T b = bw[i];
    if (!INTERIOR) {
#pragma unroll
        for (int d = 0; d < DEG; ++d) {
            lin[d] = ok[d] ? lin[d] : (T)0;
            tin[d] = ok[d] ? tin[d] : (T)0;
        }
    }
    T sl = 0, st = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        sl += lin[d];
        st += tin[d];
    }
    const T bl = fmadd(c, sl, a);
    const T bt = fmadd(c, st, b);
    const T li = ALPHA == 2 ? ell<T>(L, x, y) : (T)0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const T q = q_over_c<T, ALPHA>(L, d, li, xs[d], ys[d]);
        const T lc = bl - lin[d];
        const T tc = bt - tin[d];
        const T g = edge_gain(q, lc);
        const T dl = fmadd(eta, g * q, keep * ol[d]);
        const T dt = fmadd(eta, g * tc, keep * ot[d]);
        if (ok[d]) {
            bad |= !(lc > (T)0) || !isfinite(dl) || !isfinite(dt);
            (m_out + (size_t)d * L.plane)[i] = dl;
            (m_out + (size_t)(DEG + d) * L.plane)[i] = dt;
        }
    }
}

template <typename T, int ALPHA, bool INTERIOR>
__device__ __forceinline__ void iter_theta_node(const Lattice &L, const T *__restrict__ m_in,
                                                T *__restrict__ m_out,
                                                const T *__restrict__ gain,
                                                const T *__restrict__ bw, T eta, bool &bad,
                                                int x, int y) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    const T c = (T)L.c, keep = (T)1 - eta;
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    bool ok[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, xs, ys, ok);
    T tin[DEG], ot[DEG], g[DEG];
#pragma unroll
    for (int d = 0; d < DEG; ++d) tin[d] = (m_in + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        ot[d] = (m_in + (size_t)(DEG + d) * L.plane)[i];
        g[d] = (gain + (size_t)d * L.plane)[i];
    }
    const T b = bw[i];
    if (!INTERIOR) {
#pragma unroll
        for (int d = 0; d < DEG; ++d) tin[d] = ok[d] ? tin[d] : (T)0;
    }
    T st = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) st += tin[d];
    const T bt = fmadd(c, st, b);
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const T tc = bt - tin[d];
        const T dt = fmadd(eta, g[d] * tc, keep * ot[d]);
        if (ok[d]) {
            bad |= !isfinite(dt);
            (m_out + (size_t)(DEG + d) * L.plane)[i] = dt;
        }
    }
}

}  // namespace gabp
