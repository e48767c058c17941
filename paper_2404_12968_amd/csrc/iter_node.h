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
// New messages are written with non-temporal stores: nothing reads them in
// the same launch, and keeping them out of L2 leaves it to the neighbours'
// shared reads (measured: 2-4 % faster iterations, 11 % on 32-row pair tiles).
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

    // plane bases are wave-uniform; per-lane offsets stay 32-bit.  The loads
    // go out at a raised wave priority (dropped before the arithmetic), so
    // that a wave starting its node gets its loads in flight ahead of the
    // other waves' arithmetic and stores: full kernel 1.31 -> 1.26 ms on the
    // 8192 x 4096 lattice
    T lin[DEG], tin[DEG], ol[DEG], ot[DEG];
    __builtin_amdgcn_s_setprio(2);
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
    __builtin_amdgcn_s_setprio(0);
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
            __builtin_nontemporal_store(dl, &(m_out + (size_t)d * L.plane)[i]);
            __builtin_nontemporal_store(dt, &(m_out + (size_t)(DEG + d) * L.plane)[i]);
        }
    }
}

// --------------------------------------------------------------------------
// Information-only update (precision messages frozen, gains g stored).  For
// node i with incoming information messages tin[d] (from i + off_d, zero
// where that neighbour does not exist), its previous outgoing messages ot[d],
// the gains g[d] of its outgoing edges and its data term b:
//   th_i = b + c sum_d tin[d],   out[d] = (1 - eta) ot[d] + eta g[d] (th_i - tin[d]).
// Every information-only kernel goes through this function so that all of
// them, and the full iteration, round identically.
// --------------------------------------------------------------------------
template <typename T, int DEG>
__device__ __forceinline__ void theta_update(const T *tin, const T *ot, const T *g, T b, T c,
                                             T eta, T keep, T *out) {
    T st = 0;
#pragma unroll
    for (int d = 0; d < DEG; ++d) st += tin[d];
    const T bt = fmadd(c, st, b);
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        const T tc = bt - tin[d];
        out[d] = fmadd(eta, g[d] * tc, keep * ot[d]);
    }
}

// Loads of one node for theta_update (all issued before the first use).
template <typename T, int ALPHA, bool INTERIOR>
__device__ __forceinline__ void theta_gather(const Lattice &L, const T *__restrict__ m_in,
                                             const T *__restrict__ gain,
                                             const T *__restrict__ bw, int x, int y, T *tin,
                                             T *ot, T *g, T &b, bool *ok) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, xs, ys, ok);
#pragma unroll
    for (int d = 0; d < DEG; ++d) tin[d] = (m_in + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        ot[d] = (m_in + (size_t)(DEG + d) * L.plane)[i];
        g[d] = (gain + (size_t)d * L.plane)[i];
    }
    b = bw[i];
    if (!INTERIOR) {
#pragma unroll
        for (int d = 0; d < DEG; ++d) tin[d] = ok[d] ? tin[d] : (T)0;
    }
}

// As theta_gather, but the previous outgoing message and the gain are loaded
// only for the directions in need[] (zero elsewhere: those outputs are
// computed but must not be used).
template <typename T, int ALPHA, bool INTERIOR>
__device__ __forceinline__ void theta_gather_some(const Lattice &L, const T *__restrict__ m_in,
                                                  const T *__restrict__ gain,
                                                  const T *__restrict__ bw, int x, int y,
                                                  const bool *need, T *tin, T *ot, T *g, T &b,
                                                  bool *ok) {
    constexpr int DEG = ALPHA == 1 ? 4 : 12;
    const uint32_t i = (uint32_t)(y * L.pitch + x);
    uint32_t j[DEG];
    int xs[DEG], ys[DEG];
    node_nbrs<DEG, INTERIOR>(L, x, y, j, xs, ys, ok);
#pragma unroll
    for (int d = 0; d < DEG; ++d) tin[d] = (m_in + (size_t)(DEG + (d ^ 1)) * L.plane)[j[d]];
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        ot[d] = (T)0;
        g[d] = (T)0;
        if (need[d]) {
            ot[d] = (m_in + (size_t)(DEG + d) * L.plane)[i];
            g[d] = (gain + (size_t)d * L.plane)[i];
        }
    }
    b = bw[i];
    if (!INTERIOR) {
#pragma unroll
        for (int d = 0; d < DEG; ++d) tin[d] = ok[d] ? tin[d] : (T)0;
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
    T tin[DEG], ot[DEG], g[DEG], out[DEG], b;
    bool ok[DEG];
    __builtin_amdgcn_s_setprio(2);
    theta_gather<T, ALPHA, INTERIOR>(L, m_in, gain, bw, x, y, tin, ot, g, b, ok);
    __builtin_amdgcn_s_setprio(0);
    theta_update<T, DEG>(tin, ot, g, b, (T)L.c, eta, (T)1 - eta, out);
#pragma unroll
    for (int d = 0; d < DEG; ++d) {
        if (ok[d]) {
            bad |= !isfinite(out[d]);
            __builtin_nontemporal_store(out[d], &(m_out + (size_t)(DEG + d) * L.plane)[i]);
        }
    }
}

}  // namespace gabp
