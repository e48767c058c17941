// Host-side helpers shared by the single-lattice and batched C ABI
// implementations: workspace layout and argument validation.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>

#include "gabp.h"
#include "lattice.h"

namespace gabp {
namespace host {

constexpr int kNumPartials = 2048;       // workgroups of the residual reduction
constexpr size_t kAlign = 256;           // byte alignment of rows and planes

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Device workspace layout.  Every plane has the same row pitch (elements);
// message planes are separated by `plane` elements, which adds one 256-byte
// skew so that the 2*deg concurrent streams do not start on the same HBM
// channel.
struct Layout {
    int32_t pitch = 0;
    int64_t plane = 0;        // message-plane stride, elements
    size_t msg[2] = {0, 0};
    size_t gain = 0;
    size_t adiag64 = 0, b64 = 0, mu64 = 0, bel64 = 0, adiag_w = 0, b_w = 0;
    size_t partials = 0, red = 0, flags = 0, total = 0;
};

// Freeze decision from one precision-change probe: `changed` messages
// differed bitwise between the last two iterations, the largest relative
// change being the float with bits `maxrel_bits`.  With max_slots = 0 only a
// bitwise stationary iteration freezes (the information-only iteration is
// then bitwise the full one); otherwise at most max_slots changes of at most
// max_rel each are tolerated.
inline bool freeze_now(uint64_t changed, uint32_t maxrel_bits, int64_t max_slots,
                       double max_rel) {
    if (changed == 0u) return true;
    if (max_slots <= 0 || changed > (uint64_t)max_slots) return false;
    float rel;
    static_assert(sizeof rel == sizeof maxrel_bits, "float bits");
    std::memcpy(&rel, &maxrel_bits, sizeof rel);
    return std::isfinite(rel) && (double)rel <= max_rel;
}

// State kept after a divergence.  Kernels record the first invalid iteration
// t and every later launch returns without writing, so the messages kept are
// those written by the launch that produced t: its last iteration, in the
// buffer it wrote.  HeldState says which (iteration, buffer) that is.
struct HeldState {
    int64_t iter;
    int buf;
};

// Single-lattice runs: from iteration `start` in buffer `buf0`, `pairs`
// two-iteration launches then single ones, each launch writing the other
// buffer.  t in (start, start + 2 pairs + singles].
inline HeldState held_after_run(int64_t start, int buf0, int64_t pairs, int64_t t) {
    const int64_t rel = t - start;
    if (rel <= 2 * pairs) {
        const int64_t k = (rel + 1) / 2;      // 1-based index of the pair launch
        return {start + 2 * k, buf0 ^ (int)(k & 1)};
    }
    const int64_t k = pairs + (rel - 2 * pairs);
    return {t, buf0 ^ (int)(k & 1)};
}

// Batched runs: an instance at iteration t0 (its state in buffer t0 & 1)
// runs `couples` couples of two-iteration launches if it is frozen (the
// first reads buffer t0' & 1 and writes the other, the second writes back;
// t0' the couple's start), then single iterations, each writing buffer
// t & 1.  Instances not frozen run single iterations throughout.
inline HeldState held_after_batch_run(int64_t t0, bool frozen, int64_t couples, int64_t t) {
    const int64_t rel = t - t0;
    if (frozen && rel >= 1 && rel <= 4 * couples) {
        const int64_t cc = (rel - 1) / 4, q = (rel - 1) % 4;
        const int64_t start = t0 + 4 * cc;
        if (q < 2) return {start + 2, (int)((start & 1) ^ 1)};
        return {start + 4, (int)(start & 1)};
    }
    return {t, (int)(t & 1)};
}

inline Layout make_layout(int64_t nx, int64_t ny, int deg, size_t esize, bool f32) {
    Layout l;
    const size_t row_elems = kAlign / esize;
    l.pitch = (int32_t)round_up((size_t)nx, row_elems);
    const size_t node_elems = (size_t)l.pitch * (size_t)ny;
    l.plane = (int64_t)(round_up(node_elems, row_elems) + row_elems);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = round_up(off + bytes, kAlign);
        return o;
    };
    const size_t buf_bytes = (size_t)(2 * deg) * (size_t)l.plane * esize;
    l.msg[0] = take(buf_bytes);
    l.msg[1] = take(buf_bytes);
    l.gain = take((size_t)deg * (size_t)l.plane * esize);
    l.adiag64 = take(node_elems * 8);
    l.b64 = take(node_elems * 8);
    l.mu64 = take(node_elems * 8);
    l.bel64 = take(node_elems * 8);
    if (f32) {
        l.adiag_w = take(node_elems * esize);
        l.b_w = take(node_elems * esize);
    }
    l.partials = take((size_t)kNumPartials * 2 * sizeof(double));
    l.red = take(8 * sizeof(double));
    l.flags = take(8 * sizeof(uint32_t));
    l.total = off;
    return l;
}

inline gabp_status check_grid_stencil(const gabp_grid *g, const gabp_stencil *s, int32_t dtype,
                               std::string &why) {
    if (!g || !s) return why = "grid and stencil are required", GABP_E_INVALID;
    if (g->nx < 1 || g->ny < 1) return why = "nx and ny must be >= 1", GABP_E_INVALID;
    if (!(g->hx > 0) || !(g->hy > 0) || !std::isfinite(g->hx) || !std::isfinite(g->hy))
        return why = "hx and hy must be positive and finite", GABP_E_INVALID;
    for (int32_t bc : {g->bc_x, g->bc_y})
        if (bc < 0 || bc > 2) return why = "unknown boundary type", GABP_E_INVALID;
    if (s->alpha != 1 && s->alpha != 2) return why = "alpha must be 1 or 2", GABP_E_INVALID;
    const int64_t minp = s->alpha == 1 ? 3 : 5;
    if ((g->bc_x == GABP_BC_PERIODIC && g->nx < minp) ||
        (g->bc_y == GABP_BC_PERIODIC && g->ny < minp))
        return why = "a periodic axis needs >= 3 cells (alpha 1) or >= 5 (alpha 2)",
               GABP_E_INVALID;
    const bool dirichlet = g->bc_x == GABP_BC_DIRICHLET || g->bc_y == GABP_BC_DIRICHLET;
    if (!std::isfinite(s->kappa) || s->kappa < 0 || (s->kappa == 0 && !dirichlet))
        return why = "kappa must be > 0 (>= 0 with a Dirichlet axis)", GABP_E_INVALID;
    if (!(s->tau > 0) || !std::isfinite(s->tau)) return why = "tau must be > 0", GABP_E_INVALID;
    if (!std::isfinite(s->c) || s->c == 0) return why = "c must be finite and non-zero", GABP_E_INVALID;
    if (dtype != GABP_F32 && dtype != GABP_F64) return why = "unknown dtype", GABP_E_INVALID;
    const int64_t pitch = (int64_t)round_up((size_t)g->nx, 64);
    if (g->nx > (1 << 30) || g->ny > (1 << 30) || pitch * g->ny >= ((int64_t)1 << 31) - 4096)
        return why = "grid too large for 32-bit in-plane indices", GABP_E_INVALID;
    return GABP_OK;
}

inline Lattice make_lattice(const gabp_grid *g, const gabp_stencil *s, const Layout &lay) {
    Lattice L{};
    L.nx = (int32_t)g->nx;
    L.ny = (int32_t)g->ny;
    L.pitch = lay.pitch;
    L.bcx = g->bc_x;
    L.bcy = g->bc_y;
    L.alpha = s->alpha;
    L.deg = s->alpha == 1 ? 4 : 12;
    L.tiles_x = (int32_t)((g->nx + 63) / 64);
    L.plane = lay.plane;
    L.kappa2 = s->kappa * s->kappa;
    L.tau = s->tau;
    L.ihx2 = 1.0 / (g->hx * g->hx);
    L.ihy2 = 1.0 / (g->hy * g->hy);
    L.c = s->c;
    L.inv_c = 1.0 / s->c;
    return L;
}

}  // namespace host
}  // namespace gabp
