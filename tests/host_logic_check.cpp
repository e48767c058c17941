// Host-side checks of the library's host logic, compiled and run by
// tests/test_host_logic.py: the precision-freeze decision
// (gabp::host::freeze_now), the device workspace layout
// (gabp::host::make_layout) and the tile ranges of the two-iteration pass
// (gabp::interior_tiles, TileRange::ring).  Exit status 0
// and "ok" when every case holds.
#include <cmath>
#include <cstdio>
#include <cstring>

#include <vector>

#include "host_common.h"
#include "lattice.h"

using gabp::host::freeze_now;
using gabp::host::held_after_batch_run;
using gabp::host::held_after_run;
using gabp::host::HeldState;
using gabp::host::Layout;
using gabp::host::make_layout;

static uint32_t bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, sizeof u);
    return u;
}

#define CHECK(cond)                                             \
    do {                                                        \
        if (!(cond)) {                                          \
            std::printf("failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                           \
        }                                                       \
    } while (0)

static bool held_is(HeldState h, int64_t iter, int buf) { return h.iter == iter && h.buf == buf; }

int main() {
    // state kept after a divergence at t.  Single lattice: from iteration 10
    // in buffer 0, three two-iteration launches (writing buffers 1, 0, 1 with
    // iterations 12, 14, 16), then single launches (17 -> buffer 0, ...).
    CHECK(held_is(held_after_run(10, 0, 3, 11), 12, 1));   // first half of launch 1
    CHECK(held_is(held_after_run(10, 0, 3, 12), 12, 1));
    CHECK(held_is(held_after_run(10, 0, 3, 13), 14, 0));
    CHECK(held_is(held_after_run(10, 0, 3, 16), 16, 1));
    CHECK(held_is(held_after_run(10, 0, 3, 17), 17, 0));   // first single
    CHECK(held_is(held_after_run(10, 0, 3, 18), 18, 1));
    CHECK(held_is(held_after_run(10, 1, 0, 11), 11, 0));   // singles only
    CHECK(held_is(held_after_run(10, 1, 0, 14), 14, 1));
    // Batch: a frozen instance at iteration 10 runs two couples (launches
    // write buffers 1, 0 with iterations 12, 14, then 1, 0 with 16, 18), then
    // singles writing buffer t & 1
    CHECK(held_is(held_after_batch_run(10, true, 2, 11), 12, 1));
    CHECK(held_is(held_after_batch_run(10, true, 2, 12), 12, 1));
    CHECK(held_is(held_after_batch_run(10, true, 2, 13), 14, 0));
    CHECK(held_is(held_after_batch_run(10, true, 2, 14), 14, 0));
    CHECK(held_is(held_after_batch_run(10, true, 2, 15), 16, 1));
    CHECK(held_is(held_after_batch_run(10, true, 2, 18), 18, 0));
    CHECK(held_is(held_after_batch_run(10, true, 2, 19), 19, 1));
    CHECK(held_is(held_after_batch_run(11, true, 1, 12), 13, 0));   // odd start
    CHECK(held_is(held_after_batch_run(11, true, 1, 14), 15, 1));
    // an instance that is not frozen runs single iterations throughout
    CHECK(held_is(held_after_batch_run(10, false, 2, 11), 11, 1));
    CHECK(held_is(held_after_batch_run(10, false, 2, 14), 14, 0));
    // after every whole couple the kept buffer is the iteration's parity
    for (int64_t t0 = 0; t0 < 4; ++t0)
        for (int64_t t = t0 + 1; t <= t0 + 8; ++t) {
            const HeldState h = held_after_batch_run(t0, true, 2, t);
            CHECK(h.iter >= t && h.iter - t <= 1 && ((h.iter - t0) % 4 == 0 ? h.buf == (int)(h.iter & 1) : h.buf != (int)(h.iter & 1)));
        }
    // a bitwise stationary iteration freezes under any tolerance
    CHECK(freeze_now(0, 0, 0, 0.0));
    CHECK(freeze_now(0, bits(INFINITY), 64, 1e-6));
    // max_slots = 0: only a bitwise stationary iteration freezes
    CHECK(!freeze_now(1, 0, 0, 1.0));
    CHECK(!freeze_now(1, bits(0.0f), 0, 1.0));
    // within the tolerance
    CHECK(freeze_now(64, bits(1e-7f), 64, 1e-6));
    CHECK(freeze_now(1, bits(1e-6f), 64, 1e-6));   // float(1e-6) <= 1e-6
    // too many messages changed, or one by too much
    CHECK(!freeze_now(65, bits(1e-7f), 64, 1e-6));
    CHECK(!freeze_now(10, bits(2e-6f), 64, 1e-6));
    // a non-finite change never freezes
    CHECK(!freeze_now(1, bits(INFINITY), 64, 1e30));
    CHECK(!freeze_now(1, bits(NAN), 64, 1e30));
    // counts beyond 32 bits are compared as they are
    CHECK(!freeze_now((uint64_t)1 << 33, bits(1e-9f), 64, 1e-6));
    CHECK(!freeze_now(((uint64_t)1 << 32) + 1, bits(1e-9f), 64, 1e-6));
    // workspace layout: rows and planes 256-byte aligned, each message plane
    // one 256-byte skew longer than the node area, regions in order and
    // disjoint, for both precisions, both stencils and ragged sizes
    const int64_t sizes[][2] = {{8192, 4096}, {1, 1}, {5, 7}, {65, 3}, {1000, 999}, {32768, 64}};
    for (const auto &sz : sizes) {
        for (int deg : {4, 12}) {
            for (int f32 = 0; f32 < 2; ++f32) {
                const size_t es = f32 ? 4 : 8;
                const Layout l = make_layout(sz[0], sz[1], deg, es, f32 != 0);
                CHECK(l.pitch >= sz[0] && (l.pitch * es) % 256 == 0 && (l.pitch - sz[0]) * es < 256);
                const size_t node = (size_t)l.pitch * (size_t)sz[1];
                CHECK((size_t)l.plane >= node + 256 / es && ((size_t)l.plane * es) % 256 == 0);
                const size_t regions[] = {l.msg[0], l.msg[1], l.gain, l.adiag64, l.b64, l.mu64,
                                          l.bel64, l.partials, l.red, l.flags, l.total};
                for (size_t r : regions) CHECK(r % 256 == 0);
                const size_t buf = 2 * (size_t)deg * (size_t)l.plane * es;
                CHECK(l.msg[0] + buf <= l.msg[1] && l.msg[1] + buf <= l.gain);
                CHECK(l.gain + (size_t)deg * (size_t)l.plane * es <= l.adiag64);
                CHECK(l.adiag64 + node * 8 <= l.b64 && l.b64 + node * 8 <= l.mu64);
                CHECK(l.mu64 + node * 8 <= l.bel64 && l.bel64 + node * 8 <= l.partials);
                if (f32) CHECK(l.adiag_w >= l.bel64 + node * 8 && l.b_w >= l.adiag_w + node * 4);
                CHECK(l.flags + 8 * sizeof(uint32_t) <= l.total);
            }
        }
    }
    // tile ranges: the interior range is exactly the tiles whose halo of 2R
    // lies inside the grid; ring() visits every other tile once; hole and
    // ring tiles together cover every node once
    const int dims_x[] = {1, 5, 63, 64, 67, 68, 69, 131, 132, 133, 200, 1000};
    const int dims_y[] = {1, 3, 5, 7, 12, 13, 16, 17, 23, 28, 40, 97, 301};
    for (int nx : dims_x) {
        for (int ny : dims_y) {
            for (int R : {1, 2}) {
                for (int TH : {4, 8, 12, 16, 32}) {
                    const gabp::TileRange in = gabp::interior_tiles(nx, ny, R, TH);
                    CHECK(in.cols == (nx + 63) / 64 && in.rows == (ny + TH - 1) / TH);
                    int64_t inside = 0;
                    for (int ty = 0; ty < in.rows; ++ty)
                        for (int tx = 0; tx < in.cols; ++tx) {
                            const int x0 = 64 * tx, y0 = TH * ty;
                            const bool want = x0 >= 2 * R && x0 + 64 + 2 * R <= nx &&
                                              y0 >= 2 * R && y0 + TH + 2 * R <= ny;
                            CHECK(in.interior(tx, ty) == want);
                            inside += want;
                        }
                    CHECK(in.hole_count() == inside);
                    std::vector<int> seen((size_t)in.cols * in.rows, 0);
                    for (int b = 0; b < (int)in.ring_count(); ++b) {
                        int tx = -1, ty = -1;
                        in.ring(b, tx, ty);
                        CHECK(tx >= 0 && tx < in.cols && ty >= 0 && ty < in.rows);
                        CHECK(!in.interior(tx, ty));
                        CHECK(seen[(size_t)ty * in.cols + tx]++ == 0);
                    }
                    // nodes written: hole tiles and ring tiles, each node once
                    std::vector<int> cover((size_t)nx * ny, 0);
                    for (int ty = 0; ty < in.rows; ++ty)
                        for (int tx = 0; tx < in.cols; ++tx) {
                            if (!in.interior(tx, ty)) continue;
                            for (int y = TH * ty; y < std::min(ny, TH * ty + TH); ++y)
                                for (int x = 64 * tx; x < std::min(nx, 64 * tx + 64); ++x)
                                    ++cover[(size_t)y * nx + x];
                        }
                    for (int b = 0; b < (int)in.ring_count(); ++b) {
                        int tx = -1, ty = -1;
                        in.ring(b, tx, ty);
                        for (int y = TH * ty; y < std::min(ny, TH * ty + TH); ++y)
                            for (int x = 64 * tx; x < std::min(nx, 64 * tx + 64); ++x)
                                ++cover[(size_t)y * nx + x];
                    }
                    for (int c : cover) CHECK(c == 1);
                }
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
