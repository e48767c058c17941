// Host-side check of the precision-freeze decision (gabp::host::freeze_now),
// compiled and run by tests/test_host_logic.py.  Exit status 0 and "ok" when
// every case holds.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "host_common.h"

using gabp::host::freeze_now;

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

int main() {
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
    std::printf("ok\n");
    return 0;
}
