// Index arithmetic of the per-wave deferred-tap queue of the lit forward kernels: which slot a
// lane's queued sample takes, the count and step-start words after a step, when the queue must
// be resolved first, and where each step's run of samples ends.  Pure integer functions,
// constexpr so that one definition serves the kernels and host code (a host model of the queue
// protocol drives exactly these functions).
#pragma once

#include <cstdint>

namespace amr {

constexpr int kTapQ = 96;   // queued samples per wave

// Lanes below `lane` in a wave64 mask.
constexpr uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

constexpr uint32_t popc64(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }

// Lowest set bit of a non-zero mask.
constexpr uint32_t ctz64(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// The queue holding `count` samples must be resolved before the lanes of `marching` each queue
// one more sample in a step.
constexpr bool tapq_full(uint32_t count, uint64_t marching) { return count + popc64(marching) > (uint32_t)kTapQ; }

// Slot of lane `lane`'s sample when the lanes of `need` queue one sample each in a step that
// starts at count c0 (lower lanes first).
constexpr uint32_t tapq_slot(uint32_t c0, uint64_t need, int lane) { return c0 + popc64(need & lanes_below(lane)); }

// Count after such a step; a slot at or beyond kTapQ is dropped (tapq_full prevents it).
constexpr uint32_t tapq_count_after(uint32_t c0, uint64_t need) {
    return c0 + popc64(need) < (uint32_t)kTapQ ? c0 + popc64(need) : (uint32_t)kTapQ;
}

// Step-start words (bit j of the 128-bit pair: a step's samples start at slot j) after a step
// whose samples start at slot c0 < kTapQ.
struct TapqStarts {
    uint64_t w0, w1;
};
constexpr TapqStarts tapq_mark(uint64_t b0, uint64_t b1, uint32_t c0) {
    return c0 < 64u ? TapqStarts{b0 | (1ull << c0), b1} : TapqStarts{b0, b1 | (1ull << (c0 - 64u))};
}

// End of the run of samples queued by the step that starts at slot s: the next step's start,
// else the count n.
constexpr uint32_t tapq_run_end(uint64_t b0, uint64_t b1, uint32_t s, uint32_t n) {
    if (s < 64u) {
        const uint64_t above = s == 63u ? 0ull : b0 & ~((2ull << s) - 1ull);
        if (above) return ctz64(above);
        return b1 ? 64u + ctz64(b1) : n;
    }
    const uint32_t t = s - 64u;
    const uint64_t above = t == 63u ? 0ull : b1 & ~((2ull << t) - 1ull);
    return above ? 64u + ctz64(above) : n;
}

// The stepped lit loop fetches segments (instead of sampling) in a step where every live lane
// waits for one, or at least half of them do.
constexpr bool stepped_fetch(uint64_t live, uint64_t waiting) {
    return waiting == live || 2u * popc64(waiting) >= popc64(live);
}

static_assert(tapq_slot(5, 0b1011ull, 3) == 7, "slot of lane 3 after lanes 0 and 1");
static_assert(tapq_run_end(0b101ull, 0ull, 0, 9) == 2 && tapq_run_end(0b101ull, 0ull, 2, 9) == 9, "runs");
static_assert(tapq_run_end(1ull << 63, 1ull, 63, 70) == 64 && tapq_run_end(0ull, 0b11ull, 64, 70) == 65, "runs");
static_assert(!tapq_full(32, ~0ull) && tapq_full(33, ~0ull), "a step of 64 lanes fits 96 - 32 slots");

}  // namespace amr
