// Host model of the lit forward kernels' per-wave deferred-tap queue (test code).
//
// It plays the wave-level control flow of the two kernels that use the queue, with 64 lanes as
// arrays and ballots as masks, and calls the kernels' own index functions (amr_tapq_index.h):
//   mode 0: the single-camera kernel's stepped loop (every lane of the wave steps together; the
//           queue is resolved at the top of a step when it cannot take one sample from every
//           sampling lane, and, with checkpoints, before each segment fetch);
//   mode 1: the persistent kernel's per-segment loop (the lanes still sampling a segment
//           reserve slots and resolve the queue themselves; four such waves share a block but
//           each has its own queue, so one wave is modelled at a time);
//   mode 2: the stepped loop of the non-recording single-camera kernels: after a step's sample,
//           the lanes that still have one take their next sample in the same step when the
//           queue has a slot for each of them whose sample is queued;
//   mode 3: the per-segment loop of the non-recording persistent kernel, with the same second
//           sample per round for the lanes still in their segment.
// Every slot, owner, run bound, leaf, patch and pool index is checked; every queued sample
// must be resolved exactly once, and each owner's deferred contributions must arrive in its
// sample order.  Input (stdin, whitespace separated):
//   mode ckpt nleaves npatches pool_floats nwaves
//   then per wave, per lane (64): nseg, then per segment: n leaf patch off, then n flags
//   (0 sampled at once, 1 queued, 2 queued and the ray ends after it, 3 the ray ends after it).
// Prints one summary line; exits non-zero (an assertion or the sanitizers) on any violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "amr_tapq_index.h"

using namespace amr;

#define CHECK(c)                                                                                   \
    do {                                                                                           \
        if (!(c)) {                                                                                \
            std::fprintf(stderr, "violated: %s (line %d, wave %d, step %ld)\n", #c, __LINE__, g_wave, \
                         g_step);                                                                  \
            std::exit(3);                                                                          \
        }                                                                                          \
    } while (0)

static int g_wave = 0;
static long g_step = 0;
static int g_nleaves, g_npatches;
static long g_pool;

struct Seg {
    int n, leaf, patch;
    long off;
    std::vector<int> flag;
};

struct Lane {
    std::vector<Seg> segs;
    size_t next = 0;          // next segment to fetch
    int cur = -1, k = 0;      // segment being sampled, next sample
    bool alive = true, has = false;
    long sampled = 0, queued = 0, resolved = 0;
    long last_ord = -1;       // ordinal of the last deferred contribution added to this lane
    long ord = 0;             // ordinal of the next queued sample of this lane
};

struct Slot {
    int owner = -1, leaf = -1, patch = -1;
    long off = -1, ord = -1;
    bool written = false, done = false;
};

struct Queue {
    Slot slot[kTapQ];
    uint32_t count = 0;
    uint64_t b0 = 0, b1 = 0;
    long flushes = 0, max_fill = 0, resolved = 0;
};

// The resolving lanes (mask act) resolve every queued sample and add the contributions run by
// run, each run's owners distinct (the kernel's tapq_flush).
static void flush(Queue &Q, uint64_t act, std::vector<Lane> &L) {
    CHECK(act != 0);
    const uint32_t n = Q.count, nact = popc64(act);
    CHECK(n <= (uint32_t)kTapQ);
    Q.flushes++;
    if ((long)n > Q.max_fill) Q.max_fill = n;
    // resolution: lane of rank r takes slots r, r + nact, ... (every slot below n exactly once)
    std::vector<int> seen(n, 0);
    for (int lane = 0; lane < 64; lane++) {
        if (!((act >> lane) & 1ull)) continue;
        const uint32_t rank = popc64(act & lanes_below(lane));
        for (uint32_t j = rank; j < n; j += nact) {
            CHECK(j < (uint32_t)kTapQ);
            Slot &s = Q.slot[j];
            CHECK(s.written && !s.done);
            CHECK(s.owner >= 0 && s.owner < 64);
            CHECK(s.leaf >= 0 && s.leaf < g_nleaves);
            CHECK(s.patch >= 0 && s.patch < g_npatches);
            CHECK(s.off >= 0 && s.off < g_pool);
            seen[j]++;
        }
    }
    for (uint32_t j = 0; j < n; j++) CHECK(seen[j] == 1);
    // contributions: steps one after the other, each step's samples from distinct owners
    std::vector<int> covered(n, 0);
    const uint64_t b0 = Q.b0, b1 = Q.b1;
    for (int w = 0; w < 2; w++) {
        uint64_t bs = w ? b1 : b0;
        while (bs) {
            const uint32_t s = 64u * w + ctz64(bs);
            bs &= bs - 1ull;
            const uint32_t e = tapq_run_end(b0, b1, s, n);
            CHECK(s < n && s < e && e <= n);
            uint64_t owners = 0;
            for (uint32_t j = s; j < e; j++) {
                Slot &sl = Q.slot[j];
                CHECK(!((owners >> sl.owner) & 1ull));
                owners |= 1ull << sl.owner;
                Lane &o = L[sl.owner];
                CHECK(sl.ord == o.last_ord + 1);     // the owner's sample order
                o.last_ord = sl.ord;
                o.resolved++;
                sl.done = true;
                covered[j]++;
            }
        }
    }
    for (uint32_t j = 0; j < n; j++) CHECK(covered[j] == 1);
    Q.resolved += n;
    for (int j = 0; j < kTapQ; j++) Q.slot[j] = Slot();
    Q.count = 0;
    Q.b0 = Q.b1 = 0;
}

// One sample by every lane of mask `samp` (each with a segment and a sample left); lanes whose
// sample is queued take slots (the kernel's tapq_push), then the lanes advance.
static void sample_step(Queue &Q, uint64_t samp, std::vector<Lane> &L) {
    uint64_t need = 0;
    for (int lane = 0; lane < 64; lane++) {
        if (!((samp >> lane) & 1ull)) continue;
        const Lane &l = L[lane];
        CHECK(l.has && l.cur >= 0 && l.k < l.segs[l.cur].n);
        const int f = l.segs[l.cur].flag[l.k];
        if (f == 1 || f == 2) need |= 1ull << lane;
    }
    const uint32_t c0 = Q.count;
    for (int lane = 0; lane < 64; lane++) {
        if (!((need >> lane) & 1ull)) continue;
        Lane &l = L[lane];
        const uint32_t j = tapq_slot(c0, need, lane);
        CHECK(j < (uint32_t)kTapQ);                  // a slot per sampling lane was reserved
        Slot &s = Q.slot[j];
        CHECK(!s.written);
        const Seg &g = l.segs[l.cur];
        s.owner = lane;
        s.leaf = g.leaf;
        s.patch = g.patch;
        s.off = g.off;
        s.ord = l.ord++;
        s.written = true;
        l.queued++;
    }
    if (need && c0 < (uint32_t)kTapQ) {
        const TapqStarts b = tapq_mark(Q.b0, Q.b1, c0);
        Q.b0 = b.w0;
        Q.b1 = b.w1;
        Q.count = tapq_count_after(c0, need);
    }
    for (int lane = 0; lane < 64; lane++) {
        if (!((samp >> lane) & 1ull)) continue;
        Lane &l = L[lane];
        const int f = l.segs[l.cur].flag[l.k];
        l.sampled++;
        l.k++;
        if (f == 2 || f == 3) {
            l.alive = false;
            l.has = false;
        } else if (l.k == l.segs[l.cur].n) {
            l.has = false;
        }
    }
}

// The next segment with samples of a waiting lane, or the end of its ray.
static void fetch(Lane &l) {
    while (true) {
        if (l.next >= l.segs.size()) {
            l.alive = false;
            return;
        }
        const int s = (int)l.next++;
        if (l.segs[s].n > 0) {
            l.cur = s;
            l.k = 0;
            l.has = true;
            return;
        }
    }
}

static void run_stepped(Queue &Q, std::vector<Lane> &L, bool ckpt, bool two) {
    while (true) {
        uint64_t live = 0, samp = 0, wait = 0;
        for (int i = 0; i < 64; i++) {
            live |= (uint64_t)L[i].alive << i;
            samp |= (uint64_t)L[i].has << i;
            wait |= (uint64_t)(L[i].alive && !L[i].has) << i;
        }
        if (!live) break;
        g_step++;
        if (tapq_full(Q.count, samp)) flush(Q, ~0ull, L);
        if (stepped_fetch(live, wait)) {
            if (ckpt && Q.count) flush(Q, ~0ull, L);
            for (int i = 0; i < 64; i++)
                if ((wait >> i) & 1ull) fetch(L[i]);
            continue;
        }
        CHECK(samp != 0);
        sample_step(Q, samp, L);
        if (two) {
            uint64_t samp2 = 0, need2 = 0;
            for (int i = 0; i < 64; i++) {
                if (!L[i].has) continue;
                samp2 |= 1ull << i;
                const int f = L[i].segs[L[i].cur].flag[L[i].k];
                if (f == 1 || f == 2) need2 |= 1ull << i;
            }
            if (samp2 && !tapq_full(Q.count, need2)) sample_step(Q, samp2, L);
        }
    }
    if (Q.count) flush(Q, ~0ull, L);
}

static void run_per_segment(Queue &Q, std::vector<Lane> &L, bool two) {
    while (true) {
        // the lanes still marching fetch their next segment together
        uint64_t outer = 0;
        for (int i = 0; i < 64; i++) {
            Lane &l = L[i];
            if (!l.alive) continue;
            if (l.next >= l.segs.size()) {
                l.alive = false;
                continue;
            }
            l.cur = (int)l.next++;
            l.k = 0;
            l.has = l.segs[l.cur].n > 0;
            outer |= 1ull << i;
        }
        if (!outer) break;
        // the inner sample loop: the lanes with samples left step together
        while (true) {
            uint64_t act = 0;
            for (int i = 0; i < 64; i++)
                if (((outer >> i) & 1ull) && L[i].has) act |= 1ull << i;
            if (!act) break;
            g_step++;
            if (tapq_full(Q.count, act)) flush(Q, act, L);
            sample_step(Q, act, L);
            if (two) {
                uint64_t act2 = 0, need2 = 0;
                for (int i = 0; i < 64; i++) {
                    if (!((act >> i) & 1ull) || !L[i].has) continue;
                    act2 |= 1ull << i;
                    const int f = L[i].segs[L[i].cur].flag[L[i].k];
                    if (f == 1 || f == 2) need2 |= 1ull << i;
                }
                if (act2 && !tapq_full(Q.count, need2)) sample_step(Q, act2, L);
            }
        }
    }
    if (Q.count) flush(Q, ~0ull, L);
}

int main() {
    int mode, ckpt, nwaves;
    if (std::scanf("%d %d %d %d %ld %d", &mode, &ckpt, &g_nleaves, &g_npatches, &g_pool, &nwaves) != 6) return 2;
    long samples = 0, queued = 0, flushes = 0, max_fill = 0, steps = 0;
    for (g_wave = 0; g_wave < nwaves; g_wave++) {
        std::vector<Lane> L(64);
        for (int i = 0; i < 64; i++) {
            int nseg;
            if (std::scanf("%d", &nseg) != 1) return 2;
            L[i].segs.resize(nseg);
            for (int s = 0; s < nseg; s++) {
                Seg &g = L[i].segs[s];
                if (std::scanf("%d %d %d %ld", &g.n, &g.leaf, &g.patch, &g.off) != 4) return 2;
                g.flag.resize(g.n);
                for (int k = 0; k < g.n; k++)
                    if (std::scanf("%d", &g.flag[k]) != 1) return 2;
            }
            L[i].alive = nseg > 0;
        }
        Queue Q;
        g_step = 0;
        if (mode == 1 || mode == 3) run_per_segment(Q, L, mode == 3);
        else run_stepped(Q, L, ckpt != 0, mode == 2);
        for (int i = 0; i < 64; i++) {
            CHECK(!L[i].alive && !L[i].has);
            CHECK(L[i].resolved == L[i].queued && L[i].last_ord + 1 == L[i].queued);
            samples += L[i].sampled;
            queued += L[i].queued;
        }
        CHECK(Q.resolved == [&] { long q = 0; for (auto &l : L) q += l.queued; return q; }());
        flushes += Q.flushes;
        if (Q.max_fill > max_fill) max_fill = Q.max_fill;
        steps += g_step;
    }
    std::printf("ok waves=%d samples=%ld queued=%ld flushes=%ld max_fill=%ld steps=%ld\n", nwaves, samples, queued,
                flushes, max_fill, steps);
    return 0;
}
