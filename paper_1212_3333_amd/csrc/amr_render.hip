// Device side of libamr: the single-pass raycaster (Section 5.3), its adjoint, and launchers.
//
// One lane owns one ray and a wave64 covers an 8x8 pixel tile; the forward kernel runs one wave
// per block, the adjoint four.
// The FP64 parts (ray generation, slab clip, kD-restart planes, sample positions of gradient
// taps) are written with contraction disabled so that every operation is correctly rounded
// exactly once; the per-sample arithmetic (trilinear, LUT, exp, compositing) is fp32 in
// patch-local cell coordinates.  Forward and adjoint evaluate samples with the same device
// functions (stencil, tap resolution, LUT, shading), so the adjoint replays the forward's sample
// values; the lit forward defers samples whose taps leave the brick to a per-wave queue and
// sums their colour separately, which changes a pixel by rounding only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "amr_render_common.h"

namespace amr {

// ------------------------------------------------------------------------------------------
// Forward kernel
// ------------------------------------------------------------------------------------------

// At least 3 waves per SIMD: the timed lit kernel fits in 158 VGPRs without spilling and 12 KB
// of LDS (its tap queue), so 12 waves share a CU; the unlit one needs 78 VGPRs and runs 6.
// LAY: the brick layout fixed at compile time for the timed variants (-1: read at run time).
// Lit variants defer the samples whose gradient taps leave the brick (trilinear) or need the
// tree (nearest cell) to a per-wave queue (TapQueue).
// While recording checkpoints for the adjoint, the queue is resolved before each segment fetch
// that writes one, so a checkpoint's colour holds every earlier sample; the gradients the queue
// resolves are written to the ray's tape, so the adjoint reads them instead of resolving taps.
// CK: checkpoints (and the tape) without the other recording outputs, for the adjoint's forward
// pass at the layout's compiled addressing.
template <bool LIT, bool REC, bool NEAR, int LAY, bool CK = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void render_fwd(RenderArgs A, CamGroup G) {
    // scheduled launches: this block's camera and super-tile from the order (or, before a call
    // has recorded it, camera by camera, super-tiles row by row)
    int gc = (int)blockIdx.y;
    uint32_t sst = 0xffffffffu;
    constexpr uint32_t kSide = sched_side(LIT);
    if (G.sched) {
        const uint32_t rank = (blockIdx.x / (8u * kSide * kSide)) * 8u + blockIdx.x % 8u;
        if (rank >= G.nst) return;
        uint32_t e;
        if (A.sched_hdr[4 * G.cam0 + 1] == G.sig) {
            e = A.sched_order[G.order0 + rank];
        } else {
            int c = 0;
            while (c + 1 < kCamGroup && c + 1 < G.n && rank >= G.stpre[c + 1]) c++;
            e = ((uint32_t)c << 24) | (rank - G.stpre[c]);
        }
        gc = (int)(e >> 24);
        sst = e & 0xffffffu;
        if (gc >= (G.n > 0 ? G.n : 1)) return;       // never for an order the library wrote
    }
    take_camera(A, G, gc);
    constexpr bool kDefer = LIT;
    constexpr bool kCk = REC || CK;             // checkpoints (and the tape) may be recorded
    __shared__ float4 s_lut[256];
    TapQueue *tq = nullptr;
    if constexpr (kDefer) tq = tap_queues<1>();
    for (int i = threadIdx.x; i < 256; i += 64) s_lut[i] = A.lut[i];
    __syncthreads();

    // One wave per block, one 8x8 pixel tile per wave.  Tiles are grouped in 4x4 super-tiles
    // (32x32 pixels) numbered along a Morton curve; blocks are dealt round-robin to the 8 XCDs
    // and XCD x renders super-tiles x, x + 8, x + 16, ...  Every XCD thus gets a share of every
    // part of the image (the work per tile varies by 10x and more across the screen), while
    // the tiles in flight on one XCD stay grouped in a few compact 32x32 patches whose rays
    // share bricks in that XCD's L2.  With a tile schedule, the super-tiles of all the launch's
    // cameras (kSide x kSide tiles) are dealt the same way in the schedule's order (longest tile
    // of the last call first) instead.
    int col, row;
    if (G.sched) {
        const uint32_t sgw = ((uint32_t)A.t8x + kSide - 1u) / kSide;
        const uint32_t li = blockIdx.x / 8u;
        col = (int)((sst % sgw) * kSide + (li % (kSide * kSide)) / kSide);
        row = (int)((sst / sgw) * kSide + li % kSide);
    } else {
        const int xcd = (int)(blockIdx.x % 8), li = (int)(blockIdx.x / 8);
        const int sidx = (li >> 4) * 8 + xcd;          // Morton index of the super-tile
        int sx = 0, sy = 0;
        #pragma unroll
        for (int bit = 0; bit < 12; bit++) {
            sx |= ((sidx >> (2 * bit)) & 1) << bit;
            sy |= ((sidx >> (2 * bit + 1)) & 1) << bit;
        }
        col = sx * 4 + ((li & 15) >> 2);
        row = sy * 4 + (li & 3);
    }
    if (col >= A.t8x || row >= A.t8y) return;
    const unsigned long long tile_t0 = A.sched_time ? wall_clock64() : 0ull;
    const int lane = threadIdx.x & 63;
    const int pi = col * 8 + (lane & 7);
    const int pj = row * 8 + (lane >> 3);
    const bool valid = pi < A.width && pj < A.height;
    const int64_t ray = (int64_t)pj * A.width + pi;

    Counters cnt;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    int nseg = 0, nsamp_total = 0;
    Ray R;
    bool alive = valid && setup_ray(A, pi, pj, R);
    if (REC) cnt.hit = alive ? 1 : 0;
    // checkpoints for the adjoint: (t, T, C) at the start of every `every`-th data segment
    CkptHeader *ckh = nullptr;
    Ckpt *ck = nullptr;
    int nck = 0, every = A.ckpt_every, dseg = 0;
    // the tape (lit, with checkpoints): the ray's row and its records so far; tape_base is the row
    // of the tile's lane 0, which the queue resolution addresses owners from
    uint32_t tpos = 0;
    const int64_t tape_base = (kCk && LIT && A.tape) ? A.ckpt_ray0 + (int64_t)(row * 8) * A.width + col * 8 : -1;
    float4 *trow = (kCk && LIT && A.tape && valid) ? A.tape + (A.ckpt_ray0 + ray) * A.tape_cap : nullptr;
    if (kCk && A.ckpt && valid) {
        ckh = reinterpret_cast<CkptHeader *>(A.ckpt + (A.ckpt_ray0 + ray) * A.ckpt_stride);
        ck = reinterpret_cast<Ckpt *>(ckh + 1);
    }
    if constexpr (kDefer) {
        // Lit, deferred taps: the wave's lanes step together.  A step either fetches the next
        // data segment of the lanes that have none (once half of the live lanes wait, or
        // all do) or takes one sample on every lane that has a segment; the tap queue is
        // resolved at the top of a step, where every lane of the wave works on it.  Segments,
        // sample positions and traces are those of the per-segment loop of the unlit variants
        // below.
        TapQueue &Q = *tq;
        tapq_init(Q, lane);
        double tcur = R.t0;
        uint32_t start = 0;
        Segment S;
        int k = 0;
        bool has = false;                 // a data segment with samples left
        while (true) {
            const unsigned long long live = __ballot(alive);
            if (!live) break;
            const unsigned long long samp = __ballot(has);
            if (tapq_full(tq_count(Q), samp)) tapq_flush<REC, LAY, NEAR, kCk>(A, s_lut, Q, lane, cnt, tape_base);
            const bool waiting = alive && !has;
            const unsigned long long wait = __ballot(waiting);
            if (stepped_fetch(live, wait)) {
                if (kCk && A.ckpt && tq_count(Q)) tapq_flush<REC, LAY, NEAR, kCk>(A, s_lut, Q, lane, cnt, tape_base);
                if (waiting) {
                    while (true) {            // next segment with samples, or the end of the ray
                        if (!(tcur < R.t1)) { alive = false; break; }
                        double tb = R.t1;
                        const int leaf = descend(A, R, tcur, tb, start);
                        if (leaf < 0) { alive = false; break; }
                        if (REC) cnt.segments++;
                        if (REC && A.touch_meta) touch_segment_meta(A, R, tcur, leaf);
                        const DLeaf &L = A.leaves[leaf];
                        const int p = L.patch;
                        int n = 0;
                        if (p >= 0) {
                            if (kCk && ck) {
                                if (dseg % every == 0) {
                                    if (nck == A.ckpt_max) {     // full: keep every other, halve the rate
                                        for (int i = 0; i < A.ckpt_max / 2; i++) ck[i] = ck[2 * i];
                                        nck = A.ckpt_max / 2;
                                        every *= 2;
                                        if (REC) cnt.ckover++;
                                    }
                                    if (dseg % every == 0) {     // colour: shaded at once + deferred, all resolved
                                        Ckpt c;
                                        c.t = tcur;
                                        c.T = T;
                                        c.C[0] = C0 + Q.cd[0][lane];
                                        c.C[1] = C1 + Q.cd[1][lane];
                                        c.C[2] = C2 + Q.cd[2][lane];
                                        c.rec = (int32_t)tpos;
                                        c.sidx = nsamp_total;
                                        ck[nck++] = c;
                                    }
                                }
                                dseg++;
                            }
                            setup_segment<LIT, LAY>(A, R, L, leaf, tcur, tb, S);
                            n = S.n;
                            if (kCk && trow && n > 0) {
                                if (tpos < (uint32_t)A.tape_cap) trow[tpos] = tape_segment(S.delta, S.dl, n);
                                tpos++;
                            }
                        }
                        if (REC && A.trace) {
                            if (nseg < A.trace_cap) {
                                amr_trace_rec rec;
                                rec.leaf = leaf;
                                rec.patch = p;
                                rec.n = n;
                                rec.level = leaf_level(L);
                                rec.ta = tcur;
                                rec.tb = tb;
                                A.trace[ray * A.trace_cap + nseg] = rec;
                            } else {
                                cnt.tover++;
                            }
                        }
                        nseg++;
                        if (tb <= tcur) {   // never expected: keep the walk moving forward
                            if (REC) cnt.guard++;
                            tb = nextafter(tcur, INFINITY);
                        }
                        tcur = tb;
                        if (n > 0) {
                            k = 0;
                            has = true;
                            break;
                        }
                    }
                }
                continue;
            }
            if constexpr (!REC && !NEAR) {
                // Two samples per step: the stencils of a lane's next two samples are read
                // together (one round of brick reads for both), the first is taken as above,
                // and the second too when the queue has a slot for each lane whose second
                // sample defers (tapq_full over those lanes); otherwise it is read again in the
                // next step.  The samples are taken in order and each lane's queued samples
                // stay in its sample order (one run per push), so results are those of one
                // sample per step.
                float qa[3], qb[3], Fa, Fpa[3], Fma[3], Fb, Fpb[3], Fmb[3];
                uint32_t cla = 0u, clb = 0u;
                if (has) {
                    const int kb = min(k + 1, S.n - 1);
                    const float kka = (float)k + 0.5f, kkb = (float)kb + 0.5f;
                    #pragma unroll
                    for (int a = 0; a < 3; a++) {
                        qa[a] = S.q0[a] + kka * S.dq[a];
                        qb[a] = S.q0[a] + kkb * S.dq[a];
                    }
                    cla = lit_stencil<REC, LAY>(A, S, qa[0], qa[1], qa[2], Fa, Fpa, Fma);
                    clb = lit_stencil<REC, LAY>(A, S, qb[0], qb[1], qb[2], Fb, Fpb, Fmb);
                    const float alpha = lit_consume<REC>(A, s_lut, Q, lane, R, S, k, nullptr, qa[0], qa[1], qa[2], Fa,
                                                         Fpa, Fma, cla, pending_taps(cla), T, C0, C1, C2, cnt, trow,
                                                         &tpos);
                    T *= 1.f - alpha;
                    nsamp_total++;
                    k++;
                    if (T < A.t_min) {
                        alive = false;
                        has = false;
                    } else if (k == S.n) {
                        has = false;
                    }
                }
                const unsigned long long second = __ballot(has);
                const unsigned long long needb = __ballot(has && pending_taps(clb) != 0u);
                if (second && !tapq_full(tq_count(Q), needb) && has) {
                    const float alpha = lit_consume<REC>(A, s_lut, Q, lane, R, S, k, nullptr, qb[0], qb[1], qb[2], Fb,
                                                         Fpb, Fmb, clb, pending_taps(clb), T, C0, C1, C2, cnt, trow,
                                                         &tpos);
                    T *= 1.f - alpha;
                    nsamp_total++;
                    k++;
                    if (T < A.t_min) {
                        alive = false;
                        has = false;
                    } else if (k == S.n) {
                        has = false;
                    }
                }
            } else if (has) {
                const float alpha = lit_sample_deferred<REC, LAY, NEAR>(A, s_lut, Q, lane, R, S, k, T, C0, C1, C2, cnt,
                                                                       trow, &tpos);
                T *= 1.f - alpha;
                nsamp_total++;
                k++;
                if (T < A.t_min) {
                    alive = false;
                    has = false;
                } else if (k == S.n) {
                    has = false;
                }
            }
        }
        float D0, D1, D2;
        tapq_finish<REC, LAY, NEAR, kCk>(A, s_lut, Q, lane, cnt, D0, D1, D2, tape_base);
        C0 += D0;
        C1 += D1;
        C2 += D2;
    } else {
        double tcur = R.t0;
        uint32_t start = 0;
        while (alive && tcur < R.t1) {
            double tb = R.t1;
            int leaf = descend(A, R, tcur, tb, start);
            if (leaf < 0) break;
            if (REC) cnt.segments++;
            if (REC && A.touch_meta) touch_segment_meta(A, R, tcur, leaf);
            const DLeaf &L = A.leaves[leaf];
            const int p = L.patch;
            int nsm = 0;
            if (p >= 0) {
                if (kCk && ck) {
                    if (dseg % every == 0) {
                        if (nck == A.ckpt_max) {             // full: keep every other, halve the rate
                            for (int i = 0; i < A.ckpt_max / 2; i++) ck[i] = ck[2 * i];
                            nck = A.ckpt_max / 2;
                            every *= 2;
                            if (REC) cnt.ckover++;
                        }
                        if (dseg % every == 0) {
                            Ckpt c;
                            c.t = tcur;
                            c.T = T;
                            c.C[0] = C0;
                            c.C[1] = C1;
                            c.C[2] = C2;
                            c.rec = 0;
                            c.sidx = nsamp_total;
                            ck[nck++] = c;
                        }
                    }
                    dseg++;
                }
                Segment S;
                setup_segment<LIT, LAY>(A, R, L, leaf, tcur, tb, S);
                nsm = S.n;
                if constexpr (!REC && !kCk && !NEAR) {
                    float tseg = 1.f;
                    bool stop;
                    nsamp_total += composite_unlit<LAY>(A, s_lut, R, S, T, C0, C1, C2, tseg, stop, cnt);
                    if (stop) alive = false;
                } else {
                    for (int k = 0; k < nsm; k++) {
                        SampleVals v;
                        eval_sample<LIT, REC, NEAR, LAY>(A, s_lut, R, S, k, v, cnt);
                        float wgt = T * v.alpha * v.shade;
                        C0 += wgt * v.r;
                        C1 += wgt * v.g;
                        C2 += wgt * v.b;
                        T *= 1.f - v.alpha;
                        nsamp_total++;
                        if (T < A.t_min) { alive = false; break; }
                    }
                }
            }
            if (REC && A.trace) {
                if (nseg < A.trace_cap) {
                    amr_trace_rec rec;
                    rec.leaf = leaf;
                    rec.patch = p;
                    rec.n = p >= 0 ? nsm : 0;
                    rec.level = leaf_level(L);
                    rec.ta = tcur;
                    rec.tb = tb;
                    A.trace[ray * A.trace_cap + nseg] = rec;
                } else {
                    cnt.tover++;
                }
            }
            nseg++;
            if (tb <= tcur) {   // never expected: keep the walk moving forward
                if (REC) cnt.guard++;
                tb = nextafter(tcur, INFINITY);
            }
            tcur = tb;
        }
    }
    if (A.sched_time && lane == 0) {
        const unsigned long long dt = wall_clock64() - tile_t0;
        A.sched_time[A.tile0 + (int64_t)row * A.t8x + col] = dt < 0xffffffffull ? (uint32_t)dt : 0xffffffffu;
    }
    if (valid) {
        reinterpret_cast<float4 *>(A.rgba)[ray] = make_float4(C0, C1, C2, 1.f - T);
        if (REC && A.trace_n) A.trace_n[ray] = nseg;
        if (REC && A.nsamp) A.nsamp[ray] = nsamp_total;
        if (kCk && ckh) {
            CkptHeader hd;
            hd.T = T;
            hd.C[0] = C0;
            hd.C[1] = C1;
            hd.C[2] = C2;
            hd.nsamp = nsamp_total;
            hd.nck = nck;
            hd.every = every;
            hd.nrec = (int32_t)tpos;
            *ckh = hd;
        }
    }
    if (REC) {
        cnt.samples = nsamp_total;
        if (A.stats) flush_counters(A.stats, cnt, lane);
    }
}

// ------------------------------------------------------------------------------------------
// Adjoint kernels: one work item = one (ray, checkpoint interval).  Given (T, C) at the
// interval's start and the ray's final (T_N, C_N), every sample's derivatives are local:
//   dL/dsigma_k = delta_k [ gC . (T_{k+1} e_k - (C_N - C_<=k)) + gA T_N ],
//   dL/drgb_k   = gC T_k alpha_k shade_k,   dL/dshade_k = T_k alpha_k (gC . rgb_k),
// with e_k = shade_k rgb_k and C_<=k the colour accumulated up to and including sample k.
// LUT gradients are accumulated per wave in LDS and combined per block in a fixed order.
// The lit intervals whose tape records all fit are replayed from the tape (render_bwd_tape);
// the others walk the tree and evaluate their samples again (render_bwd).
// ------------------------------------------------------------------------------------------

// An interval's pixel gradient, the ray's final transmittance and colour, and (T, C) at the
// current sample.
struct AdjRay {
    float4 g4;
    float TN, CN0, CN1, CN2;
    float T, C0, C1, C2;
};

// A lane's sums of the shading-parameter gradients: light direction, k_a, k_d.
struct AdjSums {
    float gl0 = 0.f, gl1 = 0.f, gl2 = 0.f, gka = 0.f, gkd = 0.f;
};

// LUT-gradient terms x of consecutive samples in one LUT interval [b, b + 1], summed in
// registers (s = sum x, sf = sum f x with f the sample's position in the interval) and added
// to the wave's LDS accumulator when the interval changes: entry b takes s - sf, b + 1 takes
// sf.  Samples along a ray often stay in one interval, so this saves most LDS atomics, which
// collide when the lanes of a wave hit the same entries.  b < 0: nothing held.
struct LutRun {
    int b = -1;
    float s[4] = {0.f, 0.f, 0.f, 0.f}, sf[4] = {0.f, 0.f, 0.f, 0.f};
};

__device__ __forceinline__ void lut_run_flush(float *acc, const LutRun &r) {
    if (r.b < 0) return;
    float *a0 = acc + 4 * r.b;
    #pragma unroll
    for (int c = 0; c < 4; c++) {
        atomicAdd(a0 + c, r.s[c] - r.sf[c]);
        atomicAdd(a0 + 4 + c, r.sf[c]);
    }
}

// One sample's adjoint: advances (T, C) past the sample and accumulates its LUT and
// shading-parameter gradients.  RUN: LUT terms through the register run (else straight to LDS).
template <bool LIT, bool RUN>
__device__ __forceinline__ void adjoint_sample(const RenderArgs &A, const SampleVals &v, float dlt, AdjRay &a,
                                               float *acc, LutRun &run, AdjSums &gs) {
    const float ta = a.T * v.alpha;
    const float e0 = v.shade * v.r, e1 = v.shade * v.g, e2 = v.shade * v.b;
    a.C0 += ta * e0;
    a.C1 += ta * e1;
    a.C2 += ta * e2;
    const float Tn = a.T * (1.f - v.alpha);
    const float dsig = dlt * (a.g4.x * (Tn * e0 - (a.CN0 - a.C0)) + a.g4.y * (Tn * e1 - (a.CN1 - a.C1)) +
                              a.g4.z * (Tn * e2 - (a.CN2 - a.C2)) + a.g4.w * a.TN);
    const float wr = ta * v.shade;
    const float x[4] = {a.g4.x * wr, a.g4.y * wr, a.g4.z * wr, dsig};
    if (RUN) {
        if (v.i0 != run.b) {
            lut_run_flush(acc, run);
            run = LutRun();
            run.b = v.i0;
        }
        #pragma unroll
        for (int c = 0; c < 4; c++) {
            run.s[c] += x[c];
            run.sf[c] += v.f * x[c];
        }
    } else {
        const float w1 = v.f, w0 = 1.f - v.f;
        float *a0 = acc + 4 * v.i0;
        #pragma unroll
        for (int c = 0; c < 4; c++) {
            atomicAdd(a0 + c, w0 * x[c]);
            atomicAdd(a0 + 4 + c, w1 * x[c]);
        }
    }
    if (LIT) {
        const float dshade = ta * (a.g4.x * v.r + a.g4.y * v.g + a.g4.z * v.b);
        gs.gka += dshade;
        if (v.den > 0.f) {
            const float sg = v.dot > 0.f ? 1.f : (v.dot < 0.f ? -1.f : 0.f);
            const float q = dshade / v.den;
            const float cf = q * A.k_d * sg * A.inv_lnorm;
            gs.gl0 += cf * (v.gv[0] - v.dot * A.lhat[0]);
            gs.gl1 += cf * (v.gv[1] - v.dot * A.lhat[1]);
            gs.gl2 += cf * (v.gv[2] - v.dot * A.lhat[2]);
            gs.gkd += q * fabsf(v.dot);
        }
    }
    a.T = Tn;
}

// Start of an adjoint block (256 threads, four waves): the LUT and the wave accumulators in LDS.
__device__ __forceinline__ void adjoint_block_begin(const RenderArgs &A, float4 *s_lut, float (*s_acc)[kGradLen]) {
    s_lut[threadIdx.x] = A.lut[threadIdx.x];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = lane; i < kGradLen; i += 64) s_acc[wave][i] = 0.f;
    __syncthreads();
}

// End of an adjoint block: the shading-parameter sums reduced over each wave, the four wave
// accumulators combined in a fixed order, then written as the block's partial sum
// (deterministic mode) or added to the result.
template <bool LIT>
__device__ __forceinline__ void adjoint_block_end(const BwdArgs &B, float (*s_acc)[kGradLen], AdjSums gs) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (LIT) {
        gs.gl0 = wave_sumf(gs.gl0);
        gs.gl1 = wave_sumf(gs.gl1);
        gs.gl2 = wave_sumf(gs.gl2);
        gs.gka = wave_sumf(gs.gka);
        gs.gkd = wave_sumf(gs.gkd);
        if (lane == 0) {
            s_acc[wave][1024] += gs.gl0;
            s_acc[wave][1025] += gs.gl1;
            s_acc[wave][1026] += gs.gl2;
            s_acc[wave][1027] += gs.gka;
            s_acc[wave][1028] += gs.gkd;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kGradLen; i += blockDim.x) {
        float v = ((s_acc[0][i] + s_acc[1][i]) + s_acc[2][i]) + s_acc[3][i];
        if (B.partials) B.partials[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kGradLen + i] = v;
        else if (v != 0.f) atomicAdd(&B.grad[i], v);
    }
}

// The tape records of an interval: [rec0, end) with end the next checkpoint's position or the
// ray's total; the interval is on the tape when all of them were written.
__device__ __forceinline__ int interval_records_end(const CkptHeader &hd, const Ckpt *ck, int interval, int nck) {
    return interval + 1 < nck ? ck[interval + 1].rec : hd.nrec;
}

// In place: every sample of the interval is evaluated again (tree walk from the checkpoint,
// stencil, tap resolution).  Serves the unlit adjoint, lit renders without a tape, and the lit
// intervals whose tape records did not all fit.  Up to kCamGroup cameras per launch, one per
// blockIdx.y (their blocks split the fixed grid).  Work items run interval by interval (the
// lanes of a wave take neighbouring rays at one interval) when every interval is served here,
// and ray by ray (consecutive lanes take one ray's intervals) when only the tape's leftovers
// are: those are the late intervals of the longest rays, which would otherwise queue up on
// few threads.
// LAY: the brick layout fixed at compile time (-1: read at run time).
template <bool LIT, int LAY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LIT ? 3 : 4))) void render_bwd(RenderArgs A, BwdArgs B,
                                                                                                     CamGroup G) {
    take_camera(A, G, (int)blockIdx.y);
    if (G.n) B.grad_rgba += 4 * G.cam[blockIdx.y].ray0;
    __shared__ float4 s_lut[256];
    __shared__ float s_acc[4][kGradLen];      // one accumulator per wave
    adjoint_block_begin(A, s_lut, s_acc);
    float *acc = s_acc[threadIdx.x >> 6];
    AdjSums gs;
    LutRun run;
    Counters cnt;
    const int64_t nrays = (int64_t)A.width * A.height;
    const int64_t nitems = nrays * A.ckpt_max;
    for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < nitems;
         item += (int64_t)gridDim.x * blockDim.x) {
        int interval;
        int64_t ray;
        if (B.ray_major) {
            ray = item / A.ckpt_max;
            interval = (int)(item - ray * A.ckpt_max);
        } else {
            interval = (int)(item / nrays);
            ray = item - (int64_t)interval * nrays;
        }
        const CkptHeader *ckh = reinterpret_cast<const CkptHeader *>(A.ckpt + (A.ckpt_ray0 + ray) * A.ckpt_stride);
        const CkptHeader hd = *ckh;
        const int nck = min(hd.nck, A.ckpt_max);
        if (interval >= nck) continue;
        const Ckpt *ck = reinterpret_cast<const Ckpt *>(ckh + 1);
        const Ckpt c0 = ck[interval];
        const int s_end = interval + 1 < nck ? ck[interval + 1].sidx : hd.nsamp;
        if (LIT && A.tape && (int64_t)interval_records_end(hd, ck, interval, nck) <= A.tape_cap) continue;   // on the tape
        const int pi = (int)(ray % A.width), pj = (int)(ray / A.width);
        Ray R;
        if (!setup_ray(A, pi, pj, R)) continue;
        AdjRay a;
        a.g4 = reinterpret_cast<const float4 *>(B.grad_rgba)[ray];
        a.TN = hd.T;
        a.CN0 = hd.C[0];
        a.CN1 = hd.C[1];
        a.CN2 = hd.C[2];
        a.T = c0.T;
        a.C0 = c0.C[0];
        a.C1 = c0.C[1];
        a.C2 = c0.C[2];
        int s = c0.sidx;
        double tcur = c0.t;
        while (s < s_end && tcur < R.t1) {
            double tb = R.t1;
            int leaf = descend(A, R, tcur, tb);
            if (leaf < 0) break;
            const DLeaf &L = A.leaves[leaf];
            if (L.patch >= 0) {
                Segment S;
                setup_segment<LIT, LAY>(A, R, L, leaf, tcur, tb, S);
                const float dlt = (float)S.delta;
                for (int k = 0; k < S.n && s < s_end; k++, s++) {
                    SampleVals v;
                    eval_sample<LIT, false, false, LAY>(A, s_lut, R, S, k, v, cnt);
                    adjoint_sample<LIT, false>(A, v, dlt, a, acc, run, gs);
                }
            }
            if (tb <= tcur) tb = nextafter(tcur, INFINITY);
            tcur = tb;
        }
    }
    adjoint_block_end<LIT>(B, s_acc, gs);
}

// From the tape: the lit intervals whose records all fit are replayed from their segment and
// sample records alone (no tree walk, no brick reads), for every camera of the call in one launch
// (a ray's records need no camera).  Each lane reads its ray's records a
// group of kTapeGroup at a time (the group's records share cache lines, aligned in the tape):
// the group arrives with one fetch of its lines, where reading a record at a time would have
// the lines of the other lanes' streams evict them between reads.
constexpr int kTapeGroup = 8;

__global__ __launch_bounds__(256) void render_bwd_tape(RenderArgs A, BwdArgs B) {
    __shared__ float4 s_lut[256];
    __shared__ float s_acc[4][kGradLen];
    adjoint_block_begin(A, s_lut, s_acc);
    float *acc = s_acc[threadIdx.x >> 6];
    AdjSums gs;
    LutRun run;
    const int64_t nrays = B.nrays;
    const int64_t nitems = nrays * A.ckpt_max;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t item = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; item < nitems;
         item += (int64_t)gridDim.x * blockDim.x) {
        const int interval = (int)(item / nrays);
        const int64_t ray = item - (int64_t)interval * nrays;
        const CkptHeader *ckh = reinterpret_cast<const CkptHeader *>(A.ckpt + (A.ckpt_ray0 + ray) * A.ckpt_stride);
        const CkptHeader hd = *ckh;
        const int nck = min(hd.nck, A.ckpt_max);
        if (interval >= nck) continue;
        const Ckpt *ck = reinterpret_cast<const Ckpt *>(ckh + 1);
        const Ckpt c0 = ck[interval];
        const int s_end = interval + 1 < nck ? ck[interval + 1].sidx : hd.nsamp;
        const int r_end = interval_records_end(hd, ck, interval, nck);
        if ((int64_t)r_end > A.tape_cap || c0.rec < 0) continue;      // the in-place kernel's
        const int64_t row0 = (A.ckpt_ray0 + ray) * A.tape_cap;    // the ray's first record
        AdjRay a;
        a.g4 = reinterpret_cast<const float4 *>(B.grad_rgba)[ray];
        a.TN = hd.T;
        a.CN0 = hd.C[0];
        a.CN1 = hd.C[1];
        a.CN2 = hd.C[2];
        a.T = c0.T;
        a.C0 = c0.C[0];
        a.C1 = c0.C[1];
        a.C2 = c0.C[2];
        // absolute record indices: the interval's records are [p, e)
        int64_t p = row0 + c0.rec;
        const int64_t e = row0 + r_end;
        int s = c0.sidx, left = 0;        // left: samples of the current segment still to come
        float dlt = 0.f, dl = 0.f;
        bool more = s < s_end && p < e;
        while (more) {
            const int64_t g0 = p & ~(int64_t)(kTapeGroup - 1);
            float4 buf[kTapeGroup];
            #pragma unroll
            for (int j = 0; j < kTapeGroup; j++) buf[j] = (g0 + j >= p && g0 + j < e) ? A.tape[g0 + j] : zero;
            #pragma unroll
            for (int j = 0; j < kTapeGroup; j++) {
                if (more && g0 + j == p) {
                    const float4 r = buf[j];
                    p++;
                    if (left <= 0) {              // a segment record
                        left = __float_as_int(r.z);
                        dlt = r.x;
                        dl = r.y;
                    } else {                      // a sample record
                        SampleVals v;
                        v.gv[0] = r.y;
                        v.gv[1] = r.z;
                        v.gv[2] = r.w;
                        lut_classify(A, s_lut, r.x, dl, v);
                        v.shade = lit_shade(A, v.gv, v.dot, v.den);
                        adjoint_sample<true, true>(A, v, dlt, a, acc, run, gs);
                        left--;
                        s++;
                    }
                    more = s < s_end && p < e;
                }
            }
        }
    }
    lut_run_flush(acc, run);
    adjoint_block_end<true>(B, s_acc, gs);
}

// Tile schedule for the next call: the super-tiles (sched_side) of all cameras of a launch ordered by
// the time of their longest tile, longest first (a counting sort over 512 logarithmic buckets, 16
// per octave of the wall clock's ticks; the order within a bucket is arbitrary), one block; the
// header of the group's first camera then records the order's key, a signature of the call's
// camera sizes and of the group's place among them.  A super-tile keeps its tiles together on one
// XCD, as in the default order, so the schedule reorders the image's regions without scattering
// their tiles.  The first group's sort of a call whose camera sizes differ from the previous
// call's (word 2 of camera 0's header) first clears the keys of the call's other groups: their
// order slots may hold another list's entries.
struct SchedGroup {
    int64_t tile0[kCamGroup];        // each camera's first tile time
    int32_t t8x[kCamGroup], t8y[kCamGroup];
    uint32_t stpre[kCamGroup + 1];   // each camera's first super-tile in the group
    int32_t n, cam0;
    uint32_t sig, list_sig;
    int64_t order0;
    int32_t ncams;
    uint32_t side;                   // super-tile side in tiles (sched_side)
};
constexpr int kSchedBuckets = 512;

__device__ __forceinline__ int sched_bucket(uint32_t t) {
    if (t < 16u) return (int)t;
    const int msb = 31 - __builtin_clz(t);
    return min(kSchedBuckets - 1, (msb - 3) * 16 + (int)((t >> (msb - 4)) & 15u));
}

__global__ __launch_bounds__(1024) void sched_sort(uint32_t *hdr, const uint32_t *time, uint32_t *order,
                                                   SchedGroup G) {
    __shared__ uint32_t cnt[kSchedBuckets], cur[kSchedBuckets];
    const uint32_t n = G.stpre[G.n];
    // rank r of the default order: camera c with stpre[c] <= r < stpre[c + 1], its super-tile r - stpre[c]
    auto entry = [&](uint32_t r) {
        int c = 0;
        while (c + 1 < G.n && r >= G.stpre[c + 1]) c++;
        return ((uint32_t)c << 24) | (r - G.stpre[c]);
    };
    auto stime = [&](uint32_t e) {
        const int c = (int)(e >> 24);
        const uint32_t st = e & 0xffffffu;
        const int t8x = G.t8x[c], t8y = G.t8y[c];
        const uint32_t side = G.side;
        const uint32_t sgw = ((uint32_t)t8x + side - 1u) / side;
        const int sx = (int)((st % sgw) * side), sy = (int)((st / sgw) * side);
        uint32_t m = 0u;
        for (int j = 0; j < (int)(side * side); j++) {
            const int cx = sx + j / (int)side, cy = sy + j % (int)side;
            if (cx < t8x && cy < t8y) m = max(m, time[G.tile0[c] + (int64_t)cy * t8x + cx]);
        }
        return m;
    };
    for (int i = threadIdx.x; i < kSchedBuckets; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&cnt[sched_bucket(stime(entry(i)))], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0u;
        for (int b = kSchedBuckets - 1; b >= 0; b--) {
            cur[b] = s;
            s += cnt[b];
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t e = entry(i);
        const uint32_t pos = atomicAdd(&cur[sched_bucket(stime(e))], 1u);
        order[G.order0 + pos] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (G.cam0 == 0 && hdr[2] != G.list_sig) {
            for (int c = kCamGroup; c < G.ncams; c += kCamGroup) hdr[4 * c + 1] = 0u;
            hdr[2] = G.list_sig;
        }
        hdr[4 * G.cam0 + 1] = G.sig;
    }
}

// Fixed-order sum of per-block partials (deterministic adjoint).
__global__ void reduce_partials(const float *partials, int nblocks, float *grad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kGradLen) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; b++) s += partials[(int64_t)b * kGradLen + i];
    grad[i] += s;
}

__global__ void zero_f32(float *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void zero_u64(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void split_grad(const float *grad, float *grad_lut, float *grad_light) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 1024) grad_lut[i] = grad[i];
    else if (i < kGradLen) grad_light[i - 1024] = grad[i];
}

// The adjoint's launches with the gradient accumulators at `work` (device, at least
// amr_backward_work_bytes(deterministic) bytes): zero the accumulator, one render_bwd launch per
// camera (plus the fixed-order partial reduction in deterministic mode), then split the result
// into the LUT and shading gradients.  Enqueued on `stream`; no allocation, no synchronisation.
int backward_launch(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
                    const float *d_grad_rgba, float *d_grad_lut, float *d_grad_light, int32_t deterministic,
                    float *work, void *stream) {
    if (!S || !cams || !P || !d_grad_rgba || !d_grad_lut || !d_grad_light || ncams <= 0 || !work) {
        set_error("null argument or ncams <= 0");
        return AMR_EINVAL;
    }
    if (!P->d_ckpt) { set_error("the adjoint needs the forward's checkpoints (params.d_ckpt)"); return AMR_EINVAL; }
    if (P->interp != 0) { set_error("the adjoint is defined for trilinear sampling (interp = 0)"); return AMR_EINVAL; }
    if (P->lighting == 2) { set_error("the adjoint is defined for lighting 0 and 1"); return AMR_EINVAL; }
    int64_t total = 0;
    for (int c = 0; c < ncams; c++) total += (int64_t)cams[c].width * cams[c].height;
    if (P->ckpt_max < 2 || P->ckpt_bytes < amr_ckpt_bytes(total, P->ckpt_max)) {
        set_error("checkpoint buffer too small");
        return AMR_ECAPACITY;
    }
    if (P->d_tape && (P->tape_cap < 0 || P->tape_cap > kTapeCapMax || (reinterpret_cast<uintptr_t>(P->d_tape) & 15u))) {
        set_error("d_tape needs 16-byte alignment and tape_cap in [0, %lld]", (long long)kTapeCapMax);
        return AMR_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    float *grad = work;
    float *partials = deterministic ? work + kGradLen : nullptr;
    hipLaunchKernelGGL(zero_f32, dim3((kGradLen + 255) / 256), dim3(256), 0, s, grad, kGradLen);
    int rc = check_hip(hipGetLastError(), "adjoint accumulator reset");
    const dim3 g(kBwdGrid), b(256);
    // lit with a tape: the intervals the tape holds, every camera in one launch; then, per
    // camera, the others in place.  Otherwise one launch per camera, every interval in place.
    bool taped = false;
    if (rc == AMR_OK && P->lighting == 1 && P->d_tape && P->tape_cap > 0) {
        RenderArgs A;
        rc = fill_args(S, &cams[0], P, &A);
        if (rc == AMR_OK) {
            A.ckpt_ray0 = 0;
            BwdArgs B;
            B.grad_rgba = d_grad_rgba;
            B.grad = grad;
            B.partials = partials;
            B.ray_major = 0;
            B.nrays = total;
            hipLaunchKernelGGL(render_bwd_tape, g, b, 0, s, A, B);
            rc = check_hip(hipGetLastError(), "render_bwd_tape launch");
            if (rc == AMR_OK && deterministic)
                hipLaunchKernelGGL(reduce_partials, dim3((kGradLen + 255) / 256), dim3(256), 0, s, partials, kBwdGrid,
                                   grad);
            taped = true;
        }
    }
    // in place, up to kCamGroup cameras per launch, the fixed grid's blocks split among them
    int64_t pix_off = 0;
    for (int c0 = 0; c0 < ncams && rc == AMR_OK; c0 += kCamGroup) {
        const int n = std::min(kCamGroup, ncams - c0);
        RenderArgs A;
        CamGroup G;
        memset(&G, 0, sizeof(G));
        int64_t rel = 0;
        for (int i = 0; i < n && rc == AMR_OK; i++) {
            RenderArgs Ai;
            rc = fill_args(S, &cams[c0 + i], P, &Ai);
            if (rc) break;
            if (i == 0) A = Ai;
            G.cam[i] = cam_args_of(Ai, rel);
            rel += (int64_t)cams[c0 + i].width * cams[c0 + i].height;
        }
        if (rc) break;
        G.n = n > 1 ? n : 0;
        A.ckpt_ray0 = pix_off;
        BwdArgs B;
        B.grad_rgba = d_grad_rgba + 4 * pix_off;
        B.grad = grad;
        B.partials = partials;
        B.nrays = (int64_t)A.width * A.height;     // one camera's (taken per block)
        B.ray_major = taped;
        const dim3 gg(kBwdGrid / n, n);
        if (A.lighting) {
            if (A.layout == 0) hipLaunchKernelGGL((render_bwd<true, 0>), gg, b, 0, s, A, B, G);
            else if (A.layout == 1) hipLaunchKernelGGL((render_bwd<true, 1>), gg, b, 0, s, A, B, G);
            else hipLaunchKernelGGL((render_bwd<true, 2>), gg, b, 0, s, A, B, G);
        } else {
            if (A.layout == 0) hipLaunchKernelGGL((render_bwd<false, 0>), gg, b, 0, s, A, B, G);
            else if (A.layout == 1) hipLaunchKernelGGL((render_bwd<false, 1>), gg, b, 0, s, A, B, G);
            else hipLaunchKernelGGL((render_bwd<false, 2>), gg, b, 0, s, A, B, G);
        }
        rc = check_hip(hipGetLastError(), "render_bwd launch");
        if (rc == AMR_OK && deterministic)
            hipLaunchKernelGGL(reduce_partials, dim3((kGradLen + 255) / 256), dim3(256), 0, s, partials,
                               (int)(gg.x * gg.y), grad);
        pix_off += rel;
    }
    if (rc == AMR_OK) {
        hipLaunchKernelGGL(split_grad, dim3((kGradLen + 255) / 256), dim3(256), 0, s, grad, d_grad_lut, d_grad_light);
        rc = check_hip(hipGetLastError(), "adjoint gradient split");
    }
    return rc;
}

// Workspace of amr_render_backward_static: the adjoint's gradient accumulators (1029 floats)
// and deterministic partial sums (one 1029-float row per block of the fixed grid), in a
// fixed array of the library's code object.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as a device address; it takes
// each device's address once from hipGetSymbolAddress, with that device current.
constexpr size_t kStaticWorkFloats = (size_t)kGradLen * (1 + (size_t)kBwdGrid);
static __device__ __align__(256) float scratch[kStaticWorkFloats];

constexpr int kMaxDevices = 64;
static std::mutex g_static_work_mu;
static float *g_static_work[kMaxDevices];

// Device address of this device's copy of `scratch` (the current device), looked up on the
// first call on that device; nullptr (with the error set) if HIP fails.
static float *static_work_ptr() {
    int dev = -1;
    if (check_hip(hipGetDevice(&dev), "hipGetDevice")) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d devices the static workspace serves", dev, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_static_work_mu);
    if (!g_static_work[dev]) {
        void *ptr = nullptr;
        if (check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return nullptr;
        g_static_work[dev] = (float *)ptr;
    }
    return g_static_work[dev];
}

}  // namespace amr

using namespace amr;

extern "C" {

int64_t amr_backward_static_bytes(void) { return (int64_t)sizeof(scratch); }

int amr_render_backward_static(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
                               const float *d_grad_rgba, float *d_grad_lut, float *d_grad_light, int32_t deterministic,
                               void *stream) {
    const int64_t need = amr_backward_work_bytes(deterministic);
    if (need > (int64_t)sizeof(scratch)) {
        set_error("the adjoint needs %lld workspace bytes, more than the %lld of the static workspace", (long long)need,
                  (long long)sizeof(scratch));
        return AMR_ECAPACITY;
    }
    float *work = static_work_ptr();
    if (!work) return AMR_EHIP;
    return backward_launch(S, cams, ncams, P, d_grad_rgba, d_grad_lut, d_grad_light, deterministic, work, stream);
}

int64_t amr_sched_bytes(const amr_camera *cams, int32_t ncams) {
    if (!cams || ncams <= 0) return -1;
    int64_t ntot = 0;
    for (int c = 0; c < ncams; c++) {
        if (cams[c].width <= 0 || cams[c].height <= 0) return -1;
        ntot += sched_tiles(cams[c]);
    }
    return 4 * (sched_header_words(ncams) + 2 * ntot);
}

int64_t amr_tape_bytes(int64_t nrays, int64_t tape_cap) {
    if (nrays < 0 || tape_cap < 0) return 0;
    return nrays * tape_cap * (int64_t)sizeof(float4);
}

int64_t amr_ckpt_bytes(int64_t nrays, int32_t ckpt_max) {
    if (nrays < 0 || ckpt_max < 2) return 0;
    return nrays * (int64_t)sizeof(Ckpt) * (1 + (int64_t)ckpt_max);
}

int64_t amr_render_work_bytes(const amr_camera *cams, int32_t ncams, const amr_render_params *P) {
    if (!cams || !P || ncams <= 0 || P->light_jobs < 0) return -1;
    if (P->lighting != 2) return 0;
    int64_t npix = 0;
    for (int c = 0; c < ncams; c++) npix = std::max<int64_t>(npix, (int64_t)cams[c].width * cams[c].height);
    return shadow_work_bytes(npix, P->light_jobs);
}

int amr_render(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
               float *d_rgba, amr_render_stats *d_stats, void *stream) {
    if (!S || !cams || !P || !d_rgba || ncams <= 0) { set_error("null argument or ncams <= 0"); return AMR_EINVAL; }
    if (!S->pool || !S->nodes || !S->leaves || !S->patches) { set_error("scene not packed"); return AMR_EINVAL; }
    if (P->d_trace && P->trace_cap <= 0) { set_error("trace_cap must be positive with d_trace"); return AMR_EINVAL; }
    int64_t total = 0;
    for (int c = 0; c < ncams; c++) total += (int64_t)cams[c].width * cams[c].height;
    if (P->d_ckpt) {
        if (P->ckpt_max < 2 || (P->ckpt_max & 1) || P->ckpt_every < 1) {
            set_error("checkpoints need an even ckpt_max >= 2 and ckpt_every >= 1");
            return AMR_EINVAL;
        }
        if (P->ckpt_bytes < amr_ckpt_bytes(total, P->ckpt_max)) {
            set_error("ckpt_bytes %lld < %lld", (long long)P->ckpt_bytes, (long long)amr_ckpt_bytes(total, P->ckpt_max));
            return AMR_ECAPACITY;
        }
        if (P->d_tape && (P->tape_cap < 0 || P->tape_cap > kTapeCapMax)) {
            set_error("tape_cap must lie in [0, %lld]", (long long)kTapeCapMax);
            return AMR_EINVAL;
        }
        if (P->d_tape && (reinterpret_cast<uintptr_t>(P->d_tape) & 15u)) {
            set_error("d_tape must be 16-byte aligned");
            return AMR_EINVAL;
        }
    }
    const bool learned = P->d_mlp || P->d_seglog || P->bound_only;
    if (P->d_sched) {
        if (P->persistent || learned || P->lighting == 2) {
            set_error("the tile schedule (d_sched) serves the raycaster's single-camera kernels only (not persistent "
                      "mode, learned proposals or the point light)");
            return AMR_EINVAL;
        }
        const int64_t need = amr_sched_bytes(cams, ncams);
        if (need < 0 || P->sched_bytes < need) {
            set_error("sched_bytes %lld < %lld", (long long)P->sched_bytes, (long long)need);
            return AMR_ECAPACITY;
        }
        if (reinterpret_cast<uintptr_t>(P->d_sched) & 3u) {
            set_error("d_sched must be 4-byte aligned");
            return AMR_EINVAL;
        }
        const int64_t sp = 8 * (int64_t)sched_side(P->lighting == 1);   // super-tile side in pixels
        for (int c = 0; c < ncams; c++) {      // an order entry holds the super-tile in 24 bits
            const int64_t nst = ((cams[c].width + sp - 1) / sp) * ((cams[c].height + sp - 1) / sp);
            if (nst >= ((int64_t)1 << 24)) {
                set_error("the tile schedule takes cameras of fewer than 2^24 super-tiles (16x16 pixels lit, "
                          "32x32 unlit)");
                return AMR_EINVAL;
            }
        }
    }
    if (P->d_mlp && (reinterpret_cast<uintptr_t>(P->d_mlp) & 15u)) {
        set_error("d_mlp must be 16-byte aligned");
        return AMR_EINVAL;
    }
    if (P->bound_only && P->d_mlp) {
        set_error("bound_only skips by the analytic bound alone: d_mlp must be NULL");
        return AMR_EINVAL;
    }
    if (P->lighting == 2 && (P->persistent || learned || P->d_ckpt || P->interp != 0 || P->lod > 0.f)) {
        set_error("point-light lighting (lighting = 2) is rendered by its own forward kernel only, with trilinear "
                  "sampling and no level of detail (not persistent, learned, logging or checkpointed)");
        return AMR_EINVAL;
    }
    if (P->interp == 1 && (P->persistent || learned || P->d_ckpt)) {
        set_error("nearest-cell sampling (interp = 1) is rendered by the plain forward kernel only "
                  "(not persistent, learned, logging or checkpointed)");
        return AMR_EINVAL;
    }
    if (P->persistent && learned) {
        set_error("learned proposals and segment logging run in their own kernel (not persistent)");
        return AMR_EINVAL;
    }
    if (P->persistent) return launch_persistent(S, cams, ncams, P, d_rgba, d_stats, stream);
    hipStream_t s = (hipStream_t)stream;
    if (d_stats) {
        int n = (int)(sizeof(amr_render_stats) / 8);
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)d_stats, n);
    }
    // learned proposals and the point light: one launch per camera
    if (learned || P->lighting == 2) {
        int64_t pix_off = 0;
        for (int c = 0; c < ncams; c++) {
            RenderArgs A;
            int rc = fill_args(S, &cams[c], P, &A);
            if (rc) return rc;
            A.rgba = d_rgba + 4 * pix_off;
            A.trace = P->d_trace ? P->d_trace + pix_off * P->trace_cap : nullptr;
            A.trace_cap = P->trace_cap;
            A.trace_n = P->d_trace_n ? P->d_trace_n + pix_off : nullptr;
            A.nsamp = P->d_nsamp ? P->d_nsamp + pix_off : nullptr;
            A.stats = d_stats;
            A.touch = P->d_touch;
            A.ckpt_ray0 = pix_off;
            if (learned) {
                if (P->d_trace || P->d_ckpt || P->d_touch || P->d_touch_meta) {
                    set_error("learned proposals / segment logging do not record traces, checkpoints or touch maps");
                    return AMR_EINVAL;
                }
                rc = launch_learned(A, P, S->lmax, stream, c == 0);
            } else {
                const bool rec = A.trace || A.trace_n || A.nsamp || A.stats || A.touch || A.touch_meta || A.ckpt;
                rc = launch_shadow(A, rec, stream, P->d_work, P->work_bytes, P->light_jobs);
            }
            if (rc) return rc;
            pix_off += (int64_t)cams[c].width * cams[c].height;
        }
        return AMR_OK;
    }
    // the raycaster: up to kCamGroup cameras per launch (blockIdx.y picks the camera), so that
    // the blocks of several images share the GPU and one image's last blocks do not leave it idle
    uint32_t *sched = (uint32_t *)P->d_sched;
    int64_t sched_ntot = 0;
    for (int c = 0; c < ncams; c++) sched_ntot += sched_tiles(cams[c]);
    uint32_t *sched_time = sched ? sched + sched_header_words(ncams) : nullptr;
    uint32_t *sched_order = sched ? sched_time + sched_ntot : nullptr;
    // the key of an order: FNV-1a over the super-tile side, the call's camera count and every
    // camera's tile grid, then the group's first camera (0 is left for a zeroed schedule)
    const uint32_t side = sched_side(P->lighting == 1);
    uint32_t list_sig = (((2166136261u ^ side) * 16777619u) ^ (uint32_t)ncams) * 16777619u;
    for (int c = 0; c < ncams; c++)
        for (uint32_t w : {(uint32_t)(cams[c].width + 7) / 8u, (uint32_t)(cams[c].height + 7) / 8u})
            list_sig = (list_sig ^ w) * 16777619u;
    int64_t pix_off = 0, tile_off = 0;
    for (int c0 = 0; c0 < ncams; c0 += kCamGroup) {
        const int n = std::min(kCamGroup, ncams - c0);
        RenderArgs A;
        CamGroup G;
        memset(&G, 0, sizeof(G));
        SchedGroup SG;
        memset(&SG, 0, sizeof(SG));
        int gx = 0;
        int64_t rel = 0;
        const int64_t order0 = tile_off;
        uint32_t nst = 0;
        for (int i = 0; i < n; i++) {
            RenderArgs Ai;
            int rc = fill_args(S, &cams[c0 + i], P, &Ai);
            if (rc) return rc;
            Ai.tile0 = tile_off;
            Ai.cam = c0 + i;
            if (i == 0) A = Ai;
            G.cam[i] = cam_args_of(Ai, rel);
            gx = std::max(gx, 8 * ((Ai.sgrid * Ai.sgrid + 7) / 8) * 16);
            SG.tile0[i] = tile_off;
            SG.t8x[i] = Ai.t8x;
            SG.t8y[i] = Ai.t8y;
            SG.stpre[i] = G.stpre[i] = nst;
            nst += (((uint32_t)Ai.t8x + side - 1u) / side) * (((uint32_t)Ai.t8y + side - 1u) / side);
            rel += (int64_t)cams[c0 + i].width * cams[c0 + i].height;
            tile_off += sched_tiles(cams[c0 + i]);
        }
        SG.stpre[n] = G.stpre[n] = nst;
        uint32_t sig = (list_sig ^ (uint32_t)c0) * 16777619u;
        if (sig == 0u) sig = 1u;
        G.n = n > 1 ? n : 0;
        if (sched) {
            G.sched = 1;
            G.nst = nst;
            G.sig = sig;
            G.cam0 = c0;
            G.order0 = order0;
            SG.n = n;
            SG.cam0 = c0;
            SG.sig = sig;
            SG.order0 = order0;
            SG.list_sig = list_sig;
            SG.ncams = ncams;
            SG.side = side;
        }
        A.sched_hdr = sched;
        A.sched_time = sched_time;
        A.sched_order = sched_order;
        A.rgba = d_rgba + 4 * pix_off;
        A.trace = P->d_trace ? P->d_trace + pix_off * P->trace_cap : nullptr;
        A.trace_cap = P->trace_cap;
        A.trace_n = P->d_trace_n ? P->d_trace_n + pix_off : nullptr;
        A.nsamp = P->d_nsamp ? P->d_nsamp + pix_off : nullptr;
        A.stats = d_stats;
        A.touch = P->d_touch;
        A.ckpt_ray0 = pix_off;
        const bool rec = A.trace || A.trace_n || A.nsamp || A.stats || A.touch || A.touch_meta || A.ckpt;
        // scheduled: one-dimensional, 16 blocks per super-tile, ranks dealt to the 8 XCDs in turn
        const dim3 g(sched ? 8 * side * side * ((nst + 7) / 8) : gx, sched ? 1 : n), b(64);
        if (A.nearest) {
            if (A.lighting) {
                if (rec) hipLaunchKernelGGL((render_fwd<true, true, true, -1>), g, b, 0, s, A, G);
                else hipLaunchKernelGGL((render_fwd<true, false, true, -1>), g, b, 0, s, A, G);
            } else {
                if (rec) hipLaunchKernelGGL((render_fwd<false, true, true, -1>), g, b, 0, s, A, G);
                else hipLaunchKernelGGL((render_fwd<false, false, true, -1>), g, b, 0, s, A, G);
            }
        } else if (rec && !(A.ckpt && !A.trace && !A.trace_n && !A.nsamp && !A.stats && !A.touch && !A.touch_meta)) {
            if (A.lighting) hipLaunchKernelGGL((render_fwd<true, true, false, -1>), g, b, 0, s, A, G);
            else hipLaunchKernelGGL((render_fwd<false, true, false, -1>), g, b, 0, s, A, G);
        } else if (A.ckpt) {       // checkpoints (and the tape) only: the adjoint's forward pass
            if (A.lighting) {
                if (A.layout == 0) hipLaunchKernelGGL((render_fwd<true, false, false, 0, true>), g, b, 0, s, A, G);
                else if (A.layout == 1) hipLaunchKernelGGL((render_fwd<true, false, false, 1, true>), g, b, 0, s, A, G);
                else hipLaunchKernelGGL((render_fwd<true, false, false, 2, true>), g, b, 0, s, A, G);
            } else {
                if (A.layout == 0) hipLaunchKernelGGL((render_fwd<false, false, false, 0, true>), g, b, 0, s, A, G);
                else if (A.layout == 1) hipLaunchKernelGGL((render_fwd<false, false, false, 1, true>), g, b, 0, s, A, G);
                else hipLaunchKernelGGL((render_fwd<false, false, false, 2, true>), g, b, 0, s, A, G);
            }
        } else if (A.lighting) {   // the timed variants, one per brick layout
            if (A.layout == 0) hipLaunchKernelGGL((render_fwd<true, false, false, 0>), g, b, 0, s, A, G);
            else if (A.layout == 1) hipLaunchKernelGGL((render_fwd<true, false, false, 1>), g, b, 0, s, A, G);
            else hipLaunchKernelGGL((render_fwd<true, false, false, 2>), g, b, 0, s, A, G);
        } else {
            if (A.layout == 0) hipLaunchKernelGGL((render_fwd<false, false, false, 0>), g, b, 0, s, A, G);
            else if (A.layout == 1) hipLaunchKernelGGL((render_fwd<false, false, false, 1>), g, b, 0, s, A, G);
            else hipLaunchKernelGGL((render_fwd<false, false, false, 2>), g, b, 0, s, A, G);
        }
        int rc = check_hip(hipGetLastError(), "render_fwd launch");
        if (rc) return rc;
        if (sched) {
            hipLaunchKernelGGL(sched_sort, dim3(1), dim3(1024), 0, s, sched, sched_time, sched_order, SG);
            rc = check_hip(hipGetLastError(), "tile schedule sort");
            if (rc) return rc;
        }
        pix_off += rel;
    }
    return AMR_OK;
}

int64_t amr_backward_work_bytes(int32_t deterministic) {
    return (int64_t)sizeof(float) * ((int64_t)kGradLen + (deterministic ? (int64_t)kBwdGrid * kGradLen : 0));
}

int amr_render_backward(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
                        const float *d_grad_rgba, float *d_grad_lut, float *d_grad_light, int32_t deterministic,
                        void *stream) {
    if (P && !P->d_work) {
        set_error("amr_render_backward needs a workspace: params.d_work of amr_backward_work_bytes(deterministic) bytes");
        return AMR_EINVAL;
    }
    if (P && P->work_bytes < amr_backward_work_bytes(deterministic)) {
        set_error("work_bytes %lld < %lld", (long long)P->work_bytes, (long long)amr_backward_work_bytes(deterministic));
        return AMR_ECAPACITY;
    }
    return backward_launch(S, cams, ncams, P, d_grad_rgba, d_grad_lut, d_grad_light, deterministic,
                           P ? (float *)P->d_work : nullptr, stream);
}

}  // extern "C"
