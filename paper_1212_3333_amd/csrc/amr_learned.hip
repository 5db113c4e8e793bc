// Learned segment proposals (an addition to the paper's method) and the training-data logger.
//
// The outer loop is wave-uniform: in every round each live lane takes its next leaf segment
// (kD-restart), computes 12 features, and the wave decides per lane whether to
//   skip the segment        (B + T * alpha_hi < tau_e, where B sums T * alpha_hi over the ray's
//                            earlier skips, so the skipped opacity of a whole ray stays below
//                            tau_e),
//   sample it coarsely      (alpha_lo > 1 - tau_s: step h^l instead of step_frac h^l, then
//                            terminate the ray), or
//   sample it as the plain traversal does (the fallback).
// Every sample of the leaf lies in the leaf's value range, so the segment opacity is at most
// alpha_max = 1 - exp(-sigma_max L) with sigma_max the largest extinction of the LUT over that
// range; a lane whose bound already proves the skip needs no network (and with bound_only
// the network is never asked: the same kernel then shows what the network adds).  The network
// (12 -> 64 -> 64 -> 2, fp16 matrix cores, fp32 accumulation) predicts quantiles of the ratio
// alpha / alpha_max in [0, 1], so its error scales with the bound instead of being a fixed
// absolute error at the fp16 resolution; it runs on the 16-lane row tiles that hold
// undecided lanes.  With d_mlp == NULL and d_seglog set, the
// kernel renders plainly and logs (features, true segment opacity) for training.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "amr_mlp.h"
#include "amr_render_common.h"

namespace amr {

struct SeglogHeader {
    unsigned long long count;
    unsigned long long pad_[31];
};
static_assert(sizeof(SeglogHeader) == 256, "seglog header");

struct LearnArgs {
    const MlpLds *mlp;         // packed network, NULL: log-only mode
    float tau_e, tau_s;
    uint8_t *seglog;           // SeglogHeader then amr_seglog_rec[cap]
    int64_t seglog_cap;
    int32_t lmax;
};

struct LearnLds {               // every variant: the LUT and its extinction tables
    float4 lut[256];
    float bmax[16], bmin[16];  // extinction max/min per 16-entry bucket
    float prefix[257];         // prefix sums of extinction
};

struct __attribute__((aligned(16))) NetLds {   // the network variant: per-wave inference buffers
                                // (the weights, 12 KB read by every query, stay in global memory
                                // and the caches)
    _Float16 feat[64 * 16];
    _Float16 hid[16 * 64];     // layer 1 output, then layer 2 output in place
    float out[64 * 2];
};

// The block's network buffers; a variant that never calls this allocates no LDS for them.
__device__ __forceinline__ NetLds *net_lds() {
    __shared__ NetLds n;
    return &n;
}

// Extinction range [smin, smax] and mean over LUT entries [i0, i1] (bucket-conservative bounds).
__device__ __forceinline__ void sigma_range(const LearnLds &s, int i0, int i1, float &smin, float &smax, float &smean) {
    const int b0 = i0 >> 4, b1 = i1 >> 4;
    float mx = s.bmax[b0], mn = s.bmin[b0];
    for (int b = b0 + 1; b <= b1; b++) {
        mx = fmaxf(mx, s.bmax[b]);
        mn = fminf(mn, s.bmin[b]);
    }
    smax = mx;
    smin = mn;
    smean = (s.prefix[i1 + 1] - s.prefix[i0]) / (float)(i1 - i0 + 1);
}

// Wave-level inference for row tile rt (lanes 16 rt .. 16 rt + 15) of the wave's features.
__device__ __forceinline__ void infer_tile(NetLds &s, const MlpLds *__restrict__ w, int rt) {
    const int lane = threadIdx.x & 63, lr = lane & 15, lq = lane >> 4;
    const _Float16 *x16 = s.feat + rt * 16 * 16;
    _Float16 *hid = s.hid;
    half4 a = *reinterpret_cast<const half4 *>(x16 + lr * 16 + 4 * lq);
    #pragma unroll 1
    for (int ct = 0; ct < 4; ct++) {
        half4 b = *reinterpret_cast<const half4 *>(w->w1t + (ct * 16 + lr) * 16 + 4 * lq);
        float4v acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma_k16(a, b, acc);
        #pragma unroll
        for (int j = 0; j < 4; j++) hid[(4 * lq + j) * 64 + ct * 16 + lr] = (_Float16)fmaxf(acc[j] + w->b1[ct * 16 + lr], 0.f);
    }
    __builtin_amdgcn_wave_barrier();
    // layer 2: the A fragments of h1 are the same for every output block, so read them once and
    // overwrite the buffer with h2
    half8 a2[2];
    #pragma unroll
    for (int ks = 0; ks < 2; ks++) a2[ks] = *reinterpret_cast<const half8 *>(hid + lr * 64 + ks * 32 + 8 * lq);
    __builtin_amdgcn_wave_barrier();
    #pragma unroll 1
    for (int ct = 0; ct < 4; ct++) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
        #pragma unroll
        for (int ks = 0; ks < 2; ks++) {
            half8 b = *reinterpret_cast<const half8 *>(w->w2t + (ct * 16 + lr) * 64 + ks * 32 + 8 * lq);
            acc = mfma_k32(a2[ks], b, acc);
        }
        #pragma unroll
        for (int j = 0; j < 4; j++) hid[(4 * lq + j) * 64 + ct * 16 + lr] = (_Float16)fmaxf(acc[j] + w->b2[ct * 16 + lr], 0.f);
    }
    __builtin_amdgcn_wave_barrier();
    float4v acc = {0.f, 0.f, 0.f, 0.f};
    #pragma unroll
    for (int ks = 0; ks < 2; ks++) {
        half8 a3 = *reinterpret_cast<const half8 *>(hid + lr * 64 + ks * 32 + 8 * lq);
        half8 b = *reinterpret_cast<const half8 *>(w->w3t + lr * 64 + ks * 32 + 8 * lq);
        acc = mfma_k32(a3, b, acc);
    }
    if (lr < kOut) {
        #pragma unroll
        for (int j = 0; j < 4; j++)
            s.out[(rt * 16 + 4 * lq + j) * 2 + lr] = 1.f / (1.f + __expf(-(acc[j] + w->b3[lr])));
    }
    __builtin_amdgcn_wave_barrier();
}

enum { kModePlain = 0, kModeSkip = 1, kModeCoarse = 2 };
// Segments shorter than this are never worth a query: a query round costs the wave about as
// much as 30 unlit samples (measured on the deep-range view at 1024^2: with a threshold of 8
// the network removed 29% more samples than the bound alone but the frame took 10% longer).
constexpr int kNetMinSamples = 32;

// DEC: how data segments are decided: 0 all sampled plainly (logging), 1 skipped by the
// analytic bound alone, 2 the bound and then the network (G.mlp set).  LOG: segments are logged
// for training (G.seglog set).  LAY: the brick layout (-1: read at run time).
template <bool LIT, int DEC, bool LOG, int LAY>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LIT ? 2 : (LOG ? 4 : 5)))) void render_learned(RenderArgs A, LearnArgs G) {
    __shared__ LearnLds s;
    NetLds *sn = nullptr;
    for (int i = threadIdx.x; i < 256; i += 64) s.lut[i] = A.lut[i];
    if constexpr (DEC == 2) sn = net_lds();
    __syncthreads();
    if (threadIdx.x < 16) {
        float mx = -INFINITY, mn = INFINITY;
        for (int i = 0; i < 16; i++) {
            float v = s.lut[threadIdx.x * 16 + i].w;
            mx = fmaxf(mx, v);
            mn = fminf(mn, v);
        }
        s.bmax[threadIdx.x] = mx;
        s.bmin[threadIdx.x] = mn;
    }
    if (threadIdx.x == 32) {
        float acc = 0.f;
        s.prefix[0] = 0.f;
        for (int i = 0; i < 256; i++) { acc += s.lut[i].w; s.prefix[i + 1] = acc; }
    }
    __syncthreads();
    const float4 *s_lut = s.lut;

    // One wave per block and one 8x8 pixel tile per wave, tiles grouped in 4x4 super-tiles along
    // a Morton curve and dealt round-robin to the 8 XCDs, as in the plain forward kernel (a
    // wave's slot frees as soon as its rays end).
    const int xcd = (int)(blockIdx.x % 8), li = (int)(blockIdx.x / 8);
    const int sidx = (li >> 4) * 8 + xcd;
    int sx = 0, sy = 0;
    #pragma unroll
    for (int bit = 0; bit < 12; bit++) {
        sx |= ((sidx >> (2 * bit)) & 1) << bit;
        sy |= ((sidx >> (2 * bit + 1)) & 1) << bit;
    }
    const int col = sx * 4 + ((li & 15) >> 2), row = sy * 4 + (li & 3);
    if (col >= A.t8x || row >= A.t8y) return;
    const int lane = threadIdx.x & 63;
    const int pi = col * 8 + (lane & 7);
    const int pj = row * 8 + (lane >> 3);
    const bool valid = pi < A.width && pj < A.height;
    const int64_t ray = (int64_t)pj * A.width + pi;

    Counters cnt;
    unsigned int c_skip = 0, c_coarse = 0, c_net = 0;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    float budget = 0.f;                   // sum of T * alpha_hi over the segments skipped so far
    int nsamp_total = 0;
    Ray R;
    bool alive = valid && setup_ray(A, pi, pj, R);
    cnt.hit = alive ? 1 : 0;
    double tcur = R.t0;
    uint32_t start = 0;
    SeglogHeader *lh = reinterpret_cast<SeglogHeader *>(G.seglog);
    amr_seglog_rec *lrec = reinterpret_cast<amr_seglog_rec *>(G.seglog + sizeof(SeglogHeader));
    const float inv_lmax = 1.f / (float)(G.lmax > 0 ? G.lmax : 1);
    while (true) {
        const bool active = alive && tcur < R.t1;
        if (!__any(active)) break;
        double tb = R.t1;
        int leaf = -1;
        bool data = false;
        Segment S;
        float a_bound_hi = 1.f;           // analytic bound on the segment opacity
        float a_bound_lo = 0.f;           // and its analytic lower bound
        float a_use = 1.f;                // upper bound charged to the skip budget
        float len = 0.f, umin = 0.f, umax = 0.f, smin = 0.f, smax = 0.f, smean = 0.f;
        int nsm = 0;                      // the segment's plain sample count
        if (active) {
            leaf = descend(A, R, tcur, tb, start);
            if (leaf < 0) {
                alive = false;
            } else {
                cnt.segments++;
                const DLeaf &L = A.leaves[leaf];
                data = L.patch >= 0;
                if (data) {
                    // the full sampling state is set up after the decision, for segments sampled
                    nsm = segment_samples(A, A.patches[L.patch], tcur, tb);
                    len = (float)(tb - tcur);
                    umin = __saturatef((L.vmin - A.v_lo) * A.inv_range);
                    umax = __saturatef((L.vmax - A.v_lo) * A.inv_range);
                    const int i0 = min((int)(255.f * umin), 255);
                    const int i1 = min((int)ceilf(255.f * umax), 255);
                    sigma_range(s, i0, max(i0, i1), smin, smax, smean);
                    a_bound_hi = 1.f - __expf(-smax * 1.00001f * len);
                    a_bound_lo = 1.f - __expf(-smin * len);
                    a_use = a_bound_hi;
                }
            }
        }
        // the 12 features of a data segment (logged for training and fed to the network)
        auto features = [&](float *feat) {
            const DLeaf &L = A.leaves[leaf];
            const DPatch &P = A.patches[L.patch];
            feat[0] = (float)leaf_level(L) * inv_lmax;
            feat[1] = log2f(fmaxf(len / (float)P.step, 1e-3f)) * 0.125f;
            feat[2] = umin;
            feat[3] = umax;
            feat[4] = a_bound_hi;
            feat[5] = 1.f - __expf(-smean * len);
            feat[6] = a_bound_lo;
            feat[7] = (float)min(nsm, 256) * (1.f / 256.f);
            feat[8] = (float)fabs(R.d[0]);
            feat[9] = (float)fabs(R.d[1]);
            feat[10] = (float)fabs(R.d[2]);
            feat[11] = log2f((float)min(P.n[0], min(P.n[1], P.n[2]))) * (1.f / 6.f);
        };
        // decide: skip by the analytic bound, else ask the network (wave-level MFMA)
        int mode = kModePlain;
        if constexpr (DEC == 1) {
            if (data && budget + T * a_bound_hi < G.tau_e) {
                mode = kModeSkip;
                budget += T * a_bound_hi;
            }
        }
        if constexpr (DEC == 2) {
            NetLds &sw = *sn;
            const bool bound_skip = data && budget + T * a_bound_hi < G.tau_e;
            // the network is asked only where its answer can change the decision and skipping
            // pays for it: segments of at least kNetMinSamples samples whose bound did not
            // already decide and whose analytic lower bound still fits the budget (or whose
            // upper bound reaches the coarse threshold)
            const bool undecided = data && !bound_skip && nsm >= kNetMinSamples &&
                                   (budget + T * a_bound_lo < G.tau_e || a_bound_hi > 1.f - G.tau_s);
            if (undecided) c_net++;
            if (bound_skip) mode = kModeSkip;
            const unsigned long long need = __ballot(undecided);
            if (need) {
                float feat[kIn];
                #pragma unroll
                for (int j = 0; j < kIn; j++) feat[j] = 0.f;
                if (undecided) features(feat);
                #pragma unroll
                for (int j = 0; j < 16; j++) sw.feat[lane * 16 + j] = (_Float16)(j < kIn ? feat[j < kIn ? j : 0] : 0.f);
                __builtin_amdgcn_wave_barrier();
                #pragma unroll 1
                for (int rt = 0; rt < 4; rt++)
                    if ((need >> (16 * rt)) & 0xffffull) infer_tile(sw, G.mlp, rt);
                if (undecided) {
                    a_use = __saturatef(sw.out[lane * 2 + 1]) * a_bound_hi;
                    const float a_lo = __saturatef(sw.out[lane * 2]) * a_bound_hi;
                    if (budget + T * a_use < G.tau_e) mode = kModeSkip;
                    else if (a_lo > 1.f - G.tau_s) mode = kModeCoarse;
                }
            }
            if (mode == kModeSkip) budget += T * a_use;   // skipped opacity mass of this ray
        }
        float tseg = 1.f;
        const float t_in = T;
        bool full = true;
        if (data && mode != kModeSkip) {
            setup_segment<LIT, LAY>(A, R, A.leaves[leaf], leaf, tcur, tb, S, nsm);
            if (mode == kModeCoarse) {
                // one step per cell of the leaf's level, then the ray stops after this segment
#pragma clang fp contract(off)
                const DPatch &P = A.patches[S.patch];
                const double step = A.uniform_step ? A.step_fine : P.step;
                const double nn = ceil((tb - tcur) / step - 0x1p-20);
                S.n = nn < 1.0 ? 1 : (int)nn;
                S.delta = (tb - tcur) / (double)S.n;
                #pragma unroll
                for (int a = 0; a < 3; a++) S.dq[a] = (float)(S.delta * R.d[a] * P.inv_h[a]);
                S.dl = (float)S.delta * 1.44269504088896340736f;
                c_coarse++;
            }
            if constexpr (!LIT && !LOG) {
                bool stop;
                const int done = composite_unlit<LAY>(A, s_lut, R, S, T, C0, C1, C2, tseg, stop, cnt);
                nsamp_total += done;
                if (stop) { alive = false; full = done == S.n; }
            } else {
                for (int k = 0; k < S.n; k++) {
                    SampleVals v;
                    eval_sample<LIT, false, false, LAY>(A, s_lut, R, S, k, v, cnt);
                    float wgt = T * v.alpha * v.shade;
                    C0 += wgt * v.r;
                    C1 += wgt * v.g;
                    C2 += wgt * v.b;
                    T *= 1.f - v.alpha;
                    tseg *= 1.f - v.alpha;
                    nsamp_total++;
                    if (T < A.t_min) { alive = false; full = k + 1 == S.n; break; }
                }
            }
            if (mode == kModeCoarse) alive = false;
        } else if (data) {
            c_skip++;
        }
        // training log: every plainly sampled data segment
        if (LOG) {
            const bool want = data && mode == kModePlain;
            const unsigned long long mask = __ballot(want);
            if (mask) {
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(&lh->count, (unsigned long long)__popcll(mask));
                base = __shfl(base, 0, 64);
                if (want) {
                    const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
                    if (slot < (unsigned long long)G.seglog_cap) {
                        amr_seglog_rec r;
                        features(r.feat);
                        r.alpha_seg = 1.f - tseg;
                        r.t_in = full ? t_in : -t_in;
                        r.ray = (int32_t)ray;
                        r.n = S.n;
                        lrec[slot] = r;
                    }
                }
            }
        }
        if (active && leaf >= 0) {
            if (tb <= tcur) {
                cnt.guard++;
                tb = nextafter(tcur, INFINITY);
            }
            tcur = tb;
        }
    }
    if (valid) reinterpret_cast<float4 *>(A.rgba)[ray] = make_float4(C0, C1, C2, 1.f - T);
    if (A.nsamp && valid) A.nsamp[ray] = nsamp_total;
    if (A.stats) {
        cnt.samples = nsamp_total;
        flush_counters(A.stats, cnt, lane);
        typedef unsigned long long u64;
        u64 sk = wave_sum((u64)c_skip), co = wave_sum((u64)c_coarse), nn = wave_sum((u64)c_net);
        if (lane == 0) {
            if (sk) atomicAdd(&A.stats->skipped_segments, sk);
            if (co) atomicAdd(&A.stats->coarse_segments, co);
            if (nn) atomicAdd(&A.stats->net_segments, nn);
        }
    }
}

__global__ void seglog_reset(uint8_t *seglog) {
    if (threadIdx.x == 0 && blockIdx.x == 0) reinterpret_cast<SeglogHeader *>(seglog)->count = 0ull;
}

int launch_learned(const RenderArgs &A, const amr_render_params *P, int lmax, void *stream, bool first_camera) {
    LearnArgs G;
    G.mlp = (const MlpLds *)P->d_mlp;
    G.tau_e = P->tau_e;
    G.tau_s = P->tau_s;
    G.seglog = (uint8_t *)P->d_seglog;
    G.seglog_cap = P->d_seglog ? (P->seglog_cap - (int64_t)sizeof(SeglogHeader)) / (int64_t)sizeof(amr_seglog_rec) : 0;
    G.lmax = lmax;
    hipStream_t s = (hipStream_t)stream;
    if (G.seglog && first_camera) hipLaunchKernelGGL(seglog_reset, dim3(1), dim3(64), 0, s, G.seglog);
    const int grid = 8 * ((A.sgrid * A.sgrid + 7) / 8) * 16;
    const bool log = G.seglog != nullptr;
    const int dec = P->bound_only ? 1 : (G.mlp ? 2 : 0);
    const dim3 g(grid), b(64);
    // the timed forms (deciding, not logging) are compiled for the brick layout
    auto timed = [&](auto lit, auto decc) {
        constexpr bool L = decltype(lit)::value;
        constexpr int D = decltype(decc)::value;
        if (A.layout == 0) hipLaunchKernelGGL((render_learned<L, D, false, 0>), g, b, 0, s, A, G);
        else if (A.layout == 1) hipLaunchKernelGGL((render_learned<L, D, false, 1>), g, b, 0, s, A, G);
        else hipLaunchKernelGGL((render_learned<L, D, false, 2>), g, b, 0, s, A, G);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    using D1 = std::integral_constant<int, 1>;
    using D2 = std::integral_constant<int, 2>;
    if (A.lighting) {
        if (dec == 2 && log) hipLaunchKernelGGL((render_learned<true, 2, true, -1>), g, b, 0, s, A, G);
        else if (dec == 1 && log) hipLaunchKernelGGL((render_learned<true, 1, true, -1>), g, b, 0, s, A, G);
        else if (dec == 2) timed(T_{}, D2{});
        else if (dec == 1) timed(T_{}, D1{});
        else hipLaunchKernelGGL((render_learned<true, 0, true, -1>), g, b, 0, s, A, G);
    } else {
        if (dec == 2 && log) hipLaunchKernelGGL((render_learned<false, 2, true, -1>), g, b, 0, s, A, G);
        else if (dec == 1 && log) hipLaunchKernelGGL((render_learned<false, 1, true, -1>), g, b, 0, s, A, G);
        else if (dec == 2) timed(F_{}, D2{});
        else if (dec == 1) timed(F_{}, D1{});
        else hipLaunchKernelGGL((render_learned<false, 0, true, -1>), g, b, 0, s, A, G);
    }
    return check_hip(hipGetLastError(), "render_learned launch");
}

}  // namespace amr
