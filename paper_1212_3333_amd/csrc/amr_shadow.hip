// Point-light secondary rays (lighting = 2): the paper's global-illumination example traces,
// from every sampling location, a secondary ray to a central point-like light source
// (Section 6, Figure 5).  Here each primary sample is shaded by k_a + k_d T_L(x), where T_L is
// the transmittance of the segment from x to the light inside B, sampled with the primary rule
// (kD-restart segments, midpoints, step proportional to each leaf level's cell size).
//
// The secondary rays are not marched inside the primary sample loop: there a wave holds one
// shadow ray per pixel, lanes finish at very different times and a small image leaves most of
// the machine idle.  Instead the render runs as passes over the same primary march (whose
// samples and early termination do not depend on the shading):
//   1. count the samples of every ray; an exclusive scan gives each ray its first job;
//   2. record the ray parameter of every sample as a job;
//   3. trace every job's shadow ray, one per lane: consecutive lanes hold consecutive samples of
//      a ray, whose shadow rays run side by side to the light;
//   4. march again and composite with the stored transmittances.
// The per-ray counts and offsets and the job arrays (16 bytes per sample) live in the caller's
// workspace; a sample whose job does not fit traces its secondary ray in the shading pass, so
// the image never depends on the workspace's size.  Nothing is read back to the host: the job
// count stays on the device and bounds the secondary-ray pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "amr_render_common.h"

namespace amr {

// exp(-integral of sigma) from world point x to the light, over the part of the segment in B.
template <int LAY>
__device__ __forceinline__ float light_transmittance(const RenderArgs &A, const float4 *s_lut, const double x[3]) {
#pragma clang fp contract(off)
    double v[3];
    #pragma unroll
    for (int a = 0; a < 3; a++) v[a] = A.plight[a] - x[a];
    double dist2 = v[0] * v[0] + v[1] * v[1];
    dist2 = dist2 + v[2] * v[2];
    const double dist = sqrt(dist2);
    if (!(dist > 0.0)) return 1.f;
    Ray Q;
    double lo_t = 0.0, hi_t = dist;
    #pragma unroll
    for (int a = 0; a < 3; a++) {
        Q.o[a] = x[a];
        Q.d[a] = v[a] / dist;
        const double lo = A.box_lo[a], hi = A.box_hi[a];
        if (Q.d[a] == 0.0) {
            Q.invd[a] = 0.0;
            if (!(x[a] >= lo && x[a] < hi)) return 1.f;
            continue;
        }
        const double inv = 1.0 / Q.d[a];
        Q.invd[a] = inv;
        const double ta = (lo - x[a]) * inv, tb = (hi - x[a]) * inv;
        const double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > lo_t) lo_t = tn;
        if (tf < hi_t) hi_t = tf;
    }
    if (!(hi_t > lo_t)) return 1.f;
    Q.t0 = lo_t;
    Q.t1 = hi_t;
    float tau = 0.f;                      // sum of sigma delta, in units of ln 2
    double tcur = lo_t;
    uint32_t start = 0;
    while (tcur < hi_t) {
        double tb = hi_t;
        const int leaf = descend(A, Q, tcur, tb, start);
        if (leaf < 0) break;
        const DLeaf &L = A.leaves[leaf];
        if (L.patch >= 0) {
            Segment S;
            setup_segment<false, LAY>(A, Q, L, leaf, tcur, tb, S);
            for (int j = 0; j < S.n; j++) {
                const float kk = (float)j + 0.5f;
                const float F = trilinear<false, LAY>(A, S.pv, S.q0[0] + kk * S.dq[0], S.q0[1] + kk * S.dq[1],
                                                 S.q0[2] + kk * S.dq[2]);
                const float u = __saturatef((F - A.v_lo) * A.inv_range);
                const float xs = 255.f * u;
                const int i0 = min((int)xs, 254);
                const float f = xs - (float)i0;
                tau += lerpf(s_lut[i0].w, s_lut[i0 + 1].w, f) * S.dl;
            }
        }
        if (tb <= tcur) tb = nextafter(tcur, INFINITY);
        tcur = tb;
    }
    return exp2f(-tau);
}

struct ShadowWork {
    int32_t *cnt;       // [npix] samples per ray (pass 1)
    int64_t *off;       // [npix] first job of each ray
    int64_t *total;     // [1] jobs of the frame (all samples), written by the scan
    double *tk;         // [cap] ray parameter of each sample
    int32_t *ray;       // [cap] the sample's ray
    float *tl;          // [cap] transmittance to the light
    int64_t cap;        // jobs the arrays hold
};

enum { kPassCount = 0, kPassRecord = 1, kPassShade = 2 };

// One march of the primary rays (one wave per 8x8 tile, tiles dealt to XCDs as in the forward
// kernel): PASS counts, records or shades the samples; the samples and the termination are the
// same in every pass.
template <int PASS, bool REC, int LAY>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void shadow_march(RenderArgs A, ShadowWork W) {
    __shared__ float4 s_lut[256];
    for (int i = threadIdx.x; i < 256; i += 64) s_lut[i] = A.lut[i];
    __syncthreads();
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
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    int nseg = 0, nsamp_total = 0;
    Ray R;
    bool alive = valid && setup_ray(A, pi, pj, R);
    if (REC) cnt.hit = alive ? 1 : 0;
    const int64_t base = (PASS != kPassCount && valid) ? W.off[ray] : 0;
    // the later passes stay inside this ray's jobs even if a sample count came out differently
    const int njob = (PASS != kPassCount && valid) ? W.cnt[ray] : 0;
    double tcur = R.t0;
    uint32_t start = 0;
    while (alive && tcur < R.t1) {
        double tb = R.t1;
        const int leaf = descend(A, R, tcur, tb, start);
        if (leaf < 0) break;
        if (REC) cnt.segments++;
        const DLeaf &L = A.leaves[leaf];
        int nsm = 0;
        if (L.patch >= 0) {
            Segment S;
            setup_segment<false, LAY>(A, R, L, leaf, tcur, tb, S);
            nsm = S.n;
            for (int k = 0; k < nsm; k++) {
                SampleVals v;
                eval_sample<false, REC, false, LAY>(A, s_lut, R, S, k, v, cnt);
                const bool job = nsamp_total < njob && base + nsamp_total < W.cap;
                if (PASS == kPassRecord && job) {
#pragma clang fp contract(off)
                    W.tk[base + nsamp_total] = S.ta + ((double)k + 0.5) * S.delta;
                    W.ray[base + nsamp_total] = (int32_t)ray;
                }
                if (PASS == kPassShade) {
                    float tl;
                    if (job) {
                        tl = W.tl[base + nsamp_total];
                    } else {
                        // no job slot: the secondary ray from the same FP64 sample position
#pragma clang fp contract(off)
                        const double tk = S.ta + ((double)k + 0.5) * S.delta;
                        double x[3];
                        #pragma unroll
                        for (int b = 0; b < 3; b++) x[b] = R.o[b] + tk * R.d[b];
                        tl = light_transmittance<LAY>(A, s_lut, x);
                        if (REC) cnt.linl++;
                    }
                    const float shade = A.k_a + A.k_d * tl;
                    const float wgt = T * v.alpha * shade;
                    C0 += wgt * v.r;
                    C1 += wgt * v.g;
                    C2 += wgt * v.b;
                }
                T *= 1.f - v.alpha;
                nsamp_total++;
                if (T < A.t_min) { alive = false; break; }
            }
        }
        if (REC && A.trace) {
            if (nseg < A.trace_cap) {
                amr_trace_rec rec;
                rec.leaf = leaf;
                rec.patch = L.patch;
                rec.n = L.patch >= 0 ? nsm : 0;
                rec.level = leaf_level(L);
                rec.ta = tcur;
                rec.tb = tb;
                A.trace[ray * A.trace_cap + nseg] = rec;
            } else {
                cnt.tover++;
            }
        }
        nseg++;
        if (tb <= tcur) {
            if (REC) cnt.guard++;
            tb = nextafter(tcur, INFINITY);
        }
        tcur = tb;
    }
    if (PASS == kPassCount && valid) W.cnt[ray] = nsamp_total;
    if (PASS == kPassShade && valid) {
        reinterpret_cast<float4 *>(A.rgba)[ray] = make_float4(C0, C1, C2, 1.f - T);
        if (REC && A.trace_n) A.trace_n[ray] = nseg;
        if (REC && A.nsamp) A.nsamp[ray] = nsamp_total;
    }
    if (REC) {
        cnt.samples = nsamp_total;
        if (A.stats) flush_counters(A.stats, cnt, lane);
    }
}

// Pass 3: one shadow ray per lane, from the recorded sample position to the light.  The grid
// covers the job arrays; lanes beyond the frame's job count (read on the device) return.
template <int LAY>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void shadow_rays(RenderArgs A, ShadowWork W) {
#pragma clang fp contract(off)
    const int64_t njobs = min(*W.total, W.cap);
    if ((int64_t)blockIdx.x * 64 >= njobs) return;
    __shared__ float4 s_lut[256];
    for (int i = threadIdx.x; i < 256; i += 64) s_lut[i] = A.lut[i];
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= njobs) return;
    const int r = W.ray[j];
    float tl = 1.f;
    if (r >= 0 && (int64_t)r < (int64_t)A.width * A.height) {   // every job below the count was recorded
        Ray R;
        setup_ray(A, r % A.width, r / A.width, R);   // a ray with samples, so it meets the clip box
        const double tk = W.tk[j];
        double x[3];
        #pragma unroll
        for (int b = 0; b < 3; b++) x[b] = R.o[b] + tk * R.d[b];
        tl = light_transmittance<LAY>(A, s_lut, x);
    }
    W.tl[j] = tl;
}

// Block-wise exclusive scan of the per-ray counts (1024 per block), then of the block sums.
__global__ __launch_bounds__(1024) void scan_counts(const int32_t *cnt, int64_t n, int64_t *off, int64_t *bsum) {
    __shared__ int64_t t[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int64_t v = i < n ? (int64_t)cnt[i] : 0;
    t[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d *= 2) {
        const int64_t add = threadIdx.x >= (unsigned)d ? t[threadIdx.x - d] : 0;
        __syncthreads();
        t[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < n) off[i] = t[threadIdx.x] - v;
    if (threadIdx.x == 1023) bsum[blockIdx.x] = t[1023];
}

__global__ __launch_bounds__(1024) void scan_block_sums(int64_t *bsum, int64_t nb, int64_t *total) {
    __shared__ int64_t t[1024];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        t[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d *= 2) {
            const int64_t add = threadIdx.x >= (unsigned)d ? t[threadIdx.x - d] : 0;
            __syncthreads();
            t[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + t[threadIdx.x] - v;
        carry += t[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(1024) void add_block_offsets(int64_t *off, int64_t n, const int64_t *bsum) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) off[i] += bsum[blockIdx.x];
}

template <int LAY>
static void launch_march(int pass, bool rec, int grid, hipStream_t s, const RenderArgs &A, const ShadowWork &W) {
    if (pass == kPassCount) hipLaunchKernelGGL((shadow_march<kPassCount, false, LAY>), dim3(grid), dim3(64), 0, s, A, W);
    else if (pass == kPassRecord) hipLaunchKernelGGL((shadow_march<kPassRecord, false, LAY>), dim3(grid), dim3(64), 0, s, A, W);
    else if (rec) hipLaunchKernelGGL((shadow_march<kPassShade, true, -1>), dim3(grid), dim3(64), 0, s, A, W);
    else hipLaunchKernelGGL((shadow_march<kPassShade, false, LAY>), dim3(grid), dim3(64), 0, s, A, W);
}

// Workspace of the point-light passes for npix rays and `jobs` job slots: counts, offsets,
// scan block sums and the job total, then the three job arrays, each 256-byte aligned.
static inline int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

int64_t shadow_work_bytes(int64_t npix, int64_t jobs) {
    const int64_t nb = (npix + 1023) / 1024;
    return align256(4 * npix) + align256(8 * npix) + align256(8 * nb) + 256 + align256(8 * jobs) + align256(4 * jobs) +
           align256(4 * jobs);
}

int launch_shadow(const RenderArgs &A, bool rec, void *stream, void *work, int64_t work_bytes, int64_t jobs) {
    hipStream_t s = (hipStream_t)stream;
    const int grid = 8 * ((A.sgrid * A.sgrid + 7) / 8) * 16;
    const int64_t npix = (int64_t)A.width * A.height;
    const int64_t nb = (npix + 1023) / 1024;
    if (!work || jobs < 0 || work_bytes < shadow_work_bytes(npix, jobs)) {
        set_error("point-light lighting needs a workspace of amr_render_work_bytes() bytes (params.d_work, "
                  "params.work_bytes, params.light_jobs)");
        return work ? AMR_ECAPACITY : AMR_EINVAL;
    }
    if ((jobs + 63) / 64 > 0x7fffffffLL) {
        set_error("light_jobs %lld exceeds one launch of the secondary-ray pass", (long long)jobs);
        return AMR_EINVAL;
    }
    RenderArgs Ap = A;                      // counting and recording passes record nothing else
    Ap.trace = nullptr;
    Ap.trace_n = nullptr;
    Ap.nsamp = nullptr;
    Ap.stats = nullptr;
    Ap.touch = nullptr;
    Ap.touch_meta = nullptr;
    char *p = (char *)work;
    ShadowWork W{};
    W.cnt = (int32_t *)p;
    p += align256(4 * npix);
    W.off = (int64_t *)p;
    p += align256(8 * npix);
    int64_t *bsum = (int64_t *)p;
    p += align256(8 * nb);
    W.total = (int64_t *)p;
    p += 256;
    W.tk = (double *)p;
    p += align256(8 * jobs);
    W.ray = (int32_t *)p;
    p += align256(4 * jobs);
    W.tl = (float *)p;
    W.cap = jobs;
    auto march = [&](int pass, const RenderArgs &Aa) {
        if (Aa.layout == 0) launch_march<0>(pass, rec, grid, s, Aa, W);
        else if (Aa.layout == 1) launch_march<1>(pass, rec, grid, s, Aa, W);
        else launch_march<2>(pass, rec, grid, s, Aa, W);
    };
    march(kPassCount, Ap);
    hipLaunchKernelGGL(scan_counts, dim3(nb), dim3(1024), 0, s, W.cnt, npix, W.off, bsum);
    hipLaunchKernelGGL(scan_block_sums, dim3(1), dim3(1024), 0, s, bsum, nb, W.total);
    hipLaunchKernelGGL(add_block_offsets, dim3(nb), dim3(1024), 0, s, W.off, npix, bsum);
    if (jobs > 0) {
        march(kPassRecord, Ap);
        const int64_t nj = (jobs + 63) / 64;
        if (A.layout == 0) hipLaunchKernelGGL((shadow_rays<0>), dim3(nj), dim3(64), 0, s, Ap, W);
        else if (A.layout == 1) hipLaunchKernelGGL((shadow_rays<1>), dim3(nj), dim3(64), 0, s, Ap, W);
        else hipLaunchKernelGGL((shadow_rays<2>), dim3(nj), dim3(64), 0, s, Ap, W);
    }
    march(kPassShade, A);
    return check_hip(hipGetLastError(), "point-light passes");
}

}  // namespace amr
