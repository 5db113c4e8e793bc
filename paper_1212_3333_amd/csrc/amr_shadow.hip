// Point-light secondary rays (lighting = 2): the paper's global-illumination example traces,
// from every sampling location, a secondary ray to a central point-like light source
// (Section 6, Figure 5).  Here each primary sample is shaded by k_a + k_d T_L(x), where T_L is
// the transmittance of the segment from x to the light inside B, sampled with the primary rule
// (kD-restart segments, midpoints, step proportional to each leaf level's cell size).
//
// One wave per block and one 8x8 pixel tile per wave, dealt to XCDs like the forward kernel.
// The secondary march runs inside the primary sample loop, so the cost is (primary samples) x
// (secondary samples); the images are for the workloads that need the lighting, not a timed path.
#include <hip/hip_runtime.h>

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

template <bool REC, int LAY>
__global__ __launch_bounds__(64) void render_shadow(RenderArgs A) {
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
                double x[3];
                {
#pragma clang fp contract(off)
                    const double tk = S.ta + ((double)k + 0.5) * S.delta;
                    #pragma unroll
                    for (int b = 0; b < 3; b++) x[b] = R.o[b] + tk * R.d[b];
                }
                const float shade = A.k_a + A.k_d * light_transmittance<LAY>(A, s_lut, x);
                const float wgt = T * v.alpha * shade;
                C0 += wgt * v.r;
                C1 += wgt * v.g;
                C2 += wgt * v.b;
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
    if (valid) {
        reinterpret_cast<float4 *>(A.rgba)[ray] = make_float4(C0, C1, C2, 1.f - T);
        if (REC && A.trace_n) A.trace_n[ray] = nseg;
        if (REC && A.nsamp) A.nsamp[ray] = nsamp_total;
    }
    if (REC) {
        cnt.samples = nsamp_total;
        if (A.stats) flush_counters(A.stats, cnt, lane);
    }
}

int launch_shadow(const RenderArgs &A, bool rec, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const int grid = 8 * ((A.sgrid * A.sgrid + 7) / 8) * 16;
    if (rec) hipLaunchKernelGGL((render_shadow<true, -1>), dim3(grid), dim3(64), 0, s, A);
    else if (A.layout == 0) hipLaunchKernelGGL((render_shadow<false, 0>), dim3(grid), dim3(64), 0, s, A);
    else if (A.layout == 1) hipLaunchKernelGGL((render_shadow<false, 1>), dim3(grid), dim3(64), 0, s, A);
    else hipLaunchKernelGGL((render_shadow<false, 2>), dim3(grid), dim3(64), 0, s, A);
    return check_hip(hipGetLastError(), "render_shadow launch");
}

}  // namespace amr
