// Persistent multi-camera raycasting: one launch renders many cameras of different sizes.
//
// Work unit: a 64-pixel tile (tile_w x tile_h) rendered by one wave, one ray per lane, with
// the per-ray code of the single-camera kernel.  Waves take tiles from one global atomic
// queue that lists the cameras largest first, so the short images of a batch fill the tail of
// the long ones.  The wave that finishes an image's last tile writes the device clock into
// stamps[camera]; the wave that takes tile 0 writes stamps[ncams] (launch start).  Everything
// the launch needs (queue reset, camera order, tile prefix sums) is computed on the device
// from the device camera table, so the sequence can be captured in a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include "amr_render_common.h"

namespace amr {

// Queue scratch layout (amr_queue_bytes): counters first, then per-camera tables.  There are
// kQueues tile queues: with XCD-aware tiles, queue x serves the waves of blocks x, x + 8, ...
// (the hardware deals blocks to the 8 XCDs in turn) and lists, image by image, the 4x4-tile
// super-tiles x, x + 8, x + 16, ... of each image along a Morton curve, as the single-camera
// kernel deals them; otherwise queue 0 lists every image's tiles row by row.
constexpr int kQueues = 8;

struct QueueView {
    unsigned int *next;          // [kQueues] next tile of each queue, 64 bytes apart
    unsigned int *done;          // [ncams] tiles finished per camera
    unsigned int *ntiles;        // [ncams] tiles of each camera over all queues
    int *order;                  // [ncams] cameras in queue order
    long long *tile0;            // [kQueues][ncams + 1] first tile of the k-th camera in `order`
    long long *pix0;             // [ncams] first pixel of camera c in the rgba output
    int *tiles_x, *tiles_y;      // [ncams]
    int *sgrid;                  // [ncams] side of the power-of-two super-tile grid
};

__host__ __device__ __forceinline__ int64_t q_align(int64_t b) { return (b + 255) / 256 * 256; }

__host__ __device__ __forceinline__ QueueView queue_view(void *base, int ncams) {
    char *p = (char *)base;
    QueueView q;
    q.next = (unsigned int *)p;
    p += 64 * kQueues;
    q.done = (unsigned int *)p;
    p += q_align(4 * (int64_t)ncams);
    q.ntiles = (unsigned int *)p;
    p += q_align(4 * (int64_t)ncams);
    q.order = (int *)p;
    p += q_align(4 * (int64_t)ncams);
    q.tile0 = (long long *)p;
    p += q_align(8 * (int64_t)kQueues * (ncams + 1));
    q.pix0 = (long long *)p;
    p += q_align(8 * (int64_t)ncams);
    q.tiles_x = (int *)p;
    p += q_align(4 * (int64_t)ncams);
    q.tiles_y = (int *)p;
    p += q_align(4 * (int64_t)ncams);
    q.sgrid = (int *)p;
    return q;
}

inline int64_t queue_bytes(int ncams) {
    return 64 * kQueues + 3 * q_align(4 * (int64_t)ncams) + q_align(8 * (int64_t)kQueues * (ncams + 1)) +
           q_align(8 * (int64_t)ncams) + 3 * q_align(4 * (int64_t)ncams);
}

// One thread: reset the queues, order the cameras by pixel count (largest first, or smallest
// first with `smallest`; ties by index) and build the tile and pixel prefix tables.
__global__ void queue_setup(const amr_camera *cams, int ncams, void *qbase, int tw, int th,
                            unsigned long long *stamps, int smallest, int xcd_tiles) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    QueueView q = queue_view(qbase, ncams);
    for (int x = 0; x < kQueues; x++) q.next[16 * x] = 0u;
    long long pix = 0;
    for (int c = 0; c < ncams; c++) {
        q.done[c] = 0u;
        q.order[c] = c;
        q.pix0[c] = pix;
        pix += (long long)cams[c].width * cams[c].height;
        q.tiles_x[c] = (cams[c].width + tw - 1) / tw;
        q.tiles_y[c] = (cams[c].height + th - 1) / th;
        int sg = 1;
        while (sg * 4 < q.tiles_x[c] || sg * 4 < q.tiles_y[c]) sg *= 2;
        q.sgrid[c] = sg;
        q.ntiles[c] = xcd_tiles ? (unsigned int)(16 * sg * sg) : (unsigned int)(q.tiles_x[c] * q.tiles_y[c]);
        if (stamps) stamps[c] = 0ull;
    }
    if (stamps) stamps[ncams] = 0ull;
    for (int i = 1; i < ncams; i++) {          // insertion sort by pixel count
        int c = q.order[i];
        long long sz = (long long)cams[c].width * cams[c].height;
        int j = i - 1;
        while (j >= 0) {
            const long long sj = (long long)cams[q.order[j]].width * cams[q.order[j]].height;
            if (!(smallest ? sj > sz : sj < sz)) break;
            q.order[j + 1] = q.order[j];
            j--;
        }
        q.order[j + 1] = c;
    }
    for (int x = 0; x < kQueues; x++) {
        long long t = 0;
        for (int k = 0; k < ncams; k++) {
            q.tile0[x * (ncams + 1) + k] = t;
            const int c = q.order[k];
            if (xcd_tiles) {
                const long long S = (long long)q.sgrid[c] * q.sgrid[c];      // super-tiles x, x + 8, ...
                t += x < S ? 16 * ((S - x + kQueues - 1) / kQueues) : 0;
            } else if (x == 0) {
                t += q.ntiles[c];
            }
        }
        q.tile0[x * (ncams + 1) + ncams] = t;
    }
}

struct BatchArgs {
    RenderArgs base;                 // scene, LUT and shading parameters; camera fields unused
    const amr_camera *cams;          // device camera table
    int ncams, tw, th, xcd_tiles;
    void *queue;
    unsigned long long *stamps;
};

__device__ __forceinline__ void set_camera(RenderArgs &A, const amr_camera &C) {
    for (int a = 0; a < 3; a++) {
        A.eye[a] = C.eye[a];
        A.u[a] = C.u[a];
        A.v[a] = C.v[a];
        A.w[a] = C.w[a];
    }
    A.tanf = C.tan_half_fov;
    A.win0 = C.win[0];
    A.win1 = C.win[1];
    A.ortho = C.ortho;
    A.width = C.width;
    A.height = C.height;
    A.lod_pix = C.ortho ? (2.0 * C.win[1]) / (double)C.height : (2.0 * C.tan_half_fov) / (double)C.height;
}

// LAY: the brick layout fixed at compile time (-1: read at run time, for the recording variants).
// WPS: waves per SIMD the register allocation must allow (the lit kernel: 3 fits 168 VGPRs and
// spills about 120 bytes per lane, 2 keeps everything in registers with a third fewer waves).
template <bool LIT, bool REC, int LAY, int WPS = 3>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPS))) void render_batched(BatchArgs B) {
    __shared__ float4 s_lut[256];
    TapQueue *tq = nullptr;                        // lit: one deferred-tap queue per wave
    if constexpr (LIT) tq = tap_queues<4>() + (threadIdx.x >> 6);
    s_lut[threadIdx.x] = B.base.lut[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    QueueView q = queue_view(B.queue, B.ncams);
    const int qx = B.xcd_tiles ? (int)(blockIdx.x % kQueues) : 0;   // this wave's queue
    const long long *tile0 = q.tile0 + (long long)qx * (B.ncams + 1);
    const long long total = tile0[B.ncams];
    Counters cnt;
    RenderArgs A = B.base;
    while (true) {
        unsigned int tile = 0;
        if (lane == 0) tile = atomicAdd(q.next + 16 * qx, 1u);
        tile = __shfl(tile, 0, 64);
        if ((long long)tile >= total) break;           // every wave leaves once its queue is empty
        if (tile == 0 && lane == 0 && B.stamps && qx == 0) B.stamps[B.ncams] = wall_clock64();
        int k = 0;                                     // camera slot: largest k with tile0[k] <= tile
        int lo = 0, hi = B.ncams - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (tile0[mid] <= (long long)tile) lo = mid;
            else hi = mid - 1;
        }
        k = lo;
        const int c = q.order[k];
        const amr_camera C = B.cams[c];
        set_camera(A, C);
        const long long local = (long long)tile - tile0[k];
        int tx, ty;
        if (B.xcd_tiles) {
            // super-tile qx + 8 (local / 16) along the Morton curve, tile local % 16 in it
            const long long st = qx + (long long)kQueues * (local / 16);
            const int sub = (int)(local % 16);
            int sx = 0, sy = 0;
            #pragma unroll
            for (int bit = 0; bit < 15; bit++) {
                sx |= (int)((st >> (2 * bit)) & 1) << bit;
                sy |= (int)((st >> (2 * bit + 1)) & 1) << bit;
            }
            tx = sx * 4 + (sub >> 2);
            ty = sy * 4 + (sub & 3);
        } else {
            const int txs = q.tiles_x[c];
            tx = (int)(local % txs);
            ty = (int)(local / txs);
        }
        const int pi = tx * B.tw + lane % B.tw;
        const int pj = ty * B.th + lane / B.tw;
        const bool valid = pi < C.width && pj < C.height;
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
        int nsamp_total = 0;
        Ray R;
        bool alive = valid && setup_ray(A, pi, pj, R);
        if (REC) cnt.hit += alive ? 1 : 0;
        if (LIT) tapq_init(*tq, lane);
        double tcur = R.t0;
        uint32_t start = 0;
        while (alive && tcur < R.t1) {
            double tb = R.t1;
            int leaf = descend(A, R, tcur, tb, start);
            if (leaf < 0) break;
            if (REC) cnt.segments++;
            const DLeaf &L = A.leaves[leaf];
            if (L.patch >= 0) {
                Segment S;
                setup_segment<LIT, LAY>(A, R, L, leaf, tcur, tb, S);
                if constexpr (!LIT && !REC) {
                    float tseg = 1.f;
                    bool stop;
                    nsamp_total += composite_unlit<LAY>(A, s_lut, R, S, T, C0, C1, C2, tseg, stop, cnt);
                    if (stop) alive = false;
                } else if constexpr (LIT && !REC) {
                    // as the single-camera kernel: the stencils of a lane's next two samples are
                    // read together; after the first, the lanes still in this loop (each with a
                    // second sample) take it when the queue has a slot for those of them whose
                    // second sample defers, else they read it again in the next round
                    TapQueue &Q = *tq;
                    for (int k2 = 0; k2 < S.n;) {
                        tapq_reserve<REC, LAY>(A, s_lut, Q, lane, cnt);
                        const int kb = min(k2 + 1, S.n - 1);
                        const float kka = (float)k2 + 0.5f, kkb = (float)kb + 0.5f;
                        float qa[3], qb[3], Fa, Fpa[3], Fma[3], Fb, Fpb[3], Fmb[3];
                        #pragma unroll
                        for (int a = 0; a < 3; a++) {
                            qa[a] = S.q0[a] + kka * S.dq[a];
                            qb[a] = S.q0[a] + kkb * S.dq[a];
                        }
                        const uint32_t cla = lit_stencil<REC, LAY>(A, S, qa[0], qa[1], qa[2], Fa, Fpa, Fma);
                        const uint32_t clb = lit_stencil<REC, LAY>(A, S, qb[0], qb[1], qb[2], Fb, Fpb, Fmb);
                        float alpha = lit_consume<REC>(A, s_lut, Q, lane, R, S, k2, nullptr, qa[0], qa[1], qa[2], Fa,
                                                       Fpa, Fma, cla, pending_taps(cla), T, C0, C1, C2, cnt, nullptr,
                                                       nullptr);
                        T *= 1.f - alpha;
                        nsamp_total++;
                        k2++;
                        if (T < A.t_min) { alive = false; break; }
                        if (k2 == S.n) break;
                        const unsigned long long needb = __ballot(pending_taps(clb) != 0u);
                        if (tapq_full(tq_count(Q), needb)) continue;
                        alpha = lit_consume<REC>(A, s_lut, Q, lane, R, S, k2, nullptr, qb[0], qb[1], qb[2], Fb, Fpb,
                                                 Fmb, clb, pending_taps(clb), T, C0, C1, C2, cnt, nullptr, nullptr);
                        T *= 1.f - alpha;
                        nsamp_total++;
                        k2++;
                        if (T < A.t_min) { alive = false; break; }
                    }
                } else {
                    for (int k2 = 0; k2 < S.n; k2++) {
                        float alpha;
                        if (LIT) {
                            // as the single-camera kernel: taps that leave the brick are deferred
                            TapQueue &Q = *tq;
                            tapq_reserve<REC, LAY>(A, s_lut, Q, lane, cnt);
                            alpha = lit_sample_deferred<REC, LAY>(A, s_lut, Q, lane, R, S, k2, T, C0, C1, C2, cnt);
                        } else {
                            SampleVals v;
                            eval_sample<false, REC, false, LAY>(A, s_lut, R, S, k2, v, cnt);
                            float wgt = T * v.alpha * v.shade;
                            C0 += wgt * v.r;
                            C1 += wgt * v.g;
                            C2 += wgt * v.b;
                            alpha = v.alpha;
                        }
                        T *= 1.f - alpha;
                        nsamp_total++;
                        if (T < A.t_min) { alive = false; break; }
                    }
                }
            }
            if (tb <= tcur) {
                if (REC) cnt.guard++;
                tb = nextafter(tcur, INFINITY);
            }
            tcur = tb;
        }
        if (LIT) {
            float D0, D1, D2;
            tapq_finish<REC, LAY>(A, s_lut, *tq, lane, cnt, D0, D1, D2);
            C0 += D0;
            C1 += D1;
            C2 += D2;
        }
        if (REC) cnt.samples += nsamp_total;
        if (valid) reinterpret_cast<float4 *>(B.base.rgba)[q.pix0[c] + (long long)pj * C.width + pi] =
            make_float4(C0, C1, C2, 1.f - T);
        // completion: the wave that finishes the image's last tile stamps it
        __threadfence();
        if (lane == 0) {
            unsigned int d = atomicAdd(&q.done[c], 1u) + 1u;
            if (d == q.ntiles[c] && B.stamps) B.stamps[c] = wall_clock64();
        }
    }
    if (REC && B.base.stats) flush_counters(B.base.stats, cnt, lane);
}

__global__ void zero_stats(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Compute units of the current device (queried once per device).
static int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        cached[dev] = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0 ? n : 256;
    }
    return cached[dev];
}

int launch_persistent(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
                      float *d_rgba, amr_render_stats *d_stats, void *stream) {
    if (!P->d_queue || !P->d_cams) {
        set_error("persistent mode needs params.d_queue (amr_queue_bytes) and params.d_cams (device cameras)");
        return AMR_EINVAL;
    }
    if (P->d_trace || P->d_ckpt || P->d_nsamp || P->d_touch || P->d_touch_meta) {
        set_error("persistent mode renders images only (no trace, checkpoints, sample counts or touch map)");
        return AMR_EINVAL;
    }
    int tw = P->tile_w > 0 ? P->tile_w : 8, th = P->tile_h > 0 ? P->tile_h : 8;
    if (tw * th != 64) { set_error("tile_w * tile_h must be 64 (one wave)"); return AMR_EINVAL; }
    BatchArgs B;
    int rc = fill_args(S, &cams[0], P, &B.base);   // scene/LUT/shading; camera fields come per tile
    if (rc) return rc;
    for (int c = 0; c < ncams; c++)
        if (cams[c].width <= 0 || cams[c].height <= 0) { set_error("camera %d has no pixels", c); return AMR_EINVAL; }
    B.base.rgba = d_rgba;
    B.base.stats = d_stats;
    B.cams = P->d_cams;
    B.ncams = ncams;
    B.tw = tw;
    B.th = th;
    B.queue = P->d_queue;
    B.stamps = P->d_stamps;
    if (P->queue_order < 0 || P->queue_order > 1 || P->xcd_tiles < 0 || P->xcd_tiles > 1) {
        set_error("queue_order and xcd_tiles must be 0 or 1");
        return AMR_EINVAL;
    }
    if (P->waves_per_simd != 0 && P->waves_per_simd != 2 && P->waves_per_simd != 3) {
        set_error("waves_per_simd must be 0 (default 3), 2 or 3");
        return AMR_EINVAL;
    }
    const bool two = P->waves_per_simd == 2;
    B.xcd_tiles = P->xcd_tiles;
    hipStream_t s = (hipStream_t)stream;
    if (d_stats)
        hipLaunchKernelGGL(zero_stats, dim3(1), dim3(64), 0, s, (unsigned long long *)d_stats,
                           (int)(sizeof(amr_render_stats) / 8));
    hipLaunchKernelGGL(queue_setup, dim3(1), dim3(64), 0, s, P->d_cams, ncams, P->d_queue, tw, th, P->d_stamps,
                       (int)P->queue_order, (int)P->xcd_tiles);
    int bpc = P->blocks_per_cu > 0 ? P->blocks_per_cu : 4;
    dim3 grid(device_cus() * bpc);
    const bool rec = d_stats != nullptr;
    if (B.base.lighting) {
        if (rec) hipLaunchKernelGGL((render_batched<true, true, -1>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 0 && two) hipLaunchKernelGGL((render_batched<true, false, 0, 2>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 0) hipLaunchKernelGGL((render_batched<true, false, 0>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 1 && two) hipLaunchKernelGGL((render_batched<true, false, 1, 2>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 1) hipLaunchKernelGGL((render_batched<true, false, 1>), grid, dim3(256), 0, s, B);
        else if (two) hipLaunchKernelGGL((render_batched<true, false, 2, 2>), grid, dim3(256), 0, s, B);
        else hipLaunchKernelGGL((render_batched<true, false, 2>), grid, dim3(256), 0, s, B);
    } else {
        if (rec) hipLaunchKernelGGL((render_batched<false, true, -1>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 0) hipLaunchKernelGGL((render_batched<false, false, 0>), grid, dim3(256), 0, s, B);
        else if (B.base.layout == 1) hipLaunchKernelGGL((render_batched<false, false, 1>), grid, dim3(256), 0, s, B);
        else hipLaunchKernelGGL((render_batched<false, false, 2>), grid, dim3(256), 0, s, B);
    }
    return check_hip(hipGetLastError(), "render_batched launch");
}

}  // namespace amr

extern "C" int64_t amr_queue_bytes(int32_t ncams) { return ncams > 0 ? amr::queue_bytes(ncams) : 0; }

extern "C" int64_t amr_wall_clock_khz(void) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return khz;
}
