// Measurement probe (not a step of the method): sustained read bandwidth of the cache level a
// buffer fits in, for the rooflines the frame time is compared with.  A buffer of a few MB per
// XCD stays in the XCD's L2 across repetitions while each CU's share exceeds its L1, so the
// rate measured is the L2's; a buffer far larger than the L2s and the MALL measures HBM.
#include <hip/hip_runtime.h>

#include "amr_internal.h"

namespace amr {

// Every block reads the same float4 elements in every repetition (a fixed grid striding over
// the buffer), so each XCD keeps its blocks' share cached; an empty asm statement with a memory
// clobber between repetitions makes the compiler load again.  The sum is written only under a
// condition the data never meets, which keeps the loads without storing anything.
__global__ __launch_bounds__(256) void read_probe(const float4 *buf, int64_t n4, int reps, float *sink) {
    float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int r = 0; r < reps; r++) {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
            const float4 v = buf[i];
            ax += v.x;
            ay += v.y;
            az += v.z;
            aw += v.w;
        }
        __asm__ volatile("" ::: "memory");   // each repetition reads the buffer again
    }
    const float s = (ax + ay) + (az + aw);
    if (s == -1.f) sink[0] = s;   // the probe's buffers hold non-negative values
}

}  // namespace amr

extern "C" int amr_probe_read(const void *d_buf, int64_t bytes, int32_t reps, int32_t blocks, float *d_sink,
                              void *stream) {
    if (!d_buf || !d_sink || bytes < 16 || reps < 1 || blocks < 1) {
        amr::set_error("amr_probe_read: null buffer, fewer than 16 bytes, or reps/blocks < 1");
        return AMR_EINVAL;
    }
    hipLaunchKernelGGL(amr::read_probe, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)d_buf,
                       bytes / 16, reps, d_sink);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        amr::set_error("read_probe launch: %s", hipGetErrorString(e));
        return AMR_EHIP;
    }
    return AMR_OK;
}
