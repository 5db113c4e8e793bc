// Layout of the segment-proposal network shared by its training kernels and the renderer.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "amr_internal.h"

namespace amr {

constexpr int kIn = AMR_MLP_IN, kHid = AMR_MLP_HID, kOut = AMR_MLP_OUT;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kOut;
constexpr int kParams = kOffB3 + kOut;
static_assert(kHid == 64 && kIn <= 16 && kOut <= 16, "tile shapes assume 64 hidden units");

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float4v __attribute__((ext_vector_type(4)));

// The two matrix-core shapes the network uses (fp16 operands, fp32 accumulation, wave64):
//   v_mfma_f32_16x16x16f16 (layer 1, K = 16): lane l holds A[l % 16][4 (l / 16) + j] and
//     B[4 (l / 16) + j][l % 16], j = 0..3;
//   v_mfma_f32_16x16x32_f16 (gfx950; the K = 64 products in two steps): lane l holds
//     A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7.
// Both return D[4 (l / 16) + j][l % 16], j = 0..3, in lane l.
__device__ __forceinline__ float4v mfma_k16(half4 a, half4 b, float4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ float4v mfma_k32(half8 a, half8 b, float4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// fp16 operand copies of the weights (MFMA-friendly layouts) and fp32 biases.  This is also
// the packed inference format (amr_mlp_pack) that the renderer copies into LDS.
struct __attribute__((aligned(16))) MlpLds {
    _Float16 w1t[64 * 16];   // [u][i]  = W1[i][u], i >= 12 zero
    _Float16 w2t[64 * 64];   // [v][u]  = W2[u][v]
    _Float16 w2[64 * 64];    // [u][v]
    _Float16 w3t[16 * 64];   // [j][u]  = W3[u][j], j >= 2 zero
    float b1[64], b2[64], b3[4];
};

inline int check_hip_mlp(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return AMR_EHIP;
    }
    return AMR_OK;
}

}  // namespace amr
