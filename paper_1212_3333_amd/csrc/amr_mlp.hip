// The segment-proposal network (an addition to the paper's method): 12 -> 64 -> 64 -> 2,
// ReLU hidden layers, sigmoid outputs (alpha_lo, alpha_hi), trained with a pinball loss.
//
// GEMMs run on the matrix cores, fp16 operands and fp32 accumulation: the 16x16x16 shape for
// layer 1 (K = 16, the 12 inputs padded), gfx950's 16x16x32 shape for every K = 64 product
// (operand layouts in amr_mlp.h).  A wave handles a 64-row tile.
// Parameters are fp32 masters packed as W1 [12][64], b1 [64], W2 [64][64], b2 [64],
// W3 [64][2], b3 [2] (input-major); the fp16 operands are rounded from them.
#include <hip/hip_runtime.h>

#include "amr_mlp.h"

namespace amr {

// Stage the fp16 operand copies of the weights in LDS, in the layouts the MFMA loads want.
__device__ inline void stage_weights(const float *W, MlpLds &s) {
    const float *W1 = W + kOffW1, *W2 = W + kOffW2, *W3 = W + kOffW3;
    for (int i = threadIdx.x; i < 64 * 16; i += blockDim.x) {       // W1T[u][i], i >= 12 zero
        int u = i / 16, k = i % 16;
        s.w1t[i] = (_Float16)(k < kIn ? W1[k * 64 + u] : 0.f);
    }
    for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        int a = i / 64, b = i % 64;
        s.w2t[i] = (_Float16)W2[b * 64 + a];                          // W2T[v][u] = W2[u][v]
        s.w2[i] = (_Float16)W2[i];                                    // W2[u][v]
    }
    for (int i = threadIdx.x; i < 16 * 64; i += blockDim.x) {       // W3T[j][u], j >= 2 zero
        int j = i / 64, u = i % 64;
        s.w3t[i] = (_Float16)(j < kOut ? W3[u * 2 + j] : 0.f);
    }
    for (int i = threadIdx.x; i < 64; i += blockDim.x) {
        s.b1[i] = W[kOffB1 + i];
        s.b2[i] = W[kOffB2 + i];
    }
    if (threadIdx.x < 2) s.b3[threadIdx.x] = W[kOffB3 + threadIdx.x];
}

// Forward of one 64-row tile whose fp16 inputs sit in x16 ([64][16], row-major, zero padded).
// Writes post-ReLU activations to h1/h2 (fp16, [64][64]) and returns the pre-sigmoid logits of
// rows 4 (l/16) + j of row tile rt in z3[rt][j] for column l % 16 (columns 0, 1 are valid).
__device__ inline void mlp_tile_forward(const MlpLds &s, const _Float16 *x16, _Float16 *h1, _Float16 *h2,
                                        float z3[4][4], float *h1f, float *h2f) {
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    // layer 1: [64 x 16] . [16 x 64]
    for (int rt = 0; rt < 4; rt++) {
        half4 a = *reinterpret_cast<const half4 *>(x16 + (rt * 16 + lr) * 16 + 4 * lq);
        for (int ct = 0; ct < 4; ct++) {
            half4 b = *reinterpret_cast<const half4 *>(s.w1t + (ct * 16 + lr) * 16 + 4 * lq);
            float4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma_k16(a, b, acc);
            for (int j = 0; j < 4; j++) {
                int row = rt * 16 + 4 * lq + j, col = ct * 16 + lr;
                float hv = fmaxf(acc[j] + s.b1[col], 0.f);
                h1[row * 64 + col] = (_Float16)hv;
                if (h1f) h1f[row * 64 + col] = hv;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    // layer 2: [64 x 64] . [64 x 64]
    for (int rt = 0; rt < 4; rt++)
        for (int ct = 0; ct < 4; ct++) {
            float4v acc = {0.f, 0.f, 0.f, 0.f};
            for (int ks = 0; ks < 2; ks++) {
                half8 a = *reinterpret_cast<const half8 *>(h1 + (rt * 16 + lr) * 64 + ks * 32 + 8 * lq);
                half8 b = *reinterpret_cast<const half8 *>(s.w2t + (ct * 16 + lr) * 64 + ks * 32 + 8 * lq);
                acc = mfma_k32(a, b, acc);
            }
            for (int j = 0; j < 4; j++) {
                int row = rt * 16 + 4 * lq + j, col = ct * 16 + lr;
                float hv = fmaxf(acc[j] + s.b2[col], 0.f);
                h2[row * 64 + col] = (_Float16)hv;
                if (h2f) h2f[row * 64 + col] = hv;
            }
        }
    __builtin_amdgcn_wave_barrier();
    // layer 3: [64 x 64] . [64 x 16] (two valid columns)
    for (int rt = 0; rt < 4; rt++) {
        float4v acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < 2; ks++) {
            half8 a = *reinterpret_cast<const half8 *>(h2 + (rt * 16 + lr) * 64 + ks * 32 + 8 * lq);
            half8 b = *reinterpret_cast<const half8 *>(s.w3t + lr * 64 + ks * 32 + 8 * lq);
            acc = mfma_k32(a, b, acc);
        }
        for (int j = 0; j < 4; j++) z3[rt][j] = acc[j] + (lr < kOut ? s.b3[lr] : 0.f);
    }
}

__device__ inline float sigmoidf_(float z) { return 1.f / (1.f + __expf(-z)); }

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *X, const float *W, float *Y, float *H,
                                                         int64_t n) {
    __shared__ MlpLds s;
    __shared__ __attribute__((aligned(16))) _Float16 xs[4][64 * 16];
    __shared__ __attribute__((aligned(16))) _Float16 hs1[4][64 * 64], hs2[4][64 * 64];
    stage_weights(W, s);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t ntiles = (n + 63) / 64;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntiles; t += (int64_t)gridDim.x * 4) {
        const int64_t row0 = t * 64;
        for (int i = lane; i < 64 * 16; i += 64) {
            int r = i / 16, k = i % 16;
            int64_t g = row0 + r;
            xs[wave][i] = (_Float16)(g < n && k < kIn ? X[g * kIn + k] : 0.f);
        }
        __builtin_amdgcn_wave_barrier();
        float z3[4][4];
        float *h1f = nullptr, *h2f = nullptr;
        mlp_tile_forward(s, xs[wave], hs1[wave], hs2[wave], z3, h1f, h2f);
        for (int rt = 0; rt < 4; rt++)
            for (int j = 0; j < 4; j++) {
                int64_t g = row0 + rt * 16 + 4 * lq + j;
                if (lr < kOut && g < n) Y[g * 2 + lr] = sigmoidf_(z3[rt][j]);
            }
        if (H) {   // activations for the backward pass: [n][128] = h1 (64) then h2 (64), fp32
            __builtin_amdgcn_wave_barrier();
            for (int i = lane; i < 64 * 64; i += 64) {
                int r = i / 64, c = i % 64;
                int64_t g = row0 + r;
                if (g < n) {
                    H[g * 128 + c] = (float)hs1[wave][i];
                    H[g * 128 + 64 + c] = (float)hs2[wave][i];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Backward of the mean pinball loss.  dZ values are kept unscaled (no 1/n) through the fp16
// products and scaled at the end, so they stay in fp16's normal range.
__global__ __launch_bounds__(256) void mlp_backward_kernel(const float *X, const float *W, const float *H,
                                                          const float *Y, const float *Tg, int64_t n, float q_lo,
                                                          float q_hi, float *dW, float *loss) {
    __shared__ MlpLds s;
    __shared__ __attribute__((aligned(16))) _Float16 hs1[4][64 * 64], dz2s[4][64 * 64];
    __shared__ float acc_s[kParams];
    stage_weights(W, s);
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) acc_s[i] = 0.f;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lq = lane >> 4;
    const int64_t ntiles = (n + 63) / 64;
    // per-lane fp32 accumulators: dW2 tiles (MFMA D layout) and the VALU parts
    float4v dw2[4][4];
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) dw2[a][b] = float4v{0.f, 0.f, 0.f, 0.f};
    float dw1[kIn], db1 = 0.f, db2 = 0.f, dw3[2] = {0.f, 0.f}, db3[2] = {0.f, 0.f}, lsum = 0.f;
    for (int k = 0; k < kIn; k++) dw1[k] = 0.f;
    const float *W3 = W + kOffW3;
    const float w3u0 = W3[lane * 2], w3u1 = W3[lane * 2 + 1];   // lane = hidden unit u
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < ntiles; t += (int64_t)gridDim.x * 4) {
        const int64_t row0 = t * 64;
        // lane = hidden unit: dZ2 column for all 64 rows; dW3 and db3 on the VALU
        for (int r = 0; r < 64; r++) {
            int64_t g = row0 + r;
            float dz2 = 0.f;
            if (g < n) {
                float y0 = Y[g * 2], y1 = Y[g * 2 + 1], tg = Tg[g];
                float d0 = tg > y0 ? -q_lo : 1.f - q_lo;
                float d1 = tg > y1 ? -q_hi : 1.f - q_hi;
                if (lane == 0) {
                    float r0 = tg - y0, r1 = tg - y1;
                    lsum += fmaxf(q_lo * r0, (q_lo - 1.f) * r0) + fmaxf(q_hi * r1, (q_hi - 1.f) * r1);
                }
                float dz30 = d0 * y0 * (1.f - y0), dz31 = d1 * y1 * (1.f - y1);
                float h2 = H[g * 128 + 64 + lane], h1 = H[g * 128 + lane];
                dw3[0] += h2 * dz30;
                dw3[1] += h2 * dz31;
                if (lane < 2) db3[lane] += lane == 0 ? dz30 : dz31;
                dz2 = h2 > 0.f ? dz30 * w3u0 + dz31 * w3u1 : 0.f;
                db2 += dz2;
                hs1[wave][r * 64 + lane] = (_Float16)h1;
            } else {
                hs1[wave][r * 64 + lane] = (_Float16)0.f;
            }
            dz2s[wave][r * 64 + lane] = (_Float16)dz2;
        }
        __builtin_amdgcn_wave_barrier();
        // dW2 += H1^T dZ2: M = unit u, K = row, N = unit v
        for (int mt = 0; mt < 4; mt++)
            for (int nt = 0; nt < 4; nt++)
                for (int ks = 0; ks < 2; ks++) {
                    half8 a, b;
                    for (int j = 0; j < 8; j++) {
                        int row = ks * 32 + 8 * lq + j;
                        a[j] = hs1[wave][row * 64 + mt * 16 + lr];
                        b[j] = dz2s[wave][row * 64 + nt * 16 + lr];
                    }
                    dw2[mt][nt] = mfma_k32(a, b, dw2[mt][nt]);
                }
        // dH1 = dZ2 W2^T (M = row, K = unit v, N = unit u), then dZ1 = dH1 (H1 > 0);
        // dW1 += X^T dZ1 and db1 on the VALU (lane = unit u after the shuffle through LDS)
        for (int rt = 0; rt < 4; rt++)
            for (int ct = 0; ct < 4; ct++) {
                float4v acc = {0.f, 0.f, 0.f, 0.f};
                for (int ks = 0; ks < 2; ks++) {
                    half8 a = *reinterpret_cast<const half8 *>(&dz2s[wave][(rt * 16 + lr) * 64 + ks * 32 + 8 * lq]);
                    half8 b = *reinterpret_cast<const half8 *>(&s.w2[(ct * 16 + lr) * 64 + ks * 32 + 8 * lq]);
                    acc = mfma_k32(a, b, acc);
                }
                __builtin_amdgcn_wave_barrier();
                for (int j = 0; j < 4; j++) {
                    int row = rt * 16 + 4 * lq + j, col = ct * 16 + lr;
                    float h1 = (float)hs1[wave][row * 64 + col];
                    // reuse dz2s rows already consumed? no: stash dZ1 in hs1 (h1 no longer needed
                    // after its sign is read)
                    hs1[wave][row * 64 + col] = (_Float16)(h1 > 0.f ? acc[j] : 0.f);
                }
            }
        __builtin_amdgcn_wave_barrier();
        for (int r = 0; r < 64; r++) {
            int64_t g = row0 + r;
            if (g >= n) break;
            float dz1 = (float)hs1[wave][r * 64 + lane];
            db1 += dz1;
            for (int k = 0; k < kIn; k++) dw1[k] += X[g * kIn + k] * dz1;
        }
        __builtin_amdgcn_wave_barrier();
    }
    // reduce per block in LDS, then one global atomic per parameter and block
    for (int k = 0; k < kIn; k++) atomicAdd(&acc_s[kOffW1 + k * 64 + lane], dw1[k]);
    atomicAdd(&acc_s[kOffB1 + lane], db1);
    for (int mt = 0; mt < 4; mt++)
        for (int nt = 0; nt < 4; nt++)
            for (int j = 0; j < 4; j++)
                atomicAdd(&acc_s[kOffW2 + (mt * 16 + 4 * lq + j) * 64 + nt * 16 + lr], dw2[mt][nt][j]);
    atomicAdd(&acc_s[kOffB2 + lane], db2);
    atomicAdd(&acc_s[kOffW3 + lane * 2], dw3[0]);
    atomicAdd(&acc_s[kOffW3 + lane * 2 + 1], dw3[1]);
    if (lane < 2) atomicAdd(&acc_s[kOffB3 + lane], db3[lane]);
    __syncthreads();
    const float inv_n = 1.f / (float)n;
    for (int i = threadIdx.x; i < kParams; i += blockDim.x) atomicAdd(&dW[i], acc_s[i] * inv_n);
    if (lane == 0 && lsum != 0.f) atomicAdd(loss, lsum * inv_n);
}

__global__ void mlp_zero(float *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void mlp_adam_kernel(float *W, const float *dW, float *M, float *V, int n, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float g = dW[i];
    float m = b1 * M[i] + (1.f - b1) * g;
    float v = b2 * V[i] + (1.f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    W[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// Packed inference layout: the LDS image of MlpLds (fp16 operand copies + fp32 biases).
__global__ void mlp_pack_kernel(const float *W, MlpLds *out) {
    __shared__ MlpLds s;
    stage_weights(W, s);
    __syncthreads();
    const uint32_t *src = reinterpret_cast<const uint32_t *>(&s);
    uint32_t *dst = reinterpret_cast<uint32_t *>(out);
    for (int i = threadIdx.x; i < (int)(sizeof(MlpLds) / 4); i += blockDim.x) dst[i] = src[i];
}

}  // namespace amr

using namespace amr;

extern "C" {

int32_t amr_mlp_param_count(void) { return kParams; }
int64_t amr_mlp_packed_bytes(void) { return (int64_t)sizeof(MlpLds); }

int amr_mlp_forward(const float *X, const float *W, float *Y, float *H, int64_t n, void *stream) {
    if (!X || !W || !Y || n <= 0) { set_error("amr_mlp_forward: null argument or n <= 0"); return AMR_EINVAL; }
    int64_t tiles = (n + 63) / 64;
    int grid = (int)std::min<int64_t>((tiles + 3) / 4, 4096);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, X, W, Y, H, n);
    return check_hip_mlp(hipGetLastError(), "mlp_forward launch");
}

int amr_mlp_backward(const float *X, const float *W, const float *H, const float *Y, const float *T, int64_t n,
                     float q_lo, float q_hi, float *dW, float *loss, void *stream) {
    if (!X || !W || !H || !Y || !T || !dW || !loss || n <= 0) {
        set_error("amr_mlp_backward: null argument or n <= 0");
        return AMR_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mlp_zero, dim3((kParams + 255) / 256), dim3(256), 0, s, dW, kParams);
    hipLaunchKernelGGL(mlp_zero, dim3(1), dim3(64), 0, s, loss, 1);
    int64_t tiles = (n + 63) / 64;
    int grid = (int)std::min<int64_t>((tiles + 3) / 4, 512);
    hipLaunchKernelGGL(mlp_backward_kernel, dim3(grid), dim3(256), 0, s, X, W, H, Y, T, n, q_lo, q_hi, dW, loss);
    return check_hip_mlp(hipGetLastError(), "mlp_backward launch");
}

int amr_mlp_adam_step(float *W, const float *dW, float *M, float *V, int32_t t, float lr, float beta1, float beta2,
                      float eps, void *stream) {
    if (!W || !dW || !M || !V || t < 1) { set_error("amr_mlp_adam_step: null argument or t < 1"); return AMR_EINVAL; }
    float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, W, dW, M, V,
                       kParams, lr, beta1, beta2, eps, c1, c2);
    return check_hip_mlp(hipGetLastError(), "mlp_adam launch");
}

int amr_mlp_pack(const float *W, void *d_out, void *stream) {
    if (!W || !d_out) { set_error("amr_mlp_pack: null argument"); return AMR_EINVAL; }
    if (reinterpret_cast<uintptr_t>(d_out) & 15u) { set_error("amr_mlp_pack: d_out must be 16-byte aligned"); return AMR_EINVAL; }
    hipLaunchKernelGGL(mlp_pack_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, W, (MlpLds *)d_out);
    return check_hip_mlp(hipGetLastError(), "mlp_pack launch");
}

}  // extern "C"
