// Entry points whose kernels are not in this build yet: they fail with AMR_EINVAL and a message.
#include "amr_internal.h"

using namespace amr;

extern "C" {

int amr_render_backward(const amr_scene *, const amr_camera *, int32_t, const amr_render_params *, const float *,
                        float *, float *, int32_t, void *) {
    set_error("amr_render_backward: not available in this build");
    return AMR_EINVAL;
}
int64_t amr_queue_bytes(int32_t ncams) { return 256 + 64 * (int64_t)(ncams > 0 ? ncams : 0); }
int64_t amr_ckpt_bytes(int64_t nrays, int32_t ckpt_max) { return nrays * (16 + 32 * (int64_t)ckpt_max); }
int32_t amr_mlp_param_count(void) { return 12 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2; }
int amr_mlp_forward(const float *, const float *, float *, float *, int64_t, void *) {
    set_error("amr_mlp_forward: not available in this build");
    return AMR_EINVAL;
}
int amr_mlp_backward(const float *, const float *, const float *, const float *, const float *, int64_t, float, float,
                     float *, float *, void *) {
    set_error("amr_mlp_backward: not available in this build");
    return AMR_EINVAL;
}
int amr_mlp_adam_step(float *, const float *, float *, float *, int32_t, float, float, float, float, void *) {
    set_error("amr_mlp_adam_step: not available in this build");
    return AMR_EINVAL;
}
int64_t amr_mlp_packed_bytes(void) { return 0; }
int amr_mlp_pack(const float *, void *, void *) {
    set_error("amr_mlp_pack: not available in this build");
    return AMR_EINVAL;
}
}
