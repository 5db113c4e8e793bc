// Device side of libamr: the single-pass raycaster (Section 5.3) and its launchers.
//
// One lane owns one ray. A wave64 covers an 8x8 pixel tile, a 256-thread block 16x16 pixels.
// The FP64 parts (ray generation, slab clip, kD-restart planes, sample positions of gradient
// taps) are written with contraction disabled so that every operation is correctly rounded
// exactly once; the per-sample arithmetic (trilinear, LUT, exp, compositing) is fp32 in
// patch-local cell coordinates.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "amr_internal.h"

namespace amr {

struct RenderArgs {
    const float *pool;
    const DNode *nodes;
    const DLeaf *leaves;
    const DPatch *patches;
    const float4 *lut;
    double box_lo[3], box_hi[3];     // B (closed, for gradient taps)
    double clip_lo[3], clip_hi[3];   // B ∩ clip box
    double step_fine;
    double eye[3], u[3], v[3], w[3];
    double tanf, win0, win1;
    int32_t ortho, width, height, depth;
    float v_lo, inv_range, step_frac, t_min;
    float lhat[3], k_a, k_d, eps2;
    int32_t uniform_step, lighting;
    float *rgba;
    amr_trace_rec *trace;
    int32_t *trace_n;
    int32_t *nsamp;
    int64_t trace_cap;
    amr_render_stats *stats;
    int32_t tiles_x, tiles_y, nblocks;
};

// ------------------------------------------------------------------------------------------
// FP64 geometry: rays, clip, kD-restart, point location
// ------------------------------------------------------------------------------------------

__device__ inline double sel3(int a, double x, double y, double z) { return a == 0 ? x : (a == 1 ? y : z); }

__device__ inline void make_ray(const RenderArgs &A, int i, int j, double o[3], double d[3]) {
#pragma clang fp contract(off)
    double s = (double)(2 * i + 1) / (double)A.width - 1.0;
    double t = 1.0 - (double)(2 * j + 1) / (double)A.height;
    double dd[3];
    if (A.ortho) {
        double a = s * A.win0, b = t * A.win1;
        for (int k = 0; k < 3; k++) {
            double e = A.eye[k] + a * A.u[k];
            o[k] = e + b * A.v[k];
            dd[k] = A.w[k];
        }
    } else {
        double aspect = (double)A.width / (double)A.height;
        double a = (s * A.tanf) * aspect, b = t * A.tanf;
        for (int k = 0; k < 3; k++) {
            o[k] = A.eye[k];
            double e = A.w[k] + a * A.u[k];
            dd[k] = e + b * A.v[k];
        }
    }
    double n2 = dd[0] * dd[0] + dd[1] * dd[1];
    n2 = n2 + dd[2] * dd[2];
    double nr = sqrt(n2);
    for (int k = 0; k < 3; k++) d[k] = dd[k] / nr;
}

__device__ inline bool clip_ray(const RenderArgs &A, const double o[3], const double d[3], double *t0, double *t1) {
#pragma clang fp contract(off)
    double lo_t = 0.0, hi_t = INFINITY;
    for (int a = 0; a < 3; a++) {
        double lo = A.clip_lo[a], hi = A.clip_hi[a];
        if (d[a] == 0.0) {
            if (!(o[a] >= lo && o[a] < hi)) return false;
            continue;
        }
        double inv = 1.0 / d[a];
        double ta = (lo - o[a]) * inv, tb = (hi - o[a]) * inv;
        double tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > lo_t) lo_t = tn;
        if (tf < hi_t) hi_t = tf;
    }
    *t0 = lo_t;
    *t1 = hi_t;
    return hi_t > lo_t;
}

// kD-restart: descend from the root for the ray interval [tmin, tmax]; returns the leaf id
// and shrinks tmax to the leaf's exit.  Returns -1 if the walk exceeds the tree depth.
__device__ inline int descend(const RenderArgs &A, const double o[3], const double d[3], const double invd[3],
                              double tmin, double &tmax) {
#pragma clang fp contract(off)
    uint32_t ni = 0;
    for (int it = 0; it <= A.depth; it++) {
        DNode n = A.nodes[ni];
        uint32_t axis = n.meta & 3u;
        if (axis == kLeafAxis) return (int)n.child;
        double oa = sel3(axis, o[0], o[1], o[2]);
        double da = sel3(axis, d[0], d[1], d[2]);
        double s = n.split;
        uint32_t low = n.child, high = low + 1;
        if (da == 0.0) {
            ni = oa < s ? low : high;
            continue;
        }
        bool near_low = (oa < s) || (oa == s && da < 0.0);
        uint32_t nearc = near_low ? low : high, farc = near_low ? high : low;
        double ts = (s - oa) * sel3(axis, invd[0], invd[1], invd[2]);
        if (ts <= 0.0 || ts >= tmax) ni = nearc;
        else if (ts <= tmin) ni = farc;
        else { ni = nearc; tmax = ts; }
    }
    return -1;
}

// Leaf holding point x (half-open comparisons against the split planes).
__device__ inline int locate_leaf(const RenderArgs &A, const double x[3]) {
    uint32_t ni = 0;
    for (int it = 0; it <= A.depth; it++) {
        DNode n = A.nodes[ni];
        uint32_t axis = n.meta & 3u;
        if (axis == kLeafAxis) return (int)n.child;
        ni = sel3(axis, x[0], x[1], x[2]) < n.split ? n.child : n.child + 1;
    }
    return -1;
}

// ------------------------------------------------------------------------------------------
// FP32 sampling
// ------------------------------------------------------------------------------------------

__device__ inline float lerpf(float a, float b, float f) { return a + f * (b - a); }

// Trilinear value of a padded brick at patch-local continuous index q (cell centres at
// integers; index -1 and n are the ghost layer).
__device__ inline float trilinear(const float *__restrict__ brick, int px, int pxy, int nx, int ny, int nz,
                                  float qx, float qy, float qz) {
    float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    int ix = min(max((int)fx, -1), nx - 1);
    int iy = min(max((int)fy, -1), ny - 1);
    int iz = min(max((int)fz, -1), nz - 1);
    fx = qx - (float)ix;
    fy = qy - (float)iy;
    fz = qz - (float)iz;
    const float *b = brick + (ix + 1) + (iy + 1) * px + (iz + 1) * pxy;
    float v000 = b[0], v100 = b[1], v010 = b[px], v110 = b[px + 1];
    float v001 = b[pxy], v101 = b[pxy + 1], v011 = b[pxy + px], v111 = b[pxy + px + 1];
    float c00 = lerpf(v000, v100, fx), c10 = lerpf(v010, v110, fx);
    float c01 = lerpf(v001, v101, fx), c11 = lerpf(v011, v111, fx);
    float c0 = lerpf(c00, c10, fy), c1 = lerpf(c01, c11, fy);
    return lerpf(c0, c1, fz);
}

struct PatchView {
    const float *brick;
    int px, pxy, nx, ny, nz;
};

__device__ inline PatchView patch_view(const RenderArgs &A, const DPatch &P) {
    PatchView v;
    v.brick = A.pool + P.off;
    v.nx = P.n[0];
    v.ny = P.n[1];
    v.nz = P.n[2];
    v.px = v.nx + 2;
    v.pxy = v.px * (v.ny + 2);
    return v;
}

// Field value at world point x located in the tree; false where no patch holds data or x is
// outside B (closed).
__device__ inline bool field_at(const RenderArgs &A, const double x[3], float *val, unsigned long long *descents) {
#pragma clang fp contract(off)
    for (int a = 0; a < 3; a++)
        if (x[a] < A.box_lo[a] || x[a] > A.box_hi[a]) return false;
    int leaf = locate_leaf(A, x);
    (*descents)++;
    if (leaf < 0) return false;
    int p = A.leaves[leaf].patch;
    if (p < 0) return false;
    const DPatch &P = A.patches[p];
    PatchView pv = patch_view(A, P);
    float q[3];
    for (int a = 0; a < 3; a++) q[a] = (float)((x[a] - P.lo[a]) * P.inv_h[a] - 0.5);
    *val = trilinear(pv.brick, pv.px, pv.pxy, pv.nx, pv.ny, pv.nz, q[0], q[1], q[2]);
    return true;
}

__device__ inline unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------------------------------
// The forward kernel
// ------------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void render_fwd(RenderArgs A) {
    __shared__ float4 s_lut[256];
    s_lut[threadIdx.x] = A.lut[threadIdx.x];
    __syncthreads();

    // XCD-aware tile order: blocks are dealt round-robin to the 8 XCDs, so give each XCD a
    // contiguous band of tiles (neighbouring rays share bricks in that XCD's L2).
    const int per = (A.nblocks + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= A.nblocks) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int pi = tx * 16 + (wave & 1) * 8 + (lane & 7);
    const int pj = ty * 16 + (wave >> 1) * 8 + (lane >> 3);
    const bool valid = pi < A.width && pj < A.height;
    const int64_t ray = (int64_t)pj * A.width + pi;

    unsigned long long c_samples = 0, c_segments = 0, c_hit = 0, c_desc = 0, c_guard = 0, c_tover = 0;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, T = 1.f;
    int nseg = 0;
    int nsamp_total = 0;
    double o[3], d[3], t0 = 0.0, t1 = 0.0;
    bool alive = false;
    if (valid) {
        make_ray(A, pi, pj, o, d);
        alive = clip_ray(A, o, d, &t0, &t1);
    }
    double invd[3];
    for (int a = 0; a < 3; a++) invd[a] = alive && d[a] != 0.0 ? 1.0 / d[a] : 0.0;
    c_hit = alive ? 1 : 0;
    const float inv_range = A.inv_range, v_lo = A.v_lo;
    double tcur = t0;
    while (alive && tcur < t1) {
        double tb = t1;
        int leaf = descend(A, o, d, invd, tcur, tb);
        if (leaf < 0) break;
        c_segments++;
        const DLeaf &L = A.leaves[leaf];
        int p = L.patch;
        int nsm = 0;
        if (p >= 0) {
            const DPatch &P = A.patches[p];
            double ratio, delta;
            {
#pragma clang fp contract(off)
                double step = (double)A.step_frac * (A.uniform_step ? A.step_fine : P.step);
                ratio = (tb - tcur) / step;
                double nn = ceil(ratio - 0x1p-20);
                nsm = nn < 1.0 ? 1 : (int)nn;
                delta = (tb - tcur) / (double)nsm;
            }
            PatchView pv = patch_view(A, P);
            float q0[3], dq[3];
            for (int a = 0; a < 3; a++) {
                q0[a] = (float)(((o[a] - P.lo[a]) + tcur * d[a]) * P.inv_h[a] - 0.5);
                dq[a] = (float)(delta * d[a] * P.inv_h[a]);
            }
            const float dl = (float)delta * 1.44269504088896340736f;   // delta * log2(e)
            double lbox_lo[3], lbox_hi[3], hl[3];
            if (A.lighting)
                for (int a = 0; a < 3; a++) { lbox_lo[a] = L.lo[a]; lbox_hi[a] = L.hi[a]; hl[a] = P.h[a]; }
            for (int k = 0; k < nsm; k++) {
                float kk = (float)k + 0.5f;
                float qx = q0[0] + kk * dq[0], qy = q0[1] + kk * dq[1], qz = q0[2] + kk * dq[2];
                float F = trilinear(pv.brick, pv.px, pv.pxy, pv.nx, pv.ny, pv.nz, qx, qy, qz);
                float u = __saturatef((F - v_lo) * inv_range);
                float xs = 255.f * u;
                int i0 = min((int)xs, 254);
                float f = xs - (float)i0;
                float4 La = s_lut[i0], Lb = s_lut[i0 + 1];
                float r = lerpf(La.x, Lb.x, f), g = lerpf(La.y, Lb.y, f), b = lerpf(La.z, Lb.z, f);
                float sig = lerpf(La.w, Lb.w, f);
                float alpha = 1.f - exp2f(-sig * dl);
                float shade = 1.f;
                if (A.lighting) {
                    double x[3];
                    {
#pragma clang fp contract(off)
                        double tk = tcur + ((double)k + 0.5) * delta;
                        for (int a = 0; a < 3; a++) x[a] = o[a] + tk * d[a];
                    }
                    float gv[3];
                    float qc[3] = {qx, qy, qz};
                    for (int a = 0; a < 3; a++) {
                        float Fs[2];
                        bool ok[2];
                        for (int sgn = 0; sgn < 2; sgn++) {
                            double xt[3] = {x[0], x[1], x[2]};
                            {
#pragma clang fp contract(off)
                                xt[a] = sgn ? x[a] - hl[a] : x[a] + hl[a];
                            }
                            bool in_leaf = xt[0] >= lbox_lo[0] && xt[0] < lbox_hi[0] && xt[1] >= lbox_lo[1] &&
                                           xt[1] < lbox_hi[1] && xt[2] >= lbox_lo[2] && xt[2] < lbox_hi[2];
                            if (in_leaf) {
                                float qq[3] = {qc[0], qc[1], qc[2]};
                                qq[a] += sgn ? -1.f : 1.f;
                                Fs[sgn] = trilinear(pv.brick, pv.px, pv.pxy, pv.nx, pv.ny, pv.nz, qq[0], qq[1], qq[2]);
                                ok[sgn] = true;
                            } else {
                                ok[sgn] = field_at(A, xt, &Fs[sgn], &c_desc);
                            }
                        }
                        float gr;
                        if (ok[0] && ok[1]) gr = (Fs[0] - Fs[1]) * (0.5f * inv_range);
                        else if (ok[0]) gr = (Fs[0] - F) * inv_range;
                        else if (ok[1]) gr = (F - Fs[1]) * inv_range;
                        else gr = 0.f;
                        gv[a] = gr;
                    }
                    float dot = gv[0] * A.lhat[0] + gv[1] * A.lhat[1] + gv[2] * A.lhat[2];
                    float den = sqrtf(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2] + A.eps2);
                    shade = A.k_a + (den > 0.f ? A.k_d * fabsf(dot) / den : 0.f);
                }
                float wgt = T * alpha * shade;
                C0 += wgt * r;
                C1 += wgt * g;
                C2 += wgt * b;
                T *= 1.f - alpha;
                nsamp_total++;
                if (T < A.t_min) { alive = false; break; }
            }
        }
        if (A.trace) {
            if (nseg < A.trace_cap) {
                amr_trace_rec rec;
                rec.leaf = leaf;
                rec.patch = p;
                rec.n = p >= 0 ? nsm : 0;
                rec.level = L.level;
                rec.ta = tcur;
                rec.tb = tb;
                A.trace[ray * A.trace_cap + nseg] = rec;
            } else {
                c_tover++;
            }
        }
        nseg++;
        if (tb <= tcur) {   // never expected: keep the walk moving forward
            c_guard++;
            tb = nextafter(tcur, INFINITY);
        }
        tcur = tb;
    }
    if (valid) {
        reinterpret_cast<float4 *>(A.rgba)[ray] = make_float4(C0, C1, C2, 1.f - T);
        if (A.trace_n) A.trace_n[ray] = nseg;
        if (A.nsamp) A.nsamp[ray] = nsamp_total;
    }
    if (A.stats) {
        c_samples = wave_sum((unsigned long long)nsamp_total);
        c_segments = wave_sum(c_segments);
        c_hit = wave_sum(c_hit);
        c_desc = wave_sum(c_desc);
        c_guard = wave_sum(c_guard);
        c_tover = wave_sum(c_tover);
        if (lane == 0) {
            atomicAdd(&A.stats->samples, c_samples);
            atomicAdd(&A.stats->segments, c_segments);
            atomicAdd(&A.stats->rays_hit, c_hit);
            if (c_desc) atomicAdd(&A.stats->tap_descents, c_desc);
            if (c_guard) atomicAdd(&A.stats->guard_hits, c_guard);
            if (c_tover) atomicAdd(&A.stats->trace_overflow, c_tover);
        }
    }
}

__global__ void zero_u64(unsigned long long *p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

static int check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return AMR_EHIP;
    }
    return AMR_OK;
}

static int fill_args(const amr_scene *S, const amr_camera *C, const amr_render_params *P, RenderArgs *A) {
    memset(A, 0, sizeof(*A));
    if (!P->d_lut) { set_error("d_lut is NULL"); return AMR_EINVAL; }
    if (!(P->v_hi > P->v_lo)) { set_error("v_hi must exceed v_lo"); return AMR_EINVAL; }
    if (!(P->step_frac > 0.f) || !std::isfinite(P->step_frac)) { set_error("step_frac must be positive"); return AMR_EINVAL; }
    if (C->width <= 0 || C->height <= 0) { set_error("camera size must be positive"); return AMR_EINVAL; }
    A->pool = S->pool;
    A->nodes = (const DNode *)S->nodes;
    A->leaves = (const DLeaf *)S->leaves;
    A->patches = (const DPatch *)S->patches;
    A->lut = (const float4 *)P->d_lut;
    for (int a = 0; a < 3; a++) {
        A->box_lo[a] = S->box_lo[a];
        A->box_hi[a] = S->box_hi[a];
        A->clip_lo[a] = S->box_lo[a] > P->clip_lo[a] ? S->box_lo[a] : P->clip_lo[a];
        A->clip_hi[a] = S->box_hi[a] < P->clip_hi[a] ? S->box_hi[a] : P->clip_hi[a];
        A->eye[a] = C->eye[a];
        A->u[a] = C->u[a];
        A->v[a] = C->v[a];
        A->w[a] = C->w[a];
    }
    A->step_fine = S->step_fine;
    A->tanf = C->tan_half_fov;
    A->win0 = C->win[0];
    A->win1 = C->win[1];
    A->ortho = C->ortho;
    A->width = C->width;
    A->height = C->height;
    A->depth = S->depth;
    A->v_lo = P->v_lo;
    A->inv_range = 1.0f / (P->v_hi - P->v_lo);
    A->step_frac = P->step_frac;
    A->t_min = P->t_min;
    float ln = sqrtf(P->light[0] * P->light[0] + P->light[1] * P->light[1] + P->light[2] * P->light[2]);
    for (int a = 0; a < 3; a++) A->lhat[a] = ln > 0.f ? P->light[a] / ln : 0.f;
    A->k_a = P->k_a;
    A->k_d = P->k_d;
    A->eps2 = P->eps_g * P->eps_g;
    A->uniform_step = P->uniform_step;
    A->lighting = P->lighting;
    A->tiles_x = (C->width + 15) / 16;
    A->tiles_y = (C->height + 15) / 16;
    A->nblocks = A->tiles_x * A->tiles_y;
    return AMR_OK;
}

}  // namespace amr

using namespace amr;

extern "C" {

int amr_render(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
               float *d_rgba, amr_render_stats *d_stats, void *stream) {
    if (!S || !cams || !P || !d_rgba || ncams <= 0) { set_error("null argument or ncams <= 0"); return AMR_EINVAL; }
    if (!S->pool || !S->nodes || !S->leaves || !S->patches) { set_error("scene not packed"); return AMR_EINVAL; }
    if (P->d_trace && P->trace_cap <= 0) { set_error("trace_cap must be positive with d_trace"); return AMR_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    if (d_stats) {
        int n = (int)(sizeof(amr_render_stats) / 8);
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, s, (unsigned long long *)d_stats, n);
    }
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
        int grid = ((A.nblocks + 7) / 8) * 8;
        hipLaunchKernelGGL(render_fwd, dim3(grid), dim3(256), 0, s, A);
        rc = check_hip(hipGetLastError(), "render_fwd launch");
        if (rc) return rc;
        pix_off += (int64_t)cams[c].width * cams[c].height;
    }
    return AMR_OK;
}

}  // extern "C"
