// Shared device code of the raycasting kernels: FP64 ray geometry and kD-restart traversal,
// patch-local FP32 sampling, LUT classification and gradient lighting (Sections 5.3 and 6).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "amr_internal.h"
#include "amr_tapq_index.h"

namespace amr {

constexpr int kGradLen = 1024 + 5;   // dL/dLUT [256][4] then dL/d(light xyz, k_a, k_d)
constexpr int kBwdGrid = 2048;       // adjoint blocks: fixed, so deterministic mode sums a fixed set of partials

struct CkptHeader {                  // per ray, written at the end of the forward
    float T, C[3];
    int32_t nsamp, nck, every, nrec;  // nrec: the ray's tape records (those beyond the cap unwritten)
};
struct Ckpt {                        // (t, T, C) at the start of a data segment
    double t;
    float T, C[3];
    int32_t rec, sidx;               // tape records and samples of the ray before this point
};
static_assert(sizeof(CkptHeader) == 32 && sizeof(Ckpt) == 32, "checkpoint layout");

// The tape of the checkpointed lit forward: per ray, in the ray's order, one 16-byte record
// at the start of each data segment, (delta, delta log2(e), n as int bits, 0), then one per
// sample, (F, g_x, g_y, g_z): the sampled value and the central-difference gradient the
// forward shaded with.  The adjoint replays an interval from these records alone.  Records
// at or beyond tape_cap are not written; the header counts them all.
constexpr int64_t kTapeCapMax = (1 << 26) - 1;   // tape positions travel in 26 bits of the queue
__device__ __forceinline__ float4 tape_segment(double delta, float dl, int n) {
    return make_float4((float)delta, dl, __int_as_float(n), 0.f);
}

struct RenderArgs {
    const float *pool;
    const DNode *nodes;
    const DLeaf *leaves;
    const DPatch *patches;
    const DFaceXf *face_xf;          // [nleaves][6] gradient-tap records
    int32_t nearest;                 // 1: nearest-cell sampling instead of trilinear
    int32_t lod_on, nleaves;         // level of detail enabled; real leaves (kind-(a) records follow)
    int32_t nrec, npatches;          // leaf records (real + kind-(a)); patch headers
    double lod;                      // pixels
    double lod_pix;                  // pixel footprint per unit distance (perspective) or per pixel
    double plight[3];                // lighting = 2: point-light position
    const float4 *lut;
    double box_lo[3], box_hi[3];     // B (closed, for gradient taps)
    double clip_lo[3], clip_hi[3];   // B ∩ clip box
    double step_fine;
    double eye[3], u[3], v[3], w[3];
    double tanf, win0, win1;
    int32_t ortho, width, height, depth;
    float v_lo, inv_range, step_frac, t_min;
    float lhat[3], inv_lnorm, k_a, k_d, eps2;
    int32_t uniform_step, lighting, layout;   // layout: 0 linear, 1 micro-bricks, 2 halo rows
    float *rgba;
    amr_trace_rec *trace;
    int32_t *trace_n;
    int32_t *nsamp;
    int64_t trace_cap;
    amr_render_stats *stats;
    uint32_t *touch;
    uint32_t *touch_meta;            // measurement: one bit per 16 bytes of the scene's metadata
    const uint8_t *meta_base;        // start of the metadata buffer (the node array)
    uint8_t *ckpt;                   // checkpoint buffer base (all cameras)
    int64_t ckpt_ray0;               // first ray of this camera in the buffer
    int64_t ckpt_stride;             // bytes per ray
    int32_t ckpt_every, ckpt_max;
    float4 *tape;                    // checkpointed lit forward: per ray, a record per data
    int64_t tape_cap;                // segment and per sample ([rays][tape_cap]; see TapeSeg)
    uint32_t *sched_hdr;             // tile schedule (null: none): per camera the tile count its
    uint32_t *sched_time;            // order was sorted for (4 words each); per tile its time in
    uint32_t *sched_order;           // the last call; per camera its tiles, longest first
    int64_t tile0;                   // this camera's first tile in the schedule
    int32_t cam;                     // this camera's index in the call
    int32_t tiles_x, tiles_y, nblocks;     // 16x16 tiles of four waves (learned kernel)
    int32_t t8x, t8y, sgrid;               // 8x8 one-wave tiles; side of the power-of-two
                                           // grid of 4x4-tile super-tiles covering them
};

// The per-camera fields of RenderArgs, for launches that render a group of cameras (one camera
// per blockIdx.y): each block takes its camera's fields and its pixel offset in the outputs.
struct CamArgs {
    double eye[3], u[3], v[3], w[3];
    double tanf, win0, win1, lod_pix;
    int32_t ortho, width, height, t8x, t8y, sgrid;
    int64_t ray0;                    // the camera's first pixel, relative to the group's first
    int64_t tile0;                   // the camera's first tile in the schedule
    int32_t cam, pad_;               // the camera's index in the call
};
constexpr int kCamGroup = 8;
// Side of a tile schedule's super-tile in 8x8 tiles: 2 (16x16 pixels) for lit renders, whose
// longest tiles are long enough that a finer order shortens the launch's tail, 4 (32x32 pixels)
// for unlit ones, whose short tiles gain more from sharing bricks in an XCD's L2.
__host__ __device__ constexpr uint32_t sched_side(bool lit) { return lit ? 2u : 4u; }

struct CamGroup {
    CamArgs cam[kCamGroup];
    int32_t n;                       // cameras in the group; 0: one camera, RenderArgs as given
    // with a tile schedule: the launch is one-dimensional over the group's super-tiles of
    // s x s tiles (s = sched_side), block b taking rank (b / (8 s^2)) * 8 + b % 8 of the order
    // and tile (b / 8) % s^2 of that super-tile; an order entry is camera << 24 | super-tile
    int32_t sched;                   // 1: a scheduled launch
    uint32_t nst;                    // super-tiles of the group
    uint32_t sig;                    // signature of the group's camera sizes, the order's key
    int32_t cam0;                    // the group's first camera in the call (its header holds sig)
    int64_t order0;                  // the group's first order slot
    uint32_t stpre[kCamGroup + 1];   // first super-tile of each camera in the default order
};
static_assert(sizeof(RenderArgs) + sizeof(CamGroup) <= 4096, "kernel arguments of a group launch");

inline CamArgs cam_args_of(const RenderArgs &A, int64_t ray0) {
    CamArgs C;
    C.tile0 = A.tile0;
    C.cam = A.cam;
    C.pad_ = 0;
    for (int a = 0; a < 3; a++) {
        C.eye[a] = A.eye[a];
        C.u[a] = A.u[a];
        C.v[a] = A.v[a];
        C.w[a] = A.w[a];
    }
    C.tanf = A.tanf;
    C.win0 = A.win0;
    C.win1 = A.win1;
    C.lod_pix = A.lod_pix;
    C.ortho = A.ortho;
    C.width = A.width;
    C.height = A.height;
    C.t8x = A.t8x;
    C.t8y = A.t8y;
    C.sgrid = A.sgrid;
    C.ray0 = ray0;
    return C;
}

// A block of a group launch takes its camera (c, for unscheduled launches blockIdx.y) into A.
__device__ __forceinline__ void take_camera(RenderArgs &A, const CamGroup &G, int c) {
    if (G.n == 0) return;
    const CamArgs &C = G.cam[c];
    #pragma unroll
    for (int a = 0; a < 3; a++) {
        A.eye[a] = C.eye[a];
        A.u[a] = C.u[a];
        A.v[a] = C.v[a];
        A.w[a] = C.w[a];
    }
    A.tanf = C.tanf;
    A.win0 = C.win0;
    A.win1 = C.win1;
    A.lod_pix = C.lod_pix;
    A.ortho = C.ortho;
    A.width = C.width;
    A.height = C.height;
    A.t8x = C.t8x;
    A.t8y = C.t8y;
    A.sgrid = C.sgrid;
    A.tile0 = C.tile0;
    A.cam = C.cam;
    A.rgba += 4 * C.ray0;
    if (A.trace) A.trace += C.ray0 * A.trace_cap;
    if (A.trace_n) A.trace_n += C.ray0;
    if (A.nsamp) A.nsamp += C.ray0;
    A.ckpt_ray0 += C.ray0;
}

// Tile schedule layout (words of 4 bytes): a 4-word header per camera, padded to 256 bytes, then
// one time per tile of every camera (camera by camera, tiles row-major), then one order slot per
// tile.
inline int64_t sched_header_words(int64_t ncams) { return (4 * ncams + 63) / 64 * 64; }
inline int64_t sched_tiles(const amr_camera &C) { return (int64_t)((C.width + 7) / 8) * ((C.height + 7) / 8); }

struct BwdArgs {
    const float *grad_rgba;
    float *grad;                     // kGradLen accumulator
    float *partials;                 // deterministic: [grid][kGradLen]
    int32_t ray_major;               // work items numbered ray by ray (else interval by interval)
    int64_t nrays;                   // rays the launch covers, from A.ckpt_ray0 (the tape kernel
                                     // covers every camera of the call at once)
};

struct Counters {   // per lane (32-bit); summed over the wave in 64 bits when flushed
    unsigned int samples = 0, segments = 0, hit = 0, desc = 0, guard = 0, tover = 0, ckover = 0;
    unsigned int split = 0, face = 0, unsure = 0, linl = 0;
};

// ------------------------------------------------------------------------------------------
// FP64 geometry
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ double sel3(int a, double x, double y, double z) { return a == 0 ? x : (a == 1 ? y : z); }

struct Ray {
    double o[3], d[3], invd[3], t0, t1;
};

__device__ __forceinline__ void make_ray(const RenderArgs &A, int i, int j, double o[3], double d[3]) {
#pragma clang fp contract(off)
    double s = (double)(2 * i + 1) / (double)A.width - 1.0;
    double t = 1.0 - (double)(2 * j + 1) / (double)A.height;
    double dd[3];
    if (A.ortho) {
        double a = s * A.win0, b = t * A.win1;
        #pragma unroll
        for (int k = 0; k < 3; k++) {
            double e = A.eye[k] + a * A.u[k];
            o[k] = e + b * A.v[k];
            dd[k] = A.w[k];
        }
    } else {
        double aspect = (double)A.width / (double)A.height;
        double a = (s * A.tanf) * aspect, b = t * A.tanf;
        #pragma unroll
        for (int k = 0; k < 3; k++) {
            o[k] = A.eye[k];
            double e = A.w[k] + a * A.u[k];
            dd[k] = e + b * A.v[k];
        }
    }
    double n2 = dd[0] * dd[0] + dd[1] * dd[1];
    n2 = n2 + dd[2] * dd[2];
    double nr = sqrt(n2);
    #pragma unroll
    for (int k = 0; k < 3; k++) d[k] = dd[k] / nr;
}

__device__ __forceinline__ bool clip_ray(const RenderArgs &A, const double o[3], const double d[3], double *t0, double *t1) {
#pragma clang fp contract(off)
    double lo_t = 0.0, hi_t = INFINITY;
    #pragma unroll
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

__device__ __forceinline__ bool setup_ray(const RenderArgs &A, int i, int j, Ray &R) {
    make_ray(A, i, j, R.o, R.d);
    if (!clip_ray(A, R.o, R.d, &R.t0, &R.t1)) return false;
    #pragma unroll
    for (int a = 0; a < 3; a++) R.invd[a] = R.d[a] != 0.0 ? 1.0 / R.d[a] : 0.0;
    return true;
}

// Measurement only: marks the metadata bytes [p, p + bytes) as read (16-byte granules).
__device__ __forceinline__ void touch_meta(const RenderArgs &A, const void *p, int bytes) {
    const int64_t off = (const uint8_t *)p - A.meta_base;
    for (int64_t g = off >> 4; g <= (off + bytes - 1) >> 4; g++) atomicOr(&A.touch_meta[g >> 5], 1u << (g & 31));
}

// kD-restart with push-down: `start` is the deepest node known to hold the rest of the ray.
// While the descent has not clipped tmax, every decision on the way down was independent of
// tmin (the split lay outside [tmin, tmax], or behind tmin), so a later restart with a larger
// tmin and the same tmax takes the same way: the walk can begin at the node reached so far.  The
// leaves and exits found are exactly those of a restart from the root.  Level-of-detail walks
// always start at the root (they must see every kind-(a) node on the way).
// MARK (measurement): every node read is marked in A.touch_meta.
template <bool LOD, bool MARK = false>
__device__ __forceinline__ int descend_walk(const RenderArgs &A, const Ray &R, double tmin, double &tmax,
                                            uint32_t &start) {
#pragma clang fp contract(off)
    uint32_t ni = LOD ? 0u : start;
    bool open = !LOD;
    for (int it = 0; it <= A.depth; it++) {
        DNode n = A.nodes[ni];
        if (MARK) touch_meta(A, &A.nodes[ni], (int)sizeof(DNode));
        uint32_t axis = n.meta & 3u;
        if (axis == kLeafAxis) return (int)n.child;
        if (LOD && (n.meta >> 8)) {
            // a kind-(a) node: stop here when the cells of its coarse patch project to fewer than
            // lod pixels at the segment start; the segment is then [tmin, tmax] across the node
            const int vl = A.nleaves + (int)(n.meta >> 8) - 1;
            if (MARK) {
                touch_meta(A, &A.leaves[vl], (int)sizeof(DLeaf));
                touch_meta(A, &A.patches[A.leaves[vl].patch], (int)sizeof(DPatch));
            }
            const double h = A.patches[A.leaves[vl].patch].step;
            const double foot = A.ortho ? A.lod_pix : tmin * A.lod_pix;
            if (h < A.lod * foot) return vl;
        }
        double oa = sel3(axis, R.o[0], R.o[1], R.o[2]);
        double da = sel3(axis, R.d[0], R.d[1], R.d[2]);
        double s = n.split;
        uint32_t low = n.child, high = low + 1;
        if (da == 0.0) {
            ni = oa < s ? low : high;
        } else {
            bool near_low = (oa < s) || (oa == s && da < 0.0);
            uint32_t nearc = near_low ? low : high, farc = near_low ? high : low;
            double ts = (s - oa) * sel3(axis, R.invd[0], R.invd[1], R.invd[2]);
            if (ts <= 0.0 || ts >= tmax) ni = nearc;
            else if (ts <= tmin) ni = farc;
            else { ni = nearc; tmax = ts; open = false; }
        }
        if (open) start = ni;
    }
    return -1;
}

// kD-restart: descend for the ray interval [tmin, tmax] (tmax the ray's exit from the clip box,
// the same on every call for one ray; `start` 0 before the first call); returns the leaf id and
// shrinks tmax to the leaf's exit.  Returns -1 if the walk exceeds the tree depth.
__device__ __forceinline__ int descend(const RenderArgs &A, const Ray &R, double tmin, double &tmax, uint32_t &start) {
    return A.lod_on ? descend_walk<true>(A, R, tmin, tmax, start) : descend_walk<false>(A, R, tmin, tmax, start);
}

// The same from the root (no push-down).
__device__ __forceinline__ int descend(const RenderArgs &A, const Ray &R, double tmin, double &tmax) {
    uint32_t start = 0;
    return descend(A, R, tmin, tmax, start);
}

// The metadata a recorded segment read: the nodes from the root to its leaf (the push-down
// walks read a subset of them, the restarts before it the rest), its leaf record and the
// patch header.
__device__ __forceinline__ void touch_segment_meta(const RenderArgs &A, const Ray &R, double tcur, int leaf) {
    double tmax = R.t1;
    uint32_t start = 0;
    if (A.lod_on) descend_walk<true, true>(A, R, tcur, tmax, start);
    else descend_walk<false, true>(A, R, tcur, tmax, start);
    touch_meta(A, &A.leaves[leaf], (int)sizeof(DLeaf));
    if (A.leaves[leaf].patch >= 0) touch_meta(A, &A.patches[A.leaves[leaf].patch], (int)sizeof(DPatch));
}

// Leaf holding point x (half-open comparisons against the split planes), descending from
// node `start` (the root, or a node known to hold x).  MARK: nodes read are marked.
template <bool MARK = false>
__device__ __forceinline__ int locate_leaf(const RenderArgs &A, const double x[3], uint32_t start = 0) {
    uint32_t ni = start;
    for (int it = 0; it <= A.depth; it++) {
        DNode n = A.nodes[ni];
        if (MARK) touch_meta(A, &A.nodes[ni], (int)sizeof(DNode));
        uint32_t axis = n.meta & 3u;
        if (axis == kLeafAxis) return (int)n.child;
        ni = sel3(axis, x[0], x[1], x[2]) < n.split ? n.child : n.child + 1;
    }
    return -1;
}

__device__ __forceinline__ int leaf_level(const DLeaf &L) { return (int)(L.level_flags & 0xffu); }

// ------------------------------------------------------------------------------------------
// FP32 sampling
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ float lerpf(float a, float b, float f) { return a + f * (b - a); }

struct PatchView {
    const float *brick;
    int px, pxy, nx, ny, nz;          // linear: row and slab strides; micro-bricks: 64 nbx, 64 nbx nby;
                                      // halo rows: 128 nbx, 128 nbx nby
};

// Halo-row layout (2): the padded brick is cut into 4x4x4-cell blocks; a block stores its 16
// x-rows (y fastest, then z) of 8 floats each, holding padded x indices 4 bx - 1 .. 4 bx + 6, so
// the four x cells a stencil row needs lie in one row of the block chosen by the stencil's first
// core cell, and load as one vector.  Offset of padded x index x in the block column bx:
__device__ __forceinline__ int halo_x(int x, int bx) { return x + 1 + 124 * bx; }
__device__ __forceinline__ int halo_y(const PatchView &pv, int j) { return (j >> 2) * pv.px + (j & 3) * 8; }
__device__ __forceinline__ int halo_z(const PatchView &pv, int k) { return (k >> 2) * pv.pxy + (k & 3) * 32; }

// LAY: the brick layout when known at compile time (0, 1, 2), else -1 (read from A.layout).
template <int LAY = -1>
__device__ __forceinline__ int layout_of(const RenderArgs &A) { return LAY >= 0 ? LAY : A.layout; }

template <int LAY = -1>
__device__ __forceinline__ PatchView patch_view(const RenderArgs &A, const DPatch &P) {
    const int lay = layout_of<LAY>(A);
    PatchView v;
    v.brick = A.pool + P.off;
    v.nx = P.n[0];
    v.ny = P.n[1];
    v.nz = P.n[2];
    if (lay == 1) {
        v.px = 64 * P.nb[0];
        v.pxy = v.px * P.nb[1];
    } else if (lay == 2) {
        v.px = 128 * P.nb[0];
        v.pxy = v.px * P.nb[1];
    } else {
        v.px = v.nx + 2;
        v.pxy = v.px * (v.ny + 2);
    }
    return v;
}

// Trilinear value of a padded brick at patch-local continuous index q (cell centres at
// integers; index -1 and n are the ghost layer).  Indices are clamped into the brick.
template <bool REC, int LAY = -1>
__device__ __forceinline__ float trilinear(const RenderArgs &A, const PatchView &pv, float qx, float qy, float qz) {
    const int lay = layout_of<LAY>(A);
    float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    int ix = min(max((int)fx, -1), pv.nx - 1);
    int iy = min(max((int)fy, -1), pv.ny - 1);
    int iz = min(max((int)fz, -1), pv.nz - 1);
    fx = qx - (float)ix;
    fy = qy - (float)iy;
    fz = qz - (float)iz;
    typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
    float v000, v100, v010, v110, v001, v101, v011, v111;
    if (lay == 1) {
        // 4^3 micro-bricks: the +1 neighbour is in the same block unless the index is 3 mod 4
        const int i = ix + 1, j = iy + 1, k = iz + 1;
        const float *b = pv.brick + ((k >> 2) * pv.pxy + (j >> 2) * pv.px + (i >> 2) * 64 + (k & 3) * 16 + (j & 3) * 4 + (i & 3));
        const int dx = (i & 3) == 3 ? 61 : 1;
        const int dy = (j & 3) == 3 ? pv.px - 12 : 4;
        const int dz = (k & 3) == 3 ? pv.pxy - 48 : 16;
        if (REC && A.touch) {   // measurement only: mark the eight cells read
            const uint64_t base = (uint64_t)(b - A.pool);
            const uint64_t offs[8] = {0, (uint64_t)dx, (uint64_t)dy, (uint64_t)(dx + dy), (uint64_t)dz, (uint64_t)(dz + dx),
                                      (uint64_t)(dz + dy), (uint64_t)(dz + dy + dx)};
            #pragma unroll
            for (int c = 0; c < 8; c++) atomicOr(&A.touch[(base + offs[c]) >> 5], 1u << ((base + offs[c]) & 31));
        }
        v000 = b[0]; v100 = b[dx]; v010 = b[dy]; v110 = b[dy + dx];
        v001 = b[dz]; v101 = b[dz + dx]; v011 = b[dz + dy]; v111 = b[dz + dy + dx];
    } else {
        // linear and halo-row layouts: each x pair is one 8-byte row load (the packer pads the
        // pool on both ends; a halo row always holds the pair)
        const float *r[2][2];
        if (lay == 2) {
            const float *bx0 = pv.brick + halo_x(ix + 1, (ix + 1) >> 2);
            const int y0 = halo_y(pv, iy + 1), y1 = halo_y(pv, iy + 2), z0 = halo_z(pv, iz + 1), z1 = halo_z(pv, iz + 2);
            r[0][0] = bx0 + y0 + z0; r[1][0] = bx0 + y1 + z0; r[0][1] = bx0 + y0 + z1; r[1][1] = bx0 + y1 + z1;
        } else {
            const float *b = pv.brick + (ix + 1) + (iy + 1) * pv.px + (iz + 1) * pv.pxy;
            r[0][0] = b; r[1][0] = b + pv.px; r[0][1] = b + pv.pxy; r[1][1] = b + pv.pxy + pv.px;
        }
        if (REC && A.touch) {
            #pragma unroll
            for (int c = 0; c < 8; c++) {
                const uint64_t e = (uint64_t)(r[(c >> 1) & 1][(c >> 2) & 1] + (c & 1) - A.pool);
                atomicOr(&A.touch[e >> 5], 1u << (e & 31));
            }
        }
        const f2u r00 = *(const f2u *)r[0][0], r10 = *(const f2u *)r[1][0], r01 = *(const f2u *)r[0][1], r11 = *(const f2u *)r[1][1];
        v000 = r00.x; v100 = r00.y; v010 = r10.x; v110 = r10.y; v001 = r01.x; v101 = r01.y; v011 = r11.x; v111 = r11.y;
    }
    float c00 = lerpf(v000, v100, fx), c10 = lerpf(v010, v110, fx);
    float c01 = lerpf(v001, v101, fx), c11 = lerpf(v011, v111, fx);
    float c0 = lerpf(c00, c10, fy), c1 = lerpf(c01, c11, fy);
    return lerpf(c0, c1, fz);
}

// Trilinear value F(q) and the six tap values F(q + e_a) (Fp) and F(q - e_a) (Fm) of a padded
// brick.  The taps use the centre's weights shifted by one cell, so the seven stencils read 32
// distinct cells: the 2x2x2 core and a 2x2 pair of cells beyond it on each side of each axis.
// The centre must lie in the brick's interior (patch-local index range [-0.5, n - 0.5]); a tap
// is exact when it also lies there, and the arm reads of a tap that does not are clamped into
// the brick (the caller replaces that tap's value).
template <bool REC, int LAY = -1>
__device__ __forceinline__ float trilinear_taps(const RenderArgs &A, const PatchView &pv, float qx, float qy,
                                                float qz, float Fp[3], float Fm[3]) {
    const int lay = layout_of<LAY>(A);
    float fx = floorf(qx), fy = floorf(qy), fz = floorf(qz);
    const int ix = min(max((int)fx, -1), pv.nx - 1);
    const int iy = min(max((int)fy, -1), pv.ny - 1);
    const int iz = min(max((int)fz, -1), pv.nz - 1);
    fx = qx - (float)ix;
    fy = qy - (float)iy;
    fz = qz - (float)iz;
    // padded index ix + d holds cell ix - 1 + d; the arms (d = 0, 3) are clamped to [0, n + 1]
    int xo[4], yo[4], zo[4];
    const int hbx = (ix + 1) >> 2;        // halo rows: the block column of the first core cell
    #pragma unroll
    for (int d = 0; d < 4; d++) {
        const int i = d == 0 ? max(ix, 0) : (d == 3 ? min(ix + 3, pv.nx + 1) : ix + d);
        const int j = d == 0 ? max(iy, 0) : (d == 3 ? min(iy + 3, pv.ny + 1) : iy + d);
        const int k = d == 0 ? max(iz, 0) : (d == 3 ? min(iz + 3, pv.nz + 1) : iz + d);
        if (lay == 1) {
            xo[d] = (i >> 2) * 64 + (i & 3);
            yo[d] = (j >> 2) * pv.px + (j & 3) * 4;
            zo[d] = (k >> 2) * pv.pxy + (k & 3) * 16;
        } else if (lay == 2) {
            xo[d] = halo_x(ix + d, hbx);
            yo[d] = halo_y(pv, j);
            zo[d] = halo_z(pv, k);
        } else {
            xo[d] = i;
            yo[d] = j * pv.px;
            zo[d] = k * pv.pxy;
        }
    }
    const float *b = pv.brick;
    // c[x][y][z] for the core (indices 1, 2 on every axis) and the arms (0 or 3 on one axis)
    float core[2][2][2], ax[2][2][2], ay[2][2][2], az[2][2][2];
    if (lay != 1) {
        // linear and halo-row layouts: the four x cells of a core row are one 16-byte load and
        // each arm row pair one 8-byte load (12 loads instead of 32).  In the linear layout a
        // row load may touch the float before or after the brick row (the arms of a tap that
        // leaves the brick, replaced later); the packer pads the pool by 64 floats on both ends
        // so such reads stay in the allocation.  A halo row holds all four.
        typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
        typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
        // padded x index ix (holding cell ix - 1), unclamped
        const float *row0 = b + (lay == 2 ? halo_x(ix, hbx) : ix);
        #pragma unroll
        for (int v = 0; v < 2; v++)
            #pragma unroll
            for (int w = 0; w < 2; w++) {
                const f4u r = *(const f4u *)(row0 + yo[1 + v] + zo[1 + w]);
                ax[0][v][w] = r.x; core[0][v][w] = r.y; core[1][v][w] = r.z; ax[1][v][w] = r.w;
            }
        #pragma unroll
        for (int u = 0; u < 2; u++)
            #pragma unroll
            for (int w = 0; w < 2; w++) {
                const f2u ry = *(const f2u *)(row0 + 1 + yo[3 * u] + zo[1 + w]);
                ay[u][0][w] = ry.x; ay[u][1][w] = ry.y;
                const f2u rz = *(const f2u *)(row0 + 1 + yo[1 + w] + zo[3 * u]);
                az[u][0][w] = rz.x; az[u][1][w] = rz.y;
            }
    } else
    #pragma unroll
    for (int u = 0; u < 2; u++)
        #pragma unroll
        for (int v = 0; v < 2; v++)
            #pragma unroll
            for (int w = 0; w < 2; w++) {
                core[u][v][w] = b[xo[1 + u] + yo[1 + v] + zo[1 + w]];
                ax[u][v][w] = b[xo[3 * u] + yo[1 + v] + zo[1 + w]];      // x arm: side u, core (y, z)
                ay[u][v][w] = b[xo[1 + v] + yo[3 * u] + zo[1 + w]];      // y arm: side u, core (x, z)
                az[u][v][w] = b[xo[1 + v] + yo[1 + w] + zo[3 * u]];      // z arm: side u, core (x, y)
            }
    if (REC && A.touch) {   // measurement only: mark the 32 cells read
        const uint64_t base = (uint64_t)(b - A.pool);
        #pragma unroll
        for (int u = 0; u < 2; u++)
            #pragma unroll
            for (int v = 0; v < 2; v++)
                #pragma unroll
                for (int w = 0; w < 2; w++) {
                    const uint64_t e[4] = {base + (uint64_t)(xo[1 + u] + yo[1 + v] + zo[1 + w]),
                                           base + (uint64_t)(xo[3 * u] + yo[1 + v] + zo[1 + w]),
                                           base + (uint64_t)(xo[1 + v] + yo[3 * u] + zo[1 + w]),
                                           base + (uint64_t)(xo[1 + v] + yo[1 + w] + zo[3 * u])};
                    #pragma unroll
                    for (int c = 0; c < 4; c++) atomicOr(&A.touch[e[c] >> 5], 1u << (e[c] & 31));
                }
    }
    // value: the core's trilinear
    const float c00 = lerpf(core[0][0][0], core[1][0][0], fx), c10 = lerpf(core[0][1][0], core[1][1][0], fx);
    const float c01 = lerpf(core[0][0][1], core[1][0][1], fx), c11 = lerpf(core[0][1][1], core[1][1][1], fx);
    const float F = lerpf(lerpf(c00, c10, fy), lerpf(c01, c11, fy), fz);
    // F(q +- e_x): the x-lerp moves one cell, the (y, z) weights stay
    float px[2][2], mx[2][2], py[2][2], my[2][2], pz[2][2], mz[2][2];
    #pragma unroll
    for (int v = 0; v < 2; v++)
        #pragma unroll
        for (int w = 0; w < 2; w++) {
            px[v][w] = lerpf(core[1][v][w], ax[1][v][w], fx);
            mx[v][w] = lerpf(ax[0][v][w], core[0][v][w], fx);
            py[v][w] = lerpf(core[v][1][w], ay[1][v][w], fy);
            my[v][w] = lerpf(ay[0][v][w], core[v][0][w], fy);
            pz[v][w] = lerpf(core[v][w][1], az[1][v][w], fz);
            mz[v][w] = lerpf(az[0][v][w], core[v][w][0], fz);
        }
    Fp[0] = lerpf(lerpf(px[0][0], px[1][0], fy), lerpf(px[0][1], px[1][1], fy), fz);
    Fm[0] = lerpf(lerpf(mx[0][0], mx[1][0], fy), lerpf(mx[0][1], mx[1][1], fy), fz);
    Fp[1] = lerpf(lerpf(py[0][0], py[1][0], fx), lerpf(py[0][1], py[1][1], fx), fz);
    Fm[1] = lerpf(lerpf(my[0][0], my[1][0], fx), lerpf(my[0][1], my[1][1], fx), fz);
    Fp[2] = lerpf(lerpf(pz[0][0], pz[1][0], fx), lerpf(pz[0][1], pz[1][1], fx), fy);
    Fm[2] = lerpf(lerpf(mz[0][0], mz[1][0], fx), lerpf(mz[0][1], mz[1][1], fx), fy);
    return F;
}

// Brick and patch-local position of world point x located in the tree; false where no patch
// holds data or x is outside B (closed).
template <bool REC, int LAY = -1>
__device__ __forceinline__ bool locate_brick(const RenderArgs &A, const double x[3], PatchView &pv, float q[3],
                                             Counters &cnt, uint32_t start = 0) {
#pragma clang fp contract(off)
    #pragma unroll
    for (int a = 0; a < 3; a++)
        if (x[a] < A.box_lo[a] || x[a] > A.box_hi[a]) return false;
    int leaf = (REC && A.touch_meta) ? locate_leaf<true>(A, x, start) : locate_leaf(A, x, start);
    if (REC) cnt.desc++;
    if (leaf < 0) return false;
    if (REC && A.touch_meta) touch_meta(A, &A.leaves[leaf], (int)sizeof(DLeaf));
    int p = A.leaves[leaf].patch;
    if (p < 0) return false;
    const DPatch &P = A.patches[p];
    if (REC && A.touch_meta) touch_meta(A, &P, (int)sizeof(DPatch));
    pv = patch_view<LAY>(A, P);
    #pragma unroll
    for (int a = 0; a < 3; a++) q[a] = (float)((x[a] - P.lo[a]) * P.inv_h[a] - 0.5);
    return true;
}

// Per-segment sampling state: n midpoint samples of step delta on [ta, tb] (Section 5.3:
// the step is proportional to the leaf level's cell size).
enum { kTapSame = 0, kTapLocate = 1, kTapUnsure = 2, kTapFace = 3 };
constexpr float kTapMargin = 1e-3f;   // cells; far above the fp32 error of patch-local positions

struct Segment {
    PatchView pv;
    float q0[3], dq[3], dl;           // patch-local start, step, delta * log2(e)
    double ta, delta;
    float fs_lo[3], fs_hi[3];         // all six taps of a sample stay in this brick (with the
                                      // classification margin) when every q_a is in [fs_lo, fs_hi);
                                      // seg_box() recovers the leaf box from them
    uint32_t safe;                    // faces across which a gradient tap stays in this brick
    int leaf, patch, n;
};

// Sample count of a segment [ta, tb] of a leaf of patch P: n = max(1, ceil((tb - ta) / step -
// 2^-20)) with step = step_frac h^l (Section 5.3; the 2^-20 keeps ratios within rounding of an
// integer from gaining a sample).
__device__ __forceinline__ int segment_samples(const RenderArgs &A, const DPatch &P, double ta, double tb) {
#pragma clang fp contract(off)
    const double step = (double)A.step_frac * (A.uniform_step ? A.step_fine : P.step);
    const double ratio = (tb - ta) / step;
    const double nn = ceil(ratio - 0x1p-20);
    return nn < 1.0 ? 1 : (int)nn;
}

// The sampling state of a segment [ta, tb] of leaf L; n: its sample count when known
// (segment_samples), else 0.
template <bool LIT, int LAY = -1>
__device__ __forceinline__ void setup_segment(const RenderArgs &A, const Ray &R, const DLeaf &L, int leaf, double ta,
                                              double tb, Segment &S, int n = 0) {
    const DPatch &P = A.patches[L.patch];
    S.n = n > 0 ? n : segment_samples(A, P, ta, tb);
    {
#pragma clang fp contract(off)
        S.delta = (tb - ta) / (double)S.n;
    }
    S.ta = ta;
    S.pv = patch_view<LAY>(A, P);
    #pragma unroll
    for (int a = 0; a < 3; a++) {
        S.q0[a] = (float)(((R.o[a] - P.lo[a]) + ta * R.d[a]) * P.inv_h[a] - 0.5);
        S.dq[a] = (float)(S.delta * R.d[a] * P.inv_h[a]);
    }
    S.dl = (float)S.delta * 1.44269504088896340736f;
    if (LIT) {
        S.safe = (L.level_flags >> 8) & 0x3fu;
        #pragma unroll
        for (int a = 0; a < 3; a++) {
            // leaf box in patch-local continuous cell coordinates; a tap q -+ 1 stays in the brick
            // while inside it, or inside the one-cell slab beyond a face whose slab belongs to
            // the same patch
            const float lq_lo = (float)((L.lo[a] - P.lo[a]) * P.inv_h[a] - 0.5);
            const float lq_hi = (float)((L.hi[a] - P.lo[a]) * P.inv_h[a] - 0.5);
            const float lo = lq_lo - (((S.safe >> (2 * a)) & 1u) ? 1.f : 0.f);
            const float hi = lq_hi + (((S.safe >> (2 * a + 1)) & 1u) ? 1.f : 0.f);
            S.fs_lo[a] = lo + 1.f + kTapMargin;
            S.fs_hi[a] = hi - 1.f - kTapMargin;
        }
    }
    S.leaf = leaf;
    S.patch = L.patch;
}

struct SampleVals {
    float F, r, g, b, sig, alpha, shade, f;
    int i0;
    float gv[3], dot, den;
};


// Leaf box along axis b in patch-local cell coordinates, recovered from the tap window (within
// a few fp32 ulps, far below the classification margin).
__device__ __forceinline__ void seg_box(const Segment &S, int b, float &lo, float &hi) {
    lo = S.fs_lo[b] - (1.f + kTapMargin) + (((S.safe >> (2 * b)) & 1u) ? 1.f : 0.f);
    hi = S.fs_hi[b] + (1.f + kTapMargin) - (((S.safe >> (2 * b + 1)) & 1u) ? 1.f : 0.f);
}

// Where does the gradient tap q (the sample moved by +-1 cell along axis a) read its value?
// Decided in fp32 patch-local coordinates when every comparison clears the margin.
__device__ __forceinline__ int classify_tap_fp32(const Segment &S, const float q[3], int a, int sgn) {
    int out_axis = -1;
    #pragma unroll
    for (int b = 0; b < 3; b++) {
        float lo, hi;
        seg_box(S, b, lo, hi);
        const bool in_sure = q[b] >= lo + kTapMargin && q[b] < hi - kTapMargin;
        const bool out_sure = q[b] < lo - kTapMargin || q[b] >= hi + kTapMargin;
        if (!in_sure && !out_sure) return kTapUnsure;
        if (out_sure) {
            if (b != a) return kTapLocate;
            out_axis = b;
        }
    }
    if (out_axis < 0) return kTapSame;
    const uint32_t face = 2u * a + (sgn ? 0u : 1u);
    // inside the one-cell slab beyond the face?
    float alo, ahi;
    seg_box(S, a, alo, ahi);
    const float lim = sgn ? alo - 1.f : ahi + 1.f;
    const float qa = q[a];
    const bool in_slab = sgn ? qa >= lim + kTapMargin : qa < lim - kTapMargin;
    const bool out_slab = sgn ? qa < lim - kTapMargin : qa >= lim + kTapMargin;
    if (in_slab) return ((S.safe >> face) & 1u) ? kTapSame : kTapFace;
    if (out_slab) return kTapLocate;
    return kTapUnsure;
}

// Exact FP64 decision (same comparisons as the oracle's point location), for taps near a face.
__device__ __forceinline__ int classify_tap_fp64(const RenderArgs &A, int leaf, int patch, uint32_t safe,
                                                 const double xt[3], int a, int sgn) {
#pragma clang fp contract(off)
    const DLeaf &L = A.leaves[leaf];
    const DPatch &P = A.patches[patch];
    bool in_leaf = true, others = true;
    #pragma unroll
    for (int b = 0; b < 3; b++) {
        const bool inb = xt[b] >= L.lo[b] && xt[b] < L.hi[b];
        in_leaf = in_leaf && inb;
        if (b != a) others = others && inb;
    }
    if (in_leaf) return kTapSame;
    const uint32_t face = 2u * a + (sgn ? 0u : 1u);
    if (!others) return kTapLocate;
    const double lim = sgn ? L.lo[a] - P.h[a] : L.hi[a] + P.h[a];
    const bool in_slab = sgn ? (xt[a] >= lim && xt[a] < L.lo[a]) : (xt[a] >= L.hi[a] && xt[a] < lim);
    if (!in_slab) return kTapLocate;
    return ((safe >> face) & 1u) ? kTapSame : kTapFace;
}

__device__ __forceinline__ int classify_tap_fp64(const RenderArgs &A, const Segment &S, const double xt[3], int a,
                                                 int sgn) {
    return classify_tap_fp64(A, S.leaf, S.patch, S.safe, xt, a, sgn);
}

// Interior cell (i, j, k) of a padded brick (0 <= index < n).
template <int LAY = -1>
__device__ __forceinline__ float brick_cell(const RenderArgs &A, const PatchView &pv, int i, int j, int k) {
    const int lay = layout_of<LAY>(A);
    i++;
    j++;
    k++;
    if (lay == 1) return pv.brick[(k >> 2) * pv.pxy + (j >> 2) * pv.px + (i >> 2) * 64 + (k & 3) * 16 + (j & 3) * 4 + (i & 3)];
    if (lay == 2) return pv.brick[halo_x(i, i >> 2) + halo_y(pv, j) + halo_z(pv, k)];
    return pv.brick[i + j * pv.px + k * pv.pxy];
}

// Index of the cell holding world coordinate x along one axis of a patch, as the definition
// reads: floor((x - lo) / h), clamped into the patch (FP64, correctly rounded).
__device__ __forceinline__ int cell_index(double x, double lo, double h, int n) {
#pragma clang fp contract(off)
    const double c = floor((x - lo) / h);
    return c < 0.0 ? 0 : (c >= (double)n ? n - 1 : (int)c);
}

// Nearest-cell value of world point x located in the tree; false where no patch holds data or
// x is outside B (closed).
template <bool REC, int LAY = -1>
__device__ __forceinline__ bool nearest_at(const RenderArgs &A, const double x[3], float *val, Counters &cnt,
                                           uint32_t start = 0) {
    #pragma unroll
    for (int a = 0; a < 3; a++)
        if (x[a] < A.box_lo[a] || x[a] > A.box_hi[a]) return false;
    const int leaf = locate_leaf(A, x, start);
    if (REC) cnt.desc++;
    if (leaf < 0) return false;
    const int p = A.leaves[leaf].patch;
    if (p < 0) return false;
    const DPatch &P = A.patches[p];
    const PatchView pv = patch_view<LAY>(A, P);
    *val = brick_cell<LAY>(A, pv, cell_index(x[0], P.lo[0], P.h[0], P.n[0]), cell_index(x[1], P.lo[1], P.h[1], P.n[1]),
                      cell_index(x[2], P.lo[2], P.h[2], P.n[2]));
    return true;
}

// Classes of the six gradient taps q +- e_a of a sample at patch-local q (2 bits per tap
// t = 2 a + sgn, sgn = 1 for the minus side; 0: in the brick), decided in fp32 against the tap
// window; a class of kTapUnsure is decided later in FP64.
__device__ __forceinline__ uint32_t classify_taps(const Segment &S, float qx, float qy, float qz) {
    const float qc[3] = {qx, qy, qz};
    uint32_t clsbits = 0;
    const bool inner = qx >= S.fs_lo[0] && qx < S.fs_hi[0] && qy >= S.fs_lo[1] && qy < S.fs_hi[1] &&
                       qz >= S.fs_lo[2] && qz < S.fs_hi[2];
    if (!inner) {
        // With the sample inside the leaf box by the margin on every axis, a tap can only leave
        // the box along its own axis, so that axis alone decides (the same classes as the full
        // test below, which the rare samples within the margin of a box face take).
        float lo[3], hi[3];
        bool boxed = true;
        #pragma unroll
        for (int b = 0; b < 3; b++) {
            seg_box(S, b, lo[b], hi[b]);
            boxed = boxed && qc[b] >= lo[b] + kTapMargin && qc[b] < hi[b] - kTapMargin;
        }
        if (boxed) {
            #pragma unroll
            for (int a = 0; a < 3; a++)
                #pragma unroll
                for (int sgn = 0; sgn < 2; sgn++) {
                    const float x = qc[a] + (sgn ? -1.f : 1.f);
                    int c;
                    if (x >= lo[a] + kTapMargin && x < hi[a] - kTapMargin) {
                        c = kTapSame;
                    } else if (x < lo[a] - kTapMargin || x >= hi[a] + kTapMargin) {
                        // beyond the face: inside the one-cell slab there?
                        const uint32_t face = 2u * a + (sgn ? 0u : 1u);
                        const float lim = sgn ? lo[a] - 1.f : hi[a] + 1.f;
                        const bool in_slab = sgn ? x >= lim + kTapMargin : x < lim - kTapMargin;
                        const bool out_slab = sgn ? x < lim - kTapMargin : x >= lim + kTapMargin;
                        c = in_slab ? (((S.safe >> face) & 1u) ? kTapSame : kTapFace)
                                    : (out_slab ? kTapLocate : kTapUnsure);
                    } else {
                        c = kTapUnsure;
                    }
                    clsbits |= (uint32_t)c << (2 * (2 * a + sgn));
                }
        } else {
            #pragma unroll
            for (int a = 0; a < 3; a++)
                #pragma unroll
                for (int sgn = 0; sgn < 2; sgn++) {
                    float qt[3] = {qc[0], qc[1], qc[2]};
                    qt[a] += sgn ? -1.f : 1.f;
                    clsbits |= (uint32_t)classify_tap_fp32(S, qt, a, sgn) << (2 * (2 * a + sgn));
                }
        }
    }
    return clsbits;
}

// In-brick part of a lit sample at patch-local q: the value F and the six taps F(q +- e_a) from
// one fused stencil of the segment's brick, and the classes of the taps (classify_taps).
template <bool REC, int LAY = -1>
__device__ __forceinline__ uint32_t lit_stencil(const RenderArgs &A, const Segment &S, float qx, float qy, float qz,
                                                float &F, float Fp[3], float Fm[3]) {
    const uint32_t clsbits = classify_taps(S, qx, qy, qz);
    F = trilinear_taps<REC, LAY>(A, S.pv, qx, qy, qz, Fp, Fm);
    return clsbits;
}

// FP64 position of sample k of a segment, o + t_k d (the point the gradient taps move from).
__device__ __forceinline__ void sample_point(const Ray &R, const Segment &S, int k, double xs[3]) {
#pragma clang fp contract(off)
    const double tk = S.ta + ((double)k + 0.5) * S.delta;
    #pragma unroll
    for (int b = 0; b < 3; b++) xs[b] = R.o[b] + tk * R.d[b];
}

// Gradient tap point xs +- h^l e_a of a sample at FP64 position xs in patch `patch`.
__device__ __forceinline__ void tap_point(const RenderArgs &A, int patch, const double xs[3], int a, int sgn,
                                          double xt[3]) {
#pragma clang fp contract(off)
    const double hl = A.patches[patch].h[a];
    const double xa = sel3(a, xs[0], xs[1], xs[2]);
    const double xn = sgn ? xa - hl : xa + hl;
    #pragma unroll
    for (int b = 0; b < 3; b++) xt[b] = b == a ? xn : xs[b];
}

// The taps of a lit sample that leave its brick (classes in clsbits, as lit_stencil returns
// them), one at a time: each chooses a brick and a position in it, then one trilinear read
// replaces Fp or Fm.  A tap beyond a face whose one-cell slab has a single owner patch is
// mapped into that patch's brick (the face record of the leaf); otherwise the exact FP64 tap
// point xs +- h^l e_a is located by a descent from the rope node holding the slab, else from
// the root.  leaf, patch and safe describe the sample's segment, own its brick (null: read
// from the patch header when a tap needs it); xs is the sample's FP64 position, (qx, qy, qz)
// its patch-local position.  Returns bit t set where tap t holds data.
template <bool REC, int LAY = -1>
__device__ __forceinline__ uint32_t resolve_taps(const RenderArgs &A, int leaf, int patch, uint32_t safe,
                                                 const PatchView *own, const double xs[3], float qx, float qy,
                                                 float qz, uint32_t clsbits, float Fp[3], float Fm[3],
                                                 Counters &cnt) {
    uint32_t okbits = 0x3fu;
    uint32_t todo = 0;
    #pragma unroll
    for (int t = 0; t < 6; t++) todo |= ((clsbits >> (2 * t)) & 3u) ? (1u << t) : 0u;
    while (todo) {
        const int t = __builtin_ctz(todo);
        todo &= todo - 1u;
        const int a = t >> 1, sgn = t & 1;
        int c = (int)((clsbits >> (2 * t)) & 3u);
        const float step = sgn ? -1.f : 1.f;
        const float qt0 = qx + (a == 0 ? step : 0.f), qt1 = qy + (a == 1 ? step : 0.f),
                    qt2 = qz + (a == 2 ? step : 0.f);
        // the exact FP64 tap point, formed near a face and for descents only
        double xt[3] = {0.0, 0.0, 0.0};
        const bool exact = c != kTapFace;
        if (exact) tap_point(A, patch, xs, a, sgn, xt);
        if (REC && c == kTapUnsure) cnt.unsure++;
        if (c == kTapUnsure) c = classify_tap_fp64(A, leaf, patch, safe, xt, a, sgn);
        PatchView pv;
        float q0 = qt0, q1 = qt1, q2 = qt2;
        bool ok = true;
        if (c == kTapSame) {
            pv = own ? *own : patch_view<LAY>(A, A.patches[patch]);
        } else {
            const DFaceXf X = c == kTapFace ? A.face_xf[6 * leaf + 2 * a + (sgn ? 0 : 1)] : DFaceXf{};
            if (REC && A.touch_meta && c == kTapFace)
                touch_meta(A, &A.face_xf[6 * leaf + 2 * a + (sgn ? 0 : 1)], (int)sizeof(DFaceXf));
            if (c == kTapFace && X.n[0] > 0) {
                // the slab's single owner: its brick at the mapped position
                if (REC) cnt.face++;
                pv.brick = A.pool + X.off;
                pv.px = X.px;
                pv.pxy = X.pxy;
                pv.nx = X.n[0];
                pv.ny = X.n[1];
                pv.nz = X.n[2];
                q0 = qt0 * X.r + X.t[0];
                q1 = qt1 * X.r + X.t[1];
                q2 = qt2 * X.r + X.t[2];
            } else {
                // descend from the rope node holding the slab, else from the root (a slab beyond
                // B fails the box test there, except on B's closed upper faces)
                if (!exact) tap_point(A, patch, xs, a, sgn, xt);
                float qq[3];
                ok = locate_brick<REC, LAY>(A, xt, pv, qq, cnt, c == kTapFace && X.rope > 0 ? (uint32_t)X.rope : 0u);
                q0 = qq[0];
                q1 = qq[1];
                q2 = qq[2];
            }
        }
        const float Fs = ok ? trilinear<REC, LAY>(A, pv, q0, q1, q2) : 0.f;
        if (!ok) okbits &= ~(1u << t);
        // write the tap back (selects keep the arrays in registers)
        #pragma unroll
        for (int b = 0; b < 3; b++) {
            Fp[b] = (t == 2 * b) ? Fs : Fp[b];
            Fm[b] = (t == 2 * b + 1) ? Fs : Fm[b];
        }
    }
    return okbits;
}

// The pending taps (bit t of pend) of a nearest-cell lit sample, one at a time: each reads the
// cell of the finest patch holding the exact FP64 tap point xs +- h^l e_a.  A tap classified
// in the sample's own patch takes its cell from the FP64 position; beyond a face whose slab has
// a single owner, the cell under the mapped position when that is clear of the owner's cell
// faces; otherwise a descent from the slab's rope node, else from the root.  leaf, patch and
// safe describe the sample's segment, q its patch-local position, cls the fp32 classes.
// Returns bit t set where tap t holds data.
template <bool REC, int LAY = -1>
__device__ __forceinline__ uint32_t resolve_taps_nearest(const RenderArgs &A, int leaf, int patch, uint32_t safe,
                                                         const double xs[3], const float q[3], uint32_t cls,
                                                         uint32_t pend, float Fp[3], float Fm[3], Counters &cnt) {
    const DPatch &P = A.patches[patch];
    uint32_t okbits = 0x3fu;
    while (pend) {
        const int t = __builtin_ctz(pend);
        pend &= pend - 1u;
        const int a = t >> 1, sgn = t & 1;
        float qt[3] = {q[0], q[1], q[2]};
        qt[a] += sgn ? -1.f : 1.f;
        const int c = (int)((cls >> (2 * t)) & 3u);
        double xt[3] = {xs[0], xs[1], xs[2]};
        {
#pragma clang fp contract(off)
            xt[a] = sgn ? xs[a] - P.h[a] : xs[a] + P.h[a];
        }
        float val = 0.f;
        bool ok = true, done = false;
        if (REC && c == kTapUnsure) cnt.unsure++;
        const int c2 = c == kTapUnsure ? classify_tap_fp64(A, leaf, patch, safe, xt, a, sgn) : c;
        uint32_t from = 0;
        if (c2 == kTapSame) {
            // the tap lies where the sample's own patch is the finest: its cell, in FP64
            const PatchView pv = patch_view<LAY>(A, P);
            val = brick_cell<LAY>(A, pv, cell_index(xt[0], P.lo[0], P.h[0], P.n[0]),
                                  cell_index(xt[1], P.lo[1], P.h[1], P.n[1]), cell_index(xt[2], P.lo[2], P.h[2], P.n[2]));
            done = true;
        } else if (c2 == kTapFace) {
            const DFaceXf X = A.face_xf[6 * leaf + 2 * a + (sgn ? 0 : 1)];
            if (X.n[0] > 0) {
                const float qo[3] = {qt[0] * X.r + X.t[0], qt[1] * X.r + X.t[1], qt[2] * X.r + X.t[2]};
                int co[3];
                bool clear = true;
                #pragma unroll
                for (int b = 0; b < 3; b++) {
                    const float u = qo[b] + 0.5f, fl = floorf(u), fr = u - fl;
                    clear = clear && fr >= kTapMargin && fr <= 1.f - kTapMargin;
                    co[b] = min(max((int)fl, 0), X.n[b] - 1);
                }
                if (clear) {
                    PatchView pv;
                    pv.brick = A.pool + X.off;
                    pv.px = X.px;
                    pv.pxy = X.pxy;
                    pv.nx = X.n[0];
                    pv.ny = X.n[1];
                    pv.nz = X.n[2];
                    val = brick_cell<LAY>(A, pv, co[0], co[1], co[2]);
                    if (REC) cnt.face++;
                    done = true;
                }
            } else if (X.rope > 0) {
                from = (uint32_t)X.rope;
            }
        }
        if (!done) ok = nearest_at<REC, LAY>(A, xt, &val, cnt, from);
        if (!ok) okbits &= ~(1u << t);
        #pragma unroll
        for (int b = 0; b < 3; b++) {
            Fp[b] = (t == 2 * b) ? val : Fp[b];
            Fm[b] = (t == 2 * b + 1) ? val : Fm[b];
        }
    }
    return okbits;
}

// Normalised-value gradient by central differences of the taps, one-sided where a tap holds no
// data, zero where neither does.
__device__ __forceinline__ float lit_gradient_axis(const RenderArgs &A, float F, float fp, float fm, bool okp, bool okm) {
    if (okp && okm) return (fp - fm) * (0.5f * A.inv_range);
    if (okp) return (fp - F) * A.inv_range;
    if (okm) return (F - fm) * A.inv_range;
    return 0.f;
}

__device__ __forceinline__ void lit_gradient(const RenderArgs &A, float F, const float Fp[3], const float Fm[3],
                                             uint32_t okbits, float gv[3]) {
    #pragma unroll
    for (int a = 0; a < 3; a++)
        gv[a] = lit_gradient_axis(A, F, Fp[a], Fm[a], (okbits >> (2 * a)) & 1u, (okbits >> (2 * a + 1)) & 1u);
}

// Diffuse shading factor k_a + k_d |g . l| / sqrt(|g|^2 + eps^2) (Section 6), the fraction 0
// where the denominator is 0.  The reciprocal square root is the hardware's (within 1 ulp),
// which replaces a correctly rounded square root and division (some 30 instructions per lit
// sample); den = n2 / sqrt(n2) is kept for the adjoint.
__device__ __forceinline__ float lit_shade(const RenderArgs &A, const float gv[3], float &dot, float &den) {
    dot = gv[0] * A.lhat[0] + gv[1] * A.lhat[1] + gv[2] * A.lhat[2];
    const float n2 = gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2] + A.eps2;
    const float r = n2 > 0.f ? __builtin_amdgcn_rsqf(n2) : 0.f;
    den = n2 * r;
    return A.k_a + A.k_d * fabsf(dot) * r;
}

// Transfer function: colour and extinction by linear interpolation in the 256-entry LUT at the
// normalised value, and the opacity 1 - exp(-sigma delta) of one step (Sections 3 and 5.3).
__device__ __forceinline__ void lut_classify(const RenderArgs &A, const float4 *s_lut, float F, float dl, SampleVals &v) {
    v.F = F;
    const float u = __saturatef((F - A.v_lo) * A.inv_range);
    const float xs = 255.f * u;
    const int i0 = min((int)xs, 254);
    const float f = xs - (float)i0;
    const float4 La = s_lut[i0], Lb = s_lut[i0 + 1];
    v.i0 = i0;
    v.f = f;
    v.r = lerpf(La.x, Lb.x, f);
    v.g = lerpf(La.y, Lb.y, f);
    v.b = lerpf(La.z, Lb.z, f);
    v.sig = lerpf(La.w, Lb.w, f);
    // the hardware exp2 (1 ulp); its results below the normal range flush to 0, where 1 - exp2
    // is 1 either way
    v.alpha = 1.f - __builtin_amdgcn_exp2f(-v.sig * dl);
}

// Nearest-cell sampling (interp = 1): F(x) is the value of the cell of the finest patch that
// holds x.  The cell index is taken in fp32 patch-local coordinates when the point is at least
// the classification margin away from every cell face, else from the FP64 position exactly as
// defined.  (Lit nearest-cell samples take their taps through the tap queue.)
template <int LAY = -1>
__device__ __forceinline__ float nearest_value(const RenderArgs &A, const Ray &R, const Segment &S, int k, float qx,
                                               float qy, float qz) {
    const float qc[3] = {qx, qy, qz};
    int ci[3];
    bool sure = true;
    #pragma unroll
    for (int a = 0; a < 3; a++) {
        const float u = qc[a] + 0.5f, fl = floorf(u), fr = u - fl;
        sure = sure && fr >= kTapMargin && fr <= 1.f - kTapMargin;
        ci[a] = (int)fl;
    }
    if (!sure) {
        const DPatch &P = A.patches[S.patch];
        double x[3];
        sample_point(R, S, k, x);
        #pragma unroll
        for (int a = 0; a < 3; a++) ci[a] = cell_index(x[a], P.lo[a], P.h[a], P.n[a]);
    }
    ci[0] = min(max(ci[0], 0), S.pv.nx - 1);
    ci[1] = min(max(ci[1], 0), S.pv.ny - 1);
    ci[2] = min(max(ci[2], 0), S.pv.nz - 1);
    return brick_cell<LAY>(A, S.pv, ci[0], ci[1], ci[2]);
}

// Sample k of a segment, every part in place: value, LUT classification, opacity over the step,
// and (LIT) the gradient shading with taps at x +- h^l e_a, those outside the brick read where
// they land.  The adjoint, the learned kernel and the unlit forward variants sample this way.
template <bool LIT, bool REC, bool NEAR = false, int LAY = -1>
__device__ __forceinline__ void eval_sample(const RenderArgs &A, const float4 *s_lut, const Ray &R, const Segment &S,
                                            int k, SampleVals &v, Counters &cnt) {
    const float kk = (float)k + 0.5f;
    const float qx = S.q0[0] + kk * S.dq[0], qy = S.q0[1] + kk * S.dq[1], qz = S.q0[2] + kk * S.dq[2];
    float F;
    if constexpr (NEAR) {
        static_assert(!LIT, "lit nearest-cell samples take the tap queue (lit_sample_deferred)");
        F = nearest_value<LAY>(A, R, S, k, qx, qy, qz);
    } else if (LIT) {
        // value and the six taps x +- h^l e_a from this brick in one fused stencil; a tap that
        // leaves the brick is then read where it lands
        float Fp[3], Fm[3];
        const uint32_t clsbits = lit_stencil<REC, LAY>(A, S, qx, qy, qz, F, Fp, Fm);
        uint32_t okbits = 0x3fu;
        if (clsbits) {
            if (REC) cnt.split++;
            double xs[3];
            sample_point(R, S, k, xs);
            okbits = resolve_taps<REC, LAY>(A, S.leaf, S.patch, S.safe, &S.pv, xs, qx, qy, qz, clsbits, Fp, Fm, cnt);
        }
        lit_gradient(A, F, Fp, Fm, okbits, v.gv);
    } else {
        F = trilinear<REC, LAY>(A, S.pv, qx, qy, qz);
    }
    lut_classify(A, s_lut, F, S.dl, v);
    v.shade = LIT ? lit_shade(A, v.gv, v.dot, v.den) : 1.f;
}

// Unlit samples of one data segment, composited front to back (emission-absorption with early
// termination, Section 5.3).  A ray's samples depend on each other only through T, so the
// values of kUnlitBatch samples are evaluated (their brick loads in flight together) before
// they are composited one by one in sample order; the ray's dependent memory round trips fall
// by that factor.  A batch that runs past the segment's end repeats its last sample, which is
// not composited, and samples past early termination are not composited either: results are
// bit-identical to one sample at a time.  tseg: the segment's own transmittance, multiplied
// alike.  Returns the samples composited; stop: the ray terminated in this segment.
constexpr int kUnlitBatch = 4;
template <int LAY>
__device__ __forceinline__ int composite_unlit(const RenderArgs &A, const float4 *s_lut, const Ray &R,
                                               const Segment &S, float &T, float &C0, float &C1, float &C2,
                                               float &tseg, bool &stop, Counters &cnt) {
    int done = 0;
    stop = false;
    for (int k = 0; k < S.n; k += kUnlitBatch) {
        SampleVals v[kUnlitBatch];
        #pragma unroll
        for (int u = 0; u < kUnlitBatch; u++)
            eval_sample<false, false, false, LAY>(A, s_lut, R, S, min(k + u, S.n - 1), v[u], cnt);
        #pragma unroll
        for (int u = 0; u < kUnlitBatch; u++) {
            if (!stop && k + u < S.n) {
                const float wgt = T * v[u].alpha * v[u].shade;
                C0 += wgt * v[u].r;
                C1 += wgt * v[u].g;
                C2 += wgt * v[u].b;
                T *= 1.f - v[u].alpha;
                tseg *= 1.f - v[u].alpha;
                done++;
                if (T < A.t_min) stop = true;
            }
        }
        if (stop) break;
    }
    return done;
}

// ------------------------------------------------------------------------------------------
// Deferred gradient taps (lit forward kernels)
// ------------------------------------------------------------------------------------------
//
// About a fifth of the lit samples of a large view have a gradient tap outside their brick
// (trilinear), or one that needs the tree (nearest cell).  Served where they occur, nearly every
// step of a wave waits on such a tap's dependent loads (face record or tree descent, then a
// brick read) with one or two lanes busy.  Instead, the in-brick part of such a sample is
// evaluated at once (value, colour and opacity from the LUT, the in-brick taps).  Opacity and
// transmittance do not depend on the shading, so the ray marches on, and the sample's pending
// taps, gradient, shading and colour contribution wait in a per-wave queue in LDS.  When the
// queue could not take one more sample from every marching lane, the calling lanes resolve all
// queued samples together, one sample per lane.
//
// Each ray sums its colour in two accumulators, each in its own sample order: the samples
// shaded at once (in registers), and the deferred ones (in LDS, added per owner in queue
// order, which is the owner's sample order); the pixel is their sum.  So a ray's result does
// not depend on which rays share its wave or on when the queue is resolved.

// A queued sample.  Per axis, g holds the finished central difference when neither tap of
// the axis is pending, else the value of the tap that is not (or nothing).
struct TapQueue {
    double xs[3][kTapQ];           // FP64 sample position
    float q[3][kTapQ];             // patch-local position; after resolution the contribution (r, g, b)
    float g[4][kTapQ];             // F, then per axis as above
    float ta[kTapQ], lf[kTapQ];    // T alpha; LUT fraction
    int32_t leaf[kTapQ], patch[kTapQ];
    uint32_t meta[kTapQ];          // owner lane | tap classes << 6 | LUT index << 18 | safe faces << 26
    uint32_t pend[kTapQ];          // taps left to resolve (bit t)
    float cd[3][64];               // per lane: colour of its resolved deferred samples
    uint32_t count, pad_;
    unsigned long long bstart[2];  // bit j: the samples queued by one step start at slot j
};

// The block's queues (NW waves); a kernel that never calls this allocates no LDS for them.
template <int NW>
__device__ __forceinline__ TapQueue *tap_queues() {
    __shared__ TapQueue q[NW];
    return q;
}

// Orders this wave's LDS accesses (the queue is written by some lanes and read by others).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t tq_count(TapQueue &Q) {
    return __hip_atomic_load(&Q.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ unsigned long long tq_bstart(TapQueue &Q, int w) {
    return __hip_atomic_load(&Q.bstart[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ void tq_set(TapQueue &Q, uint32_t count, unsigned long long b0, unsigned long long b1) {
    __hip_atomic_store(&Q.count, count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __hip_atomic_store(&Q.bstart[0], b0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __hip_atomic_store(&Q.bstart[1], b1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// All lanes of the wave: empty queue, zero deferred colour.
__device__ __forceinline__ void tapq_init(TapQueue &Q, int lane) {
    Q.cd[0][lane] = 0.f;
    Q.cd[1][lane] = 0.f;
    Q.cd[2][lane] = 0.f;
    if (lane == 0) tq_set(Q, 0u, 0ull, 0ull);
    wave_lds_fence();
}

// The calling (active) lanes resolve every queued sample: remaining taps, gradient, shading,
// contribution; then each owner's deferred colour takes its contributions in queue order.
// TAPE (checkpointed single-camera forward, one 8x8 pixel tile per wave): each resolved sample's
// record (value, gradient) is also written to the owner ray's tape at the sample's position, so
// the adjoint need not evaluate it again.  tape_base: the tape row (ray) of lane 0, whose tile
// row holds lanes 0..7; lane o's ray is tape_base + (o / 8) * width + o % 8.
template <bool REC, int LAY = -1, bool NEAR = false, bool TAPE = false>
__device__ __forceinline__ void tapq_flush(const RenderArgs &A, const float4 *s_lut, TapQueue &Q, int lane,
                                           Counters &cnt, int64_t tape_base = -1) {
    const unsigned long long act = __ballot(1);
    const uint32_t nact = popc64(act), rank = popc64(act & lanes_below(lane));
    wave_lds_fence();
    const uint32_t n = tq_count(Q);
    for (uint32_t j = rank; j < n; j += nact) {
        const double xs[3] = {Q.xs[0][j], Q.xs[1][j], Q.xs[2][j]};
        const float F = Q.g[0][j];
        const uint32_t m = Q.meta[j], pend = Q.pend[j] & 63u;
        const uint32_t cls = (m >> 6) & 0xfffu, safe = m >> 26;
        float Fp[3], Fm[3];
        #pragma unroll
        for (int a = 0; a < 3; a++) {
            const float v = Q.g[1 + a][j];
            Fp[a] = v;                 // the in-brick side; the other is replaced below
            Fm[a] = v;
        }
        const int leaf = Q.leaf[j], patch = Q.patch[j];
        uint32_t ok = 0u;
        if ((uint32_t)leaf < (uint32_t)A.nrec && (uint32_t)patch < (uint32_t)A.npatches) {   // always
            if (NEAR) {
                const float q[3] = {Q.q[0][j], Q.q[1][j], Q.q[2][j]};
                ok = resolve_taps_nearest<REC, LAY>(A, leaf, patch, safe, xs, q, cls, pend, Fp, Fm, cnt);
            } else {
                ok = resolve_taps<REC, LAY>(A, leaf, patch, safe, nullptr, xs, Q.q[0][j], Q.q[1][j], Q.q[2][j], cls,
                                            Fp, Fm, cnt);
            }
        } else if (REC) {
            cnt.guard++;
        }
        float gv[3];
        #pragma unroll
        for (int a = 0; a < 3; a++) {
            const bool pp = (pend >> (2 * a)) & 1u, pm = (pend >> (2 * a + 1)) & 1u;
            gv[a] = (pp || pm) ? lit_gradient_axis(A, F, Fp[a], Fm[a], (ok >> (2 * a)) & 1u, (ok >> (2 * a + 1)) & 1u)
                               : Q.g[1 + a][j];
        }
        if (TAPE && tape_base >= 0) {
            const int o = (int)(m & 63u);
            const int64_t row = tape_base + (int64_t)(o >> 3) * A.width + (o & 7);
            const int64_t pos = (int64_t)(Q.pend[j] >> 6);
            if (pos < A.tape_cap) A.tape[row * A.tape_cap + pos] = make_float4(F, gv[0], gv[1], gv[2]);
        }
        float dot, den;
        const float wgt = Q.ta[j] * lit_shade(A, gv, dot, den);
        const int i0 = (int)((m >> 18) & 0xffu);
        const float f = Q.lf[j];
        const float4 La = s_lut[i0], Lb = s_lut[i0 + 1];
        Q.q[0][j] = wgt * lerpf(La.x, Lb.x, f);
        Q.q[1][j] = wgt * lerpf(La.y, Lb.y, f);
        Q.q[2][j] = wgt * lerpf(La.z, Lb.z, f);
    }
    wave_lds_fence();
    // the samples of one step have distinct owners; steps are added one after the other
    const unsigned long long b0 = tq_bstart(Q, 0), b1 = tq_bstart(Q, 1);
    #pragma unroll
    for (int w = 0; w < 2; w++) {
        unsigned long long bs = w ? b1 : b0;
        while (bs) {
            const uint32_t s = 64u * w + ctz64(bs);
            bs &= bs - 1ull;
            const uint32_t e = tapq_run_end(b0, b1, s, n);
            for (uint32_t j = s + rank; j < e; j += nact) {
                const uint32_t o = Q.meta[j] & 63u;
                Q.cd[0][o] += Q.q[0][j];
                Q.cd[1][o] += Q.q[1][j];
                Q.cd[2][o] += Q.q[2][j];
            }
            wave_lds_fence();
        }
    }
    if (rank == 0) tq_set(Q, 0u, 0ull, 0ull);
    wave_lds_fence();
}

// At the top of a step, by the marching lanes: resolve the queue first unless it has a free
// slot for each of them.
template <bool REC, int LAY = -1, bool NEAR = false>
__device__ __forceinline__ void tapq_reserve(const RenderArgs &A, const float4 *s_lut, TapQueue &Q, int lane,
                                             Counters &cnt) {
    const unsigned long long act = __ballot(1);
    if (tapq_full(tq_count(Q), act)) tapq_flush<REC, LAY, NEAR>(A, s_lut, Q, lane, cnt);
}

// Queues a lit sample whose taps in `pend` are left to resolve (all marching lanes call it in
// the same step, with a slot reserved for each; lanes with want = false queue nothing).
// Fp/Fm hold the in-brick tap values; an axis with neither tap pending is stored as its
// finished central difference, else as the in-brick side's value.
// ord: the sample's tape position (below 2^26; tape_cap, which is never written, when beyond it;
// 0 without a tape).
template <bool REC>
__device__ __forceinline__ void tapq_push(const RenderArgs &A, TapQueue &Q, int lane, bool want, const Ray &R,
                                          const Segment &S, int k, const double *xs_known, float qx, float qy,
                                          float qz, float F, const float Fp[3], const float Fm[3], uint32_t cls,
                                          uint32_t pend, float Ta, const SampleVals &v, Counters &cnt,
                                          uint32_t ord = 0) {
    const unsigned long long need = __ballot(want);
    if (!need) return;
    const unsigned long long act = __ballot(1);
    const uint32_t c0 = tq_count(Q);
    if (want) {
        if (REC) cnt.split++;
        const uint32_t j = tapq_slot(c0, need, lane);
        if (j < (uint32_t)kTapQ) {          // always: a slot per lane was reserved
            double xs[3];
            if (xs_known) {
                xs[0] = xs_known[0];
                xs[1] = xs_known[1];
                xs[2] = xs_known[2];
            } else {
                sample_point(R, S, k, xs);
            }
            Q.xs[0][j] = xs[0];
            Q.xs[1][j] = xs[1];
            Q.xs[2][j] = xs[2];
            Q.q[0][j] = qx;
            Q.q[1][j] = qy;
            Q.q[2][j] = qz;
            Q.g[0][j] = F;
            #pragma unroll
            for (int a = 0; a < 3; a++) {
                const bool pp = (pend >> (2 * a)) & 1u, pm = (pend >> (2 * a + 1)) & 1u;
                Q.g[1 + a][j] = !(pp || pm) ? lit_gradient_axis(A, F, Fp[a], Fm[a], true, true) : (pp ? Fm[a] : Fp[a]);
            }
            Q.ta[j] = Ta;
            Q.lf[j] = v.f;
            Q.leaf[j] = S.leaf;
            Q.patch[j] = S.patch;
            Q.meta[j] = (uint32_t)lane | (cls << 6) | ((uint32_t)v.i0 << 18) | (S.safe << 26);
            Q.pend[j] = pend | (ord << 6);
        } else if (REC) {
            cnt.guard++;
        }
    }
    wave_lds_fence();
    if (lane == (int)ctz64(act) && c0 < (uint32_t)kTapQ) {
        const TapqStarts b = tapq_mark(tq_bstart(Q, 0), tq_bstart(Q, 1), c0);
        tq_set(Q, tapq_count_after(c0, need), b.w0, b.w1);
    }
    wave_lds_fence();
}

// Pending taps of a classified sample: bit t where tap t leaves the brick.
__device__ __forceinline__ uint32_t pending_taps(uint32_t cls) {
    uint32_t pend = 0;
    #pragma unroll
    for (int t = 0; t < 6; t++) pend |= ((cls >> (2 * t)) & 3u) ? (1u << t) : 0u;
    return pend;
}

// The part of a lit sample after its stencil: LUT classification, then either the shading and
// colour at once (every tap in the brick) or a queue slot (tapq_push: every lane of the calling
// set takes part).  xs: the sample's FP64 position if already known (else null).  With a tape
// row, the sample's record is written (at once) or its tape position queued.  Returns alpha.
template <bool REC>
__device__ __forceinline__ float lit_consume(const RenderArgs &A, const float4 *s_lut, TapQueue &Q, int lane,
                                             const Ray &R, const Segment &S, int k, const double *xs, float qx,
                                             float qy, float qz, float F, const float Fp[3], const float Fm[3],
                                             uint32_t cls, uint32_t pend, float T, float &C0, float &C1, float &C2,
                                             Counters &cnt, float4 *trow, uint32_t *tpos) {
    SampleVals v;
    lut_classify(A, s_lut, F, S.dl, v);
    const float Ta = T * v.alpha;
    const bool defer = pend != 0;
    const uint32_t pos = trow ? *tpos : 0u;
    const uint32_t cap = (uint32_t)A.tape_cap;
    if (!defer) {
        float gv[3], dot, den;
        lit_gradient(A, F, Fp, Fm, 0x3fu, gv);
        const float wgt = Ta * lit_shade(A, gv, dot, den);
        C0 += wgt * v.r;
        C1 += wgt * v.g;
        C2 += wgt * v.b;
        if (trow && pos < cap) trow[pos] = make_float4(F, gv[0], gv[1], gv[2]);
    }
    const uint32_t ord = pos < cap ? pos : cap;
    if (trow) *tpos = pos + 1u;
    tapq_push<REC>(A, Q, lane, defer, R, S, k, xs, qx, qy, qz, F, Fp, Fm, cls, pend, Ta, v, cnt, ord);
    return v.alpha;
}

// One lit sample of a marching lane with deferred taps: the in-brick part now; the sample is
// queued when a tap leaves the brick (trilinear) or needs the tree (nearest cell), else shaded
// and added to (C0, C1, C2) at once.  Returns the opacity.  All marching lanes call it in the
// same step, after tapq_reserve.
// trow, tpos (checkpointed forward with a tape): the lane's tape row and the sample's position in
// it, advanced here; a sample shaded at once writes its record now, a queued one when resolved.
template <bool REC, int LAY = -1, bool NEAR = false>
__device__ __forceinline__ float lit_sample_deferred(const RenderArgs &A, const float4 *s_lut, TapQueue &Q, int lane,
                                                     const Ray &R, const Segment &S, int k, float T, float &C0,
                                                     float &C1, float &C2, Counters &cnt, float4 *trow = nullptr,
                                                     uint32_t *tpos = nullptr) {
    const float kk = (float)k + 0.5f;
    const float qx = S.q0[0] + kk * S.dq[0], qy = S.q0[1] + kk * S.dq[1], qz = S.q0[2] + kk * S.dq[2];
    float F, Fp[3], Fm[3];
    uint32_t cls, pend;
    double xs[3] = {0.0, 0.0, 0.0};
    bool have_xs = false;
    if (NEAR) {
        // the sample's cell and the taps one cell over in this brick; the rest needs the tree
        const float qc[3] = {qx, qy, qz};
        int ci[3];
        bool sure = true;
        #pragma unroll
        for (int a = 0; a < 3; a++) {
            const float u = qc[a] + 0.5f, fl = floorf(u), fr = u - fl;
            sure = sure && fr >= kTapMargin && fr <= 1.f - kTapMargin;
            ci[a] = (int)fl;
        }
        cls = classify_taps(S, qx, qy, qz);
        pend = sure ? pending_taps(cls) : 0x3fu;
        if (pend) {
            sample_point(R, S, k, xs);
            have_xs = true;
        }
        if (!sure) {
            const DPatch &P = A.patches[S.patch];
            #pragma unroll
            for (int a = 0; a < 3; a++) ci[a] = cell_index(xs[a], P.lo[a], P.h[a], P.n[a]);
        }
        ci[0] = min(max(ci[0], 0), S.pv.nx - 1);
        ci[1] = min(max(ci[1], 0), S.pv.ny - 1);
        ci[2] = min(max(ci[2], 0), S.pv.nz - 1);
        F = brick_cell<LAY>(A, S.pv, ci[0], ci[1], ci[2]);
        #pragma unroll
        for (int t = 0; t < 6; t++) {
            const int a = t >> 1, sgn = t & 1;
            float val = F;
            if (!((pend >> t) & 1u)) {
                int cj[3] = {ci[0], ci[1], ci[2]};
                cj[a] += sgn ? -1 : 1;
                cj[0] = min(max(cj[0], 0), S.pv.nx - 1);
                cj[1] = min(max(cj[1], 0), S.pv.ny - 1);
                cj[2] = min(max(cj[2], 0), S.pv.nz - 1);
                val = brick_cell<LAY>(A, S.pv, cj[0], cj[1], cj[2]);
            }
            if (sgn) Fm[a] = val;
            else Fp[a] = val;
        }
    } else {
        cls = lit_stencil<REC, LAY>(A, S, qx, qy, qz, F, Fp, Fm);
        pend = pending_taps(cls);
    }
    return lit_consume<REC>(A, s_lut, Q, lane, R, S, k, have_xs ? xs : nullptr, qx, qy, qz, F, Fp, Fm, cls, pend, T,
                            C0, C1, C2, cnt, trow, tpos);
}

// After the march, by all lanes of the wave: resolve what is queued; returns the lane's
// deferred colour.
template <bool REC, int LAY = -1, bool NEAR = false, bool TAPE = false>
__device__ __forceinline__ void tapq_finish(const RenderArgs &A, const float4 *s_lut, TapQueue &Q, int lane,
                                            Counters &cnt, float &D0, float &D1, float &D2, int64_t tape_base = -1) {
    if (tq_count(Q)) tapq_flush<REC, LAY, NEAR, TAPE>(A, s_lut, Q, lane, cnt, tape_base);
    wave_lds_fence();
    D0 = Q.cd[0][lane];
    D1 = Q.cd[1][lane];
    D2 = Q.cd[2][lane];
}

// ------------------------------------------------------------------------------------------
// Reductions and counters
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sumf(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void flush_counters(amr_render_stats *st, Counters c, int lane) {
    typedef unsigned long long u64;
    u64 s = wave_sum((u64)c.samples), g = wave_sum((u64)c.segments), h = wave_sum((u64)c.hit);
    u64 d = wave_sum((u64)c.desc), gu = wave_sum((u64)c.guard), to = wave_sum((u64)c.tover);
    u64 co = wave_sum((u64)c.ckover);
    u64 sp = wave_sum((u64)c.split), fa = wave_sum((u64)c.face), un = wave_sum((u64)c.unsure);
    u64 li = wave_sum((u64)c.linl);
    if (lane == 0) {
        if (s) atomicAdd(&st->samples, s);
        if (g) atomicAdd(&st->segments, g);
        if (h) atomicAdd(&st->rays_hit, h);
        if (d) atomicAdd(&st->tap_descents, d);
        if (gu) atomicAdd(&st->guard_hits, gu);
        if (to) atomicAdd(&st->trace_overflow, to);
        if (co) atomicAdd(&st->ckpt_overflow, co);
        if (sp) atomicAdd(&st->split_samples, sp);
        if (fa) atomicAdd(&st->face_taps, fa);
        if (un) atomicAdd(&st->unsure_taps, un);
        if (li) atomicAdd(&st->light_inline, li);
    }
}

// ------------------------------------------------------------------------------------------
// Host helpers
// ------------------------------------------------------------------------------------------

inline int check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return AMR_EHIP;
    }
    return AMR_OK;
}

inline int fill_args(const amr_scene *S, const amr_camera *C, const amr_render_params *P, RenderArgs *A) {
    memset(A, 0, sizeof(*A));
    if (!P->d_lut) { set_error("d_lut is NULL"); return AMR_EINVAL; }
    if (!(P->v_hi > P->v_lo)) { set_error("v_hi must exceed v_lo"); return AMR_EINVAL; }
    if (!(P->step_frac > 0.f) || !std::isfinite(P->step_frac)) { set_error("step_frac must be positive"); return AMR_EINVAL; }
    if (C->width <= 0 || C->height <= 0) { set_error("camera size must be positive"); return AMR_EINVAL; }
    A->pool = S->pool;
    A->nodes = (const DNode *)S->nodes;
    A->leaves = (const DLeaf *)S->leaves;
    A->patches = (const DPatch *)S->patches;
    A->face_xf = (const DFaceXf *)S->face_taps;
    if (P->interp != 0 && P->interp != 1) { set_error("interp must be 0 (trilinear) or 1 (nearest cell)"); return AMR_EINVAL; }
    if (P->interp == 1 && S->centering != 0) { set_error("nearest-cell sampling needs cell-centred data"); return AMR_EINVAL; }
    A->nearest = P->interp;
    if (!(P->lod >= 0.f)) { set_error("lod must be >= 0"); return AMR_EINVAL; }
    A->lod_on = P->lod > 0.f && S->nlod > 0;
    A->lod = (double)P->lod;
    A->nleaves = S->nleaves;
    A->nrec = S->nleaves + S->nlod;
    A->npatches = S->npatches;
    A->lod_pix = C->ortho ? (2.0 * C->win[1]) / (double)C->height : (2.0 * C->tan_half_fov) / (double)C->height;
    A->lut = (const float4 *)P->d_lut;
    A->touch_meta = P->d_touch_meta;
    A->meta_base = (const uint8_t *)S->nodes;
    #pragma unroll
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
    #pragma unroll
    for (int a = 0; a < 3; a++) A->lhat[a] = ln > 0.f ? P->light[a] / ln : 0.f;
    A->inv_lnorm = ln > 0.f ? 1.f / ln : 0.f;
    A->k_a = P->k_a;
    A->k_d = P->k_d;
    A->eps2 = P->eps_g * P->eps_g;
    A->uniform_step = P->uniform_step;
    if (P->lighting < 0 || P->lighting > 2) { set_error("lighting must be 0, 1 (gradient) or 2 (point light)"); return AMR_EINVAL; }
    A->lighting = P->lighting;
    for (int a = 0; a < 3; a++) A->plight[a] = (double)P->light[a];
    if (S->brick_layout < 0 || S->brick_layout > 2) { set_error("unknown brick layout"); return AMR_EINVAL; }
    A->layout = S->brick_layout;
    A->tiles_x = (C->width + 15) / 16;
    A->tiles_y = (C->height + 15) / 16;
    A->nblocks = A->tiles_x * A->tiles_y;
    A->t8x = (C->width + 7) / 8;
    A->t8y = (C->height + 7) / 8;
    A->sgrid = 1;
    while (A->sgrid * 4 < A->t8x || A->sgrid * 4 < A->t8y) A->sgrid *= 2;
    A->ckpt = (uint8_t *)P->d_ckpt;
    A->ckpt_stride = (int64_t)sizeof(Ckpt) * (1 + (int64_t)P->ckpt_max);
    A->ckpt_every = P->ckpt_every > 0 ? P->ckpt_every : 1;
    A->ckpt_max = P->ckpt_max;
    A->tape = P->d_ckpt && P->d_tape && P->tape_cap > 0 ? reinterpret_cast<float4 *>(P->d_tape) : nullptr;
    A->tape_cap = A->tape ? P->tape_cap : 0;
    return AMR_OK;
}

// Point-light secondary-ray launch for one camera (amr_shadow.hip), with its workspace of
// shadow_work_bytes(npix, jobs) bytes.
int64_t shadow_work_bytes(int64_t npix, int64_t jobs);
int launch_shadow(const RenderArgs &A, bool rec, void *stream, void *work, int64_t work_bytes, int64_t jobs);

// Learned-proposal / segment-logging launch for one camera (amr_learned.hip).
int launch_learned(const RenderArgs &A, const amr_render_params *P, int lmax, void *stream, bool first_camera);

// Persistent multi-camera launch (amr_batched.hip).
int launch_persistent(const amr_scene *S, const amr_camera *cams, int32_t ncams, const amr_render_params *P,
                      float *d_rgba, amr_render_stats *d_stats, void *stream);

}  // namespace amr
