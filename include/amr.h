/*
 * amr.h — C ABI of libamr: single-pass raycasting of structured AMR data on MI355X (gfx950).
 *
 * Method: Kaehler & Abel, "Single-Pass GPU-Raycasting for Structured Adaptive Mesh
 * Refinement Data" (arXiv 1212.3333).  The library
 *   1. partitions the overlapping refinement levels into non-overlapping same-level leaf
 *      blocks with an adaptive kD-tree built level by level        (amr_build_kdtree, Sec. 4.1)
 *   2. stores one padded brick per subgrid in a linear HBM pool and encodes the tree for the
 *      device                                                          (amr_pack_pool, Sec. 4.2, 5)
 *   3. renders every pixel in one pass: kD-restart descent, per-leaf sampling at a rate
 *      proportional to the leaf level's cell size, trilinear sampling, 1D RGBA transfer
 *      function with on-the-fly gradient lighting across blocks, front-to-back
 *      emission-absorption compositing with early termination      (amr_render, Sec. 5.3, 6)
 *   4. differentiates the image with respect to the transfer function and lighting
 *      parameters                                                     (amr_render_backward)
 *
 * Conventions for every function:
 *   - returns AMR_OK (0) or an error code; amr_last_error() gives a thread-local message;
 *   - "host" pointers are CPU memory, "device" pointers are HIP device memory owned by the
 *     caller; the library never frees caller memory and allocates device memory only where
 *     a function says so;
 *   - `stream` is a hipStream_t (passed as void*); device work is enqueued asynchronously on
 *     it, with no implicit synchronisation unless stated;
 *   - integers describing the hierarchy are in cells; coordinates of world space are FP64.
 */
#ifndef AMR_H
#define AMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    AMR_OK = 0,
    AMR_EINVAL = 1,       /* bad argument (NULL, size, range) */
    AMR_EHIERARCHY = 2,   /* invalid hierarchy (overlap, outside root box, empty patch) */
    AMR_ECAPACITY = 3,    /* caller buffer too small */
    AMR_ENOMEM = 4,       /* host allocation failed */
    AMR_EHIP = 5          /* HIP runtime error (launch, copy) */
};

const char *amr_last_error(void);

/* ---------------------------------------------------------------------------------------- */
/* Hierarchy (Section 3): subgrids on levels l = 0..nlevels-1, h^l = h^0 / refine^l.          */
/* ---------------------------------------------------------------------------------------- */

typedef struct {
    int32_t level;        /* 0 = root level */
    int32_t pad_;
    int64_t lo[3];        /* lower corner, level-l cell coordinates */
    int64_t dims[3];      /* cells per axis, >= 1 */
    const float *cells;   /* host, dims[0]*dims[1]*dims[2] values, x fastest; may be NULL
                             for amr_build_kdtree */
} amr_patch;

typedef struct {
    double origin[3];     /* world position of level-0 cell coordinate 0 */
    double h0[3];         /* root cell size */
    int32_t refine;       /* r >= 2, constant over levels and axes */
    int32_t nlevels;      /* 1..32 */
} amr_domain;

/* ---------------------------------------------------------------------------------------- */
/* kD-tree (Section 4.1)                                                                     */
/* ---------------------------------------------------------------------------------------- */

typedef struct amr_tree amr_tree;   /* opaque, immutable after the build, shareable */

typedef struct {
    int64_t nodes, leaves;          /* leaves = kind (b) */
    int64_t n_a, n_b, n_c;          /* node kinds: (a) fully refined inside one subgrid,
                                       (b) leaf, (c) other internal */
    int64_t depth;                  /* longest root-to-leaf path in edges */
    int64_t empty_leaves;           /* leaves covered by no root subgrid (transparent) */
    int64_t npatches;
} amr_tree_info;

typedef struct {                    /* one node, depth-first pre-order, low child first */
    int32_t axis;                   /* 0,1,2; -1 for a leaf */
    int32_t level;                  /* leaf: level of its patch; internal: level inserted
                                       when the node was split */
    int64_t split;                  /* internal: plane position in finest-level cells */
    int32_t patch;                  /* leaf: patch id or -1 (no data); internal: -1 */
    int32_t cover;                  /* internal: patch the node held before it was split */
    int32_t kind;                   /* 0 = (a), 1 = (b), 2 = (c) */
    int32_t pad_;
} amr_node_host;

typedef struct {                    /* one leaf, ids in depth-first pre-order */
    int64_t lo[3], hi[3];           /* finest-level cells, half open */
    int32_t patch, level;
} amr_leaf_host;

/* Builds the kD-tree of Section 4.1: the root is the bounding box B of the level-0 patches;
 * each node is split by the axis-aligned plane through a face of the boxes being inserted
 * that cuts the fewest of them, then splits the node's cells most evenly, then lowest axis,
 * then lowest position; a node stops when it holds cells of one subgrid.  Levels are inserted
 * one after another, refining every leaf that overlaps the next level.
 * Validates the hierarchy first (AMR_EHIERARCHY: same-level overlap, a patch outside B,
 * an empty patch, a level out of range, no level-0 patch).  Host only; *out must be freed
 * with amr_tree_free. */
int amr_build_kdtree(const amr_domain *dom, const amr_patch *patches, int32_t npatches, amr_tree **out);
int amr_tree_stats(const amr_tree *tree, amr_tree_info *out);
/* Copies the nodes and leaves (host arrays of at least stats.nodes / stats.leaves entries;
 * AMR_ECAPACITY if smaller; either pointer may be NULL to skip it). */
int amr_tree_export(const amr_tree *tree, amr_node_host *nodes, size_t ncap, amr_leaf_host *leaves, size_t lcap);
void amr_tree_free(amr_tree *tree);

/* ---------------------------------------------------------------------------------------- */
/* Pool and device scene (Sections 4.2 and 5)                                                */
/* ---------------------------------------------------------------------------------------- */

typedef struct {
    int32_t host_dst;     /* 1: d_pool and d_meta are host pointers (plain memcpy, no HIP) */
    int32_t nthreads;     /* host threads for the ghost fill; 0 = hardware concurrency */
    int32_t brick_layout; /* 0: each padded brick x-fastest (the pool keeps 64 spare floats
                             before the first and after the last brick, so the lit kernel reads
                             whole rows); 1: padded brick stored as 4x4x4-cell micro-bricks
                             (256 bytes each, x-fastest inside and between them); 2: halo rows,
                             4x4x4-cell blocks of 16 rows of 8 floats (512 bytes), row (j, k) of
                             block column bx holding padded x indices 4 bx - 1 .. 4 bx + 6, so a
                             stencil row loads as one vector from one block (twice the floats) */
    int32_t centering;    /* 0: cell-centred data, `cells` holds dims[0]*dims[1]*dims[2] values;
                             1: vertex-centred data (Section 5), `cells` holds the
                             (dims[0]+1)(dims[1]+1)(dims[2]+1) samples at the grid vertices
                             lo + i h, i = 0..dims, x fastest.  The field is their trilinear
                             interpolant.  Samples on a patch face that abuts coarser data
                             (dangling nodes) are replaced, at pack time and in FP64, by the
                             value of the abutting coarse patch: for each vertex on a patch's
                             boundary, the eight finest-level cells around it that lie in B are
                             each owned by the finest patch holding them, and when the coarsest
                             owner is coarser than the patch the sample becomes that owner's
                             trilinear value at the vertex (the first such owner with octant
                             bit a set for the + side of axis a).  Coarser levels are fixed
                             first.  Same-level neighbours are expected to carry equal values at
                             shared vertices.  The brick holds the n+1 samples per axis plus a
                             one-sample shell replicating the nearest sample. */
    int32_t reserved_[4];
} amr_pack_opts;

/* Device view of a packed scene.  Filled by amr_pack_pool; every pointer points into the
 * caller's d_pool / d_meta buffers, which must outlive the scene. */
typedef struct {
    const float *pool;          /* padded bricks, fp32, one per patch, 256-byte aligned */
    const void *nodes;          /* device tree, breadth-first, 16 bytes per node */
    const void *leaves;         /* leaf records, 64 bytes each */
    const void *patches;        /* patch headers, 128 bytes each */
    const void *leaf_faces;     /* per leaf, 6 int32 for the one-cell slab beyond each face:
                                   v >= 0 the single patch owning it; v <= -2 several owners, and
                                   node -2-v is the smallest tree node holding the slab; -1 the
                                   slab leaves B */
    const void *face_taps;      /* per leaf, 6 records of 64 bytes for gradient taps beyond each
                                   face: the single owner's brick and the affine map from the
                                   leaf's patch-local cell coordinates into it, or the node to
                                   descend from */
    int64_t pool_bytes, meta_bytes;
    int32_t nnodes, nleaves, npatches, nlevels;
    int32_t lmax, refine, depth, brick_layout;
    int32_t nlod;               /* kind-(a) nodes (inside one subgrid, all of its cells refined
                                   further; Section 4.1): records nleaves .. nleaves + nlod - 1 of
                                   `leaves` (and of the face tables) describe them in pre-order,
                                   with the covering coarse patch, for level-of-detail renders */
    int32_t centering;          /* 0 cell-centred, 1 vertex-centred (amr_pack_opts) */
    double box_lo[3], box_hi[3];        /* B in world coordinates */
    double origin[3], h0[3], hfine[3];  /* hfine = h0 / refine^lmax */
    double step_fine;                   /* min_a h^lmax_a */
    float v_min, v_max;                 /* range of all cell values */
} amr_scene;

/* Packs every patch into one padded brick, computed in FP64 and stored as fp32: cell-centred
 * data gets one ghost layer (same-level copy, edge replication outside B, coarse trilinear
 * interpolant, nearest interior cell); vertex-centred data holds its samples after the
 * dangling-node fix described at amr_pack_opts.centering.  Writes the device tree, leaf table
 * and patch headers to d_meta.  Two-call protocol: with d_pool == NULL and d_meta == NULL it
 * only writes the required sizes to *pool_bytes and *meta_bytes.  Otherwise the buffers
 * must hold at least those sizes (AMR_ECAPACITY).  The copies are enqueued on `stream` and
 * the function waits for them before returning (host staging memory is freed).
 * `patches` must be the array passed to amr_build_kdtree, with cells != NULL. */
int amr_pack_pool(const amr_tree *tree, const amr_patch *patches, int32_t npatches,
                  const amr_pack_opts *opts, void *d_pool, int64_t *pool_bytes,
                  void *d_meta, int64_t *meta_bytes, amr_scene *out_scene, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Rendering (Section 5.3)                                                                   */
/* ---------------------------------------------------------------------------------------- */

typedef struct {
    double eye[3], u[3], v[3], w[3];    /* explicit frame: right u, up v, forward w */
    double tan_half_fov;                /* perspective half-angle tangent (vertical) */
    double win[2];                      /* orthographic half extents (x, y) */
    int32_t ortho, width, height, pad_;
} amr_camera;

typedef struct {                        /* per ray segment, for parity tests */
    int32_t leaf, patch, n, level;      /* n = samples taken on the leaf (0 if no data) */
    double ta, tb;                      /* FP64 ray parameters of the segment */
} amr_trace_rec;

typedef struct {                        /* device counters, accumulated by amr_render */
    unsigned long long samples, segments, rays_hit, tap_descents, guard_hits, trace_overflow;
    unsigned long long skipped_segments, coarse_segments, seglog_count, ckpt_overflow;
    unsigned long long split_samples;   /* lit samples with a tap outside the sample's brick */
    unsigned long long face_taps;       /* taps read from a leaf face's single slab owner */
    unsigned long long unsure_taps;     /* taps classified in FP64 (within 1e-3 cell of a face) */
    unsigned long long net_segments;    /* learned form: segments the network was asked about */
    unsigned long long light_inline;    /* lighting = 2: samples whose secondary ray did not fit
                                           the workspace's job arrays (params.light_jobs) and was
                                           traced in the shading pass instead */
    unsigned long long reserved_[1];
} amr_render_stats;

typedef struct {
    const float *d_lut;                 /* device [256][4]: r, g, b, extinction per unit length */
    float v_lo, v_hi;                   /* u = clamp((F - v_lo) / (v_hi - v_lo), 0, 1); v_hi > v_lo */
    float step_frac;                    /* step = step_frac * min_a h^l_a of the leaf level */
    float t_min;                        /* early termination once T < t_min; 0 disables */
    int32_t uniform_step;               /* 1: every leaf uses the finest level's step */
    int32_t lighting;                   /* 0: none; 1: gradient shading (light = direction);
                                           2: point light at position `light`: shade =
                                           k_a + k_d T_L(x), T_L the transmittance of a secondary
                                           ray from the sample to the light inside B (the paper's
                                           global-illumination example, Section 6); forward only,
                                           trilinear, no level of detail */
    float light[3];                     /* light direction (need not be normalised) */
    float k_a, k_d, eps_g;              /* shade = k_a + k_d |g.l| / sqrt(|g|^2 + eps_g^2) */
    double clip_lo[3], clip_hi[3];      /* world clip box intersected with B */
    /* optional per-ray outputs (device, NULL to skip) */
    amr_trace_rec *d_trace;             /* [nrays][trace_cap] */
    int32_t *d_trace_n;                 /* [nrays]: segments met (may exceed trace_cap) */
    int32_t *d_nsamp;                   /* [nrays]: samples evaluated */
    int64_t trace_cap;
    /* adjoint checkpoints (device, NULL to skip; see amr_render_backward) */
    void *d_ckpt;
    int64_t ckpt_bytes;
    int32_t ckpt_every;                 /* checkpoint every k-th data segment (>= 1) */
    int32_t ckpt_max;                   /* checkpoints per ray */
    float *d_tape;                      /* optional with d_ckpt, lit: [nrays][tape_cap][4] fp32 (device,
                                           16-byte aligned), written by the forward: per ray, in
                                           order, a record (delta, delta log2 e, n as int32 bits, 0)
                                           at each data segment with n samples, then a record
                                           (F, g_x, g_y, g_z) per sample: the value and the gradient
                                           it was shaded with.  amr_render_backward replays the
                                           checkpoint intervals whose records all fit from the tape
                                           and evaluates the rest in place; records beyond tape_cap
                                           are not written */
    int64_t tape_cap;                   /* records per ray (amr_tape_bytes), at most 2^26 - 1 */
    /* learned segment proposals (NULL = plain traversal).  alpha_max = 1 - exp(-sigma_max L)
       is the analytic bound on a segment's opacity from the leaf's value range; the network
       predicts quantiles (r_lo, r_hi) of alpha / alpha_max, clamped to [0, 1], and
       alpha_hi = r_hi alpha_max, alpha_lo = r_lo alpha_max.  A data segment entered with
       transmittance T is skipped if B + T * alpha_hi < tau_e (alpha_hi = alpha_max when the
       bound alone decides), B being the sum of T * alpha_hi over the ray's earlier skips, so
       the charged opacity of a ray stays below tau_e; it is sampled with one step per cell
       and ends the ray if alpha_lo > 1 - tau_s; otherwise it is sampled plainly */
    const void *d_mlp;                  /* packed network, see amr_mlp_pack (16-byte aligned) */
    float tau_e, tau_s;
    /* segment log for training (device): a 256-byte header whose first 8 bytes count the
       segments met, then amr_seglog_rec records; seglog_cap is the buffer size in bytes */
    void *d_seglog;
    int64_t seglog_cap;
    /* scheduling */
    int32_t persistent;                 /* 1: persistent tile-queue kernel */
    int32_t tile_w, tile_h;             /* pixels per wave tile (0 = default 8 x 8) */
    int32_t blocks_per_cu;              /* persistent grid = 256 CUs x this (0 = default) */
    int32_t interp;                     /* sampling of the cell-centred data: 0 trilinear with the
                                           ghost layer, 1 the value of the cell holding the point
                                           (nearest cell, as Section 5 samples cell data; plain
                                           forward kernel only, AMR_EINVAL elsewhere and on
                                           vertex-centred scenes) */
    float lod;                          /* level of detail (Sections 4.1 and 5.3): the kD-restart
                                           descent stops at a kind-(a) node when the cells of its
                                           covering coarse patch project to fewer than lod pixels
                                           at the segment start (perspective: h < lod t (2 tan /
                                           height); orthographic: h < lod (2 win_y / height)), and
                                           renders the node's segment from that patch; 0 = off */
    void *d_queue;                      /* persistent: device scratch, >= amr_queue_bytes(ncams) */
    unsigned long long *d_stamps;       /* persistent: [ncams + 1] device clock when each image
                                           completed, then the launch start (optional) */
    const amr_camera *d_cams;           /* persistent: device copy of `cams` (read by the kernel,
                                           so a captured graph can be replayed with new cameras) */
    /* measurement (device, NULL to skip): one bit per pool float, set for every cell a sample
       or gradient tap reads; its population count gives a frame's compulsory pool bytes */
    uint32_t *d_touch;
    /* caller-owned device workspace (the library allocates no device memory during a render):
       amr_render with lighting = 2 needs amr_render_work_bytes(...) bytes, amr_render_backward
       needs amr_backward_work_bytes(deterministic); other calls ignore it.  NULL or too small
       where needed: AMR_EINVAL / AMR_ECAPACITY, nothing enqueued.  Its contents on entry do not
       matter; calls that share one workspace must be ordered (one stream). */
    void *d_work;
    int64_t work_bytes;
    int64_t light_jobs;                 /* lighting = 2: secondary rays the workspace holds per
                                           camera (16 bytes each); a sample beyond this count has
                                           its secondary ray traced in the shading pass (same
                                           value, slower; counted in light_inline) */
    uint32_t *d_touch_meta;             /* measurement (device, NULL to skip): one bit per 16 bytes
                                           of the scene's metadata buffer (from scene.nodes), set for
                                           the node, leaf, patch-header and face records the frame
                                           reads */
    int32_t bound_only;                 /* 1: skip segments by the analytic bound alone (the learned
                                           kernel with the network never consulted; d_mlp must be
                                           NULL): a data segment is skipped if B + T * alpha_max <
                                           tau_e, with B and alpha_max as for learned proposals; no
                                           coarse sampling.  0: learned proposals when d_mlp is set */
    int32_t queue_order;                /* persistent: 0 cameras largest image first, 1 smallest first */
    int32_t xcd_tiles;                  /* persistent: 0 one tile queue, images row by row; 1 one queue per
                                           XCD (blocks b with b mod 8 = x take queue x), holding the
                                           4x4-tile super-tiles x, x + 8, ... of each image along a
                                           Morton curve, so the tiles in flight on an XCD stay close */
    int32_t waves_per_simd;             /* persistent, lit: the register budget of the kernel, 2 or 3
                                           waves per SIMD (0 = 3; 3 spills part of the state to
                                           scratch, 2 holds it in registers); AMR_EINVAL otherwise */
    int32_t pad3_;
    /* tile schedule (device, NULL to skip; amr_sched_bytes bytes, caller-owned, zeroed before its
       first use and kept across calls for the same cameras): every call records how long each
       8x8 tile of each camera took and sorts the super-tiles (16x16 pixels lit, 32x32 unlit) of
       each launch's cameras (up to 8 per launch) together by their longest tile; the next call
       with the same lighting and cameras
       of the same sizes starts them in that order, longest first, so that the launch does not
       end waiting on long tiles started late.  A call whose lighting or camera sizes differ
       renders in the default order and records a new order.  Images do not depend on the order.  The
       raycaster only: AMR_EINVAL with persistent mode, learned proposals or the point light, or
       for a camera of 2^24 or more super-tiles.  Calls that overlap on one schedule
       race on it */
    void *d_sched;
    int64_t sched_bytes;
} amr_render_params;

/* Renders ncams cameras (host array) into d_rgba (device, premultiplied RGBA fp32, images
 * concatenated, image i has width_i*height_i*4 floats, row 0 at the top).  d_stats
 * (device, optional) is zeroed and then accumulated.  Asynchronous on `stream`: no device
 * allocation, no host synchronisation (the point light's passes included). */
int amr_render(const amr_scene *scene, const amr_camera *cams, int32_t ncams,
               const amr_render_params *params, float *d_rgba, amr_render_stats *d_stats, void *stream);

/* Persistent mode (params.persistent = 1): one launch renders all cameras; waves take 64-pixel
 * tiles (tile_w x tile_h) from a device queue ordered largest image first; the launch and its
 * setup are device-only work, so the call may be captured in a hipGraph.  Needs d_queue and
 * d_cams; images are identical to the non-persistent path's.  Trilinear sampling with
 * lighting 0 or 1 only: nearest-cell sampling, the point light, learned proposals, segment
 * logging, traces and checkpoints are rejected with AMR_EINVAL. */
/* Bytes of device scratch the persistent batched kernel needs for ncams cameras. */
int64_t amr_queue_bytes(int32_t ncams);
/* Rate of the device clock written to d_stamps, in kHz. */
int64_t amr_wall_clock_khz(void);

/* Checkpoint buffer bytes for nrays rays with ckpt_max checkpoints each. */
int64_t amr_ckpt_bytes(int64_t nrays, int32_t ckpt_max);
/* Tile schedule bytes (params->d_sched) for these cameras: a 16-byte header per camera (padded to
 * 256 bytes), then a time and an order slot of 4 bytes each per 8x8 tile; -1 on invalid
 * arguments. */
int64_t amr_sched_bytes(const amr_camera *cams, int32_t ncams);
/* Tape bytes for nrays rays with tape_cap records each (16 bytes per record). */
int64_t amr_tape_bytes(int64_t nrays, int64_t tape_cap);

/* Workspace bytes (params->d_work) amr_render needs for these cameras and params: with
 * lighting = 2, per-ray sample counts and job offsets for the largest camera plus
 * params->light_jobs jobs of 16 bytes (the cameras are rendered one after another and reuse
 * it); 0 otherwise.  -1 on invalid arguments (NULL, ncams <= 0, negative light_jobs). */
int64_t amr_render_work_bytes(const amr_camera *cams, int32_t ncams, const amr_render_params *params);
/* Workspace bytes (params->d_work) amr_render_backward needs: the 1029-float gradient
 * accumulator, plus one partial sum per block of the adjoint's fixed grid when
 * deterministic = 1. */
int64_t amr_backward_work_bytes(int32_t deterministic);

/* Adjoint of amr_render for a loss L(RGBA): given dL/dRGBA (device, same layout as d_rgba),
 * accumulates dL/dLUT into d_grad_lut (device [256][4], fp32, zeroed by the call) and
 * dL/d(light_x, light_y, light_z, k_a, k_d) into d_grad_light (device [5]).  `params` must be
 * the ones of the forward call that filled params->d_ckpt (same scene, cameras, LUT).
 * The early-termination point of each ray is the forward's.  deterministic = 1 reduces
 * per-block partial sums in a fixed order (bit-reproducible); 0 uses atomics.  The gradient
 * accumulators live in params->d_work (amr_backward_work_bytes(deterministic) bytes, caller
 * owned; AMR_EINVAL if NULL, AMR_ECAPACITY if smaller).  Asynchronous: no device allocation,
 * no host synchronisation. */
int amr_render_backward(const amr_scene *scene, const amr_camera *cams, int32_t ncams,
                        const amr_render_params *params, const float *d_grad_rgba,
                        float *d_grad_lut, float *d_grad_light, int32_t deterministic, void *stream);

/* For callers that cannot allocate device memory or pass a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): amr_render_backward with its
 * gradient accumulators in a fixed device array inside the library instead of params->d_work
 * (ignored here).  The array holds amr_backward_static_bytes() bytes (the deterministic
 * mode's need, 8.4 MB) on every GPU the library runs on, until the process ends; a need beyond
 * it returns AMR_ECAPACITY.  Its address on a device is looked up on the first call there.
 * The call allocates nothing and clears the accumulators itself (with a kernel, no memset),
 * so each call starts from zero; every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (different streams, or threads without ordering) race and must not be
 * made.  Arguments, outputs and errors otherwise as amr_render_backward. */
int64_t amr_backward_static_bytes(void);
int amr_render_backward_static(const amr_scene *scene, const amr_camera *cams, int32_t ncams,
                               const amr_render_params *params, const float *d_grad_rgba,
                               float *d_grad_lut, float *d_grad_light, int32_t deterministic,
                               void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Measurement (not a step of the method)                                                     */
/* ---------------------------------------------------------------------------------------- */

/* Read-bandwidth probe for the rooflines: `blocks` blocks of 256 threads stride over d_buf
 * (device, `bytes` bytes of non-negative floats, 16-byte aligned; the tail beyond a multiple
 * of 16 bytes is not read) `reps` times, each block reading the same elements every time, and
 * store nothing (d_sink, device [1], is written only if the sum of the data is -1).  Timed by
 * the caller around the launch on `stream`: bytes/16*16 * reps / time is the sustained read
 * rate of the cache level the buffer fits in (a few MB per XCD: L2). */
int amr_probe_read(const void *d_buf, int64_t bytes, int32_t reps, int32_t blocks, float *d_sink, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Proposal network for learned segment skipping (an addition to the paper)                 */
/* ---------------------------------------------------------------------------------------- */

#define AMR_MLP_IN 12
#define AMR_MLP_HID 64
#define AMR_MLP_OUT 2

typedef struct {                        /* one logged leaf segment (training data) */
    float feat[AMR_MLP_IN];             /* level/lmax, log2(L/h)/8, u_min, u_max, analytic
                                           alpha bounds (max, mean, min extinction of the LUT over
                                           the leaf's value range times L), n/256, |d_x|, |d_y|,
                                           |d_z|, log2(min patch dim)/6 */
    float alpha_seg;                    /* true segment opacity 1 - prod(1 - alpha_k) */
    float t_in;                         /* transmittance entering the segment; negative if early
                                           termination cut the segment short */
    int32_t ray, n;
} amr_seglog_rec;

/* Forward pass of the 12-64-64-2 ReLU network on n rows: X (device, [n][12] fp32),
 * W (device, packed fp32 master weights, amr_mlp_param_count floats), Y (device, [n][2],
 * sigmoid outputs (alpha_lo, alpha_hi)); H (device scratch [n][128] fp32 activations, kept
 * for the backward pass, may be NULL for inference).  fp16 MFMA with fp32 accumulation. */
int32_t amr_mlp_param_count(void);
int amr_mlp_forward(const float *X, const float *W, float *Y, float *H, int64_t n, void *stream);
/* Backward of the pinball (quantile) loss mean over rows: q_lo for output 0, q_hi for
 * output 1, targets T (device [n]); writes dW (device, zeroed by the call), loss (device [1]). */
int amr_mlp_backward(const float *X, const float *W, const float *H, const float *Y, const float *T,
                     int64_t n, float q_lo, float q_hi, float *dW, float *loss, void *stream);
/* One Adam step on W with moments M, V (device, param_count each), step index t >= 1. */
int amr_mlp_adam_step(float *W, const float *dW, float *M, float *V, int32_t t, float lr,
                      float beta1, float beta2, float eps, void *stream);
/* Packs fp32 master weights W into the fp16 inference layout used by amr_render (d_out of
 * amr_mlp_packed_bytes() bytes, device, 16-byte aligned as amr_render requires of d_mlp). */
int64_t amr_mlp_packed_bytes(void);
int amr_mlp_pack(const float *W, void *d_out, void *stream);

/* ---------------------------------------------------------------------------------------- */
/* Out-of-core residency (Sections 5.2 and 7)                                                */
/* ---------------------------------------------------------------------------------------- */

/* The paper keeps one texture brick per subgrid, and with bindless access an out-of-core
 * renderer can upload the subsets of bricks it needs.  A store holds every brick on the host,
 * packed once as amr_pack_pool packs them; amr_store_update makes a subset resident in a device
 * brick cache and writes a scene in which each leaf (and kind-(a) node) of an absent patch is
 * drawn from the finest resident patch whose box holds the leaf's box, with that patch's cells
 * and sample step; a leaf with no resident holder is empty, and a kind-(a) node without one is
 * never a level-of-detail stop.  Gradient taps read the finest resident patch holding the tap
 * point.  Ghost layers and vertex samples stay those of the full hierarchy.  The render entry
 * points take the scene unchanged. */
typedef struct amr_store amr_store;   /* opaque; not thread-safe */

typedef struct {
    int64_t npatches;
    int64_t meta_bytes;        /* device metadata buffer amr_store_update needs */
    int64_t full_cache_bytes;  /* cache that holds every brick at once */
    int64_t pad_bytes;         /* bytes of a cache outside the bricks (row-load pads) */
} amr_store_info;

typedef struct {
    int64_t uploaded_bricks, uploaded_bytes;   /* host-to-device brick copies of this update */
    int64_t evicted_bricks;                    /* bricks dropped from the cache */
    int64_t resident_bricks, resident_bytes;   /* after the update */
    int64_t remapped_leaves;                   /* leaf records drawn from another patch */
    int32_t repacked;                          /* 1: every resident brick was laid out again */
    int32_t reserved_;
} amr_store_report;

/* Packs every patch into a host store (same options as amr_pack_pool; opts->host_dst = 1 makes
 * amr_store_update write plain host memory, for tests without a GPU).  `tree` and `patches`
 * are read only during the call.  Free with amr_store_free. */
int amr_store_create(const amr_tree *tree, const amr_patch *patches, int32_t npatches,
                     const amr_pack_opts *opts, amr_store **out);
int amr_store_stats(const amr_store *s, amr_store_info *info);
/* Cache bytes of each patch's brick (bytes[npatches]; AMR_ECAPACITY if cap < npatches). */
int amr_store_brick_bytes(const amr_store *s, int64_t *bytes, int64_t cap);
/* A resident set for `cam` within cache_bytes: levels coarse to fine, inside a level the
 * patches whose bounding sphere meets the view volume nearest first; refinements out of view
 * are left out; a brick that does not fit is skipped.  Writes resident[npatches] (0/1). */
int amr_store_select(const amr_store *s, const amr_camera *cam, int64_t cache_bytes, uint8_t *resident);
/* Makes the patches with resident[p] != 0 resident in the device cache d_cache (cache_bytes,
 * 256-byte aligned; a cache never seen before, or of another size, is cleared and laid out from
 * the start).  Bricks already in the cache stay where they are; new ones take the first free
 * slot that fits, and when none does every resident brick is laid out again.  Writes the
 * metadata to d_meta (>= amr_store_info.meta_bytes) and the scene to *out_scene, whose pool is
 * d_cache.  The copies are enqueued on `stream` and waited for.  AMR_ECAPACITY when the
 * resident bricks exceed the cache (the cache and the previous scene are unchanged).  Renders
 * of an earlier scene must have finished before the call. */
int amr_store_update(amr_store *s, const uint8_t *resident, void *d_cache, int64_t cache_bytes,
                     void *d_meta, int64_t meta_bytes, amr_scene *out_scene, amr_store_report *report,
                     void *stream);
void amr_store_free(amr_store *s);

#ifdef __cplusplus
}
#endif
#endif /* AMR_H */
