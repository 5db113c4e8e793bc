// Internal layouts shared by the host library and the HIP kernels of libamr.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/amr.h"

namespace amr {

// Device tree node, 16 bytes, breadth-first order; the two children of an internal node are
// adjacent (high = low + 1), as in the paper's implicit-sibling encoding (Section 4.2).
struct DNode {
    double split;      // internal: split plane in world coordinates (FP64, exact for dyadic grids)
    uint32_t child;    // internal: index of the low child; leaf: leaf id
    uint32_t meta;     // bits 0-1 axis (3 = leaf), bits 2-7 level
};
static_assert(sizeof(DNode) == 16, "DNode layout");

// Leaf record, 64 bytes: world box (for gradient-tap containment tests), owning patch,
// level (bits 0-7) with six face flags (bits 8-13, face 2a+side): a face is "safe" when the
// one-cell slab beyond it lies inside the leaf's patch and holds no finer data, so a gradient
// tap crossing it reads the same brick.  vmin/vmax: value range of the leaf's cells plus one
// halo cell.
struct DLeaf {
    double lo[3], hi[3];
    int32_t patch;
    uint32_t level_flags;
    float vmin, vmax;
};
static_assert(sizeof(DLeaf) == 64, "DLeaf layout");

// Patch header, 128 bytes.
struct DPatch {
    uint64_t off;        // first float of the padded brick in the pool
    int32_t n[3];        // interior cells per axis (brick is n+2 per axis, x fastest)
    int32_t level;
    double lo[3];        // world lower corner of the interior
    double inv_h[3];     // 1 / h^l
    double h[3];         // h^l
    double step;         // min_a h^l_a
    float vmin, vmax;
    int32_t nb[3];       // micro-brick and halo-row layouts: 4^3-cell blocks per axis of the padded brick
    int32_t layout;      // 0 linear, 1 micro-bricks, 2 halo rows
};
static_assert(sizeof(DPatch) == 128, "DPatch layout");

// Gradient-tap record of one leaf face, 64 bytes.  When the one-cell slab beyond the face has a
// single owner patch (n[0] > 0), a tap in the slab reads that patch's brick at
// q_owner = r q + t[a], q being the tap in the leaf's own patch-local cell coordinates.
// Otherwise n[0] == 0 and rope is the node to descend from (0: the root; -1: the slab leaves B).
struct DFaceXf {
    uint64_t off;        // first float of the owner's padded brick
    int32_t n[3];        // owner's interior cells per axis (0: no single owner)
    int32_t px, pxy;     // owner brick's row and slab strides (layout dependent)
    float r;             // h_own / h_owner
    float t[3];
    int32_t rope;
    int32_t pad_[4];
};
static_assert(sizeof(DFaceXf) == 64, "DFaceXf layout");

constexpr uint32_t kLeafAxis = 3u;

// Offset (in floats) of padded-brick cell (i, j, k) (0 <= index <= n + 1) in each layout; for
// the halo-row layout, the copy in the block column i / 4 (a cell also sits in the halo of the
// neighbouring block row when i mod 4 is 0, 1, 2 or 3: see halo_row_fill).
inline int64_t brick_index(int layout, const int32_t *n, const int32_t *nb, int64_t i, int64_t j, int64_t k) {
    if (layout == 0) return i + (int64_t)(n[0] + 2) * (j + (int64_t)(n[1] + 2) * k);
    if (layout == 2)
        return (((k >> 2) * nb[1] + (j >> 2)) * nb[0] + (i >> 2)) * 128 + ((k & 3) * 4 + (j & 3)) * 8 + (i & 3) + 1;
    return (((k >> 2) * nb[1] + (j >> 2)) * nb[0] + (i >> 2)) * 64 + (k & 3) * 16 + (j & 3) * 4 + (i & 3);
}

// Floats of one brick in each layout (before 64-float alignment).
inline int64_t brick_floats(int layout, const int32_t *n, const int32_t *nb) {
    if (layout == 0) return (int64_t)(n[0] + 2) * (n[1] + 2) * (n[2] + 2);
    return (int64_t)nb[0] * nb[1] * nb[2] * (layout == 2 ? 128 : 64);
}

// Halo-row layout: each 4x4x4-cell block stores 16 rows of 8 floats, row (j, k) of block column
// bx holding padded x indices 4 bx - 1 .. 4 bx + 6 (zero outside the padded brick).  `at(i, j, k)`
// returns the padded-brick value.
template <typename F>
inline void halo_row_fill(const int32_t *n, const int32_t *nb, float *dst, F at) {
    const int64_t P[3] = {n[0] + 2, n[1] + 2, n[2] + 2};
    for (int64_t bz = 0; bz < nb[2]; bz++)
        for (int64_t by = 0; by < nb[1]; by++)
            for (int64_t bx = 0; bx < nb[0]; bx++) {
                float *blk = dst + ((bz * nb[1] + by) * nb[0] + bx) * 128;
                for (int64_t kk = 0; kk < 4; kk++)
                    for (int64_t jj = 0; jj < 4; jj++) {
                        const int64_t j = 4 * by + jj, k = 4 * bz + kk;
                        float *row = blk + (kk * 4 + jj) * 8;
                        for (int64_t t = 0; t < 8; t++) {
                            const int64_t i = 4 * bx - 1 + t;
                            row[t] = (i >= 0 && i < P[0] && j < P[1] && k < P[2]) ? at(i, j, k) : 0.0f;
                        }
                    }
            }
}

inline uint32_t node_meta(int axis, int level) { return (uint32_t)(axis & 3) | ((uint32_t)(level & 63) << 2); }

void set_error(const char *fmt, ...);

}  // namespace amr
