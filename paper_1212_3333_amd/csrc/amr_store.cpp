// Out-of-core residency (Sections 5.2 and 7): the paper keeps one texture brick per subgrid so
// that, with bindless access, an out-of-core renderer can upload the subsets of bricks it needs.
// Here a host store holds every brick once, packed exactly as amr_pack_pool packs the pool; a
// subset is made resident in a device brick cache (first-fit slots, 256-byte aligned), and the
// metadata is rewritten so that each leaf of an absent patch is drawn from the finest resident
// patch holding the leaf's box.  The render kernels are unchanged: the cache is the scene's pool
// and the patch headers carry each resident brick's cache offset.
//
// Compiled with -ffp-contract=off like the rest of the host code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <unordered_map>
#include <utility>
#include <vector>

#include "amr.h"
#include "amr_internal.h"

using namespace amr;

namespace {

constexpr int64_t kPadFloats = 64;   // spare floats before and after the bricks (row loads)

int64_t align64(int64_t x) { return (x + 63) / 64 * 64; }

}  // namespace

struct amr_store {
    int np = 0, layout = 0, centering = 0, host_dst = 0, refine = 2, lmax = 0;
    amr_scene full{};                    // scene of the host pack (pointers into pool/meta)
    std::vector<float> pool;             // every brick (host copy of a full pool)
    std::vector<uint8_t> meta;           // metadata of the full hierarchy
    int64_t o_nodes = 0, o_leaves = 0, o_patch = 0, o_faces = 0, o_fxf = 0;
    std::vector<int64_t> bsz;            // per patch: cache floats of its brick (64-float multiple)
    std::vector<int32_t> plevel;
    std::vector<int64_t> pbox;           // per patch: lo[3], hi[3] in finest-level cells
    int64_t nrec = 0, nl0 = 0;           // leaf records: leaves, then kind-(a) nodes
    std::vector<int64_t> rbox;           // per record: lo[3], hi[3]
    std::vector<int32_t> chain_at, chain;  // per record: patches holding its box, coarse to fine
    std::vector<int32_t> lod_node;       // per kind-(a) record: its device node index
    // value range of record k drawn from holder patch h, keyed (k << 32) | h (the scan of the
    // holder's cells depends on nothing else, and an orbit remaps the same records again)
    std::unordered_map<uint64_t, std::pair<float, float>> range_memo;
    // cache state
    void *cache = nullptr;
    int64_t cache_floats = 0;
    std::vector<int64_t> slot;           // per patch: float offset in the cache, -1 if absent
    std::map<int64_t, int64_t> free_;    // free intervals: start -> length (floats)
};

namespace {

void free_reset(amr_store *s) {
    s->free_.clear();
    if (s->cache_floats > 2 * kPadFloats) s->free_[kPadFloats] = s->cache_floats - 2 * kPadFloats;
    std::fill(s->slot.begin(), s->slot.end(), (int64_t)-1);
}

bool free_take(amr_store *s, int64_t len, int64_t *at) {   // best fit: the smallest hole that fits
    auto best = s->free_.end();
    for (auto it = s->free_.begin(); it != s->free_.end(); ++it)
        if (it->second >= len && (best == s->free_.end() || it->second < best->second)) best = it;
    if (best == s->free_.end()) return false;
    *at = best->first;
    const int64_t rest = best->second - len, start = best->first + len;
    s->free_.erase(best);
    if (rest > 0) s->free_[start] = rest;
    return true;
}

void free_give(amr_store *s, int64_t at, int64_t len) {
    auto next = s->free_.lower_bound(at);
    if (next != s->free_.end() && next->first == at + len) {
        len += next->second;
        next = s->free_.erase(next);
    }
    if (next != s->free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == at) {
            prev->second += len;
            return;
        }
    }
    s->free_[at] = len;
}

// Value range a sample in record box [lo, hi) can read from patch h's brick (the rule of the
// packer: cell-centred, the box's cells plus one halo cell; vertex-centred, the vertices of its
// cells).
void leaf_range(const amr_store *s, int h, const int64_t *lo, const int64_t *hi, float *vmin, float *vmax) {
    const DPatch *P = (const DPatch *)(s->meta.data() + s->o_patch) + h;
    int64_t S = 1;
    for (int k = 0; k < s->lmax - s->plevel[h]; k++) S *= s->refine;
    int64_t i0[3], i1[3];
    for (int a = 0; a < 3; a++) {
        i0[a] = (lo[a] - s->pbox[6 * h + a]) / S;
        i1[a] = (hi[a] - s->pbox[6 * h + a] + S - 1) / S;
    }
    const int64_t first = s->centering ? 0 : 1;
    const int64_t base = (int64_t)P->off;   // the full pack's pool offset
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t z = i0[2] - first; z <= i1[2]; z++)
        for (int64_t y = i0[1] - first; y <= i1[1]; y++)
            for (int64_t x = i0[0] - first; x <= i1[0]; x++) {
                const float v = s->pool[(size_t)(base + brick_index(s->layout, P->n, P->nb, x + 1, y + 1, z + 1))];
                mn = std::min(mn, v);
                mx = std::max(mx, v);
            }
    *vmin = mn;
    *vmax = mx;
}

int copy_out(const amr_store *s, void *dst, const void *src, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return AMR_OK;
    if (s->host_dst) {
        memcpy(dst, src, bytes);
        return AMR_OK;
    }
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) { set_error("HIP copy failed: %s", hipGetErrorString(e)); return AMR_EHIP; }
    return AMR_OK;
}

// Does the sphere (c, r) meet the camera's view volume?  Perspective: the four side planes
// through the eye; orthographic: the window's slab.  Conservative (near and far unbounded).
bool sphere_visible(const amr_camera *cam, const double c[3], double r) {
    double v[3];
    for (int a = 0; a < 3; a++) v[a] = c[a] - cam->eye[a];
    const double x = v[0] * cam->u[0] + v[1] * cam->u[1] + v[2] * cam->u[2];
    const double y = v[0] * cam->v[0] + v[1] * cam->v[1] + v[2] * cam->v[2];
    const double z = v[0] * cam->w[0] + v[1] * cam->w[1] + v[2] * cam->w[2];
    if (cam->ortho) return std::fabs(x) <= cam->win[0] + r && std::fabs(y) <= cam->win[1] + r && z >= -r;
    const double ty = cam->tan_half_fov, tx = ty * (double)cam->width / (double)cam->height;
    // plane normals (unnormalised) of x = tx z and y = ty z; distance = (|x| - t z) / sqrt(1 + t^2)
    return (std::fabs(x) - tx * z) <= r * std::sqrt(1.0 + tx * tx) && (std::fabs(y) - ty * z) <= r * std::sqrt(1.0 + ty * ty) &&
           z >= -r;
}

}  // namespace

extern "C" {

int amr_store_create(const amr_tree *tree, const amr_patch *patches, int32_t npatches, const amr_pack_opts *opts,
                     amr_store **out) {
    if (!tree || !patches || !out) { set_error("null argument"); return AMR_EINVAL; }
    *out = nullptr;
    amr_pack_opts o{};
    if (opts) o = *opts;
    const int host_dst = o.host_dst;
    o.host_dst = 1;
    amr_store *s = nullptr;
    try {
        s = new amr_store();
        s->np = npatches;
        s->host_dst = host_dst;
        s->layout = o.brick_layout;
        s->centering = o.centering;
        int64_t pb = 0, mb = 0;
        int rc = amr_pack_pool(tree, patches, npatches, &o, nullptr, &pb, nullptr, &mb, nullptr, nullptr);
        if (rc != AMR_OK) { delete s; return rc; }
        s->pool.assign((size_t)(pb / 4), 0.0f);
        s->meta.assign((size_t)mb, 0);
        rc = amr_pack_pool(tree, patches, npatches, &o, s->pool.data(), &pb, s->meta.data(), &mb, &s->full, nullptr);
        if (rc != AMR_OK) { delete s; return rc; }
        const uint8_t *mbase = s->meta.data();
        s->o_nodes = (const uint8_t *)s->full.nodes - mbase;
        s->o_leaves = (const uint8_t *)s->full.leaves - mbase;
        s->o_patch = (const uint8_t *)s->full.patches - mbase;
        s->o_faces = (const uint8_t *)s->full.leaf_faces - mbase;
        s->o_fxf = (const uint8_t *)s->full.face_taps - mbase;
        s->refine = s->full.refine;
        s->lmax = s->full.lmax;
        // brick sizes and patch boxes (finest-level cells)
        const DPatch *P = (const DPatch *)(mbase + s->o_patch);
        int64_t fine = 1;
        for (int k = 0; k < s->lmax; k++) fine *= s->refine;
        s->bsz.resize(npatches);
        s->plevel.resize(npatches);
        s->pbox.resize(6 * (size_t)npatches);
        for (int p = 0; p < npatches; p++) {
            s->bsz[p] = align64(brick_floats(s->layout, P[p].n, P[p].nb));
            s->plevel[p] = patches[p].level;
            int64_t S = 1;
            for (int k = 0; k < s->lmax - patches[p].level; k++) S *= s->refine;
            for (int a = 0; a < 3; a++) {
                s->pbox[6 * p + a] = patches[p].lo[a] * S;
                s->pbox[6 * p + 3 + a] = (patches[p].lo[a] + patches[p].dims[a]) * S;
            }
        }
        // record boxes: leaves in pre-order, then kind-(a) nodes in pre-order (as the packer)
        amr_tree_info ti;
        amr_tree_stats(tree, &ti);
        std::vector<amr_node_host> nodes((size_t)ti.nodes);
        std::vector<amr_leaf_host> leaves((size_t)ti.leaves);
        amr_tree_export(tree, nodes.data(), nodes.size(), leaves.data(), leaves.size());
        s->nl0 = ti.leaves;
        s->nrec = ti.leaves + ti.n_a;
        s->rbox.resize(6 * (size_t)s->nrec);
        for (int64_t k = 0; k < s->nl0; k++)
            for (int a = 0; a < 3; a++) {
                s->rbox[6 * k + a] = leaves[k].lo[a];
                s->rbox[6 * k + 3 + a] = leaves[k].hi[a];
            }
        {   // node boxes by a pre-order walk from B (the level-0 patches' bounding box)
            int64_t B[6];
            bool first = true;
            for (int p = 0; p < npatches; p++) {
                if (patches[p].level != 0) continue;
                for (int a = 0; a < 3; a++) {
                    if (first || s->pbox[6 * p + a] < B[a]) B[a] = s->pbox[6 * p + a];
                    if (first || s->pbox[6 * p + 3 + a] > B[3 + a]) B[3 + a] = s->pbox[6 * p + 3 + a];
                }
                first = false;
            }
            std::vector<std::array<int64_t, 6>> pending;   // high-child boxes awaiting their turn
            std::array<int64_t, 6> box;
            std::copy(B, B + 6, box.begin());
            int64_t ka = s->nl0;
            for (size_t i = 0; i < nodes.size(); i++) {
                const amr_node_host &n = nodes[i];
                if (n.kind == 0) {
                    std::copy(box.begin(), box.end(), &s->rbox[6 * ka]);
                    ka++;
                }
                if (n.axis >= 0) {
                    std::array<int64_t, 6> lo_box = box, hi_box = box;
                    lo_box[3 + n.axis] = n.split;
                    hi_box[n.axis] = n.split;
                    pending.push_back(hi_box);
                    box = lo_box;
                } else if (!pending.empty()) {
                    box = pending.back();
                    pending.pop_back();
                }
            }
        }
        // holders of each record box, from a coarse bin grid over the patch boxes
        const int G = 32;
        int64_t Blo[3], ext[3];
        for (int a = 0; a < 3; a++) {
            Blo[a] = INT64_MAX;
            int64_t hi = INT64_MIN;
            for (int p = 0; p < npatches; p++) {
                Blo[a] = std::min(Blo[a], s->pbox[6 * p + a]);
                hi = std::max(hi, s->pbox[6 * p + 3 + a]);
            }
            ext[a] = std::max<int64_t>(1, hi - Blo[a]);
        }
        auto bin_of = [&](int a, int64_t x) {
            int64_t c = (x - Blo[a]) * G / ext[a];
            return (int)std::min<int64_t>(std::max<int64_t>(c, 0), G - 1);
        };
        std::vector<std::vector<int32_t>> bins((size_t)G * G * G);
        for (int p = 0; p < npatches; p++)
            for (int z = bin_of(2, s->pbox[6 * p + 2]); z <= bin_of(2, s->pbox[6 * p + 5] - 1); z++)
                for (int y = bin_of(1, s->pbox[6 * p + 1]); y <= bin_of(1, s->pbox[6 * p + 4] - 1); y++)
                    for (int x = bin_of(0, s->pbox[6 * p]); x <= bin_of(0, s->pbox[6 * p + 3] - 1); x++)
                        bins[(size_t)x + G * (y + G * z)].push_back(p);
        s->chain_at.assign((size_t)s->nrec + 1, 0);
        for (int64_t k = 0; k < s->nrec; k++) {
            const int64_t *b = &s->rbox[6 * k];
            const auto &cand = bins[(size_t)bin_of(0, b[0]) + G * (bin_of(1, b[1]) + G * bin_of(2, b[2]))];
            std::vector<int32_t> hold;
            for (int32_t q : cand) {
                bool in = true;
                for (int a = 0; a < 3; a++) in = in && s->pbox[6 * q + a] <= b[a] && b[3 + a] <= s->pbox[6 * q + 3 + a];
                if (in) hold.push_back(q);
            }
            std::sort(hold.begin(), hold.end(), [&](int32_t x, int32_t y) {
                return s->plevel[x] != s->plevel[y] ? s->plevel[x] < s->plevel[y] : x < y;
            });
            s->chain.insert(s->chain.end(), hold.begin(), hold.end());
            s->chain_at[k + 1] = (int32_t)s->chain.size();
        }
        // device node of each kind-(a) record (its level-of-detail bits name the record)
        s->lod_node.assign((size_t)(s->nrec - s->nl0), -1);
        const DNode *dn = (const DNode *)(mbase + s->o_nodes);
        for (int64_t i = 0; i < s->full.nnodes; i++) {
            const uint32_t a = dn[i].meta >> 8;
            if (a) s->lod_node[a - 1] = (int32_t)i;
        }
        s->slot.assign(npatches, -1);
    } catch (const std::bad_alloc &) {
        delete s;
        set_error("out of host memory");
        return AMR_ENOMEM;
    }
    *out = s;
    return AMR_OK;
}

int amr_store_stats(const amr_store *s, amr_store_info *info) {
    if (!s || !info) { set_error("null argument"); return AMR_EINVAL; }
    memset(info, 0, sizeof(*info));
    info->npatches = s->np;
    info->meta_bytes = (int64_t)s->meta.size();
    int64_t tot = 0;
    for (int64_t b : s->bsz) tot += b;
    info->full_cache_bytes = 4 * (tot + 2 * kPadFloats);
    info->pad_bytes = 4 * 2 * kPadFloats;
    return AMR_OK;
}

int amr_store_brick_bytes(const amr_store *s, int64_t *bytes, int64_t cap) {
    if (!s || !bytes) { set_error("null argument"); return AMR_EINVAL; }
    if (cap < s->np) { set_error("capacity %lld < %d patches", (long long)cap, s->np); return AMR_ECAPACITY; }
    for (int p = 0; p < s->np; p++) bytes[p] = 4 * s->bsz[p];
    return AMR_OK;
}

int amr_store_select(const amr_store *s, const amr_camera *cam, int64_t cache_bytes, uint8_t *resident) {
    if (!s || !cam || !resident) { set_error("null argument"); return AMR_EINVAL; }
    const amr_scene &F = s->full;
    std::vector<int> order(s->np);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> dist(s->np);
    std::vector<char> vis(s->np);
    for (int p = 0; p < s->np; p++) {
        double c[3], r2 = 0.0, d2 = 0.0;
        for (int a = 0; a < 3; a++) {
            const double lo = F.origin[a] + (double)s->pbox[6 * p + a] * F.hfine[a];
            const double hi = F.origin[a] + (double)s->pbox[6 * p + 3 + a] * F.hfine[a];
            c[a] = 0.5 * (lo + hi);
            r2 += 0.25 * (hi - lo) * (hi - lo);
            d2 += (c[a] - cam->eye[a]) * (c[a] - cam->eye[a]);
        }
        dist[p] = std::sqrt(d2);
        vis[p] = sphere_visible(cam, c, std::sqrt(r2));
    }
    // coarse levels first; inside a level, patches in view before the others, nearest first
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (s->plevel[x] != s->plevel[y]) return s->plevel[x] < s->plevel[y];
        if (vis[x] != vis[y]) return vis[x] > vis[y];
        return dist[x] < dist[y];
    });
    int64_t left = cache_bytes / 4 - 2 * kPadFloats;
    memset(resident, 0, (size_t)s->np);
    for (int p : order) {
        if (!vis[p] && s->plevel[p] > 0) continue;   // out-of-view refinements never help
        if (s->bsz[p] <= left) {
            resident[p] = 1;
            left -= s->bsz[p];
        }
    }
    return AMR_OK;
}

int amr_store_update(amr_store *s, const uint8_t *resident, void *d_cache, int64_t cache_bytes, void *d_meta,
                     int64_t meta_bytes, amr_scene *out, amr_store_report *rep, void *stream) {
    if (!s || !resident || !d_cache || !d_meta || !out) { set_error("null argument"); return AMR_EINVAL; }
    if (meta_bytes < (int64_t)s->meta.size()) {
        set_error("meta buffer %lld < %lld bytes", (long long)meta_bytes, (long long)s->meta.size());
        return AMR_ECAPACITY;
    }
    if (cache_bytes % 4 != 0 || ((uintptr_t)d_cache & 255) != 0) {
        set_error("the cache must be 256-byte aligned and a whole number of floats");
        return AMR_EINVAL;
    }
    amr_store_report R{};
    hipStream_t st = (hipStream_t)stream;
    const int64_t cap = cache_bytes / 4;
    int64_t need = 0;
    for (int p = 0; p < s->np; p++)
        if (resident[p]) need += s->bsz[p];
    if (need > cap - 2 * kPadFloats) {
        set_error("resident bricks need %lld bytes, the cache holds %lld", (long long)(4 * (need + 2 * kPadFloats)),
                  (long long)cache_bytes);
        return AMR_ECAPACITY;
    }
    const bool new_cache = d_cache != s->cache || cap != s->cache_floats;
    if (new_cache) {
        s->cache = d_cache;
        s->cache_floats = cap;
        free_reset(s);
        R.repacked = 1;
    }
    try {
        for (int p = 0; p < s->np; p++)
            if (s->slot[p] >= 0 && !resident[p]) {
                free_give(s, s->slot[p], s->bsz[p]);
                s->slot[p] = -1;
                R.evicted_bricks++;
            }
        // new bricks, largest first, into the best-fitting holes
        std::vector<int> fresh;
        for (int p = 0; p < s->np; p++)
            if (resident[p] && s->slot[p] < 0) fresh.push_back(p);
        std::stable_sort(fresh.begin(), fresh.end(), [&](int x, int y) { return s->bsz[x] > s->bsz[y]; });
        bool fits = true;
        for (int p : fresh) {
            int64_t at;
            if (!free_take(s, s->bsz[p], &at)) { fits = false; break; }
            s->slot[p] = at;
        }
        if (!fits) {
            // fragmented: slide the kept bricks down in slot order (re-sent from the host copy,
            // only those that move), then place the new ones after them
            for (int p : fresh) s->slot[p] = -1;
            std::vector<int> kept;
            for (int p = 0; p < s->np; p++)
                if (s->slot[p] >= 0) kept.push_back(p);
            std::sort(kept.begin(), kept.end(), [&](int x, int y) { return s->slot[x] < s->slot[y]; });
            int64_t cursor = kPadFloats;
            std::vector<int> moved;
            for (int p : kept) {
                if (s->slot[p] != cursor) moved.push_back(p);
                s->slot[p] = cursor;
                cursor += s->bsz[p];
            }
            for (int p : fresh) {
                s->slot[p] = cursor;
                cursor += s->bsz[p];
            }
            s->free_.clear();
            if (cursor < s->cache_floats - kPadFloats) s->free_[cursor] = s->cache_floats - kPadFloats - cursor;
            fresh.insert(fresh.begin(), moved.begin(), moved.end());
            R.repacked = 1;
        }
        if (new_cache) {   // a cache laid out from scratch: pads and free slots hold zeros
            if (s->host_dst) memset(d_cache, 0, (size_t)cache_bytes);
            else {
                hipError_t e = hipMemsetAsync(d_cache, 0, (size_t)cache_bytes, st);
                if (e != hipSuccess) { set_error("HIP memset failed: %s", hipGetErrorString(e)); return AMR_EHIP; }
            }
        }
        const DPatch *P0 = (const DPatch *)(s->meta.data() + s->o_patch);
        float *cache = (float *)d_cache;
        for (int p : fresh) {
            int rc = copy_out(s, cache + s->slot[p], s->pool.data() + P0[p].off, 4 * (size_t)s->bsz[p], st);
            if (rc != AMR_OK) return rc;
            R.uploaded_bricks++;
            R.uploaded_bytes += 4 * s->bsz[p];
        }
        // metadata: slot offsets, leaves of absent patches moved to their finest resident holder
        std::vector<uint8_t> m = s->meta;
        uint8_t *mb = m.data();
        DPatch *P = (DPatch *)(mb + s->o_patch);
        for (int p = 0; p < s->np; p++) {
            P[p].off = resident[p] ? (uint64_t)s->slot[p] : 0;
            if (resident[p]) {
                R.resident_bricks++;
                R.resident_bytes += 4 * s->bsz[p];
            }
        }
        DLeaf *L = (DLeaf *)(mb + s->o_leaves);
        int32_t *own = (int32_t *)(mb + s->o_faces);
        DFaceXf *fx = (DFaceXf *)(mb + s->o_fxf);
        DNode *dn = (DNode *)(mb + s->o_nodes);
        auto to_root = [&](int64_t k, int f) {
            own[6 * k + f] = -2;
            memset(&fx[6 * k + f], 0, sizeof(DFaceXf));
        };
        for (int64_t k = 0; k < s->nrec; k++) {
            const int p0 = L[k].patch;
            if (p0 < 0) continue;
            int h = -1;
            for (int32_t c = s->chain_at[k]; c < s->chain_at[k + 1]; c++)
                if (resident[s->chain[c]]) h = s->chain[c];   // coarse to fine: the last is the finest
            if (h == p0) {
                for (int f = 0; f < 6; f++)
                    if (own[6 * k + f] >= 0 && !resident[own[6 * k + f]]) to_root(k, f);
                continue;
            }
            R.remapped_leaves++;
            for (int f = 0; f < 6; f++) to_root(k, f);
            if (h >= 0) {
                L[k].patch = h;
                L[k].level_flags = (uint32_t)s->plevel[h];
                const uint64_t key = ((uint64_t)k << 32) | (uint32_t)h;
                auto it = s->range_memo.find(key);
                if (it == s->range_memo.end()) {
                    float mn, mx;
                    leaf_range(s, h, &s->rbox[6 * k], &s->rbox[6 * k + 3], &mn, &mx);
                    it = s->range_memo.emplace(key, std::make_pair(mn, mx)).first;
                }
                L[k].vmin = it->second.first;
                L[k].vmax = it->second.second;
            } else {
                L[k].patch = -1;
                L[k].level_flags &= 0xffu;
                L[k].vmin = L[k].vmax = 0.0f;
                if (k >= s->nl0) {   // a level-of-detail node with nothing to draw it from
                    DNode &d = dn[s->lod_node[k - s->nl0]];
                    d.meta &= 0xffu;
                }
            }
        }
        // single-owner face records name the owner's brick by its offset: now its cache slot
        for (int64_t k = 0; k < 6 * s->nrec; k++)
            if (own[k] >= 0) fx[k].off = (uint64_t)s->slot[own[k]];
        int rc = copy_out(s, d_meta, mb, m.size(), st);
        if (rc != AMR_OK) return rc;
        if (!s->host_dst) {
            hipError_t e = hipStreamSynchronize(st);
            if (e != hipSuccess) { set_error("HIP copy failed: %s", hipGetErrorString(e)); return AMR_EHIP; }
        }
        *out = s->full;
        uint8_t *dm = (uint8_t *)d_meta;
        out->pool = (const float *)d_cache;
        out->nodes = dm + s->o_nodes;
        out->leaves = dm + s->o_leaves;
        out->patches = dm + s->o_patch;
        out->leaf_faces = dm + s->o_faces;
        out->face_taps = dm + s->o_fxf;
        out->pool_bytes = cache_bytes;
    } catch (const std::bad_alloc &) {
        s->cache = nullptr;   // the next update lays the cache out again
        set_error("out of host memory");
        return AMR_ENOMEM;
    }
    if (rep) *rep = R;
    return AMR_OK;
}

void amr_store_free(amr_store *s) { delete s; }

}  // extern "C"
