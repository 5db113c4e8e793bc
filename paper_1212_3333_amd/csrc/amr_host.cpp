// Host side of libamr: hierarchy validation, kD-tree construction (Section 4.1), device tree
// encoding (Section 4.2) and the brick pool with ghost layers (Section 5).
//
// Compiled with -ffp-contract=off: split planes, patch corners and ghost interpolants are
// fixed sequences of correctly rounded FP64 operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "amr_internal.h"

namespace amr {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

namespace {

constexpr int kMaxLevels = 32;
constexpr int64_t kMaxCoord = int64_t(1) << 40;   // finest-level coordinates stay exact in FP64

struct Box {
    int64_t lo[3], hi[3];
    int32_t id;
};

struct Node {
    int64_t lo[3], hi[3];
    int64_t split = 0;
    int32_t axis = -1;
    int32_t level = 0;     // leaf: level of its patch; internal: level of the split
    int32_t patch = -1;    // leaf: owning patch (-1: no data)
    int32_t cover = -1;    // internal: patch held before the split
    int32_t low = -1, high = -1;
};

bool box_overlap(const int64_t *alo, const int64_t *ahi, const int64_t *blo, const int64_t *bhi) {
    for (int a = 0; a < 3; a++)
        if (std::min(ahi[a], bhi[a]) <= std::max(alo[a], blo[a])) return false;
    return true;
}

}  // namespace
}  // namespace amr

struct amr_tree {
    amr_domain dom;
    int lmax = 0;
    std::vector<int64_t> scale;              // r^(lmax - l)
    std::vector<amr::Box> pbox;              // patch boxes, finest-level cells (id = patch)
    std::vector<int32_t> plevel;
    std::vector<amr::Node> nodes;            // index 0 = root
    std::vector<int32_t> preorder;           // node indices, depth-first pre-order
    std::vector<int32_t> leaves;             // node indices of leaves, pre-order
    std::vector<int32_t> kind;               // per node (pool index)
    int64_t B_lo[3], B_hi[3];
    int64_t depth = 0;
};

namespace amr {
namespace {

// ---------------------------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------------------------

int validate(const amr_domain *dom, const amr_patch *patches, int32_t np, amr_tree *T) {
    if (!dom || (!patches && np > 0) || np <= 0) { set_error("null domain/patches or npatches <= 0"); return AMR_EINVAL; }
    if (dom->refine < 2 || dom->nlevels < 1 || dom->nlevels > kMaxLevels) {
        set_error("refine must be >= 2 and nlevels in [1, %d]", kMaxLevels);
        return AMR_EINVAL;
    }
    for (int a = 0; a < 3; a++)
        if (!(dom->h0[a] > 0) || !std::isfinite(dom->h0[a]) || !std::isfinite(dom->origin[a])) {
            set_error("h0 must be positive and finite, origin finite");
            return AMR_EINVAL;
        }
    T->dom = *dom;
    T->lmax = dom->nlevels - 1;
    T->scale.assign(dom->nlevels, 1);
    __int128 s = 1;
    for (int l = T->lmax; l >= 0; l--) {
        if (s > kMaxCoord) { set_error("refine^(nlevels-1) too large"); return AMR_EINVAL; }
        T->scale[l] = (int64_t)s;
        s *= dom->refine;
    }
    T->pbox.resize(np);
    T->plevel.resize(np);
    bool have0 = false;
    for (int i = 0; i < np; i++) {
        const amr_patch &p = patches[i];
        if (p.level < 0 || p.level >= dom->nlevels) { set_error("patch %d: level %d out of range", i, p.level); return AMR_EHIERARCHY; }
        T->plevel[i] = p.level;
        Box &b = T->pbox[i];
        b.id = i;
        for (int a = 0; a < 3; a++) {
            if (p.dims[a] < 1) { set_error("patch %d: empty (dims < 1)", i); return AMR_EHIERARCHY; }
            __int128 lo = (__int128)p.lo[a] * T->scale[p.level];
            __int128 hi = ((__int128)p.lo[a] + p.dims[a]) * T->scale[p.level];
            if (lo < -kMaxCoord || hi > kMaxCoord) { set_error("patch %d: coordinates too large", i); return AMR_EHIERARCHY; }
            b.lo[a] = (int64_t)lo;
            b.hi[a] = (int64_t)hi;
        }
        if (p.level == 0) {
            for (int a = 0; a < 3; a++) {
                if (!have0 || b.lo[a] < T->B_lo[a]) T->B_lo[a] = b.lo[a];
                if (!have0 || b.hi[a] > T->B_hi[a]) T->B_hi[a] = b.hi[a];
            }
            have0 = true;
        }
    }
    if (!have0) { set_error("no level-0 patch"); return AMR_EHIERARCHY; }
    for (int i = 0; i < np; i++)
        for (int a = 0; a < 3; a++)
            if (T->pbox[i].lo[a] < T->B_lo[a] || T->pbox[i].hi[a] > T->B_hi[a]) {
                set_error("patch %d (level %d) lies outside the root bounding box", i, T->plevel[i]);
                return AMR_EHIERARCHY;
            }
    // same-level disjointness: sweep over x per level
    for (int l = 0; l < dom->nlevels; l++) {
        std::vector<int> ids;
        for (int i = 0; i < np; i++) if (T->plevel[i] == l) ids.push_back(i);
        std::sort(ids.begin(), ids.end(), [&](int x, int y) { return T->pbox[x].lo[0] < T->pbox[y].lo[0]; });
        std::vector<int> active;
        for (int id : ids) {
            const Box &b = T->pbox[id];
            size_t w = 0;
            for (size_t k = 0; k < active.size(); k++) {
                const Box &c = T->pbox[active[k]];
                if (c.hi[0] <= b.lo[0]) continue;   // no longer active
                active[w++] = active[k];
                if (box_overlap(b.lo, b.hi, c.lo, c.hi)) {
                    set_error("patches %d and %d of level %d overlap", active[k], id, l);
                    return AMR_EHIERARCHY;
                }
            }
            active.resize(w);
            active.push_back(id);
        }
    }
    return AMR_OK;
}

// ---------------------------------------------------------------------------------------------
// kD construction (Section 4.1)
// ---------------------------------------------------------------------------------------------

struct Builder {
    amr_tree *T;

    int new_node(const int64_t *lo, const int64_t *hi, int patch, int level) {
        Node n;
        for (int a = 0; a < 3; a++) { n.lo[a] = lo[a]; n.hi[a] = hi[a]; }
        n.patch = patch;
        n.level = level;
        T->nodes.push_back(n);
        return (int)T->nodes.size() - 1;
    }

    // Picks the plane minimising (boxes cut, -balance, axis, position) among the faces of
    // the boxes strictly inside the node. Cut counts come from sorted face lists:
    // cut(c) = #{lo < c} - #{hi <= c}.
    bool choose(const Node &nd, const std::vector<Box> &S, int *axis, int64_t *pos) {
        bool have = false;
        int64_t bcost = 0, bmn = 0, bmx = 1;
        int ba = 0;
        int64_t bc = 0;
        std::vector<int64_t> los(S.size()), his(S.size()), faces;
        for (int a = 0; a < 3; a++) {
            for (size_t i = 0; i < S.size(); i++) { los[i] = S[i].lo[a]; his[i] = S[i].hi[a]; }
            std::sort(los.begin(), los.end());
            std::sort(his.begin(), his.end());
            faces.clear();
            std::merge(los.begin(), los.end(), his.begin(), his.end(), std::back_inserter(faces));
            faces.erase(std::unique(faces.begin(), faces.end()), faces.end());
            for (int64_t c : faces) {
                if (c <= nd.lo[a] || c >= nd.hi[a]) continue;
                int64_t cost = (int64_t)(std::lower_bound(los.begin(), los.end(), c) - los.begin()) -
                               (int64_t)(std::upper_bound(his.begin(), his.end(), c) - his.begin());
                int64_t l = c - nd.lo[a], r = nd.hi[a] - c;
                int64_t mn = std::min(l, r), mx = std::max(l, r);
                bool better;
                if (!have) better = true;
                else if (cost != bcost) better = cost < bcost;
                else {
                    __int128 x = (__int128)mn * bmx, y = (__int128)bmn * mx;
                    if (x != y) better = x > y;
                    else better = (a < ba) || (a == ba && c < bc);
                }
                if (better) { have = true; bcost = cost; bmn = mn; bmx = mx; ba = a; bc = c; }
            }
        }
        *axis = ba;
        *pos = bc;
        return have;
    }

    static std::vector<Box> clip(const std::vector<Box> &S, const int64_t *lo, const int64_t *hi) {
        std::vector<Box> out;
        out.reserve(S.size());
        for (const Box &b : S) {
            Box c = b;
            bool ok = true;
            for (int a = 0; a < 3; a++) {
                c.lo[a] = std::max(b.lo[a], lo[a]);
                c.hi[a] = std::min(b.hi[a], hi[a]);
                if (c.hi[a] <= c.lo[a]) { ok = false; break; }
            }
            if (ok) out.push_back(c);
        }
        return out;
    }

    int split(int ni, int level, const std::vector<Box> &S) {
        if (S.empty()) return AMR_OK;
        {
            const Node &nd = T->nodes[ni];
            if (S.size() == 1) {
                bool same = true;
                for (int a = 0; a < 3; a++) same = same && S[0].lo[a] == nd.lo[a] && S[0].hi[a] == nd.hi[a];
                if (same) {
                    T->nodes[ni].patch = S[0].id;
                    T->nodes[ni].level = level;
                    return AMR_OK;
                }
            }
        }
        int axis;
        int64_t c;
        if (!choose(T->nodes[ni], S, &axis, &c)) {
            set_error("no admissible split plane at level %d", level);
            return AMR_EHIERARCHY;
        }
        Node nd = T->nodes[ni];   // copy: push_back below may reallocate
        int64_t lhi[3] = {nd.hi[0], nd.hi[1], nd.hi[2]}, hlo[3] = {nd.lo[0], nd.lo[1], nd.lo[2]};
        lhi[axis] = c;
        hlo[axis] = c;
        int lo_i = new_node(nd.lo, lhi, nd.patch, nd.level);
        int hi_i = new_node(hlo, nd.hi, nd.patch, nd.level);
        Node &me = T->nodes[ni];
        me.cover = nd.patch;
        me.axis = axis;
        me.split = c;
        me.level = level;
        me.patch = -1;
        me.low = lo_i;
        me.high = hi_i;
        int rc = split(lo_i, level, clip(S, T->nodes[lo_i].lo, T->nodes[lo_i].hi));
        if (rc) return rc;
        return split(hi_i, level, clip(S, T->nodes[hi_i].lo, T->nodes[hi_i].hi));
    }

    // Leaves overlapping box b, found top-down from the root visiting only children that
    // intersect b (Section 4.1).
    void overlapping_leaves(const Box &b, std::vector<int> &out) {
        std::vector<int> stack{0};
        while (!stack.empty()) {
            int i = stack.back();
            stack.pop_back();
            const Node &n = T->nodes[i];
            if (!box_overlap(n.lo, n.hi, b.lo, b.hi)) continue;
            if (n.axis < 0) out.push_back(i);
            else { stack.push_back(n.high); stack.push_back(n.low); }
        }
    }

    int build() {
        T->nodes.clear();
        T->nodes.reserve(T->pbox.size() * 16 + 16);
        new_node(T->B_lo, T->B_hi, -1, 0);
        std::vector<Box> lev0;
        for (size_t i = 0; i < T->pbox.size(); i++) if (T->plevel[i] == 0) lev0.push_back(T->pbox[i]);
        int rc = split(0, 0, clip(lev0, T->B_lo, T->B_hi));
        if (rc) return rc;
        for (int l = 1; l <= T->lmax; l++) {
            std::vector<std::vector<Box>> per_leaf_boxes;
            std::vector<int> leaf_of;           // node index per list
            std::vector<int> slot(T->nodes.size(), -1);
            std::vector<int> hits;
            for (size_t i = 0; i < T->pbox.size(); i++) {
                if (T->plevel[i] != l) continue;
                hits.clear();
                overlapping_leaves(T->pbox[i], hits);
                for (int leaf : hits) {
                    if (slot[leaf] < 0) {
                        slot[leaf] = (int)per_leaf_boxes.size();
                        per_leaf_boxes.emplace_back();
                        leaf_of.push_back(leaf);
                    }
                    per_leaf_boxes[slot[leaf]].push_back(T->pbox[i]);
                }
            }
            for (size_t k = 0; k < leaf_of.size(); k++) {
                int leaf = leaf_of[k];
                Node nd = T->nodes[leaf];
                rc = split(leaf, l, clip(per_leaf_boxes[k], nd.lo, nd.hi));
                if (rc) return rc;
            }
        }
        return AMR_OK;
    }

    void finish() {
        // pre-order (low first), leaf ids, depth, kinds
        T->preorder.clear();
        T->leaves.clear();
        std::vector<std::pair<int, int>> stack{{0, 0}};
        T->depth = 0;
        while (!stack.empty()) {
            auto [i, d] = stack.back();
            stack.pop_back();
            T->preorder.push_back(i);
            const Node &n = T->nodes[i];
            if (n.axis < 0) {
                T->leaves.push_back(i);
                T->depth = std::max<int64_t>(T->depth, d);
            } else {
                stack.push_back({n.high, d + 1});
                stack.push_back({n.low, d + 1});
            }
        }
        // kinds: (a) = internal node inside one subgrid whose cells are all refined further
        std::vector<int> minlev(T->nodes.size(), 0);
        for (auto it = T->preorder.rbegin(); it != T->preorder.rend(); ++it) {
            const Node &n = T->nodes[*it];
            minlev[*it] = n.axis < 0 ? n.level : std::min(minlev[n.low], minlev[n.high]);
        }
        T->kind.assign(T->nodes.size(), 1);
        for (size_t i = 0; i < T->nodes.size(); i++) {
            const Node &n = T->nodes[i];
            if (n.axis < 0) T->kind[i] = 1;
            else if (n.cover >= 0 && minlev[i] > T->plevel[n.cover]) T->kind[i] = 0;
            else T->kind[i] = 2;
        }
    }
};

// ---------------------------------------------------------------------------------------------
// Ghost layers and pool (Section 5)
// ---------------------------------------------------------------------------------------------

inline int64_t fdiv(int64_t a, int64_t b) {  // floor division, b > 0
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

struct Packer {
    const amr_tree *T;
    const amr_patch *P;
    int np;
    int vertex;                               // 1: vertex-centred samples, n+1 per axis
    std::vector<std::vector<double>> brick;   // FP64 padded bricks (samples + 2 per axis)
    std::vector<std::vector<int>> nbr;        // patches of level <= own meeting the dilated box

    // brick entry of sample (i, j, k); -1 and n (cells) or n + 1 (vertices) are the shell
    double &at(int p, int64_t i, int64_t j, int64_t k) {
        const int64_t *n = P[p].dims;
        const int64_t sx = n[0] + vertex + 2, sy = n[1] + vertex + 2;
        return brick[p][(size_t)((i + 1) + sx * ((j + 1) + sy * (k + 1)))];
    }

    // Interior cell of patch q holding the level-l cell centre c2 (twice the finest coordinate).
    double copy_cell(int q, const int64_t *c2, int64_t S) {
        int64_t m[3];
        for (int a = 0; a < 3; a++) m[a] = (c2[a] - S) / (2 * S) - P[q].lo[a];
        return (double)P[q].cells[m[0] + P[q].dims[0] * (m[1] + P[q].dims[1] * m[2])];
    }

    bool holds(int q, const int64_t *c2) const {
        for (int a = 0; a < 3; a++)
            if (c2[a] < 2 * T->pbox[q].lo[a] || c2[a] >= 2 * T->pbox[q].hi[a]) return false;
        return true;
    }

    double coarse_interp(int q, const int64_t *c2) {
        int64_t Sq = T->scale[T->plevel[q]];
        int64_t i0[3];
        double f[3];
        for (int a = 0; a < 3; a++) {
            // level-q continuous index of the point minus one half, as (num / den)
            int64_t num = c2[a] - 2 * T->pbox[q].lo[a] - Sq, den = 2 * Sq;
            i0[a] = fdiv(num, den);
            f[a] = (double)(num - i0[a] * den) / (double)den;
        }
        double v[2][2][2];
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) v[dz][dy][dx] = at(q, i0[0] + dx, i0[1] + dy, i0[2] + dz);
        double x00 = v[0][0][0] + f[0] * (v[0][0][1] - v[0][0][0]);
        double x10 = v[0][1][0] + f[0] * (v[0][1][1] - v[0][1][0]);
        double x01 = v[1][0][0] + f[0] * (v[1][0][1] - v[1][0][0]);
        double x11 = v[1][1][0] + f[0] * (v[1][1][1] - v[1][1][0]);
        double y0 = x00 + f[1] * (x10 - x00);
        double y1 = x01 + f[1] * (x11 - x01);
        return y0 + f[2] * (y1 - y0);
    }

    double ghost(int p, int64_t i, int64_t j, int64_t k) {
        int l = T->plevel[p];
        int64_t S = T->scale[l];
        int64_t idx[3] = {i, j, k};
        int64_t c2[3];
        for (int a = 0; a < 3; a++) c2[a] = (2 * (P[p].lo[a] + idx[a]) + 1) * S;
        for (int pass = 0; pass < 2; pass++) {
            for (int q : nbr[p])        // same level: exact copy
                if (T->plevel[q] == l && holds(q, c2)) return copy_cell(q, c2, S);
            bool moved = false;
            for (int a = 0; a < 3; a++) {   // outside B: clamp the centre into B, retry
                int64_t lo = 2 * T->B_lo[a] + S, hi = 2 * T->B_hi[a] - S;
                if (c2[a] < lo) { c2[a] = lo; moved = true; }
                if (c2[a] > hi) { c2[a] = hi; moved = true; }
            }
            if (moved && pass == 0) continue;
            int best = -1;             // finest coarser patch holding the centre
            for (int q : nbr[p])
                if (T->plevel[q] < l && holds(q, c2) && (best < 0 || T->plevel[q] > T->plevel[best])) best = q;
            if (best >= 0) return coarse_interp(best, c2);
            break;
        }
        int64_t m[3];                  // no coarser data: nearest interior cell
        for (int a = 0; a < 3; a++) m[a] = std::min<int64_t>(std::max<int64_t>(idx[a], 0), P[p].dims[a] - 1);
        return (double)P[p].cells[m[0] + P[p].dims[0] * (m[1] + P[p].dims[1] * m[2])];
    }

    void fill_patch(int p) {
        const int64_t *n = P[p].dims;
        brick[p].assign((size_t)((n[0] + 2) * (n[1] + 2) * (n[2] + 2)), 0.0);
        for (int64_t k = 0; k < n[2]; k++)
            for (int64_t j = 0; j < n[1]; j++)
                for (int64_t i = 0; i < n[0]; i++) at(p, i, j, k) = (double)P[p].cells[i + n[0] * (j + n[1] * k)];
        for (int64_t k = -1; k <= n[2]; k++)
            for (int64_t j = -1; j <= n[1]; j++) {
                bool inner_row = (k >= 0 && k < n[2] && j >= 0 && j < n[1]);
                for (int64_t i = -1; i <= n[0]; i++) {
                    if (inner_row && i >= 0 && i < n[0]) { i = n[0] - 1; continue; }
                    at(p, i, j, k) = ghost(p, i, j, k);
                }
            }
    }

    void neighbours(int nthreads) {
        nbr.assign(np, {});
        // bin patches on a coarse grid over B to find box neighbours quickly
        const int G = 32;
        int64_t ext[3];
        for (int a = 0; a < 3; a++) ext[a] = T->B_hi[a] - T->B_lo[a];
        auto cell_of = [&](int a, int64_t x) {
            int64_t c = fdiv((x - T->B_lo[a]) * G, ext[a]);
            return (int)std::min<int64_t>(std::max<int64_t>(c, 0), G - 1);
        };
        std::vector<std::vector<int>> bins((size_t)G * G * G);
        for (int q = 0; q < np; q++) {
            const Box &b = T->pbox[q];
            for (int z = cell_of(2, b.lo[2]); z <= cell_of(2, b.hi[2]); z++)
                for (int y = cell_of(1, b.lo[1]); y <= cell_of(1, b.hi[1]); y++)
                    for (int x = cell_of(0, b.lo[0]); x <= cell_of(0, b.hi[0]); x++) bins[(size_t)x + G * (y + G * z)].push_back(q);
        }
        auto work = [&](int t) {
            std::vector<char> seen(np, 0);
            for (int p = t; p < np; p += nthreads) {
                int64_t S = T->scale[T->plevel[p]];
                int64_t lo[3], hi[3];
                for (int a = 0; a < 3; a++) { lo[a] = T->pbox[p].lo[a] - S; hi[a] = T->pbox[p].hi[a] + S; }
                std::vector<int> &out = nbr[p];
                for (int z = cell_of(2, lo[2]); z <= cell_of(2, hi[2]); z++)
                    for (int y = cell_of(1, lo[1]); y <= cell_of(1, hi[1]); y++)
                        for (int x = cell_of(0, lo[0]); x <= cell_of(0, hi[0]); x++)
                            for (int q : bins[(size_t)x + G * (y + G * z)]) {
                                if (seen[q] || T->plevel[q] > T->plevel[p]) continue;
                                const Box &b = T->pbox[q];
                                bool meet = true;
                                for (int a = 0; a < 3; a++) meet = meet && b.hi[a] >= lo[a] && b.lo[a] <= hi[a];
                                if (meet) { seen[q] = 1; out.push_back(q); }
                            }
                for (int q : out) seen[q] = 0;
            }
        };
        std::vector<std::thread> th;
        for (int t = 0; t < nthreads; t++) th.emplace_back(work, t);
        for (auto &x : th) x.join();
    }

    // Vertex-centred data (Section 5).  Patch owning the finest-level cell c: the kD leaf
    // holding it (half-open split planes); -1 for a leaf without data.
    int cell_owner(const int64_t *c) const {
        int ni = 0;
        while (T->nodes[ni].axis >= 0) {
            const Node &n = T->nodes[ni];
            ni = c[n.axis] < n.split ? n.low : n.high;
        }
        return T->nodes[ni].patch;
    }

    // Trilinear value of patch q's samples at the vertex with finest-level coordinates G, a
    // point of q's closed box (base index kept in [0, n-1], so a point on the upper face takes
    // the last cell with weight one).
    double vertex_value(int q, const int64_t *G) {
        const int64_t Sq = T->scale[T->plevel[q]];
        int64_t i0[3];
        double f[3];
        for (int a = 0; a < 3; a++) {
            const int64_t num = G[a] - T->pbox[q].lo[a];
            i0[a] = std::min<int64_t>(std::max<int64_t>(fdiv(num, Sq), 0), P[q].dims[a] - 1);
            f[a] = (double)(num - i0[a] * Sq) / (double)Sq;
        }
        double v[2][2][2];
        for (int dz = 0; dz < 2; dz++)
            for (int dy = 0; dy < 2; dy++)
                for (int dx = 0; dx < 2; dx++) v[dz][dy][dx] = at(q, i0[0] + dx, i0[1] + dy, i0[2] + dz);
        double x00 = v[0][0][0] + f[0] * (v[0][0][1] - v[0][0][0]);
        double x10 = v[0][1][0] + f[0] * (v[0][1][1] - v[0][1][0]);
        double x01 = v[1][0][0] + f[0] * (v[1][0][1] - v[1][0][0]);
        double x11 = v[1][1][0] + f[0] * (v[1][1][1] - v[1][1][0]);
        double y0 = x00 + f[1] * (x10 - x00);
        double y1 = x01 + f[1] * (x11 - x01);
        return y0 + f[2] * (y1 - y0);
    }

    // Samples of a vertex-centred patch with the dangling-node fix: a sample on the patch
    // boundary whose eight surrounding finest cells (those in B) have a coarsest owner coarser
    // than the patch takes that owner's interpolated value (first such owner in octant order,
    // bit a of the octant set for the + side of axis a).  Coarser levels are final before this
    // runs.  The shell replicates the nearest sample: the kernels read it only with weight zero,
    // or with a rounding-sized weight for a position a few ulps outside the box.
    void fill_vertex(int p) {
        const int64_t *n = P[p].dims;
        const int64_t nx = n[0] + 1, ny = n[1] + 1, nz = n[2] + 1;
        brick[p].assign((size_t)((nx + 2) * (ny + 2) * (nz + 2)), 0.0);
        const int l = T->plevel[p];
        const int64_t S = T->scale[l];
        for (int64_t k = 0; k < nz; k++)
            for (int64_t j = 0; j < ny; j++)
                for (int64_t i = 0; i < nx; i++) {
                    double v = (double)P[p].cells[i + nx * (j + ny * k)];
                    if (i == 0 || j == 0 || k == 0 || i == n[0] || j == n[1] || k == n[2]) {
                        const int64_t G[3] = {T->pbox[p].lo[0] + i * S, T->pbox[p].lo[1] + j * S,
                                              T->pbox[p].lo[2] + k * S};
                        int m = l, own = -1;
                        for (int o = 0; o < 8; o++) {
                            int64_t c[3];
                            bool inB = true;
                            for (int a = 0; a < 3; a++) {
                                c[a] = ((o >> a) & 1) ? G[a] : G[a] - 1;
                                inB = inB && c[a] >= T->B_lo[a] && c[a] < T->B_hi[a];
                            }
                            if (!inB) continue;
                            const int q = cell_owner(c);
                            if (q >= 0 && T->plevel[q] < m) { m = T->plevel[q]; own = q; }
                        }
                        if (own >= 0) v = vertex_value(own, G);
                    }
                    at(p, i, j, k) = v;
                }
        for (int64_t k = -1; k <= nz; k++)
            for (int64_t j = -1; j <= ny; j++)
                for (int64_t i = -1; i <= nx; i++) {
                    if (i >= 0 && j >= 0 && k >= 0 && i < nx && j < ny && k < nz) continue;
                    at(p, i, j, k) = at(p, std::min<int64_t>(std::max<int64_t>(i, 0), nx - 1),
                                        std::min<int64_t>(std::max<int64_t>(j, 0), ny - 1),
                                        std::min<int64_t>(std::max<int64_t>(k, 0), nz - 1));
                }
    }

    void run(int nthreads) {
        brick.assign(np, {});
        if (!vertex) neighbours(nthreads);
        for (int l = 0; l <= T->lmax; l++) {      // coarser bricks are complete before finer ones
            std::vector<int> ids;
            for (int p = 0; p < np; p++) if (T->plevel[p] == l) ids.push_back(p);
            std::atomic<size_t> next{0};
            auto work = [&]() {
                for (size_t k; (k = next.fetch_add(1)) < ids.size();) {
                    if (vertex) fill_vertex(ids[k]);
                    else fill_patch(ids[k]);
                }
            };
            std::vector<std::thread> th;
            for (int t = 0; t < nthreads; t++) th.emplace_back(work);
            for (auto &x : th) x.join();
        }
    }
};

// For each face 2a+side of a leaf: the patch owning the whole one-cell slab (cells of the
// leaf's level) beyond the face when a single patch holds every leaf meeting it and the slab
// lies inside B, else -1.  The returned mask has bit 2a+side set when that owner is the leaf's
// own patch (the gradient tap then reads the same brick).
uint32_t face_owners(const amr_tree *T, const Node &lf, const std::vector<int32_t> &bfs_index, int32_t owner[6]) {
    for (int f = 0; f < 6; f++) owner[f] = -1;
    if (lf.patch < 0) return 0;
    const int64_t S = T->scale[T->plevel[lf.patch]];
    uint32_t mask = 0;
    std::vector<int> stack;
    for (int a = 0; a < 3; a++)
        for (int side = 0; side < 2; side++) {
            int64_t lo[3] = {lf.lo[0], lf.lo[1], lf.lo[2]}, hi[3] = {lf.hi[0], lf.hi[1], lf.hi[2]};
            if (side) { lo[a] = lf.hi[a]; hi[a] = lf.hi[a] + S; }
            else { lo[a] = lf.lo[a] - S; hi[a] = lf.lo[a]; }
            bool ok = true;
            for (int b = 0; b < 3; b++) ok = ok && lo[b] >= T->B_lo[b] && hi[b] <= T->B_hi[b];
            const bool inB = ok;
            int own = -2;
            stack.assign(1, 0);
            while (ok && !stack.empty()) {
                int i = stack.back();
                stack.pop_back();
                const Node &n = T->nodes[i];
                if (!box_overlap(n.lo, n.hi, lo, hi)) continue;
                if (n.axis >= 0) { stack.push_back(n.low); stack.push_back(n.high); continue; }
                if (n.patch < 0 || (own != -2 && own != n.patch)) ok = false;
                else own = n.patch;
            }
            if (ok && own >= 0) {
                owner[2 * a + side] = own;
                if (own == lf.patch) mask |= 1u << (2 * a + side);
            } else if (inB) {
                // several owners: the smallest node whose box holds the whole slab (a rope)
                int ni = 0;
                while (T->nodes[ni].axis >= 0) {
                    const Node &n = T->nodes[ni];
                    const Node &lo_c = T->nodes[n.low];
                    if (hi[n.axis] <= lo_c.hi[n.axis]) ni = n.low;
                    else if (lo[n.axis] >= lo_c.hi[n.axis]) ni = n.high;
                    else break;
                }
                owner[2 * a + side] = -2 - bfs_index[ni];
            }
        }
    return mask;
}

double world_plane(const amr_tree *T, int a, int64_t G) {
    double g = (double)G;
    double hf = T->dom.h0[a] / (double)T->scale[0];
    double m = g * hf;
    return T->dom.origin[a] + m;
}

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

}  // namespace
}  // namespace amr

using namespace amr;

extern "C" {

const char *amr_last_error(void) { return g_err.c_str(); }

int amr_build_kdtree(const amr_domain *dom, const amr_patch *patches, int32_t npatches, amr_tree **out) {
    if (!out) { set_error("out is NULL"); return AMR_EINVAL; }
    *out = nullptr;
    amr_tree *T = new (std::nothrow) amr_tree();
    if (!T) { set_error("out of host memory"); return AMR_ENOMEM; }
    try {
        int rc = validate(dom, patches, npatches, T);
        if (rc) { delete T; return rc; }
        Builder b{T};
        rc = b.build();
        if (rc) { delete T; return rc; }
        b.finish();
    } catch (const std::bad_alloc &) {
        delete T;
        set_error("out of host memory");
        return AMR_ENOMEM;
    }
    *out = T;
    return AMR_OK;
}

int amr_tree_stats(const amr_tree *T, amr_tree_info *s) {
    if (!T || !s) { set_error("null argument"); return AMR_EINVAL; }
    memset(s, 0, sizeof(*s));
    s->nodes = (int64_t)T->nodes.size();
    s->leaves = (int64_t)T->leaves.size();
    for (size_t i = 0; i < T->nodes.size(); i++) {
        if (T->kind[i] == 0) s->n_a++;
        else if (T->kind[i] == 1) s->n_b++;
        else s->n_c++;
    }
    for (int li : T->leaves) if (T->nodes[li].patch < 0) s->empty_leaves++;
    s->depth = T->depth;
    s->npatches = (int64_t)T->pbox.size();
    return AMR_OK;
}

int amr_tree_export(const amr_tree *T, amr_node_host *nodes, size_t ncap, amr_leaf_host *leaves, size_t lcap) {
    if (!T) { set_error("null tree"); return AMR_EINVAL; }
    if (nodes) {
        if (ncap < T->preorder.size()) { set_error("node capacity %zu < %zu", ncap, T->preorder.size()); return AMR_ECAPACITY; }
        for (size_t k = 0; k < T->preorder.size(); k++) {
            const Node &n = T->nodes[T->preorder[k]];
            amr_node_host &o = nodes[k];
            memset(&o, 0, sizeof(o));
            o.axis = n.axis;
            o.level = n.level;
            o.split = n.axis >= 0 ? n.split : 0;
            o.patch = n.axis < 0 ? n.patch : -1;
            o.cover = n.axis >= 0 ? n.cover : -1;
            o.kind = T->kind[T->preorder[k]];
        }
    }
    if (leaves) {
        if (lcap < T->leaves.size()) { set_error("leaf capacity %zu < %zu", lcap, T->leaves.size()); return AMR_ECAPACITY; }
        for (size_t k = 0; k < T->leaves.size(); k++) {
            const Node &n = T->nodes[T->leaves[k]];
            amr_leaf_host &o = leaves[k];
            for (int a = 0; a < 3; a++) { o.lo[a] = n.lo[a]; o.hi[a] = n.hi[a]; }
            o.patch = n.patch;
            o.level = n.level;
        }
    }
    return AMR_OK;
}

void amr_tree_free(amr_tree *T) { delete T; }

int amr_pack_pool(const amr_tree *T, const amr_patch *patches, int32_t npatches, const amr_pack_opts *opts,
                  void *d_pool, int64_t *pool_bytes, void *d_meta, int64_t *meta_bytes, amr_scene *out,
                  void *stream) {
    if (!T || !patches || !pool_bytes || !meta_bytes) { set_error("null argument"); return AMR_EINVAL; }
    if (npatches != (int32_t)T->pbox.size()) { set_error("npatches differs from the tree's"); return AMR_EINVAL; }
    const int np = npatches;
    const int layout = opts ? opts->brick_layout : 0;
    if (layout < 0 || layout > 2) { set_error("brick_layout must be 0, 1 or 2"); return AMR_EINVAL; }
    const int vertex = opts ? opts->centering : 0;
    if (vertex != 0 && vertex != 1) { set_error("centering must be 0 (cells) or 1 (vertices)"); return AMR_EINVAL; }
    // kernels see a vertex-centred patch of n cells as n + 1 samples at integer positions of
    // its patch-local index (the header's lower corner moves down by half a cell)
    // pool layout: 256-byte aligned padded bricks (linear, or 4^3 micro-bricks)
    std::vector<int64_t> off(np);
    int64_t nfl = 64;   // leading pad: row loads of the linear layout may start one float early
    for (int p = 0; p < np; p++) {
        const int64_t n[3] = {patches[p].dims[0] + vertex, patches[p].dims[1] + vertex, patches[p].dims[2] + vertex};
        if (patches[p].level != T->plevel[p]) { set_error("patch %d differs from the tree's", p); return AMR_EINVAL; }
        off[p] = nfl;
        const int32_t n32[3] = {(int32_t)n[0], (int32_t)n[1], (int32_t)n[2]};
        const int32_t nb[3] = {(n32[0] + 5) / 4, (n32[1] + 5) / 4, (n32[2] + 5) / 4};
        const int64_t cells = brick_floats(layout, n32, nb);
        nfl = align_up(nfl + cells, 64);
    }
    const int64_t nn = (int64_t)T->nodes.size(), nl0 = (int64_t)T->leaves.size();
    // kind-(a) nodes in pre-order: level-of-detail records nl0 + k after the leaves
    std::vector<int32_t> aidx(T->nodes.size(), -1);
    std::vector<int32_t> anodes;
    for (int32_t i : T->preorder)
        if (T->kind[i] == 0) { aidx[i] = (int32_t)anodes.size(); anodes.push_back(i); }
    const int64_t na = (int64_t)anodes.size(), nl = nl0 + na;
    const int64_t o_nodes = 0;
    const int64_t o_leaves = align_up(o_nodes + nn * (int64_t)sizeof(DNode), 256);
    const int64_t o_patch = align_up(o_leaves + nl * (int64_t)sizeof(DLeaf), 256);
    const int64_t o_faces = align_up(o_patch + np * (int64_t)sizeof(DPatch), 256);
    const int64_t o_fxf = align_up(o_faces + nl * 6 * (int64_t)sizeof(int32_t), 256);
    const int64_t mbytes = align_up(o_fxf + nl * 6 * (int64_t)sizeof(DFaceXf), 256);
    const int64_t pbytes = std::max<int64_t>((nfl + 64) * 4, 256);   // trailing pad
    if (!d_pool && !d_meta) {
        *pool_bytes = pbytes;
        *meta_bytes = mbytes;
        return AMR_OK;
    }
    if (!d_pool || !d_meta || !out) { set_error("d_pool, d_meta and out_scene are required"); return AMR_EINVAL; }
    if (*pool_bytes < pbytes || *meta_bytes < mbytes) {
        set_error("buffers too small: pool %lld < %lld or meta %lld < %lld", (long long)*pool_bytes,
                  (long long)pbytes, (long long)*meta_bytes, (long long)mbytes);
        return AMR_ECAPACITY;
    }
    for (int p = 0; p < np; p++)
        if (!patches[p].cells) { set_error("patch %d has no cells", p); return AMR_EINVAL; }
    int nthreads = opts && opts->nthreads > 0 ? opts->nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    bool host_dst = opts && opts->host_dst;

    std::vector<float> pool;
    std::vector<uint8_t> meta;
    try {
        pool.assign((size_t)nfl, 0.0f);
        meta.assign((size_t)mbytes, 0);
        Packer pk{T, patches, np, vertex, {}, {}};
        pk.run(nthreads);
        float vmin = INFINITY, vmax = -INFINITY;
        for (int p = 0; p < np; p++) {
            const std::vector<double> &b = pk.brick[p];
            int32_t n32[3], nb[3];
            for (int a = 0; a < 3; a++) {
                n32[a] = (int32_t)patches[p].dims[a] + vertex;
                nb[a] = (n32[a] + 5) / 4;
            }
            const int64_t px = n32[0] + 2, py = n32[1] + 2, pz = n32[2] + 2;
            if (layout == 2) {
                halo_row_fill(n32, nb, pool.data() + off[p],
                              [&](int64_t i, int64_t j, int64_t k) { return (float)b[(size_t)(i + px * (j + py * k))]; });
                continue;
            }
            for (int64_t k = 0; k < pz; k++)
                for (int64_t j = 0; j < py; j++)
                    for (int64_t i = 0; i < px; i++)
                        pool[(size_t)(off[p] + brick_index(layout, n32, nb, i, j, k))] = (float)b[(size_t)(i + px * (j + py * k))];
        }
        // device tree, breadth first with adjacent children
        DNode *dn = (DNode *)(meta.data() + o_nodes);
        std::vector<int32_t> bfs_index(T->nodes.size(), -1);
        std::vector<int32_t> leaf_id(T->nodes.size(), -1);
        for (size_t k = 0; k < T->leaves.size(); k++) leaf_id[T->leaves[k]] = (int32_t)k;
        std::vector<int32_t> order{0};
        order.reserve(nn);
        for (size_t h = 0; h < order.size(); h++) {
            const Node &n = T->nodes[order[h]];
            bfs_index[order[h]] = (int32_t)h;
            DNode &d = dn[h];
            if (n.axis < 0) {
                d.split = 0.0;
                d.child = (uint32_t)leaf_id[order[h]];
                d.meta = node_meta(kLeafAxis, n.level);
            } else {
                d.split = world_plane(T, n.axis, n.split);
                d.child = (uint32_t)order.size();
                d.meta = node_meta(n.axis, n.level) | (aidx[order[h]] >= 0 ? (uint32_t)(aidx[order[h]] + 1) << 8 : 0u);
                order.push_back(n.low);
                order.push_back(n.high);
            }
        }
        DPatch *dp = (DPatch *)(meta.data() + o_patch);
        for (int p = 0; p < np; p++) {
            DPatch &h = dp[p];
            int l = T->plevel[p];
            h.off = (uint64_t)off[p];
            h.level = l;
            float pmin = INFINITY, pmax = -INFINITY;
            for (double v : pk.brick[p]) { pmin = std::min(pmin, (float)v); pmax = std::max(pmax, (float)v); }
            h.vmin = pmin;
            h.vmax = pmax;
            for (int a = 0; a < 3; a++) h.nb[a] = ((int32_t)patches[p].dims[a] + vertex + 5) / 4;
            h.layout = layout;
            vmin = std::min(vmin, pmin);
            vmax = std::max(vmax, pmax);
            double hmin = INFINITY;
            for (int a = 0; a < 3; a++) {
                h.n[a] = (int32_t)patches[p].dims[a] + vertex;
                double rl = 1.0;
                for (int k = 0; k < l; k++) rl *= (double)T->dom.refine;
                h.h[a] = T->dom.h0[a] / rl;
                h.inv_h[a] = 1.0 / h.h[a];
                h.lo[a] = world_plane(T, a, T->pbox[p].lo[a]);
                if (vertex) h.lo[a] = h.lo[a] - 0.5 * h.h[a];
                hmin = std::min(hmin, T->dom.h0[a]);
            }
            double rl = 1.0;
            for (int k = 0; k < l; k++) rl *= (double)T->dom.refine;
            h.step = hmin / rl;
        }
        DLeaf *dl = (DLeaf *)(meta.data() + o_leaves);
        for (int64_t k = 0; k < nl; k++) {
            const bool virt = k >= nl0;           // a kind-(a) node, rendered from its cover patch
            const Node &n = virt ? T->nodes[anodes[k - nl0]] : T->nodes[T->leaves[k]];
            const int32_t np_k = virt ? n.cover : n.patch;
            DLeaf &L = dl[k];
            for (int a = 0; a < 3; a++) { L.lo[a] = world_plane(T, a, n.lo[a]); L.hi[a] = world_plane(T, a, n.hi[a]); }
            L.patch = np_k;
            int32_t *own = (int32_t *)(meta.data() + o_faces) + 6 * k;
            if (virt) {
                // gradient taps leaving the node are located from the root
                for (int f = 0; f < 6; f++) own[f] = -2;
                L.level_flags = (uint32_t)T->plevel[np_k];
            } else {
                L.level_flags = (uint32_t)n.level | (face_owners(T, n, bfs_index, own) << 8);
            }
            L.vmin = 0.0f;
            L.vmax = 0.0f;
            if (np_k >= 0) {
                // value range over what a sample in the leaf can read: cell-centred, the leaf's
                // cells plus one halo cell; vertex-centred, the vertices of the leaf's cells
                int p = np_k;
                int64_t S = T->scale[T->plevel[p]];
                int64_t i0[3], i1[3];
                for (int a = 0; a < 3; a++) {
                    i0[a] = (n.lo[a] - T->pbox[p].lo[a]) / S;        // first interior index
                    i1[a] = (n.hi[a] - T->pbox[p].lo[a] + S - 1) / S;  // one past the last cell
                }
                const int64_t d[3] = {patches[p].dims[0] + vertex, patches[p].dims[1] + vertex,
                                      patches[p].dims[2] + vertex};
                const int64_t first = vertex ? 0 : 1;
                const std::vector<double> &bk = pk.brick[p];
                float mn = INFINITY, mx = -INFINITY;
                for (int64_t z = i0[2] - first; z <= i1[2]; z++)
                    for (int64_t y = i0[1] - first; y <= i1[1]; y++)
                        for (int64_t x = i0[0] - first; x <= i1[0]; x++) {
                            float v = (float)bk[(size_t)((x + 1) + (d[0] + 2) * ((y + 1) + (d[1] + 2) * (z + 1)))];
                            mn = std::min(mn, v);
                            mx = std::max(mx, v);
                        }
                L.vmin = mn;
                L.vmax = mx;
            }
        }
        // gradient-tap records per leaf face (after the patch headers, which they read)
        DFaceXf *fx = (DFaceXf *)(meta.data() + o_fxf);
        const int32_t *own_all = (const int32_t *)(meta.data() + o_faces);
        for (int64_t k = 0; k < nl; k++) {
            const int p = dl[k].patch;
            for (int f = 0; f < 6; f++) {
                DFaceXf &X = fx[6 * k + f];
                memset(&X, 0, sizeof(X));
                const int32_t o = own_all[6 * k + f];
                if (o >= 0 && p >= 0) {
                    const DPatch &Po = dp[o], &Pp = dp[p];
                    X.off = Po.off;
                    for (int a = 0; a < 3; a++) X.n[a] = Po.n[a];
                    if (layout == 1 || layout == 2) {
                        X.px = (layout == 1 ? 64 : 128) * Po.nb[0];
                        X.pxy = X.px * Po.nb[1];
                    } else {
                        X.px = Po.n[0] + 2;
                        X.pxy = X.px * (Po.n[1] + 2);
                    }
                    // x = lo_p + (q + 1/2) h_p  =>  q_o = (x - lo_o) / h_o - 1/2 = r q + t
                    const double r = Pp.h[0] / Po.h[0];
                    X.r = (float)r;
                    for (int a = 0; a < 3; a++) X.t[a] = (float)((Pp.lo[a] - Po.lo[a]) * Po.inv_h[a] + 0.5 * r - 0.5);
                    X.rope = 0;
                } else {
                    X.rope = o <= -2 ? -2 - o : (o == -1 ? -1 : 0);
                }
            }
        }
        // scene
        memset(out, 0, sizeof(*out));
        out->pool = (const float *)d_pool;
        out->nodes = (const uint8_t *)d_meta + o_nodes;
        out->leaves = (const uint8_t *)d_meta + o_leaves;
        out->patches = (const uint8_t *)d_meta + o_patch;
        out->leaf_faces = (const uint8_t *)d_meta + o_faces;
        out->face_taps = (const uint8_t *)d_meta + o_fxf;
        out->pool_bytes = pbytes;
        out->meta_bytes = mbytes;
        out->nnodes = (int32_t)nn;
        out->nleaves = (int32_t)nl0;
        out->nlod = (int32_t)na;
        out->npatches = np;
        out->nlevels = T->dom.nlevels;
        out->lmax = T->lmax;
        out->refine = T->dom.refine;
        out->depth = (int32_t)T->depth;
        out->brick_layout = layout;
        out->centering = vertex;
        double hmin = std::min(T->dom.h0[0], std::min(T->dom.h0[1], T->dom.h0[2]));
        double rl = 1.0;
        for (int k = 0; k < T->lmax; k++) rl *= (double)T->dom.refine;
        out->step_fine = hmin / rl;
        for (int a = 0; a < 3; a++) {
            out->box_lo[a] = world_plane(T, a, T->B_lo[a]);
            out->box_hi[a] = world_plane(T, a, T->B_hi[a]);
            out->origin[a] = T->dom.origin[a];
            out->h0[a] = T->dom.h0[a];
            out->hfine[a] = T->dom.h0[a] / (double)T->scale[0];
        }
        out->v_min = vmin;
        out->v_max = vmax;
    } catch (const std::bad_alloc &) {
        set_error("out of host memory");
        return AMR_ENOMEM;
    }
    if (host_dst) {
        memcpy(d_pool, pool.data(), pool.size() * 4);
        memcpy(d_meta, meta.data(), meta.size());
        return AMR_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_pool, pool.data(), pool.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_meta, meta.data(), meta.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error("HIP copy failed: %s", hipGetErrorString(e)); return AMR_EHIP; }
    return AMR_OK;
}

}  // extern "C"
