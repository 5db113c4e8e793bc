"""Out-of-core residency on the host (amr_store_*, host_dst = 1, no GPU): the cache holds exactly
the resident bricks at non-overlapping aligned slots, the metadata draws each leaf of an absent
patch from its brute-force finest resident holder (level, value range, faces), updates upload
only new bricks, and capacity errors leave the store usable."""
import numpy as np
import pytest

import paper_1212_3333_amd as amr
from paper_1212_3333_amd import _lib as L
import oracle
import workloads


def _hier(name):
    if name == "lod":
        return workloads.lod_blocks(1)
    if name == "lodv":
        return workloads.lod_blocks(2).with_vertex_field(workloads.gaussian_sum_field(np.random.default_rng(3)))
    if name == "tiny":
        return workloads.tiny_samr(2)
    return workloads.random_tiny(int(name[4]), multi_root=name.endswith("m"), max_patches=8)


def _mask(h, seed, keep=0.5, root=True):
    rng = np.random.default_rng(seed)
    m = rng.random(len(h.patches)) < keep
    if root:
        m |= np.array([p.level == 0 for p in h.patches])
    return m


def _holder(boxes, mask, lo, hi):
    best = -1
    for q in range(len(boxes)):
        if mask[q] and np.all(boxes[q, 1:4] <= lo) and np.all(hi <= boxes[q, 4:7]):
            if best < 0 or boxes[q, 0] > boxes[best, 0]:
                best = q
    return best


def _records(sc):
    """Leaf records incl. the kind-(a) ones after the leaves."""
    dt = np.dtype([("lo", np.float64, 3), ("hi", np.float64, 3), ("patch", np.int32),
                   ("level_flags", np.uint32), ("vmin", np.float32), ("vmax", np.float32)])
    return sc._records(sc.scene.leaves, dt, sc.scene.nleaves + sc.scene.nlod)


def _faces(sc):
    n = sc.scene.nleaves + sc.scene.nlod
    own = sc._records(sc.scene.leaf_faces, np.dtype(np.int32), 6 * n).reshape(n, 6)
    dt = np.dtype([("off", np.uint64), ("n", np.int32, 3), ("px", np.int32), ("pxy", np.int32),
                   ("r", np.float32), ("t", np.float32, 3), ("rope", np.int32), ("pad", np.int32, 4)])
    return own, sc._records(sc.scene.face_taps, dt, 6 * n).reshape(n, 6)


def _record_boxes(tree, h):
    """Integer boxes of the leaves (pre-order) then the kind-(a) nodes (pre-order)."""
    nodes, leaves = tree.export()
    boxes = [np.concatenate([l["lo"], l["hi"]]) for l in leaves]
    fb = oracle.finest_boxes(h)
    root = fb[fb[:, 0] == 0]
    box = np.concatenate([root[:, 1:4].min(0), root[:, 4:7].max(0)])
    pending, abox = [], []
    for n in nodes:
        if n["kind"] == 0:
            abox.append(box.copy())
        if n["axis"] >= 0:
            lo_b, hi_b = box.copy(), box.copy()
            lo_b[3 + n["axis"]] = n["split"]
            hi_b[n["axis"]] = n["split"]
            pending.append(hi_b)
            box = lo_b
        elif pending:
            box = pending.pop()
    return np.array(boxes + abox, dtype=np.int64).reshape(-1, 6)


def _brick_range(full, h, p, lo, hi, vertex):
    b = full.brick(p).astype(np.float32)
    s = h.refine ** (h.lmax - h.patches[p].level)
    plo = np.asarray(h.patches[p].lo) * s
    i0 = (lo - plo) // s
    i1 = -((-(hi - plo)) // s)
    f = 0 if vertex else 1
    sub = b[i0[2] - f + 1:i1[2] + 2, i0[1] - f + 1:i1[1] + 2, i0[0] - f + 1:i1[0] + 2]
    return sub.min(), sub.max()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("name", ["tiny", "lod", "lodv", "rand0", "rand1m", "rand2", "rand3m"])
def test_remap_matches_brute_force(name, layout):
    h = _hier(name)
    vertex = getattr(h, "centering", "cell") == "vertex"
    tree = amr.build_tree(h)
    full = amr.pack(tree, h, host=True, brick_layout=layout)
    st = amr.Store(tree, h, host=True, brick_layout=layout)
    info = st.info()
    cache, meta = st.alloc(info["full_cache_bytes"])
    fb = oracle.finest_boxes(h)
    rb = _record_boxes(tree, h)
    fr, (fown, ffx) = _records(full), _faces(full)
    nl = full.scene.nleaves
    for seed in range(4):
        mask = _mask(h, seed, keep=0.4, root=seed != 3)
        sc, rep = st.update(mask, cache, meta)
        rr, (own, fx) = _records(sc), _faces(sc)
        ph = sc.patch_headers()
        bb = st.brick_bytes()
        remapped = 0
        for k in range(len(rr)):
            p0 = int(fr["patch"][k])
            if p0 < 0:
                assert rr["patch"][k] == -1
                continue
            want = _holder(fb, mask, rb[k, :3], rb[k, 3:])
            assert rr["patch"][k] == want, (seed, k)
            if want == p0:
                assert rr["level_flags"][k] == fr["level_flags"][k]
                assert rr["vmin"][k] == fr["vmin"][k] and rr["vmax"][k] == fr["vmax"][k]
                for f in range(6):
                    o = int(fown[k, f])
                    if o >= 0 and not mask[o]:
                        assert own[k, f] == -2 and fx[k, f]["n"][0] == 0 and fx[k, f]["rope"] == 0
                    else:
                        assert own[k, f] == o
                continue
            remapped += 1
            assert np.all(own[k] == -2) and np.all(fx[k]["n"][:, 0] == 0) and np.all(fx[k]["rope"] == 0)
            if want >= 0:
                assert rr["level_flags"][k] == h.patches[want].level
                lo_v, hi_v = _brick_range(full, h, want, rb[k, :3], rb[k, 3:], vertex)
                assert rr["vmin"][k] == lo_v and rr["vmax"][k] == hi_v
            elif k >= nl:
                # a level-of-detail node with no holder is never a stop
                nodes = sc.node_records()
                assert not np.any((nodes["meta"] >> 8) == (k - nl + 1))
        assert rep["remapped_leaves"] == remapped
        # single-owner face records carry the owner's cache slot (a resident brick)
        single = own >= 0
        assert np.all(mask[own[single]])
        assert np.array_equal(fx["off"][single], ph["off"][own[single]])
        # the cache holds each resident brick at its slot; slots are aligned and disjoint
        pool = cache.view(np.float32)
        spans = []
        for p in range(len(h.patches)):
            if not mask[p]:
                continue
            off = int(ph["off"][p])
            assert off % 64 == 0 and off >= 64 and off * 4 + bb[p] <= len(cache) - 256
            spans.append((off, off + bb[p] // 4))
            src = full.pool.view(np.float32)[int(full.patch_headers()["off"][p]):][: bb[p] // 4]
            assert np.array_equal(pool[off:off + bb[p] // 4], src)
        spans.sort()
        assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))


def test_incremental_updates_and_capacity():
    h = workloads.random_tiny(5, max_patches=8)
    tree = amr.build_tree(h)
    st = amr.Store(tree, h, host=True)
    bb = st.brick_bytes()
    info = st.info()
    assert info["full_cache_bytes"] == bb.sum() + info["pad_bytes"]
    cache, meta = st.alloc(info["full_cache_bytes"])
    m0 = _mask(h, 0, keep=0.3)
    sc, rep = st.update(m0, cache, meta)
    assert rep["repacked"] == 1 and rep["uploaded_bricks"] == m0.sum() and rep["evicted_bricks"] == 0
    off0 = sc.patch_headers()["off"].copy()
    m1 = m0.copy()
    more = np.flatnonzero(~m0)[:2]
    assert len(more) > 0
    m1[more] = True
    sc, rep = st.update(m1, cache, meta)
    assert rep["repacked"] == 0 and rep["uploaded_bricks"] == len(more)
    assert rep["uploaded_bytes"] == bb[m1 & ~m0].sum()
    assert np.array_equal(sc.patch_headers()["off"][m0], off0[m0])      # bricks stay put
    m2 = m1.copy()
    drop = np.flatnonzero(m1 & np.array([p.level > 0 for p in h.patches]))[:1]
    m2[drop] = False
    sc, rep = st.update(m2, cache, meta)
    assert rep["evicted_bricks"] == len(drop) and rep["uploaded_bricks"] == 0
    assert rep["resident_bricks"] == m2.sum() and rep["resident_bytes"] == bb[m2].sum()
    # too small a cache: AMR_ECAPACITY, and the store still serves the old cache afterwards
    small = amr.Store.host_buffer(int(bb[m2].sum()))
    with pytest.raises(amr.AMRError, match="ECAPACITY"):
        st.update(m2, small, meta)
    sc, rep = st.update(m2, cache, meta)
    assert rep["uploaded_bricks"] == 0 and rep["repacked"] == 0
    # a fragmented cache is laid out again
    tight = amr.Store.host_buffer(int(bb.max() * 2 + info["pad_bytes"] + 4096))
    order = np.argsort(-bb)
    a = np.zeros(len(bb), bool); a[order[1]] = True
    st.update(a, tight, meta)
    b = np.zeros(len(bb), bool); b[order[0]] = True
    sc, rep = st.update(b, tight, meta)
    assert rep["resident_bricks"] == 1


def test_select_respects_budget_and_levels():
    """The selection fits the budget, always starts with the level-0 patches, leaves out
    refinements whose bounding sphere misses the view volume, and with room for everything
    takes every patch in view."""
    h, lut, cam, prm = workloads.cosmology_view(0, 256, 256)
    tree = amr.build_tree(h)
    st = amr.Store(tree, h, host=True)
    bb = st.brick_bytes()
    lev = np.array([p.level for p in h.patches])
    info = st.info()
    full = st.select(cam, info["full_cache_bytes"])
    assert np.all(full[lev == 0]) and 0 < full.sum() <= len(bb)
    for frac in (0.15, 0.4):
        budget = int(info["full_cache_bytes"] * frac)
        m = st.select(cam, budget)
        assert bb[m].sum() <= budget - info["pad_bytes"]
        assert np.all(m[lev == 0])
        assert not np.any(m & ~full)          # nothing out of view
        assert m.sum() < full.sum()
        # the finest level reached is not started before a coarser visible level fits
        top = lev[m].max()
        left = budget - info["pad_bytes"] - bb[m].sum()
        assert np.all(bb[full & ~m & (lev < top)] > left)


def test_store_arguments():
    h = workloads.tiny_samr(0)
    tree = amr.build_tree(h)
    st = amr.Store(tree, h, host=True)
    cache, meta = st.alloc(st.info()["full_cache_bytes"])
    with pytest.raises(ValueError):
        st.update(np.ones(3, bool), cache, meta)
    with pytest.raises(amr.AMRError, match="ECAPACITY"):
        st.update(np.ones(len(h.patches), bool), cache, meta[:16])


@pytest.mark.parametrize("layout", [0, 1])
def test_random_update_sequence_keeps_the_cache_consistent(layout):
    """Thirty random resident sets through a cache of 60% of all bricks (holes and compaction):
    after each update every resident brick sits intact at its slot, slots are disjoint, kept
    bricks move only when the cache was compacted, and the report counts what happened."""
    h = workloads.cosmology_like(1, root=32, nlevels=4, target_patches=60, sides=(8, 16, 32), side_probs=(0.4, 0.4, 0.2))
    tree = amr.build_tree(h)
    full = amr.pack(tree, h, host=True, brick_layout=layout)
    st = amr.Store(tree, h, host=True, brick_layout=layout)
    bb = st.brick_bytes()
    info = st.info()
    cap = int(0.6 * info["full_cache_bytes"]) // 256 * 256
    cache, meta = st.alloc(cap)
    src = full.pool.view(np.float32)
    foff = full.patch_headers()["off"].astype(np.int64)
    rng = np.random.default_rng(layout)
    prev_mask, prev_off = np.zeros(len(bb), bool), None
    compactions = 0
    for it in range(30):
        # keep part of the previous set, then fill up to the cache size in random order
        mask = prev_mask & (rng.random(len(bb)) < 0.7)
        for p in rng.permutation(len(bb)):
            if not mask[p] and bb[mask].sum() + bb[p] <= cap - info["pad_bytes"]:
                mask[p] = True
        sc, rep = st.update(mask, cache, meta)
        off = sc.patch_headers()["off"].astype(np.int64)
        pool = cache.view(np.float32)
        spans = sorted((off[p], off[p] + bb[p] // 4) for p in np.flatnonzero(mask))
        assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
        assert all(a[0] >= 64 and a[1] <= cap // 4 - 64 for a in spans)
        for p in np.flatnonzero(mask):
            assert np.array_equal(pool[off[p]:off[p] + bb[p] // 4], src[foff[p]:foff[p] + bb[p] // 4]), (it, p)
        kept = mask & prev_mask
        moved = kept & (off != prev_off) if prev_off is not None else np.zeros_like(kept)
        if moved.any():
            assert rep["repacked"] == 1
        compactions += rep["repacked"] and it > 0
        new = mask & ~prev_mask
        assert rep["uploaded_bricks"] == new.sum() + moved.sum()
        assert rep["evicted_bricks"] == (prev_mask & ~mask).sum()
        prev_mask, prev_off = mask, off
    assert compactions > 0
