"""Host side of libamr on the CPU: exported symbols, validation errors, the kD builder against the
oracle's naive builder (node by node), the pool's ghost layers against the oracle's FP64 ghosts
(bit-exact after fp32 rounding) and the device tree encoding.  No GPU is used: the pool is
packed into host memory (amr_pack_opts.host_dst)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1212_3333_amd as amr
from paper_1212_3333_amd import _lib as L
import workloads
from oracle import Oracle, finest_boxes, kdbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    src = open(os.path.join(ROOT, "include", "amr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(amr_[a-z0-9_]+)\s*\(", src))
    assert len(names) >= 15
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    assert names == set(L.SIGNATURES), "binding signatures out of sync with include/amr.h"


def _compare_trees(h):
    tree = amr.build_tree(h)
    nodes, leaves = tree.export()
    ref = kdbuild.build(finest_boxes(h), h.nlevels)
    na = ref.node_array()
    assert len(nodes) == len(na)
    assert np.array_equal(nodes["axis"], na[:, 0])
    assert np.array_equal(nodes["split"], np.where(na[:, 0] >= 0, na[:, 1], 0))
    assert np.array_equal(nodes["level"], na[:, 2])
    assert np.array_equal(nodes["patch"], na[:, 3])
    assert np.array_equal(nodes["cover"], na[:, 4])
    assert np.array_equal(nodes["kind"], ref.kinds())
    la = ref.leaf_array()
    assert np.array_equal(leaves["lo"], la[:, 0:3]) and np.array_equal(leaves["hi"], la[:, 3:6])
    assert np.array_equal(leaves["patch"], la[:, 6]) and np.array_equal(leaves["level"], la[:, 7])
    info = tree.info()
    assert info["nodes"] == len(na) and info["leaves"] == len(la)
    assert info["n_a"] + info["n_b"] + info["n_c"] == info["nodes"]
    return tree


def test_builder_equals_naive_small_nested():
    _compare_trees(workloads.tiny_samr(0))


@pytest.mark.parametrize("seed", range(100))
def test_builder_equals_naive_random(seed):
    _compare_trees(workloads.random_tiny(seed, multi_root=(seed % 3 == 0)))


def test_builder_shuffle_invariance():
    h = workloads.tiny_samr(2)
    perm = np.random.default_rng(1).permutation(len(h.patches))
    hs = workloads.Hierarchy(h.origin, h.h0, h.refine, h.nlevels, [h.patches[i] for i in perm])
    n1, _ = amr.build_tree(h).export()
    n2, _ = amr.build_tree(hs).export()
    assert np.array_equal(n1["axis"], n2["axis"]) and np.array_equal(n1["split"], n2["split"])
    p2 = np.where(n2["patch"] >= 0, perm[np.maximum(n2["patch"], 0)], -1)
    assert np.array_equal(n1["patch"], p2)


def _compare_ghosts(h):
    tree = amr.build_tree(h)
    O = Oracle(h)
    for layout in (0, 1, 2):
        scene = amr.pack(tree, h, host=True, nthreads=3, brick_layout=layout)
        for p in range(len(h.patches)):
            got = scene.brick(p)
            ref = O.padded_brick(p).astype(np.float32)
            assert np.array_equal(got, ref), (layout, p)
    return scene


def test_ghosts_bit_exact_small_nested():
    _compare_ghosts(workloads.tiny_samr(0))


@pytest.mark.parametrize("seed", range(12))
def test_ghosts_bit_exact_random(seed):
    _compare_ghosts(workloads.random_tiny(seed, multi_root=(seed % 2 == 0)))


def test_ghosts_bit_exact_nonnested():
    p0 = workloads._empty_patch(0, [0, 0, 0], [4, 8, 8])
    p1 = workloads._empty_patch(0, [4, 0, 0], [4, 4, 8])
    p2 = workloads._empty_patch(1, [6, 6, 4], [6, 6, 4])       # spans p0, p1 and the hole
    p3 = workloads._empty_patch(1, [12, 10, 0], [3, 4, 4])     # inside the hole
    h = workloads.Hierarchy(np.zeros(3), np.full(3, 1.0 / 8), 2, 2, [p0, p1, p2, p3])
    h = h.with_field(lambda X, Y, Z: np.sin(9 * X) * Y + Z * Z)
    _compare_ghosts(h)


def test_device_encoding():
    h = workloads.random_tiny(5, multi_root=True)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    nodes, leaves = tree.export()
    dn = scene.node_records()
    assert len(dn) == len(nodes)
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    # breadth-first: children adjacent and after their parent; every node reached once
    seen = np.zeros(len(dn), dtype=int)
    seen[0] = 1
    leaf_ids = []
    for i, n in enumerate(dn):
        axis = n["meta"] & 3
        if axis == 3:
            leaf_ids.append(int(n["child"]))
        else:
            c = int(n["child"])
            assert c > i and c + 1 < len(dn)
            seen[c] += 1
            seen[c + 1] += 1
    assert np.all(seen == 1)
    assert sorted(leaf_ids) == list(range(len(leaves)))
    # split planes: world coordinate of an integer finest-grid plane (product, then sum)
    splits = sorted(set((int(n["axis"]), int(n["split"])) for n in nodes if n["axis"] >= 0))
    dsplits = sorted(set((int(n["meta"] & 3), float(n["split"])) for n in dn if (n["meta"] & 3) != 3))
    expect = sorted(set((a, float(h.origin[a] + np.float64(G) * hf[a])) for a, G in splits))
    assert dsplits == expect
    lr = scene.leaf_records()
    for k, lf in enumerate(leaves):
        assert np.array_equal(lr[k]["lo"], h.origin + lf["lo"] * hf)
        assert lr[k]["patch"] == lf["patch"] and (lr[k]["level_flags"] & 0xFF) == lf["level"]
    hdr = scene.patch_headers()
    for p, ph in enumerate(h.patches):
        assert np.array_equal(hdr[p]["n"], ph.dims)
        assert hdr[p]["off"] % 64 == 0
        assert np.allclose(hdr[p]["h"], h.h0 / h.refine ** ph.level, rtol=0, atol=0)


def _h_from_boxes(boxes, nlevels=2, refine=2, root=8):
    ps = [workloads._empty_patch(l, lo, d) for (l, lo, d) in boxes]
    return workloads.Hierarchy(np.zeros(3), np.full(3, 1.0 / root), refine, nlevels, ps)


@pytest.mark.parametrize("boxes,code", [
    ([(0, [0, 0, 0], [8, 8, 8]), (1, [0, 0, 0], [4, 4, 4]), (1, [2, 2, 2], [4, 4, 4])], L.AMR_EHIERARCHY),  # overlap
    ([(0, [0, 0, 0], [8, 8, 8]), (1, [14, 0, 0], [4, 4, 4])], L.AMR_EHIERARCHY),                          # outside B
    ([(0, [0, 0, 0], [8, 8, 8]), (1, [0, 0, 0], [0, 4, 4])], L.AMR_EHIERARCHY),                           # empty
    ([(1, [0, 0, 0], [4, 4, 4])], L.AMR_EHIERARCHY),                                                      # no root
    ([(0, [0, 0, 0], [8, 8, 8]), (2, [0, 0, 0], [4, 4, 4])], L.AMR_EHIERARCHY),                           # level range
    ([(0, [0, 0, 0], [4, 8, 8]), (0, [3, 0, 0], [4, 8, 8])], L.AMR_EHIERARCHY),                           # root overlap
])
def test_validation_errors(boxes, code):
    h = _h_from_boxes(boxes)
    with pytest.raises(amr.AMRError) as e:
        amr.build_tree(h)
    assert L.ERRNAMES[code] in str(e.value)


def test_domain_errors():
    lib = L.load()
    h = _h_from_boxes([(0, [0, 0, 0], [8, 8, 8])])
    arr, keep = amr._patch_array(h)
    dom = amr._domain(h)
    out = ctypes.c_void_p()
    dom.refine = 1
    assert lib.amr_build_kdtree(ctypes.byref(dom), arr, 1, ctypes.byref(out)) == L.AMR_EINVAL
    dom.refine = 2
    dom.h0[1] = 0.0
    assert lib.amr_build_kdtree(ctypes.byref(dom), arr, 1, ctypes.byref(out)) == L.AMR_EINVAL
    dom.h0[1] = 0.125
    assert lib.amr_build_kdtree(ctypes.byref(dom), arr, 0, ctypes.byref(out)) == L.AMR_EINVAL
    assert lib.amr_build_kdtree(ctypes.byref(dom), arr, 1, None) == L.AMR_EINVAL
    assert b"null" in lib.amr_last_error() or len(lib.amr_last_error()) > 0


def test_pack_capacity_and_size_query():
    lib = L.load()
    h = workloads.tiny_samr(0)
    tree = amr.build_tree(h)
    pb, mb = ctypes.c_int64(0), ctypes.c_int64(0)
    opts = L.amr_pack_opts()
    opts.host_dst = 1
    assert lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts), None, ctypes.byref(pb),
                             None, ctypes.byref(mb), None, None) == 0
    # padded bricks rounded to 64 floats, plus 64 spare floats before the first and after the last
    expect_pool = sum(((int(p.dims[0]) + 2) * (int(p.dims[1]) + 2) * (int(p.dims[2]) + 2) + 63) // 64 * 64 * 4
                      for p in h.patches) + 2 * 64 * 4
    opts.brick_layout = 0
    assert pb.value == expect_pool
    pool = np.zeros(pb.value - 4, dtype=np.uint8)
    meta = np.zeros(mb.value, dtype=np.uint8)
    small = ctypes.c_int64(pb.value - 4)
    sc = L.amr_scene()
    assert lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts), pool.ctypes.data,
                             ctypes.byref(small), meta.ctypes.data, ctypes.byref(mb), ctypes.byref(sc),
                             None) == L.AMR_ECAPACITY
    assert lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches) - 1, ctypes.byref(opts), pool.ctypes.data,
                             ctypes.byref(small), meta.ctypes.data, ctypes.byref(mb), ctypes.byref(sc),
                             None) == L.AMR_EINVAL


def test_tree_export_capacity():
    lib = L.load()
    tree = amr.build_tree(workloads.tiny_samr(0))
    inf = tree.info()
    nodes = (L.amr_node_host * (inf["nodes"] - 1))()
    assert lib.amr_tree_export(tree.ptr, nodes, inf["nodes"] - 1, None, 0) == L.AMR_ECAPACITY


def test_leaf_value_range():
    h = workloads.tiny_samr(1)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    _, leaves = tree.export()
    lr = scene.leaf_records()
    s = h.refine ** (h.nlevels - 1)
    for k, lf in enumerate(leaves):
        p = int(lf["patch"])
        b = scene.brick(p)
        sc = h.refine ** (h.lmax - int(lf["level"]))
        lo = (lf["lo"] - h.patches[p].lo * sc) // sc
        hi = -((-(lf["hi"] - h.patches[p].lo * sc)) // sc)
        sub = b[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2]
        assert lr[k]["vmin"] == sub.min() and lr[k]["vmax"] == sub.max()
    assert s > 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_leaf_face_owners(seed):
    """Where the table names an owner, every point of the one-cell slab beyond the face lies in
    that patch's data (checked with the oracle's point location); the safe bits mark the faces
    owned by the leaf's own patch."""
    h = workloads.random_tiny(seed, multi_root=(seed == 1)) if seed < 2 else workloads.tiny_samr(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    _, leaves = tree.export()
    own = scene.leaf_face_owners()
    flags = scene.leaf_records()["level_flags"]
    O = Oracle(h)
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    rng = np.random.default_rng(seed)
    named = 0
    ropes = []
    for k, lf in enumerate(leaves):
        if lf["patch"] < 0:
            assert np.all(own[k] == -1)
            continue
        S = h.refine ** (h.lmax - int(lf["level"]))
        for f in range(6):
            a, side = f // 2, f % 2
            assert bool((flags[k] >> (8 + f)) & 1) == (own[k, f] == lf["patch"])
            if own[k, f] <= -2:
                ropes.append((k, f, -2 - own[k, f]))
            if own[k, f] < 0:
                continue
            named += 1
            lo, hi = lf["lo"].astype(np.float64), lf["hi"].astype(np.float64)
            if side:
                lo[a], hi[a] = hi[a], hi[a] + S
            else:
                lo[a], hi[a] = lo[a] - S, lo[a]
            for _ in range(4):
                x = h.origin + (lo + rng.random(3) * (hi - lo)) * hf
                assert O.locate(x) == own[k, f]
    assert named > 0
    # ropes: descending from the stored node reaches the same leaf as descending from the root
    dn = scene.node_records()

    def descend(x, start):
        ni = start
        while (dn[ni]["meta"] & 3) != 3:
            ax = dn[ni]["meta"] & 3
            ni = dn[ni]["child"] + (0 if x[ax] < dn[ni]["split"] else 1)
        return dn[ni]["child"]
    for k, f, node in ropes:
        a, side = f // 2, f % 2
        S = h.refine ** (h.lmax - int(leaves[k]["level"]))
        lo, hi = leaves[k]["lo"].astype(np.float64), leaves[k]["hi"].astype(np.float64)
        if side:
            lo[a], hi[a] = hi[a], hi[a] + S
        else:
            lo[a], hi[a] = lo[a] - S, lo[a]
        for _ in range(4):
            x = h.origin + (lo + rng.random(3) * (hi - lo)) * hf
            assert descend(x, node) == descend(x, 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_face_tap_records(seed):
    """Each single-owner face record maps a point of the slab from the leaf's patch-local cell
    coordinates into the owner's (q_o = r q + t) as the FP64 world-coordinate formula does, and
    names the owner's brick; the other faces carry the rope node of the face table."""
    h = workloads.random_tiny(seed, multi_root=(seed == 1)) if seed < 2 else workloads.tiny_samr(0)
    tree = amr.build_tree(h)
    for layout in (0, 1, 2):
        scene = amr.pack(tree, h, host=True, brick_layout=layout)
        own = scene.leaf_face_owners()
        rec = scene.face_tap_records()
        ph = scene.patch_headers()
        lr = scene.leaf_records()
        rng = np.random.default_rng(seed)
        mapped = 0
        for k in range(len(lr)):
            p = int(lr["patch"][k])
            for f in range(6):
                X, o = rec[k, f], int(own[k, f])
                if p < 0 or o < 0:
                    assert X["n"][0] == 0
                    assert X["rope"] == (-2 - o if o <= -2 else (-1 if o == -1 else 0))
                    continue
                mapped += 1
                assert X["off"] == ph["off"][o] and np.array_equal(X["n"], ph["n"][o])
                if layout in (1, 2):
                    w = 64 if layout == 1 else 128
                    assert X["px"] == w * ph["nb"][o][0] and X["pxy"] == X["px"] * ph["nb"][o][1]
                else:
                    assert X["px"] == ph["n"][o][0] + 2 and X["pxy"] == X["px"] * (ph["n"][o][1] + 2)
                a, side = f // 2, f % 2
                lo, hi = lr["lo"][k].copy(), lr["hi"][k].copy()
                hl = ph["h"][p]
                if side:
                    lo[a], hi[a] = hi[a], hi[a] + hl[a]
                else:
                    lo[a], hi[a] = lo[a] - hl[a], lo[a]
                for _ in range(4):
                    x = lo + rng.random(3) * (hi - lo)
                    q = (x - ph["lo"][p]) * ph["inv_h"][p] - 0.5
                    qo = (x - ph["lo"][o]) * ph["inv_h"][o] - 0.5
                    got = q * np.float64(X["r"]) + X["t"].astype(np.float64)
                    assert np.allclose(got, qo, rtol=0, atol=1e-9 * (1 + np.abs(qo).max()))
        assert mapped > 0



def _vertex_h(name):
    fn = workloads.gaussian_sum_field(np.random.default_rng(17), n=4, smin=0.08, smax=0.25)
    if name == "tiny":
        h = workloads.tiny_samr(2)
    elif name == "lod":
        h = workloads.lod_blocks(0)
    elif name.startswith("aligned"):
        h = workloads.random_tiny(int(name[-1]), root_aligned=True)
    else:
        h = workloads.random_tiny(int(name[4]), multi_root=name.endswith("m"))
    return h.with_vertex_field(fn)


@pytest.mark.parametrize("name", ["tiny", "lod", "aligned0", "aligned5", "rand1", "rand2m", "rand3", "rand4m"])
def test_vertex_bricks_match_oracle(name):
    """Vertex-centred pack: each brick holds the oracle's samples after the dangling-node fix
    (FP64 on both sides, then fp32) with a shell replicating the nearest sample; the header
    presents the n+1 samples to the kernels as cells whose centres are the vertices (lower
    corner half a cell down), and the leaf value range covers the vertices of the leaf's cells."""
    h = _vertex_h(name)
    tree = amr.build_tree(h)
    O = Oracle(h)
    for layout in (0, 1, 2):
        scene = amr.pack(tree, h, host=True, nthreads=3, brick_layout=layout)
        assert scene.scene.centering == 1
        ph = scene.patch_headers()
        for p, pt in enumerate(h.patches):
            ref = O.vertex_values(p).astype(np.float32)
            got = scene.brick(p)
            assert got.shape == tuple(int(d) + 3 for d in pt.dims[::-1])
            assert np.array_equal(got[1:-1, 1:-1, 1:-1], ref), (layout, p)
            assert np.array_equal(got, np.pad(ref, 1, mode="edge")), (layout, p)
            hl = h.h0 / float(h.refine) ** pt.level
            assert np.array_equal(ph["n"][p], pt.dims + 1)
            assert np.allclose(ph["lo"][p], h.origin + pt.lo * hl - 0.5 * hl, rtol=0, atol=1e-15)
    _, leaves = tree.export()
    lr = scene.leaf_records()
    for k, lf in enumerate(leaves):
        p = int(lf["patch"])
        if p < 0:
            continue
        sc = h.refine ** (h.lmax - int(lf["level"]))
        lo = (lf["lo"] - h.patches[p].lo * sc) // sc
        hi = -((-(lf["hi"] - h.patches[p].lo * sc)) // sc)
        sub = O.vertex_values(p)[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1].astype(np.float32)
        assert lr[k]["vmin"] == sub.min() and lr[k]["vmax"] == sub.max()


def test_vertex_sample_shape_checked():
    h = workloads.tiny_samr(0)
    bad = workloads.Hierarchy(h.origin, h.h0, h.refine, h.nlevels, h.patches, "vertex")
    tree = amr.build_tree(bad)
    with pytest.raises(ValueError):
        amr.pack(tree, bad, host=True)
    opts = L.amr_pack_opts()
    opts.host_dst = 1
    opts.centering = 2
    pb, mb = ctypes.c_int64(0), ctypes.c_int64(0)
    lib = amr.load()
    assert lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts), None, ctypes.byref(pb),
                             None, ctypes.byref(mb), None, None) == L.AMR_EINVAL


@pytest.mark.parametrize("name", ["tiny", "vertex"])
def test_halo_rows_layout(name):
    """Halo-row layout: row (j, k) of block column bx holds padded x indices 4 bx - 1 .. 4 bx + 6
    of the padded brick (zero beyond it), so every row also carries its neighbours' edge cells."""
    h = workloads.tiny_samr(1)
    if name == "vertex":
        h = h.with_vertex_field(workloads.gaussian_sum_field(np.random.default_rng(2)))
    tree = amr.build_tree(h)
    lin = amr.pack(tree, h, host=True, brick_layout=0)
    halo = amr.pack(tree, h, host=True, brick_layout=2)
    for p in range(len(h.patches)):
        ref = lin.brick(p)
        assert np.array_equal(halo.brick(p), ref)
        rows = halo.halo_rows(p)
        nbz, nby, nbx = rows.shape[:3]
        P = ref.shape
        padded = np.zeros((4 * nbz, 4 * nby, 4 * nbx + 8), np.float32)
        padded[:P[0], :P[1], 1:P[2] + 1] = ref          # x shifted by one: index -1 -> column 0
        for bx in range(nbx):
            want = padded[:, :, 4 * bx:4 * bx + 8].reshape(nbz, 4, nby, 4, 8).transpose(0, 2, 1, 3, 4)
            assert np.array_equal(rows[:, :, bx], want), (p, bx)


def test_persistent_mode_argument_checks():
    """amr_render rejects, before touching any device memory, the requests the persistent kernel
    does not serve: learned proposals, nearest-cell sampling and the point light.  Host buffers
    stand in for the device pointers, so the test runs only where no GPU is visible."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("host buffers stand in for device pointers: CPU only")
    h, lut, cams, prm = workloads.small_nested(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    lib = amr.load()
    two = [cams[0], cams[1]]
    carr = (L.amr_camera * 2)(*[amr.make_camera(c) for c in two])
    lutbuf = np.zeros((256, 4), np.float32)
    rgba = np.zeros(4 * sum(c["width"] * c["height"] for c in two), np.float32)
    scratch = np.zeros(4096, np.uint8)
    for extra, words in [(dict(), "learned proposals"), (dict(interp=1), "nearest-cell"),
                         (dict(lighting=2), "point-light")]:
        q = amr.make_params(dict(prm, persistent=1, **extra), lutbuf)
        q.d_queue = scratch.ctypes.data
        q.d_cams = ctypes.cast(carr, ctypes.c_void_p).value
        if not extra:
            q.d_mlp = scratch.ctypes.data
        rc = lib.amr_render(ctypes.byref(scene.scene), carr, 2, ctypes.byref(q), rgba.ctypes.data, None, None)
        assert rc == 1, extra
        msg = lib.amr_last_error().decode()
        assert words in msg and "persistent" in msg, msg


def _render_call(lib, scene, cams, prm, set_fields=None, lut_ok=True):
    """amr_render on host buffers standing in for device pointers (rejected calls only)."""
    carr = (L.amr_camera * len(cams))(*[amr.make_camera(c) for c in cams])
    lutbuf = np.zeros((256, 4), np.float32)
    # never written (every call here is rejected first), so capped for the huge-camera cases
    rgba = np.zeros(min(1 << 20, 4 * max(1, sum(max(0, c["width"]) * max(0, c["height"]) for c in cams))), np.float32)
    scratch = np.zeros(1 << 16, np.uint8)
    q = amr.make_params(prm, lutbuf)
    if not lut_ok:
        q.d_lut = None
    for k, v in (set_fields or {}).items():
        # "buf": a host buffer standing in for a device one; "buf+4": the same, 4-byte misaligned
        setattr(q, k, scratch.ctypes.data + (4 if v == "buf+4" else 0) if v in ("buf", "buf+4") else v)
    if q.persistent and not (set_fields and "d_cams" in set_fields):
        q.d_cams = ctypes.cast(carr, ctypes.c_void_p).value
    rc = lib.amr_render(ctypes.byref(scene.scene), carr, len(cams), ctypes.byref(q), rgba.ctypes.data, None, None)
    return rc, lib.amr_last_error().decode()


@pytest.mark.parametrize("case", ["v_range", "step", "cam_size", "interp", "lighting", "lod", "lut", "trace_cap",
                                  "ckpt_odd", "ckpt_small", "tile", "no_queue", "light_no_work", "light_work_small",
                                  "tape_cap", "tape_align", "waves_per_simd", "sched_small", "sched_persistent",
                                  "sched_huge", "sched_huge_lit"])
def test_render_argument_checks(case):
    """amr_render's argument checks, each of which returns before any device access (host buffers
    stand in for device pointers, so the test runs only where no GPU is visible)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("host buffers stand in for device pointers: CPU only")
    h, lut, cams, prm = workloads.small_nested(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    lib = amr.load()
    cam = cams[0]
    want_code, words = 1, None
    fields, p, cl, lut_ok = {}, dict(prm), [cam], True
    if case == "v_range":
        p, words = dict(prm, v_hi=prm["v_lo"]), "v_hi"
    elif case == "step":
        p, words = dict(prm, step_frac=0.0), "step_frac"
    elif case == "cam_size":
        cl, words = [dict(cam, width=0)], "camera size"
    elif case == "interp":
        p, words = dict(prm, interp=2), "interp"
    elif case == "lighting":
        p, words = dict(prm, lighting=3), "lighting"
    elif case == "lod":
        p, words = dict(prm, lod=-1.0), "lod"
    elif case == "lut":
        lut_ok, words = False, "d_lut"
    elif case == "trace_cap":
        fields, words = dict(d_trace="buf", trace_cap=0), "trace_cap"
    elif case == "ckpt_odd":
        fields, words = dict(d_ckpt="buf", ckpt_bytes=1 << 16, ckpt_every=2, ckpt_max=3), "ckpt_max"
    elif case == "ckpt_small":
        fields, words, want_code = dict(d_ckpt="buf", ckpt_bytes=64, ckpt_every=2, ckpt_max=4), "ckpt_bytes", 3
    elif case == "tile":
        p, fields, words = dict(prm, persistent=1, tile_w=16, tile_h=8), dict(d_queue="buf"), "tile_w * tile_h"
    elif case == "no_queue":
        p, words = dict(prm, persistent=1), "d_queue"
    elif case == "light_no_work":
        p, words = dict(prm, lighting=2), "workspace"
    elif case == "light_work_small":
        p, words, want_code = dict(prm, lighting=2), "workspace", 3
        fields = dict(d_work="buf", work_bytes=1 << 16, light_jobs=1 << 20)
    elif case == "sched_small":
        p, words, want_code = dict(prm), "sched_bytes", 3
        fields = dict(d_sched="buf", sched_bytes=64)
    elif case == "sched_persistent":
        p, words = dict(prm, persistent=1), "tile schedule"
        fields = dict(d_queue="buf", d_sched="buf", sched_bytes=1 << 16)
    elif case == "sched_huge":
        # 4096 x 4097 super-tiles of 32x32 pixels (unlit): past the 24 bits an order entry holds
        cl, words = [cam, dict(cam, width=4096 * 32, height=4096 * 32 + 1)], "2^24 super-tiles"
        fields = dict(d_sched="buf", sched_bytes=1 << 40)
    elif case == "sched_huge_lit":
        # lit super-tiles are 16x16 pixels: a camera of half that size is already past the limit
        p, words = dict(prm, lighting=1), "2^24 super-tiles"
        cl = [cam, dict(cam, width=4096 * 16, height=4096 * 16 + 1)]
        fields = dict(d_sched="buf", sched_bytes=1 << 40)
    elif case == "waves_per_simd":
        p, fields, words = dict(prm, persistent=1, lighting=1, waves_per_simd=4), dict(d_queue="buf"), "waves_per_simd"
    elif case == "tape_cap":
        p, words = dict(prm, lighting=1), "tape_cap"
        fields = dict(d_ckpt="buf", ckpt_bytes=1 << 40, ckpt_every=2, ckpt_max=4, d_tape="buf", tape_cap=1 << 26)
    elif case == "tape_align":
        p, words = dict(prm, lighting=1), "16-byte"
        fields = dict(d_ckpt="buf", ckpt_bytes=1 << 40, ckpt_every=2, ckpt_max=4, d_tape="buf+4", tape_cap=8)
    rc, msg = _render_call(lib, scene, cl, p, fields, lut_ok)
    assert rc == want_code, (case, rc, msg)
    assert words in msg, (case, msg)


@pytest.mark.parametrize("case", ["no_ckpt", "nearest", "point_light", "ckpt_small", "no_work", "work_small",
                                  "work_small_det"])
def test_backward_argument_checks(case):
    """amr_render_backward's checks that precede any launch: a caller workspace of
    amr_backward_work_bytes(deterministic) bytes, checkpoints required, trilinear sampling and
    gradient lighting only, a checkpoint buffer of the forward's size (host buffers stand in
    for device pointers: CPU only)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("host buffers stand in for device pointers: CPU only")
    h, lut, cams, prm = workloads.small_nested(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, host=True)
    lib = amr.load()
    cam = cams[0]
    npix = cam["width"] * cam["height"]
    carr = (L.amr_camera * 1)(amr.make_camera(cam))
    lutbuf = np.zeros((256, 4), np.float32)
    g = np.zeros(4 * npix, np.float32)
    glut = np.zeros((256, 4), np.float32)
    glight = np.zeros(5, np.float32)
    ck = np.zeros(1 << 16, np.uint8)
    p = dict(prm, lighting=True)
    if case == "nearest":
        p["interp"] = 1
    elif case == "point_light":
        p["lighting"] = 2
    q = amr.make_params(p, lutbuf)
    if case != "no_ckpt":
        q.d_ckpt, q.ckpt_every, q.ckpt_max = ck.ctypes.data, 2, 4
        q.ckpt_bytes = 64 if case == "ckpt_small" else int(lib.amr_ckpt_bytes(npix, 4))
    det = 1 if case == "work_small_det" else 0
    need = int(lib.amr_backward_work_bytes(det))
    assert need == 4 * 1029 * (1 + 2048 * det)
    work = np.zeros(need, np.uint8)
    if case != "no_work":
        q.d_work = work.ctypes.data
        q.work_bytes = int(lib.amr_backward_work_bytes(0)) if case == "work_small_det" else (
            need - 4 if case == "work_small" else need)
    rc = lib.amr_render_backward(ctypes.byref(scene.scene), carr, 1, ctypes.byref(q), g.ctypes.data, glut.ctypes.data,
                                 glight.ctypes.data, det, None)
    msg = lib.amr_last_error().decode()
    want = {"no_ckpt": (1, "checkpoints"), "nearest": (1, "trilinear"), "point_light": (1, "lighting 0 and 1"),
            "ckpt_small": (3, "too small"), "no_work": (1, "workspace"), "work_small": (3, "work_bytes"),
            "work_small_det": (3, "work_bytes")}[case]
    assert rc == want[0] and want[1] in msg, (case, rc, msg)


def test_render_work_bytes():
    """Workspace size queries: the point light's per-ray counts, offsets, scan sums and job total
    for the largest camera plus 16 bytes per job slot, each section 256-byte aligned; nothing for
    the other lighting modes; -1 for invalid arguments.  The adjoint's: 1029 floats, plus one
    partial sum of 1029 floats per block of its 2048-block grid when deterministic."""
    lib = amr.load()
    h, lut, cams, prm = workloads.small_nested(0)
    two = [dict(cams[0], width=300, height=200), dict(cams[1], width=100, height=700)]
    carr = (L.amr_camera * 2)(*[amr.make_camera(c) for c in two])
    lutbuf = np.zeros((256, 4), np.float32)

    def a256(b):
        return (b + 255) // 256 * 256
    for jobs in (0, 1, 1000, 123457):
        q = amr.make_params(dict(prm, lighting=2), lutbuf)
        q.light_jobs = jobs
        n = 100 * 700
        nb = (n + 1023) // 1024
        want = a256(4 * n) + a256(8 * n) + a256(8 * nb) + 256 + a256(8 * jobs) + 2 * a256(4 * jobs)
        assert lib.amr_render_work_bytes(carr, 2, ctypes.byref(q)) == want
    for lighting in (0, 1):
        q = amr.make_params(dict(prm, lighting=lighting), lutbuf)
        assert lib.amr_render_work_bytes(carr, 2, ctypes.byref(q)) == 0
    q = amr.make_params(dict(prm, lighting=2), lutbuf)
    q.light_jobs = -1
    assert lib.amr_render_work_bytes(carr, 2, ctypes.byref(q)) == -1
    assert lib.amr_render_work_bytes(carr, 0, ctypes.byref(q)) == -1
    assert lib.amr_backward_work_bytes(0) == 4 * 1029
    assert lib.amr_backward_work_bytes(1) == 4 * 1029 * 2049
    # the tape: 16-byte records, tape_cap of them per ray; by default as many as fit in 30 % of the
    # device's memory (multiples of 8, at most 2048)
    assert lib.amr_tape_bytes(1000, 7) == 1000 * 7 * 16
    assert amr.default_tape_cap(8 * 512 * 512, total_memory=288 * 10**9) == 2048
    assert amr.default_tape_cap(8 * 1024 * 1024, total_memory=288 * 10**9) == 640
    assert amr.default_tape_cap(8 * 2048 * 2048, total_memory=288 * 10**9) == 160
    assert amr.default_tape_cap(10**12, total_memory=288 * 10**9) == 0
    # the tile schedule: 16 bytes per camera (a 256-byte multiple), then 8 bytes per 8x8 tile
    assert lib.amr_sched_bytes(carr, 2) == 256 + 8 * ((38 * 25) + (13 * 88))
    assert lib.amr_sched_bytes(carr, 0) == -1
    assert lib.amr_tape_bytes(0, 7) == 0 and lib.amr_tape_bytes(-1, 7) == 0 and lib.amr_tape_bytes(5, -1) == 0
