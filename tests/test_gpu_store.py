"""Out-of-core residency on the GPU (amr_store_update + the unchanged render kernels) against the
FP64 oracle restricted to the same resident subset, through the C ABI.  Bars as for full scenes:
segment traces bit-exact, RGBA within 1e-4."""
import numpy as np
import pytest

import oracle
import workloads
from _parity import compare_traces

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _hier(name):
    if name == "lod":
        return workloads.lod_blocks(1)
    if name == "vertex":
        return workloads.random_tiny(2, root_aligned=True).with_vertex_field(
            workloads.gaussian_sum_field(np.random.default_rng(5), n=5, smin=0.06, smax=0.2))
    if name == "tiny":
        return workloads.tiny_samr(3)
    return workloads.random_tiny(int(name[4]), multi_root=name.endswith("m"), max_patches=8)


def _mask(h, seed, keep=0.5):
    rng = np.random.default_rng(seed)
    m = rng.random(len(h.patches)) < keep
    m |= np.array([p.level == 0 for p in h.patches])
    if seed % 3 == 2:
        m[np.flatnonzero(m)[0]] = False       # a hole with no holder: empty leaves
    return m


def _check_bounds(st, sc, mask):
    """Host-side check before any launch: every brick a leaf or face record can reach is
    resident and lies inside the cache."""
    bb = st.brick_bytes()
    ph = sc.patch_headers()
    n = sc.scene.nleaves + sc.scene.nlod
    dt = np.dtype([("lo", np.float64, 3), ("hi", np.float64, 3), ("patch", np.int32),
                   ("level_flags", np.uint32), ("vmin", np.float32), ("vmax", np.float32)])
    leaves = sc._records(sc.scene.leaves, dt, n)
    own = sc._records(sc.scene.leaf_faces, np.dtype(np.int32), 6 * n)
    fdt = np.dtype([("off", np.uint64), ("n", np.int32, 3), ("px", np.int32), ("pxy", np.int32),
                    ("r", np.float32), ("t", np.float32, 3), ("rope", np.int32), ("pad", np.int32, 4)])
    fx = sc._records(sc.scene.face_taps, fdt, 6 * n)
    cap = sc.scene.pool_bytes
    used = leaves["patch"][leaves["patch"] >= 0]
    assert np.all(mask[used])
    for p in np.unique(used):
        assert 64 * 4 <= 4 * int(ph["off"][p]) and 4 * int(ph["off"][p]) + bb[p] <= cap - 256
    single = own >= 0
    assert np.all(mask[own[single]])
    assert np.array_equal(fx["off"][single], ph["off"][own[single]])




@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("name", ["tiny", "lod", "vertex", "rand0", "rand1m", "rand3"])
def test_resident_subsets_vs_oracle(gpu, name, lit, layout):
    """Several resident subsets in a row through one cache (incremental updates): images and
    traces against the oracle restricted to the same subset."""
    import torch
    amr = gpu
    h = _hier(name)
    tree = amr.build_tree(h)
    st = amr.Store(tree, h, brick_layout=layout)
    cache, meta = st.alloc(st.info()["full_cache_bytes"])
    lut = workloads.lut_bumps(np.random.default_rng(len(name)), sigma_scale=10.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    lod = 3.0 if name == "lod" else 0.0
    prm = workloads.default_params(v_hi=vmax, lighting=lit, lod=lod)
    lut_t = torch.from_numpy(lut).cuda()
    cam = workloads.perspective_orbit(35, 27, 0.6 + len(name), 0.25, radius=1.7)
    for seed in range(3):
        mask = _mask(h, seed + 7 * layout)
        sc, rep = st.update(mask, cache, meta)
        _check_bounds(st, sc, mask)
        out = amr.render(sc, cam, lut_t, prm, trace_cap=128, stats=True)
        torch.cuda.synchronize()
        ores = oracle.Oracle(h, resident=mask).render(cam, prm, lut, trace_cap=128)
        err = np.abs(out["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max()
        print("store %s lit=%d layout=%d seed=%d: %d resident, %d remapped, max|err| = %.3g" % (
            name, lit, layout, seed, rep["resident_bricks"], rep["remapped_leaves"], err))
        assert err <= TOL
        compare_traces(amr, out, ores)
        assert amr.stats_dict(out)["guard_hits"] == 0


def test_all_resident_equals_packed_scene(gpu):
    """Every brick resident: the store's scene renders bit-identically to amr_pack_pool's, lit
    and unlit, single camera and persistent batch."""
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(2)
    tree = amr.build_tree(h)
    ref_scene = amr.pack(tree, h, device="cuda", brick_layout=0)
    st = amr.Store(tree, h, brick_layout=0)
    cache, meta = st.alloc(st.info()["full_cache_bytes"] + 8192)
    sc, rep = st.update(np.ones(len(h.patches), bool), cache, meta)
    _check_bounds(st, sc, np.ones(len(h.patches), bool))
    assert rep["remapped_leaves"] == 0
    lut_t = torch.from_numpy(lut).cuda()
    cam_list = [workloads.perspective_orbit(w, hh, 0.3 * k, 0.2, radius=1.8) for k, (w, hh) in
                enumerate([(24, 16), (40, 40), (64, 32)])]
    for lit in (False, True):
        p = dict(prm, lighting=lit)
        a = amr.render(sc, cams[1], lut_t, p)["rgba"]
        b = amr.render(ref_scene, cams[1], lut_t, p)["rgba"]
        c = amr.render(sc, cam_list, lut_t, dict(p, persistent=1, tile_w=8, tile_h=8, blocks_per_cu=2),
                       d_cams=amr.camera_table(cam_list), d_queue=amr.queue_buffer(len(cam_list)))["rgba"]
        d = amr.render(ref_scene, cam_list, lut_t, p)["rgba"]
        torch.cuda.synchronize()
        assert torch.equal(a, b) and torch.equal(c, d)


def test_streaming_cosmology_orbit(gpu):
    """The 1024^2 cosmology-like view family under a cache of 30% of the bricks: a short orbit
    where each frame selects its subset (90% of the cache, the rest is slack against
    fragmentation) and updates the cache incrementally; the last frame is checked against the
    restricted oracle on sampled pixels, and uploads after the first frame stay far below it."""
    import torch
    amr = gpu
    h, lut, cam, prm = workloads.cosmology_view(0)
    tree = amr.build_tree(h)
    st = amr.Store(tree, h, brick_layout=0)
    info = st.info()
    budget = int(0.3 * info["full_cache_bytes"]) // 256 * 256
    cache, meta = st.alloc(budget)
    lut_t = torch.from_numpy(lut).cuda()
    up = []
    rng = np.random.default_rng(4)
    for k in range(4):
        c = workloads.perspective_orbit(1024, 1024, 0.9 + 0.15 * k, 0.2, radius=2.0, fov_deg=40.0)
        mask = st.select(c, int(0.9 * budget))
        sc, rep = st.update(mask, cache, meta)
        _check_bounds(st, sc, mask)
        out = amr.render(sc, c, lut_t, prm, trace_cap=192)
        torch.cuda.synchronize()
        up.append(rep["uploaded_bytes"])
        print("frame %d: %d resident (%.2f GB), uploaded %.3f GB, %d remapped, repacked %d" % (
            k, rep["resident_bricks"], rep["resident_bytes"] / 1e9, rep["uploaded_bytes"] / 1e9,
            rep["remapped_leaves"], rep["repacked"]))
    assert max(up[1:]) < 0.25 * up[0]
    pix = np.stack([rng.integers(0, 1024, 1200), rng.integers(0, 1024, 1200)], 1).astype(np.int32)
    idx = torch.from_numpy(pix[:, 1].astype(np.int64) * 1024 + pix[:, 0]).cuda()
    rgba = out["rgba"].view(-1, 4)[idx].cpu().numpy()
    sub = dict(trace_raw=out["trace_raw"][idx], trace_n=out["trace_n"][idx])
    ores = oracle.Oracle(h, resident=mask).render(c, prm, lut, pixels=pix, trace_cap=192)
    err = np.abs(rgba - ores["rgba"]).max()
    print("streamed frame vs restricted oracle: max|err| = %.3g" % err)
    assert err <= TOL
    compare_traces(amr, sub, ores)
