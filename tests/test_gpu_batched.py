"""Persistent multi-camera kernel: every image of a batch is bit-identical to its single-camera
render; per-image completion stamps; hipGraph capture and replay; the autotuner."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda")
    torch.cuda.synchronize()
    return h, lut, prm, tree, scene


def _cams(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w, hh = int(rng.choice([16, 24, 40, 64, 100])), int(rng.choice([8, 32, 48, 64]))
        out.append(workloads.perspective_orbit(w, hh, float(rng.uniform(0, 6.28)), float(rng.uniform(-0.6, 0.6)),
                                               radius=float(rng.uniform(1.5, 2.5))))
    return out


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("xcd", [0, 1])
@pytest.mark.parametrize("tile", [(8, 8), (16, 4), (4, 16), (32, 2)])
@pytest.mark.parametrize("lit", [False, True])
def test_batched_bit_identical(gpu, tiny, tile, lit, xcd, order):
    """Every image of a persistent batch equals its single-camera render bit for bit, for every
    tile shape, both tile queues (one row-major queue; per-XCD Morton super-tiles) and both
    camera orders; every image gets a completion stamp after the launch-start stamp."""
    import torch
    amr = gpu
    h, lut, prm, tree, scene = tiny
    prm = dict(prm, lighting=lit)
    cams = _cams(9, seed=3)
    lut_t = torch.from_numpy(lut).cuda()
    dc = amr.camera_table(cams)
    q = amr.queue_buffer(len(cams))
    stamps = torch.zeros(len(cams) + 1, dtype=torch.int64, device="cuda")
    out = amr.render(scene, cams, lut_t, dict(prm, persistent=1, tile_w=tile[0], tile_h=tile[1], blocks_per_cu=2,
                                              xcd_tiles=xcd, queue_order=order),
                     d_cams=dc, d_queue=q, d_stamps=stamps, stats=True)
    ref = amr.render(scene, cams, lut_t, prm, stats=True)
    torch.cuda.synchronize()
    assert torch.equal(out["rgba"], ref["rgba"])
    s_b, s_r = amr.stats_dict(out), amr.stats_dict(ref)
    assert s_b["samples"] == s_r["samples"] and s_b["segments"] == s_r["segments"]
    st = stamps.cpu().numpy()
    assert np.all(st[:-1] > 0) and np.all(st[:-1] >= st[-1])


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("wps", [2, 3])
def test_batched_waves_per_simd(gpu, tiny, layout, wps):
    """The lit persistent kernel compiled for 2 or 3 waves per SIMD (its timed variants, no
    statistics) renders every image of a batch bit for bit as the single-camera kernel does, in
    every brick layout."""
    import torch
    amr = gpu
    h, lut, prm, tree, scene = tiny
    prm = dict(prm, lighting=True)
    sc = amr.pack(tree, h, device="cuda", brick_layout=layout)
    cams = _cams(7, seed=5)
    lut_t = torch.from_numpy(lut).cuda()
    dc = amr.camera_table(cams)
    q = amr.queue_buffer(len(cams))
    out = amr.render(sc, cams, lut_t, dict(prm, persistent=1, blocks_per_cu=2, waves_per_simd=wps), d_cams=dc,
                     d_queue=q)["rgba"]
    ref = amr.render(sc, cams, lut_t, prm)["rgba"]
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_graph_capture_replay(gpu, tiny):
    import torch
    amr = gpu
    h, lut, prm, tree, scene = tiny
    prm = dict(prm, lighting=True)
    cams = _cams(6, seed=5)
    lut_t = torch.from_numpy(lut).cuda()
    dc = amr.camera_table(cams)
    q = amr.queue_buffer(len(cams))
    npix = sum(c["width"] * c["height"] for c in cams)
    out = torch.zeros(npix * 4, dtype=torch.float32, device="cuda")
    bprm = dict(prm, persistent=1)
    ref = amr.render(scene, cams, lut_t, prm)["rgba"].clone()
    amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q)     # warm up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q)
    for rep in range(4):
        out.fill_(-1.0)                       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(-1, 4), ref), rep
    # new cameras through the same device table: the replay renders them
    cams2 = _cams(6, seed=5)
    cams2[0] = dict(cams2[0], eye=cams2[0]["eye"] + 0.01)
    dc.copy_(amr.camera_table(cams2))
    g.replay()
    ref2 = amr.render(scene, cams2, lut_t, prm)["rgba"]
    torch.cuda.synchronize()
    assert torch.equal(out.view(-1, 4), ref2)


def test_autotune_picks_a_candidate(gpu, tiny, tmp_path):
    import torch
    amr = gpu
    from paper_1212_3333_amd import autotune
    h, lut, prm, tree, scene = tiny
    cams = _cams(5, seed=8)
    lut_t = torch.from_numpy(lut).cuda()
    dc = amr.camera_table(cams)
    q = amr.queue_buffer(len(cams))
    npix = sum(c["width"] * c["height"] for c in cams)
    out = torch.empty(npix * 4, dtype=torch.float32, device="cuda")
    scenes = {1: scene, 2: amr.pack(tree, h, device="cuda", brick_layout=2)}
    res = autotune.tune(scene, cams, lut_t, prm, dc, q, out, "tiny-test", reps=1,
                        cache_path=str(tmp_path / "cache.json"), scenes=scenes)
    assert (res["tile_w"], res["tile_h"]) in autotune.CANDIDATE_TILES
    assert res["xcd_tiles"] in (0, 1) and res["brick_layout"] in (1, 2)
    assert len(res["table"]) == len(autotune.candidates((1, 2), int(prm.get("lighting", 0)) == 1))
    assert res["waves_per_simd"] in autotune.CANDIDATE_WPS
    again = autotune.tune(scene, cams, lut_t, prm, dc, q, out, "tiny-test", cache_path=str(tmp_path / "cache.json"))
    assert again == res
    # the chosen configuration renders what the single-camera kernel renders
    best = dict(prm, persistent=1, tile_w=res["tile_w"], tile_h=res["tile_h"], blocks_per_cu=res["blocks_per_cu"],
                waves_per_simd=res["waves_per_simd"], xcd_tiles=res["xcd_tiles"], queue_order=res["queue_order"])
    got = amr.render(scenes[res["brick_layout"]], cams, lut_t, best, d_cams=dc, d_queue=q)["rgba"]
    ref = amr.render(scene, cams, lut_t, prm)["rgba"]
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_serving_batch_latency(gpu, tmp_path):
    """Serving-style batch on the cosmology-like hierarchy: 64 orbit cameras with resolutions from
    {256^2, 512^2, 768^2, 1024^2} in one persistent launch captured in a hipGraph, with the tile
    shape and blocks per CU chosen by the autotuner.  Reports per-image latency (launch start to
    the image's completion stamp) p50/p99 and aggregate Mrays/s; sampled images are bit-identical
    to single-camera renders."""
    import torch
    amr = gpu
    from paper_1212_3333_amd import autotune
    h, lut, cam0, prm = workloads.cosmology_view(0)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda")
    lut_t = torch.from_numpy(lut).cuda()
    cams = workloads.serving_cameras(0, 64)
    dc = amr.camera_table(cams)
    q = amr.queue_buffer(len(cams))
    npix = sum(c["width"] * c["height"] for c in cams)
    out = torch.zeros(npix * 4, dtype=torch.float32, device="cuda")
    best = autotune.tune(scene, cams, lut_t, prm, dc, q, out, workload_key="serving64", reps=1,
                         cache_path=str(tmp_path / "tune.json"))
    print("autotuned:", {k: best[k] for k in ("tile_w", "tile_h", "blocks_per_cu", "xcd_tiles", "queue_order", "ms")})
    stamps = torch.zeros(len(cams) + 1, dtype=torch.int64, device="cuda")
    bprm = dict(prm, persistent=1, tile_w=best["tile_w"], tile_h=best["tile_h"], blocks_per_cu=best["blocks_per_cu"],
                xcd_tiles=best["xcd_tiles"], queue_order=best["queue_order"])
    amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q, d_stamps=stamps)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q, d_stamps=stamps)
    lat, agg = [], []
    for rep in range(3):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        st = stamps.cpu().numpy()
        khz = amr.wall_clock_khz()
        assert np.all(st[:-1] >= st[-1]) and st[-1] > 0
        lat.append((st[:-1] - st[-1]) / khz)                 # ms
        agg.append(npix / (e0.elapsed_time(e1) * 1e-3) / 1e6)
    lat = np.concatenate(lat)
    print("batch %d rays: p50 %.2f ms, p99 %.2f ms, aggregate %.1f Mrays/s" % (
        npix, np.percentile(lat, 50), np.percentile(lat, 99), float(np.median(agg))))
    # images: the smallest and the largest camera against single-camera renders
    offs = np.cumsum([0] + [c["width"] * c["height"] for c in cams])
    sizes = [c["width"] * c["height"] for c in cams]
    for c in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        ref = amr.render(scene, cams[c], lut_t, prm)["rgba"].reshape(-1, 4)
        torch.cuda.synchronize()
        assert torch.equal(out.view(-1, 4)[offs[c]:offs[c + 1]], ref)

