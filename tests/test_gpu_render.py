"""GPU parity of amr_render against the FP64 oracle, through the C ABI.

Bars: per-ray segment lists (leaf, patch, sample count, FP64 t_a, t_b) bit-exact; RGBA within
1e-4 max abs; closed forms within 1e-5."""
import math

import numpy as np
import pytest

import oracle
import workloads
from _parity import compare_traces, pixel_set

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _setup(amr, h, layout=1):
    import torch
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda", brick_layout=layout)
    torch.cuda.synchronize()
    return tree, scene


def _gpu_render(amr, scene, cam, lut, prm, trace_cap=0, stats=False, nsamp=False):
    import torch
    out = amr.render(scene, cam, torch.from_numpy(np.asarray(lut, np.float32)).cuda(), prm, trace_cap=trace_cap,
                     stats=stats, nsamp=nsamp)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("uniform", [False, True])
@pytest.mark.parametrize("cam_idx", [0, 1])
def test_small_nested_full_image(gpu, cam_idx, uniform, lit, layout):
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    cam = cams[cam_idx]
    prm = dict(prm, uniform_step=uniform, lighting=lit)
    tree, scene = _setup(amr, h, layout)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=64, stats=True, nsamp=True)
    O = oracle.Oracle(h)
    ores = O.render(cam, prm, lut, trace_cap=64)
    rgba = gout["rgba"].cpu().numpy().reshape(-1, 4).astype(np.float64)
    err = np.abs(rgba - ores["rgba"]).max()
    print("small_nested cam%d uniform=%d lit=%d max|err|=%.3g" % (cam_idx, uniform, lit, err))
    assert err <= TOL
    compare_traces(amr, gout, ores)
    st = amr.stats_dict(gout)
    assert st["guard_hits"] == 0 and st["trace_overflow"] == 0
    ns = gout["nsamp"].cpu().numpy()
    # sample counts agree except where fp32 and fp64 transmittance cross t_min at different samples
    assert np.mean(ns == ores["nsamp"]) > 0.999


@pytest.mark.parametrize("lit", [False, True])
def test_constant_field_gpu(gpu, lit):
    amr = gpu
    cv = 0.6
    h = workloads.tiny_samr(2).with_field(workloads.constant_field(cv))
    lut = workloads.lut_small_nested(3)
    prm = workloads.default_params(v_lo=0.0, v_hi=1.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75)
    cam = workloads.perspective_orbit(48, 40, 0.4, 0.35, radius=1.6)
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=64)
    rgba = gout["rgba"].cpu().numpy().reshape(-1, 4)
    xs = np.arange(256) / 255.0
    u = float(np.float32(cv))
    sig = np.interp(u, xs, lut[:, 3].astype(np.float64))
    rgb = np.array([np.interp(u, xs, lut[:, c].astype(np.float64)) for c in range(3)])
    g = amr.trace_records(gout)
    gn = gout["trace_n"].cpu().numpy()
    for q in range(len(rgba)):
        if gn[q] == 0:
            assert np.all(rgba[q] == 0)
            continue
        L = g[q, gn[q] - 1]["tb"] - g[q, 0]["ta"]      # chord: first entry to last exit
        A = 1 - math.exp(-sig * L)
        assert abs(rgba[q, 3] - A) < 1e-5
        assert np.all(np.abs(rgba[q, :3] - rgb * A * (0.25 if lit else 1.0)) < 1e-5)


@pytest.mark.parametrize("lit", [False, True])
def test_linear_field_gpu(gpu, lit):
    amr = gpu
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    h = workloads.tiny_samr(4).with_field(workloads.linear_field(a, b))
    s = 255.0 / 64
    lut = workloads.lut_linear_sigma(s, rgb=(0.75, 0.5, 0.25))
    m = 3.0 / 32
    prm = workloads.default_params(v_lo=0.0, v_hi=2.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75, eps_g=0.0,
                                   light=(1.0, 2.0, -0.5), clip_lo=(m, m, m), clip_hi=(1 - m, 1 - m, 1 - m))
    cam = workloads.ortho_oblique(48, 48)
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=64)
    rgba = gout["rgba"].cpu().numpy().reshape(-1, 4)
    g = amr.trace_records(gout)
    gn = gout["trace_n"].cpu().numpy()
    l = np.array(prm["light"], dtype=np.float64)
    shade = 0.25 + 0.75 * abs(a @ l) / (np.linalg.norm(a) * np.linalg.norm(l)) if lit else 1.0
    hits = 0
    for q in range(len(rgba)):
        if gn[q] == 0:
            continue
        hits += 1
        i, j = q % 48, q // 48
        o, d = oracle.ray(cam, i, j)
        ta, tb = g[q, 0]["ta"], g[q, gn[q] - 1]["tb"]
        xm = o + 0.5 * (ta + tb) * d
        A = 1 - math.exp(-s * (tb - ta) * (a @ xm + b) / 2.0)
        assert abs(rgba[q, 3] - A) < 1e-5
        assert np.all(np.abs(rgba[q, :3] - np.array([0.75, 0.5, 0.25]) * shade * A) < 1e-5)
    assert hits > 500


@pytest.mark.parametrize("seed", range(6))
def test_random_hierarchies(gpu, seed):
    amr = gpu
    h = workloads.random_tiny(seed, multi_root=(seed % 2 == 1))
    lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=12.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    m = 0.05 * (seed % 3)
    prm = workloads.default_params(v_hi=vmax, lighting=(seed % 2 == 0), clip_lo=(m, 0, m), clip_hi=(1, 1 - m, 1))
    cam = workloads.perspective_orbit(37, 23, 0.3 + seed, 0.2 * seed - 0.4, radius=1.8)   # ragged tiles
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=256)
    ores = oracle.Oracle(h).render(cam, prm, lut, trace_cap=256)
    rgba = gout["rgba"].cpu().numpy().reshape(-1, 4)
    assert np.abs(rgba - ores["rgba"]).max() <= TOL
    compare_traces(amr, gout, ores)


def test_degenerate_views(gpu):
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    tree, scene = _setup(amr, h)
    # one pixel
    cam = workloads.ortho_axis_z(1, 1)
    out = _gpu_render(amr, scene, cam, lut, prm)
    ref = oracle.Oracle(h).render(cam, prm, lut)["rgba"]
    assert np.abs(out["rgba"].cpu().numpy().reshape(-1, 4) - ref).max() <= TOL
    # a camera looking away from the domain: every pixel transparent
    away = workloads.camera([0.5, 0.5, -1.0], [1, 0, 0], [0, 1, 0], [0, 0, -1], 20, 20, tan_half_fov=0.3)
    out = _gpu_render(amr, scene, away, lut, prm, stats=True)
    assert np.all(out["rgba"].cpu().numpy() == 0) and amr.stats_dict(out)["rays_hit"] == 0
    # empty clip box
    out = _gpu_render(amr, scene, cams[0], lut, dict(prm, clip_lo=(0.6, 0, 0), clip_hi=(0.4, 1, 1)))
    assert np.all(out["rgba"].cpu().numpy() == 0)


def test_invalid_arguments(gpu):
    amr = gpu
    import torch
    h, lut, cams, prm = workloads.small_nested(0)
    tree, scene = _setup(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    with pytest.raises(amr.AMRError):
        amr.render(scene, cams[0], lut_t, dict(prm, v_hi=prm["v_lo"]))
    with pytest.raises(amr.AMRError):
        amr.render(scene, dict(cams[0], width=0), lut_t, prm)
    with pytest.raises(amr.AMRError):
        amr.render(scene, cams[0], lut_t, dict(prm, step_frac=0.0))


@pytest.fixture(scope="module")
def cosmology_scene(gpu):
    amr = gpu
    h, lut, cam, prm = workloads.cosmology_view(0)
    tree, scene = _setup(amr, h)
    return h, lut, cam, prm, tree, scene


def test_cosmology_linear_layout_sampled(gpu, cosmology_scene):
    """The linear brick layout (row loads in the lit stencil) on the cosmology-like view, lit and
    unlit: a pixel sample against the oracle, and the image within 1e-5 of the micro-brick one."""
    import torch
    amr = gpu
    h, lut, cam, prm, tree, scene1 = cosmology_scene
    scene0 = amr.pack(tree, h, device="cuda", brick_layout=0)
    lut_t = torch.from_numpy(lut).cuda()
    rng = np.random.default_rng(21)
    pix = np.stack([rng.integers(0, cam["width"], 1500), rng.integers(0, cam["height"], 1500)], 1).astype(np.int32)
    O = oracle.Oracle(h)
    for lit in (True, False):
        p = dict(prm, lighting=lit)
        a = amr.render(scene0, cam, lut_t, p)["rgba"].clone()
        b = amr.render(scene1, cam, lut_t, p)["rgba"]
        torch.cuda.synchronize()
        ref = O.render(cam, p, lut, pixels=pix)["rgba"]
        err = np.abs(a.cpu().numpy()[pix[:, 1], pix[:, 0]] - ref).max()
        print("linear layout lit=%d: max|err| vs oracle %.3g, vs micro-bricks %.3g" % (lit, err, (a - b).abs().max().item()))
        assert err <= TOL
        assert (a - b).abs().max().item() <= 1e-5
    del scene0


@pytest.mark.parametrize("lit", [True, False])
def test_cosmology_full_size_sampled(gpu, cosmology_scene, lit):
    """The 1024x1024 cosmology-like frame through the recording forward variant (trace and
    counters on, brick layout read at run time) on the micro-brick pool: 16,384 seeded pixels,
    four full rows and a 64x64 crop against the oracle, RGBA within 1e-4 and segment traces
    bit-exact.  The benchmark's own launch (halo-row pool, non-recording kernel) is checked in
    test_gpu_timed_config.py."""
    import torch
    amr = gpu
    h, lut, cam, prm, tree, scene = cosmology_scene
    prm = dict(prm, lighting=lit)
    W, H = cam["width"], cam["height"]
    cap = 192
    out = _gpu_render(amr, scene, cam, lut, prm, trace_cap=cap, stats=True)
    pix = pixel_set(W, H, 11)
    idx = torch.from_numpy(pix[:, 1].astype(np.int64) * W + pix[:, 0]).cuda()
    rgba = out["rgba"].view(-1, 4)[idx].cpu().numpy().astype(np.float64)
    sub = dict(trace_raw=out["trace_raw"][idx], trace_n=out["trace_n"][idx])
    del out
    ores = oracle.Oracle(h).render(cam, prm, lut, pixels=pix, trace_cap=cap)
    err = np.abs(rgba - ores["rgba"]).max()
    print("cosmology_view lit=%d: %d pixels, max|err| = %.3g, max segments %d" % (lit, len(pix), err, ores["trace_n"].max()))
    assert err <= TOL
    assert ores["trace_n"].max() <= cap
    compare_traces(amr, sub, ores, "cosmology micro-bricks lit=%d" % lit)


@pytest.mark.parametrize("interp", [0, 1])
def test_deferred_taps_do_not_depend_on_scheduling(gpu, cosmology_scene, interp):
    """Lit samples whose gradient taps leave the brick wait in a per-wave queue; each ray sums its
    deferred colour separately in sample order, so the image must not depend on when the queue
    is resolved or which rays share a wave.  On the 1024x1024 cosmology-like view: the plain
    render, the recording variant, the checkpointed render (which resolves the queue before
    every segment fetch that writes a checkpoint) and, for trilinear sampling, the persistent
    kernel with 16x4 tiles (which resolves it inside its per-segment loop) give bit-identical
    images; the queue never runs out of slots."""
    import torch
    amr = gpu
    h, lut, cam, prm, tree, scene = cosmology_scene
    prm = dict(prm, lighting=True, interp=interp)
    lut_t = torch.from_numpy(lut).cuda()
    plain = amr.render(scene, cam, lut_t, prm)["rgba"].clone()
    rec = amr.render(scene, cam, lut_t, prm, stats=True)
    torch.cuda.synchronize()
    st = amr.stats_dict(rec)
    print("interp=%d: %d samples, %d with deferred taps, guard hits %d" % (
        interp, st["samples"], st["split_samples"], st["guard_hits"]))
    assert st["guard_hits"] == 0
    assert 0.05 * st["samples"] < st["split_samples"] < 0.5 * st["samples"]
    assert torch.equal(plain, rec["rgba"])
    del rec
    if interp == 0:
        out, ck = amr.render_checkpointed(scene, cam, lut_t, prm, ckpt_every=2, ckpt_max=8)
        torch.cuda.synchronize()
        assert torch.equal(plain, out["rgba"])
        del out, ck
        cams = [cam]
        per = amr.render(scene, cams, lut_t, dict(prm, persistent=1, tile_w=16, tile_h=4, blocks_per_cu=2),
                         d_cams=amr.camera_table(cams), d_queue=amr.queue_buffer(1))["rgba"]
        torch.cuda.synchronize()
        assert torch.equal(plain, per.view(-1, 4).view_as(plain))


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("cam_idx", [0, 1])
def test_nearest_small_nested(gpu, cam_idx, lit):
    """Nearest-cell sampling (interp = 1): full images against the oracle, traces bit-exact."""
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    prm = dict(prm, lighting=lit, interp=1)
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cams[cam_idx], lut, prm, trace_cap=64, stats=True)
    ores = oracle.Oracle(h).render(cams[cam_idx], prm, lut, trace_cap=64)
    err = np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max()
    print("nearest cam%d lit=%d max|err|=%.3g" % (cam_idx, lit, err))
    assert err <= TOL
    compare_traces(amr, gout, ores)


@pytest.mark.parametrize("seed", range(4))
def test_nearest_random_hierarchies(gpu, seed):
    amr = gpu
    h = workloads.random_tiny(seed, multi_root=(seed % 2 == 1))
    lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=12.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=(seed % 2 == 0), interp=1)
    cam = workloads.perspective_orbit(37, 23, 0.3 + seed, 0.2 * seed - 0.4, radius=1.8)
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=256)
    ores = oracle.Oracle(h).render(cam, prm, lut, trace_cap=256)
    assert np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max() <= TOL
    compare_traces(amr, gout, ores)


def test_nearest_cosmology_sampled(gpu, cosmology_scene):
    """Nearest-cell sampling on the cosmology-like hierarchy at 1024^2, lit: a seeded pixel sample
    against the oracle."""
    import torch
    amr = gpu
    h, lut, cam, prm, tree, scene = cosmology_scene
    prm = dict(prm, interp=1)
    out = amr.render(scene, cam, torch.from_numpy(lut).cuda(), prm)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pix = np.stack([rng.integers(0, cam["width"], 1500), rng.integers(0, cam["height"], 1500)], 1).astype(np.int32)
    ref = oracle.Oracle(h).render(cam, prm, lut, pixels=pix)["rgba"]
    got = out["rgba"].cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = np.abs(got - ref).max()
    print("nearest cosmology: max|err| = %.3g" % err)
    assert err <= TOL


def test_nearest_rejected_outside_plain_forward(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    tree, scene = _setup(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    with pytest.raises(amr.AMRError, match="nearest"):
        amr.render_checkpointed(scene, cams[0], lut_t, dict(prm, interp=1))
    with pytest.raises(amr.AMRError, match="interp"):
        amr.render(scene, cams[0], lut_t, dict(prm, interp=2))
    two = [cams[0], cams[1]]
    with pytest.raises(amr.AMRError, match="nearest"):
        amr.render(scene, two, lut_t, dict(prm, interp=1, persistent=1), d_cams=amr.camera_table(two),
                   d_queue=amr.queue_buffer(2))


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("lod", [1.5, 3.0, 1e6])
@pytest.mark.parametrize("seed", range(3))
def test_lod_vs_oracle(gpu, seed, lod, lit):
    """Level-of-detail renders (the descent stops at kind-(a) nodes whose coarse cells project
    below `lod` pixels): images against the oracle, traces bit-exact including the ids of the
    level-of-detail segments (nleaves + the node's pre-order rank among kind-(a) nodes)."""
    amr = gpu
    h = workloads.lod_blocks(seed)
    lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=6.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=lit, lod=lod)
    tree, scene = _setup(amr, h)
    assert scene.scene.nlod > 0
    for cam in (workloads.perspective_orbit(33, 25, 0.7 + seed, 0.3 - 0.2 * seed, radius=1.7),
                workloads.ortho_oblique(24, 24)):
        gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=128)
        ores = oracle.Oracle(h).render(cam, prm, lut, trace_cap=128)
        assert np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max() <= TOL
        compare_traces(amr, gout, ores)
        if lod >= 3.0:
            assert np.any(ores["trace"]["leaf"] >= scene.scene.nleaves)


def test_lod_cosmology_sampled(gpu, cosmology_scene):
    """Level of detail (lod = 2 pixels) on the cosmology-like hierarchy at 1024^2, lit: a pixel
    sample against the oracle; fewer samples than the full-detail render."""
    import torch
    amr = gpu
    h, lut, cam, prm, tree, scene = cosmology_scene
    lprm = dict(prm, lod=2.0)
    lut_t = torch.from_numpy(lut).cuda()
    out = amr.render(scene, cam, lut_t, lprm, stats=True)
    full = amr.render(scene, cam, lut_t, prm, stats=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    pix = np.stack([rng.integers(0, cam["width"], 1500), rng.integers(0, cam["height"], 1500)], 1).astype(np.int32)
    ref = oracle.Oracle(h).render(cam, lprm, lut, pixels=pix)["rgba"]
    got = out["rgba"].cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = np.abs(got - ref).max()
    sl, sf = amr.stats_dict(out)["samples"], amr.stats_dict(full)["samples"]
    print("lod cosmology: max|err| = %.3g, samples %d vs %d at full detail" % (err, sl, sf))
    assert err <= TOL
    assert sl < sf


@pytest.mark.parametrize("light", [(0.5, 0.45, 0.55), (1.6, -0.3, 0.4)])
@pytest.mark.parametrize("case", ["small0", "small1", "rand0", "rand1"])
def test_point_light_vs_oracle(gpu, case, light):
    """Point-light secondary rays (lighting = 2): every primary sample shaded by the
    transmittance of a secondary ray to the light; images against the oracle, traces bit-exact."""
    amr = gpu
    if case.startswith("small"):
        h, lut, cams, prm = workloads.small_nested(0)
        cam = workloads.small_nested_cameras(48, 48)[int(case[-1])]
        prm = dict(prm, lighting=2, light=light, k_a=0.2, k_d=0.8)
    else:
        seed = int(case[-1])
        h = workloads.random_tiny(seed, multi_root=(seed == 1))
        lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=12.0)
        vmax = float(max(p.cells.max() for p in h.patches))
        prm = workloads.default_params(v_hi=vmax, lighting=2, light=light, k_a=0.2, k_d=0.8)
        cam = workloads.perspective_orbit(37, 23, 0.3 + seed, 0.2 * seed - 0.4, radius=1.8)
    tree, scene = _setup(amr, h)
    gout = _gpu_render(amr, scene, cam, lut, prm, trace_cap=128)
    ores = oracle.Oracle(h).render(cam, prm, lut, trace_cap=128)
    err = np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max()
    print("point light %s %s: max|err| = %.3g" % (case, light, err))
    assert err <= TOL
    compare_traces(amr, gout, ores)


def test_point_light_rejected_elsewhere(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    tree, scene = _setup(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    with pytest.raises(amr.AMRError, match="point-light"):
        amr.render_checkpointed(scene, cams[0], lut_t, dict(prm, lighting=2))
    with pytest.raises(amr.AMRError, match="point-light"):
        amr.render(scene, cams[0], lut_t, dict(prm, lighting=2, lod=2.0))
    with pytest.raises(amr.AMRError, match="lighting"):
        amr.render(scene, cams[0], lut_t, dict(prm, lighting=3))
    two = [cams[0], cams[1]]
    with pytest.raises(amr.AMRError, match="point-light"):
        amr.render(scene, two, lut_t, dict(prm, lighting=2, persistent=1), d_cams=amr.camera_table(two),
                   d_queue=amr.queue_buffer(2))



def _orbit_cams(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(40, 24), (64, 64), (17, 33), (48, 40), (8, 8), (72, 56), (33, 17), (56, 48), (24, 40), (64, 24)]
    return [workloads.perspective_orbit(sizes[i % len(sizes)][0], sizes[i % len(sizes)][1],
                                        float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(-0.6, 0.6)),
                                        radius=float(rng.uniform(1.5, 2.5))) for i in range(n)]


@pytest.mark.parametrize("mode", ["timed", "recording", "checkpoints"])
@pytest.mark.parametrize("lit", [False, True])
def test_camera_groups_match_single_camera_launches(gpu, lit, mode):
    """Several cameras in one amr_render call are rendered up to 8 per launch (one camera per
    blockIdx.y).  Ten cameras of different sizes (two launches: 8 and 2) against one call per
    camera: images, per-ray sample counts and segment traces (recording kernels), checkpoint
    records and the lit tape (checkpointed kernels) are bit-identical."""
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=lit)
    tree, scene = _setup(amr, h, layout=2)
    lut_t = torch.from_numpy(lut).cuda()
    cl = _orbit_cams(10, seed=21)
    npix = [c["width"] * c["height"] for c in cl]
    if mode == "checkpoints":
        out, ck = amr.render_checkpointed(scene, cl, lut_t, prm, ckpt_every=2, ckpt_max=8, tape_cap=256 if lit else 0)
        torch.cuda.synchronize()
        off = 0
        for c, cam in enumerate(cl):
            o1, k1 = amr.render_checkpointed(scene, cam, lut_t, prm, ckpt_every=2, ckpt_max=8,
                                             tape_cap=256 if lit else 0)
            torch.cuda.synchronize()
            assert torch.equal(out["rgba"].view(-1, 4)[off:off + npix[c]], o1["rgba"].view(-1, 4)), c
            # per ray a 32-byte header and up to 8 32-byte checkpoints, of which the first nck are
            # written; the tape rows hold nrec records, of which the first 256 are written
            a = ck.buf.view(sum(npix), 9, 32)[off:off + npix[c]].cpu().numpy()
            b = k1.buf.view(npix[c], 9, 32).cpu().numpy()
            assert np.array_equal(a[:, 0], b[:, 0]), c
            nck = b[:, 0].copy().view(np.int32)[:, 5]
            for r in range(npix[c]):
                assert np.array_equal(a[r, 1:1 + nck[r]], b[r, 1:1 + nck[r]]), (c, r)
            if lit:
                nrec = np.minimum(b[:, 0].copy().view(np.int32)[:, 7], 256)
                ta = ck.tape.view(sum(npix), 256, 4)[off:off + npix[c]].cpu().numpy()
                tb = k1.tape.view(npix[c], 256, 4).cpu().numpy()
                for r in range(npix[c]):
                    assert np.array_equal(ta[r, :nrec[r]], tb[r, :nrec[r]]), (c, r)
            off += npix[c]
        return
    kw = dict(trace_cap=64, nsamp=True, stats=True) if mode == "recording" else {}
    out = amr.render(scene, cl, lut_t, prm, **kw)
    torch.cuda.synchronize()
    off = 0
    for c, cam in enumerate(cl):
        o1 = amr.render(scene, cam, lut_t, prm, **kw)
        torch.cuda.synchronize()
        assert torch.equal(out["rgba"].view(-1, 4)[off:off + npix[c]], o1["rgba"].view(-1, 4)), c
        if mode == "recording":
            assert torch.equal(out["nsamp"][off:off + npix[c]], o1["nsamp"]), c
            assert torch.equal(out["trace_n"][off:off + npix[c]], o1["trace_n"]), c
            assert torch.equal(out["trace_raw"][off:off + npix[c]], o1["trace_raw"]), c
        off += npix[c]


def _sched_bucket(t):
    t = int(t)
    if t < 16:
        return t
    msb = t.bit_length() - 1
    return min(511, (msb - 3) * 16 + ((t >> (msb - 4)) & 15))


@pytest.mark.parametrize("mode", ["timed", "recording", "checkpoints"])
@pytest.mark.parametrize("lit", [False, True])
def test_tile_schedule(gpu, lit, mode):
    """With a tile schedule, each call records every tile's time and sorts the super-tiles (2x2
    tiles lit, 4x4 unlit) of each launch's cameras (up to 8) by their longest tile; the next call
    starts them in that order.  Over three calls of ten cameras of different sizes (two launches), images, sample
    counts and traces (recording kernels), checkpoint records and tape records (checkpointed
    kernels) are bit-identical to the calls without a schedule; afterwards each launch's order
    holds every (camera, super-tile) of its cameras once, in non-increasing buckets of their
    longest tile's time, and its first camera's header holds the order's key (non-zero)."""
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=lit)
    tree, scene = _setup(amr, h, layout=2)
    lut_t = torch.from_numpy(lut).cuda()
    cl = _orbit_cams(10, seed=22)
    npix = sum(c["width"] * c["height"] for c in cl)
    sch = amr.Schedule(cl, "cuda")

    def run(**kw):
        if mode == "checkpoints":
            out, ck = amr.render_checkpointed(scene, cl, lut_t, prm, ckpt_every=2, ckpt_max=8,
                                              tape_cap=256 if lit else 0, **kw)
            torch.cuda.synchronize()
            return out, ck
        extra = dict(trace_cap=64, nsamp=True, stats=True) if mode == "recording" else {}
        out = amr.render(scene, cl, lut_t, prm, **extra, **kw)
        torch.cuda.synchronize()
        return out, None
    ref, rck = run()
    for call in range(3):
        out, ck = run(**sch.params())
        assert torch.equal(out["rgba"], ref["rgba"]), call
        if mode == "recording":
            for k in ("nsamp", "trace_n", "trace_raw"):
                assert torch.equal(out[k], ref[k]), (call, k)
        if mode == "checkpoints":
            a = ck.buf.view(npix, 9, 32).cpu().numpy()
            b = rck.buf.view(npix, 9, 32).cpu().numpy()
            assert np.array_equal(a[:, 0], b[:, 0])
            nck = b[:, 0].copy().view(np.int32)[:, 5]
            nrec = np.minimum(b[:, 0].copy().view(np.int32)[:, 7], 256)
            for r in range(0, npix, 7):
                assert np.array_equal(a[r, 1:1 + nck[r]], b[r, 1:1 + nck[r]]), r
                if lit:
                    ta = ck.tape.view(npix, 256, 4)[r, :nrec[r]].cpu().numpy()
                    tb = rck.tape.view(npix, 256, 4)[r, :nrec[r]].cpu().numpy()
                    assert np.array_equal(ta, tb), r
    words = sch.buf.view(torch.int32).cpu().numpy().view(np.uint32)
    hw = (4 * len(cl) + 63) // 64 * 64
    t8 = [((c["width"] + 7) // 8, (c["height"] + 7) // 8) for c in cl]
    toff = np.concatenate([[0], np.cumsum([x * y for x, y in t8])])
    ntot = int(toff[-1])
    tm, order = words[hw:hw + ntot], words[hw + ntot:hw + 2 * ntot]
    side = 2 if lit else 4
    for c0 in range(0, len(cl), 8):
        grp = list(range(c0, min(c0 + 8, len(cl))))
        assert words[4 * c0 + 1] != 0, c0
        pairs = [(i, s) for i, c in enumerate(grp)
                 for s in range(((t8[c][0] + side - 1) // side) * ((t8[c][1] + side - 1) // side))]
        o = order[toff[c0]:toff[c0] + len(pairs)]
        got = [(int(e) >> 24, int(e) & 0xffffff) for e in o]
        assert sorted(got) == sorted(pairs), c0

        def longest(i, s):
            c = grp[i]
            tx, ty = t8[c]
            sgw = (tx + side - 1) // side
            times = tm[toff[c]:toff[c] + tx * ty].reshape(ty, tx)
            y0, x0 = (s // sgw) * side, (s % sgw) * side
            return int(times[y0:y0 + side, x0:x0 + side].max())
        bk = [_sched_bucket(longest(i, s)) for (i, s) in got]
        assert all(bk[j] >= bk[j + 1] for j in range(len(bk) - 1)), c0


def test_tile_schedule_camera_list_change(gpu):
    """One schedule buffer used with 18 cameras (three launches), then 9 other cameras of other
    sizes, whose header, times and orders overwrite parts of the first list's, then the 18 again,
    then the 18 unlit (other super-tiles) and lit again: every call's images equal those of calls
    without a schedule (a call after a change renders in the default order and records afresh;
    the next one uses the new order)."""
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=True)
    tree, scene = _setup(amr, h, layout=2)
    lut_t = torch.from_numpy(lut).cuda()
    l1 = _orbit_cams(18, seed=5)
    l2 = _orbit_cams(12, seed=6)[3:]
    sch = amr.Schedule(l1, "cuda")
    assert int(amr.load().amr_sched_bytes(amr._cams(l2)[1], len(l2))) <= sch.nbytes

    def img(cl, **kw):
        r = amr.render(scene, cl, lut_t, prm, **kw)["rgba"].clone()
        torch.cuda.synchronize()
        return r
    ref1, ref2 = img(l1), img(l2)
    for i, cl in enumerate([l1, l1, l2, l2, l1, l1, l2, l1]):
        assert torch.equal(img(cl, **sch.params()), ref1 if cl is l1 else ref2), i
    words = sch.buf.view(torch.int32).cpu().numpy().view(np.uint32)
    assert all(words[4 * c0 + 1] != 0 for c0 in (0, 8, 16))
    # unlit calls use larger super-tiles: the lit order is not reused, and back again
    prm_u = dict(prm, lighting=False)
    ref_u = amr.render(scene, l1, lut_t, prm_u)["rgba"].clone()
    for i in range(2):
        got = amr.render(scene, l1, lut_t, prm_u, **sch.params())["rgba"]
        torch.cuda.synchronize()
        assert torch.equal(got, ref_u), i
    assert torch.equal(img(l1, **sch.params()), ref1)
