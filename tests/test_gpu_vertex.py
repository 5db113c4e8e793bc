"""GPU parity of vertex-centred scenes (Section 5: samples on the grid vertices, trilinear
interpolation, dangling nodes replaced at pack time) against the FP64 oracle, through the C ABI.

The kernels are the cell-centred ones: the packer presents a patch of n cells as n + 1 samples at
integer positions.  Bars as for cell-centred data: per-ray segment lists bit-exact (the tree does
not depend on the centring), RGBA within 1e-4, closed forms within 1e-5, gradients as in the
adjoint tests."""
import math

import numpy as np
import pytest

import oracle
import workloads
from _parity import compare_traces

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _field(seed):
    return workloads.gaussian_sum_field(np.random.default_rng(seed + 31), n=5, smin=0.06, smax=0.2)


def _hier(name):
    if name == "tiny":
        h = workloads.tiny_samr(1)
    elif name == "lod":
        h = workloads.lod_blocks(2)
    elif name.startswith("aligned"):
        h = workloads.random_tiny(int(name[-1]), root_aligned=True)
    else:
        h = workloads.random_tiny(int(name[4]), multi_root=name.endswith("m"))
    return h.with_vertex_field(_field(len(name)))


def _setup(amr, h, layout=1):
    import torch
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda", brick_layout=layout)
    torch.cuda.synchronize()
    assert scene.scene.centering == 1
    return tree, scene


def _render(amr, scene, cam, lut, prm, **kw):
    import torch
    out = amr.render(scene, cam, torch.from_numpy(np.asarray(lut, np.float32)).cuda(), prm, **kw)
    torch.cuda.synchronize()
    return out




@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("name", ["tiny", "lod", "aligned0", "aligned5", "rand1", "rand2m", "rand3"])
def test_vertex_vs_oracle(gpu, name, lit, layout):
    """Full images (ragged tiles) and segment traces against the oracle, all three brick layouts."""
    amr = gpu
    h = _hier(name)
    lut = workloads.lut_bumps(np.random.default_rng(len(name)), sigma_scale=10.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=lit)
    tree, scene = _setup(amr, h, layout)
    O = oracle.Oracle(h)
    for cam in (workloads.perspective_orbit(37, 29, 0.4 + len(name), 0.3, radius=1.7),
                workloads.ortho_oblique(24, 24)):
        gout = _render(amr, scene, cam, lut, prm, trace_cap=128, stats=True)
        ores = O.render(cam, prm, lut, trace_cap=128)
        err = np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max()
        print("vertex %s lit=%d layout=%d: max|err| = %.3g" % (name, lit, layout, err))
        assert err <= TOL
        compare_traces(amr, gout, ores)
        assert amr.stats_dict(gout)["guard_hits"] == 0


@pytest.mark.parametrize("lit", [False, True])
def test_vertex_linear_field_closed_form(gpu, lit):
    """A linear field on vertex data is reproduced exactly on all of B, so the closed form of
    the oracle pin holds for the GPU image without a clip margin."""
    amr = gpu
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    h = workloads.tiny_samr(4).with_vertex_field(workloads.linear_field(a, b))
    s = 255.0 / 64
    lut = workloads.lut_linear_sigma(s, rgb=(0.75, 0.5, 0.25))
    prm = workloads.default_params(v_lo=0.0, v_hi=2.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75,
                                   eps_g=0.0, light=(1.0, 2.0, -0.5))
    cam = workloads.perspective_orbit(40, 30, 0.4, 0.35, radius=1.6)
    tree, scene = _setup(amr, h)
    rgba = _render(amr, scene, cam, lut, prm)["rgba"].cpu().numpy().reshape(cam["height"], cam["width"], 4)
    l = np.array([float(np.float32(x)) for x in prm["light"]])
    shade = 0.25 + 0.75 * abs(a @ l) / (np.linalg.norm(a) * np.linalg.norm(l)) if lit else 1.0
    hits, worst = 0, 0.0
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            o, d = oracle.ray(cam, i, j)
            t0, t1 = 0.0, math.inf
            for ax in range(3):
                ta, tb = (0.0 - o[ax]) / d[ax], (1.0 - o[ax]) / d[ax]
                t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
            if not t1 > t0:
                continue
            hits += 1
            um = (a @ (o + 0.5 * (t0 + t1) * d) + b) / 2.0
            A = 1 - math.exp(-s * (t1 - t0) * um)
            want = np.array([0.75 * shade * A, 0.5 * shade * A, 0.25 * shade * A, A])
            worst = max(worst, float(np.abs(rgba[j, i] - want).max()))
    print("vertex linear closed form lit=%d: max|err| = %.3g over %d rays" % (lit, worst, hits))
    assert hits > 100 and worst <= 1e-5


def test_vertex_nearest_rejected(gpu):
    import torch
    amr = gpu
    h = _hier("tiny")
    tree, scene = _setup(amr, h)
    lut_t = torch.from_numpy(workloads.lut_small_nested(0)).cuda()
    with pytest.raises(amr.AMRError, match="cell-centred"):
        amr.render(scene, workloads.ortho_axis_z(8, 8), lut_t, workloads.default_params(interp=1))


@pytest.mark.parametrize("lit", [False, True])
def test_vertex_lod_and_batched(gpu, lit):
    """Level of detail on vertex data against the oracle; the persistent multi-camera kernel
    bit-identical to single-camera renders."""
    import torch
    amr = gpu
    h = _hier("lod")
    lut = workloads.lut_bumps(np.random.default_rng(5), sigma_scale=8.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=lit, lod=3.0)
    tree, scene = _setup(amr, h)
    cam = workloads.perspective_orbit(33, 25, 1.1, 0.2, radius=1.7)
    gout = _render(amr, scene, cam, lut, prm, trace_cap=128)
    ores = oracle.Oracle(h).render(cam, prm, lut, trace_cap=128)
    assert np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max() <= TOL
    compare_traces(amr, gout, ores)
    assert np.any(ores["trace"]["leaf"] >= scene.scene.nleaves)
    cams = [workloads.perspective_orbit(w, hh, 0.5 * k, 0.1 * k - 0.2, radius=1.9)
            for k, (w, hh) in enumerate([(16, 8), (40, 32), (24, 48), (64, 64)])]
    prm = dict(prm, lod=0.0)
    lut_t = torch.from_numpy(lut).cuda()
    out = amr.render(scene, cams, lut_t, dict(prm, persistent=1, tile_w=8, tile_h=8, blocks_per_cu=2),
                     d_cams=amr.camera_table(cams), d_queue=amr.queue_buffer(len(cams)))
    ref = amr.render(scene, cams, lut_t, prm)
    torch.cuda.synchronize()
    assert torch.equal(out["rgba"], ref["rgba"])


@pytest.mark.parametrize("lit", [False, True])
def test_vertex_adjoint_vs_oracle(gpu, lit):
    """The adjoint on vertex data: LUT (and light) gradients against the oracle's reverse mode."""
    import torch
    amr = gpu
    h = _hier("aligned0")
    lut = workloads.lut_bumps(np.random.default_rng(3), sigma_scale=6.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=lit, t_min=0.0, light=(0.3, 1.0, -0.6))
    cam = workloads.perspective_orbit(40, 32, 0.9, 0.25, radius=1.7)
    tree, scene = _setup(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    out, ck = amr.render_checkpointed(scene, cam, lut_t, prm)
    G = np.random.default_rng(4).normal(size=(40 * 32, 4))
    glut, glight = amr.render_backward(scene, cam, lut_t, prm, ck, torch.from_numpy(G.astype(np.float32)).cuda())
    ref_lut, ref_light = oracle.Oracle(h).grad(cam, prm, lut.astype(np.float64), G)
    got = glut.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref_lut) <= 1e-3 * np.abs(ref_lut) + 1e-5 * np.abs(ref_lut).max())
    if lit:
        gl = glight.cpu().numpy()
        assert np.all(np.abs(gl - ref_light) <= 1e-3 * np.abs(ref_light) + 1e-4 * np.abs(ref_light).max())


def test_vertex_point_light(gpu):
    """Secondary rays to a point light read vertex data through the same sampling."""
    amr = gpu
    h = _hier("tiny")
    lut = workloads.lut_bumps(np.random.default_rng(2), sigma_scale=6.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=2, light=(0.5, 0.45, 0.55), k_a=0.2, k_d=0.8)
    cam = workloads.perspective_orbit(24, 20, 0.7, 0.3, radius=1.8)
    tree, scene = _setup(amr, h)
    gout = _render(amr, scene, cam, lut, prm)
    ores = oracle.Oracle(h).render(cam, prm, lut)
    assert np.abs(gout["rgba"].cpu().numpy().reshape(-1, 4) - ores["rgba"]).max() <= TOL


def test_vertex_cosmology_full_size_sampled(gpu):
    """The 1024x1024 cosmology-like frame with vertex-centred data (2008 patches, the
    benchmark's launch configuration), lit: 1500 random pixels and a full row against the
    oracle, segment traces bit-exact."""
    import torch
    amr = gpu
    h, lut, cam, prm = workloads.cosmology_vertex_view(0)
    tree, scene = _setup(amr, h, layout=0)
    W, H = cam["width"], cam["height"]
    cap = 192
    out = _render(amr, scene, cam, lut, prm, trace_cap=cap)
    rng = np.random.default_rng(13)
    pix = np.concatenate([np.stack([rng.integers(0, W, 1500), rng.integers(0, H, 1500)], 1),
                          np.stack([np.arange(W), np.full(W, H // 2 + 3)], 1)]).astype(np.int32)
    idx = torch.from_numpy(pix[:, 1].astype(np.int64) * W + pix[:, 0]).cuda()
    rgba = out["rgba"].view(-1, 4)[idx].cpu().numpy().astype(np.float64)
    sub = dict(trace_raw=out["trace_raw"][idx], trace_n=out["trace_n"][idx])
    del out, scene
    ores = oracle.Oracle(h).render(cam, prm, lut, pixels=pix, trace_cap=cap)
    err = np.abs(rgba - ores["rgba"]).max()
    print("cosmology vertex view: %d pixels, max|err| = %.3g" % (len(pix), err))
    assert err <= TOL
    compare_traces(amr, sub, ores)
