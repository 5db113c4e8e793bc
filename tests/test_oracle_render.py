"""Pins of the oracle's rays, segments, sampling, lighting, compositing and gradients against
closed forms, a textbook routine (scipy trilinear on a single level), brute force and finite
differences.  None of the expected values below comes from the oracle's own formulas."""
import math

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle
import workloads
from oracle import Oracle, finest_boxes


def _f32(x):
    return float(np.float32(x))


def _inside(lo, hi, x):
    return bool(np.all(x >= lo) and np.all(x <= hi))


def _chord_faces(o, d, lo, hi):
    """Entry/exit parameters of the ray in the closed box [lo, hi], from the points where the
    line meets each of the six face rectangles (a face-by-face test, not the slab formula).
    Returns None on a miss."""
    ts = []
    for a in range(3):
        if d[a] == 0:
            continue
        for pl in (lo[a], hi[a]):
            t = (pl - o[a]) / d[a]
            x = o + t * d
            others = [b for b in range(3) if b != a]
            if all(lo[b] - 1e-12 <= x[b] <= hi[b] + 1e-12 for b in others):
                ts.append(t)
    inside_o = bool(np.all(o >= lo) and np.all(o <= hi))
    if inside_o:
        return 0.0, max(ts)
    ts = [t for t in ts if t >= 0]
    if len(ts) < 2:
        return None
    return min(ts), max(ts)


def test_rays_ortho_axis_exact():
    cam = workloads.ortho_axis_z(16, 8)
    for j in range(8):
        for i in range(16):
            o, d = oracle.ray(cam, i, j)
            assert np.array_equal(d, [0, 0, 1])
            assert np.array_equal(o, [(i + 0.5) / 16, 1 - (j + 0.5) / 8, -1.0])   # row 0 at the top


def test_rays_perspective_direction():
    cam = workloads.perspective_orbit(40, 30, 0.7, 0.3)
    t = cam["tan_half_fov"]
    for (i, j) in [(0, 0), (39, 29), (20, 15), (7, 22)]:
        o, d = oracle.ray(cam, i, j)
        assert np.array_equal(o, cam["eye"])
        assert abs(np.linalg.norm(d) - 1) < 1e-15
        s = (2 * i + 1) / 40 - 1
        tt = 1 - (2 * j + 1) / 30
        expect = cam["w"] + s * t * (40 / 30) * cam["u"] + tt * t * cam["v"]
        assert np.allclose(d, expect / np.linalg.norm(expect), rtol=0, atol=1e-15)


CAMS = {
    "ortho_z": workloads.ortho_axis_z(32, 32),
    "oblique": workloads.ortho_oblique(32, 32),
    "persp": workloads.perspective_orbit(32, 24, 0.4, 0.35, radius=1.6),
    "persp_inside": workloads.camera([0.3, 0.6, 0.4], *workloads.look_at([0.3, 0.6, 0.4], [0.9, 0.2, 0.8])[1:],
                                     24, 24, tan_half_fov=0.6),
}


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("cam_name", list(CAMS))
def test_constant_field_closed_form(cam_name, lit):
    """F = c everywhere => A = 1 - exp(-sigma(c) L) with L the chord length, C = rgb(c) A shade,
    shade = k_a when lit (the gradient vanishes exactly), 1 when unlit."""
    cv = 0.6
    h = workloads.tiny_samr(2).with_field(workloads.constant_field(cv))
    lut = workloads.lut_small_nested(3)
    prm = workloads.default_params(v_lo=0.0, v_hi=1.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75)
    cam = CAMS[cam_name]
    O = Oracle(h)
    res = O.render(cam, prm, lut)
    xs = np.arange(256) / 255.0
    u = float(np.float32(cv))
    sig = np.interp(u, xs, lut[:, 3].astype(np.float64))
    rgb = np.array([np.interp(u, xs, lut[:, c].astype(np.float64)) for c in range(3)])
    shade = 0.25 if lit else 1.0
    rgba = res["rgba"].reshape(cam["height"], cam["width"], 4)
    hits = 0
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            o, d = oracle.ray(cam, i, j)
            ch = _chord_faces(o, d, np.zeros(3), np.ones(3))
            L = 0.0 if ch is None else max(0.0, ch[1] - ch[0])
            A = 1 - math.exp(-sig * L)
            hits += L > 0
            assert abs(rgba[j, i, 3] - A) < 1e-12
            assert np.all(np.abs(rgba[j, i, :3] - rgb * A * shade) < 1e-12)
    assert hits > 0


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("uniform", [False, True])
@pytest.mark.parametrize("cam_name", ["ortho_z", "oblique", "persp"])
def test_linear_field_closed_form(cam_name, uniform, lit):
    """F = a.x + b with dyadic a, b (cell values exact in fp32), sigma linear in u, constant
    rgb: the midpoint rule integrates sigma exactly over every segment, so
    A = 1 - exp(-s L u(x_mid)); with eps_g = 0 the shade is k_a + k_d |a.l|/(|a||l|); C = rgb shade A.
    The clip box keeps samples and gradient taps >= 1.5 root cells from B's faces, where the
    ghost layers reproduce the linear field exactly."""
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    h = workloads.tiny_samr(4).with_field(workloads.linear_field(a, b))
    s = 255.0 / 64      # sigma_i = i / 64: exact in fp32
    lut = workloads.lut_linear_sigma(s, rgb=(0.75, 0.5, 0.25))
    m = 3.0 / 32
    prm = workloads.default_params(v_lo=0.0, v_hi=2.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75,
                                   eps_g=0.0, light=(1.0, 2.0, -0.5), uniform_step=uniform,
                                   clip_lo=(m, m, m), clip_hi=(1 - m, 1 - m, 1 - m))
    cam = CAMS[cam_name]
    O = Oracle(h)
    res = O.render(cam, prm, lut)
    l = np.array([_f32(x) for x in prm["light"]])
    shade = 0.25 + 0.75 * abs(a @ l) / (np.linalg.norm(a) * np.linalg.norm(l)) if lit else 1.0
    rgb = np.array([0.75, 0.5, 0.25])
    rgba = res["rgba"].reshape(cam["height"], cam["width"], 4)
    hits = 0
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            o, d = oracle.ray(cam, i, j)
            ch = _chord_faces(o, d, np.full(3, m), np.full(3, 1 - m))
            if ch is None or ch[1] - ch[0] <= 0:
                assert np.all(rgba[j, i] == 0)
                continue
            hits += 1
            L = ch[1] - ch[0]
            xm = o + 0.5 * (ch[0] + ch[1]) * d
            um = (a @ xm + b) / 2.0
            A = 1 - math.exp(-s * L * um)
            assert abs(rgba[j, i, 3] - A) < 1e-10, (i, j)
            assert np.all(np.abs(rgba[j, i, :3] - rgb * shade * A) < 1e-10)
    assert hits > 0


@pytest.mark.parametrize("interp", [0, 1])
@pytest.mark.parametrize("lit", [False, True])
def test_single_level_matches_scipy(lit, interp):
    """One subgrid: the tree is a single leaf and the render reduces to a uniform-grid raycast.
    Samples are evaluated with scipy's textbook interpolation (map_coordinates, order 1 for
    trilinear and order 0 for nearest cell, edge replication outside the grid), the LUT with
    np.interp and compositing with a running product."""
    h = workloads.single_level((12, 10, 8))
    lut = workloads.lut_bumps(np.random.default_rng(9), sigma_scale=8.0)
    cells = h.patches[0].cells.astype(np.float64)
    vmax = float(cells.max())
    prm = workloads.default_params(v_lo=0.0, v_hi=vmax, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75,
                                   eps_g=2.0 ** -10, light=(0.5, 1.0, 0.25), interp=interp)
    centre = h.origin + 0.5 * h.h0 * np.array([12, 10, 8])
    e, u, v, w = workloads.look_at(centre + np.array([0.3, 0.5, -0.9]), centre)
    cam = workloads.camera(e, u, v, w, 20, 16, tan_half_fov=0.35)
    O = Oracle(h)
    res = O.render(cam, prm, lut, trace_cap=4)
    hgrid = h.h0[0]
    Blo, Bhi = h.origin, h.origin + hgrid * np.array([12, 10, 8])
    xs = np.arange(256) / 255.0
    L64 = lut.astype(np.float64)
    l = np.array([_f32(x) for x in prm["light"]]); lhat = l / np.linalg.norm(l)

    def F(pts):
        q = (pts - h.origin) / hgrid - 0.5
        return map_coordinates(cells, [q[:, 2], q[:, 1], q[:, 0]], order=1 - interp, mode="nearest")

    for q in range(len(res["pixels"])):
        i, j = res["pixels"][q]
        o, d = oracle.ray(cam, i, j)
        if res["trace_n"][q] == 0:
            assert np.all(res["rgba"][q] == 0)
            continue
        assert res["trace_n"][q] == 1
        seg = res["trace"][q, 0]
        ta, tb = seg["ta"], seg["tb"]
        n = max(1, math.ceil((tb - ta) / (0.5 * hgrid) - 2.0 ** -20))
        assert seg["n"] == n
        delta = (tb - ta) / n
        t = ta + (np.arange(n) + 0.5) * delta
        pts = o[None, :] + t[:, None] * d[None, :]
        Fv = F(pts)
        uu = np.clip(Fv / _f32(vmax), 0, 1)
        rgb = np.stack([np.interp(uu, xs, L64[:, c]) for c in range(3)], 1)
        sig = np.interp(uu, xs, L64[:, 3])
        if lit:
            g = np.zeros((n, 3))
            for ax in range(3):
                off = np.zeros(3); off[ax] = hgrid
                pp, pm = pts + off, pts - off
                okp = np.all((pp >= Blo) & (pp <= Bhi), 1)
                okm = np.all((pm >= Blo) & (pm <= Bhi), 1)
                Fp, Fm = F(pp), F(pm)
                rng_ = _f32(vmax)
                g[:, ax] = np.where(okp & okm, (Fp - Fm) / (2 * rng_),
                                    np.where(okp, (Fp - Fv) / rng_, np.where(okm, (Fv - Fm) / rng_, 0.0)))
            eps = 2.0 ** -10
            shade = 0.25 + 0.75 * np.abs(g @ lhat) / np.sqrt((g * g).sum(1) + eps * eps)
        else:
            shade = np.ones(n)
        alpha = 1 - np.exp(-sig * delta)
        T = np.concatenate([[1.0], np.cumprod(1 - alpha)])
        C = (T[:-1, None] * alpha[:, None] * shade[:, None] * rgb).sum(0)
        assert np.all(np.abs(res["rgba"][q, :3] - C) < 1e-12)
        assert abs(res["rgba"][q, 3] - (1 - T[-1])) < 1e-12


def _brute_check_segments(h, O, cam, prm, pixels):
    res = O.render(cam, prm, workloads.lut_small_nested(0), pixels=pixels, trace_cap=512)
    boxes = finest_boxes(h)
    L = O.tree.leaf_array()
    L_lo = h.origin + L[:, 0:3] * (h.h0 / h.refine ** (h.nlevels - 1))
    L_hi = h.origin + L[:, 3:6] * (h.h0 / h.refine ** (h.nlevels - 1))
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    P_lo = h.origin + boxes[:, 1:4] * hf
    P_hi = h.origin + boxes[:, 4:7] * hf
    checked = 0
    for q in range(len(pixels)):
        if res["flags"][q]:
            continue
        i, j = pixels[q]
        o, d = oracle.ray(cam, i, j)
        nseg = res["trace_n"][q]
        assert nseg <= 512
        segs = res["trace"][q, :nseg]
        if nseg == 0:
            continue
        # segments tile the chord: consecutive, ending at the box exit
        ch = _chord_faces(o, d, np.asarray(prm["clip_lo"]).clip(0, 1), np.asarray(prm["clip_hi"]).clip(0, 1))
        assert abs(segs[0]["ta"] - ch[0]) < 1e-12 and abs(segs[-1]["tb"] - ch[1]) < 1e-12
        assert np.all(segs["ta"][1:] == segs["tb"][:-1])
        for s in segs:
            if s["patch"] < 0:      # transparent leaf: no data anywhere along it
                x = o + 0.5 * (s["ta"] + s["tb"]) * d
                assert not np.any(np.all((P_lo <= x) & (x < P_hi), 1)) and s["n"] == 0
                continue
            lev = h.nlevels - 1 if prm["uniform_step"] else s["level"]
            step = _f32(prm["step_frac"]) * h.h0.min() / h.refine ** lev
            ln = s["tb"] - s["ta"]
            # n is the smallest count whose step does not exceed the nominal one (2^-20 slack)
            assert ln / s["n"] <= step * (1 + 2.0 ** -19)
            assert s["n"] == 1 or ln / (s["n"] - 1) > step * (1 - 2.0 ** -19)
            dl = ln / s["n"]
            for k in range(s["n"]):
                x = o + (s["ta"] + (k + 0.5) * dl) * d
                inl = np.flatnonzero(np.all((L_lo <= x) & (x < L_hi), 1))
                assert list(inl) == [s["leaf"]]
                inp = np.flatnonzero(np.all((P_lo <= x) & (x < P_hi), 1))
                assert s["patch"] == inp[np.argmax(boxes[inp, 0])]
                checked += 1
    return checked


@pytest.mark.parametrize("uniform", [False, True])
@pytest.mark.parametrize("cam_idx", [0, 1])
def test_segment_ids_brute_force_small_nested(cam_idx, uniform):
    h = workloads.tiny_samr(0)
    O = Oracle(h)
    cam = workloads.small_nested_cameras(64, 64)[cam_idx]
    prm = workloads.default_params(uniform_step=uniform, t_min=0.0)
    rng = np.random.default_rng(cam_idx)
    pix = np.stack([rng.integers(0, 64, 150), rng.integers(0, 64, 150)], 1).astype(np.int32)
    assert _brute_check_segments(h, O, cam, prm, pix) > 1000


@pytest.mark.parametrize("seed", range(6))
def test_segment_ids_brute_force_random(seed):
    h = workloads.random_tiny(seed, multi_root=(seed % 2 == 1))
    O = Oracle(h)
    cam = workloads.perspective_orbit(24, 24, 0.3 + seed, 0.2 * seed - 0.4, radius=1.8)
    m = 0.05 * (seed % 3)
    prm = workloads.default_params(t_min=0.0, clip_lo=(m, 0, m), clip_hi=(1, 1 - m, 1))
    rng = np.random.default_rng(seed)
    pix = np.stack([rng.integers(0, 24, 100), rng.integers(0, 24, 100)], 1).astype(np.int32)
    _brute_check_segments(h, O, cam, prm, pix)


def test_early_termination_bound():
    h, lut, cams, prm = workloads.small_nested(0)
    lut = lut.copy(); lut[:, 3] *= 20
    O = Oracle(h)
    for lit in (False, True):
        p0 = dict(prm, t_min=0.0, lighting=lit)
        p1 = dict(prm, t_min=1e-3, lighting=lit)
        r0, r1 = O.render(cams[1], p0, lut), O.render(cams[1], p1, lut)
        emax = float((lut[:, :3].max()) * (1.0 if not lit else 1.0))
        tm = _f32(1e-3)
        assert np.all(np.abs(r0["rgba"][:, :3] - r1["rgba"][:, :3]) <= tm * emax + 1e-15)
        assert np.all(np.abs(r0["rgba"][:, 3] - r1["rgba"][:, 3]) <= tm + 1e-15)
        assert (r1["nsamp"] < r0["nsamp"]).sum() > 100


def test_shuffle_invariance_image():
    h, lut, cams, prm = workloads.small_nested(0)
    hs = h.shuffled(3)
    r1 = Oracle(h).render(cams[1], dict(prm, lighting=True), lut)
    r2 = Oracle(hs).render(cams[1], dict(prm, lighting=True), lut)
    assert np.array_equal(r1["rgba"], r2["rgba"])


@pytest.mark.parametrize("lit", [False, True])
def test_gradient_vs_finite_difference(lit):
    """Reverse-mode dL/dLUT and dL/d(light, k_a, k_d) against FP64 central differences."""
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, t_min=0.0, lighting=lit, light=(0.3, 1.0, -0.6), k_a=0.3, k_d=0.7)
    O = Oracle(h)
    cam = workloads.small_nested_cameras(48, 48)[1]
    rng = np.random.default_rng(4)
    pix = np.stack([rng.integers(0, 48, 60), rng.integers(0, 48, 60)], 1).astype(np.int32)
    W = rng.normal(size=(len(pix), 4))
    lut64 = lut.astype(np.float64)
    glut, glight = O.grad(cam, prm, lut64, W, pixels=pix, f32_params=False)

    def loss(l64, p):
        return float((O.render_lut64(cam, p, l64, pixels=pix, f32_params=False) * W).sum())
    gmax = np.abs(glut).max()
    idx = np.argwhere(np.abs(glut) > 1e-3 * gmax)
    sel = idx[rng.choice(len(idx), size=min(40, len(idx)), replace=False)]
    hstep = 1e-6
    for (e, c) in sel:
        lp = lut64.copy(); lp[e, c] += hstep
        lm = lut64.copy(); lm[e, c] -= hstep
        fd = (loss(lp, prm) - loss(lm, prm)) / (2 * hstep)
        assert abs(fd - glut[e, c]) <= 1e-6 * max(abs(glut[e, c]), 1e-2 * gmax), (e, c, fd, glut[e, c])
    # untouched entries have exactly zero gradient
    assert np.count_nonzero(glut) < glut.size
    if lit:
        for k, key in enumerate(["lx", "ly", "lz", "k_a", "k_d"]):
            def with_(delta):
                p = dict(prm)
                if k < 3:
                    l = list(p["light"]); l[k] += delta; p["light"] = tuple(l)
                else:
                    p[key] += delta
                return p
            fd = (loss(lut64, with_(hstep)) - loss(lut64, with_(-hstep))) / (2 * hstep)
            assert abs(fd - glight[k]) <= 1e-6 * max(1.0, abs(glight[k])), (key, fd, glight[k])
    else:
        assert np.all(glight == 0)


def test_constant_field_sigma_derivative():
    """Constant field: dA/dsigma = L exp(-sigma L); the LUT entries bracketing u share it with
    weights (1-f, f)."""
    cv = 0.5
    h = workloads.tiny_samr(2).with_field(workloads.constant_field(cv))
    lut = workloads.lut_small_nested(3).astype(np.float64)
    prm = workloads.default_params(v_lo=0.0, v_hi=1.0, t_min=0.0)
    cam = workloads.ortho_axis_z(8, 8)
    O = Oracle(h)
    W = np.zeros((64, 4)); W[:, 3] = 1.0       # L = sum of alpha over pixels
    glut, _ = O.grad(cam, prm, lut, W)
    x = 255 * float(np.float32(cv)); i0 = int(math.floor(x)); f = x - i0
    sig = lut[i0, 3] + f * (lut[i0 + 1, 3] - lut[i0, 3])
    dA = 64 * 1.0 * math.exp(-sig * 1.0)       # chord length 1 for every pixel
    assert abs(glut[i0, 3] - (1 - f) * dA) < 1e-12
    assert abs(glut[i0 + 1, 3] - f * dA) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_nearest_field_brute_force(seed):
    """Nearest-cell field on random hierarchies: at random points (and points on cell faces) the
    value is the cell of the finest patch holding the point, found by brute force over patches
    in integer finest-level coordinates."""
    h = workloads.random_tiny(seed, multi_root=(seed % 2 == 1))
    O = Oracle(h)
    fb = oracle.finest_boxes(h)
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    Blo = fb[fb[:, 0] == 0][:, 1:4].min(0)
    Bhi = fb[fb[:, 0] == 0][:, 4:7].max(0)
    rng = np.random.default_rng(seed)
    checked = 0
    for trial in range(400):
        g = Blo + rng.random(3) * (Bhi - Blo)
        if trial % 4 == 0:
            g = np.floor(g)                  # on finest-cell faces
        x = h.origin + g * hf
        best = -1
        for p, row in enumerate(fb):
            lo, hi = row[1:4], row[4:7]
            inside = np.all((g >= lo) & ((g < hi) | ((g == hi) & (hi == Bhi))))
            if inside and (best < 0 or row[0] > fb[best][0]):
                best = p
        v = O.field(x, interp=1)
        if best < 0:
            assert v is None
            continue
        P = h.patches[best]
        S = h.refine ** (h.nlevels - 1 - P.level)
        idx = np.clip(np.floor((g - fb[best][1:4]) / S).astype(np.int64), 0, np.array(P.cells.shape[::-1]) - 1)
        assert v == float(P.cells[idx[2], idx[1], idx[0]])
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("lod", [0.0, 1.5, 3.0, 1e6])
@pytest.mark.parametrize("cam_name", ["ortho_z", "oblique", "persp"])
def test_lod_linear_closed_form(cam_name, lod, lit):
    """Level of detail on a linear field: a segment rendered from a coarse cover patch samples
    the same linear function (its cells hold the same exact values), and the midpoint rule
    integrates linear opacity exactly on any segmentation, so every pixel still obeys
    A = 1 - exp(-s L u(x_mid)) and C = rgb shade A, whatever the level-of-detail cut."""
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    h = workloads.lod_blocks(1, field=workloads.linear_field(a, b))
    s = 255.0 / 64
    lut = workloads.lut_linear_sigma(s, rgb=(0.75, 0.5, 0.25))
    m = 0.125
    prm = workloads.default_params(v_lo=0.0, v_hi=2.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75,
                                   eps_g=0.0, light=(1.0, 2.0, -0.5), lod=lod,
                                   clip_lo=(m, m, m), clip_hi=(1 - m, 1 - m, 1 - m))
    cam = CAMS[cam_name]
    O = Oracle(h)
    res = O.render(cam, prm, lut, trace_cap=64)
    nl = len(O.tree.leaves)
    l = np.array([_f32(x) for x in prm["light"]])
    shade = 0.25 + 0.75 * abs(a @ l) / (np.linalg.norm(a) * np.linalg.norm(l)) if lit else 1.0
    rgb = np.array([0.75, 0.5, 0.25])
    rgba = res["rgba"].reshape(cam["height"], cam["width"], 4)
    lod_segs = 0
    for j in range(cam["height"]):
        for i in range(cam["width"]):
            q = j * cam["width"] + i
            tr = res["trace"][q, :res["trace_n"][q]]
            lod_segs += int(np.sum(tr["leaf"] >= nl))
            o, d = oracle.ray(cam, i, j)
            ch = _chord_faces(o, d, np.full(3, m), np.full(3, 1 - m))
            if ch is None or ch[1] - ch[0] <= 0:
                continue
            xm = o + 0.5 * (ch[0] + ch[1]) * d
            A = 1 - math.exp(-s * (ch[1] - ch[0]) * (a @ xm + b) / 2.0)
            assert abs(rgba[j, i, 3] - A) < 1e-10
            assert np.all(np.abs(rgba[j, i, :3] - rgb * shade * A) < 1e-10)
    if lod >= 3.0:
        assert lod_segs > 0
    if lod == 0.0:
        assert lod_segs == 0


@pytest.mark.parametrize("seed", range(4))
def test_lod_segments_structure(seed):
    """With an unbounded threshold every kind-(a) node the ray enters away from the eye is cut:
    each ray's segments tile its chord; a level-of-detail segment spans the ray's whole
    intersection with an outermost kind-(a) node (one with no kind-(a) ancestor, found here by
    box containment), is reported with that node's id and its cover patch and level; every
    other segment is the plain render's leaf segment outside those nodes."""
    h = workloads.lod_blocks(seed)
    lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=4.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    cam = workloads.perspective_orbit(20, 16, 0.7 + seed, 0.3 - 0.2 * seed, radius=1.7)
    O = Oracle(h)
    nl = len(O.tree.leaves)
    an = O._anodes
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    lo_w, hi_w = an[:, 0:3] * hf + h.origin, an[:, 3:6] * hf + h.origin
    outer = [k for k in range(len(an)) if not any(
        j != k and np.all(an[j, 0:3] <= an[k, 0:3]) and np.all(an[j, 3:6] >= an[k, 3:6]) for j in range(len(an)))]
    base = O.render(cam, workloads.default_params(v_hi=vmax, t_min=0.0), lut, trace_cap=128)
    res = O.render(cam, workloads.default_params(v_hi=vmax, t_min=0.0, lod=1e30), lut, trace_cap=128)
    cut = 0
    for q in range(len(res["pixels"])):
        tr = res["trace"][q, :res["trace_n"][q]]
        tb0 = base["trace"][q, :base["trace_n"][q]]
        if len(tr) == 0:
            assert len(tb0) == 0
            continue
        assert tr["ta"][0] == tb0["ta"][0] and tr["tb"][-1] == tb0["tb"][-1]
        assert np.all(tr["tb"][:-1] == tr["ta"][1:])
        i, j = res["pixels"][q]
        o, d = oracle.ray(cam, i, j)
        for sg in tr:
            xm = o + 0.5 * (sg["ta"] + sg["tb"]) * d
            inside = [k for k in outer if np.all(xm >= lo_w[k]) and np.all(xm < hi_w[k])]
            if sg["leaf"] >= nl:
                k = sg["leaf"] - nl
                assert inside == [k]
                assert sg["patch"] == an[k, 6] and sg["level"] == an[k, 7]
                ch = _chord_faces(o, d, lo_w[k], hi_w[k])
                assert abs(max(ch[0], tr["ta"][0]) - sg["ta"]) < 1e-12 and abs(min(ch[1], tr["tb"][-1]) - sg["tb"]) < 1e-12
                cut += 1
            else:
                assert inside == []
                hit = (tb0["ta"] == sg["ta"]) & (tb0["tb"] == sg["tb"]) & (tb0["leaf"] == sg["leaf"])
                assert hit.sum() == 1
    assert cut > 0


@pytest.mark.parametrize("light", [(0.5, 0.45, 0.55), (1.7, -0.4, 0.3)])
@pytest.mark.parametrize("cam_name", ["ortho_z", "persp"])
def test_point_light_constant_field(cam_name, light):
    """Point-light secondary rays (lighting = 2) on one subgrid with a constant field: every
    sample's light transmittance is exp(-sigma |[x, p_L] in B|), the length taken from a
    face-by-face chord of the box; the primary composite is then a running product over the
    evenly spaced primary samples."""
    h = workloads.single_level((12, 10, 8)).with_field(workloads.constant_field(0.5))
    sig = 3.0
    lut = workloads.lut_constant(rgb=(0.8, 0.5, 0.2), sigma=sig)
    prm = workloads.default_params(v_lo=0.0, v_hi=1.0, t_min=0.0, lighting=2, light=light, k_a=0.25, k_d=0.75)
    cam = CAMS[cam_name]
    O = Oracle(h)
    res = O.render(cam, prm, lut, trace_cap=4)
    hgrid = h.h0[0]
    Blo, Bhi = h.origin, h.origin + hgrid * np.array([12, 10, 8])
    pl = np.array([_f32(v) for v in light])
    rgb = np.array([_f32(0.8), _f32(0.5), _f32(0.2)])     # the LUT holds fp32 values
    checked = 0
    for q in range(len(res["pixels"])):
        if res["trace_n"][q] == 0:
            continue
        i, j = res["pixels"][q]
        o, d = oracle.ray(cam, i, j)
        seg = res["trace"][q, 0]
        n = seg["n"]
        delta = (seg["tb"] - seg["ta"]) / n
        alpha = 1 - math.exp(-sig * delta)
        C = np.zeros(3); T = 1.0
        for k in range(n):
            x = o + (seg["ta"] + (k + 0.5) * delta) * d
            v = pl - x
            dist = np.linalg.norm(v)
            ch = _chord_faces(x, v / dist, Blo, Bhi)
            L = 0.0 if ch is None else max(0.0, min(ch[1], dist) - max(ch[0], 0.0))
            shade = 0.25 + 0.75 * math.exp(-sig * L)
            C += T * alpha * shade * rgb
            T *= 1 - alpha
        assert np.all(np.abs(res["rgba"][q, :3] - C) < 1e-10), q
        assert abs(res["rgba"][q, 3] - (1 - T)) < 1e-12
        checked += 1
    assert checked > 50

