"""Pins of the oracle's vertex-centred data mode (Section 5: texels on the grid vertices,
trilinear interpolation, shared boundary samples, dangling nodes replaced by the interpolated
value of the abutting coarse brick).  Checked against a textbook interpolator, hand-derived
dangling-node values, linear fields (reproduced exactly everywhere, B's faces included),
continuity across coarse-fine faces and a closed-form render."""
import math

import numpy as np
import pytest
from scipy.interpolate import RegularGridInterpolator

import oracle
import workloads
from oracle import Oracle
from workloads import Hierarchy, Patch


def _vertex_grid_interp(h, p):
    """scipy's trilinear interpolant of patch p's raw vertex samples (points as (x, y, z))."""
    x, y, z = h.vertex_positions(p)
    f = RegularGridInterpolator((z, y, x), p.cells.astype(np.float64), method="linear")
    return lambda pts: f(np.asarray(pts)[..., ::-1])


def _world_box(h, p):
    hl = h.h0 / float(h.refine) ** p.level
    return h.origin + p.lo * hl, h.origin + (p.lo + p.dims) * hl


def test_single_patch_matches_scipy():
    """One subgrid: F is the trilinear interpolant of the vertex samples on the closed box,
    faces and corners included."""
    h0 = workloads.single_level((12, 10, 8))
    fn = workloads.gaussian_sum_field(np.random.default_rng(4), n=5, smin=0.1, smax=0.3)
    h = h0.with_vertex_field(fn)
    O = Oracle(h)
    ref = _vertex_grid_interp(h, h.patches[0])
    lo, hi = _world_box(h, h.patches[0])
    rng = np.random.default_rng(1)
    pts = lo + rng.random((3000, 3)) * (hi - lo)
    # points on faces and at the corners too
    pts[:200, 0] = lo[0]
    pts[200:400, 1] = hi[1]
    pts[400:408] = [[(lo, hi)[(c >> a) & 1][a] for a in range(3)] for c in range(8)]
    want = ref(pts)
    got = np.array([O.field(x) for x in pts])
    assert np.max(np.abs(got - want)) < 1e-12
    # no dangling nodes in a single subgrid: the samples are the input
    assert np.array_equal(O.vertex_values(0), h.patches[0].cells.astype(np.float64))


def _corner_pair(seed):
    """Level 0: 2^3 cells of size 1/2 on [0,1]^3; level 1: 2^3 cells of size 1/4 filling the
    level-0 cell at the origin.  Integer samples so every expected value is exact."""
    rng = np.random.default_rng(seed)
    v0 = rng.integers(-50, 50, (3, 3, 3)).astype(np.float32)
    v1 = rng.integers(-50, 50, (3, 3, 3)).astype(np.float32)
    ps = [Patch(0, np.zeros(3, np.int64), np.full(3, 2, np.int64), v0),
          Patch(1, np.zeros(3, np.int64), np.full(3, 2, np.int64), v1)]
    return Hierarchy(np.zeros(3), np.full(3, 0.5), 2, 2, ps, "vertex"), v0, v1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dangling_nodes_hand_values(seed):
    """Fine vertices on the fine patch's faces at 1/2 (which abut level-0 data) take the
    level-0 interpolant: a vertex at an odd fine index along an axis sits halfway between two
    coarse vertices, so its value is the mean over 1, 2 or 4 coarse samples (coincident
    vertices take the coarse sample itself).  Fine vertices whose other side is outside B, and
    all interior and level-0 samples, keep their input."""
    h, v0, v1 = _corner_pair(seed)
    O = Oracle(h)
    fixed1 = O.vertex_values(1)
    assert np.array_equal(O.vertex_values(0), v0.astype(np.float64))
    for k in range(3):
        for j in range(3):
            for i in range(3):
                idx = (i, j, k)
                if 2 in idx:
                    # coarse position idx / 2 per axis: even -> one sample, odd -> mean of two
                    ax = [[(c // 2, 1.0)] if c % 2 == 0 else [((c - 1) // 2, 0.5), ((c + 1) // 2, 0.5)] for c in idx]
                    want = sum(wx * wy * wz * float(v0[cz, cy, cx])
                               for cx, wx in ax[0] for cy, wy in ax[1] for cz, wz in ax[2])
                else:
                    want = float(v1[k, j, i])
                assert fixed1[k, j, i] == want, (idx, fixed1[k, j, i], want)
    # just inside the fine patch, at the middle of a fine cell face on x = 1/2, the fine field
    # equals the level-0 interpolant there (coarse position (1, 1/4, 1/4))
    x = np.array([0.5 - 2.0 ** -30, 0.125, 0.125])
    assert O.locate(x) == 1
    want = 0.5625 * v0[0, 0, 1] + 0.1875 * v0[0, 1, 1] + 0.1875 * v0[1, 0, 1] + 0.0625 * v0[1, 1, 1]
    assert abs(O.field(x) - float(want)) < 1e-5


def _linear_vertex(h, a, b):
    return h.with_vertex_field(workloads.linear_field(a, b))


@pytest.mark.parametrize("name", ["tiny", "random0", "random1", "random2", "aligned3", "lod"])
def test_linear_field_exact_everywhere(name):
    """A linear field sampled at the vertices is its own trilinear interpolant on every cell,
    so the dangling-node fix must leave every sample as it was and F must equal the linear
    function at every point of B, including points on B's faces (no ghost layer involved)."""
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    if name == "tiny":
        h0 = workloads.tiny_samr(3)
    elif name == "lod":
        h0 = workloads.lod_blocks(1)
    elif name.startswith("aligned"):
        h0 = workloads.random_tiny(int(name[-1]), root_aligned=True)
    else:
        h0 = workloads.random_tiny(int(name[-1]))
    h = _linear_vertex(h0, a, b)
    O = Oracle(h)
    for pi, p in enumerate(h.patches):
        assert np.max(np.abs(O.vertex_values(pi) - p.cells.astype(np.float64))) < 1e-6, pi
    rng = np.random.default_rng(5)
    lo = h.origin.copy()
    hi = h.origin + h.h0 * np.max([p.hi for p in h.patches if p.level == 0], axis=0)
    pts = lo + rng.random((3000, 3)) * (hi - lo)
    pts[:300, 2] = hi[2]
    pts[300:600, 0] = lo[0]
    for x in pts:
        v = O.field(x)
        assert v is not None
        assert abs(v - (a @ x + b)) < 2e-6


def _face_points(h, rng, per_face=40):
    """Random points on every patch face (world), with the face axis and normal sign."""
    out = []
    for p in h.patches:
        lo, hi = _world_box(h, p)
        for a in range(3):
            for side in range(2):
                pts = lo + rng.random((per_face, 3)) * (hi - lo)
                pts[:, a] = (lo, hi)[side][a]
                out += [(x, a) for x in pts]
    return out


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_continuity_across_coarse_fine_faces(seed):
    """With every box a union of root cells, each fine cell face on an interface lies inside a
    coarse cell face and all of its vertices take the coarse interpolant, so F is continuous:
    the values just before and just after the face agree to O(eps).  Without the fix (the fine
    patch's raw samples) they do not, which keeps the pin meaningful."""
    h = workloads.random_tiny(seed, root_aligned=True).with_vertex_field(
        workloads.gaussian_sum_field(np.random.default_rng(seed + 11), n=4, smin=0.08, smax=0.2))
    O = Oracle(h)
    rng = np.random.default_rng(seed)
    eps = 1e-9
    n_if, worst, raw_gap = 0, 0.0, 0.0
    raw = {pi: _vertex_grid_interp(h, p) for pi, p in enumerate(h.patches)}
    for x, a in _face_points(h, rng):
        e = np.zeros(3); e[a] = eps
        qp, qm = O.locate(x + e), O.locate(x - e)
        if qp < 0 or qm < 0:
            continue
        lp, lm = h.patches[qp].level, h.patches[qm].level
        if lp == lm:
            continue
        n_if += 1
        worst = max(worst, abs(O.field(x + e) - O.field(x - e)))
        fine, coarse_side = (qp, x - e) if lp > lm else (qm, x + e)
        fine_pt = x + e if lp > lm else x - e
        raw_gap = max(raw_gap, abs(float(raw[fine](fine_pt[None])[0]) - O.field(coarse_side)))
    assert n_if > 50
    assert worst < 1e-7, worst
    assert raw_gap > 1e-4, raw_gap


def test_nearest_rejected_for_vertex_data():
    h = workloads.tiny_samr(0).with_vertex_field(workloads.constant_field(0.5))
    O = Oracle(h)
    with pytest.raises(ValueError):
        O.field([0.5, 0.5, 0.5], interp=1)
    with pytest.raises(ValueError):
        O.render(workloads.ortho_axis_z(4, 4), workloads.default_params(interp=1), workloads.lut_constant())


def test_sample_shape_checked():
    h = workloads.tiny_samr(0)               # cell-centred arrays
    bad = Hierarchy(h.origin, h.h0, h.refine, h.nlevels, h.patches, "vertex")
    with pytest.raises(ValueError):
        Oracle(bad)


def _chord(o, d, lo, hi):
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] <= o[a] <= hi[a]):
                return None
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return (t0, t1) if t1 > t0 else None


@pytest.mark.parametrize("lit", [False, True])
@pytest.mark.parametrize("cam", ["ortho_z", "oblique", "persp"])
def test_linear_field_render_closed_form(cam, lit):
    """Linear F, sigma linear in u, constant rgb: the midpoint rule integrates sigma exactly on
    every segment, A = 1 - exp(-s L u(x_mid)) with L the whole chord through B (vertex data
    needs no clip margin), and with eps_g = 0 the shade is k_a + k_d |a.l| / (|a| |l|) (a tap
    beyond B gives a one-sided difference, also exact)."""
    cams = {"ortho_z": workloads.ortho_axis_z(24, 24), "oblique": workloads.ortho_oblique(24, 24),
            "persp": workloads.perspective_orbit(24, 20, 0.4, 0.35, radius=1.6)}
    a = np.array([0.75, -0.375, 0.25]); b = 0.5
    h = _linear_vertex(workloads.tiny_samr(4), a, b)
    s = 255.0 / 64
    lut = workloads.lut_linear_sigma(s, rgb=(0.75, 0.5, 0.25))
    prm = workloads.default_params(v_lo=0.0, v_hi=2.0, t_min=0.0, lighting=lit, k_a=0.25, k_d=0.75,
                                   eps_g=0.0, light=(1.0, 2.0, -0.5))
    c = cams[cam]
    res = Oracle(h).render(c, prm, lut)
    l = np.array([float(np.float32(x)) for x in prm["light"]])
    shade = 0.25 + 0.75 * abs(a @ l) / (np.linalg.norm(a) * np.linalg.norm(l)) if lit else 1.0
    rgb = np.array([0.75, 0.5, 0.25])
    rgba = res["rgba"].reshape(c["height"], c["width"], 4)
    hits = 0
    for j in range(c["height"]):
        for i in range(c["width"]):
            o, d = oracle.ray(c, i, j)
            ch = _chord(o, d, np.zeros(3), np.ones(3))
            if ch is None:
                assert np.all(rgba[j, i] == 0)
                continue
            hits += 1
            L = ch[1] - ch[0]
            um = (a @ (o + 0.5 * (ch[0] + ch[1]) * d) + b) / 2.0
            A = 1 - math.exp(-s * L * um)
            assert abs(rgba[j, i, 3] - A) < 1e-10, (i, j)
            assert np.all(np.abs(rgba[j, i, :3] - rgb * shade * A) < 1e-10)
    assert hits > 0
