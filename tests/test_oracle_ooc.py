"""Pins of the oracle's out-of-core mode (per-subgrid storage, Sections 5.2 and 7): with a
subset of the patches present, every leaf keeps its place in the tree and is drawn from the
finest present patch holding its whole box.  Checked against brute-force holders, a
closed-form composite over piecewise-constant data, and the unrestricted oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle import Oracle


def _mask(h, seed, keep=0.5):
    rng = np.random.default_rng(seed)
    m = rng.random(len(h.patches)) < keep
    for i, p in enumerate(h.patches):
        if p.level == 0:
            m[i] = True
    return m


def _holder(boxes, mask, lo, hi):
    """Finest present patch whose box holds [lo, hi) (brute force); -1 if none."""
    best = -1
    for q in range(len(boxes)):
        if mask[q] and np.all(boxes[q, 1:4] <= lo) and np.all(hi <= boxes[q, 4:7]):
            if best < 0 or boxes[q, 0] > boxes[best, 0]:
                best = q
    return best


def test_all_present_is_the_plain_oracle():
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=True)
    a = Oracle(h).render(cams[1], prm, lut, trace_cap=64)
    b = Oracle(h, resident=np.ones(len(h.patches), bool)).render(cams[1], prm, lut, trace_cap=64)
    assert np.array_equal(a["rgba"], b["rgba"])
    assert np.array_equal(a["trace"], b["trace"])


def _nested_lod(seed):
    """Level-of-detail geometry (level-2 patches inside a level-1 patch) with every level-2
    patch absent: their leaves must fall back to the level-1 patch, not to the root."""
    h = workloads.lod_blocks(seed)
    return h, np.array([p.level < 2 for p in h.patches])


@pytest.mark.parametrize("seed", list(range(6)) + [10, 11])
def test_segments_take_the_finest_present_holder(seed):
    """Each traced segment names the brute-force holder of its leaf's box, that patch's level,
    and the sample count of that level's step; the segment bounds are those of the full tree."""
    if seed >= 10:
        h, mask = _nested_lod(seed - 10)
    else:
        h = workloads.random_tiny(seed, multi_root=(seed % 2 == 1), max_patches=8)
        mask = _mask(h, seed)
    boxes = oracle.finest_boxes(h)
    O = Oracle(h, resident=mask)
    full = Oracle(h)
    leaves = O.tree.leaf_array()
    prm = workloads.default_params(v_hi=1.0, t_min=0.0)
    cam = workloads.perspective_orbit(20, 16, 0.5 + seed, 0.3, radius=1.7)
    r = O.render(cam, prm, workloads.lut_constant(sigma=0.5), trace_cap=128)
    f = full.render(cam, prm, workloads.lut_constant(sigma=0.5), trace_cap=128)
    hs = min(h.h0) / h.refine ** np.arange(h.nlevels)
    checked = 0
    for q in range(len(r["trace_n"])):
        assert r["trace_n"][q] == f["trace_n"][q]
        for s, sf in zip(r["trace"][q, :r["trace_n"][q]], f["trace"][q, :f["trace_n"][q]]):
            assert s["leaf"] == sf["leaf"] and s["ta"] == sf["ta"] and s["tb"] == sf["tb"]
            L = leaves[s["leaf"]]
            want = -1 if L[6] < 0 else _holder(boxes, mask, L[0:3], L[3:6])
            assert s["patch"] == want
            if want >= 0:
                lev = h.patches[want].level
                if seed >= 10 and h.patches[L[6]].level == 2:
                    assert lev == 1
                assert s["level"] == lev
                n = max(1, math.ceil((s["tb"] - s["ta"]) / (prm["step_frac"] * hs[lev]) - 2.0 ** -20))
                assert s["n"] == n
                checked += 1
    assert checked > 50


@pytest.mark.parametrize("seed", range(4))
def test_piecewise_constant_closed_form(seed):
    """Each patch holds one constant c_p (cell values, nearest-cell sampling, unlit): a segment
    of length L drawn from holder p contributes rgb(c_p) (T_in - T_in e^{-sigma(c_p) L}), so the
    pixel is a closed-form product/sum over the traced segments with brute-force holders."""
    h0 = workloads.random_tiny(seed + 10, max_patches=8)
    cs = np.linspace(0.1, 0.9, len(h0.patches))
    ps = [workloads.Patch(p.level, p.lo, p.dims, np.full(p.cells.shape, cs[i], np.float32))
          for i, p in enumerate(h0.patches)]
    h = workloads.Hierarchy(h0.origin, h0.h0, h0.refine, h0.nlevels, ps)
    mask = _mask(h, seed + 3)
    boxes = oracle.finest_boxes(h)
    lut = workloads.lut_bumps(np.random.default_rng(seed), sigma_scale=4.0)
    prm = workloads.default_params(v_hi=1.0, t_min=0.0, interp=1)
    cam = workloads.ortho_oblique(18, 18)
    O = Oracle(h, resident=mask)
    r = O.render(cam, prm, lut, trace_cap=128)
    leaves = O.tree.leaf_array()
    xs = np.arange(256) / 255.0
    lut64 = lut.astype(np.float64)
    for q in range(len(r["trace_n"])):
        T, C = 1.0, np.zeros(3)
        for s in r["trace"][q, :r["trace_n"][q]]:
            L = leaves[s["leaf"]]
            p = -1 if L[6] < 0 else _holder(boxes, mask, L[0:3], L[3:6])
            if p < 0:
                continue
            u = float(np.float32(cs[p]))
            sig = np.interp(u, xs, lut64[:, 3])
            rgb = np.array([np.interp(u, xs, lut64[:, c]) for c in range(3)])
            Tn = T * math.exp(-sig * (s["tb"] - s["ta"]))
            C += rgb * (T - Tn)
            T = Tn
        assert abs(r["rgba"][q, 3] - (1 - T)) < 1e-12
        assert np.all(np.abs(r["rgba"][q, :3] - C) < 1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_field_reads_the_finest_present_patch(seed):
    """Gradient taps read F at the finest present patch holding the point (brute force over the
    patch boxes, half-open)."""
    h = workloads.random_tiny(seed + 20, max_patches=8)
    mask = _mask(h, seed)
    O = Oracle(h, resident=mask)
    full = Oracle(h)
    rng = np.random.default_rng(seed)
    boxes = oracle.finest_boxes(h)
    hf = h.h0 / h.refine ** (h.nlevels - 1)
    for x in rng.random((800, 3)):
        g = np.floor((x - h.origin) / hf).astype(np.int64)
        p = _holder(boxes, mask, g, g + 1)
        assert O.locate(x) == p
        assert O.locate(x, brute=True) == p
        if p >= 0 and full.locate(x) == p:
            assert O.field(x) == full.field(x)
