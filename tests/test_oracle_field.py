"""Pins of the oracle's field: patch lookup, ghost cells (g1-g4) and trilinear interpolation,
against closed forms (constant and linear fields are reproduced exactly by trilinear
interpolation of cell-centred samples) and brute force."""
import numpy as np
import pytest

import workloads
from oracle import Oracle, finest_boxes


def _world_box(h, p):
    hl = h.h0 / float(h.refine) ** p.level
    return h.origin + p.lo * hl, h.origin + (p.lo + p.dims) * hl


@pytest.mark.parametrize("seed", range(8))
def test_locate_binned_equals_brute(seed):
    h = workloads.random_tiny(seed, multi_root=(seed % 2 == 0))
    O = Oracle(h)
    rng = np.random.default_rng(seed)
    Bw_lo, Bw_hi = O._origin, O._origin + 8 * h.h0   # root_cells = 8
    for _ in range(2000):
        x = Bw_lo + (Bw_hi - Bw_lo) * rng.uniform(-0.05, 1.05, 3)
        assert O.locate(x) == O.locate(x, brute=True)
    # points exactly on patch faces
    for p in h.patches:
        lo, hi = _world_box(h, p)
        for x in (lo, hi, 0.5 * (lo + hi)):
            assert O.locate(x) == O.locate(x, brute=True)


def test_locate_brute_matches_definition():
    """locate = the patch of maximum level whose half-open box holds x (upper faces of B closed)."""
    h = workloads.tiny_samr(0)
    O = Oracle(h)
    rng = np.random.default_rng(1)
    for _ in range(3000):
        x = rng.uniform(0, 1, 3)
        best, blev = -1, -1
        for i, p in enumerate(h.patches):
            lo, hi = _world_box(h, p)
            if np.all(x >= lo) and np.all(x < hi) and p.level > blev:
                best, blev = i, p.level
        assert O.locate(x) == best
    assert O.locate(np.array([1.0, 1.0, 1.0])) >= 0       # closed at B's upper faces
    assert O.locate(np.array([1.0 + 1e-12, 0.5, 0.5])) == -1


def test_constant_field_everywhere():
    h = workloads.random_tiny(3, multi_root=True).with_field(workloads.constant_field(0.375))
    O = Oracle(h)
    for p in range(len(h.patches)):
        assert np.all(O.padded_brick(p) == np.float32(0.375))
    rng = np.random.default_rng(0)
    for _ in range(500):
        v = O.field(rng.uniform(0, 1, 3))
        assert v is None or v == np.float32(0.375)


def _linear_hierarchy(seed):
    a = np.array([0.7, -0.4, 0.25])
    # a properly nested hierarchy (the small nested geometry); the linear function takes values that
    # are exact in fp32 at cell centres when a and the centres are dyadic
    h = workloads.tiny_samr(seed)
    return h.with_field(workloads.linear_field(a, 0.5)), a


def test_linear_field_ghosts_exact():
    """g1 copies and g3 coarse interpolants of a linear field are exact; g2 (outside B) replicates
    the boundary value of the clamped centre."""
    h, a = _linear_hierarchy(0)
    O = Oracle(h)
    lin = lambda x: a @ x + 0.5
    for pi, p in enumerate(h.patches):
        brick = O.padded_brick(pi)
        hl = h.h0 / 2.0 ** p.level
        nx, ny, nz = p.dims
        for k in range(-1, nz + 1):
            for j in range(-1, ny + 1):
                for i in range(-1, nx + 1):
                    if 0 <= i < nx and 0 <= j < ny and 0 <= k < nz:
                        continue
                    c = h.origin + (p.lo + np.array([i, j, k]) + 0.5) * hl
                    cc = np.clip(c, 0.5 * hl, 1.0 - 0.5 * hl)       # g2: clamp into B
                    expect = lin(cc)
                    # the centre lies in a coarser patch whose stencil stays inside B (>= one
                    # root cell from the faces) or is a same-level copy: exact up to rounding
                    inner = np.all(np.minimum(cc, 1 - cc) > 1.0 / 32)
                    if inner or p.level == 0:
                        assert abs(brick[k + 1, j + 1, i + 1] - expect) < 1e-6, (pi, i, j, k)


def test_linear_field_pointwise_exact():
    h, a = _linear_hierarchy(1)
    O = Oracle(h)
    rng = np.random.default_rng(2)
    for _ in range(4000):
        # exact region: ghosts near B take replicated (g2) values, and a fine ghost's coarse
        # stencil reaches half a root cell further; 1.5 root cells from the faces is safe
        x = rng.uniform(3.0 / 64, 1 - 3.0 / 64, 3)
        v = O.field(x)
        # cell values are fp32-rounded linear samples: error bound = max |fp32 rounding| ~ 1e-7
        assert abs(v - (a @ x + 0.5)) < 2e-7


def test_g2_edge_replication_single_patch():
    h = workloads.single_level((5, 4, 3))
    O = Oracle(h)
    cells = h.patches[0].cells.astype(np.float64)          # (nz, ny, nx)
    brick = O.padded_brick(0)
    expect = np.pad(cells, 1, mode="edge")
    assert np.array_equal(brick, expect)


def test_g4_nearest_interior_without_coarse_data():
    """A level-1 patch over a hole of the root level: ghosts not covered by any coarser patch
    and not by same-level patches take the nearest interior cell of the patch (g4)."""
    p0 = workloads._empty_patch(0, [0, 0, 0], [4, 8, 8])
    p1 = workloads._empty_patch(0, [4, 0, 0], [4, 4, 8])
    # level-1 patch entirely inside the hole x in [4,8), y in [4,8) (level-0 units)
    p2 = workloads._empty_patch(1, [10, 10, 4], [4, 4, 4])
    h = workloads.Hierarchy(np.zeros(3), np.full(3, 1.0 / 8), 2, 2, [p0, p1, p2])
    h = h.with_field(lambda X, Y, Z: X + 10 * Y + 100 * Z)
    O = Oracle(h)
    brick = O.padded_brick(2)
    cells = h.patches[2].cells.astype(np.float64)
    # on the z faces (k = -1, nz) with interior i, j: no same-level patch and no coarser patch
    # holds those centres (they are inside the hole), so g4 copies the nearest interior cell
    assert np.array_equal(brick[0, 1:-1, 1:-1], cells[0])
    assert np.array_equal(brick[-1, 1:-1, 1:-1], cells[-1])
    # on the x = -1 face the centres lie inside root patch p0's x-range? no: x = 9.5 level-1 cells
    # = 4.75 level-0 cells, i.e. inside the hole as well -> g4
    assert np.array_equal(brick[1:-1, 1:-1, 0], cells[:, :, 0])


def test_g3_coarse_interpolant_hand_value():
    """A level-1 patch inside a 2x2x2 root: ghost values are trilinear interpolants of the
    root's cell-centred values, checked against a value computed by hand."""
    root = workloads._empty_patch(0, [0, 0, 0], [2, 2, 2])
    root.cells[:] = np.arange(8, dtype=np.float32).reshape(2, 2, 2)   # v[k,j,i] = i + 2j + 4k
    fine = workloads._empty_patch(1, [1, 1, 1], [2, 2, 2])
    fine.cells[:] = 100.0
    h = workloads.Hierarchy(np.zeros(3), np.ones(3), 2, 2, [root, fine])
    O = Oracle(h)
    # ghost (i,j,k) = (-1,-1,-1) of the fine patch: centre at level-1 coords 0.5 -> world 0.25;
    # in root coordinates q = 0.25 - 0.5 = -0.25 on each axis: i0 = -1 (root ghost), f = 0.75.
    # Root ghosts replicate the edge (g2), so the value equals root value at (0,0,0) = 0.
    assert O.patch_value(1, -1, -1, -1) == 0.0
    # ghost (2, 0, 0) of the fine patch: centre at level-1 (1+2+0.5, 1.5, 1.5) = world (1.75, .75, .75)
    # root q = (1.25, 0.25, 0.25): i0 = (1,0,0), f = (.25,.25,.25); x index 2 is a root ghost
    # replicating index 1. Values: v(1,0,0)=1, v(2->1,0,0)=1, v(1,1,0)=3, v(1,0,1)=5, v(1,1,1)=7
    # lerp in x gives (1, 3, 5, 7); y: 1 + .25*2 = 1.5, 5.5; z: 1.5 + .25*4 = 2.5
    assert O.patch_value(1, 2, 0, 0) == 2.5
    # interior values are untouched
    assert O.patch_value(1, 0, 0, 0) == 100.0


def test_same_level_copy_g1():
    """Two abutting level-1 patches: each one's ghost layer on the shared face is an exact copy
    of the neighbour's first cell layer (g1), never a coarse interpolant."""
    root = workloads._empty_patch(0, [0, 0, 0], [4, 4, 4])
    a = workloads._empty_patch(1, [2, 2, 2], [2, 3, 2])
    b = workloads._empty_patch(1, [4, 2, 2], [3, 3, 2])
    h = workloads.Hierarchy(np.zeros(3), np.full(3, 0.25), 2, 2, [root, a, b])
    h = h.with_field(lambda X, Y, Z: np.sin(7 * X) + Y * Y - Z)
    O = Oracle(h)
    ba, bb = O.padded_brick(1), O.padded_brick(2)
    ca, cb = h.patches[1].cells, h.patches[2].cells
    assert np.array_equal(ba[1:-1, 1:-1, -1], cb[:, :, 0].astype(np.float64))
    assert np.array_equal(bb[1:-1, 1:-1, 0], ca[:, :, -1].astype(np.float64))
