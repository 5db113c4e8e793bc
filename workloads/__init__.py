"""Seeded synthetic SAMR workloads.

This module only *constructs inputs*: patch boxes, cell values, transfer
function tables and camera frames.  It holds none of the rendering method's
arithmetic (no tree building, no interpolation, no compositing), so both the
HIP library and the FP64 oracle can be fed from it without sharing any code
path of the method.

Data model (Section 3 of the paper): a hierarchy of axis-aligned subgrids
("patches") on levels l = 0..L-1 with a constant refinement factor r, mesh
spacing h^l = h^0 / r^l.  Patch boxes are given in integer level-l cell
coordinates (lo, dims); cell values are fp32, x fastest (array shape
(nz, ny, nx)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

MASTER_SEED = 12123333


@dataclasses.dataclass
class Patch:
    level: int
    lo: np.ndarray          # int64[3], level-l cell coordinates
    dims: np.ndarray        # int64[3]
    cells: np.ndarray       # float32[nz, ny, nx], x fastest

    @property
    def hi(self) -> np.ndarray:
        return self.lo + self.dims


@dataclasses.dataclass
class Hierarchy:
    origin: np.ndarray      # float64[3]
    h0: np.ndarray          # float64[3] root spacing
    refine: int
    nlevels: int
    patches: List[Patch]
    centering: str = "cell"  # "cell": dims cells per patch; "vertex": dims+1 vertex samples per axis

    @property
    def lmax(self) -> int:
        return self.nlevels - 1

    def scale(self, level: int) -> int:
        """Finest cells per level-`level` cell along one axis."""
        return self.refine ** (self.lmax - level)

    def boxes_finest(self) -> np.ndarray:
        """int64[np, 7]: level, lo[3], hi[3] in finest-level cell units."""
        out = np.zeros((len(self.patches), 7), dtype=np.int64)
        for i, p in enumerate(self.patches):
            s = self.scale(p.level)
            out[i, 0] = p.level
            out[i, 1:4] = p.lo * s
            out[i, 4:7] = (p.lo + p.dims) * s
        return out

    def cell_centres(self, p: Patch):
        """World coordinates of the cell centres of patch p (x, y, z 1-D arrays)."""
        h = self.h0 / float(self.refine) ** p.level
        ax = [self.origin[a] + (p.lo[a] + np.arange(p.dims[a]) + 0.5) * h[a] for a in range(3)]
        return ax

    def nbytes_cells(self) -> int:
        return int(sum(p.cells.nbytes for p in self.patches))

    def with_field(self, fn) -> "Hierarchy":
        """Same boxes, cells replaced by fn(X, Y, Z) evaluated at cell centres (FP64 -> fp32)."""
        ps = []
        for p in self.patches:
            x, y, z = self.cell_centres(p)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            v = np.asarray(fn(X, Y, Z), dtype=np.float64)
            v = np.broadcast_to(v, X.shape)
            ps.append(Patch(p.level, p.lo.copy(), p.dims.copy(), np.ascontiguousarray(v, dtype=np.float32)))
        return Hierarchy(self.origin.copy(), self.h0.copy(), self.refine, self.nlevels, ps)

    def shuffled(self, seed: int) -> "Hierarchy":
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(self.patches))
        return Hierarchy(self.origin.copy(), self.h0.copy(), self.refine, self.nlevels,
                         [self.patches[i] for i in perm], self.centering)

    def vertex_positions(self, p: Patch):
        """World coordinates of the grid vertices of patch p (x, y, z 1-D arrays, dims+1 each)."""
        h = self.h0 / float(self.refine) ** p.level
        return [self.origin[a] + (p.lo[a] + np.arange(p.dims[a] + 1)) * h[a] for a in range(3)]

    def with_vertex_field(self, fn) -> "Hierarchy":
        """Same boxes, vertex-centred: each patch holds fn(X, Y, Z) at its (dims+1)^3 grid
        vertices (FP64 -> fp32).  Patches sharing a vertex hold the same sample there."""
        ps = []
        for p in self.patches:
            x, y, z = self.vertex_positions(p)
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            v = np.broadcast_to(np.asarray(fn(X, Y, Z), dtype=np.float64), X.shape)
            ps.append(Patch(p.level, p.lo.copy(), p.dims.copy(), np.ascontiguousarray(v, dtype=np.float32)))
        return Hierarchy(self.origin.copy(), self.h0.copy(), self.refine, self.nlevels, ps, "vertex")


def _rng(workload: int, stream: str, seed: int = MASTER_SEED) -> np.random.Generator:
    names = ["field", "patches", "lut", "cameras", "mlp_init", "train_views", "eval_views", "misc"]
    ss = np.random.SeedSequence(seed).spawn(8)[workload]
    child = ss.spawn(len(names))[names.index(stream)]
    return np.random.default_rng(child)


def _disjoint(a_lo, a_hi, b_lo, b_hi) -> bool:
    return bool(np.any(a_hi <= b_lo) or np.any(b_hi <= a_lo))


# ----------------------------------------------------------------------------------------------
# Fields (evaluated at cell centres by Hierarchy.with_field)
# ----------------------------------------------------------------------------------------------

def gaussian_sum_field(rng: np.random.Generator, n: int = 8, smin=0.02, smax=0.1):
    c = rng.random((n, 3))
    s = rng.uniform(smin, smax, n)
    a = rng.random(n)

    def fn(X, Y, Z):
        v = np.zeros_like(X)
        for j in range(n):
            r2 = (X - c[j, 0]) ** 2 + (Y - c[j, 1]) ** 2 + (Z - c[j, 2]) ** 2
            v = v + a[j] * np.exp(-r2 / (2.0 * s[j] ** 2))
        return v
    return fn


def linear_field(a: Sequence[float], b: float):
    a = np.asarray(a, dtype=np.float64)
    return lambda X, Y, Z: a[0] * X + a[1] * Y + a[2] * Z + b


def constant_field(c: float):
    return lambda X, Y, Z: np.full_like(X, c)


# ----------------------------------------------------------------------------------------------
# Hierarchies
# ----------------------------------------------------------------------------------------------

def _empty_patch(level, lo, dims) -> Patch:
    lo = np.asarray(lo, dtype=np.int64)
    dims = np.asarray(dims, dtype=np.int64)
    return Patch(level, lo, dims, np.zeros(tuple(int(d) for d in dims[::-1]), dtype=np.float32))


def tiny_samr(seed: int = 0) -> Hierarchy:
    """Small nested geometry: root 32^3 on [0,1]^3, r = 2, four level-1 patches of 8..16
    coarse cells per axis at cell-aligned random positions, pairwise disjoint
    (same-level SAMR patches never overlap), field = sum of 8 Gaussians."""
    rng = _rng(0, "patches", MASTER_SEED + seed)
    root = _empty_patch(0, [0, 0, 0], [32, 32, 32])
    boxes = []
    while len(boxes) < 4:
        ext = rng.integers(8, 17, 3)
        lo = np.array([rng.integers(0, 32 - e + 1) for e in ext])
        hi = lo + ext
        if all(_disjoint(lo, hi, b0, b1) for b0, b1 in boxes):
            boxes.append((lo, hi))
    ps = [root] + [_empty_patch(1, 2 * lo, 2 * (hi - lo)) for lo, hi in boxes]
    h = Hierarchy(np.zeros(3), np.full(3, 1.0 / 32), 2, 2, ps)
    return h.with_field(gaussian_sum_field(_rng(0, "field", MASTER_SEED + seed)))


def lod_blocks(seed: int = 0, field=None) -> Hierarchy:
    """Level-of-detail geometry: root 16^3 on [0,1]^3 (one level-0 patch); one half of the
    domain along a seeded axis is fully tiled by k in {2, 4} abutting level-1 patches, and the
    first of them is fully tiled by two level-2 patches.  The kD tree then holds two nested
    kind-(a) nodes: the refined half, covered by the root patch, and the first level-1 patch,
    covered by itself.  Field: sum of Gaussians, or `field`."""
    rng = _rng(5, "patches", MASTER_SEED + seed)
    k = int(rng.choice([2, 4]))
    ax = int(rng.integers(0, 3))
    side = int(rng.integers(0, 2))
    b = int(rng.integers(0, 3))                 # second axis for the level-2 split
    by = (ax + 1 + b % 2) % 3

    def box(level, lo_a, len_a, other):
        lo = np.zeros(3, dtype=np.int64)
        dims = np.full(3, other, dtype=np.int64)
        lo[ax], dims[ax] = lo_a, len_a
        return lo, dims
    ps = [_empty_patch(0, [0, 0, 0], [16, 16, 16])]
    w1 = 16 // k
    x0 = 16 * side                              # level-1 start of the refined half
    for i in range(k):
        lo, dims = box(1, x0 + i * w1, w1, 32)
        ps.append(_empty_patch(1, lo, dims))
    lo, dims = box(2, 2 * x0, 2 * w1, 64)
    for j in range(2):
        l2, d2 = lo.copy(), dims.copy()
        l2[by], d2[by] = 32 * j, 32
        ps.append(_empty_patch(2, l2, d2))
    h = Hierarchy(np.zeros(3), np.full(3, 1.0 / 16), 2, 3, ps)
    return h.with_field(field if field is not None else gaussian_sum_field(_rng(5, "field", MASTER_SEED + seed)))


def random_tiny(seed: int, max_patches: int = 6, nlevels: int = 3, refine: int | None = None,
                root_cells: int = 8, multi_root: bool = False, root_aligned: bool = False) -> Hierarchy:
    """Small random hierarchies for builder/oracle pins: up to `max_patches` patches on
    `nlevels` levels, r in {2, 4}; patches need not be properly nested (a level-l patch may
    span several level-(l-1) parents or stick out of them).  With `root_aligned` every box is
    a union of root cells (its faces lie on planes of every level)."""
    rng = np.random.default_rng(np.random.SeedSequence([MASTER_SEED, 101, seed]))
    r = int(refine if refine is not None else rng.choice([2, 4]))
    ps: List[Patch] = []
    if multi_root:
        half = root_cells // 2
        for i in range(2):
            for j in range(2):
                if rng.random() < 0.85 or not ps:
                    ps.append(_empty_patch(0, [i * half, j * half, 0], [half, half, root_cells]))
    else:
        ps.append(_empty_patch(0, [0, 0, 0], [root_cells] * 3))
    count = len(ps)
    B_lo = np.min([p.lo for p in ps], axis=0)
    B_hi = np.max([p.hi for p in ps], axis=0)
    for lev in range(1, nlevels):
        n_here = rng.integers(1, 3)
        ncell = root_cells * r ** lev
        blo, bhi = B_lo * r ** lev, B_hi * r ** lev        # patches stay inside B
        boxes = [(p.lo, p.hi) for p in ps if p.level == lev]
        tries = 0
        while n_here > 0 and count < max_patches and tries < 200:
            tries += 1
            ext = np.minimum(rng.integers(1, max(2, ncell // 2) + 1, 3), bhi - blo)
            lo = np.array([rng.integers(blo[a], bhi[a] - ext[a] + 1) for a in range(3)])
            if root_aligned:
                g = r ** lev
                lo = lo // g * g
                ext = np.maximum(ext // g, 1) * g
                ext = np.minimum(ext, bhi - lo)
            hi = lo + ext
            if all(_disjoint(lo, hi, b0, b1) for b0, b1 in boxes):
                boxes.append((lo, hi))
                ps.append(_empty_patch(lev, lo, hi - lo))
                count += 1
                n_here -= 1
    h = Hierarchy(np.zeros(3), np.full(3, 1.0 / root_cells), r, nlevels, ps)
    return h.with_field(gaussian_sum_field(np.random.default_rng(seed + 7), n=4, smin=0.1, smax=0.3))


def single_level(n=(12, 10, 8), seed: int = 0) -> Hierarchy:
    """One level-0 patch: the render reduces to a uniform-grid raycast."""
    p = _empty_patch(0, [0, 0, 0], list(n))
    h = Hierarchy(np.array([0.1, -0.2, 0.3]), np.array([0.05, 0.05, 0.05]), 2, 1, [p])
    return h.with_field(gaussian_sum_field(np.random.default_rng(seed + 3), n=5, smin=0.1, smax=0.3))


# ----------------------------------------------------------------------------------------------
# Transfer functions (256 x RGBA; rgb emission, alpha channel = extinction per unit length)
# ----------------------------------------------------------------------------------------------

def lut_bumps(rng: np.random.Generator, sigma_scale: float = 20.0, power: float = 2.0) -> np.ndarray:
    u = np.arange(256) / 255.0
    lut = np.zeros((256, 4))
    for c in range(3):
        v = np.zeros(256)
        for _ in range(3):
            mu, w, a = rng.random(), rng.uniform(0.05, 0.3), rng.uniform(0.3, 1.0)
            v += a * np.exp(-((u - mu) ** 2) / (2 * w * w))
        lut[:, c] = np.clip(v, 0.0, 1.0)
    lut[:, 3] = sigma_scale * u ** power
    return lut.astype(np.float32)


def lut_small_nested(seed: int = 0) -> np.ndarray:
    return lut_bumps(_rng(0, "lut", MASTER_SEED + seed))


def lut_linear_sigma(s: float, rgb=(0.8, 0.5, 0.2)) -> np.ndarray:
    """sigma_i = s * i / 255 and constant emission colour."""
    lut = np.zeros((256, 4), dtype=np.float64)
    lut[:, :3] = rgb
    lut[:, 3] = s * np.arange(256) / 255.0
    return lut.astype(np.float32)


def lut_constant(rgb=(0.8, 0.5, 0.2), sigma=3.0) -> np.ndarray:
    lut = np.zeros((256, 4), dtype=np.float32)
    lut[:, :3] = rgb
    lut[:, 3] = sigma
    return lut


# ----------------------------------------------------------------------------------------------
# Cameras: explicit FP64 frames (eye, right u, up v, forward w)
# ----------------------------------------------------------------------------------------------

def camera(eye, u, v, w, width, height, ortho=False, tan_half_fov=0.0, win=(0.0, 0.0)) -> dict:
    return dict(eye=np.asarray(eye, np.float64), u=np.asarray(u, np.float64),
                v=np.asarray(v, np.float64), w=np.asarray(w, np.float64),
                tan_half_fov=float(tan_half_fov), ortho=bool(ortho),
                win=np.asarray(win, np.float64), width=int(width), height=int(height))


def look_at(eye, centre, up=(0.0, 1.0, 0.0)):
    eye = np.asarray(eye, np.float64)
    w = np.asarray(centre, np.float64) - eye
    w /= np.linalg.norm(w)
    u = np.cross(w, np.asarray(up, np.float64))
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    return eye, u, v, w


def ortho_axis_z(width=256, height=256, lo=(0.0, 0.0), hi=(1.0, 1.0), z=-1.0) -> dict:
    """Orthographic view along +z whose window spans [lo, hi] in x, y."""
    cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
    return camera([cx, cy, z], [1, 0, 0], [0, 1, 0], [0, 0, 1], width, height, ortho=True,
                  win=(0.5 * (hi[0] - lo[0]), 0.5 * (hi[1] - lo[1])))


def ortho_oblique(width=256, height=256, az_deg=30.0, el_deg=20.0, centre=(0.5, 0.5, 0.5),
                  dist=2.0, half=0.9) -> dict:
    az, el = math.radians(az_deg), math.radians(el_deg)
    eye = np.asarray(centre) + dist * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                                -math.cos(el) * math.cos(az)])
    e, u, v, w = look_at(eye, centre)
    return camera(e, u, v, w, width, height, ortho=True, win=(half, half * height / width))


def perspective_orbit(width, height, az, el, radius=2.0, centre=(0.5, 0.5, 0.5), fov_deg=40.0) -> dict:
    eye = np.asarray(centre) + radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                                  -math.cos(el) * math.cos(az)])
    e, u, v, w = look_at(eye, centre)
    return camera(e, u, v, w, width, height, ortho=False, tan_half_fov=math.tan(math.radians(fov_deg) / 2))


def small_nested_cameras(width=256, height=256):
    return [ortho_axis_z(width, height), ortho_oblique(width, height)]


def default_params(**kw) -> dict:
    p = dict(v_lo=0.0, v_hi=1.0, step_frac=0.5, uniform_step=False, t_min=1e-5, lighting=False,
             light=(1.0, 1.0, 1.0), k_a=0.3, k_d=0.7, eps_g=1e-3,
             clip_lo=(-1e300, -1e300, -1e300), clip_hi=(1e300, 1e300, 1e300), interp=0)
    p.update(kw)
    return p


def small_nested(seed: int = 0):
    """Tiny SAMR workload: hierarchy, LUT, cameras and params (v_hi = max cell)."""
    h = tiny_samr(seed)
    vmax = float(max(p.cells.max() for p in h.patches))
    return h, lut_small_nested(seed), small_nested_cameras(), default_params(v_lo=0.0, v_hi=vmax)


# ----------------------------------------------------------------------------------------------
# Cosmology-like hierarchy: log-normal density, patches around density peaks
# ----------------------------------------------------------------------------------------------

class LogNormalField:
    """rho = exp(s g - s^2/2), g a unit-variance Gaussian random field made of K Fourier modes
    with |k| log-uniform in [2 pi, 2 pi kmax] (mode density per log k is flat, i.e. a k^-3
    power spectrum), random directions and phases.  Evaluated separably on lattices."""

    def __init__(self, rng: np.random.Generator, K: int = 64, sigma_ln: float = 2.0, kmax: float = 2048.0):
        self.K, self.s = K, sigma_ln
        kmag = 2 * math.pi * np.exp(rng.uniform(0.0, math.log(kmax), K))
        dirs = rng.normal(size=(K, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        self.k = kmag[:, None] * dirs
        self.phi = rng.uniform(0, 2 * math.pi, K)
        self.amp = math.sqrt(2.0 / K)

    def g_lattice(self, xs, ys, zs) -> np.ndarray:
        ex = np.exp(1j * np.outer(self.k[:, 0], xs))
        ey = np.exp(1j * np.outer(self.k[:, 1], ys))
        ez = np.exp(1j * (np.outer(self.k[:, 2], zs) + self.phi[:, None]))
        m = (ey[:, :, None] * ex[:, None, :]).reshape(self.K, -1)
        return (ez.T @ m).real.reshape(len(zs), len(ys), len(xs)) * self.amp

    def rho_lattice(self, xs, ys, zs) -> np.ndarray:
        return np.exp(self.s * self.g_lattice(xs, ys, zs) - 0.5 * self.s * self.s)


def _fill_cells(h: Hierarchy, fn_lattice) -> Hierarchy:
    for p in h.patches:
        x, y, z = h.cell_centres(p)
        p.cells = np.ascontiguousarray(fn_lattice(x, y, z), dtype=np.float32)
    return h


def cosmology_like(seed: int = 0, root: int = 128, nlevels: int = 6, target_patches: int = 2000,
                   root_split: int = 2, sides=(8, 16, 32, 64), side_probs=(0.01, 0.02, 0.07, 0.90),
                   weights=(0.04, 0.12, 0.22, 0.30, 0.32), min_cover: float = 0.5) -> Hierarchy:
    """Cosmology-like geometry: root `root`^3 on [0,1]^3 split into root_split^3 level-0 patches,
    r = 2.  Level l patches sit on a grid of 64/32/16/8-cell blocks shifted by a random even
    offset (so they span several parents).  Parent cells are visited densest first; for each,
    a side is drawn from `sides` with `side_probs` and the aligned block of that side holding
    the cell is taken if it is free and at least `min_cover` of it lies inside the union of the
    level-(l-1) patches (relaxed nesting), else the side is halved.  Each level stops at its
    `weights` share of `target_patches`."""
    rng = _rng(1, "patches", MASTER_SEED + seed)
    field = LogNormalField(_rng(1, "field", MASTER_SEED + seed))
    rs = root // root_split
    ps = [_empty_patch(0, [i * rs, j * rs, k * rs], [rs, rs, rs])
          for k in range(root_split) for j in range(root_split) for i in range(root_split)]
    h = Hierarchy(np.zeros(3), np.full(3, 1.0 / root), 2, nlevels, ps)
    _fill_cells(h, field.rho_lattice)
    w = np.asarray(weights[: nlevels - 1], dtype=np.float64)
    w = w / w.sum()
    big = max(sides)
    for lev in range(1, nlevels):
        n_l = root * 2 ** lev
        parents = [p for p in h.patches if p.level == lev - 1]
        plo = np.array([2 * p.lo for p in parents])
        phi = np.array([2 * p.hi for p in parents])
        want = int(round(target_patches * w[lev - 1]))
        off = rng.integers(0, big // 2, 3) * 2
        vals = np.concatenate([p.cells.reshape(-1) for p in parents])
        owner = np.concatenate([np.full(p.cells.size, k, dtype=np.int32) for k, p in enumerate(parents)])
        first = np.cumsum([0] + [p.cells.size for p in parents])
        m = min(len(vals), 400 * want)
        top = np.argpartition(-vals, m - 1)[:m]
        top = top[np.argsort(-vals[top], kind="stable")]
        taken = set()
        boxes = []
        for t in top:
            if len(boxes) >= want:
                break
            p = parents[owner[t]]
            li = int(t - first[owner[t]])
            nx, ny = int(p.dims[0]), int(p.dims[1])
            c = 2 * (p.lo + np.array([li % nx, (li // nx) % ny, li // (nx * ny)])) - off
            if tuple(c // 8) in taken:
                continue
            side = int(rng.choice(sides, p=side_probs))
            while side >= sides[0]:
                blo = c // side * side
                cells8 = [tuple(blo // 8 + np.array([a, b, d])) for d in range(side // 8)
                          for b in range(side // 8) for a in range(side // 8)]
                glo, ghi = np.maximum(blo + off, 0), np.minimum(blo + off + side, n_l)
                vol = int(np.prod(ghi - glo))
                inter = np.prod(np.clip(np.minimum(ghi, phi) - np.maximum(glo, plo), 0, None), axis=1).sum()
                if vol > 0 and inter >= min_cover * vol and not any(x in taken for x in cells8):
                    taken.update(cells8)
                    boxes.append((glo, ghi))
                    break
                side //= 2
        for glo, ghi in boxes:
            q = _empty_patch(lev, glo, ghi - glo)
            x, y, z = h.cell_centres(q)
            q.cells = np.ascontiguousarray(field.rho_lattice(x, y, z), dtype=np.float32)
            h.patches.append(q)
    return h


def straddle_fraction(h: Hierarchy, level: int) -> float:
    """Fraction of level-`level` patches overlapping two or more level-(level-1) patches."""
    boxes = h.boxes_finest()
    par = boxes[boxes[:, 0] == level - 1]
    cnt, n = 0, 0
    for b in boxes[boxes[:, 0] == level]:
        ov = np.all(np.minimum(b[4:7], par[:, 4:7]) > np.maximum(b[1:4], par[:, 1:4]), axis=1)
        cnt += int(ov.sum() >= 2)
        n += 1
    return cnt / max(n, 1)


def lut_cosmology(seed: int = 0) -> np.ndarray:
    rng = _rng(1, "lut", MASTER_SEED + seed)
    lut = lut_bumps(rng, sigma_scale=1.0)
    u = np.arange(256) / 255.0
    lut[:, 3] = (0.4 + 60.0 * u).astype(np.float32)
    return lut


def cosmology_view(seed: int = 0, width: int = 1024, height: int = 1024):
    """Cosmology-like workload: hierarchy, LUT, 1024^2 perspective orbit camera, lit params."""
    h = cosmology_like(seed)
    rng = _rng(1, "cameras", MASTER_SEED + seed)
    az = float(rng.uniform(0, 2 * math.pi))
    el = float(rng.uniform(-0.5, 0.5))
    cam = perspective_orbit(width, height, az, el, radius=2.0, fov_deg=40.0)
    sample = np.concatenate([p.cells.reshape(-1)[:: max(1, p.cells.size // 4096)] for p in h.patches])
    vhi = float(np.float32(np.percentile(sample.astype(np.float64), 99.9)))
    prm = default_params(v_lo=0.0, v_hi=vhi, lighting=True, light=(1.0, 1.0, 1.0), k_a=0.3, k_d=0.7)
    return h, lut_cosmology(seed), cam, prm


def cosmology_vertex_view(seed: int = 0, width: int = 1024, height: int = 1024):
    """The cosmology-like view with vertex-centred data (Section 5): the same boxes, LUT,
    camera and params, each patch holding the log-normal density at its (dims+1)^3 grid
    vertices."""
    h, lut, cam, prm = cosmology_view(seed, width, height)
    field = LogNormalField(_rng(1, "field", MASTER_SEED + seed))
    ps = [Patch(p.level, p.lo.copy(), p.dims.copy(),
                np.ascontiguousarray(field.rho_lattice(*h.vertex_positions(p)), dtype=np.float32)) for p in h.patches]
    return Hierarchy(h.origin.copy(), h.h0.copy(), h.refine, h.nlevels, ps, "vertex"), lut, cam, prm


def tf_fit(seed: int = 0, res: int = 512, ncams: int = 8, h: Hierarchy | None = None):
    """Differentiable transfer function: the cosmology-like hierarchy, `ncams` seeded orbit cameras at
    res^2, a hidden target LUT and a different starting LUT."""
    if h is None:
        h = cosmology_like(seed)
    rng = _rng(4, "cameras", MASTER_SEED + seed)
    cams = [perspective_orbit(res, res, float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(-0.6, 0.6)),
                              radius=2.0, fov_deg=40.0) for _ in range(ncams)]
    target = lut_bumps(_rng(4, "lut", MASTER_SEED + seed), sigma_scale=1.0)
    u = np.arange(256) / 255.0
    target[:, 3] = (0.4 + 60.0 * u).astype(np.float32)
    start = lut_bumps(_rng(4, "mlp_init", MASTER_SEED + seed), sigma_scale=1.0)
    start[:, 3] = (0.4 + 30.0 * u ** 0.7).astype(np.float32)
    sample = np.concatenate([p.cells.reshape(-1)[:: max(1, p.cells.size // 4096)] for p in h.patches])
    vhi = float(np.float32(np.percentile(sample.astype(np.float64), 99.9)))
    prm = default_params(v_lo=0.0, v_hi=vhi, lighting=True, light=(1.0, 1.0, 1.0), k_a=0.3, k_d=0.7, t_min=0.0)
    return h, cams, target, start, prm


def serving_cameras(seed: int = 0, ncams: int = 64, sizes=(256, 512, 768, 1024)):
    """Batched serving: `ncams` perspective cameras on random orbit positions, square
    resolutions drawn uniformly from `sizes`."""
    rng = _rng(3, "cameras", MASTER_SEED + seed)
    cams = []
    for _ in range(ncams):
        res = int(rng.choice(sizes))
        cams.append(perspective_orbit(res, res, float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(-0.7, 0.7)),
                                      radius=float(rng.uniform(1.8, 2.4)), fov_deg=40.0))
    return cams


# ----------------------------------------------------------------------------------------------
# Deep-range hierarchy: three collapsing cores refined over 20 levels
# ----------------------------------------------------------------------------------------------

class CoreField:
    """rho = 1 + sum_j A_j (1 + r_j^2 / s^2)^-1 exp(-r_j^2 / (2 w^2)); cells hold log10 rho."""

    def __init__(self, rng: np.random.Generator, ncores: int = 3, s: float = 2.0 ** -24, w: float = 0.05):
        self.c = rng.uniform(0.3, 0.7, (ncores, 3))
        self.A = 10.0 ** (14.0 + rng.uniform(-0.5, 0.5, ncores))
        self.s, self.w = s, w

    def log_rho_lattice(self, xs, ys, zs) -> np.ndarray:
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        rho = np.ones_like(X)
        for j in range(len(self.A)):
            r2 = (X - self.c[j, 0]) ** 2 + (Y - self.c[j, 1]) ** 2 + (Z - self.c[j, 2]) ** 2
            rho += self.A[j] / (1.0 + r2 / self.s ** 2) * np.exp(-r2 / (2 * self.w ** 2))
        return np.log10(rho)


def deep_range(seed: int = 0, root: int = 64, nlevels: int = 20, block: int = 16, radius_cells: float = 44.0):
    """Deep-range geometry: root `root`^3 on [0,1]^3 (one level-0 patch), r = 2, `nlevels` levels.
    Level l >= 1 tiles a ball of radius `radius_cells` h^l around each core with `block`^3
    blocks on a grid shifted by a random even offset (so fine blocks span several parents),
    keeping the blocks that meet a ball, clipped to the domain."""
    rng = _rng(2, "patches", MASTER_SEED + seed)
    field = CoreField(_rng(2, "field", MASTER_SEED + seed))
    h = Hierarchy(np.zeros(3), np.full(3, 1.0 / root), 2, nlevels, [_empty_patch(0, [0, 0, 0], [root] * 3)])
    for lev in range(1, nlevels):
        n_l = root * 2 ** lev
        hl = 1.0 / n_l
        off = rng.integers(0, block // 2, 3) * 2
        keys = set()
        for c in field.c:
            cc = c / hl                                   # core in level-l cell units
            lo = np.floor((cc - radius_cells - off) / block).astype(np.int64)
            hi = np.floor((cc + radius_cells - off) / block).astype(np.int64)
            for kz in range(lo[2], hi[2] + 1):
                for ky in range(lo[1], hi[1] + 1):
                    for kx in range(lo[0], hi[0] + 1):
                        b0 = np.array([kx, ky, kz]) * block + off
                        nearest = np.clip(cc, b0, b0 + block)
                        if np.sum((nearest - cc) ** 2) <= radius_cells ** 2:
                            keys.add((kx, ky, kz))
        for key in sorted(keys):
            b0 = np.array(key) * block + off
            glo, ghi = np.maximum(b0, 0), np.minimum(b0 + block, n_l)
            if np.all(ghi > glo):
                h.patches.append(_empty_patch(lev, glo, ghi - glo))
    for p in h.patches:
        x, y, z = h.cell_centres(p)
        p.cells = np.ascontiguousarray(field.log_rho_lattice(x, y, z), dtype=np.float32)
    h.cores = field.c
    return h


def lut_deep(seed: int = 0, sigma0: float = 1e-4, decades: float = 10.0) -> np.ndarray:
    """sigma_i = sigma0 10^(decades i / 255): the bulk is nearly transparent while the deep
    cores (log10 rho ~ 14) still register."""
    lut = lut_bumps(_rng(2, "lut", MASTER_SEED + seed), sigma_scale=1.0)
    u = np.arange(256) / 255.0
    lut[:, 3] = (sigma0 * 10.0 ** (decades * u)).astype(np.float32)
    return lut


def deep_range_scene(seed: int = 0, res: int = 1024):
    """Deep-range workload: hierarchy, LUT, full-domain view and a zoom on core 0 at res^2."""
    h = deep_range(seed)
    rng = _rng(2, "cameras", MASTER_SEED + seed)
    az, el = float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(-0.4, 0.4))
    full = perspective_orbit(res, res, az, el, radius=2.0, fov_deg=40.0)
    core = h.cores[0]
    zoom = perspective_orbit(res, res, az + 0.7, el, radius=4e-6, centre=tuple(core), fov_deg=40.0)
    prm = default_params(v_lo=0.0, v_hi=14.5, lighting=False, t_min=1e-5)
    return h, lut_deep(seed), [full, zoom], prm


def deep_range_orbits(h: Hierarchy, n: int, seed: int, res: int):
    """Seeded views of the deep-range hierarchy: every third a full-domain orbit (radius 2 about
    the centre), the others zooms onto the cores from log-uniform distances in [3e-6, 0.5]
    (training and held-out sets use different seeds)."""
    rng = np.random.default_rng(np.random.SeedSequence([MASTER_SEED, 3, seed]))
    out = []
    for i in range(n):
        core = h.cores[i % len(h.cores)]
        radius = float(10 ** rng.uniform(-5.5, math.log10(0.5)))
        az, el = float(rng.uniform(0, 2 * math.pi)), float(rng.uniform(-0.8, 0.8))
        if i % 3 == 0:
            out.append(perspective_orbit(res, res, az, el, radius=2.0))
        else:
            out.append(perspective_orbit(res, res, az, el, radius=radius, centre=tuple(core)))
    return out
