"""MI355X-native single-pass raycasting of structured AMR data (Kaehler & Abel, arXiv 1212.3333).

Thin Python binding over the C ABI of libamr (include/amr.h).  Every step of the hot path runs
in the library's C++/HIP code; this module only marshals arguments, and torch provides device
memory and the current stream.  If libamr.so is missing, importing this package fails.

    tree  = build_tree(h)                    # amr_build_kdtree   (Section 4.1)
    scene = pack(tree, h)                    # amr_pack_pool      (Sections 4.2, 5)
    rgba  = render(scene, cams, lut, params) # amr_render         (Section 5.3)
    gl, gL = render_backward(...)            # amr_render_backward
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import AMRError, check, load

load()

__all__ = ["AMRError", "Tree", "Scene", "Store", "ResidentScene", "build_tree", "pack", "render",
           "render_backward", "make_params", "RenderOutput", "AMRRender"]


def _vp(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(None)
    if isinstance(t, torch.Tensor):
        return ctypes.c_void_p(t.data_ptr())
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t)


def _stream(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _patch_array(h):
    """amr_patch[] for a hierarchy (keeps the fp32 cell arrays alive via the returned list)."""
    keep = []
    arr = (L.amr_patch * len(h.patches))()
    for i, p in enumerate(h.patches):
        c = np.ascontiguousarray(p.cells, dtype=np.float32)
        keep.append(c)
        arr[i].level = int(p.level)
        arr[i].lo[:] = [int(x) for x in p.lo]
        arr[i].dims[:] = [int(x) for x in p.dims]
        arr[i].cells = c.ctypes.data
    return arr, keep


def _domain(h) -> L.amr_domain:
    d = L.amr_domain()
    d.origin[:] = [float(x) for x in h.origin]
    d.h0[:] = [float(x) for x in h.h0]
    d.refine = int(h.refine)
    d.nlevels = int(h.nlevels)
    return d


class Tree:
    """Host kD-tree (immutable). Nodes and leaves are exported in depth-first pre-order."""

    def __init__(self, h):
        self.lib = load()
        self.h = h
        self._patches, self._keep = _patch_array(h)
        self._dom = _domain(h)
        ptr = ctypes.c_void_p()
        check(self.lib.amr_build_kdtree(ctypes.byref(self._dom), self._patches, len(h.patches), ctypes.byref(ptr)),
              "amr_build_kdtree")
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value:
            self.lib.amr_tree_free(self.ptr)
            self.ptr = None

    def info(self) -> dict:
        s = L.amr_tree_info()
        check(self.lib.amr_tree_stats(self.ptr, ctypes.byref(s)), "amr_tree_stats")
        return {k: int(getattr(s, k)) for k, _ in L.amr_tree_info._fields_}

    def export(self):
        """(nodes, leaves) as numpy structured arrays."""
        inf = self.info()
        nodes = (L.amr_node_host * inf["nodes"])()
        leaves = (L.amr_leaf_host * inf["leaves"])()
        check(self.lib.amr_tree_export(self.ptr, nodes, inf["nodes"], leaves, inf["leaves"]), "amr_tree_export")
        ndt = np.dtype([("axis", np.int32), ("level", np.int32), ("split", np.int64), ("patch", np.int32),
                        ("cover", np.int32), ("kind", np.int32), ("pad_", np.int32)])
        ldt = np.dtype([("lo", np.int64, 3), ("hi", np.int64, 3), ("patch", np.int32), ("level", np.int32)])
        return (np.frombuffer(bytes(nodes), dtype=ndt).copy(), np.frombuffer(bytes(leaves), dtype=ldt).copy())


def build_tree(h) -> Tree:
    return Tree(h)


class Scene:
    """Packed pool + device tree. On device, pool/meta are torch uint8 tensors on `device`;
    with host=True they are numpy arrays (no HIP involved)."""

    def __init__(self, tree: Tree, h, device="cuda", host: bool = False, nthreads: int = 0, brick_layout: int = 2):
        self.lib = load()
        self.tree = tree
        opts = _pack_opts(h, host, nthreads, brick_layout)
        pb, mb = ctypes.c_int64(0), ctypes.c_int64(0)
        check(self.lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts), None,
                                     ctypes.byref(pb), None, ctypes.byref(mb), None, None), "amr_pack_pool(size)")
        self.scene = L.amr_scene()
        self.host = host
        if host:
            self.pool = np.zeros(pb.value, dtype=np.uint8)
            self.meta = np.zeros(mb.value, dtype=np.uint8)
            stream = ctypes.c_void_p(None)
        else:
            self.pool = torch.empty(pb.value, dtype=torch.uint8, device=device)
            self.meta = torch.empty(mb.value, dtype=torch.uint8, device=device)
            stream = _stream(self.pool.device)
        check(self.lib.amr_pack_pool(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts), _vp(self.pool),
                                     ctypes.byref(pb), _vp(self.meta), ctypes.byref(mb), ctypes.byref(self.scene),
                                     stream), "amr_pack_pool")

    @property
    def nbytes(self) -> int:
        return int(self.scene.pool_bytes + self.scene.meta_bytes)

    # host-side views (host=True scenes): padded bricks and device records
    def brick(self, p: int) -> np.ndarray:
        """Padded brick of patch p as a (nz+2, ny+2, nx+2) array, whatever the pool layout
        (vertex-centred data: (nz+3, ny+3, nx+3), the samples plus their one-sample shell)."""
        assert self.host
        hdr = self.patch_headers()[p]
        nx, ny, nz = (int(v) for v in hdr["n"])
        pool = self.pool.view(np.float32)
        off = int(hdr["off"])
        if int(hdr["layout"]) == 0:
            return pool[off:off + (nx + 2) * (ny + 2) * (nz + 2)].reshape(nz + 2, ny + 2, nx + 2)
        bx, by, bz = (int(v) for v in hdr["nb"])
        if int(hdr["layout"]) == 2:
            # halo rows: block (bz, by, bx), row (k & 3, j & 3), slots 1..4 hold x = 4 bx .. 4 bx + 3
            blocks = pool[off:off + bx * by * bz * 128].reshape(bz, by, bx, 4, 4, 8)[..., 1:5]
        else:
            blocks = pool[off:off + bx * by * bz * 64].reshape(bz, by, bx, 4, 4, 4)
        full = blocks.transpose(0, 3, 1, 4, 2, 5).reshape(4 * bz, 4 * by, 4 * bx)
        return full[: nz + 2, : ny + 2, : nx + 2]

    def halo_rows(self, p: int) -> np.ndarray:
        """Halo-row layout only: the raw [nbz, nby, nbx, 4 (z), 4 (y), 8] row store of patch p."""
        assert self.host
        hdr = self.patch_headers()[p]
        assert int(hdr["layout"]) == 2
        bx, by, bz = (int(v) for v in hdr["nb"])
        off = int(hdr["off"])
        return self.pool.view(np.float32)[off:off + bx * by * bz * 128].reshape(bz, by, bx, 4, 4, 8)

    def patch_headers(self) -> np.ndarray:
        dt = np.dtype([("off", np.uint64), ("n", np.int32, 3), ("level", np.int32), ("lo", np.float64, 3),
                       ("inv_h", np.float64, 3), ("h", np.float64, 3), ("step", np.float64),
                       ("vmin", np.float32), ("vmax", np.float32), ("nb", np.int32, 3), ("layout", np.int32)])
        return self._records(self.scene.patches, dt, self.scene.npatches)

    def leaf_records(self) -> np.ndarray:
        dt = np.dtype([("lo", np.float64, 3), ("hi", np.float64, 3), ("patch", np.int32),
                       ("level_flags", np.uint32), ("vmin", np.float32), ("vmax", np.float32)])
        return self._records(self.scene.leaves, dt, self.scene.nleaves)

    def leaf_face_owners(self) -> np.ndarray:
        """[nleaves, 6] int32: patch owning the one-cell slab beyond each leaf face (-1: none/several)."""
        base = self.meta.ctypes.data if self.host else self.meta.data_ptr()
        off = self.scene.leaf_faces - base
        raw = self.meta[off:off + self.scene.nleaves * 24]
        raw = raw if self.host else raw.cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=np.int32).reshape(-1, 6)

    def face_tap_records(self) -> np.ndarray:
        """[nleaves, 6] gradient-tap records: the single slab owner's brick (n > 0) with the map
        q_owner = r q + t from the leaf's patch-local cell coordinates, else the rope node."""
        dt = np.dtype([("off", np.uint64), ("n", np.int32, 3), ("px", np.int32), ("pxy", np.int32),
                       ("r", np.float32), ("t", np.float32, 3), ("rope", np.int32), ("pad", np.int32, 4)])
        return self._records(self.scene.face_taps, dt, self.scene.nleaves * 6).reshape(-1, 6)

    def node_records(self) -> np.ndarray:
        dt = np.dtype([("split", np.float64), ("child", np.uint32), ("meta", np.uint32)])
        return self._records(self.scene.nodes, dt, self.scene.nnodes)

    def _records(self, ptr, dt, n):
        base = self.meta.ctypes.data if self.host else self.meta.data_ptr()
        off = ptr - base
        raw = self.meta[off:off + n * dt.itemsize]
        raw = raw if self.host else raw.cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=dt)


def pack(tree: Tree, h, device="cuda", host: bool = False, nthreads: int = 0, brick_layout: int = 2) -> Scene:
    return Scene(tree, h, device=device, host=host, nthreads=nthreads, brick_layout=brick_layout)


def _pack_opts(h, host: bool, nthreads: int, brick_layout: int) -> L.amr_pack_opts:
    centering = getattr(h, "centering", "cell")
    if centering not in ("cell", "vertex"):
        raise ValueError("centering must be 'cell' or 'vertex'")
    extra = 1 if centering == "vertex" else 0
    for i, p in enumerate(h.patches):
        want = tuple(int(d) + extra for d in p.dims[::-1])
        if tuple(np.shape(p.cells)) != want:
            raise ValueError("patch %d holds samples of shape %s; %s-centred data needs %s"
                             % (i, np.shape(p.cells), centering, want))
    opts = L.amr_pack_opts()
    opts.host_dst = 1 if host else 0
    opts.nthreads = int(nthreads)
    opts.brick_layout = int(brick_layout)
    opts.centering = extra
    return opts


class ResidentScene(Scene):
    """Scene of a Store update: pool = the device brick cache, meta = its metadata buffer."""

    def __init__(self, store, cache, meta, scene):
        self.lib = store.lib
        self.tree = store.tree
        self.host = store.host
        self.pool = cache
        self.meta = meta
        self.scene = scene


class Store:
    """Out-of-core residency (amr_store_*): every brick packed once on the host; `update` makes
    a subset resident in a device brick cache and returns the scene that renders it."""

    def __init__(self, tree: Tree, h, host: bool = False, nthreads: int = 0, brick_layout: int = 2):
        self.lib = load()
        self.tree = tree
        self.host = host
        self.npatches = len(h.patches)
        opts = _pack_opts(h, host, nthreads, brick_layout)
        ptr = ctypes.c_void_p()
        check(self.lib.amr_store_create(tree.ptr, tree._patches, len(h.patches), ctypes.byref(opts),
                                        ctypes.byref(ptr)), "amr_store_create")
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None) and self.ptr.value:
            self.lib.amr_store_free(self.ptr)
            self.ptr = None

    def info(self) -> dict:
        s = L.amr_store_info()
        check(self.lib.amr_store_stats(self.ptr, ctypes.byref(s)), "amr_store_stats")
        return {k: int(getattr(s, k)) for k, _ in L.amr_store_info._fields_}

    def brick_bytes(self) -> np.ndarray:
        out = np.zeros(self.npatches, dtype=np.int64)
        check(self.lib.amr_store_brick_bytes(self.ptr, _vp(out), len(out)), "amr_store_brick_bytes")
        return out

    def select(self, cam: dict, cache_bytes: int) -> np.ndarray:
        out = np.zeros(self.npatches, dtype=np.uint8)
        check(self.lib.amr_store_select(self.ptr, ctypes.byref(make_camera(cam)), int(cache_bytes), _vp(out)),
              "amr_store_select")
        return out.astype(bool)

    @staticmethod
    def host_buffer(nbytes: int) -> np.ndarray:
        """Zeroed 256-byte aligned host bytes (a cache for a host store)."""
        raw = np.zeros(int(nbytes) + 256, dtype=np.uint8)
        off = (-raw.ctypes.data) % 256
        return raw[off:off + int(nbytes)]

    def alloc(self, cache_bytes: int, device="cuda"):
        """(cache, meta) buffers: device tensors, or numpy arrays for a host store."""
        mb = self.info()["meta_bytes"]
        if self.host:
            return self.host_buffer(cache_bytes), self.host_buffer(mb)
        return (torch.zeros(int(cache_bytes), dtype=torch.uint8, device=device),
                torch.empty(mb, dtype=torch.uint8, device=device))

    def update(self, resident, cache, meta):
        """Makes the patches with resident[p] true resident in `cache`; returns (scene, report)."""
        m = np.ascontiguousarray(np.asarray(resident).astype(np.uint8))
        if m.shape != (self.npatches,):
            raise ValueError("resident mask must have one entry per patch")
        sc = L.amr_scene()
        rep = L.amr_store_report()
        nbytes = cache.numel() if isinstance(cache, torch.Tensor) else cache.nbytes
        mbytes = meta.numel() if isinstance(meta, torch.Tensor) else meta.nbytes
        stream = ctypes.c_void_p(None) if self.host else _stream(cache.device)
        check(self.lib.amr_store_update(self.ptr, _vp(m), _vp(cache), int(nbytes), _vp(meta), int(mbytes),
                                        ctypes.byref(sc), ctypes.byref(rep), stream), "amr_store_update")
        return ResidentScene(self, cache, meta, sc), {k: int(getattr(rep, k)) for k, _ in L.amr_store_report._fields_
                                                      if k != "reserved_"}


def make_camera(cam: dict) -> L.amr_camera:
    c = L.amr_camera()
    for k in ("eye", "u", "v", "w"):
        getattr(c, k)[:] = [float(x) for x in cam[k]]
    c.tan_half_fov = float(cam.get("tan_half_fov", 0.0))
    c.win[:] = [float(x) for x in cam.get("win", (0.0, 0.0))]
    c.ortho = int(bool(cam["ortho"]))
    c.width, c.height = int(cam["width"]), int(cam["height"])
    return c


def make_params(p: dict, d_lut) -> L.amr_render_params:
    q = L.amr_render_params()
    q.d_lut = _vp(d_lut).value
    q.v_lo, q.v_hi, q.step_frac, q.t_min = p["v_lo"], p["v_hi"], p["step_frac"], p["t_min"]
    q.uniform_step = int(bool(p["uniform_step"]))
    q.lighting = int(p["lighting"])
    q.light[:] = [float(x) for x in p["light"]]
    q.k_a, q.k_d, q.eps_g = p["k_a"], p["k_d"], p["eps_g"]
    q.clip_lo[:] = [float(x) for x in p["clip_lo"]]
    q.clip_hi[:] = [float(x) for x in p["clip_hi"]]
    q.tau_e = float(p.get("tau_e", 0.0))
    q.tau_s = float(p.get("tau_s", 0.0))
    q.persistent = int(p.get("persistent", 0))
    q.tile_w = int(p.get("tile_w", 0))
    q.tile_h = int(p.get("tile_h", 0))
    q.blocks_per_cu = int(p.get("blocks_per_cu", 0))
    q.interp = int(p.get("interp", 0))
    q.lod = float(p.get("lod", 0.0))
    q.bound_only = int(bool(p.get("bound_only", 0)))
    q.queue_order = int(p.get("queue_order", 0))
    q.xcd_tiles = int(p.get("xcd_tiles", 0))
    q.waves_per_simd = int(p.get("waves_per_simd", 0))
    return q


class RenderOutput(dict):
    __getattr__ = dict.__getitem__


def _cams(cams):
    if isinstance(cams, dict):
        cams = [cams]
    arr = (L.amr_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = make_camera(c)
    return cams, arr


# Default job slots of the point light's secondary-ray pass, per pixel of the largest camera
# (samples beyond them trace their secondary ray in the shading pass: same image, slower).
LIGHT_JOBS_PER_PIXEL = 512


def render(scene: Scene, cams, lut: torch.Tensor, params: dict, trace_cap: int = 0, stats: bool = False,
           nsamp: bool = False, out: torch.Tensor | None = None, **extra) -> RenderOutput:
    """Renders one camera (dict) or several (list) with amr_render.  Returns RenderOutput with
    rgba ([H,W,4] for one camera, else the concatenated flat [sum HW, 4]) and, on request,
    trace/trace_n/nsamp/stats."""
    lib = load()
    dev = scene.pool.device
    cam_list, carr = _cams(cams)
    npix = sum(int(c["width"]) * int(c["height"]) for c in cam_list)
    lut = lut.to(device=dev, dtype=torch.float32).contiguous()
    q = make_params(dict(params, **extra), lut)
    res = RenderOutput()
    rgba = out if out is not None else torch.empty(npix * 4, dtype=torch.float32, device=dev)
    if trace_cap:
        trace = torch.zeros((npix, trace_cap, 32), dtype=torch.uint8, device=dev)
        trace_n = torch.zeros(npix, dtype=torch.int32, device=dev)
        q.d_trace, q.d_trace_n, q.trace_cap = trace.data_ptr(), trace_n.data_ptr(), trace_cap
        res["trace_raw"], res["trace_n"] = trace, trace_n
    if nsamp:
        ns = torch.zeros(npix, dtype=torch.int32, device=dev)
        q.d_nsamp = ns.data_ptr()
        res["nsamp"] = ns
    st = torch.zeros(16, dtype=torch.int64, device=dev) if stats else None
    for k in ("d_ckpt", "ckpt_bytes", "ckpt_every", "ckpt_max", "d_tape", "tape_cap", "d_mlp", "d_seglog", "seglog_cap",
              "d_queue",
              "d_stamps", "d_touch", "d_touch_meta", "d_cams", "d_work", "work_bytes", "light_jobs", "d_sched",
              "sched_bytes"):
        if k in extra:
            v = extra[k]
            setattr(q, k, v.data_ptr() if isinstance(v, torch.Tensor) else v)
    if q.lighting == 2 and "d_work" not in extra:
        # point light: the job arrays of the secondary-ray pass live in a workspace owned here
        npix_max = max(int(c["width"]) * int(c["height"]) for c in cam_list)
        q.light_jobs = int(params.get("light_jobs", extra.get("light_jobs", LIGHT_JOBS_PER_PIXEL * npix_max)))
        nwork = int(lib.amr_render_work_bytes(carr, len(cam_list), ctypes.byref(q)))
        work = torch.empty(max(nwork, 1), dtype=torch.uint8, device=dev)
        q.d_work, q.work_bytes = work.data_ptr(), nwork
        res["_work"] = work
    check(lib.amr_render(ctypes.byref(scene.scene), carr, len(cam_list), ctypes.byref(q), _vp(rgba), _vp(st),
                         _stream(dev)), "amr_render")
    res["rgba"] = rgba.view(cam_list[0]["height"], cam_list[0]["width"], 4) if len(cam_list) == 1 else rgba.view(-1, 4)
    if stats:
        res["stats_raw"] = st
    res["_keep"] = (lut, carr, q)
    return res


# ----------------------------------------------------------------------------------------------
# Proposal network (training runs on the GPU through the library's kernels)
# ----------------------------------------------------------------------------------------------

def mlp_param_count() -> int:
    return int(load().amr_mlp_param_count())


def mlp_forward(X: torch.Tensor, W: torch.Tensor, keep_hidden: bool = True):
    """Y [n,2] = (alpha_lo, alpha_hi) and, if keep_hidden, the activations H [n,128]."""
    lib = load()
    n = X.shape[0]
    Y = torch.empty((n, 2), dtype=torch.float32, device=X.device)
    H = torch.empty((n, 128), dtype=torch.float32, device=X.device) if keep_hidden else None
    check(lib.amr_mlp_forward(_vp(X), _vp(W), _vp(Y), _vp(H), n, _stream(X.device)), "amr_mlp_forward")
    return Y, H


def mlp_backward(X, W, H, Y, T, q_lo=0.01, q_hi=0.99):
    """(dW, loss) of the mean pinball loss."""
    lib = load()
    dW = torch.empty_like(W)
    loss = torch.empty(1, dtype=torch.float32, device=W.device)
    check(lib.amr_mlp_backward(_vp(X), _vp(W), _vp(H), _vp(Y), _vp(T), X.shape[0], q_lo, q_hi, _vp(dW), _vp(loss),
                               _stream(W.device)), "amr_mlp_backward")
    return dW, loss


def mlp_adam_step(W, dW, M, V, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    check(load().amr_mlp_adam_step(_vp(W), _vp(dW), _vp(M), _vp(V), int(t), lr, beta1, beta2, eps, _stream(W.device)),
          "amr_mlp_adam_step")


def mlp_pack(W: torch.Tensor) -> torch.Tensor:
    """fp16 inference image of the network, for params d_mlp."""
    lib = load()
    out = torch.empty(int(lib.amr_mlp_packed_bytes()), dtype=torch.uint8, device=W.device)
    check(lib.amr_mlp_pack(_vp(W), _vp(out), _stream(W.device)), "amr_mlp_pack")
    return out


def camera_table(cams, device="cuda") -> torch.Tensor:
    """Device copy of a camera list (amr_camera records) for persistent rendering."""
    _, carr = _cams(cams)
    raw = np.frombuffer(bytes(carr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def queue_buffer(ncams: int, device="cuda") -> torch.Tensor:
    return torch.zeros(int(load().amr_queue_bytes(ncams)), dtype=torch.uint8, device=device)


def read_bandwidth(nbytes: int, reps: int, blocks: int = 2048, device="cuda") -> float:
    """Sustained read rate (GB/s) of the cache level a buffer of nbytes fits in, from the
    library's read probe timed with HIP events on the current stream (one warm-up launch)."""
    lib = load()
    buf = torch.ones(max(16, nbytes) // 4, dtype=torch.float32, device=device)
    sink = torch.zeros(1, dtype=torch.float32, device=device)
    st = _stream(device)
    check(lib.amr_probe_read(_vp(buf), buf.numel() * 4, 1, blocks, _vp(sink), st), "amr_probe_read")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    check(lib.amr_probe_read(_vp(buf), buf.numel() * 4, reps, blocks, _vp(sink), st), "amr_probe_read")
    e1.record()
    torch.cuda.synchronize(device)
    return buf.numel() * 4 // 16 * 16 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def wall_clock_khz() -> int:
    return int(load().amr_wall_clock_khz())


def trace_records(res: RenderOutput) -> np.ndarray:
    """Decodes the per-ray segment trace into a numpy structured array [nrays, cap]."""
    dt = np.dtype([("leaf", np.int32), ("patch", np.int32), ("n", np.int32), ("level", np.int32),
                   ("ta", np.float64), ("tb", np.float64)])
    raw = res["trace_raw"].cpu().numpy()
    return raw.view(dt).reshape(raw.shape[0], raw.shape[1])


def stats_dict(res: RenderOutput) -> dict:
    v = res["stats_raw"].cpu().numpy().view(np.uint64)
    return {k: int(v[i]) for i, k in enumerate(L.STATS_FIELDS)}


# Tape records per ray for lit checkpointed renders (16 bytes each: one per data segment and
# one per sample); the adjoint evaluates the intervals of a ray past its cap in place, at several
# times the cost of reading them.  The default cap is the largest multiple of 8 up to TAPE_CAP
# whose tape fits in TAPE_MEM_FRACTION of the device's memory.
TAPE_CAP = 2048
TAPE_MEM_FRACTION = 0.3


def default_tape_cap(nrays: int, device=None, total_memory: int | None = None) -> int:
    """Tape records per ray for nrays rays on `device` (or a device of total_memory bytes)."""
    total = total_memory if total_memory is not None else torch.cuda.get_device_properties(
        torch.device(device)).total_memory
    cap = int(TAPE_MEM_FRACTION * total) // (16 * max(int(nrays), 1))
    return max(0, min(TAPE_CAP, cap // 8 * 8))


class Schedule:
    """Tile schedule for repeated renders of the same cameras (amr_sched_bytes; pass **params()
    to render): every call records each 8x8 tile's time, and the next call with the same
    lighting and cameras of the same sizes starts the super-tiles (16x16 pixels lit, 32x32 unlit)
    of each launch's cameras (up to 8) with the longest tiles first.  Zeroed at creation; reset() forgets the recorded order (after a large
    change of view)."""

    def __init__(self, cams, device):
        lib = load()
        cam_list, carr = _cams(cams)
        self.nbytes = int(lib.amr_sched_bytes(carr, len(cam_list)))
        if self.nbytes < 0:
            raise ValueError("invalid cameras")
        self.buf = torch.zeros(self.nbytes, dtype=torch.uint8, device=device)

    def params(self) -> dict:
        return dict(d_sched=self.buf, sched_bytes=self.nbytes)

    def reset(self) -> None:
        self.buf.zero_()


class Checkpoints:
    """Device buffers the checkpointed forward fills and the adjoint reads: per ray a header
    (final T and C, samples, checkpoint count, tape records) and up to ckpt_max (t, T, C) records
    taken at the start of every ckpt_every-th data segment (the rate halves when a ray runs out of
    slots); with tape_cap > 0 (lit renders) the tape: per ray, a record per data segment (its
    sample spacing and count) and per sample (value and gradient), tape_cap records at most."""

    def __init__(self, nrays: int, device, ckpt_every: int = 4, ckpt_max: int = 16, tape_cap: int = 0):
        lib = load()
        self.nbytes = int(lib.amr_ckpt_bytes(nrays, ckpt_max))
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.every, self.max = int(ckpt_every), int(ckpt_max)
        self.tape_cap = int(tape_cap)
        self.tape = (torch.empty(int(lib.amr_tape_bytes(nrays, tape_cap)) // 4, dtype=torch.float32, device=device)
                     if tape_cap > 0 else None)
        assert self.tape is None or self.tape.data_ptr() % 16 == 0

    def params(self) -> dict:
        p = dict(d_ckpt=self.buf, ckpt_bytes=self.nbytes, ckpt_every=self.every, ckpt_max=self.max)
        if self.tape is not None:
            p.update(d_tape=self.tape, tape_cap=self.tape_cap)
        return p

    def tape_overflow_rays(self) -> int:
        """Rays with more tape records than tape_cap (the adjoint evaluates their later intervals in
        place); synchronises."""
        if self.tape is None:
            return 0
        hdr = self.buf.view(-1, 32 * (1 + self.max))[:, :32].contiguous().view(torch.int32)[:, 7]
        return int((hdr > self.tape_cap).sum().item())


def render_checkpointed(scene: Scene, cams, lut: torch.Tensor, params: dict, ckpt_every: int = 4,
                        ckpt_max: int = 16, tape_cap: int | None = None, **kw):
    """Forward render that also records the adjoint's checkpoints (and, lit, the tape of tape_cap
    records per ray, default default_tape_cap(); 0 for none). Returns (RenderOutput, Checkpoints)."""
    cam_list = [cams] if isinstance(cams, dict) else list(cams)
    npix = sum(int(c["width"]) * int(c["height"]) for c in cam_list)
    if tape_cap is None:
        tape_cap = default_tape_cap(npix, scene.pool.device) if int(params.get("lighting", 0)) == 1 else 0
    ck = Checkpoints(npix, scene.pool.device, ckpt_every, ckpt_max, tape_cap)
    out = render(scene, cams, lut, params, **ck.params(), **kw)
    return out, ck


def render_backward(scene: Scene, cams, lut: torch.Tensor, params: dict, ckpt: Checkpoints,
                    grad_rgba: torch.Tensor, deterministic: bool = False, static_work: bool = False):
    """dL/dLUT [256,4] and dL/d(light_x, light_y, light_z, k_a, k_d) [5] from dL/dRGBA, using the
    checkpoints of the matching forward call (amr_render_backward).  static_work: call
    amr_render_backward_static, whose accumulators live in the library's fixed device array
    (no workspace is allocated here)."""
    lib = load()
    dev = scene.pool.device
    cam_list, carr = _cams(cams)
    lut = lut.to(device=dev, dtype=torch.float32).contiguous()
    g = grad_rgba.to(device=dev, dtype=torch.float32).contiguous()
    q = make_params(params, lut)
    q.d_ckpt, q.ckpt_bytes, q.ckpt_every, q.ckpt_max = ckpt.buf.data_ptr(), ckpt.nbytes, ckpt.every, ckpt.max
    if ckpt.tape is not None:
        q.d_tape, q.tape_cap = ckpt.tape.data_ptr(), ckpt.tape_cap
    glut = torch.empty((256, 4), dtype=torch.float32, device=dev)
    glight = torch.empty(5, dtype=torch.float32, device=dev)
    if static_work:
        check(lib.amr_render_backward_static(ctypes.byref(scene.scene), carr, len(cam_list), ctypes.byref(q), _vp(g),
                                             _vp(glut), _vp(glight), int(bool(deterministic)), _stream(dev)),
              "amr_render_backward_static")
        return glut, glight
    nwork = int(lib.amr_backward_work_bytes(int(bool(deterministic))))
    work = torch.empty(nwork, dtype=torch.uint8, device=dev)
    q.d_work, q.work_bytes = work.data_ptr(), nwork
    check(lib.amr_render_backward(ctypes.byref(scene.scene), carr, len(cam_list), ctypes.byref(q), _vp(g), _vp(glut),
                                  _vp(glight), int(bool(deterministic)), _stream(dev)), "amr_render_backward")
    return glut, glight


class AMRRender(torch.autograd.Function):
    """Differentiable render: rgba = AMRRender.apply(lut [256,4], shading [5] = (light xyz, k_a,
    k_d), scene, cams, params).  Gradients flow to the LUT and the shading parameters through
    the library's adjoint kernel; the forward keeps segment checkpoints and, lit, the sample
    tape.  schedule: an optional Schedule for these cameras, kept across calls (an optimisation
    loop renders the same views every step)."""

    @staticmethod
    def forward(ctx, lut, shading, scene, cams, params, ckpt_every=4, ckpt_max=16, deterministic=False,
                schedule=None):
        sh = shading.detach().double().cpu().tolist()
        prm = dict(params, light=tuple(sh[:3]), k_a=sh[3], k_d=sh[4])
        kw = schedule.params() if schedule is not None else {}
        out, ck = render_checkpointed(scene, cams, lut.detach(), prm, ckpt_every, ckpt_max, **kw)
        ctx.scene, ctx.cams, ctx.prm, ctx.ck, ctx.det = scene, cams, prm, ck, deterministic
        ctx.lut = lut.detach().to(device=scene.pool.device, dtype=torch.float32).contiguous()
        ctx.lut_device, ctx.sh_device = lut.device, shading.device
        return out["rgba"].clone()

    @staticmethod
    def backward(ctx, grad_rgba):
        glut, glight = render_backward(ctx.scene, ctx.cams, ctx.lut, ctx.prm, ctx.ck, grad_rgba, ctx.det)
        return glut.to(ctx.lut_device), glight.to(ctx.sh_device), None, None, None, None, None, None, None
