"""ctypes mirror of include/amr.h and the loader of the in-tree libamr.so.

There is no fallback: if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamr.so")

c_double3 = ctypes.c_double * 3
c_int64_3 = ctypes.c_int64 * 3
c_float3 = ctypes.c_float * 3
VP = ctypes.c_void_p

AMR_OK, AMR_EINVAL, AMR_EHIERARCHY, AMR_ECAPACITY, AMR_ENOMEM, AMR_EHIP = range(6)
ERRNAMES = {1: "AMR_EINVAL", 2: "AMR_EHIERARCHY", 3: "AMR_ECAPACITY", 4: "AMR_ENOMEM", 5: "AMR_EHIP"}

MLP_IN, MLP_HID, MLP_OUT = 12, 64, 2


class amr_patch(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("pad_", ctypes.c_int32), ("lo", c_int64_3), ("dims", c_int64_3),
                ("cells", VP)]


class amr_domain(ctypes.Structure):
    _fields_ = [("origin", c_double3), ("h0", c_double3), ("refine", ctypes.c_int32), ("nlevels", ctypes.c_int32)]


class amr_tree_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("nodes", "leaves", "n_a", "n_b", "n_c", "depth", "empty_leaves",
                                              "npatches")]


class amr_node_host(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int32), ("level", ctypes.c_int32), ("split", ctypes.c_int64),
                ("patch", ctypes.c_int32), ("cover", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class amr_leaf_host(ctypes.Structure):
    _fields_ = [("lo", c_int64_3), ("hi", c_int64_3), ("patch", ctypes.c_int32), ("level", ctypes.c_int32)]


class amr_pack_opts(ctypes.Structure):
    _fields_ = [("host_dst", ctypes.c_int32), ("nthreads", ctypes.c_int32), ("brick_layout", ctypes.c_int32),
                ("centering", ctypes.c_int32), ("reserved_", ctypes.c_int32 * 4)]


class amr_scene(ctypes.Structure):
    _fields_ = [("pool", VP), ("nodes", VP), ("leaves", VP), ("patches", VP), ("leaf_faces", VP), ("face_taps", VP),
                ("pool_bytes", ctypes.c_int64), ("meta_bytes", ctypes.c_int64),
                ("nnodes", ctypes.c_int32), ("nleaves", ctypes.c_int32), ("npatches", ctypes.c_int32),
                ("nlevels", ctypes.c_int32), ("lmax", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("brick_layout", ctypes.c_int32), ("nlod", ctypes.c_int32),
                ("centering", ctypes.c_int32),
                ("box_lo", c_double3), ("box_hi", c_double3), ("origin", c_double3), ("h0", c_double3),
                ("hfine", c_double3), ("step_fine", ctypes.c_double), ("v_min", ctypes.c_float),
                ("v_max", ctypes.c_float)]


class amr_store_info(ctypes.Structure):
    _fields_ = [("npatches", ctypes.c_int64), ("meta_bytes", ctypes.c_int64), ("full_cache_bytes", ctypes.c_int64),
                ("pad_bytes", ctypes.c_int64)]


class amr_store_report(ctypes.Structure):
    _fields_ = [("uploaded_bricks", ctypes.c_int64), ("uploaded_bytes", ctypes.c_int64),
                ("evicted_bricks", ctypes.c_int64), ("resident_bricks", ctypes.c_int64),
                ("resident_bytes", ctypes.c_int64), ("remapped_leaves", ctypes.c_int64),
                ("repacked", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class amr_camera(ctypes.Structure):
    _fields_ = [("eye", c_double3), ("u", c_double3), ("v", c_double3), ("w", c_double3),
                ("tan_half_fov", ctypes.c_double), ("win", ctypes.c_double * 2), ("ortho", ctypes.c_int32),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class amr_trace_rec(ctypes.Structure):
    _fields_ = [("leaf", ctypes.c_int32), ("patch", ctypes.c_int32), ("n", ctypes.c_int32),
                ("level", ctypes.c_int32), ("ta", ctypes.c_double), ("tb", ctypes.c_double)]


STATS_FIELDS = ("samples", "segments", "rays_hit", "tap_descents", "guard_hits", "trace_overflow",
                "skipped_segments", "coarse_segments", "seglog_count", "ckpt_overflow", "split_samples",
                "face_taps", "unsure_taps", "net_segments", "light_inline")


class amr_render_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in STATS_FIELDS] + [("reserved_", ctypes.c_uint64 * 1)]


class amr_render_params(ctypes.Structure):
    _fields_ = [("d_lut", VP), ("v_lo", ctypes.c_float), ("v_hi", ctypes.c_float), ("step_frac", ctypes.c_float),
                ("t_min", ctypes.c_float), ("uniform_step", ctypes.c_int32), ("lighting", ctypes.c_int32),
                ("light", c_float3), ("k_a", ctypes.c_float), ("k_d", ctypes.c_float), ("eps_g", ctypes.c_float),
                ("clip_lo", c_double3), ("clip_hi", c_double3),
                ("d_trace", VP), ("d_trace_n", VP), ("d_nsamp", VP), ("trace_cap", ctypes.c_int64),
                ("d_ckpt", VP), ("ckpt_bytes", ctypes.c_int64), ("ckpt_every", ctypes.c_int32),
                ("ckpt_max", ctypes.c_int32), ("d_tape", VP), ("tape_cap", ctypes.c_int64),
                ("d_mlp", VP), ("tau_e", ctypes.c_float), ("tau_s", ctypes.c_float),
                ("d_seglog", VP), ("seglog_cap", ctypes.c_int64),
                ("persistent", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("interp", ctypes.c_int32), ("lod", ctypes.c_float),
                ("d_queue", VP), ("d_stamps", VP), ("d_cams", VP), ("d_touch", VP),
                ("d_work", VP), ("work_bytes", ctypes.c_int64), ("light_jobs", ctypes.c_int64),
                ("d_touch_meta", VP), ("bound_only", ctypes.c_int32), ("queue_order", ctypes.c_int32),
                ("xcd_tiles", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32), ("pad3_", ctypes.c_int32),
                ("d_sched", VP), ("sched_bytes", ctypes.c_int64)]


class amr_seglog_rec(ctypes.Structure):
    _fields_ = [("feat", ctypes.c_float * MLP_IN), ("alpha_seg", ctypes.c_float), ("t_in", ctypes.c_float),
                ("ray", ctypes.c_int32), ("n", ctypes.c_int32)]


# every exported entry point declared in include/amr.h, with its signature
SIGNATURES = {
    "amr_last_error": (ctypes.c_char_p, []),
    "amr_build_kdtree": (ctypes.c_int, [ctypes.POINTER(amr_domain), ctypes.POINTER(amr_patch), ctypes.c_int32,
                                        ctypes.POINTER(VP)]),
    "amr_tree_stats": (ctypes.c_int, [VP, ctypes.POINTER(amr_tree_info)]),
    "amr_tree_export": (ctypes.c_int, [VP, VP, ctypes.c_size_t, VP, ctypes.c_size_t]),
    "amr_tree_free": (None, [VP]),
    "amr_pack_pool": (ctypes.c_int, [VP, ctypes.POINTER(amr_patch), ctypes.c_int32, ctypes.POINTER(amr_pack_opts),
                                     VP, ctypes.POINTER(ctypes.c_int64), VP, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(amr_scene), VP]),
    "amr_store_create": (ctypes.c_int, [VP, ctypes.POINTER(amr_patch), ctypes.c_int32, ctypes.POINTER(amr_pack_opts),
                                        ctypes.POINTER(VP)]),
    "amr_store_stats": (ctypes.c_int, [VP, ctypes.POINTER(amr_store_info)]),
    "amr_store_brick_bytes": (ctypes.c_int, [VP, VP, ctypes.c_int64]),
    "amr_store_select": (ctypes.c_int, [VP, ctypes.POINTER(amr_camera), ctypes.c_int64, VP]),
    "amr_store_update": (ctypes.c_int, [VP, VP, VP, ctypes.c_int64, VP, ctypes.c_int64, ctypes.POINTER(amr_scene),
                                        ctypes.POINTER(amr_store_report), VP]),
    "amr_store_free": (None, [VP]),
    "amr_render": (ctypes.c_int, [ctypes.POINTER(amr_scene), ctypes.POINTER(amr_camera), ctypes.c_int32,
                                  ctypes.POINTER(amr_render_params), VP, VP, VP]),
    "amr_queue_bytes": (ctypes.c_int64, [ctypes.c_int32]),
    "amr_wall_clock_khz": (ctypes.c_int64, []),
    "amr_ckpt_bytes": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int32]),
    "amr_tape_bytes": (ctypes.c_int64, [ctypes.c_int64, ctypes.c_int64]),
    "amr_sched_bytes": (ctypes.c_int64, [ctypes.POINTER(amr_camera), ctypes.c_int32]),
    "amr_render_work_bytes": (ctypes.c_int64, [ctypes.POINTER(amr_camera), ctypes.c_int32,
                                               ctypes.POINTER(amr_render_params)]),
    "amr_backward_work_bytes": (ctypes.c_int64, [ctypes.c_int32]),
    "amr_backward_static_bytes": (ctypes.c_int64, []),
    "amr_probe_read": (ctypes.c_int, [VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, VP, VP]),
    "amr_render_backward": (ctypes.c_int, [ctypes.POINTER(amr_scene), ctypes.POINTER(amr_camera), ctypes.c_int32,
                                           ctypes.POINTER(amr_render_params), VP, VP, VP, ctypes.c_int32, VP]),
    "amr_render_backward_static": (ctypes.c_int, [ctypes.POINTER(amr_scene), ctypes.POINTER(amr_camera), ctypes.c_int32,
                                           ctypes.POINTER(amr_render_params), VP, VP, VP, ctypes.c_int32, VP]),
    "amr_mlp_param_count": (ctypes.c_int32, []),
    "amr_mlp_forward": (ctypes.c_int, [VP, VP, VP, VP, ctypes.c_int64, VP]),
    "amr_mlp_backward": (ctypes.c_int, [VP, VP, VP, VP, VP, ctypes.c_int64, ctypes.c_float, ctypes.c_float, VP, VP,
                                        VP]),
    "amr_mlp_adam_step": (ctypes.c_int, [VP, VP, VP, VP, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, VP]),
    "amr_mlp_packed_bytes": (ctypes.c_int64, []),
    "amr_mlp_pack": (ctypes.c_int, [VP, VP, VP]),
}

_lib = None


class AMRError(RuntimeError):
    pass


def load():
    """Loads libamr.so (built in-tree by paper_1212_3333_amd.build). No fallback exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libamr.so is not built; run `python paper_1212_3333_amd/build.py`")
    # torch first: the library resolves the HIP runtime to the copy torch has loaded
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, what: str = ""):
    if rc != AMR_OK:
        msg = load().amr_last_error().decode(errors="replace")
        raise AMRError("%s failed: %s (%s)" % (what, ERRNAMES.get(rc, rc), msg))
