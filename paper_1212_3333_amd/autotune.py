"""Autotuner for the persistent multi-camera kernel: times every (tile shape, blocks per CU, waves
per SIMD, tile queue, camera order, brick layout) candidate on the caller's cameras and caches the
fastest per device and workload.

The tile shape is the pixel footprint of a wave (64 rays), blocks per CU the persistent grid
(four waves per block), waves per SIMD the register budget the lit kernel is compiled for (3 with
part of its state spilled to scratch, 2 without; the unlit kernel has registers to spare and is
timed at 3 only), the tile queue either one queue over the images row by row or one queue per
XCD holding each image's Morton-ordered super-tiles, the camera order largest or smallest image
first, and the brick layout which packing of the same hierarchy is read (when the caller passes
several).  The cache is a JSON file (default: autotune_cache.json next to this module) keyed by
"<device name>|<workload key>"."""
from __future__ import annotations

import json
import os

import torch

from . import render

CANDIDATE_TILES = [(8, 8), (16, 4), (4, 16), (32, 2)]
CANDIDATE_BPC = [1, 2, 4, 8]
CANDIDATE_WPS = [2, 3]
CANDIDATE_XCD = [0, 1]
CANDIDATE_ORDER = [0, 1]
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def device_key() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s-%s-%dcu" % (p.name, getattr(p, "gcnArchName", ""), p.multi_processor_count)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def candidates(layouts=(None,), lit=True):
    """Every (tile_w, tile_h, blocks_per_cu, waves_per_simd, xcd_tiles, queue_order, layout) the tuner
    times."""
    wps = CANDIDATE_WPS if lit else [3]
    return [(tw, th, bpc, w, x, o, lay) for lay in layouts for (tw, th) in CANDIDATE_TILES for bpc in CANDIDATE_BPC
            for w in wps for x in CANDIDATE_XCD for o in CANDIDATE_ORDER]


def tune(scene, cams, lut, params, d_cams, queue, out, workload_key: str, reps: int = 3,
         cache_path: str = DEFAULT_CACHE, force: bool = False, scenes: dict | None = None) -> dict:
    """Returns {"tile_w", "tile_h", "blocks_per_cu", "waves_per_simd", "xcd_tiles", "queue_order",
    "brick_layout", "ms", "table"} for the fastest candidate.  `scenes` (optional): {brick layout: scene} packings of the same hierarchy to
    search as well; otherwise `scene` alone (its own layout)."""
    key = device_key() + "|" + workload_key
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not force:
        return cache[key]
    pool = scenes if scenes else {int(scene.scene.brick_layout): scene}
    table = []
    lit = int(params.get("lighting", 0)) == 1
    for (tw, th, bpc, w, x, o, lay) in candidates(tuple(sorted(pool)), lit):
        prm = dict(params, persistent=1, tile_w=tw, tile_h=th, blocks_per_cu=bpc, waves_per_simd=w, xcd_tiles=x,
                   queue_order=o)
        sc = pool[lay]

        def run():
            render(sc, cams, lut, prm, out=out, d_cams=d_cams, d_queue=queue)
        ms = _time(run, reps)
        table.append(dict(tile_w=tw, tile_h=th, blocks_per_cu=bpc, waves_per_simd=w, xcd_tiles=x, queue_order=o,
                          brick_layout=lay, ms=round(ms, 4)))
    best = min(table, key=lambda r: r["ms"])
    res = dict(best, table=table)
    cache[key] = res
    tmp = cache_path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return res
