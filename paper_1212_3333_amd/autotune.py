"""Autotuner for the persistent multi-camera kernel: times every (tile shape, blocks per CU)
candidate on the caller's scene and cameras and caches the fastest per device and workload.

The cache is a JSON file (default: autotune_cache.json next to this module) keyed by
"<device name>|<workload key>"."""
from __future__ import annotations

import json
import os

import torch

from . import render

CANDIDATE_TILES = [(8, 8), (16, 4), (4, 16), (32, 2)]
CANDIDATE_BPC = [1, 2, 4, 8]
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


def tune(scene, cams, lut, params, d_cams, queue, out, workload_key: str, reps: int = 3,
         cache_path: str = DEFAULT_CACHE, force: bool = False) -> dict:
    """Returns {"tile_w", "tile_h", "blocks_per_cu", "ms", "table"} for the fastest candidate."""
    key = device_key() + "|" + workload_key
    cache = {}
    if os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if key in cache and not force:
        return cache[key]
    table = []
    for (tw, th) in CANDIDATE_TILES:
        for bpc in CANDIDATE_BPC:
            prm = dict(params, persistent=1, tile_w=tw, tile_h=th, blocks_per_cu=bpc)

            def run():
                render(scene, cams, lut, prm, out=out, d_cams=d_cams, d_queue=queue)
            ms = _time(run, reps)
            table.append(dict(tile_w=tw, tile_h=th, blocks_per_cu=bpc, ms=round(ms, 4)))
    best = min(table, key=lambda r: r["ms"])
    res = dict(best, table=table)
    cache[key] = res
    tmp = cache_path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, cache_path)
    return res
