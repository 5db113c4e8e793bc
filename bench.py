"""Benchmark: single-pass AMR raycasting on one MI355X.

One step = one frame of the hot path: ray generation, kD-restart traversal, per-leaf sampling,
trilinear sampling from the HBM pool, LUT classification, gradient lighting with taps located
across patches, front-to-back compositing with early termination (one amr_render launch).
Hierarchy validation, the kD build and the pool packing run once before the timed region and
are reported as preprocessing seconds, as in the paper's tables.

Workload (default): the cosmology-like hierarchy (root 128^3, 6 levels, r = 2, ~2000 patches of
8^3..64^3 around peaks of a seeded log-normal density, ~1.5 GB pool), one 1024x1024 perspective
view, gradient lighting on, plain traversal.

Prints one JSON line (rank 0).  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "samples/s + Mrays/s at 1024², plain vs learned-skip at ≤1e-3 RGBA error"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def popcount_bytes(bitmap_u8):
    import torch
    table = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64, device=bitmap_u8.device)
    return int(table[bitmap_u8.long()].sum().item())


def time_frames(amr, scene, cam, lut_t, prm, steps, warmup, out):
    import torch
    for _ in range(warmup):
        amr.render(scene, cam, lut_t, prm, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        amr.render(scene, cam, lut_t, prm, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(h, cam, lut, prm, target_s=15.0, seed=7):
    """The FP64 oracle as it stands, on a random pixel sample of the same view."""
    import oracle
    t = time.time()
    O = oracle.Oracle(h)
    setup = time.time() - t
    rng = np.random.default_rng(seed)
    W, H = cam["width"], cam["height"]
    probe = np.stack([rng.integers(0, W, 256), rng.integers(0, H, 256)], 1).astype(np.int32)
    O.render(cam, prm, lut, pixels=probe)            # builds the ghost layers it touches
    t = time.time()
    r = O.render(cam, prm, lut, pixels=probe)
    dt = max(time.time() - t, 1e-3)
    n = int(min(W * H, max(256, 256 * target_s / dt)))
    pix = np.stack([rng.integers(0, W, n), rng.integers(0, H, n)], 1).astype(np.int32)
    O.render(cam, prm, lut, pixels=pix[: min(n, 4096)])
    t = time.time()
    r = O.render(cam, prm, lut, pixels=pix)
    dt = time.time() - t
    samples = int(r["nsamp"].sum())
    return dict(value=samples / dt, unit="samples/s", cores=oracle.num_threads(), kind="oracle",
                mrays_per_s=n / dt / 1e6,
                sample="%d random pixels of the same %dx%d view (seed %d), %.1f s of oracle work after a "
                       "warm-up pass that fills the oracle's lazily built ghost layers; oracle tree build %.1f s"
                       % (n, W, H, seed, dt, setup),
                seconds=dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-touch", action="store_true", help="skip the compulsory-bytes measurement run")
    ap.add_argument("--unlit", action="store_true", help="time the unlit kernel instead")
    ap.add_argument("--copy-calib", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build renders on one GPU only (the multi-GPU design is described in DESIGN.md); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1212_3333_amd as amr
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.time()
    h, lut, cam, prm = workloads.config2(args.seed)
    gen_s = time.time() - t
    if args.unlit:
        prm = dict(prm, lighting=False)
    log("generated %d patches, %.2f GB of cells in %.1f s" % (len(h.patches), h.nbytes_cells() / 1e9, gen_s))
    t = time.time()
    tree = amr.build_tree(h)
    build_s = time.time() - t
    t = time.time()
    scene = amr.pack(tree, h, device=dev)
    torch.cuda.synchronize()
    pack_s = time.time() - t
    info = tree.info()
    log("tree: %d nodes, %d leaves, depth %d; build %.3f s, pack+upload %.2f s" % (
        info["nodes"], info["leaves"], info["depth"], build_s, pack_s))
    lut_t = torch.from_numpy(lut).to(dev)
    W, H = cam["width"], cam["height"]
    out = torch.empty(W * H * 4, dtype=torch.float32, device=dev)

    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst

    # counts (separate run, so timing is unperturbed)
    res = amr.render(scene, cam, lut_t, prm, stats=True)
    torch.cuda.synchronize()
    st = amr.stats_dict(res)
    log("stats:", st)

    ms = time_frames(amr, scene, cam, lut_t, prm, args.steps, args.warmup, out)
    log("render %.3f ms/frame" % ms)
    samples = st["samples"]
    value = samples / (ms * 1e-3)
    mrays = W * H / (ms * 1e-3) / 1e6

    # compulsory bytes: distinct pool cells the frame's stencils read + tree/leaf/header tables
    # + the RGBA output
    roof = None
    if not args.no_touch:
        nwords = scene.scene.pool_bytes // 4 // 32 + 1
        touch = torch.zeros(nwords, dtype=torch.int32, device=dev)
        amr.render(scene, cam, lut_t, prm, d_touch=touch)
        torch.cuda.synchronize()
        cells = popcount_bytes(touch.view(torch.uint8))
        b_alg = 4 * cells + scene.scene.meta_bytes + 16 * W * H
        achieved = b_alg / (ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=None,
                    kernel="render_fwd", algorithmic_bytes=int(b_alg), distinct_cells=int(cells),
                    gather_request_bytes=int(samples * (32 + (192 if prm["lighting"] else 0))))
        log("compulsory bytes %.1f MB (%d distinct cells)" % (b_alg / 1e6, cells))
        del touch

    # the unlit kernel, as a second line of context
    unlit_ms = None
    if prm["lighting"]:
        unlit_ms = time_frames(amr, scene, cam, lut_t, dict(prm, lighting=False), max(3, args.steps // 2), 2, out)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)...")
        cpu = cpu_baseline(h, cam, lut, prm)
        log("oracle: %.3g samples/s on %d threads" % (cpu["value"], cpu["cores"]))

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cosmology-like SAMR: root 128^3, 6 levels, r=2, %d patches 8^3..64^3 around peaks of a "
                        "seeded log-normal density (sigma_ln=2), %.2f GB pool; 1024x1024 perspective view, "
                        "gradient lighting %s, plain traversal" % (len(h.patches), scene.scene.pool_bytes / 1e9,
                                                                 "on" if prm["lighting"] else "off"),
            "width": W, "height": H, "patches": len(h.patches), "nodes": info["nodes"], "leaves": info["leaves"],
            "pool_bytes": int(scene.scene.pool_bytes), "lighting": bool(prm["lighting"]),
            "step_frac": prm["step_frac"], "t_min": prm["t_min"],
        },
        "mrays_per_s": round(mrays, 3),
        "samples_per_frame": int(samples),
        "segments_per_frame": int(st["segments"]),
        "tap_descents_per_frame": int(st["tap_descents"]),
        "unlit_ms_per_step": round(unlit_ms, 4) if unlit_ms else None,
        "preprocess_s": {"generate": round(gen_s, 2), "build": round(build_s, 4), "pack_upload": round(pack_s, 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "learned_skip": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
