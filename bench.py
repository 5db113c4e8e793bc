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
FP32_PEAK_TFLOPS = 157.3
# VALU issue: each of a CU's 4 SIMDs issues one wave64 vector instruction every 4 cycles, so the
# chip issues 256 CUs x 2.4 GHz wave instructions per second
VALU_ISSUE_PEAK = 256 * 2.4e9
# algorithmic fp32 operations per sample (counted in the design notes): position, trilinear,
# value normalisation, LUT lerp, opacity, compositing; lit adds the six taps' trilinears on the
# centre's weights, the central differences and the shading
FLOPS_PER_SAMPLE = {False: 59, True: 206}
# gather request bytes per sample: 8 cells, plus 6 taps of 8 cells each when lit
GATHER_BYTES_PER_SAMPLE = {False: 32, True: 32 + 192}
# the sources of the timed kernels and the script that compiles them (its flags change the code);
# committed counter readings are used only while these match
KERNEL_SOURCES = ("paper_1212_3333_amd/csrc/amr_render.hip", "paper_1212_3333_amd/csrc/amr_render_common.h",
                  "paper_1212_3333_amd/csrc/amr_internal.h", "paper_1212_3333_amd/build.py")
COUNTERS_FILE = "profiles/render_fwd_cosmology_1024_counters.txt"


def kernel_source_hash() -> str:
    import hashlib
    hsh = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def committed_counters():
    """Per-launch counter readings of the timed kernels from the committed rocprofv3 summary:
    HBM bytes (FETCH_SIZE and WRITE_SIZE, each scaled by a copy kernel's reading), the raw
    FETCH_SIZE bytes, and VALU instructions, for the lit and the unlit kernel; None when the
    summary is missing or the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, COUNTERS_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return {lit: dict(traffic=int(float(kv[p + "traffic_bytes_per_launch"])),
                          fetch_raw=int(float(kv[p + "fetch_kib_per_dispatch"]) * 1024),
                          valu_insts=float(kv[p + "valu_insts_per_dispatch"]))
                for lit, p in ((True, "lit_"), (False, "unlit_"))}
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


METRIC = "samples/s + Mrays/s at 1024², plain vs learned-skip at ≤1e-3 RGBA error"
# The paper's own measurements (its results table and Section 6), on other hardware and data:
# context for the numbers above, not a baseline of the same workload.
PAPER_CONTEXT = {
    "hardware": "NVIDIA GeForce GTX 680 (2 GB), OpenGL/GLSL fragment shaders, Xeon E5520 host",
    "view": "1000x1000, emission-absorption, no early ray termination",
    "datasets": "three Enzo AMR snapshots: 2,666 / 18,528 / 39,061 grids; 19 M / 33 M / 140 M cells",
    "packing_fps": [3.2, 1.6, 1.2],
    "packing_mrays_per_s_at_most": [3.2, 1.6, 1.2],
    "gradient_shaded_isosurface_fps_dataset3": 0.8,
    "point_light_secondary_rays_fps_dataset3": 0.1,
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def popcount_bytes(bitmap_u8):
    import torch
    table = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64, device=bitmap_u8.device)
    return int(table[bitmap_u8.long()].sum().item())


def time_frames(amr, scene, cam, lut_t, prm, steps, warmup, out, first=None):
    """Mean ms per frame over `steps` frames after `warmup`, with a tile schedule of its own (each
    frame renders its tiles longest first by the previous frame's tile times; the order changes
    no pixel; the point light's passes take none).  first: a dict that receives the first frame's
    time, rendered in the default order (a fresh schedule), as after a change of view."""
    import torch
    sch = amr.Schedule(cam, out.device).params() if int(prm.get("lighting", 0)) != 2 else {}
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    amr.render(scene, cam, lut_t, prm, out=out, **sch)
    e1.record(stream)
    torch.cuda.synchronize()
    if first is not None:
        first["ms"] = e0.elapsed_time(e1)
    for _ in range(warmup):
        amr.render(scene, cam, lut_t, prm, out=out, **sch)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        amr.render(scene, cam, lut_t, prm, out=out, **sch)
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
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                mrays_per_s=n / dt / 1e6,
                sample="%d random pixels of the same %dx%d view (seed %d), %.1f s of oracle work after a "
                       "warm-up pass that fills the oracle's lazily built ghost layers; oracle tree build %.1f s"
                       % (n, W, H, seed, dt, setup),
                seconds=dt)


def next_rows_section(amr, dev, scene, h, cam, lut_t, prm, steps, out, seed):
    """The widened rows on the same view: nearest-cell sampling, the level-of-detail cut at
    kind-(a) nodes (2 pixels), secondary rays to a point light (light at the domain centre; the
    job arrays of the secondary-ray pass in a workspace sized for the frame's samples, allocated
    before the timed frames), out-of-core residency and vertex-centred data (the same boxes with
    samples at the grid vertices)."""
    import torch
    import workloads
    res = {}

    def stats_of(scn, c, p):
        r = amr.render(scn, c, lut_t, p, stats=True)
        torch.cuda.synchronize()
        return amr.stats_dict(r)

    unlit = dict(prm, lighting=False)
    near = dict(prm, interp=1)
    res["nearest"] = dict(lit_ms=round(time_frames(amr, scene, cam, lut_t, near, steps, 2, out), 4),
                          unlit_ms=round(time_frames(amr, scene, cam, lut_t, dict(near, lighting=False), steps, 2, out), 4),
                          samples_per_frame=int(stats_of(scene, cam, near)["samples"]))
    lod = dict(prm, lod=2.0)
    st = stats_of(scene, cam, lod)
    res["lod"] = dict(lod_pixels=2.0, lit_ms=round(time_frames(amr, scene, cam, lut_t, lod, steps, 2, out), 4),
                      samples_per_frame=int(st["samples"]), segments_per_frame=int(st["segments"]))
    pl = dict(prm, lighting=2, light=(0.5, 0.5, 0.5))
    st = stats_of(scene, cam, pl)
    pl = dict(pl, light_jobs=int(st["samples"]))
    st = stats_of(scene, cam, pl)
    ms_pl = time_frames(amr, scene, cam, lut_t, pl, 3, 1, out)
    res["point_light"] = dict(width=cam["width"], height=cam["height"], light=[0.5, 0.5, 0.5], ms=round(ms_pl, 4),
                              primary_samples_per_frame=int(st["samples"]), light_jobs=int(pl["light_jobs"]),
                              samples_traced_inline=int(st["light_inline"]),
                              secondary_rays_per_s=round(st["samples"] / (ms_pl * 1e-3), 1))
    res["out_of_core"] = out_of_core_section(amr, dev, scene, h, cam, lut_t, prm, steps, out)
    t = time.time()
    hv, _, _, _ = workloads.cosmology_vertex_view(seed)
    gen_s = time.time() - t
    t = time.time()
    tv = amr.build_tree(hv)
    sv = amr.pack(tv, hv, device=dev, brick_layout=2)
    torch.cuda.synchronize()
    pack_s = time.time() - t
    st = stats_of(sv, cam, prm)
    res["vertex_centred"] = dict(lit_ms=round(time_frames(amr, sv, cam, lut_t, prm, steps, 2, out), 4),
                                 unlit_ms=round(time_frames(amr, sv, cam, lut_t, unlit, steps, 2, out), 4),
                                 samples_per_frame=int(st["samples"]), pool_bytes=int(sv.scene.pool_bytes),
                                 generate_s=round(gen_s, 2), build_pack_upload_s=round(pack_s, 2))
    del sv
    torch.cuda.empty_cache()
    log("next rows:", res)
    return res


def out_of_core_section(amr, dev, scene, h, cam, lut_t, prm, steps, out, frac=0.3, frames=8):
    """Per-subgrid residency: a brick cache of `frac` of all bricks, an 8-frame orbit through
    the benchmark view where each frame selects its subset (90% of the cache) and updates the
    cache incrementally, then renders lit at 1024^2.  Reports the host update time, the bytes
    uploaded per frame, the render time, and the last frame's error against the render with
    every brick resident."""
    import torch
    t = time.time()
    st = amr.Store(scene.tree, h, brick_layout=2)
    create_s = time.time() - t
    info = st.info()
    cap = int(frac * info["full_cache_bytes"]) // 256 * 256
    cache, meta = st.alloc(cap, device=dev)
    upd_ms, up_b, ren_ms, remapped = [], [], [], []
    for k in range(frames):
        c = dict(cam) if k == frames - 1 else workloads_orbit(cam, k, frames)
        t = time.time()
        mask = st.select(c, int(0.9 * cap))
        sc, rep = st.update(mask, cache, meta)
        torch.cuda.synchronize()
        upd_ms.append(1e3 * (time.time() - t))
        up_b.append(rep["uploaded_bytes"])
        remapped.append(rep["remapped_leaves"])
        ren_ms.append(time_frames(amr, sc, c, lut_t, prm, max(2, steps // 2), 1, out))
    img = out.view(-1, 4).clone()
    ref = torch.empty_like(out)
    time_frames(amr, scene, cam, lut_t, prm, 1, 0, ref)
    err = float((img - ref.view(-1, 4)).abs().max().item())
    res = dict(cache_bytes=cap, full_bytes=int(info["full_cache_bytes"]), frames=frames,
               store_create_s=round(create_s, 2), first_upload_bytes=int(up_b[0]),
               mean_upload_bytes_after_first=int(np.mean(up_b[1:])), mean_update_ms_after_first=round(float(np.mean(upd_ms[1:])), 2),
               first_update_ms=round(upd_ms[0], 2), mean_render_ms=round(float(np.mean(ren_ms)), 4),
               remapped_leaves_last=int(remapped[-1]), max_rgba_err_vs_all_resident=err)
    del cache, meta, st
    torch.cuda.empty_cache()
    return res


def workloads_orbit(cam, k, frames):
    """Camera k of a short orbit ending at the benchmark view (same radius, fov, size)."""
    import workloads
    import math as _m
    eye = np.asarray(cam["eye"], np.float64)
    rel = eye - 0.5
    r = float(np.linalg.norm(rel))
    az = _m.atan2(rel[0], -rel[2]) - 0.12 * (frames - 1 - k)
    el = _m.asin(rel[1] / r)
    fov = 2.0 * _m.degrees(_m.atan(cam["tan_half_fov"]))
    c = workloads.perspective_orbit(cam["width"], cam["height"], az, el, radius=r, fov_deg=fov)
    return c


def batched_section(amr, dev, scene, lut_t, prm):
    """Serving batch on the same hierarchy: 64 orbit cameras with resolutions from {256^2, 512^2,
    768^2, 1024^2} in one persistent launch (tile shape, blocks per CU and tile queue from the
    autotuner), captured in a hipGraph and replayed; per-image latency from the kernel's
    completion stamps, for the tuned camera order and the other one."""
    import tempfile
    import torch
    import workloads
    from paper_1212_3333_amd import autotune
    cams = workloads.serving_cameras(0, 64)
    dc = amr.camera_table(cams, device=dev)
    q = amr.queue_buffer(len(cams), device=dev)
    npix = sum(c["width"] * c["height"] for c in cams)
    out = torch.zeros(npix * 4, dtype=torch.float32, device=dev)
    with tempfile.TemporaryDirectory() as td:
        best = autotune.tune(scene, cams, lut_t, prm, dc, q, out, workload_key="serving64", reps=1,
                             cache_path=td + "/tune.json")
    stamps = torch.zeros(len(cams) + 1, dtype=torch.int64, device=dev)
    khz = amr.wall_clock_khz()

    def replayed(order):
        """The tuned launch with cameras largest (0) or smallest (1) first, captured in a hipGraph
        and replayed three times: per-image latency from the stamps, aggregate Mrays/s."""
        bprm = dict(prm, persistent=1, tile_w=best["tile_w"], tile_h=best["tile_h"],
                    blocks_per_cu=best["blocks_per_cu"], waves_per_simd=best["waves_per_simd"],
                    xcd_tiles=best["xcd_tiles"], queue_order=order)
        amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q, d_stamps=stamps)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                amr.render(scene, cams, lut_t, bprm, out=out, d_cams=dc, d_queue=q, d_stamps=stamps)
        lat, agg = [], []
        for _ in range(3):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            sv = stamps.cpu().numpy()
            lat.append((sv[:-1] - sv[-1]) / khz)
            agg.append(npix / (e0.elapsed_time(e1) * 1e-3) / 1e6)
        lat = np.concatenate(lat)
        del g
        return dict(aggregate_mrays_per_s=round(float(np.median(agg)), 2),
                    latency_ms_p50=round(float(np.percentile(lat, 50)), 2),
                    latency_ms_p99=round(float(np.percentile(lat, 99)), 2))
    tuned = replayed(best["queue_order"])
    other = replayed(1 - best["queue_order"])
    res = dict(cameras=len(cams), rays=int(npix), tile_w=int(best["tile_w"]), tile_h=int(best["tile_h"]),
               blocks_per_cu=int(best["blocks_per_cu"]), waves_per_simd=int(best["waves_per_simd"]),
               xcd_tiles=int(best["xcd_tiles"]),
               queue_order="smallest first" if best["queue_order"] else "largest first",
               tuned_ms=best["ms"], candidates=len(best["table"]), **tuned,
               other_order=other)
    del out
    torch.cuda.empty_cache()
    return res


def adjoint_section(amr, dev, scene, h, steps=200):
    """Transfer-function fit on the same hierarchy: 8 orbit cameras at 512^2, lit, Adam (lr 1e-2)
    on the LUT through the checkpointed forward and the adjoint kernel, toward images rendered
    with a hidden target LUT.  Reports the time per optimisation step (forward + backward of all
    eight images) and the loss after `steps` steps.  The steps share a tile schedule: every
    forward starts the cameras' tiles longest first by the previous step's tile times."""
    import torch
    import workloads
    _, cams, target, start, prm = workloads.tf_fit(0, h=h)
    sh = torch.tensor([1.0, 1.0, 1.0, 0.3, 0.7], dtype=torch.float32)
    with torch.no_grad():
        tgt = amr.render(scene, cams, torch.from_numpy(target).to(dev), prm)["rgba"].clone()
    lut = torch.from_numpy(start).to(dev).requires_grad_(True)
    opt = torch.optim.Adam([lut], lr=1e-2)
    losses = []
    sched = amr.Schedule(cams, dev)

    def step():
        opt.zero_grad()
        rgba = amr.AMRRender.apply(lut, sh, scene, cams, prm, 4, 16, False, sched)
        loss = ((rgba - tgt) ** 2).mean()
        loss.backward()
        opt.step()
        with torch.no_grad():
            lut.clamp_(min=0.0)
        return loss
    for _ in range(3):
        losses.append(float(step().item()))
    torch.cuda.synchronize()
    t = time.time()
    for _ in range(steps - 3):
        last = step()
    torch.cuda.synchronize()
    ms = (time.time() - t) * 1e3 / (steps - 3)
    losses.append(float(last.item()))
    return dict(cameras=len(cams), width=512, height=512, steps=steps, ms_per_step=round(ms, 3),
                loss_first=losses[0], loss_last=losses[-1], tile_schedule=True)


def learned_skip_section(amr, dev, steps, warmup):
    """Deep-range hierarchy (20 levels) at 1024^2 (and 2048^2, the hierarchy's own view size):
    plain traversal vs learned segment proposals.  The network is trained on the GPU from
    segments logged by the plain kernel on 16 views and its thresholds calibrated on 6 held-out
    views (worst RGBA error <= 0.5e-3 there); the timed view is the full-domain one."""
    import torch
    import workloads
    from paper_1212_3333_amd import learned
    t = time.time()
    h, lut, cams, prm = workloads.deep_range_scene(0, res=1024)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device=dev)
    lut_t = torch.from_numpy(lut).to(dev)
    torch.cuda.synchronize()
    prep = time.time() - t
    t = time.time()
    X, alpha, t_in, met = learned.log_segments(scene, workloads.deep_range_orbits(h, 16, 1, 192), lut_t, prm)
    W, losses = learned.train(X, alpha, steps=500, batch=65536, lr=3e-3)
    net = learned.ProposalMLP(W)
    held = workloads.deep_range_orbits(h, 6, 2, 192)
    plain_held = [amr.render(scene, c, lut_t, prm)["rgba"].clone() for c in held]
    te, ts, table = learned.calibrate(scene, held, lut_t, prm, net.packed, plain_held, max_err=1e-3)
    tb, table_b = learned.calibrate_bound_only(scene, held, lut_t, prm, plain_held, max_err=1e-3)
    torch.cuda.synchronize()
    train_s = time.time() - t
    cam = cams[0]
    W_, H_ = cam["width"], cam["height"]

    def timed(c, prm_x, **kw):
        out = torch.empty(c["width"] * c["height"] * 4, dtype=torch.float32, device=dev)
        for _ in range(warmup):
            amr.render(scene, c, lut_t, prm_x, out=out, **kw)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            amr.render(scene, c, lut_t, prm_x, out=out, **kw)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def form(c, prm_x, plain_img, **kw):
        """Time, counters and error against the plain image of one form of the render."""
        r = amr.render(scene, c, lut_t, prm_x, stats=True, **kw)
        st = amr.stats_dict(r)
        err = float((r["rgba"] - plain_img).abs().max().item())
        del r
        return dict(ms=round(timed(c, prm_x, **kw), 4), samples=st["samples"], segments=st["segments"],
                    skipped_segments=st["skipped_segments"], net_segments=st["net_segments"],
                    coarse_segments=st["coarse_segments"], max_rgba_err_vs_plain=err)

    def compare(c):
        """Plain, learned (bound + network, its calibrated thresholds), bound-only at its own
        calibrated threshold and bound-only at the network's threshold, on camera c."""
        p_res = amr.render(scene, c, lut_t, prm, stats=True)
        p_stats, plain_img = amr.stats_dict(p_res), p_res["rgba"].clone()
        del p_res
        res = dict(plain=dict(ms=round(timed(c, prm), 4), samples=p_stats["samples"], segments=p_stats["segments"]))
        res["learned"] = form(c, dict(prm, tau_e=te, tau_s=ts), plain_img, d_mlp=net.packed)
        res["bound_only"] = form(c, dict(prm, tau_e=tb, tau_s=0.0, bound_only=1), plain_img)
        res["bound_only_at_learned_tau"] = form(c, dict(prm, tau_e=te, tau_s=0.0, bound_only=1), plain_img)
        return res

    r1 = compare(cam)
    r2 = compare(dict(cam, width=2048, height=2048))
    ms_p, ms_l, p_stats, l_stats, err = (r1["plain"]["ms"], r1["learned"]["ms"], r1["plain"],
                                         r1["learned"], r1["learned"]["max_rgba_err_vs_plain"])
    ms_p2, ms_l2 = r2["plain"]["ms"], r2["learned"]["ms"]
    log("learned skip: plain %.3f ms, learned %.3f ms, bound-only %.3f ms, err %.2e, tau_e %g tau_s %g (bound-only "
        "tau_e %g); 2048^2: %.3f / %.3f / %.3f ms" % (ms_p, ms_l, r1["bound_only"]["ms"], err, te, ts, tb, ms_p2, ms_l2,
                                                     r2["bound_only"]["ms"]))

    def forms(r):
        """The bound-only rows of one resolution, with their speed-up over plain."""
        out = {}
        for k in ("bound_only", "bound_only_at_learned_tau"):
            out[k] = dict(r[k], speedup=round(r["plain"]["ms"] / r[k]["ms"], 3))
        out["network_fewer_samples_than_bound_at_same_tau"] = int(r["bound_only_at_learned_tau"]["samples"] -
                                                                  r["learned"]["samples"])
        return out
    return {
        "workload": "deep-range SAMR: root 64^3, 20 levels, r=2, %d patches around 3 power-law cores; 1024x1024 "
                    "full-domain view, unlit" % len(h.patches),
        "plain_ms": round(ms_p, 4), "learned_ms": round(ms_l, 4), "speedup": round(ms_p / ms_l, 3),
        "plain_samples_per_s": round(p_stats["samples"] / (ms_p * 1e-3), 1),
        "learned_samples_per_s": round(l_stats["samples"] / (ms_l * 1e-3), 1),
        "plain_equivalent_samples_per_s": round(p_stats["samples"] / (ms_l * 1e-3), 1),
        "plain_mrays_per_s": round(W_ * H_ / (ms_p * 1e-3) / 1e6, 3),
        "learned_mrays_per_s": round(W_ * H_ / (ms_l * 1e-3) / 1e6, 3),
        "max_rgba_err_vs_plain": err, "tau_e": te, "tau_s": ts,
        "skipped_segments": l_stats["skipped_segments"], "coarse_segments": l_stats["coarse_segments"],
        "net_segments": l_stats["net_segments"], "segments": l_stats["segments"],
        "plain_samples": p_stats["samples"], "learned_samples": l_stats["samples"],
        "bound_only_tau_e": tb, **forms(r1),
        "train_segments": int(X.shape[0]), "train_calibrate_s": round(train_s, 2), "prepare_s": round(prep, 2),
        "at_2048": {"plain_ms": round(ms_p2, 4), "learned_ms": round(ms_l2, 4), "speedup": round(ms_p2 / ms_l2, 3),
                    "plain_mrays_per_s": round(2048 * 2048 / (ms_p2 * 1e-3) / 1e6, 3),
                    "learned_mrays_per_s": round(2048 * 2048 / (ms_l2 * 1e-3) / 1e6, 3),
                    "plain_samples": r2["plain"]["samples"], "learned_samples": r2["learned"]["samples"],
                    "segments": r2["plain"]["segments"],
                    "max_rgba_err_vs_plain": r2["learned"]["max_rgba_err_vs_plain"], **forms(r2)},
    }


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
    ap.add_argument("--brick-layout", type=int, default=2,
                    help="pool layout: 0 linear bricks, 1 4^3 micro-bricks, 2 halo rows (row loads from "
                         "4^3-cell blocks: the fastest, and a quarter of the linear layout's HBM traffic)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-skip section")
    ap.add_argument("--no-next", action="store_true", help="skip the widened-rows section")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the renderer runs on one GPU per process and this benchmark measures one GPU; "
              "multi-GPU runs are not supported, use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1212_3333_amd as amr
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.time()
    h, lut, cam, prm = workloads.cosmology_view(args.seed)
    gen_s = time.time() - t
    if args.unlit:
        prm = dict(prm, lighting=False)
    log("generated %d patches, %.2f GB of cells in %.1f s" % (len(h.patches), h.nbytes_cells() / 1e9, gen_s))
    t = time.time()
    tree = amr.build_tree(h)
    build_s = time.time() - t
    t = time.time()
    scene = amr.pack(tree, h, device=dev, brick_layout=args.brick_layout)
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

    first = {}
    ms = time_frames(amr, scene, cam, lut_t, prm, args.steps, args.warmup, out, first)
    log("render %.3f ms/frame (first frame, default tile order: %.3f ms)" % (ms, first["ms"]))
    samples = st["samples"]
    value = samples / (ms * 1e-3)
    mrays = W * H / (ms * 1e-3) / 1e6

    # the unlit kernel: timed, and its own roofline below
    unlit_prm = dict(prm, lighting=False)
    unlit_ms = unlit_samples = None
    if prm["lighting"]:
        unlit_first = {}
        unlit_ms = time_frames(amr, scene, cam, lut_t, unlit_prm, max(3, args.steps // 2), 2, out, unlit_first)
        r = amr.render(scene, cam, lut_t, unlit_prm, stats=True)
        torch.cuda.synchronize()
        unlit_samples = amr.stats_dict(r)["samples"]
        del r

    # compulsory bytes of each kernel: distinct pool cells its stencils read, the node, leaf,
    # patch-header and face records it reads, and the RGBA output; then the floors each roof
    # sets on the frame time, from the live timing, the live L2 probe and the committed counters
    roof = unlit_roof = None
    if not args.no_touch:
        l2_gbs = amr.read_bandwidth(16 << 20, 250, device=dev)
        log("L2 read bandwidth (16 MB probe): %.0f GB/s" % l2_gbs)
        counters = committed_counters()
        # counted on a linear-layout copy of the pool, where every padded cell is one float: the
        # halo-row layout stores edge cells twice, and which copy a stencil reads is a layout detail
        tscene = scene if args.brick_layout == 0 else amr.pack(tree, h, device=dev, brick_layout=0)

        def touched(p):
            touch = torch.zeros(tscene.scene.pool_bytes // 4 // 32 + 1, dtype=torch.int32, device=dev)
            tmeta = torch.zeros(tscene.scene.meta_bytes // 16 // 32 + 1, dtype=torch.int32, device=dev)
            amr.render(tscene, cam, lut_t, p, d_touch=touch, d_touch_meta=tmeta)
            torch.cuda.synchronize()
            cells = popcount_bytes(touch.view(torch.uint8))
            lines = int((touch != 0).sum().item())      # 128-byte lines (32 cells) holding a read cell
            meta = 16 * popcount_bytes(tmeta.view(torch.uint8))
            return cells, lines, meta

        def roofline_of(lit, t_ms, nsamp, cells, lines, meta):
            b_alg = 4 * cells + meta + 16 * W * H
            achieved = b_alg / (t_ms * 1e-3) / 1e9
            gather = nsamp * GATHER_BYTES_PER_SAMPLE[lit]
            flops = nsamp * FLOPS_PER_SAMPLE[lit]
            c = counters[lit] if counters else None
            floors = {"hbm": b_alg / (HBM_PEAK_GBS * 1e9) * 1e3,
                      "l2_gather": gather / (l2_gbs * 1e9) * 1e3,
                      "fp32_alu": flops / (FP32_PEAK_TFLOPS * 1e12) * 1e3}
            if c:
                floors["valu_issue"] = c["valu_insts"] / VALU_ISSUE_PEAK * 1e3
            binding = max(floors, key=floors.get)
            return dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 5), traffic=c["traffic"] if c else None,
                        kernel="render_fwd<%s, REC=false, NEAR=false, LAY=%d>" % ("LIT" if lit else "UNLIT",
                                                                                  args.brick_layout),
                        ms=round(t_ms, 4), algorithmic_bytes=int(b_alg), distinct_cells=int(cells),
                        metadata_bytes_read=int(meta), distinct_line_bytes=128 * lines,
                        gather_request_bytes=int(gather), algorithmic_flops=int(flops),
                        counter_gbs=round(c["traffic"] / (t_ms * 1e-3) / 1e9, 1) if c else None,
                        fetch_bytes_raw=c["fetch_raw"] if c else None,
                        line_efficiency=round(b_alg / c["traffic"], 4) if c else None,
                        valu_insts=c["valu_insts"] if c else None,
                        l2_read_gbs=round(l2_gbs, 1),
                        floors_ms={k: round(v, 4) for k, v in floors.items()},
                        binding_roof=binding, frac_of_binding_roof=round(floors[binding] / t_ms, 4))

        cells, lines, meta = touched(prm)
        roof = roofline_of(bool(prm["lighting"]), ms, samples, cells, lines, meta)
        log("compulsory bytes %.1f MB (%d distinct cells, %d metadata bytes read); floors %s" % (
            roof["algorithmic_bytes"] / 1e6, cells, meta, roof["floors_ms"]))
        if prm["lighting"]:
            cu, lu, mu = touched(unlit_prm)
            unlit_roof = roofline_of(False, unlit_ms, unlit_samples, cu, lu, mu)
            log("unlit: compulsory bytes %.1f MB; floors %s" % (unlit_roof["algorithmic_bytes"] / 1e6,
                                                              unlit_roof["floors_ms"]))
        if tscene is not scene:
            del tscene
            torch.cuda.empty_cache()

    pool_bytes, meta_bytes = int(scene.scene.pool_bytes), int(scene.scene.meta_bytes)
    batched_res = adjoint_res = None
    if not args.no_next:
        batched_res = batched_section(amr, dev, scene, lut_t, prm)
        log("batched:", batched_res)
        adjoint_res = adjoint_section(amr, dev, scene, h)
        log("adjoint:", adjoint_res)
    next_res = None
    if not args.no_next:
        next_res = next_rows_section(amr, dev, scene, h, cam, lut_t, prm, max(3, args.steps // 2), out, args.seed)
    learned_res = None
    if not args.no_learned:
        del scene
        torch.cuda.empty_cache()
        learned_res = learned_skip_section(amr, dev, max(3, args.steps // 2), 2)

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
                        "gradient lighting %s, plain traversal" % (len(h.patches), pool_bytes / 1e9,
                                                                 "on" if prm["lighting"] else "off"),
            "width": W, "height": H, "patches": len(h.patches), "nodes": info["nodes"], "leaves": info["leaves"],
            "pool_bytes": pool_bytes, "lighting": bool(prm["lighting"]),
            "step_frac": prm["step_frac"], "t_min": prm["t_min"], "brick_layout": args.brick_layout,
        },
        "mrays_per_s": round(mrays, 3),
        "samples_per_frame": int(samples),
        "segments_per_frame": int(st["segments"]),
        "tap_descents_per_frame": int(st["tap_descents"]),
        "deferred_tap_samples_per_frame": int(st["split_samples"]),
        "unlit_ms_per_step": round(unlit_ms, 4) if unlit_ms else None,
        "tile_order": "each frame renders its 8x8 tiles longest first by the previous frame's tile times "
                      "(a tile schedule kept across frames; images do not depend on it)",
        "first_frame_ms": round(first["ms"], 4),
        "unlit_first_frame_ms": round(unlit_first["ms"], 4) if unlit_ms else None,
        "preprocess_s": {"generate": round(gen_s, 2), "build": round(build_s, 4), "pack_upload": round(pack_s, 3)},
        "roofline": roof,
        "unlit_roofline": unlit_roof,
        "cpu_baseline": cpu,
        "learned_skip": learned_res,
        "batched_serving": batched_res,
        "adjoint_tf_fit": adjoint_res,
        "next_rows": next_res,
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
