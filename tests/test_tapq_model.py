"""The deferred-tap queue protocol of the lit forward kernels, played on the host.

tests/tapq_model.cpp models a wave's 64 lanes and its queue with the kernels' own index
functions (paper_1212_3333_amd/csrc/amr_tapq_index.h) and checks every slot, owner, run bound
and queued record, that every queued sample is resolved exactly once and that each ray's
deferred contributions arrive in its sample order.  It is built here with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only) and driven by (a) seeded synthetic lane streams,
from no queued sample to every sample queued, with early ray ends and empty rays, and (b) the
streams of real views: the oracle's segment lists of the tiny SAMR view and of 8x8 tiles of the
1024x1024 cosmology-like view, each sample marked as queued when one of its six gradient taps
leaves its leaf box (the kernels queue a subset of those: taps beyond a face whose one-cell slab
is the same patch's stay in the brick), and the ray's last sample marked as its end where early
termination cuts it short.  The kernels' loops are modelled: the single-camera stepped loop
with one sample per step (recording kernels) and with a second sample when the queue has room
for it (the others), each with and without checkpoints (which resolve the queue before every
segment fetch), and the persistent kernel's per-segment loop, with one sample per round
(recording) and with a second one when the queue has room."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# (mode, checkpoints): 0 stepped loop, one sample per step; 1 per-segment loop; 2 and 3 the same
# loops with a second sample per step or round when the queue has room
MODES = [(0, 0), (0, 1), (1, 0), (2, 0), (2, 1), (3, 0)]


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("tapq") / "tapq_model")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "paper_1212_3333_amd", "csrc"),
           os.path.join(ROOT, "tests", "tapq_model.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, text):
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-3000:])
    assert r.stdout.startswith("ok "), r.stdout
    return dict(kv.split("=") for kv in r.stdout.split()[1:])


def _encode(mode, ckpt, nleaves, npatches, pool, waves):
    """waves: list of 64-lane lists of segments (n, leaf, patch, off, flags)."""
    out = ["%d %d %d %d %d %d" % (mode, ckpt, nleaves, npatches, pool, len(waves))]
    for lanes in waves:
        assert len(lanes) == 64
        for segs in lanes:
            parts = [str(len(segs))]
            for (n, leaf, patch, off, flags) in segs:
                parts.append("%d %d %d %d" % (n, leaf, patch, off))
                parts.extend(str(int(f)) for f in flags)
            out.append(" ".join(parts))
    return "\n".join(out) + "\n"


def _synthetic(seed, p_queue, nwaves=24, p_end=0.002, empty_rays=0.05):
    rng = np.random.default_rng(seed)
    waves = []
    for _ in range(nwaves):
        lanes = []
        for _ in range(64):
            if rng.random() < empty_rays:
                lanes.append([])
                continue
            segs = []
            for _ in range(int(rng.integers(1, 40))):
                n = int(rng.geometric(0.08)) - 1 if rng.random() < 0.9 else 0
                flags = (rng.random(n) < p_queue).astype(int)
                ends = rng.random(n) < p_end
                if ends.any():
                    e = int(np.argmax(ends))
                    flags = flags[:e + 1]
                    flags[e] = 2 if flags[e] == 1 else 3
                    segs.append((e + 1, int(rng.integers(0, 50)), int(rng.integers(0, 20)), 64, flags))
                    break
                segs.append((n, int(rng.integers(0, 50)), int(rng.integers(0, 20)), 64, flags))
            lanes.append(segs)
        waves.append(lanes)
    return waves


@pytest.mark.parametrize("p_queue", [0.0, 0.19, 0.6, 1.0])
@pytest.mark.parametrize("mode,ckpt", MODES)
def test_queue_protocol_synthetic(model, mode, ckpt, p_queue):
    stats = _run(model, _encode(mode, ckpt, 50, 20, 4096, _synthetic(11 + int(100 * p_queue), p_queue)))
    print(mode, ckpt, p_queue, stats)
    assert int(stats["max_fill"]) <= 96
    if p_queue >= 0.6:
        assert int(stats["queued"]) > 0 and int(stats["flushes"]) > 24


def test_queue_protocol_single_lane_and_full_pressure(model):
    """One live lane queuing every sample; 64 lanes queuing every sample of one long segment."""
    one = [[] for _ in range(64)]
    one[37] = [(300, 1, 0, 0, [1] * 299 + [2])]
    full = [[(200, 0, 0, 0, [1] * 200)] for _ in range(64)]
    for mode, ckpt in MODES:
        s = _run(model, _encode(mode, ckpt, 2, 1, 64, [one, full]))
        assert int(s["queued"]) == 300 + 64 * 200


def _view_waves(h, cam, lut, prm, tiles, cap=192):
    """Lane streams of the 8x8 tiles `tiles` of a view from the oracle's segment lists."""
    O = oracle.Oracle(h)
    W = cam["width"]
    pix = []
    for (tx, ty) in tiles:
        for lane in range(64):
            pix.append((tx * 8 + (lane & 7), ty * 8 + (lane >> 3)))
    pix = np.asarray(pix, np.int32)
    res = O.render(cam, prm, lut, pixels=pix, trace_cap=cap)
    assert res["trace_n"].max() <= cap
    leaves = O.tree.leaf_array()
    lmax = h.nlevels - 1
    hfine = np.asarray(h.h0, np.float64) / float(h.refine) ** lmax
    origin = np.asarray(h.origin, np.float64)
    lo_w = origin + leaves[:, 0:3] * hfine
    hi_w = origin + leaves[:, 3:6] * hfine
    levels = np.array([p.level for p in h.patches])
    waves, lanes = [], []
    for q in range(len(pix)):
        o, d = oracle.ray(cam, int(pix[q, 0]), int(pix[q, 1]))
        o, d = np.asarray(o), np.asarray(d)
        segs, left = [], int(res["nsamp"][q])
        for rec in res["trace"][q, :res["trace_n"][q]]:
            n, leaf, patch = int(rec["n"]), int(rec["leaf"]), int(rec["patch"])
            if patch < 0 or n == 0:
                segs.append((0, leaf, max(patch, 0), 0, []))
                continue
            t = rec["ta"] + (np.arange(n) + 0.5) * (rec["tb"] - rec["ta"]) / n
            x = o[None, :] + t[:, None] * d[None, :]
            hl = np.asarray(h.h0, np.float64) / float(h.refine) ** levels[patch]
            out = np.zeros(n, bool)
            for a in range(3):
                out |= x[:, a] + hl[a] >= hi_w[leaf, a]
                out |= x[:, a] - hl[a] < lo_w[leaf, a]
            flags = out.astype(int)
            if left <= n:                        # early termination ends the ray here
                flags = flags[:left]
                flags[-1] = 2 if flags[-1] == 1 else 3
                segs.append((left, leaf, patch, patch, flags))
                break
            left -= n
            segs.append((n, leaf, patch, patch, flags))
        lanes.append(segs)
        if len(lanes) == 64:
            waves.append(lanes)
            lanes = []
    return waves, len(leaves), len(h.patches)


def test_queue_protocol_tiny_view(model):
    h, lut, cams, prm = workloads.small_nested(0)
    prm = dict(prm, lighting=True)
    tiles = [(tx, ty) for ty in range(0, 32, 3) for tx in range(0, 32, 3)]
    waves, nl, npch = _view_waves(h, cams[1], lut, prm, tiles)
    for mode, ckpt in MODES:
        s = _run(model, _encode(mode, ckpt, nl, npch, npch, waves))
        print("tiny view mode %d ckpt %d:" % (mode, ckpt), s)
        assert int(s["queued"]) > 0


def test_queue_protocol_cosmology_view(model):
    """64 tiles of the 1024x1024 cosmology-like view, around its centre and on a diagonal."""
    h, lut, cam, prm = workloads.cosmology_view(0)
    tiles = [(60 + i, 60 + j) for i in range(6) for j in range(6)] + [(8 * k, 7 * k + 3) for k in range(16)] + \
            [(100 + k, 30) for k in range(12)]
    waves, nl, npch = _view_waves(h, cam, lut, prm, tiles)
    for mode, ckpt in MODES:
        s = _run(model, _encode(mode, ckpt, nl, npch, npch, waves))
        print("cosmology view mode %d ckpt %d:" % (mode, ckpt), s)
        assert int(s["queued"]) > 1000 and int(s["flushes"]) > 0
