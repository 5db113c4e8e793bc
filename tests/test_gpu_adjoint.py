"""GPU adjoint (amr_render_backward) against the FP64 oracle's reverse mode, GPU finite
differences, and its own invariants (determinism, checkpoint-rate independence)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _scene(amr, h):
    import torch
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda")
    torch.cuda.synchronize()
    return tree, scene


# fp32 bar: |g - g_ref| <= rel |g_ref| + 1e-5 max|g_ref|.  The absolute term is the fp32 noise
# floor of a gradient entry summed from ~1e5 per-sample terms (observed worst 2.3e-6 max).
ABS_FLOOR = 1e-5
# Entries checked at the relative bar (|g_ref| >= 1e-3 max|g_ref|) must number more than
# MIN_SIGNIFICANT, so that a comparison is never carried by a handful of entries.  The views
# with a full image of dL/dRGBA reach 500-750 such entries; the pixel-subset views of the
# cosmology-like hierarchy (600-800 pixels, values concentrated in a few LUT bins by its
# log-normal density) reach 45-75, the 32x32 autograd view 578.
MIN_SIGNIFICANT = 20


def _bar_ok(got, ref, rel):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    return bool(np.all(np.abs(got - ref) <= rel * np.abs(ref) + ABS_FLOOR * np.abs(ref).max()))


def _rel_ok(got, ref, rel, floor_frac):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    big = np.abs(ref) >= floor_frac * np.abs(ref).max()
    err = np.abs(got - ref)[big] / np.abs(ref)[big]
    worst = np.argsort(-np.where(big, np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300), 0).ravel())[:8]
    for w in worst:
        print("  entry %s ref %.6g got %.6g rel %.3g abs/max %.3g" % (
            np.unravel_index(w, ref.shape), ref.ravel()[w], got.ravel()[w],
            abs(got.ravel()[w] - ref.ravel()[w]) / abs(ref.ravel()[w]),
            abs(got.ravel()[w] - ref.ravel()[w]) / np.abs(ref).max()))
    return err.max() if big.any() else 0.0, int(big.sum())


@pytest.mark.parametrize("lit", [False, True])
def test_adjoint_vs_oracle_small_nested(gpu, lit):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=lit, t_min=0.0, light=(0.3, 1.0, -0.6))
    cam = workloads.small_nested_cameras(64, 64)[1]
    tree, scene = _scene(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    out, ck = amr.render_checkpointed(scene, cam, lut_t, prm, ckpt_every=2, ckpt_max=8)
    W = np.random.default_rng(3).normal(size=(64 * 64, 4)).astype(np.float32)
    glut, glight = amr.render_backward(scene, cam, lut_t, prm, ck, torch.from_numpy(W).cuda())
    torch.cuda.synchronize()
    ref_lut, ref_light = oracle.Oracle(h).grad(cam, prm, lut.astype(np.float64), W.astype(np.float64))
    e, n = _rel_ok(glut.cpu().numpy(), ref_lut, 1e-3, 1e-3)
    print("lit=%d: LUT grad max rel err %.3g over %d entries" % (lit, e, n))
    assert _bar_ok(glut.cpu().numpy(), ref_lut, 1e-3) and n > 50
    if lit:
        gl = glight.cpu().numpy()
        assert np.all(np.abs(gl - ref_light) <= 1e-3 * np.abs(ref_light) + 1e-4 * np.abs(ref_light).max())
    else:
        assert np.all(glight.cpu().numpy() == 0)


def test_adjoint_vs_gpu_finite_differences(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(2)
    prm = dict(prm, lighting=True, t_min=0.0)
    cam = workloads.small_nested_cameras(48, 48)[1]
    tree, scene = _scene(amr, h)
    lut64 = lut.astype(np.float64)
    W = np.random.default_rng(5).normal(size=(48 * 48, 4))
    out, ck = amr.render_checkpointed(scene, cam, torch.from_numpy(lut).cuda(), prm)
    glut, _ = amr.render_backward(scene, cam, torch.from_numpy(lut).cuda(), prm, ck,
                                  torch.from_numpy(W.astype(np.float32)).cuda())
    g = glut.cpu().numpy().astype(np.float64)

    def loss(l):
        o = amr.render(scene, cam, torch.from_numpy(l.astype(np.float32)).cuda(), prm)["rgba"]
        return float((o.double().cpu().numpy().reshape(-1, 4) * W).sum())
    hstep = 1e-3
    rng = np.random.default_rng(0)
    idx = np.argwhere(np.abs(g) >= 1e-2 * np.abs(g).max())
    sel = idx[rng.choice(len(idx), size=min(60, len(idx)), replace=False)]
    fd = []
    for e, c in sel:
        lp = lut64.copy(); lp[e, c] += hstep
        lm = lut64.copy(); lm[e, c] -= hstep
        fd.append((loss(lp) - loss(lm)) / (2 * hstep))
    fd = np.array(fd)
    ad = np.array([g[e, c] for e, c in sel])
    cos = fd @ ad / (np.linalg.norm(fd) * np.linalg.norm(ad))
    print("cosine %.6f, max rel %.3g" % (cos, np.max(np.abs(fd - ad) / np.abs(ad))))
    assert cos >= 0.999
    assert np.max(np.abs(fd - ad) / np.abs(ad)) <= 1e-2


def test_adjoint_vs_gpu_finite_differences_cosmology(gpu):
    """The same check on the transfer-function fit's hierarchy (cosmology-like, 2008 patches),
    lit without early termination, one 96x96 orbit camera, the adjoint reading the tape: central
    differences of L = sum W * RGBA over the LUT entries with gradients of at least 3e-3 of the
    largest (17 here: the hierarchy's log-normal values fill few LUT bins).  The loss is
    piecewise linear in the colour entries and smooth in the extinction ones, so a step of 1 %
    of the entry (plus 1e-2) keeps the truncation error far below the fp32 noise of the renders."""
    import torch
    amr = gpu
    h, cams, target, start, prm = workloads.tf_fit(0, res=96, ncams=1)
    cam = cams[0]
    tree, scene = _scene(amr, h)
    W = np.random.default_rng(8).normal(size=(96 * 96, 4))
    lut64 = start.astype(np.float64)
    out, ck = amr.render_checkpointed(scene, cam, torch.from_numpy(start).cuda(), prm)
    assert ck.tape is not None and ck.tape_overflow_rays() == 0
    glut, _ = amr.render_backward(scene, cam, torch.from_numpy(start).cuda(), prm, ck,
                                  torch.from_numpy(W.astype(np.float32)).cuda())
    g = glut.cpu().numpy().astype(np.float64)

    def loss(l):
        o = amr.render(scene, cam, torch.from_numpy(l.astype(np.float32)).cuda(), prm)["rgba"]
        return float((o.double().cpu().numpy().reshape(-1, 4) * W).sum())
    rng = np.random.default_rng(1)
    idx = np.argwhere(np.abs(g) >= 3e-3 * np.abs(g).max())
    sel = idx[rng.choice(len(idx), size=min(40, len(idx)), replace=False)]
    fd = []
    for e, c in sel:
        hs = 1e-2 * (1.0 + abs(lut64[e, c]))
        lp = lut64.copy(); lp[e, c] += hs
        lm = lut64.copy(); lm[e, c] -= hs
        fd.append((loss(lp) - loss(lm)) / (2 * hs))
    fd = np.array(fd)
    ad = np.array([g[e, c] for e, c in sel])
    cos = fd @ ad / (np.linalg.norm(fd) * np.linalg.norm(ad))
    rel = np.abs(fd - ad) / np.abs(ad)
    print("cosmology: %d entries, cosine %.6f, max rel %.3g, median rel %.3g" % (len(sel), cos, rel.max(), np.median(rel)))
    assert len(sel) >= 12 and cos >= 0.999 and rel.max() <= 2e-2


def test_adjoint_deterministic_and_checkpoint_rate(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    prm = dict(prm, lighting=True)
    cam = workloads.small_nested_cameras(64, 64)[0]
    tree, scene = _scene(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    W = torch.from_numpy(np.random.default_rng(1).normal(size=(64 * 64, 4)).astype(np.float32)).cuda()
    res = []
    for every, cmax in ((1, 2), (1, 64), (4, 8), (1000, 2)):
        out, ck = amr.render_checkpointed(scene, cam, lut_t, prm, ckpt_every=every, ckpt_max=cmax)
        r1 = amr.render_backward(scene, cam, lut_t, prm, ck, W, deterministic=True)
        r2 = amr.render_backward(scene, cam, lut_t, prm, ck, W, deterministic=True)
        assert torch.equal(r1[0], r2[0]) and torch.equal(r1[1], r2[1]), "deterministic mode not reproducible"
        res.append(torch.cat([r1[0].flatten(), r1[1]]).cpu().numpy().astype(np.float64))
    ref = res[0]
    for r in res[1:]:
        assert np.abs(r - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("layout", [0, 1, 2])
def test_adjoint_tape_matches_in_place(gpu, layout):
    """The checkpointed lit forward writes every segment's and sample's record to the ray's tape;
    the adjoint replays the intervals whose records all fit from it and evaluates the others in
    place.  Gradients with a tape that holds every record, with one that holds the first
    intervals of most rays, with one too short for nearly all of them and with none agree to the
    fp32 bar of the adjoint, on the cosmology-like hierarchy at 96x96 (its gradient taps cross
    many patches), in every brick layout; the oracle checks the tape form on a pixel subset."""
    import torch
    amr = gpu
    h, cams, target, start, prm = workloads.tf_fit(0, res=96, ncams=1)
    cam = cams[0]
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda", brick_layout=layout)
    lut_t = torch.from_numpy(start).cuda()
    W = torch.from_numpy(np.random.default_rng(4).normal(size=(96 * 96, 4)).astype(np.float32)).cuda()
    got = {}
    for cap in (0, 3, 400, 4096):
        out, ck = amr.render_checkpointed(scene, cam, lut_t, prm, tape_cap=cap)
        glut, glight = amr.render_backward(scene, cam, lut_t, prm, ck, W, deterministic=True)
        torch.cuda.synchronize()
        got[cap] = (glut.cpu().numpy(), glight.cpu().numpy(), ck.tape_overflow_rays())
        print("layout %d tape_cap %d: %d rays beyond the tape, max |dLUT| %.4g" % (
            layout, cap, got[cap][2], np.abs(got[cap][0]).max()))
    assert got[3][2] > 100 and got[4096][2] == 0 and 0 < got[400][2] < got[3][2]
    for cap in (3, 400, 4096):
        assert _bar_ok(got[cap][0], got[0][0], 1e-4)
        assert np.all(np.abs(got[cap][1] - got[0][1]) <= 1e-4 * np.abs(got[0][1]) + 1e-5 * np.abs(got[0][1]).max())
    if layout == 2:
        # the tape form against the oracle's reverse mode on a pixel subset
        rng = np.random.default_rng(9)
        flat = rng.choice(96 * 96, 600, replace=False)
        pix = np.stack([flat % 96, flat // 96], 1).astype(np.int32)
        gsub = rng.normal(size=(600, 4)).astype(np.float32)
        G = np.zeros((96 * 96, 4), np.float32)
        G[flat] = gsub
        Gt = torch.from_numpy(G).cuda()
        out, ck = amr.render_checkpointed(scene, cam, lut_t, prm, tape_cap=4096)
        glut, glight = amr.render_backward(scene, cam, lut_t, prm, ck, Gt)
        torch.cuda.synchronize()
        ref_lut, ref_light = oracle.Oracle(h).grad(cam, prm, start.astype(np.float64), gsub.astype(np.float64),
                                                   pixels=pix)
        e, n = _rel_ok(glut.cpu().numpy(), ref_lut, 1e-3, 1e-3)
        print("tape adjoint vs oracle: LUT grad max rel err %.3g over %d entries" % (e, n))
        assert _bar_ok(glut.cpu().numpy(), ref_lut, 1e-3) and n > MIN_SIGNIFICANT


def test_tape_records_vs_oracle(gpu):
    """The tape the checkpointed lit forward writes, record by record, against the oracle: per ray
    one record per data segment, (delta, delta log2 e, n, 0) with n and the segment's sample
    spacing from the oracle's segment list, then one per sample, (F, g): the trilinear value at
    the sample and the central-difference gradient of the oracle's shading (taps one cell of the
    segment's level away, one-sided outside the domain, divided by the LUT's value range).  The
    header's record count is the number of records the ray wrote; early termination ends the
    records with the ray's last sample.  Small nested hierarchy (gradient taps cross patch and
    level boundaries), lit, 64x64 oblique view, 1000 seeded rays."""
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(1)
    prm = dict(prm, lighting=True)
    W = H = 64
    cam = workloads.small_nested_cameras(W, H)[1]
    tree, scene = _scene(amr, h)
    cap = 4096
    out, ck = amr.render_checkpointed(scene, cam, torch.from_numpy(lut).cuda(), prm, tape_cap=cap)
    torch.cuda.synchronize()
    tape = ck.tape.view(W * H, cap, 4).cpu().numpy()
    hdr = ck.buf.view(-1, 32 * (1 + ck.max))[:, :32].contiguous().view(torch.int32).cpu().numpy()
    O = oracle.Oracle(h)
    sel = np.sort(np.random.default_rng(12).choice(W * H, 1000, replace=False))
    pix = np.stack([sel % W, sel // W], 1).astype(np.int32)
    res = O.render(cam, prm, lut, pixels=pix, trace_cap=512)
    assert res["trace_n"].max() <= 512 and int(np.count_nonzero(res["flags"])) == 0
    same = hdr[sel, 4] == res["nsamp"]
    print("rays whose early termination differs (fp32 against FP64 transmittance): %d of %d" % ((~same).sum(), len(sel)))
    assert (~same).sum() <= 2
    levels = np.array([p.level for p in h.patches])
    hl = lambda lev: np.asarray(h.h0, np.float64) / float(h.refine) ** lev
    rng_v = prm["v_hi"] - prm["v_lo"]
    nrec = nsmp = 0
    dF = dg = 0.0
    for s in np.flatnonzero(same):
        q = int(sel[s])
        i, j = q % W, q // W
        o, d = (np.asarray(a) for a in oracle.ray(cam, int(i), int(j)))
        left = int(res["nsamp"][s])
        pos = 0
        for rec in res["trace"][s, :res["trace_n"][s]]:
            n, patch = int(rec["n"]), int(rec["patch"])
            if patch < 0 or n == 0 or left == 0:
                continue
            delta = (rec["tb"] - rec["ta"]) / n
            seg = tape[q, pos]
            assert seg.view(np.int32)[2] == n and seg[3] == 0.0, (q, pos)
            assert abs(seg[0] - delta) <= 1e-6 * delta and abs(seg[1] - delta * np.log2(np.e)) <= 2e-6 * delta
            pos += 1
            step = hl(levels[patch])
            for k in range(min(n, left)):
                x = o + (rec["ta"] + (k + 0.5) * delta) * d
                F = O.field(x)
                g = np.zeros(3)
                for a in range(3):
                    e = np.zeros(3)
                    e[a] = step[a]
                    Fp, Fm = O.field(x + e), O.field(x - e)
                    g[a] = ((Fp - Fm) / 2 if Fp is not None and Fm is not None else
                            (Fp - F) if Fp is not None else (F - Fm) if Fm is not None else 0.0) / rng_v
                r = tape[q, pos]
                dF = max(dF, abs(r[0] - F) / rng_v)
                dg = max(dg, float(np.abs(r[1:] - g).max()))
                pos += 1
                nsmp += 1
            left -= min(n, left)
        assert hdr[q, 7] == pos, (q, hdr[q, 7], pos)
        nrec += pos
    print("tape: %d records, %d samples; max |F - F_ref| / range %.3g, max |g - g_ref| %.3g" % (nrec, nsmp, dF, dg))
    assert nsmp > 12000
    # fp32 trilinear in patch-local coordinates against FP64: ~1e-7 of the range; the gradient is
    # a difference of two such values over two cells, so its error is of the same order
    assert dF <= 1e-6 and dg <= 1e-5


def test_autograd_function(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.small_nested(0)
    prm = dict(prm, lighting=True, t_min=0.0)
    cam = workloads.small_nested_cameras(32, 32)[1]
    tree, scene = _scene(amr, h)
    lut_p = torch.from_numpy(lut).cuda().requires_grad_(True)
    sh = torch.tensor([1.0, 1.0, 1.0, 0.3, 0.7], dtype=torch.float32, requires_grad=True)
    rgba = amr.AMRRender.apply(lut_p, sh, scene, cam, prm)
    target = torch.zeros_like(rgba)
    loss = ((rgba - target) ** 2).mean()
    loss.backward()
    ref_lut, ref_sh = oracle.Oracle(h).grad(cam, prm, lut.astype(np.float64),
                                           (2 * rgba.detach().double().cpu().numpy().reshape(-1, 4)) / rgba.numel())
    e, n = _rel_ok(lut_p.grad.cpu().numpy(), ref_lut, 2e-3, 1e-3)
    print("autograd: LUT grad max rel err %.3g over %d entries" % (e, n))
    assert _bar_ok(lut_p.grad.cpu().numpy(), ref_lut, 1e-3) and n > MIN_SIGNIFICANT
    assert np.allclose(sh.grad.numpy(), ref_sh, rtol=2e-3, atol=1e-4 * np.abs(ref_sh).max())


@pytest.mark.parametrize("lit", [True])
def test_adjoint_vs_oracle_tf_fit_subset(gpu, lit):
    """Transfer-function fit workload (cosmology-like hierarchy, 8 cameras at 512^2): dL/dRGBA nonzero on 800 random
    pixels per camera; the GPU adjoint of the full 8-camera batch against the oracle's."""
    import torch
    amr = gpu
    h, cams, target, start, prm = workloads.tf_fit(0)
    prm = dict(prm, lighting=lit)
    tree, scene = _scene(amr, h)
    lut_t = torch.from_numpy(start).cuda()
    out, ck = amr.render_checkpointed(scene, cams, lut_t, prm, ckpt_every=4, ckpt_max=16)
    rng = np.random.default_rng(2)
    npx = 512 * 512
    G = np.zeros((len(cams), npx, 4), dtype=np.float32)
    O = oracle.Oracle(h)
    ref_lut = np.zeros((256, 4)); ref_light = np.zeros(5)
    for c, cam in enumerate(cams):
        sel = rng.choice(npx, size=800, replace=False)
        G[c, sel] = rng.normal(size=(800, 4))
        pix = np.stack([sel % 512, sel // 512], 1).astype(np.int32)
        rl, rli = O.grad(cam, prm, start.astype(np.float64), G[c, sel].astype(np.float64), pixels=pix)
        ref_lut += rl
        ref_light += rli
    glut, glight = amr.render_backward(scene, cams, lut_t, prm, ck, torch.from_numpy(G.reshape(-1, 4)).cuda())
    e, n = _rel_ok(glut.cpu().numpy(), ref_lut, 1e-3, 1e-3)
    print("tf_fit: LUT grad max rel err %.3g over %d entries; light %s vs %s" % (e, n, glight.cpu().numpy(), ref_light))
    assert _bar_ok(glut.cpu().numpy(), ref_lut, 1e-3) and n > MIN_SIGNIFICANT
    assert np.all(np.abs(glight.cpu().numpy() - ref_light) <= 1e-3 * np.abs(ref_light) + 1e-4 * np.abs(ref_light).max())


def test_tf_fit_200_adam_steps(gpu):
    """Transfer-function fit (cosmology-like hierarchy, 8 cameras at 512^2, lit): 200 Adam steps
    (lr 1e-2) on the LUT through AMRRender from the starting LUT toward images rendered with a
    hidden target LUT.  The image loss falls by more than 10x and the LUT moves toward the target
    on the entries the images constrain.  The steps share a tile schedule (each forward starts the
    tiles longest first by the previous step's tile times); a second, shorter run without one must
    follow the same losses."""
    import torch
    amr = gpu
    h, cams, target, start, prm = workloads.tf_fit(0)
    tree, scene = _scene(amr, h)
    sh = torch.tensor([1.0, 1.0, 1.0, 0.3, 0.7], dtype=torch.float32)
    with torch.no_grad():
        tgt = amr.render(scene, cams, torch.from_numpy(target).cuda(), prm)["rgba"].clone()
    lut = torch.from_numpy(start).cuda().requires_grad_(True)
    opt = torch.optim.Adam([lut], lr=1e-2)
    losses = []
    touched = None
    sched = amr.Schedule(cams, "cuda")
    for step in range(200):
        opt.zero_grad()
        rgba = amr.AMRRender.apply(lut, sh, scene, cams, prm, 4, 16, False, sched)
        loss = ((rgba - tgt) ** 2).mean()
        loss.backward()
        if touched is None:
            touched = (lut.grad.abs() > 0).cpu().numpy()
        opt.step()
        with torch.no_grad():
            lut.clamp_(min=0.0)
        losses.append(float(loss.item()))
    print("loss %.4g -> %.4g (every 25: %s)" % (losses[0], losses[-1], ["%.3g" % v for v in losses[::25]]))
    assert losses[-1] < 0.1 * losses[0]
    d0 = np.abs(start - target)[touched[:, :3].any(axis=1)][:, :3].mean()
    d1 = np.abs(lut.detach().cpu().numpy() - target)[touched[:, :3].any(axis=1)][:, :3].mean()
    print("colour LUT error on constrained entries %.4g -> %.4g" % (d0, d1))
    assert d1 < d0
    # without a tile schedule (tiles in the default order): the same images, so the same first losses
    lut2 = torch.from_numpy(start).cuda().requires_grad_(True)
    opt2 = torch.optim.Adam([lut2], lr=1e-2)
    for step in range(5):
        opt2.zero_grad()
        rgba = amr.AMRRender.apply(lut2, sh, scene, cams, prm)
        loss = ((rgba - tgt) ** 2).mean()
        loss.backward()
        opt2.step()
        with torch.no_grad():
            lut2.clamp_(min=0.0)
        # step 0: the same images; later steps also carry the atomics' rounding of the gradients
        assert abs(float(loss.item()) - losses[step]) <= (0.0 if step == 0 else 1e-4) * losses[step], step


@pytest.mark.parametrize("lit", [False, True])
def test_adjoint_with_lod(gpu, lit):
    """The adjoint replays the level-of-detail segmentation: LUT and light gradients against the
    oracle's on the level-of-detail geometry with lod = 3 pixels."""
    import torch
    amr = gpu
    h = workloads.lod_blocks(0)
    lut = workloads.lut_bumps(np.random.default_rng(3), sigma_scale=6.0)
    vmax = float(max(p.cells.max() for p in h.patches))
    prm = workloads.default_params(v_hi=vmax, lighting=lit, t_min=0.0, lod=3.0)
    cam = workloads.perspective_orbit(40, 32, 0.9, 0.25, radius=1.7)
    tree, scene = _scene(amr, h)
    lut_t = torch.from_numpy(lut).cuda()
    out, ck = amr.render_checkpointed(scene, cam, lut_t, prm)
    G = np.random.default_rng(4).normal(size=(40 * 32, 4))
    glut, glight = amr.render_backward(scene, cam, lut_t, prm, ck, torch.from_numpy(G.astype(np.float32)).cuda())
    ref_lut, ref_light = oracle.Oracle(h).grad(cam, prm, lut.astype(np.float64), G)
    e, n = _rel_ok(glut.cpu().numpy(), ref_lut, 1e-3, 1e-3)
    print("lod adjoint lit=%d: LUT grad max rel err %.3g over %d entries" % (lit, e, n))
    assert _bar_ok(glut.cpu().numpy(), ref_lut, 1e-3) and n > MIN_SIGNIFICANT
    if lit:
        gl = glight.cpu().numpy()
        assert np.all(np.abs(gl - ref_light) <= 1e-3 * np.abs(ref_light) + 1e-4 * np.abs(ref_light).max())

