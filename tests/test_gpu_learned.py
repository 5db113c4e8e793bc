"""Learned segment proposals on the deep-range hierarchy: the logger's analytic bounds bracket
the true segment opacities, zero thresholds reproduce the plain render bit for bit, training on
the GPU lowers the pinball loss, calibrated thresholds keep held-out views within 1e-3 of the
plain render (which the FP64 oracle checks), the learned form takes fewer samples, and at the
same threshold it takes fewer samples than the same kernel with the network never asked
(bound_only), both within 1e-3 of the plain render."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def deep(gpu):
    import torch
    amr = gpu
    h, lut, cams, prm = workloads.deep_range_scene(0, res=256)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda")
    torch.cuda.synchronize()
    return h, lut, cams, prm, tree, scene


def _views(h, n, seed, res):
    return workloads.deep_range_orbits(h, n, seed, res)


def test_logger_bounds_bracket_truth(gpu, deep):
    import torch
    from paper_1212_3333_amd import learned
    amr = gpu
    h, lut, cams, prm, tree, scene = deep
    lut_t = torch.from_numpy(lut).cuda()
    X, alpha, t_in, count = learned.log_segments(scene, cams, lut_t, dict(prm, t_min=0.0), cap_records=1 << 18)
    assert count > 1000
    X, alpha = X.cpu().numpy(), alpha.cpu().numpy()
    full = t_in.cpu().numpy() > 0
    # analytic bounds from the leaf's value range: alpha_min <= alpha_seg <= alpha_max (fp32 slack)
    assert np.all(alpha[full] <= X[full, 4] + 1e-5)
    assert np.all(alpha[full] >= X[full, 6] - 1e-5)
    assert np.all((X[:, 2] >= 0) & (X[:, 3] <= 1) & (X[:, 2] <= X[:, 3]))


def test_zero_thresholds_bit_identical(gpu, deep):
    import torch
    from paper_1212_3333_amd import learned
    amr = gpu
    h, lut, cams, prm, tree, scene = deep
    lut_t = torch.from_numpy(lut).cuda()
    W = learned.init_weights(1, "cuda")
    packed = amr.mlp_pack(W)
    for cam in cams:
        plain = amr.render(scene, cam, lut_t, prm)["rgba"]
        lr = learned.render_learned(scene, cam, lut_t, prm, packed, 0.0, 0.0)["rgba"]
        torch.cuda.synchronize()
        assert torch.equal(plain, lr)


def test_bound_only_zero_threshold_and_bound(gpu, deep):
    """bound_only with tau_e = 0 skips nothing and reproduces the plain render bit for bit; with
    tau_e > 0 every ray's skipped opacity is charged at its analytic bound, so the image stays
    within about tau_e of the plain render; it is rejected with a network or in persistent mode."""
    import torch
    from paper_1212_3333_amd import learned
    amr = gpu
    h, lut, cams, prm = deep[:4]
    scene = deep[5]
    lut_t = torch.from_numpy(lut).cuda()
    for cam in cams:
        plain = amr.render(scene, cam, lut_t, prm, stats=True)
        b0 = learned.render_bound_only(scene, cam, lut_t, prm, 0.0, stats=True)
        b1 = learned.render_bound_only(scene, cam, lut_t, prm, 5e-4, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(plain["rgba"], b0["rgba"])
        assert amr.stats_dict(b0)["skipped_segments"] == 0 and amr.stats_dict(b0)["net_segments"] == 0
        err = float((b1["rgba"] - plain["rgba"]).abs().max().item())
        s1 = amr.stats_dict(b1)
        print("bound_only tau 5e-4: max err %.3g, samples %d of %d, skipped %d" % (
            err, s1["samples"], amr.stats_dict(plain)["samples"], s1["skipped_segments"]))
        assert err <= 1e-3 and s1["net_segments"] == 0
    W = learned.init_weights(1, "cuda")
    with pytest.raises(amr.AMRError, match="bound_only"):
        amr.render(scene, cams[0], lut_t, dict(prm, bound_only=1), d_mlp=amr.mlp_pack(W))
    two = list(cams[:2])
    with pytest.raises(amr.AMRError, match="persistent"):
        amr.render(scene, two, lut_t, dict(prm, bound_only=1, persistent=1), d_cams=amr.camera_table(two),
                   d_queue=amr.queue_buffer(2))


def test_train_calibrate_gain(gpu, deep):
    import torch
    from paper_1212_3333_amd import learned
    amr = gpu
    h, lut, cams, prm, tree, scene = deep
    lut_t = torch.from_numpy(lut).cuda()
    train_views = _views(h, 16, 1, 192)
    X, alpha, t_in, count = learned.log_segments(scene, train_views, lut_t, prm, cap_records=1 << 20)
    print("logged %d segments (%d met)" % (X.shape[0], count))
    W, losses = learned.train(X, alpha, steps=500, batch=65536, lr=3e-3, log_every=100)
    print("losses", losses)
    assert losses[-1][1] < 0.5 * losses[0][1]
    net = learned.ProposalMLP(W)
    Y = net.predict(X).cpu().numpy()
    r = learned.ratio_targets(X, alpha).cpu().numpy()
    print("below lo %.4f above hi %.4f" % (np.mean(r < Y[:, 0]), np.mean(r > Y[:, 1])))
    assert np.mean(r > Y[:, 1]) < 0.03
    held = _views(h, 6, 2, 192)
    plain_imgs = [amr.render(scene, c, lut_t, prm)["rgba"].clone() for c in held]
    te, ts, table = learned.calibrate(scene, held, lut_t, prm, net.packed, plain_imgs, max_err=1e-3)
    print("calibrated tau_e=%g tau_s=%g" % (te, ts))
    for row in table:
        print("  ", row)
    # fresh evaluation views: error vs plain and sample savings
    evalv = _views(h, 4, 3, 256) + list(cams)
    saved, worst = [], 0.0
    O = oracle.Oracle(h)
    for cam in evalv:
        p = amr.render(scene, cam, lut_t, prm, stats=True)
        q = learned.render_learned(scene, cam, lut_t, prm, net.packed, te, ts, stats=True)
        torch.cuda.synchronize()
        err = float((p["rgba"] - q["rgba"]).abs().max().item())
        worst = max(worst, err)
        sp, sq = amr.stats_dict(p)["samples"], amr.stats_dict(q)["samples"]
        saved.append(1 - sq / max(sp, 1))
        # oracle on a pixel subset: learned image within 1e-3 + 1e-4 of the FP64 reference
        rng = np.random.default_rng(0)
        pix = np.stack([rng.integers(0, cam["width"], 300), rng.integers(0, cam["height"], 300)], 1).astype(np.int32)
        ref = O.render(cam, prm, lut, pixels=pix)["rgba"]
        got = q["rgba"].cpu().numpy()[pix[:, 1], pix[:, 0]]
        assert np.abs(got - ref).max() <= 1e-3 + 1e-4
    print("eval: worst err %.3g, sample savings %s" % (worst, np.round(saved, 3)))
    assert worst <= 1e-3
    assert np.mean(saved) > 0.05
    # what the network adds: the same kernel and threshold with the network never asked
    nb, nn, worst_b = 0, 0, 0.0
    for cam in evalv:
        p = amr.render(scene, cam, lut_t, prm)["rgba"]
        b = learned.render_bound_only(scene, cam, lut_t, prm, te, stats=True)
        q = learned.render_learned(scene, cam, lut_t, prm, net.packed, te, ts, stats=True)
        torch.cuda.synchronize()
        worst_b = max(worst_b, float((b["rgba"] - p).abs().max().item()))
        nb += amr.stats_dict(b)["samples"]
        nn += amr.stats_dict(q)["samples"]
    print("tau_e %g: bound only %d samples (worst err %.3g), bound + network %d samples (%.1f%% fewer)" % (
        te, nb, worst_b, nn, 100.0 * (1 - nn / max(nb, 1))))
    assert worst_b <= 1e-3
    assert te > 0 and nn < nb
