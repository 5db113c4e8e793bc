"""Learned segment proposals on the deep-range hierarchy: the logger's analytic bounds bracket
the true segment opacities, zero thresholds reproduce the plain render bit for bit, training on
the GPU lowers the pinball loss, calibrated thresholds keep held-out views within 1e-3 of the
plain render (which the FP64 oracle checks), and the learned form takes fewer samples."""
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
