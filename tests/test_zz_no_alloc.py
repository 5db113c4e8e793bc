"""amr_render_backward_static (the adjoint with its accumulators in the library's fixed device
array, for callers that cannot allocate) against amr_render_backward (caller workspace), through
the C ABI: two calls in a row, the second on a smaller input, deterministic and atomic modes.
Deterministic mode runs the same kernels over the same fixed grid and sums the partials in the
same order, so the gradients must agree bit for bit; the atomic mode to the adjoint's fp32 bar
(|g - g_ref| <= 1e-3 |g_ref| + 1e-5 max|g_ref|)."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

ABS_FLOOR = 1e-5


def _bar_ok(got, ref, rel=1e-3):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    return bool(np.all(np.abs(got - ref) <= rel * np.abs(ref) + ABS_FLOOR * np.abs(ref).max()))


def test_static_workspace_backward_matches_workspace_backward(gpu):
    import torch
    amr = gpu
    lib = amr.load()
    assert lib.amr_backward_static_bytes() >= lib.amr_backward_work_bytes(1)
    h, lut, cams, prm = workloads.small_nested(1)
    tree = amr.build_tree(h)
    scene = amr.pack(tree, h, device="cuda")
    lut_t = torch.from_numpy(lut).cuda()
    big = workloads.small_nested_cameras(64, 48)
    small = [workloads.small_nested_cameras(24, 20)[1]]
    for lit in (True, False):
        p = dict(prm, lighting=lit, t_min=0.0, light=(0.3, 1.0, -0.6))
        for call, cams_k in enumerate((big, small)):
            npix = sum(c["width"] * c["height"] for c in cams_k)
            out, ck = amr.render_checkpointed(scene, cams_k, lut_t, p, ckpt_every=2, ckpt_max=8)
            g = torch.from_numpy(np.random.default_rng(10 + call).normal(size=(npix, 4)).astype(np.float32)).cuda()
            for det in (True, False):
                ref_lut, ref_light = amr.render_backward(scene, cams_k, lut_t, p, ck, g, deterministic=det)
                got_lut, got_light = amr.render_backward(scene, cams_k, lut_t, p, ck, g, deterministic=det,
                                                         static_work=True)
                torch.cuda.synchronize()
                a, b = got_lut.cpu().numpy(), ref_lut.cpu().numpy()
                la, lb = got_light.cpu().numpy(), ref_light.cpu().numpy()
                print("lit=%d call %d (%d pixels) det=%d: max |dLUT static - workspace| = %.3g, max |dLUT| = %.3g"
                      % (lit, call, npix, det, np.abs(a - b).max(), np.abs(b).max()))
                assert np.abs(b).max() > 0
                if det:
                    assert np.array_equal(a, b) and np.array_equal(la, lb)
                else:
                    assert _bar_ok(a, b) and _bar_ok(la, lb)
    # the static entry point keeps the checks of the workspace one
    q = amr.make_params(dict(prm, lighting=True), lut_t)
    carr = (amr._lib.amr_camera * 1)(amr.make_camera(small[0]))
    gl = torch.zeros((256, 4), dtype=torch.float32, device="cuda")
    gv = torch.zeros(5, dtype=torch.float32, device="cuda")
    gr = torch.zeros(4 * small[0]["width"] * small[0]["height"], dtype=torch.float32, device="cuda")
    import ctypes
    rc = lib.amr_render_backward_static(ctypes.byref(scene.scene), carr, 1, ctypes.byref(q), gr.data_ptr(),
                                        gl.data_ptr(), gv.data_ptr(), 0, None)
    assert rc == 1 and "checkpoints" in lib.amr_last_error().decode()
