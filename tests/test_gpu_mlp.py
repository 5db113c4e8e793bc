"""The proposal network's GPU kernels (fp16 MFMA, fp32 accumulation) against the FP64 oracle:
forward within 2e-3 absolute (oracle fed the same fp16-rounded weights, inputs and hidden
activations), weight gradients within 1e-2 relative, Adam within fp32 rounding."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _f16(a):
    return np.asarray(a, dtype=np.float16).astype(np.float64)


def _oracle_forward_f16(w, X):
    """FP64 forward on fp16-rounded operands, as the matrix cores see them."""
    p = omlp.unpack(w)
    h1 = np.maximum(_f16(X) @ _f16(p["W1"]) + p["b1"], 0)
    h2 = np.maximum(_f16(h1) @ _f16(p["W2"]) + p["b2"], 0)
    z3 = _f16(h2) @ _f16(p["W3"]) + p["b3"]
    return 1 / (1 + np.exp(-z3))


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 70001])
def test_mlp_forward(gpu, n):
    import torch
    amr = gpu
    rng = np.random.default_rng(n)
    w = omlp.init(rng).astype(np.float32)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    Y, H = amr.mlp_forward(torch.from_numpy(X).cuda(), torch.from_numpy(w).cuda())
    ref = _oracle_forward_f16(w.astype(np.float64), X)
    err = np.abs(Y.cpu().numpy() - ref).max()
    print("n=%d forward max abs err %.3g" % (n, err))
    assert err <= 2e-3
    # the fp64 reference without fp16 rounding is also close
    assert np.abs(Y.cpu().numpy() - omlp.forward(w.astype(np.float64), X)[0]).max() <= 2e-2


def test_mlp_backward_and_adam(gpu):
    import torch
    amr = gpu
    rng = np.random.default_rng(3)
    n = 20000
    w = omlp.init(rng).astype(np.float32)
    X = rng.normal(size=(n, 12)).astype(np.float32)
    T = rng.random(n).astype(np.float32)
    Wt = torch.from_numpy(w).cuda()
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    Y, H = amr.mlp_forward(Xt, Wt)
    dW, loss = amr.mlp_backward(Xt, Wt, H, Y, Tt, 0.01, 0.99)
    ref_loss, ref_g = omlp.backward(w.astype(np.float64), X.astype(np.float64), T.astype(np.float64), 0.01, 0.99)
    g = dW.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    cos = g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g))
    print("dW rel %.3g cos %.6f loss %.6g vs %.6g" % (rel, cos, loss.item(), ref_loss))
    assert rel <= 1e-2 and cos >= 0.9999
    assert abs(loss.item() - ref_loss) <= 1e-3 * abs(ref_loss)
    for name, o0, o1 in (("W2", omlp.SHAPES and 12 * 64 + 64, 12 * 64 + 64 + 4096),):
        big = np.abs(ref_g[o0:o1]) > 0.05 * np.abs(ref_g[o0:o1]).max()
        assert np.max(np.abs(g[o0:o1] - ref_g[o0:o1])[big] / np.abs(ref_g[o0:o1])[big]) <= 1e-2
    M = torch.zeros_like(Wt); V = torch.zeros_like(Wt)
    w0 = Wt.clone()
    amr.mlp_adam_step(Wt, dW, M, V, 1, lr=1e-3)
    ref_w, _, _ = omlp.adam(w0.cpu().numpy().astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(Wt.cpu().numpy() - ref_w).max() <= 1e-6


def test_mlp_training_reduces_loss(gpu):
    """A few hundred Adam steps on a synthetic target (a smooth function of the inputs) lower
    the pinball loss, and the learned bounds bracket the targets."""
    import torch
    amr = gpu
    rng = np.random.default_rng(4)
    n = 32768
    X = rng.normal(size=(n, 12)).astype(np.float32)
    T = (1 / (1 + np.exp(-(X[:, 0] - 0.5 * X[:, 1]))) * 0.9 + 0.05 * rng.random(n)).astype(np.float32)
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    W = torch.from_numpy(omlp.init(rng).astype(np.float32)).cuda()
    M = torch.zeros_like(W); V = torch.zeros_like(W)
    losses = []
    for t in range(1, 401):
        Y, H = amr.mlp_forward(Xt, W)
        dW, loss = amr.mlp_backward(Xt, W, H, Y, Tt, 0.01, 0.99)
        amr.mlp_adam_step(W, dW, M, V, t, lr=3e-3)
        losses.append(loss.item())
    Y, _ = amr.mlp_forward(Xt, W, keep_hidden=False)
    Yn = Y.cpu().numpy()
    print("loss %.4g -> %.4g; below lo %.3f above hi %.3f" % (losses[0], losses[-1], np.mean(T < Yn[:, 0]),
                                                              np.mean(T > Yn[:, 1])))
    assert losses[-1] < 0.3 * losses[0]
    assert np.mean(T < Yn[:, 0]) < 0.05 and np.mean(T > Yn[:, 1]) < 0.05
