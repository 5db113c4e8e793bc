"""Pins of the FP64 proposal-network reference: finite differences of the loss, closed forms
(zero weights give sigmoid(b3); the pinball loss of a constant predictor is minimised at the
q-quantile of the targets) and a textbook Adam step."""
import numpy as np

from oracle import mlp


def test_backward_vs_finite_differences():
    rng = np.random.default_rng(0)
    w = mlp.init(rng) * 0.5
    X = rng.normal(size=(64, mlp.NIN))
    t = rng.random(64)
    loss, g = mlp.backward(w, X, t, 0.01, 0.99)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, size=150, replace=False)
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        yp, _ = mlp.forward(wp, X)
        ym, _ = mlp.forward(wm, X)
        fd = (mlp.pinball(yp, t, 0.01, 0.99) - mlp.pinball(ym, t, 0.01, 0.99)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_zero_weights_give_sigmoid_bias():
    p = mlp.unpack(np.zeros(mlp.NPARAM))
    p["b3"] = np.array([0.3, -1.2])
    y, _ = mlp.forward(mlp.pack(p), np.ones((5, mlp.NIN)))
    assert np.allclose(y, 1 / (1 + np.exp(-np.array([0.3, -1.2]))), rtol=0, atol=1e-15)


def test_pinball_minimiser_is_quantile():
    rng = np.random.default_rng(1)
    t = rng.random(1001)
    for q in (0.01, 0.5, 0.99):
        cands = np.linspace(0, 1, 2001)
        losses = [mlp.pinball(np.full((len(t), 2), c), t, q, q) for c in cands]
        best = cands[int(np.argmin(losses))]
        assert abs(best - np.quantile(t, q, method="inverted_cdf")) <= 1e-3


def test_adam_first_step_is_sign_times_lr():
    g = np.array([0.5, -2.0, 1e-3])
    w, m, v = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    assert np.allclose(w, -0.1 * np.sign(g))


def test_pack_layout():
    p = {name: np.full(shp, k, dtype=np.float64) for k, (name, shp) in enumerate(mlp.SHAPES)}
    w = mlp.pack(p)
    assert len(w) == mlp.NPARAM == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
    assert w[0] == 0 and w[12 * 64] == 1 and w[-1] == 5
