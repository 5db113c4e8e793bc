"""Learned segment proposals: log segments with the plain traversal, train the 12-64-64-2
network on the GPU with the library's kernels, calibrate the skip thresholds on held-out views,
render with the learned form.  The plain traversal stays the fallback and the reference for the
error.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as L
from . import load, mlp_adam_step, mlp_backward, mlp_forward, mlp_pack, render

SEGLOG_HEADER = 256
REC_BYTES = 64


def seglog_buffer(cap_records: int, device) -> torch.Tensor:
    return torch.zeros(SEGLOG_HEADER + REC_BYTES * int(cap_records), dtype=torch.uint8, device=device)


def log_segments(scene, cams, lut: torch.Tensor, params: dict, cap_records: int = 1 << 20):
    """Plain render of `cams` that logs every sampled data segment.  Returns (X [n,12],
    alpha_seg [n], t_in [n], count_met) as device tensors (n <= cap_records)."""
    dev = scene.pool.device
    buf = seglog_buffer(cap_records, dev)
    render(scene, cams, lut, params, d_seglog=buf, seglog_cap=buf.numel())
    torch.cuda.synchronize(dev)
    count = int(buf[:8].view(torch.int64).item())
    n = min(count, cap_records)
    rec = buf[SEGLOG_HEADER:SEGLOG_HEADER + REC_BYTES * n].view(torch.float32).view(n, 16)
    X = rec[:, :12].contiguous()
    alpha = rec[:, 12].contiguous()
    t_in = rec[:, 13].contiguous()
    return X, alpha, t_in, count


def ratio_targets(X: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """Training target: the segment opacity as a fraction of its analytic bound (feature 4),
    in [0, 1]; the kernel multiplies the predicted quantiles back by the bound."""
    bound = X[:, 4]
    return torch.where(bound > 0, alpha / bound.clamp_min(1e-30), torch.zeros_like(alpha)).clamp(0.0, 1.0)


def init_weights(seed: int, device) -> torch.Tensor:
    """He-style initialisation (fp32 masters); the output biases start at ratios 0 and 1."""
    g = np.random.default_rng(seed)
    W1 = g.normal(0, math.sqrt(2.0 / 12), (12, 64))
    W2 = g.normal(0, math.sqrt(2.0 / 64), (64, 64))
    W3 = g.normal(0, math.sqrt(1.0 / 64), (64, 2))
    w = np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(), np.array([0.0, 1.0])])
    assert len(w) == int(load().amr_mlp_param_count())
    return torch.from_numpy(w.astype(np.float32)).to(device)


def train(X: torch.Tensor, alpha: torch.Tensor, steps: int = 600, batch: int = 65536, lr: float = 3e-3,
          q_lo: float = 0.01, q_hi: float = 0.99, seed: int = 0, log_every: int = 0):
    """Adam on the mean pinball loss of the ratio targets (`ratio_targets`) with minibatches
    drawn from the logged segments.  Returns (W, losses)."""
    dev = X.device
    T = ratio_targets(X, alpha)
    W = init_weights(seed, dev)
    M = torch.zeros_like(W)
    V = torch.zeros_like(W)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    n = X.shape[0]
    losses = []
    for t in range(1, steps + 1):
        if n > batch:
            idx = torch.randint(0, n, (batch,), device=dev, generator=gen)
            xb, tb = X[idx].contiguous(), T[idx].contiguous()
        else:
            xb, tb = X, T
        Y, H = mlp_forward(xb, W)
        dW, loss = mlp_backward(xb, W, H, Y, tb, q_lo, q_hi)
        lr_t = lr * (0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * t / steps)))
        mlp_adam_step(W, dW, M, V, t, lr=lr_t)
        if log_every and (t % log_every == 0 or t == 1):
            losses.append((t, float(loss.item())))
    return W, losses


def render_learned(scene, cams, lut, params, packed: torch.Tensor, tau_e: float, tau_s: float, **kw):
    return render(scene, cams, lut, dict(params, tau_e=tau_e, tau_s=tau_s), d_mlp=packed, **kw)


def render_bound_only(scene, cams, lut, params, tau_e: float, **kw):
    """The same kernel and skip rule with the network never consulted: a data segment is skipped
    when the ray's charged opacity plus T * alpha_max (the analytic bound) stays below tau_e."""
    return render(scene, cams, lut, dict(params, tau_e=tau_e, tau_s=0.0, bound_only=1), **kw)


def calibrate_bound_only(scene, views, lut, params, plain_images, max_err: float = 1e-3, safety: float = 0.5,
                         tau_e_grid=(0.0, 5e-5, 1e-4, 2e-4, 3e-4, 5e-4, 1e-3, 2e-3)):
    """Largest tau_e of the bound-only form whose worst RGBA error against the plain renders of
    the held-out `views` stays within safety * max_err (the same rule as `calibrate`).  Returns
    (tau_e, table)."""
    from . import stats_dict
    table = []
    best = (0.0, None)
    for te in tau_e_grid:
        err, samples = 0.0, 0
        for cam, ref in zip(views, plain_images):
            out = render_bound_only(scene, cam, lut, params, te, stats=True)
            err = max(err, float((out["rgba"] - ref).abs().max().item()))
            samples += stats_dict(out)["samples"]
        table.append(dict(tau_e=te, max_err=err, samples=samples))
        if err <= safety * max_err and (best[1] is None or samples < best[1]):
            best = (te, samples)
    return best[0], table


def calibrate(scene, views, lut, params, packed, plain_images, max_err: float = 1e-3, safety: float = 0.5,
              tau_e_grid=(0.0, 5e-5, 1e-4, 2e-4, 3e-4, 5e-4, 1e-3), tau_s_grid=(0.0, 1e-4, 1e-3, 1e-2)):
    """Largest thresholds whose worst RGBA error against the plain renders of the held-out
    `views` stays within safety * max_err; ties broken by fewer samples.  Returns
    (tau_e, tau_s, table)."""
    from . import stats_dict
    table = []
    best = (0.0, 0.0, None)
    for te in tau_e_grid:
        for ts in tau_s_grid:
            err, samples = 0.0, 0
            for cam, ref in zip(views, plain_images):
                out = render_learned(scene, cam, lut, params, packed, te, ts, stats=True)
                err = max(err, float((out["rgba"] - ref).abs().max().item()))
                samples += stats_dict(out)["samples"]
            table.append(dict(tau_e=te, tau_s=ts, max_err=err, samples=samples))
            if err <= safety * max_err and (best[2] is None or samples < best[2]):
                best = (te, ts, samples)
    return best[0], best[1], table


class ProposalMLP:
    """Trained network: fp32 masters W and the packed fp16 inference image."""

    def __init__(self, W: torch.Tensor):
        self.W = W
        self.packed = mlp_pack(W)

    def predict(self, X: torch.Tensor) -> torch.Tensor:
        Y, _ = mlp_forward(X, self.W, keep_hidden=False)
        return Y

    def save(self, path: str):
        np.savez(path, W=self.W.detach().cpu().numpy())

    @staticmethod
    def load(path: str, device="cuda") -> "ProposalMLP":
        return ProposalMLP(torch.from_numpy(np.load(path)["W"]).to(device))
