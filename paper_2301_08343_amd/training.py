"""Training loop and held-out evaluation of the tactile surrogate.

AdamW with a linear warm-up over the first epoch and cosine decay to zero,
mini-batches drawn by a seeded permutation per epoch; the loss is the MSE of
the displacement in dataset.Y_UNIT. All arithmetic runs in the tsg kernels;
the loss is read back once per epoch.
"""
from __future__ import annotations

import math
import time

import torch

from . import dataset as D
from . import native
from .surrogate import Net


def lr_at(step, total, warmup, peak):
    if step < warmup:
        return peak * (step + 1) / warmup
    t = (step - warmup) / max(1, total - warmup)
    return 0.5 * peak * (1.0 + math.cos(math.pi * t))


def augment(x, y, ops, xo, yo):
    """Symmetry copies (tsg_augment) of x, y by the int32 device tensor ops."""
    native.tsg_call("tsg_augment", x.data_ptr(), y.data_ptr(), x.shape[0], x.shape[1], ops.data_ptr(),
                    xo.data_ptr(), yo.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return xo, yo


def train(net: Net, x, y, epochs=20, batch=256, lr=2e-3, wd=1e-2, seed=0, symmetry=True, log=print):
    """Train in place; returns [(epoch, mean loss, seconds, samples/s)].
    With `symmetry` every mini-batch sample is replaced by one of its eight
    mirror/transpose copies, drawn per sample and step."""
    n = x.shape[0]
    steps_per_epoch = n // batch
    if steps_per_epoch < 1:
        raise ValueError("fewer samples than one batch")
    total = epochs * steps_per_epoch
    g = torch.Generator().manual_seed(seed)
    hist = []
    step = 0
    xa = torch.empty((batch,) + tuple(x.shape[1:]), dtype=torch.float32, device=x.device)
    ya = torch.empty((batch,) + tuple(y.shape[1:]), dtype=torch.float32, device=y.device)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(x.device)
        ops_all = torch.randint(0, 8, (steps_per_epoch, batch), generator=g, dtype=torch.int32).to(x.device)
        acc = torch.zeros(1, dtype=torch.float32, device=x.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps_per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            xb = x.index_select(0, idx)
            yb = y.index_select(0, idx)
            if symmetry:
                xb, yb = augment(xb, yb, ops_all[k], xa, ya)
            loss = net.train_step(xb, yb, lr_at(step, total, steps_per_epoch, lr), wd=wd)
            acc += loss
            step += 1
        mean = float(acc.item()) / steps_per_epoch
        el = time.perf_counter() - t0
        hist.append((ep, mean, el, steps_per_epoch * batch / el))
        if log:
            log(f"epoch {ep}: loss {mean:.4e} ({math.sqrt(mean) * D.Y_UNIT * 1e6:.2f} um rms), "
                f"{el:.2f} s, {steps_per_epoch * batch / el:.0f} samples/s")
    return hist


def predict(net: Net, x, batch=None) -> torch.Tensor:
    """Network output [n][res][res][3] in Y_UNIT (float32, a new tensor)."""
    batch = batch or net.batch
    outs = []
    for k in range(0, x.shape[0], batch):
        outs.append(net.forward(x[k:k + batch]).clone())
    return torch.cat(outs)


def per_sample_rmse(a, b, channel) -> torch.Tensor:
    """Per-sample RMSE of one channel of two [n][res][res][3] fields (same unit)."""
    n = a.shape[0]
    npix = a.shape[1] * a.shape[2]
    out = torch.empty(n, dtype=torch.float32, device=a.device)
    a, b = a.contiguous(), b.contiguous()
    native.tsg_call("tsg_channel_mse", a.data_ptr(), b.data_ptr(), n, npix, 3, channel, out.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    return out.sqrt()


def evaluate(net: Net, x, y, groups=None):
    """Held-out errors in micrometres: height (uz) RMSE over all pixels and
    samples, its per-sample distribution, and the RMSE of all components;
    with `groups` (a label per sample, e.g. the indenter family) also the
    height RMSE per label."""
    p = predict(net, x)
    um = D.Y_UNIT * 1e6
    hz = per_sample_rmse(p, y, 2) * um
    hx = per_sample_rmse(p, y, 0) * um
    hy = per_sample_rmse(p, y, 1) * um
    hz_c = hz.cpu()
    out = {
        "height_rmse_um": float((hz_c ** 2).mean().sqrt()),
        "height_rmse_um_p50": float(hz_c.median()),
        "height_rmse_um_p95": float(hz_c.quantile(0.95)),
        "all_rmse_um": float(((hz ** 2 + hx ** 2 + hy ** 2) / 3).mean().sqrt()),
        "frac_samples_under_5um": float((hz_c <= 5.0).float().mean()),
        "samples": int(x.shape[0]),
    }
    if groups is not None:
        g = torch.as_tensor(groups)
        out["height_rmse_um_by_group"] = {
            str(int(k)): float((hz_c[g == k] ** 2).mean().sqrt()) for k in torch.unique(g)}
        # per label: count, mean and standard deviation of the per-sample
        # height mean squared error (um^2), what the router's error budget
        # starts from
        sq = hz_c.double() ** 2
        out["height_ms_um2_stats_by_group"] = {
            str(int(k)): {"n": int((g == k).sum()), "mean": float(sq[g == k].mean()),
                          "sd": float(sq[g == k].std(unbiased=False))} for k in torch.unique(g)}
    return out
