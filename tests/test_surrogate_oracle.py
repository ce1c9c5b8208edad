"""Pins of the FP64 surrogate reference against independent implementations:
torch's CPU convolution and autograd in float64, finite differences, closed
forms of GELU and the optimiser, adjoint identities, and brute force."""
import math

import numpy as np
import pytest

from oracle import surrogate as R

torch = pytest.importorskip("torch")
F = torch.nn.functional


def small_specs():
    return R.layer_specs(enc=(4, 8), mid=16, cin=2, cout=3)


def to_torch_weight(w):
    """[Cout][taps][Cin] -> torch's [Cout][Cin][kh][kw]."""
    co, t, ci = w.shape
    k = int(round(math.sqrt(t)))
    return torch.from_numpy(np.ascontiguousarray(w.transpose(0, 2, 1).reshape(co, ci, k, k)))


def torch_net(P, x, contact_residual=0.0):
    """The same U-Net written with torch's float64 CPU operators (NCHW)."""
    levels = sum(1 for k in P if k.startswith("enc") and k.endswith("a"))
    T = {k: (to_torch_weight(w).requires_grad_(), torch.from_numpy(b.copy()).requires_grad_()) for k, (w, b) in P.items()}

    def cg(name, h):
        w, b = T[name]
        return F.gelu(F.conv2d(h, w, b, padding=w.shape[-1] // 2))

    h = torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))
    skips = []
    for l in range(levels):
        h = cg(f"enc{l}b", cg(f"enc{l}a", h))
        skips.append(h)
        h = F.avg_pool2d(h, 2)
    h = cg("midb", cg("mida", h))
    for l in reversed(range(levels)):
        h = cg(f"up{l}", F.interpolate(h, scale_factor=2, mode="nearest"))
        h = cg(f"dec{l}b", cg(f"dec{l}a", torch.cat([h, skips[l]], dim=1)))
    w, b = T["head"]
    out = F.conv2d(h, w, b).permute(0, 2, 3, 1)
    xt = torch.from_numpy(x)
    res = torch.zeros_like(out)
    res[..., 2] = contact_residual * torch.clamp(xt[..., 0], max=0.0)
    return out + res, T


def test_parameter_count_of_the_full_network():
    assert R.param_count() == 2_140_419


@pytest.mark.parametrize("taps", [9, 1])
def test_conv_matches_torch_conv2d(taps):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 7, 5, 6))
    w = rng.standard_normal((4, taps, 6))
    b = rng.standard_normal(4)
    ours = R.conv(x, w, b)
    ref = F.conv2d(torch.from_numpy(x.transpose(0, 3, 1, 2).copy()), to_torch_weight(w), torch.from_numpy(b),
                   padding=1 if taps == 9 else 0).permute(0, 2, 3, 1).numpy()
    assert np.abs(ours - ref).max() <= 1e-12


def test_conv_backward_matches_autograd():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 5, 3))
    w = rng.standard_normal((4, 9, 3))
    g = rng.standard_normal((2, 6, 5, 4))
    dx, dw, db = R.conv_backward(x, w, g)
    xt = torch.from_numpy(x.transpose(0, 3, 1, 2).copy()).requires_grad_()
    wt = to_torch_weight(w).requires_grad_()
    out = F.conv2d(xt, wt, padding=1)
    out.backward(torch.from_numpy(g.transpose(0, 3, 1, 2).copy()))
    assert np.abs(dx - xt.grad.permute(0, 2, 3, 1).numpy()).max() <= 1e-12
    assert np.abs(dw - wt.grad.numpy().reshape(4, 3, 9).transpose(0, 2, 1)).max() <= 1e-12
    assert np.abs(db - g.sum(axis=(0, 1, 2))).max() <= 1e-12


def test_network_forward_and_gradients_match_torch_autograd():
    rng = np.random.default_rng(5)
    P = R.init_params(rng, small_specs())
    for k in P:  # non-zero biases so their gradients are exercised
        P[k] = (P[k][0], rng.standard_normal(P[k][1].shape) * 0.1)
    x = rng.standard_normal((2, 8, 8, 2))
    y = rng.standard_normal((2, 8, 8, 3))
    loss, out, G = R.loss_and_grads(P, x, y, contact_residual=10.0)
    tout, T = torch_net(P, x, contact_residual=10.0)
    assert np.abs(out - tout.detach().numpy()).max() <= 1e-12
    tl = ((tout - torch.from_numpy(y)) ** 2).mean()
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-13
    for name, (w, b) in T.items():
        dw, db = G[name]
        co, t, ci = dw.shape
        ref = w.grad.numpy().reshape(co, ci, t).transpose(0, 2, 1)
        scale = np.abs(ref).max() + 1e-30
        assert np.abs(dw - ref).max() <= 1e-10 * scale, name
        assert np.abs(db - b.grad.numpy()).max() <= 1e-10 * (np.abs(b.grad.numpy()).max() + 1e-30), name


def test_gradients_match_central_differences():
    rng = np.random.default_rng(6)
    P = R.init_params(rng, small_specs())
    x = rng.standard_normal((1, 8, 8, 2))
    y = rng.standard_normal((1, 8, 8, 3))
    _, _, G = R.loss_and_grads(P, x, y)
    h = 1e-6
    for name in ("enc0a", "enc1b", "mida", "up0", "dec1a", "head"):
        w, b = P[name]
        for _ in range(3):
            idx = tuple(rng.integers(0, s) for s in w.shape)
            old = w[idx]
            w[idx] = old + h
            lp = R.loss_and_grads(P, x, y)[0]
            w[idx] = old - h
            lm = R.loss_and_grads(P, x, y)[0]
            w[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(G[name][0][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, idx)


def test_gelu_closed_forms():
    # GELU(x) = x Phi(x); Phi(1) = 0.841344746068542948585...
    assert abs(R.gelu(np.array(1.0)) - 0.8413447460685429) <= 1e-15
    assert abs(R.gelu(np.array(-1.0)) + 0.15865525393145705) <= 1e-15
    assert R.gelu(np.array(0.0)) == 0.0
    z = np.linspace(-4, 4, 41)
    fd = (R.gelu(z + 1e-6) - R.gelu(z - 1e-6)) / 2e-6
    assert np.abs(R.gelu_grad(z) - fd).max() <= 1e-8
    assert abs(R.gelu_grad(np.array(0.0)) - 0.5) <= 1e-15


def test_pool_and_upsample_are_adjoint_to_their_backward():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((2, 6, 4, 3))
    y = rng.standard_normal((2, 3, 2, 3))
    assert abs((R.avgpool2(x) * y).sum() - (x * R.avgpool2_backward(y)).sum()) <= 1e-12
    u = rng.standard_normal((2, 3, 2, 3))
    v = rng.standard_normal((2, 6, 4, 3))
    assert abs((R.upsample2(u) * v).sum() - (u * R.upsample2_backward(v)).sum()) <= 1e-12
    assert R.avgpool2(np.ones((1, 4, 4, 1))).tolist() == np.ones((1, 2, 2, 1)).tolist()


def test_adamw_matches_torch():
    rng = np.random.default_rng(8)
    p = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=2e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-2)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = R.adamw(p, g, m, v, step, lr=2e-3)
        tp.grad = torch.tensor(g)
        opt.step()
        assert np.abs(p - tp.detach().numpy()).max() <= 1e-14


def test_adamw_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2: p1 = p0 - lr (g / (|g| + eps) + wd p0)
    g = np.array([0.5, -2.0, 1e-3])
    p0 = np.array([1.0, -1.0, 0.25])
    p1, _, _ = R.adamw(p0, g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-8, wd=0.01)
    assert np.abs(p1 - (p0 - 0.1 * (g / (np.abs(g) + 1e-8) + 0.01 * p0))).max() <= 1e-15


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(9)
    a = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(R.round_bf16(a), ref)
    assert R.round_bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0  # tie to even
    assert R.round_bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_nearest_neighbour_brute_force():
    rng = np.random.default_rng(10)
    t = rng.standard_normal((40, 5))
    q = np.concatenate([rng.standard_normal((10, 5)), t[[3, 17]]])
    d2, idx = R.nearest(q, t)
    for i in range(len(q)):
        dd = [float(((q[i] - t[j]) ** 2).sum()) for j in range(len(t))]
        assert idx[i] == int(np.argmin(dd)) and abs(d2[i] - min(dd)) <= 1e-12
    assert idx[10] == 3 and idx[11] == 17 and d2[10] == 0.0


def test_nearest_takes_the_lowest_index_on_ties():
    """Equal distances (exact in binary) resolve to the lowest reference
    index, whichever side of the query the tied rows lie on."""
    t = np.array([[2.0, 0.0], [1.0, 0.0], [-1.0, 0.0], [1.0, 0.0], [0.0, 1.5]])
    q = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, 0.25]])
    d2, idx = R.nearest(q, t)
    assert list(idx) == [1, 1, 1] and list(d2) == [1.0, 0.0, 0.3125]


def test_initial_weights_follow_he_normal():
    """He et al. (2015): zero-mean normal weights of variance 2 / fan-in
    (fan-in = taps x input channels), zero biases."""
    P = R.init_params(np.random.default_rng(11))
    for name, ci, co, taps in R.layer_specs():
        w, b = P[name]
        assert w.shape == (co, taps, ci) and not b.any()
        if w.size >= 100_000:
            std = math.sqrt(2.0 / (ci * taps))
            assert abs(w.std() / std - 1.0) < 0.01 and abs(w.mean()) < 0.01 * std
