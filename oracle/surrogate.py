"""FP64 reference of the tactile surrogate network -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this module. Plain numpy in float64; nothing here is shared with the
HIP library.

The surrogate is a 4-level convolutional encoder-decoder (U-Net, Ronneberger
et al. 2015) mapping the indenter's height field and press depth on a 64 x 64
sensor grid to the three displacement components of the elastomer surface:
  encoder level l (channels 32, 64, 128; 256 at the bottleneck): two 3x3
  convolutions with zero padding 1, each followed by GELU; 2x2 average pooling
  between levels;
  decoder level l: nearest-neighbour x2 upsampling, a 3x3 convolution to the
  level's channels + GELU, concatenation [upsampled, skip], two 3x3
  convolutions + GELU;
  head: 1x1 convolution to 3 channels, no activation.
GELU is the exact x Phi(x) (Hendrycks and Gimpel 2016). The optimiser is AdamW
with bias correction and decoupled weight decay (Loshchilov and Hutter 2019).

Layouts: activations NHWC; a 3x3 convolution weight is [Cout][9][Cin] with
tap = 3 kh + kw and offsets (kh - 1, kw - 1); a 1x1 weight is [Cout][1][Cin].

`storage` (optional) is a function applied wherever the network stores a
tensor (inputs, weights, activations, pre-activations, gradients): the
identity gives the exact FP64 network; a bfloat16 rounding gives the same
network with a kernel's storage precision, all arithmetic still in FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

ENC = (32, 64, 128)
MID = 256
CIN = 2
COUT = 3


def _ident(a):
    return a


def round_bf16(a):
    """Round float64 values to the nearest bfloat16 (ties to even), as float64.

    bfloat16 keeps the top 16 bits of an IEEE binary32; the value is first
    rounded to binary32 (exact for values the kernels produce in FP32)."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- primitives

def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _taps(w):
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)] if w.shape[1] == 9 else [(0, 0)]


def _shifted(x, dh, dw):
    """y[n, h, w, :] = x[n, h + dh, w + dw, :], zero outside."""
    n, H, W, c = x.shape
    y = np.zeros_like(x)
    h0, h1 = max(0, -dh), min(H, H - dh)
    w0, w1 = max(0, -dw), min(W, W - dw)
    y[:, h0:h1, w0:w1] = x[:, h0 + dh:h1 + dh, w0 + dw:w1 + dw]
    return y


def conv(x, w, b=None):
    """out[n,h,w,co] = sum_{tap,ci} x[n, h+dh, w+dw, ci] w[co, tap, ci] (+ b[co])."""
    out = np.zeros(x.shape[:3] + (w.shape[0],))
    for t, (dh, dw) in enumerate(_taps(w)):
        out += _shifted(x, dh, dw) @ w[:, t, :].T
    return out if b is None else out + b


def conv_backward(x, w, gout):
    """Adjoint of conv: (dx, dw, db) for the output gradient gout.

    dx scatters each tap's contribution back to the pixel it was read from;
    dw[co, tap, ci] sums gout[..., co] x[shifted by the tap][..., ci]."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dh, dw_) in enumerate(_taps(w)):
        xs = _shifted(x, dh, dw_)
        dw[:, t, :] = gout.reshape(-1, gout.shape[-1]).T @ xs.reshape(-1, xs.shape[-1])
        dx += _shifted(gout @ w[:, t, :], -dh, -dw_)
    return dx, dw, gout.sum(axis=(0, 1, 2))


def avgpool2(x):
    n, H, W, c = x.shape
    return x.reshape(n, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4))


def avgpool2_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(g):
    n, H, W, c = g.shape
    return g.reshape(n, H // 2, 2, W // 2, 2, c).sum(axis=(2, 4))


def mse(pred, target):
    """(mean squared error, its gradient with respect to pred)."""
    e = pred - target
    return float(np.mean(e * e)), 2.0 * e / e.size


def adamw(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=1e-2):
    """One AdamW update (decoupled decay on the old parameter); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * (mh / (np.sqrt(vh) + eps) + wd * p), m, v


def nearest(q, t):
    """(squared distance, index) of each query's nearest reference row, lowest index on ties."""
    d2 = ((q[:, None, :] - t[None, :, :]) ** 2).sum(axis=2)
    idx = np.argmin(d2, axis=1)
    return d2[np.arange(len(q)), idx], idx


# ---------------------------------------------------------------- network

def layer_specs(enc=ENC, mid=MID, cin=CIN, cout=COUT):
    """(name, Cin, Cout, taps) of every convolution, in forward order."""
    specs = []
    c_prev = cin
    for l, c in enumerate(enc):
        specs += [(f"enc{l}a", c_prev, c, 9), (f"enc{l}b", c, c, 9)]
        c_prev = c
    specs += [("mida", c_prev, mid, 9), ("midb", mid, mid, 9)]
    c_prev = mid
    for l in reversed(range(len(enc))):
        c = enc[l]
        specs += [(f"up{l}", c_prev, c, 9), (f"dec{l}a", 2 * c, c, 9), (f"dec{l}b", c, c, 9)]
        c_prev = c
    specs.append(("head", c_prev, cout, 1))
    return specs


def param_count(specs=None):
    specs = specs or layer_specs()
    return sum(co * t * ci + co for _, ci, co, t in specs)


def init_params(rng, specs=None):
    """He-normal weights, zero biases (float64); rng is a numpy Generator."""
    specs = specs or layer_specs()
    P = {}
    for name, ci, co, t in specs:
        std = math.sqrt(2.0 / (ci * t))
        P[name] = (rng.standard_normal((co, t, ci)) * std, np.zeros(co))
    return P


def _levels(P):
    return sum(1 for k in P if k.startswith("enc") and k.endswith("a"))


def forward(P, x, storage=_ident, contact_residual=0.0):
    """Network output [n,H,W,Cout] and the cache the backward pass needs.

    contact_residual c adds c * min(x[..., 0], 0) to output channel 2 (the
    unrounded input, no parameters, so the backward pass is unchanged)."""
    levels = _levels(P)
    S = storage
    cache = {"x": S(x)}
    W = {k: (S(w), b) for k, (w, b) in P.items()}

    def cg(name, inp):
        zr = conv(inp, *W[name])
        z, a = S(zr), S(gelu(zr))
        cache[name] = (inp, z)
        return a

    h = cache["x"]
    skips = []
    for l in range(levels):
        h = cg(f"enc{l}b", cg(f"enc{l}a", h))
        skips.append(h)
        h = S(avgpool2(h))
    h = cg("midb", cg("mida", h))
    for l in reversed(range(levels)):
        u = S(upsample2(h))
        up = cg(f"up{l}", u)
        cat = np.concatenate([up, skips[l]], axis=-1)
        h = cg(f"dec{l}b", cg(f"dec{l}a", cat))
    out = conv(h, *W["head"])
    if contact_residual:
        out[..., 2] += contact_residual * np.minimum(x[..., 0], 0.0)
    cache["head"] = (h, None)
    cache["W"] = W
    return out, cache


def backward(cache, gout, storage=_ident):
    """Gradients {name: (dw, db)} of the loss whose output gradient is gout."""
    S = storage
    W = cache["W"]
    levels = _levels(W)
    G = {}

    def back(name, g_out_act):
        """g_out_act: gradient w.r.t. the GELU output of layer `name`; returns
        the gradient w.r.t. that layer's input."""
        inp, z = cache[name]
        gz = S(g_out_act * gelu_grad(z))
        dx, dw, db = conv_backward(inp, W[name][0], gz)
        G[name] = (dw, db)
        return S(dx)

    h, _ = cache["head"]
    dx, dw, db = conv_backward(h, W["head"][0], gout)
    G["head"] = (dw, db)
    g = S(dx)
    g_skip = [None] * levels
    for l in range(levels):
        c = W[f"up{l}"][0].shape[0]
        g = back(f"dec{l}a", back(f"dec{l}b", g))
        g_up, g_skip[l] = g[..., :c], g[..., c:]
        g = S(upsample2_backward(back(f"up{l}", g_up)))
    g = back("mida", back("midb", g))
    for l in reversed(range(levels)):
        g = S(g_skip[l] + avgpool2_backward(g))
        g = back(f"enc{l}a", back(f"enc{l}b", g))
    return G


def loss_and_grads(P, x, y, storage=_ident, contact_residual=0.0):
    out, cache = forward(P, x, storage, contact_residual)
    loss, gout = mse(out, y)
    return loss, out, backward(cache, gout, storage)
