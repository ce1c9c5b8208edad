"""Tactile surrogate network on the tsg_* kernels (argument marshalling only).

A 4-level U-Net maps the indenter's height field over the sensor and the press
depth (2 input channels on a res x res grid) to the elastomer surface's
displacement (3 channels). Encoder: two 3x3 convolutions + GELU per level
(32, 64, 128 channels), 2x2 average pooling between levels, 256 channels at
the bottleneck. Decoder: nearest x2 upsampling, a 3x3 convolution + GELU,
concatenation [upsampled, skip], two 3x3 convolutions + GELU. Head: a 1x1
convolution to 3 channels. Every convolution, pooling, gradient, loss and
optimiser step runs in the HIP library; this module owns the device buffers,
sequences the calls on the current stream and fails loudly without the
library or a GPU.

Storage: activations and gradients NHWC bfloat16, master weights, their
gradients and the AdamW moments FP32 in one flat buffer each, BF16 weight
packs refreshed after every optimiser step.
"""
from __future__ import annotations

import math

import torch

from . import native

ENC = (32, 64, 128)
MID = 256
CIN = 2
CIN_P = 8
COUT = 3
GELU, PLAIN, DGELU, F32 = 1, 0, 2, 3


def layer_specs(enc=ENC, mid=MID, cin=CIN, cout=COUT):
    """(name, Cin, Cout, taps) of every convolution in forward order."""
    specs, c_prev = [], cin
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


def forward_flops(res=64, enc=ENC, mid=MID, cin=CIN, cout=COUT):
    """Multiply-add FLOPs (2 per MAC) of one sample's forward convolutions."""
    L = len(enc)
    total = 0
    for name, ci, co, t in layer_specs(enc, mid, cin, cout):
        if name.startswith("enc"):
            r = res >> int(name[3])
        elif name.startswith("mid"):
            r = res >> L
        elif name == "head":
            r = res
        else:
            r = res >> int(name[-1] if name.startswith("up") else name[3])
        total += 2 * r * r * co * ci * t
    return total


def _ptr(t):
    return t.data_ptr()


class Net:
    """The surrogate with buffers for batches of up to `batch` samples."""

    def __init__(self, batch: int, res: int = 64, enc=ENC, mid=MID, seed: int = 0, device: str = "cuda",
                 contact_residual: float = 0.0):
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate kernels need a GPU")
        if res % (1 << len(enc)) or res < (1 << len(enc)):
            raise ValueError("res must be divisible by 2**levels")
        self.batch, self.res, self.enc, self.mid = batch, res, tuple(enc), mid
        # output channel 2 += contact_residual * min(input channel 0, 0), in FP32
        self.contact_residual = float(contact_residual)
        self.L = len(enc)
        self.dev = torch.device(device)
        self.specs = layer_specs(self.enc, mid)
        # a list to collect HIP events around each convolution launch (timing only), else None
        self.layer_timer = None
        self.N = native
        native.tsg()
        # flat FP32 master parameters, gradients and moments
        self.offsets = {}
        o = 0
        for name, ci, co, t in self.specs:
            self.offsets[name] = (o, o + co * t * ci, co, t, ci)
            o += co * t * ci + co
        self.nparams = o
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.flat = torch.zeros(o, **f32)
        self.grad = torch.zeros(o, **f32)
        self.m = torch.zeros(o, **f32)
        self.v = torch.zeros(o, **f32)
        self.step_count = 0
        g = torch.Generator().manual_seed(seed)
        for name, ci, co, t in self.specs:
            w, _ = self.param(name)
            w.copy_(torch.randn(co, t, ci, generator=g, dtype=torch.float32) * math.sqrt(2.0 / (ci * t)))
        # BF16 weight packs
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        self.cin_p = {name: (CIN_P if name == "enc0a" else ci) for name, ci, co, t in self.specs}
        self.wf, self.wt = {}, {}
        for name, ci, co, t in self.specs:
            self.wf[name] = torch.zeros(co, native.tsg().tsg_pack_k(t, self.cin_p[name]), **bf)
            if name not in ("enc0a", "head"):
                self.wt[name] = torch.zeros(self.cin_p[name], native.tsg().tsg_pack_k(t, co), **bf)
        self.repack()
        self._alloc(batch)

    # ------------------------------------------------------------ parameters

    def param(self, name):
        o, ob, co, t, ci = self.offsets[name]
        return self.flat[o:ob].view(co, t, ci), self.flat[ob:ob + co]

    def param_grad(self, name):
        o, ob, co, t, ci = self.offsets[name]
        return self.grad[o:ob].view(co, t, ci), self.grad[ob:ob + co]

    def state_dict(self):
        return {"flat": self.flat.detach().cpu(), "m": self.m.detach().cpu(), "v": self.v.detach().cpu(),
                "step": self.step_count, "res": self.res, "enc": list(self.enc), "mid": self.mid,
                "contact_residual": self.contact_residual}

    def load_state_dict(self, sd):
        if list(sd["enc"]) != list(self.enc) or sd["mid"] != self.mid or sd["res"] != self.res:
            raise ValueError("state was saved from a different architecture")
        self.flat.copy_(sd["flat"])
        self.m.copy_(sd["m"])
        self.v.copy_(sd["v"])
        self.step_count = int(sd["step"])
        self.contact_residual = float(sd.get("contact_residual", self.contact_residual))
        self.repack()

    def repack(self):
        s = self._stream()
        for name, ci, co, t in self.specs:
            w, _ = self.param(name)
            wt = self.wt.get(name)
            native.tsg_call("tsg_pack_weights", _ptr(w), co, ci, self.cin_p[name], co, t, _ptr(self.wf[name]),
                            _ptr(wt) if wt is not None else None, s)

    # ------------------------------------------------------------ buffers

    def _alloc(self, n):
        bf = dict(dtype=torch.bfloat16, device=self.dev)
        R = [self.res >> l for l in range(self.L + 1)]
        E = self.enc
        hc = [E[l + 1] if l + 1 < self.L else self.mid for l in range(self.L)]
        z = lambda r, c: torch.zeros(n, r, r, c, **bf)  # noqa: E731
        self.x = z(R[0], CIN_P)
        self.ea = [z(R[l], E[l]) for l in range(self.L)]
        self.zea = [z(R[l], E[l]) for l in range(self.L)]
        self.cat = [z(R[l], 2 * E[l]) for l in range(self.L)]
        self.zcat = [z(R[l], 2 * E[l]) for l in range(self.L)]
        self.p = [z(R[l + 1], E[l]) for l in range(self.L)]
        self.ma, self.zma = z(R[-1], self.mid), z(R[-1], self.mid)
        self.mb, self.zmb = z(R[-1], self.mid), z(R[-1], self.mid)
        self.ups = [z(R[l], hc[l]) for l in range(self.L)]
        self.da = [z(R[l], E[l]) for l in range(self.L)]
        self.zda = [z(R[l], E[l]) for l in range(self.L)]
        self.db = [z(R[l], E[l]) for l in range(self.L)]
        self.zdb = [z(R[l], E[l]) for l in range(self.L)]
        self.out = torch.zeros(n * R[0] * R[0], COUT, dtype=torch.float32, device=self.dev)
        # gradients
        self.gA = [z(R[l], E[l]) for l in range(self.L)]
        self.gB = [z(R[l], E[l]) for l in range(self.L)]
        self.gcat = [z(R[l], 2 * E[l]) for l in range(self.L)]
        self.gups = [z(R[l], hc[l]) for l in range(self.L)]
        self.gp = [z(R[l + 1], E[l]) for l in range(self.L)]
        self.gmA, self.gmB = z(R[-1], self.mid), z(R[-1], self.mid)
        self.dout = torch.zeros_like(self.out)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        self.mse_scratch = torch.zeros(1024, dtype=torch.float32, device=self.dev)
        T = native.tsg()
        ws = T.tsg_head_scratch_bytes(COUT, E[0])
        for name, ci, co, t in self.specs:
            r = self._res_of(name)
            ws = max(ws, T.tsg_wgrad_scratch_bytes(n, r, r, self.cin_p[name], co, t))
        self.ws_bytes = ws
        self.ws = torch.zeros((ws + 3) // 4, dtype=torch.float32, device=self.dev)

    def _res_of(self, name):
        if name.startswith("enc"):
            return self.res >> int(name[3])
        if name.startswith("mid"):
            return self.res >> self.L
        if name == "head":
            return self.res
        return self.res >> int(name[2] if name.startswith("up") else name[3])

    @staticmethod
    def _stream():
        return torch.cuda.current_stream().cuda_stream

    # ------------------------------------------------------------ kernels

    def _conv(self, name, n, r, src, src_ld, src_off, cin_p, out, out_ld, out_off, epi, z=None, z_ld=0, z_off=0,
              transposed=False, cout=None):
        """Forward convolution of layer `name` (or its input gradient when
        transposed) on n samples of r x r pixels."""
        _, ci, co, t = next(s for s in self.specs if s[0] == name)
        wp = self.wt[name] if transposed else self.wf[name]
        bias = None if transposed else _ptr(self.param(name)[1])
        cout = cout if cout is not None else (self.cin_p[name] if transposed else co)
        timer = getattr(self, "layer_timer", None)
        if timer is not None:
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record()
        native.tsg_call("tsg_conv", _ptr(src), n, r, r, src_ld, src_off, cin_p, _ptr(wp), bias, cout, t, epi,
                        _ptr(out) if out is not None else None, out_ld, out_off,
                        _ptr(z) if z is not None else None, z_ld, z_off,
                        _ptr(self.out) if epi == F32 else None, self._stream())
        if timer is not None:
            e1 = torch.cuda.Event(enable_timing=True)
            e1.record()
            # (layer, transposed, n, r, input channels as stored, output channels, taps, GELU z stored, events)
            timer.append((name, transposed, n, r, cin_p, cout, t, z is not None, e0, e1))

    def _wgrad(self, name, n, r, src, src_ld, src_off, cin, cin_p, g, g_ld, g_off):
        _, _, co, t = next(s for s in self.specs if s[0] == name)
        dw, db = self.param_grad(name)
        native.tsg_call("tsg_conv_wgrad", _ptr(src), n, r, r, src_ld, src_off, cin, cin_p, _ptr(g), g_ld, g_off,
                        co, t, _ptr(dw), _ptr(db), _ptr(self.ws), self.ws_bytes, self._stream())

    # ------------------------------------------------------------ forward / backward

    def set_input(self, x32):
        """x32: FP32 [n, res, res, 2] (height field, depth) on the device."""
        n = x32.shape[0]
        if n > self.batch or tuple(x32.shape[1:]) != (self.res, self.res, CIN):
            raise ValueError("input must be [n <= batch, res, res, 2]")
        x32 = x32.contiguous()
        self._x32 = x32
        native.tsg_call("tsg_to_bf16", _ptr(x32), n * self.res * self.res, CIN, _ptr(self.x), CIN_P,
                        self._stream())
        return n

    def forward(self, x32):
        """Network output, FP32 [n, res, res, 3] (a view of an internal buffer)."""
        n = self.set_input(x32)
        self._forward(n)
        return self.out[:n * self.res * self.res].view(n, self.res, self.res, COUT)

    def _forward(self, n):
        E, L = self.enc, self.L
        src, ld, cp = self.x, CIN_P, CIN_P
        for l in range(L):
            r, c = self.res >> l, E[l]
            self._conv(f"enc{l}a", n, r, src, ld, 0, cp, self.ea[l], c, 0, GELU, self.zea[l], c, 0)
            self._conv(f"enc{l}b", n, r, self.ea[l], c, 0, c, self.cat[l], 2 * c, c, GELU, self.zcat[l], 2 * c, c)
            native.tsg_call("tsg_avgpool2", _ptr(self.cat[l]), n, r, r, c, 2 * c, c, _ptr(self.p[l]), c, 0,
                            self._stream())
            src, ld, cp = self.p[l], c, c
        r = self.res >> L
        self._conv("mida", n, r, src, ld, 0, cp, self.ma, self.mid, 0, GELU, self.zma, self.mid, 0)
        self._conv("midb", n, r, self.ma, self.mid, 0, self.mid, self.mb, self.mid, 0, GELU, self.zmb, self.mid, 0)
        src, hc = self.mb, self.mid
        for l in reversed(range(L)):
            r, c = self.res >> l, E[l]
            native.tsg_call("tsg_upsample2", _ptr(src), n, r // 2, r // 2, hc, hc, 0, _ptr(self.ups[l]), hc, 0,
                            self._stream())
            self._conv(f"up{l}", n, r, self.ups[l], hc, 0, hc, self.cat[l], 2 * c, 0, GELU, self.zcat[l], 2 * c, 0)
            self._conv(f"dec{l}a", n, r, self.cat[l], 2 * c, 0, 2 * c, self.da[l], c, 0, GELU, self.zda[l], c, 0)
            self._conv(f"dec{l}b", n, r, self.da[l], c, 0, c, self.db[l], c, 0, GELU, self.zdb[l], c, 0)
            src, hc = self.db[l], c
        self._conv("head", n, self.res, self.db[0], E[0], 0, E[0], None, 0, 0, F32)
        if self.contact_residual != 0.0:
            native.tsg_call("tsg_contact_residual", _ptr(self.out), _ptr(self._x32), n * self.res * self.res,
                            self.contact_residual, self._stream())

    def _backward(self, n):
        E, L, s = self.enc, self.L, self._stream()
        r0 = self.res
        npix0 = n * r0 * r0
        wh, _ = self.param("head")
        dwh, dbh = self.param_grad("head")
        native.tsg_call("tsg_conv_wgrad_f32", _ptr(self.db[0]), n, r0, r0, E[0], 0, E[0], E[0], _ptr(self.dout), COUT,
                        _ptr(dwh), _ptr(dbh), _ptr(self.ws), self.ws_bytes, s)
        native.tsg_call("tsg_head_dgrad", _ptr(self.dout), npix0, COUT, _ptr(wh), E[0], _ptr(self.gB[0]), E[0], 0,
                        _ptr(self.zdb[0]), E[0], 0, s)
        for l in range(L):
            r, c = self.res >> l, E[l]
            hc = E[l + 1] if l + 1 < L else self.mid
            npix = n * r * r
            # dec{l}b: gradient of its pre-activation in gB[l]
            self._wgrad(f"dec{l}b", n, r, self.da[l], c, 0, c, c, self.gB[l], c, 0)
            self._conv(f"dec{l}b", n, r, self.gB[l], c, 0, c, self.gA[l], c, 0, DGELU, self.zda[l], c, 0,
                       transposed=True)
            self._wgrad(f"dec{l}a", n, r, self.cat[l], 2 * c, 0, 2 * c, 2 * c, self.gA[l], c, 0)
            self._conv(f"dec{l}a", n, r, self.gA[l], c, 0, c, self.gcat[l], 2 * c, 0, PLAIN, transposed=True)
            native.tsg_call("tsg_dgelu", _ptr(self.gcat[l]), 2 * c, 0, _ptr(self.zcat[l]), 2 * c, 0, npix, c, s)
            self._wgrad(f"up{l}", n, r, self.ups[l], hc, 0, hc, hc, self.gcat[l], 2 * c, 0)
            self._conv(f"up{l}", n, r, self.gcat[l], 2 * c, 0, c, self.gups[l], hc, 0, PLAIN, transposed=True)
            if l + 1 < L:
                dst, zdst = self.gB[l + 1], self.zdb[l + 1]
            else:
                dst, zdst = self.gmB, self.zmb
            native.tsg_call("tsg_upsample2_bwd_dgelu", _ptr(self.gups[l]), n, r // 2, r // 2, hc, hc, 0, _ptr(dst), hc, 0,
                            _ptr(zdst), hc, 0, s)
        r = self.res >> L
        cl = E[L - 1]
        self._wgrad("midb", n, r, self.ma, self.mid, 0, self.mid, self.mid, self.gmB, self.mid, 0)
        self._conv("midb", n, r, self.gmB, self.mid, 0, self.mid, self.gmA, self.mid, 0, DGELU, self.zma, self.mid, 0,
                   transposed=True)
        self._wgrad("mida", n, r, self.p[L - 1], cl, 0, cl, cl, self.gmA, self.mid, 0)
        self._conv("mida", n, r, self.gmA, self.mid, 0, self.mid, self.gp[L - 1], cl, 0, PLAIN, transposed=True)
        for l in reversed(range(L)):
            r, c = self.res >> l, E[l]
            native.tsg_call("tsg_avgpool2_bwd_dgelu", _ptr(self.gp[l]), n, r, r, c, c, 0, _ptr(self.gcat[l]), 2 * c, c, 1,
                            _ptr(self.zcat[l]), 2 * c, c, s)
            self._wgrad(f"enc{l}b", n, r, self.ea[l], c, 0, c, c, self.gcat[l], 2 * c, c)
            self._conv(f"enc{l}b", n, r, self.gcat[l], 2 * c, c, c, self.gA[l], c, 0, DGELU, self.zea[l], c, 0,
                       transposed=True)
            if l == 0:
                self._wgrad("enc0a", n, r, self.x, CIN_P, 0, CIN, CIN_P, self.gA[0], c, 0)
            else:
                cp = E[l - 1]
                self._wgrad(f"enc{l}a", n, r, self.p[l - 1], cp, 0, cp, cp, self.gA[l], c, 0)
                self._conv(f"enc{l}a", n, r, self.gA[l], c, 0, c, self.gp[l - 1], cp, 0, PLAIN, transposed=True)

    def loss_and_grads(self, x32, y32):
        """Forward, MSE against y32 (FP32 [n, res, res, 3]) and backward; the
        gradients land in self.grad. Returns the loss as a device scalar."""
        n = self.set_input(x32)
        if tuple(y32.shape) != (n, self.res, self.res, COUT):
            raise ValueError("target must be [n, res, res, 3]")
        self._forward(n)
        count = n * self.res * self.res * COUT
        y32 = y32.contiguous()
        native.tsg_call("tsg_mse", _ptr(self.out), _ptr(y32), count, _ptr(self.loss), _ptr(self.dout),
                        _ptr(self.mse_scratch), self._stream())
        self._backward(n)
        return self.loss

    def adamw(self, lr, b1=0.9, b2=0.999, eps=1e-8, wd=1e-2):
        self.step_count += 1
        native.tsg_call("tsg_adamw", _ptr(self.flat), _ptr(self.grad), _ptr(self.m), _ptr(self.v), self.nparams,
                        lr, b1, b2, eps, wd, self.step_count, self._stream())
        self.repack()

    def train_step(self, x32, y32, lr, **opt):
        loss = self.loss_and_grads(x32, y32)
        self.adamw(lr, **opt)
        return loss
