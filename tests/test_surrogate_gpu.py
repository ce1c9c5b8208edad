"""Surrogate kernels and network on the GPU against the FP64 reference.

Each kernel is compared element by element with the reference evaluated on
the same bfloat16-rounded operands. Bounds: products of two bfloat16 values
are exact in FP32, so a K-term FP32 accumulation is off by at most
K 2^-24 sum|terms|; storing a result as bfloat16 adds at most 2^-8 of its
magnitude (8-bit significand, round to nearest); an error in a pre-activation
reaches GELU's output, or GELU' times a gradient, amplified by at most 1.13
(the largest |GELU'| and |GELU''| on the reals are below that); erff and expf
add a few FP32 ulps.
"""
import math

import numpy as np
import pytest

from oracle import surrogate as R

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U_BF = 2.0 ** -8
U_32 = 2.0 ** -24
LIP = 1.13


@pytest.fixture(scope="module")
def T():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd import native
    native.tsg()
    return native


def bf16_dev(a):
    """numpy float64 -> device bfloat16 (the rounding the reference sees)."""
    return torch.tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def f32_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().double().numpy()


def stream():
    return torch.cuda.current_stream().cuda_stream


def pack(T, w, cin_p, cout_p):
    co, taps, ci = w.shape
    wd = f32_dev(w)
    kf, kt = T.tsg().tsg_pack_k(taps, cin_p), T.tsg().tsg_pack_k(taps, cout_p)
    wf = torch.zeros(co, kf, dtype=torch.bfloat16, device="cuda")
    wt = torch.zeros(cin_p, kt, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_pack_weights", wd.data_ptr(), co, ci, cin_p, cout_p, taps, wf.data_ptr(), wt.data_ptr(), stream())
    return wf, wt


def pad_channels(x, cp, off=0, ld=None):
    """Place x [n,h,w,c] at channel offset off of a zero [n,h,w,ld] array."""
    ld = ld or cp
    out = np.zeros(x.shape[:3] + (ld,))
    out[..., off:off + x.shape[-1]] = x
    return out


CONV_CASES = [
    # n, h, w, cin, cin_p, ld_in, off_in, cout, taps
    (2, 9, 7, 2, 8, 8, 0, 32, 9),        # the input layer, 126 pixels (ragged)
    (1, 13, 11, 40, 40, 56, 16, 20, 9),  # channel slice of a wider buffer, ragged cout
    (3, 8, 8, 64, 64, 64, 0, 128, 9),    # 64-channel tiles of the deep layers
    (2, 5, 6, 32, 32, 32, 0, 48, 1),     # 1x1
    # the LDS-staged kernel (rows of 4..64 pixels, channels in 32s): images
    # shorter than a workgroup's 256 pixels and a partial last workgroup,
    # 32-channel chunks of a channel slice, a ragged 32-channel output tile
    (3, 5, 8, 32, 32, 48, 8, 48, 9),
    (1, 6, 64, 64, 64, 64, 0, 32, 9),     # 64-pixel rows, 4 rows per workgroup
    (2, 7, 4, 96, 96, 96, 0, 64, 9),      # 4-pixel rows, three 32-channel chunks
    (1, 9, 32, 64, 64, 128, 64, 32, 9),   # 32-pixel rows, second half of a 128-channel buffer
    (3, 16, 16, 32, 32, 32, 0, 32, 9),    # 16-pixel rows: one whole image per workgroup
    (2, 64, 64, 32, 32, 32, 0, 32, 9),    # whole 64 x 64 images: edge taps masked on all four sides
]


@pytest.mark.parametrize("case", CONV_CASES)
@pytest.mark.parametrize("epi", [0, 1, 3])
def test_conv_forward(T, case, epi):
    n, h, w, cin, cin_p, ld, off, cout, taps = case
    rng = np.random.default_rng(7 * sum(case) + epi)
    x = R.round_bf16(rng.standard_normal((n, h, w, cin)))
    wt = R.round_bf16(rng.standard_normal((cout, taps, cin)) / math.sqrt(cin * taps))
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    xin = bf16_dev(pad_channels(x, cin_p, off, ld))
    wf, _ = pack(T, wt, cin_p, ((cout + 7) // 8) * 8)
    bd = f32_dev(b)
    out_ld, out_off = cout + 8, 4
    out = torch.zeros(n, h, w, out_ld, dtype=torch.bfloat16, device="cuda")
    z = torch.zeros(n, h, w, out_ld, dtype=torch.bfloat16, device="cuda")
    out32 = torch.zeros(n * h * w, cout, dtype=torch.float32, device="cuda")
    T.tsg_call("tsg_conv", xin.data_ptr(), n, h, w, ld, off, cin_p, wf.data_ptr(), bd.data_ptr(), cout, taps, epi,
               out.data_ptr(), out_ld, out_off, z.data_ptr(), out_ld, out_off, out32.data_ptr(), stream())
    ref = R.conv(x, wt, b)
    acc_tol = cin_p * taps * U_32 * R.conv(np.abs(x), np.abs(wt), np.abs(b)) + 1e-30
    if epi == 3:
        got = host(out32).reshape(n, h, w, cout)
        assert np.all(np.abs(got - ref) <= acc_tol)
        return
    got = host(out)
    # channels outside the output slice stay untouched
    assert np.all(got[..., :out_off] == 0) and np.all(got[..., out_off + cout:] == 0)
    got = got[..., out_off:out_off + cout]
    if epi == 0:
        assert np.all(np.abs(got - ref) <= U_BF * (np.abs(ref) + acc_tol) + acc_tol)
    else:
        zg = host(z)[..., out_off:out_off + cout]
        assert np.all(np.abs(zg - ref) <= U_BF * (np.abs(ref) + acc_tol) + acc_tol)
        g = R.gelu(ref)
        assert np.all(np.abs(got - g) <= U_BF * (np.abs(g) + LIP * acc_tol) + LIP * acc_tol + 1e-6 * (1 + np.abs(g)))


@pytest.mark.parametrize("case", [(2, 9, 7, 32, 32, 9), (1, 16, 16, 64, 128, 9), (2, 6, 5, 48, 24, 9),
                                  (2, 8, 32, 32, 64, 9), (3, 16, 16, 32, 32, 9)])
@pytest.mark.parametrize("fuse_gelu", [False, True])
def test_conv_input_gradient(T, case, fuse_gelu):
    """Transposed, flipped packs give the input gradient; DGELU multiplies by
    GELU' of the stored pre-activation of the forward input."""
    n, h, w, cin, cout, taps = case
    rng = np.random.default_rng(11 + cin + cout + fuse_gelu)
    x = R.round_bf16(rng.standard_normal((n, h, w, cin)))
    wt = R.round_bf16(rng.standard_normal((cout, taps, cin)) / math.sqrt(cin * taps))
    g = R.round_bf16(rng.standard_normal((n, h, w, cout)))
    zin = R.round_bf16(rng.standard_normal((n, h, w, cin)) * 2)
    _, wtp = pack(T, wt, cin, cout)
    gd, zd = bf16_dev(g), bf16_dev(zin)
    out = torch.zeros(n, h, w, cin, dtype=torch.bfloat16, device="cuda")
    epi = 2 if fuse_gelu else 0
    T.tsg_call("tsg_conv", gd.data_ptr(), n, h, w, cout, 0, cout, wtp.data_ptr(), None, cin, taps, epi,
               out.data_ptr(), cin, 0, zd.data_ptr() if fuse_gelu else None, cin, 0, None, stream())
    dx, _, _ = R.conv_backward(x, wt, g)
    adx, _, _ = R.conv_backward(x, np.abs(wt), np.abs(g))
    acc_tol = cout * taps * U_32 * adx + 1e-30
    got = host(out)
    if fuse_gelu:
        gg = R.gelu_grad(zin)
        ref = dx * gg
        tol = U_BF * (np.abs(ref) + LIP * acc_tol) + LIP * acc_tol + 1e-6 * np.abs(dx)
    else:
        ref = dx
        tol = U_BF * (np.abs(ref) + acc_tol) + acc_tol
    assert np.all(np.abs(got - ref) <= tol)


@pytest.mark.parametrize("case", [
    # n, h, w, cin, cin_p, ld_in, off_in, cout, ld_g, off_g, taps
    (2, 9, 7, 2, 8, 8, 0, 32, 32, 0, 9),
    (2, 16, 16, 64, 64, 64, 0, 32, 64, 32, 9),
    (1, 8, 8, 40, 40, 48, 8, 24, 24, 0, 9),
    (3, 33, 31, 32, 32, 32, 0, 64, 64, 0, 9),
    # the all-taps kernel (h w a multiple of 128, 16 <= w <= 64): widths 32 and 64,
    # partial channel blocks, strided and offset layouts, several images
    (2, 32, 32, 32, 32, 32, 0, 32, 32, 0, 9),
    (1, 64, 64, 40, 48, 48, 0, 24, 24, 0, 9),
    (3, 16, 16, 20, 24, 48, 24, 36, 40, 4, 9),
    # 8-pixel rows: the all-taps kernel with 64-pixel chunks (one 8 x 8 image each)
    (5, 8, 8, 32, 32, 64, 32, 64, 64, 0, 9),
    # 64-pixel chunks of 16- and 64-pixel rows (images of 64 pixels)
    (4, 4, 16, 32, 32, 32, 0, 32, 32, 0, 9),
    (3, 1, 64, 32, 32, 32, 0, 32, 32, 0, 9),
    # 102 splits of the 81920 pixels rounded up to 896 each: the last 10
    # would be empty (they are not launched; their halo rows lie past the batch)
    (80, 32, 32, 32, 32, 32, 0, 160, 160, 0, 9),
])
def test_conv_weight_gradient(T, case):
    n, h, w, cin, cin_p, ld, off, cout, gld, goff, taps = case
    rng = np.random.default_rng(21 + cout + cin)
    x = R.round_bf16(rng.standard_normal((n, h, w, cin)))
    g = R.round_bf16(rng.standard_normal((n, h, w, cout)))
    xin = bf16_dev(pad_channels(x, cin_p, off, ld))
    gd = bf16_dev(pad_channels(g, cout, goff, gld))
    dw = torch.zeros(cout, taps, cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nb = T.tsg().tsg_wgrad_scratch_bytes(n, h, w, cin_p, cout, taps)
    scratch = torch.zeros((nb + 3) // 4, dtype=torch.float32, device="cuda")
    T.tsg_call("tsg_conv_wgrad", xin.data_ptr(), n, h, w, ld, off, cin, cin_p, gd.data_ptr(), gld, goff, cout, taps,
               dw.data_ptr(), db.data_ptr(), scratch.data_ptr(), nb, stream())
    w0 = np.zeros((cout, taps, cin))
    _, rdw, rdb = R.conv_backward(x, w0, g)
    _, adw, adb = R.conv_backward(np.abs(x), w0, np.abs(g))
    npix = n * h * w
    assert np.all(np.abs(host(dw) - rdw) <= npix * U_32 * adw + 1e-30)
    assert np.all(np.abs(host(db) - rdb) <= npix * U_32 * adb + 1e-30)
    # deterministic: a second call gives identical bits
    dw2 = dw.clone()
    T.tsg_call("tsg_conv_wgrad", xin.data_ptr(), n, h, w, ld, off, cin, cin_p, gd.data_ptr(), gld, goff, cout, taps,
               dw.data_ptr(), db.data_ptr(), scratch.data_ptr(), nb, stream())
    assert torch.equal(dw, dw2)


@pytest.mark.parametrize("cin,with_z", [(32, True), (32, False), (20, True)])  # 8-channel path, and per channel
def test_head_gradients(T, cin, with_z):
    n, h, w, cout = 2, 16, 12, 3
    rng = np.random.default_rng(31 + cin)
    x = R.round_bf16(rng.standard_normal((n, h, w, cin)))
    z = R.round_bf16(rng.standard_normal((n, h, w, cin)))
    g = rng.standard_normal((n, h, w, cout)).astype(np.float32).astype(np.float64)
    wt = rng.standard_normal((cout, 1, cin)).astype(np.float32).astype(np.float64)
    xd, zd, gdv, wd = bf16_dev(x), bf16_dev(z), f32_dev(g.reshape(-1, cout)), f32_dev(wt)
    dw = torch.zeros(cout, cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    nb = T.tsg().tsg_head_scratch_bytes(cout, cin)
    scratch = torch.zeros((nb + 3) // 4, dtype=torch.float32, device="cuda")
    T.tsg_call("tsg_conv_wgrad_f32", xd.data_ptr(), n, h, w, cin, 0, cin, cin, gdv.data_ptr(), cout, dw.data_ptr(),
               db.data_ptr(), scratch.data_ptr(), nb, stream())
    din = torch.zeros(n, h, w, cin, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_head_dgrad", gdv.data_ptr(), n * h * w, cout, wd.data_ptr(), cin, din.data_ptr(), cin, 0,
               zd.data_ptr() if with_z else None, cin, 0, stream())
    dx, rdw, rdb = R.conv_backward(x, wt, g)
    _, adw, adb = R.conv_backward(np.abs(x), wt, np.abs(g))
    adx, _, _ = R.conv_backward(x, np.abs(wt), np.abs(g))
    npix = n * h * w
    assert np.all(np.abs(host(dw) - rdw[:, 0, :]) <= 2 * npix * U_32 * adw[:, 0, :])
    assert np.all(np.abs(host(db) - rdb) <= 2 * npix * U_32 * adb)
    ref = dx * R.gelu_grad(z) if with_z else dx
    acc = cout * U_32 * adx
    assert np.all(np.abs(host(din) - ref) <= U_BF * (np.abs(ref) + LIP * acc) + LIP * acc + 1e-6 * np.abs(dx))


@pytest.mark.parametrize("c,ld,off", [(16, 24, 8), (4, 6, 2)])  # 8-channel vector path, scalar path
def test_pool_upsample_and_elementwise(T, c, ld, off):
    n, h, w = 2, 6, 10
    rng = np.random.default_rng(41)
    x = R.round_bf16(rng.standard_normal((n, h, w, c)))
    xd = bf16_dev(pad_channels(x, c, off, ld))
    s = stream()
    # pooling into a channel slice
    p = torch.zeros(n, h // 2, w // 2, 2 * c, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_avgpool2", xd.data_ptr(), n, h, w, c, ld, off, p.data_ptr(), 2 * c, c, s)
    ref = R.avgpool2(x)
    got = host(p)
    assert np.all(got[..., :c] == 0)
    assert np.all(np.abs(got[..., c:] - ref) <= U_BF * np.abs(ref) + 4 * U_32 * R.avgpool2(np.abs(x)))
    # pooling backward, written then accumulated
    g = R.round_bf16(rng.standard_normal((n, h // 2, w // 2, c)))
    gd = bf16_dev(g)
    din = torch.zeros(n, h, w, c, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_avgpool2_bwd", gd.data_ptr(), n, h, w, c, c, 0, din.data_ptr(), c, 0, 0, s)
    assert np.array_equal(host(din), R.avgpool2_backward(g))  # quarter of a bf16 value is exact
    T.tsg_call("tsg_avgpool2_bwd", gd.data_ptr(), n, h, w, c, c, 0, din.data_ptr(), c, 0, 1, s)
    ref2 = 2 * R.avgpool2_backward(g)
    assert np.array_equal(host(din), ref2)
    # upsampling copies exactly; its backward sums four children
    up = torch.zeros(n, 2 * h, 2 * w, c, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_upsample2", xd.data_ptr(), n, h, w, c, ld, off, up.data_ptr(), c, 0, s)
    assert np.array_equal(host(up), R.upsample2(x))
    big = R.round_bf16(rng.standard_normal((n, 2 * h, 2 * w, c)))
    bd = bf16_dev(big)
    ub = torch.zeros(n, h, w, c, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_upsample2_bwd", bd.data_ptr(), n, h, w, c, c, 0, ub.data_ptr(), c, 0, s)
    ref = R.upsample2_backward(big)
    assert np.all(np.abs(host(ub) - ref) <= U_BF * np.abs(ref) + 4 * U_32 * R.upsample2_backward(np.abs(big)))
    # add in place and GELU' on channel slices
    a = R.round_bf16(rng.standard_normal((n * h * w, c)))
    b = R.round_bf16(rng.standard_normal((n * h * w, c)))
    ad = bf16_dev(pad_channels(a.reshape(n, h, w, c), c, off, ld))
    bdv = bf16_dev(b)
    T.tsg_call("tsg_add_inplace", ad.data_ptr(), ld, off, bdv.data_ptr(), c, 0, n * h * w, c, s)
    ref = (a + b).reshape(n, h, w, c)
    assert np.all(np.abs(host(ad)[..., off:off + c] - ref) <= U_BF * np.abs(ref))
    zz = R.round_bf16(rng.standard_normal((n * h * w, c)) * 2)
    zd = bf16_dev(zz)
    dd = bf16_dev(a)
    T.tsg_call("tsg_dgelu", dd.data_ptr(), c, 0, zd.data_ptr(), c, 0, n * h * w, c, s)
    ref = a * R.gelu_grad(zz)
    assert np.all(np.abs(host(dd) - ref) <= U_BF * np.abs(ref) + 1e-6 * np.abs(a))
    # the pooling and upsampling gradients with GELU' fused (z in its own
    # strided layout): one rounding of the product, or two on the scalar path
    zf = R.round_bf16(rng.standard_normal((n, h, w, c)) * 2)
    zfd = bf16_dev(pad_channels(zf, c, off, ld))
    gg = R.gelu_grad(zf)
    d0 = R.round_bf16(rng.standard_normal((n, h, w, c)))
    din = bf16_dev(d0)
    T.tsg_call("tsg_avgpool2_bwd_dgelu", gd.data_ptr(), n, h, w, c, c, 0, din.data_ptr(), c, 0, 1, zfd.data_ptr(), ld,
               off, s)
    pre = d0 + R.avgpool2_backward(g)
    ref = pre * gg
    assert np.all(np.abs(host(din) - ref) <= 2 * U_BF * np.abs(ref) + 1e-6 * np.abs(pre))
    ub = torch.zeros(n, h, w, c, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_upsample2_bwd_dgelu", bd.data_ptr(), n, h, w, c, c, 0, ub.data_ptr(), c, 0, zfd.data_ptr(), ld, off,
               s)
    pre = R.upsample2_backward(big)
    ref = pre * gg
    bound = 2 * U_BF * np.abs(ref) + 4 * U_32 * R.upsample2_backward(np.abs(big)) * np.abs(gg) + 1e-6 * np.abs(pre)
    assert np.all(np.abs(host(ub) - ref) <= bound)


def test_to_bf16_pads_channels(T):
    rng = np.random.default_rng(51)
    a = rng.standard_normal((77, 2)) * 3
    src = f32_dev(a)
    dst = torch.full((77, 8), 7.0, dtype=torch.bfloat16, device="cuda")
    T.tsg_call("tsg_to_bf16", src.data_ptr(), 77, 2, dst.data_ptr(), 8, stream())
    got = host(dst)
    assert np.array_equal(got[:, :2], R.round_bf16(a.astype(np.float32)))
    assert np.all(got[:, 2:] == 0)


@pytest.mark.parametrize("count", [1, 1000, 3 * 64 * 64 * 5 + 17])
def test_mse(T, count):
    rng = np.random.default_rng(61 + count)
    p = rng.standard_normal(count).astype(np.float32).astype(np.float64)
    t = rng.standard_normal(count).astype(np.float32).astype(np.float64)
    pd, td = f32_dev(p), f32_dev(t)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dp = torch.zeros(count, dtype=torch.float32, device="cuda")
    scratch = torch.zeros(1024, dtype=torch.float32, device="cuda")
    T.tsg_call("tsg_mse", pd.data_ptr(), td.data_ptr(), count, loss.data_ptr(), dp.data_ptr(), scratch.data_ptr(),
               stream())
    rl, rg = R.mse(p, t)
    assert abs(host(loss)[0] - rl) <= (count + 1030) * U_32 * rl * 2
    assert np.all(np.abs(host(dp) - rg) <= 4 * U_32 * np.abs(rg))


def test_adamw(T):
    rng = np.random.default_rng(71)
    n = 10_000
    pd = f32_dev(rng.standard_normal(n))
    md = torch.zeros(n, dtype=torch.float32, device="cuda")
    vd = torch.zeros(n, dtype=torch.float32, device="cuda")
    for step in range(1, 4):
        p0, m0, v0 = host(pd), host(md), host(vd)
        g = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        gd = f32_dev(g)
        T.tsg_call("tsg_adamw", pd.data_ptr(), gd.data_ptr(), md.data_ptr(), vd.data_ptr(), n, 2e-3, 0.9, 0.999,
                   1e-8, 1e-2, step, stream())
        # the hyperparameters are FP32 arguments: the reference takes their FP32 values
        f = lambda a: float(np.float32(a))  # noqa: E731
        p, m, v = R.adamw(p0, g, m0, v0, step, lr=f(2e-3), b1=f(0.9), b2=f(0.999), eps=f(1e-8), wd=f(1e-2))
        # a step moves p by about lr; FP32 arithmetic is off by a few ulps of p and of the step
        assert np.all(np.abs(host(pd) - p) <= 8 * 2.0 ** -23 * (np.abs(p) + 2e-3)), step
        # m = b1 m0 + (1 - b1) g can cancel: bound by the magnitudes of its two terms
        assert np.all(np.abs(host(md) - m) <= 2.0 ** -22 * (f(0.9) * np.abs(m0) + (1 - f(0.9)) * np.abs(g)))
        assert np.all(np.abs(host(vd) - v) <= 4 * 2.0 ** -23 * np.abs(v) + 1e-30)


def test_nearest_neighbour(T):
    rng = np.random.default_rng(81)
    t = rng.standard_normal((3000, 257)).astype(np.float32).astype(np.float64)
    q = np.concatenate([rng.standard_normal((40, 257)), t[[5, 2999]] + 1e-3]).astype(np.float32).astype(np.float64)
    qd, td = f32_dev(q), f32_dev(t)
    d2 = torch.zeros(len(q), dtype=torch.float32, device="cuda")
    idx = torch.zeros(len(q), dtype=torch.int32, device="cuda")
    T.tsg_call("tsg_nn_dist", qd.data_ptr(), len(q), td.data_ptr(), len(t), 257, d2.data_ptr(), idx.data_ptr(),
               stream())
    rd, ri = R.nearest(q, t)
    # the index is unique where the runner-up is farther than the FP32 error of a distance
    all_d = ((q[:, None, :] - t[None, :, :]) ** 2).sum(axis=2)
    second = np.partition(all_d, 1, axis=1)[:, 1]
    sure = second - rd > 1e-4 * (1 + rd)
    gi = idx.cpu().numpy()
    assert np.all(gi[sure] == ri[sure])
    assert np.all(np.abs(host(d2) - rd) <= 257 * 4 * U_32 * (rd + (q ** 2).sum(1) + 1))
    assert gi[-2] == 5 and gi[-1] == 2999


# ---------------------------------------------------------------- whole network


def net_params(net):
    P = {}
    for name, ci, co, t in net.specs:
        w, b = net.param(name)
        P[name] = (w.detach().cpu().double().numpy(), b.detach().cpu().double().numpy())
    return P


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30))


@pytest.mark.parametrize("n,res", [(2, 64), (3, 32)])
def test_network_forward_and_gradients_match_reference(T, n, res):
    """Whole-network parity with the reference evaluated at the kernels'
    storage precision (every stored tensor rounded to bfloat16, FP64
    arithmetic). What remains is FP32 accumulation order, erff, and the odd
    rounding flip where an FP32 value sits at a bfloat16 rounding boundary;
    those stay far below the 2^-8 storage rounding per layer, so relative L2
    errors of 1e-2 (output) and 3e-2 (each weight gradient) bound them with
    margin while a wrong index, tap or operand shows up as O(1)."""
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=4, res=res, seed=3, contact_residual=10.0)
    rng = np.random.default_rng(91 + n)
    # biases away from zero so their gradients and the epilogue are exercised
    for name, ci, co, t in net.specs:
        net.param(name)[1].copy_(torch.tensor(rng.standard_normal(co) * 0.05, dtype=torch.float32))
    net.repack()
    x = rng.standard_normal((n, res, res, 2)).astype(np.float32)
    y = rng.standard_normal((n, res, res, 3)).astype(np.float32)
    loss = net.loss_and_grads(torch.tensor(x).cuda(), torch.tensor(y).cuda())
    out = host(net.out)[:n * res * res].reshape(n, res, res, 3)
    P = net_params(net)
    rl, rout, G = R.loss_and_grads(P, x.astype(np.float64), y.astype(np.float64), storage=R.round_bf16,
                                   contact_residual=10.0)
    e_out = rel_l2(out, rout)
    print(f"n={n} res={res}: output rel L2 {e_out:.2e}, loss {host(loss)[0]:.6f} vs {rl:.6f}")
    assert e_out <= 1e-2
    assert abs(host(loss)[0] - rl) <= 2e-2 * rl
    worst = 0.0
    for name, ci, co, t in net.specs:
        dw, db = net.param_grad(name)
        ew = rel_l2(host(dw), G[name][0])
        eb = rel_l2(host(db), G[name][1])
        worst = max(worst, ew, eb)
        assert ew <= 3e-2 and eb <= 3e-2, (name, ew, eb)
    print(f"worst gradient rel L2 {worst:.2e}")


def test_network_gradients_are_deterministic(T):
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=2, res=32, seed=4)
    rng = np.random.default_rng(101)
    x = torch.tensor(rng.standard_normal((2, 32, 32, 2)).astype(np.float32)).cuda()
    y = torch.tensor(rng.standard_normal((2, 32, 32, 3)).astype(np.float32)).cuda()
    net.loss_and_grads(x, y)
    g1 = net.grad.clone()
    net.loss_and_grads(x, y)
    assert torch.equal(g1, net.grad)


def test_training_reduces_the_loss(T):
    """A fixed smooth target field: 150 AdamW steps cut the MSE by 10x
    (measured 20x: 1.21e-2 -> 6.0e-4)."""
    from paper_2301_08343_amd.surrogate import Net
    net = Net(batch=8, res=32, seed=5)
    rng = np.random.default_rng(111)
    yy, xx = np.meshgrid(np.linspace(-1, 1, 32), np.linspace(-1, 1, 32), indexing="ij")
    xs, ys = [], []
    for _ in range(8):
        c = rng.uniform(-0.5, 0.5, 2)
        d = rng.uniform(0.2, 1.0)
        hgt = np.exp(-((xx - c[0]) ** 2 + (yy - c[1]) ** 2) / 0.1)
        xs.append(np.stack([hgt, np.full_like(hgt, d)], -1))
        ys.append(np.stack([0.3 * d * np.gradient(hgt, axis=1), 0.3 * d * np.gradient(hgt, axis=0), -d * hgt], -1))
    x = torch.tensor(np.array(xs, dtype=np.float32)).cuda()
    y = torch.tensor(np.array(ys, dtype=np.float32)).cuda()
    first = float(net.train_step(x, y, lr=2e-3).item())
    for _ in range(149):
        last = net.train_step(x, y, lr=2e-3)
    last = float(last.item())
    print(f"loss {first:.4e} -> {last:.4e}")
    assert last < 0.1 * first


def test_router_features_and_per_sample_mse(T):
    rng = np.random.default_rng(121)
    n, h, w, f = 3, 16, 12, 4
    gap = rng.standard_normal((n, h, w)).astype(np.float32).astype(np.float64)
    depth = rng.uniform(0.2, 1.5, n).astype(np.float32).astype(np.float64)
    out = torch.zeros(n, (h // f) * (w // f) + 1, dtype=torch.float32, device="cuda")
    gd, dd = f32_dev(gap), f32_dev(depth)  # held: a temporary's memory could be reused before the kernel runs
    T.tsg_call("tsg_features", gd.data_ptr(), n, h, w, f, dd.data_ptr(), 2.0, out.data_ptr(), stream())
    box = gap.reshape(n, h // f, f, w // f, f).mean(axis=(2, 4)).reshape(n, -1)
    got = host(out)
    assert np.all(np.abs(got[:, :-1] - box) <= 16 * U_32 * np.abs(gap).max())
    assert np.array_equal(got[:, -1], (2.0 * depth).astype(np.float32).astype(np.float64))
    a = rng.standard_normal((n, 50, 3)).astype(np.float32).astype(np.float64)
    b = rng.standard_normal((n, 50, 3)).astype(np.float32).astype(np.float64)
    mse = torch.zeros(n, dtype=torch.float32, device="cuda")
    ad, bd = f32_dev(a), f32_dev(b)
    for ch in range(3):
        T.tsg_call("tsg_channel_mse", ad.data_ptr(), bd.data_ptr(), n, 50, 3, ch, mse.data_ptr(), stream())
        ref = ((a[..., ch] - b[..., ch]) ** 2).mean(axis=1)
        assert np.all(np.abs(host(mse) - ref) <= 60 * U_32 * ref)


def test_symmetry_copies(T):
    rng = np.random.default_rng(131)
    n, res = 8, 6
    x = rng.standard_normal((n, res, res, 2)).astype(np.float32)
    y = rng.standard_normal((n, res, res, 3)).astype(np.float32)
    ops = np.arange(8, dtype=np.int32)
    xd, yd, od = f32_dev(x), f32_dev(y), torch.tensor(ops).cuda()
    xo, yo = torch.empty_like(xd), torch.empty_like(yd)
    T.tsg_call("tsg_augment", xd.data_ptr(), yd.data_ptr(), n, res, od.data_ptr(), xo.data_ptr(), yo.data_ptr(),
               stream())
    gx, gy = host(xo), host(yo)
    for k in range(n):
        ex, ey = x[k].copy(), y[k].copy()  # [row = y][col = x][ch]
        if ops[k] & 4:
            ex, ey = ex.transpose(1, 0, 2).copy(), ey.transpose(1, 0, 2)[..., [1, 0, 2]].copy()
        if ops[k] & 1:
            ex, ey = ex[:, ::-1].copy(), ey[:, ::-1].copy()
            ey[..., 0] *= -1
        if ops[k] & 2:
            ex, ey = ex[::-1].copy(), ey[::-1].copy()
            ey[..., 1] *= -1
        assert np.array_equal(gx[k], ex) and np.array_equal(gy[k], ey), k


def test_contact_residual(T):
    rng = np.random.default_rng(141)
    npix = 1000
    out = rng.standard_normal((npix, 3)).astype(np.float32)
    x = rng.standard_normal((npix, 2)).astype(np.float32)
    od, xd = f32_dev(out), f32_dev(x)
    T.tsg_call("tsg_contact_residual", od.data_ptr(), xd.data_ptr(), npix, 10.0, stream())
    ref = out.astype(np.float64)
    ref[:, 2] += np.float32(10.0) * np.minimum(x[:, 0], 0).astype(np.float64)
    got = host(od)
    assert np.array_equal(got[:, :2], out[:, :2].astype(np.float64))
    assert np.all(np.abs(got[:, 2] - ref[:, 2]) <= 2.0 ** -23 * (np.abs(ref[:, 2]) + 10 * np.abs(x[:, 0])))
