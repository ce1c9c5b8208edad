"""tacchi_indenter_gap_noalloc (the gap field for callers that cannot
allocate device memory) against tacchi_indenter_gap with a caller workspace,
through the C ABI: two calls in a row, the second smaller, each bit for bit
equal to the workspace entry point (same kernel, same descriptors); device
free memory does not move across the no-alloc calls; more queries than its
fixed array holds are refused."""
import ctypes

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _args(contacts):
    from paper_2301_08343_amd import native as N
    n = len(contacts)
    carr = (N.Config * n)()
    parr = (N.Pose * n)()
    for k, c in enumerate(contacts):
        carr[k] = N.make_config(c["cfg"], c["poses"][-1], N.F32, 0)
        parr[k] = N.make_pose(c["poses"][-1])
    return carr, parr


def test_gap_noalloc_matches_workspace_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd import native as N
    L = N.lib()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    assert L.tacchi_indenter_gap_noalloc_max() == 2048
    calls = [
        # 24 upright GelSight contacts of every family, 64 x 64 cells of 2 x 2 points
        ([W.gelsight_contact(s, steps=10) for s in range(24)], 64, 2, -2e-3, 0.0),
        # then 5 tilted uneven-batch contacts, 16 x 16 cell centres, two-sided clamp
        ([W.batch_contact(s, steps=10) for s in range(100, 105)], 16, 1, -1.5e-3, 1.5e-3),
    ]
    outs = [(torch.full((len(cs), res, res), float("nan"), dtype=torch.float32, device="cuda"),
             torch.full((len(cs), res, res), float("nan"), dtype=torch.float32, device="cuda"))
            for cs, res, _, _, _ in calls]
    ws_bytes = int(L.tacchi_indenter_gap_workspace_bytes(24))
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
    ws_ptr = ctypes.c_void_p(ws.data_ptr() + ((-ws.data_ptr()) % 256))
    # the first no-alloc call on this GPU looks up the array's address
    cs0, res0, sub0, lo0, hi0 = calls[0]
    c0, p0 = _args(cs0[:1])
    warm = torch.empty(1, res0, res0, dtype=torch.float32, device="cuda")
    N.check(L.tacchi_indenter_gap_noalloc(c0, p0, 1, res0, sub0, lo0, hi0, ctypes.c_void_p(warm.data_ptr()), sp))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for (cs, res, sub, lo, hi), (got, ref) in zip(calls, outs):
        carr, parr = _args(cs)
        print(f"no-alloc gap: {len(cs)} contacts, {res} x {res} cells, {sub} x {sub} points", flush=True)
        N.check(L.tacchi_indenter_gap_noalloc(carr, parr, len(cs), res, sub, lo, hi, ctypes.c_void_p(got.data_ptr()),
                                              sp))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    for (cs, res, sub, lo, hi), (got, ref) in zip(calls, outs):
        carr, parr = _args(cs)
        N.check(L.tacchi_indenter_gap(carr, parr, len(cs), res, sub, lo, hi, ctypes.c_void_p(ref.data_ptr()),
                                      ws_ptr, ws_bytes, sp))
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
        assert float(got.min()) < hi  # the indenters are seen over the faces
    # the second, smaller call left the first call's cells of later contacts alone
    assert outs[0][0].shape[0] == 24 and outs[1][0].shape[0] == 5
    big = [W.gelsight_contact(0, steps=10)] * (L.tacchi_indenter_gap_noalloc_max() + 1)
    carr, parr = _args(big)
    tmp = torch.empty(len(big), 4, 4, dtype=torch.float32, device="cuda")
    with pytest.raises(N.TacchiError) as e:
        N.check(L.tacchi_indenter_gap_noalloc(carr, parr, len(big), 4, 1, -2e-3, 0.0, ctypes.c_void_p(tmp.data_ptr()),
                                              sp))
    assert e.value.status == N.E_ARG
