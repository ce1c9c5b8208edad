"""What the trained surrogate gains over the method without it, on held-out
contacts (seeds the network was not trained on) solved by the batched MPM at
the data spacing: the committed network's height error is a small fraction
of the error of the same prediction without the network (the FP32 contact
term alone: the face follows the indenter where they touch) and of zero
displacement, and the network answers the batch in a small fraction of the
MPM's time."""
import os
import time

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2301_08343_amd", "weights",
                       "surrogate_h0.2mm.safetensors")


def test_trained_network_gains_over_contact_term_and_mpm_time():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights")
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import surrogate_pipeline as SP
    from paper_2301_08343_amd import training as TR
    net, meta = SP.load_compact(WEIGHTS, batch=64)
    assert meta["contact_residual"] == D.X_UNIT / D.Y_UNIT
    seeds = range(SP.HELDOUT_SEED0, SP.HELDOUT_SEED0 + 64)
    cs = D.contacts_for(seeds, meta["h_m"])
    x = D.inputs(cs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    y = D.solve(cs)
    torch.cuda.synchronize()
    t_mpm = time.perf_counter() - t0
    TR.predict(net, x)  # first call sets up the network's buffers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = TR.predict(net, x)
    torch.cuda.synchronize()
    t_net = time.perf_counter() - t0
    contact = torch.zeros_like(y)
    contact[..., 2] = meta["contact_residual"] * x[..., 0]
    um = D.Y_UNIT * 1e6

    def height_rmse(a):
        e = TR.per_sample_rmse(a, y, 2) * um
        return float((e ** 2).mean().sqrt())

    e_net, e_contact, e_zero = height_rmse(p), height_rmse(contact), height_rmse(torch.zeros_like(y))
    print(f"held-out height RMSE: network {e_net:.2f} um, contact term alone {e_contact:.2f} um, "
          f"zero {e_zero:.2f} um; 64 frames: MPM {t_mpm:.2f} s, network {t_net * 1e3:.2f} ms")
    assert e_net < 0.5 * e_contact
    assert e_net < 0.1 * e_zero
    assert t_net * 100 < t_mpm
