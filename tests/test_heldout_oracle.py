"""The surrogate's held-out data against the FP64 oracle.

tests/golden/heldout_oracle_h0.2mm.npz holds the oracle's solves of the
held-out contacts 50000-50009 (two per indenter family) at the data spacing
(0.2 mm lattice, 1000 substeps), resampled to the 64 x 64 target grid; it is
written by tests/golden/make_heldout_oracle.py, which calls only the oracle
and the seeded workload generator. Here the batched FP32 MPM that produces
the training and held-out data solves the same contacts: its targets must
match the oracle's to the trajectory bounds (1e-5 of the 20 mm block for
every displacement component, 0.1 um for the height), and the committed
surrogate's height error is reported per family against the oracle-verified
solves.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "heldout_oracle_h0.2mm.npz")
WEIGHTS = os.path.join(HERE, "..", "paper_2301_08343_amd", "weights", "surrogate_h0.2mm.safetensors")


@pytest.fixture(scope="module")
def solved():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd import dataset as D
    ref = np.load(FIXTURE)
    seeds = [int(s) for s in ref["seeds"]]
    assert float(ref["h"]) == D.H_DATA and int(ref["res"]) == D.RES and int(ref["sub"]) == D.SUB
    cs = D.contacts_for(seeds, D.H_DATA)
    print(f"held-out seeds {seeds[0]}-{seeds[-1]}: batched MPM at {D.H_DATA * 1e3:.1f} mm", flush=True)
    x = D.inputs(cs)
    y = D.solve(cs)
    return ref, seeds, x, y


def test_heldout_targets_match_oracle(solved):
    from paper_2301_08343_amd import dataset as D
    ref, seeds, _, y = solved
    u_gpu = y.double().cpu().numpy() * D.Y_UNIT
    u_orc = ref["u"]
    assert u_gpu.shape == u_orc.shape == (len(seeds), D.RES, D.RES, 3)
    err = np.abs(u_gpu - u_orc)
    for k, s in enumerate(seeds):
        print(f"seed {s} family {s % 5}: max |du| = {err[k].max():.3e} m, max |du_z| = {err[k, ..., 2].max():.3e} m, "
              f"deepest u_z {u_orc[k, ..., 2].min():.3e} m", flush=True)
    assert err.max() <= 1e-5 * 20e-3
    assert err[..., 2].max() <= 0.1e-6
    assert (u_orc[..., 2].min(axis=(1, 2)) < -0.1e-3).all()  # every press indents the face


def test_surrogate_error_against_oracle_verified_solves(solved):
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights")
    from paper_2301_08343_amd import dataset as D
    from paper_2301_08343_amd import surrogate_pipeline as SP
    from paper_2301_08343_amd import training as TR
    ref, seeds, x, y = solved
    net, meta = SP.load_compact(WEIGHTS, batch=64)
    p = TR.predict(net, x)
    y_orc = torch.tensor(ref["u"] / D.Y_UNIT, dtype=torch.float32, device=p.device)
    um = D.Y_UNIT * 1e6
    e_orc = (TR.per_sample_rmse(p, y_orc, 2) * um).cpu().numpy()
    e_gpu = (TR.per_sample_rmse(p, y, 2) * um).cpu().numpy()
    fam = np.array([s % 5 for s in seeds])
    for f in range(5):
        sel = fam == f
        print(f"family {f}: surrogate height RMSE vs oracle solves {np.sqrt((e_orc[sel] ** 2).mean()):.2f} um, "
              f"vs the MPM data {np.sqrt((e_gpu[sel] ** 2).mean()):.2f} um", flush=True)
    # the oracle-verified targets differ from the data by < 0.1 um, so the
    # surrogate's error is the same against either
    assert np.abs(e_orc - e_gpu).max() <= 0.1
