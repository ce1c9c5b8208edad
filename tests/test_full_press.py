"""The whole benchmark press against the FP64 oracle: every indenter family's
1.6M-particle GelSight press (200 x 200 x 40 lattice, 256 x 256 x 64 grid,
0.1 mm, FP32, 8-node blocks: the configuration bench.py times) through all
2000 substeps, compared with the oracle's end state in
tests/golden/full_press_seed{0..4}.npz (written by
tests/golden/make_full_press.py, which runs only the oracle and the seeded
workload generator): the 200 x 200 depth map within 0.1 um and 8,000 sampled
particle positions (half under the indenter near the top face) within 1e-5
of the 20 mm block width."""
import os

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4], ids=["sphere", "cylinder", "cone", "edge", "textured_plate"])
def test_whole_press_matches_oracle(seed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd.sim import Sim
    ref = np.load(os.path.join(HERE, "golden", f"full_press_seed{seed}.npz"))
    steps = int(ref["steps"])
    wl = W.gelsight_contact(seed=seed, steps=steps)
    print(f"whole press {wl['name']}: {steps} substeps, FP32", flush=True)
    sim = Sim(wl["cfg"], wl["poses"][0], precision="f32", tile=8)
    for k in range(0, steps, 50):  # 50-substep frames, as the benchmark runs them
        sim.run(wl["poses"][k + 1:k + 51], wl["dt"])
    H = sim.heightmap().double().cpu().numpy()
    x = sim.read_particles()[0].double().cpu().numpy().T
    err_h = np.abs(H - ref["H"]).max()
    err_x = np.abs(x[ref["idx"]] - ref["x"]).max()
    f = sim.force()
    print(f"  max |dH| = {err_h:.3e} m, max |dx| (sampled) = {err_x:.3e} m, indent "
          f"{W.top_z(wl['cfg']) - ref['H'].min():.3e} m, force z {f[2]:.4f} N (oracle {ref['force'][2]:.4f} N)")
    assert W.top_z(wl["cfg"]) - ref["H"].min() > 0.2e-3  # the press shows in the map
    assert err_h <= 0.1e-6
    assert err_x <= 1e-5 * 20e-3
