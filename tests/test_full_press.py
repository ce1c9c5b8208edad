"""The whole benchmark press against the FP64 oracle: every indenter family's
1.6M-particle GelSight press (200 x 200 x 40 lattice, 256 x 256 x 64 grid,
0.1 mm, 8-node blocks: the configuration bench.py times) through all 2000
substeps, compared with the oracle's end state in
tests/golden/full_press_seed{0..4}.npz (written by
tests/golden/make_full_press.py, which runs only the oracle and the seeded
workload generator): the 200 x 200 depth map within 0.1 um and 8,000 sampled
particle positions (half under the indenter near the top face) within 1e-5
of the 20 mm block width.

* FP64: every family, to those bounds.
* FP32: the sphere, flat-punch and cone presses to those bounds. The edge and
  textured-plate presses at this time step (2 us, 0.48 of the undeformed
  gel's CFL limit) are locally unstable where the indenter's sharp features
  compress the gel hardest (compression stiffens the neo-Hookean gel, which
  raises its wave speed past what the step resolves): a 1 nm random change of
  the initial positions, run in FP64, grows to micrometres there (gain
  10^3-10^5 against ~25 for the other three), and the growth collapses when
  the same press runs at a quarter of the step. The FP64 path still follows
  the oracle's arithmetic to 1e-13 m; FP32 rounding (~1 nm per substep) cannot,
  and its deviation on these two presses exceeds the bound (measured: edge
  0.14 um in the map and 1.9 um in positions, plate 6.6 um and 3.2 um). Those
  two FP32 cases are expected failures (strict: a pass would be reported),
  and the instability itself is a test of its own. (Within 2000 substeps no
  other step fixes it: at 0.5 us the 1 ms press turns dynamic and FP32 drifts
  0.1-0.2 um on the plate and punch; a stable 4 ms press needs 8000 substeps.)
"""
import os

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
FAMILIES = [0, 1, 2, 3, 4]
IDS = ["sphere", "cylinder", "cone", "edge", "textured_plate"]
ILL_CONDITIONED = (3, 4)


def run_press(seed, precision):
    """End state (depth map, positions [N][3], force) of the whole press on
    the GPU, in 50-substep frames as the benchmark runs it."""
    from paper_2301_08343_amd.sim import Sim
    wl = W.gelsight_contact(seed=seed, steps=2000)
    sim = Sim(wl["cfg"], wl["poses"][0], precision=precision, tile=8)
    for k in range(0, 2000, 50):
        sim.run(wl["poses"][k + 1:k + 51], wl["dt"])
    H = sim.heightmap().double().cpu().numpy()
    x = sim.read_particles()[0].double().cpu().numpy().T
    f = sim.force()
    sim.close()
    torch.cuda.empty_cache()
    return wl, H, x, f


def errors(ref, H, x):
    return float(np.abs(H - ref["H"]).max()), float(np.abs(x[ref["idx"]] - ref["x"]).max())


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def load(seed):
    return np.load(os.path.join(HERE, "golden", f"full_press_seed{seed}.npz"))


@pytest.mark.parametrize("seed", FAMILIES, ids=IDS)
def test_whole_press_fp64_matches_oracle(gpu, seed):
    ref = load(seed)
    print(f"whole press seed {seed}: FP64, 2000 substeps", flush=True)
    wl, H, x, f = run_press(seed, "f64")
    err_h, err_x = errors(ref, H, x)
    print(f"  FP64: max |dH| = {err_h:.3e} m, max |dx| (sampled) = {err_x:.3e} m, force z {f[2]:.5f} N "
          f"(oracle {ref['force'][2]:.5f} N)")
    assert W.top_z(wl["cfg"]) - ref["H"].min() > 0.2e-3  # the press shows in the map
    assert err_h <= 0.1e-6
    assert err_x <= 1e-5 * 20e-3


FP32_CASES = [pytest.param(s, id=i, marks=pytest.mark.xfail(
    strict=True, reason="the press is unstable at its 2 us step (gain > 1e3 to a 1 nm perturbation, "
                        "test_sharp_presses_are_unstable_at_the_configured_step): only the FP64 path follows the "
                        "oracle there")) if s in ILL_CONDITIONED else pytest.param(s, id=i)
              for s, i in zip(FAMILIES, IDS)]


@pytest.mark.parametrize("seed", FP32_CASES)
def test_whole_press_fp32_matches_oracle(gpu, seed):
    ref = load(seed)
    print(f"whole press seed {seed}: FP32, 2000 substeps", flush=True)
    wl, H, x, f = run_press(seed, "f32")
    err_h, err_x = errors(ref, H, x)
    print(f"  FP32: max |dH| = {err_h:.3e} m, max |dx| (sampled) = {err_x:.3e} m, force z {f[2]:.4f} N "
          f"(oracle {ref['force'][2]:.4f} N)")
    assert err_h <= 0.1e-6
    assert err_x <= 1e-5 * 20e-3


def perturbation_gain(seed, split):
    """Largest particle displacement at the end of the whole press, run in
    FP64 at dt = 2 us / split over 2000 split substeps (the same 4 ms press),
    between a start perturbed by 1 nm (uniform per coordinate) and the exact
    start, over 1 nm."""
    from paper_2301_08343_amd.sim import Sim
    wl = W.gelsight_contact(seed=seed, steps=2000 * split)
    dt, n = 2e-6 / split, 2000 * split
    ends = []
    for perturb in (0.0, 1e-9):
        sim = Sim(wl["cfg"], wl["poses"][0], precision="f64", tile=8)
        if perturb > 0:
            x, v, C, F = sim.read_particles()
            g = torch.Generator(device=x.device).manual_seed(1000 + seed)
            x = x + perturb * (2 * torch.rand(x.shape, generator=g, device=x.device, dtype=x.dtype) - 1)
            sim.write_particles(x, v, C, F)
        for k in range(0, n, 50):
            sim.run(wl["poses"][k + 1:k + 51], dt)
        ends.append(sim.read_particles()[0].double().cpu().numpy())
        sim.close()
        torch.cuda.empty_cache()
    return float(np.abs(ends[1] - ends[0]).max()) / 1e-9


def test_sharp_presses_are_unstable_at_the_configured_step(gpu):
    """The edge and plate presses amplify a 1 nm perturbation more than 1000
    times at the configured 2 us step while the sphere press stays below 100;
    at a quarter of the step the plate's gain falls by more than 10x (the
    growth is the step's, not the elastomer's)."""
    g_sphere = perturbation_gain(0, 1)
    g_edge = perturbation_gain(3, 1)
    g_plate = perturbation_gain(4, 1)
    g_plate_q = perturbation_gain(4, 4)
    print(f"gain of a 1 nm perturbation over the press: sphere {g_sphere:.0f}, edge {g_edge:.0f}, plate {g_plate:.0f}; "
          f"plate at dt/4 {g_plate_q:.0f}", flush=True)
    assert g_sphere < 100
    assert g_edge > 1e3 and g_plate > 1e3
    assert g_plate_q < 0.1 * g_plate
