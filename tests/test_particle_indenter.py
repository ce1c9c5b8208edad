"""The indenter as particles (Eq. 10, point clouds of Sec. IV-B) on the GPU
against the oracle: a sphere's point cloud pressed into the 18,432-particle
block in FP64 (tight) and FP32 (the press's position bound), a cleared cloud
returning to the shape's contact, and the argument checks."""
import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

S = 300


@pytest.fixture(scope="module")
def press(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = W.small_sphere_contact(seed=0, steps=1000, jitter=False)
    cfg = wl["cfg"]
    mass = 10 * cfg["rho"] * (cfg["block_size"][0] / cfg["n"][0]) ** 3
    pts = W.sphere_points(3e-3, 20000, 1e-3, 0)
    orc = oracle_lib.OracleSim(cfg, wl["poses"][0])
    orc.set_indenter_points(pts, mass)
    orc.run(wl["poses"], wl["dt"], 0, S)
    return wl, pts, mass, orc.particles()[0], orc.force()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_point_cloud_press_matches_oracle(press, precision):
    from paper_2301_08343_amd.sim import Sim
    wl, pts, mass, x_ref, f_ref = press
    sim = Sim(wl["cfg"], wl["poses"][0], precision=precision)
    sim.set_indenter_points(pts, mass)
    sim.run(wl["poses"][1:S + 1], wl["dt"])
    x, _, _, _ = sim.read_particles()
    err = np.abs(x.cpu().double().numpy().T - x_ref).max()
    f = sim.force()
    print(f"{precision}: max |dx| = {err:.3e} m, force {f} vs {f_ref}")
    assert f_ref[2] > 0
    if precision == "f64":
        assert err <= 1e-12
        np.testing.assert_allclose(f, f_ref, rtol=1e-6, atol=1e-9)
    else:
        assert err <= 1e-5 * wl["cfg"]["block_size"][0]


def test_cleared_cloud_is_the_shape_contact(press):
    from paper_2301_08343_amd.sim import Sim
    # FP32: its fixed-point P2G makes runs bit-reproducible (FP64 LDS atomics
    # round in arrival order)
    wl, pts, mass, _, _ = press
    a = Sim(wl["cfg"], wl["poses"][0], precision="f32")
    a.set_indenter_points(pts, mass)
    a.set_indenter_points(np.zeros((0, 3)), 0.0)
    b = Sim(wl["cfg"], wl["poses"][0], precision="f32")
    a.run(wl["poses"][1:101], wl["dt"])
    b.run(wl["poses"][1:101], wl["dt"])
    assert torch.equal(a.read_particles()[0], b.read_particles()[0])


def test_point_cloud_arguments(press):
    from paper_2301_08343_amd import native as N
    from paper_2301_08343_amd.sim import Sim
    wl, pts, _, _, _ = press
    sim = Sim(wl["cfg"], wl["poses"][0], precision="f32")
    with pytest.raises(N.TacchiError):
        sim.set_indenter_points(pts, -1.0)
    bad = pts.copy()
    bad[3, 1] = np.nan
    with pytest.raises(N.TacchiError):
        sim.set_indenter_points(bad, 1e-6)
