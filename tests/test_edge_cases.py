"""Degenerate and boundary cases through the C ABI on the GPU: runs of zero
substeps, a press whose indenter never reaches the gel, the smallest block
the library accepts inside a batch, and the marker count's limits."""
import math

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd.batch import Batch
    from paper_2301_08343_amd.sim import Sim
    return Batch, Sim


def state(sim):
    return [t.clone() for t in sim.read_particles()]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_empty_runs_leave_the_state_alone(gpu, precision):
    """tacchi_run over zero poses changes nothing, bit for bit, and keeps the
    indenter where the last substep left it."""
    _, Sim = gpu
    wl = W.small_sphere_contact(seed=1, steps=60)
    poses, dt = wl["poses"], wl["dt"]
    sim = Sim(wl["cfg"], poses[0], precision=precision)
    sim.run(poses[1:51], dt)
    before, H = state(sim), sim.heightmap().clone()
    sim.run(poses[51:51], dt)
    for a, b in zip(before, state(sim)):
        assert torch.equal(a, b)
    assert torch.equal(H, sim.heightmap())
    np.testing.assert_array_equal(sim.pose(), poses[50])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_press_without_contact_stays_at_rest(gpu, precision):
    """The sphere's path lifted 10 mm: no grid node is ever inside it, the
    reaction is exactly zero, and the gel at rest (v = 0, F = I, no gravity)
    stays at rest bit for bit over 200 substeps: the undeformed gel has
    exactly zero stress and every transfer of zero momentum is zero."""
    _, Sim = gpu
    wl = W.small_sphere_contact(seed=1, steps=200)
    poses = np.array(wl["poses"], dtype=np.float64)
    poses[:, 2] += 10e-3
    sim = Sim(wl["cfg"], poses[0], precision=precision)
    x0, H0 = sim.read_particles()[0].clone(), sim.heightmap().clone()
    sim.run(poses[1:], wl["dt"])
    assert np.all(sim.force() == 0.0)
    assert torch.equal(sim.read_particles()[0], x0)
    assert torch.equal(sim.heightmap(), H0)


def minimal_contact(steps):
    """A 2 x 2 x 2 lattice at 0.25 mm (one particle per cell, the bottom layer
    bonded), the smallest block whose top layer has markers, pressed by a
    1 mm sphere."""
    h = 0.25e-3
    n = (2, 2, 2)
    pad = 5
    cfg = W._contact(block_origin=(pad * h, pad * h, 3 * h), block_size=(n[0] * h, n[1] * h, n[2] * h), n=n,
                     grid_origin=(0, 0, 0), dx=h, gn=(n[0] + 2 * pad, n[1] + 2 * pad, n[2] + 12),
                     E=0.15e6, nu=0.45, rho=1000.0, model=W.NEOHOOKEAN, shape=W.SPHERE, sp=[1e-3], seed=5)
    cx, cy = W.block_center_xy(cfg)
    poses = W.press_trajectory((cx, cy, W.top_z(cfg)), W.IDENTITY_QUAT, 0.1e-3, steps)
    lam = cfg["E"] * cfg["nu"] / ((1 + cfg["nu"]) * (1 - 2 * cfg["nu"]))
    mu = cfg["E"] / (2 * (1 + cfg["nu"]))
    dt = 0.45 * h / math.sqrt((lam + 2 * mu) / cfg["rho"])
    return dict(cfg=cfg, poses=poses, dt=dt)


def test_smallest_block_in_a_batch(gpu):
    """Eight particles in a batch of one contact and in a batch with a
    200,000-particle contact: each matches its solo run (the bound of the
    batch tests), and the press moves the top layer."""
    Batch, Sim = gpu
    S = 120
    tiny = minimal_contact(S)
    big = W.batch_contact(3, steps=S)
    for contacts in ([tiny], [tiny, big]):
        batch = Batch(contacts, S)
        batch.run(S)
        batch.sync()
        tuning = batch.tuning()
        for i, c in enumerate(contacts):
            solo = Sim(c["cfg"], c["poses"][0], precision="f32", tile=tuning[i][0])
            solo.run(c["poses"][1:S + 1], c["dt"])
            xs = solo.read_particles()[0].double().cpu().numpy()
            xb = batch.contact(i).read_particles()[0].double().cpu().numpy()
            assert np.abs(xs - xb).max() <= 2e-9
        x0 = Sim(tiny["cfg"], tiny["poses"][0], precision="f32").read_particles()[0].double().cpu().numpy()
        xt = batch.contact(0).read_particles()[0].double().cpu().numpy()
        assert np.abs(xt - x0).max() > 1e-7


def test_marker_count_limits(gpu):
    """At least one marker (zero is an argument error); a marker on the rim of
    the top face is accepted and one just outside it is not."""
    from paper_2301_08343_amd.native import E_ARG, TacchiError
    _, Sim = gpu
    wl = W.small_sphere_contact(seed=1, steps=10)
    cfg = wl["cfg"]
    sim = Sim(cfg, wl["poses"][0], precision="f64")
    with pytest.raises(TacchiError) as e:
        sim.markers(np.zeros((0, 2)))
    assert e.value.status == E_ARG
    x0, y0 = cfg["block_origin"][:2]
    out = sim.markers([[x0, y0]])
    assert out.shape == (1, 3) and torch.all(out == 0)
    with pytest.raises(TacchiError) as e:
        sim.markers([[x0 - 1e-6, y0]])
    assert e.value.status == E_ARG
