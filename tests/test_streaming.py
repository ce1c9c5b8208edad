"""The scripted press with a terminal condition on the contact force
(Sec. III-C) on the GPU against the oracle: the run stops after the same
substep, in the same state, and stepping on afterwards matches the oracle
(the bin-list double buffer and the pose are left consistent)."""
import math

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_SUB = 240


@pytest.fixture(scope="module")
def press(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = W.small_sphere_contact(seed=3, steps=1000)
    cfg, poses, dt = wl["cfg"], wl["poses"], wl["dt"]
    orc = oracle_lib.OracleSim(cfg, poses[0])
    f = []
    for k in range(N_SUB):
        assert orc.step(poses[k + 1], dt) == 0
        f.append(orc.force()[2])
    f = np.array(f)
    # a limit crossed at a substep whose force jumps clear of it (the GPU's
    # force agrees with the oracle's to ~1e-9 relative in FP64)
    i = next(i for i in range(150, N_SUB) if f[i] > f[:i].max() * (1 + 1e-4))
    limit = 0.5 * (f[:i].max() + f[i])
    stop = oracle_lib.OracleSim(cfg, poses[0])
    assert stop.run_until_force(poses, dt, limit, 0, N_SUB) == i + 1
    x_stop = stop.particles()[0]
    stop.run(poses, dt, i + 1, i + 1 + 40)
    return dict(wl=wl, limit=limit, steps=i + 1, x_stop=x_stop, x_after=stop.particles()[0])


def test_force_terminated_run_matches_oracle(press):
    from paper_2301_08343_amd.sim import Sim
    wl, limit = press["wl"], press["limit"]
    poses, dt = wl["poses"], wl["dt"]
    sim = Sim(wl["cfg"], poses[0], precision="f64")
    done = sim.run_until_force(poses[1:N_SUB + 1], dt, limit)
    assert done == press["steps"]
    x, _, _, _ = sim.read_particles()
    err = np.abs(x.cpu().numpy().T - press["x_stop"]).max()
    print(f"stopped after {done} substeps at {limit:.4e} N: max |dx| = {err:.3e} m")
    assert err <= 1e-12
    assert sim.force()[2] >= limit
    # stepping on from the stop: the next 40 substeps as the oracle's
    sim.run(poses[done + 1:done + 41], dt)
    x, _, _, _ = sim.read_particles()
    err = np.abs(x.cpu().numpy().T - press["x_after"]).max()
    print(f"40 substeps later: max |dx| = {err:.3e} m")
    assert err <= 1e-12


def test_force_terminated_run_limits(press):
    from paper_2301_08343_amd.sim import Sim
    wl = press["wl"]
    poses, dt = wl["poses"], wl["dt"]
    sim = Sim(wl["cfg"], poses[0], precision="f32")
    assert sim.run_until_force(poses[1:31], dt, math.inf) == 30
    assert sim.run_until_force(poses[31:61], dt, -math.inf) == 1
    # after an early stop the handle keeps stepping normally
    sim.run(poses[32:40], dt)
    sim.sync()
