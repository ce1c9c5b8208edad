"""The sampled one-substep check used at full size, validated against a whole
oracle run: on a down-scaled GelSight press that the oracle steps whole, the
small per-sample oracle runs reproduce the whole run's next substep for every
sampled particle (both FP64, so to rounding)."""
import numpy as np

from paper_2301_08343_amd import workloads as W

from _local_oracle import local_oracle_step, samples


def test_local_runs_reproduce_the_whole_substep(oracle_lib):
    wl = W.gelsight_contact(seed=0, steps=2000, scale=8)
    cfg, poses, dt = wl["cfg"], wl["poses"], wl["dt"]
    k = 300
    sim = oracle_lib.OracleSim(cfg, poses[0])
    sim.run(poses, dt, 0, k)
    x, v, C, F = sim.particles()
    assert sim.step(poses[k + 1], dt) == 0
    assert abs(sim.force()[2]) > 0
    x1, v1, C1, F1 = sim.particles()
    picks = samples(cfg, x, poses[k])
    assert len(picks) >= 40
    for p in picks:
        xo, vo, Co, Fo = local_oracle_step(oracle_lib, cfg, x, v, C, F, p, poses[k], poses[k + 1], dt)
        np.testing.assert_allclose(xo, x1[p], rtol=0, atol=1e-15)
        np.testing.assert_allclose(vo, v1[p], rtol=0, atol=1e-12)
        np.testing.assert_allclose(Fo, F1[p], rtol=0, atol=1e-13)
        np.testing.assert_allclose(Co, C1[p], rtol=0, atol=1e-9 * max(np.abs(C1[p]).max(), 1.0))
