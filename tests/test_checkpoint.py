"""Checkpoint/resume on the CPU: the particles (x, v, C, F) and the indenter
pose are the whole state of a press. The FP64 oracle saved to an .npz file
after 40 substeps of the sphere press and loaded into a new simulator
continues bit for bit as the uninterrupted run; a state that leaves out the
affine velocity C (or the deformation gradient F) does not, so the check
sees a missing field. (The GPU simulator's .npz checkpoints are compared with
its uninterrupted runs in tests/test_gpu_parity.py.)"""
import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W


def run_and_save(oracle_lib, path, n_save=40, n_more=30):
    wl = W.small_sphere_contact(seed=2, steps=n_save + n_more)
    cfg, poses, dt = wl["cfg"], wl["poses"], wl["dt"]
    a = oracle_lib.OracleSim(cfg, poses[0])
    a.run(poses, dt, 0, n_save)
    x, v, C, F = a.particles()
    np.savez(path, x=x, v=v, C=C, F=F, pose=a.pose())
    a.run(poses, dt, n_save, n_save + n_more)
    return wl, a.particles(), a.heightmap()


def resume(oracle_lib, wl, path, n_save=40, n_more=30, drop=None):
    with np.load(path, allow_pickle=False) as d:
        state = {k: d[k] for k in ("x", "v", "C", "F", "pose")}
    if drop == "C":
        state["C"] = np.zeros_like(state["C"])
    if drop == "F":
        state["F"] = np.broadcast_to(np.eye(3), state["F"].shape).copy()
    b = oracle_lib.OracleSim(wl["cfg"], state["pose"])
    b.set_particles(state["x"], state["v"], state["C"], state["F"])
    b.run(wl["poses"], wl["dt"], n_save, n_save + n_more)
    return b.particles(), b.heightmap()


def test_resumed_press_is_bitwise_the_uninterrupted_one(oracle_lib, tmp_path):
    path = tmp_path / "press.npz"
    wl, ref, H = run_and_save(oracle_lib, path)
    got, Hb = resume(oracle_lib, wl, path)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    assert np.array_equal(H, Hb)
    # the 30 substeps after the checkpoint move the particles
    with np.load(path, allow_pickle=False) as d:
        assert np.abs(ref[0] - d["x"]).max() > 1e-7


@pytest.mark.parametrize("drop", ["C", "F"])
def test_a_state_without_C_or_F_does_not_resume(oracle_lib, tmp_path, drop):
    path = tmp_path / "press.npz"
    wl, ref, _ = run_and_save(oracle_lib, path)
    got, _ = resume(oracle_lib, wl, path, drop=drop)
    assert np.abs(ref[0] - got[0]).max() > 1e-12
