"""The seeded input generators: the random stream against its published test
vectors, and the workloads against the recipe they state (sizes, ranges,
trajectories), deterministic per seed."""
import math

import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W


def test_splitmix64_matches_its_published_outputs():
    """SplitMix64 (Steele, Lea and Flood 2014; Vigna's reference code) from
    state 0: the first outputs of the reference generator."""
    rng = W.SplitMix64(0)
    assert [rng.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_draws_stay_in_range_and_are_uniform():
    rng = W.SplitMix64(12345)
    u = np.array([rng.uniform(-2.0, 3.0) for _ in range(20000)])
    assert u.min() >= -2.0 and u.max() < 3.0
    assert abs(u.mean() - 0.5) < 0.05 and abs(u.var() - 25.0 / 12.0) < 0.08


@pytest.mark.parametrize("seed", range(10))
def test_gelsight_press_recipe(seed):
    wl = W.gelsight_contact(seed=seed, steps=2000)
    cfg = wl["cfg"]
    assert cfg["n"] == (200, 200, 40) and cfg["gn"] == (256, 256, 64)
    assert cfg["dx"] == pytest.approx(1e-4) and cfg["block_size"] == pytest.approx((20e-3, 20e-3, 4e-3))
    assert cfg["shape"] == seed % 5 and cfg["model"] == W.NEOHOOKEAN
    assert (cfg["E"], cfg["nu"], cfg["rho"]) == (0.15e6, 0.45, 1000.0)
    assert wl["dt"] == 2e-6 and 0.2e-3 <= wl["depth"] <= 1.5e-3
    poses = wl["poses"]
    assert poses.shape == (2001, 7)
    cx, cy = W.block_center_xy(cfg)
    assert abs(poses[0, 0] - cx) <= 3e-3 and abs(poses[0, 1] - cy) <= 3e-3
    assert poses[0, 2] == pytest.approx(W.top_z(cfg))
    assert poses[-1, 2] == pytest.approx(W.top_z(cfg) - wl["depth"])
    assert np.all(np.diff(poses[:, 2]) < 0) and np.all(poses[:, :2] == poses[0, :2])
    assert wl["render"]["h"] == 480 and wl["render"]["w"] == 640
    assert wl["render"]["pitch"] == pytest.approx(20e-3 / 640)
    # the block sits on whole grid nodes, inside the grid with room for the walls
    o = np.array(cfg["block_origin"]) / cfg["dx"]
    assert np.allclose(o, np.round(o)) and (np.round(o) >= 3).all()
    assert (np.round(o[:2]) + 200 <= 256 - 3).all()


def test_indenter_draws_follow_their_ranges():
    rng = W.SplitMix64(7)
    for _ in range(200):
        assert 2e-3 <= W.draw_indenter(rng, W.SPHERE)[0] <= 5e-3
        assert 1e-3 <= W.draw_indenter(rng, W.CYLINDER)[0] <= 4e-3
        th, rt = W.draw_indenter(rng, W.CONE)
        assert math.radians(30) <= th <= math.radians(60) and rt == 0.2e-3
        hw, amp, lam = W.draw_indenter(rng, W.TEXTURED_PLATE)
        assert 3e-3 <= hw <= 6e-3 and (amp, lam) == (50e-6, 1e-3)
    assert W.draw_indenter(rng, W.EDGE) == [math.pi / 4, 0.2e-3]


def test_batch_contacts_follow_their_recipe():
    counts = []
    for seed in range(64):
        wl = W.batch_contact(seed, steps=100)
        cfg = wl["cfg"]
        h = cfg["dx"]
        assert 0.1e-3 <= h <= 0.3e-3
        assert cfg["model"] == W.COROTATED and 0.1e6 <= cfg["E"] <= 0.3e6 and 0.40 <= cfg["nu"] <= 0.48
        nxy, _, nz = cfg["n"]
        assert wl["particles"] == nxy * nxy * nz
        counts.append(wl["particles"])
        # CFL: dt = 0.45 dx / c_p with c_p the P-wave speed
        lam = cfg["E"] * cfg["nu"] / ((1 + cfg["nu"]) * (1 - 2 * cfg["nu"]))
        mu = cfg["E"] / (2 * (1 + cfg["nu"]))
        assert wl["dt"] == pytest.approx(0.45 * h / math.sqrt((lam + 2 * mu) / cfg["rho"]))
        # tilt of at most 5 degrees about a horizontal axis
        q = wl["poses"][0, 3:]
        assert abs(np.linalg.norm(q) - 1) < 1e-12 and q[3] == pytest.approx(0.0, abs=1e-15)
        assert 2 * math.acos(min(1.0, abs(q[0]))) <= math.radians(5) + 1e-12
        assert 0.2e-3 <= wl["depth"] <= min(1.5e-3, 0.35 * nz * h) + 1e-15
    counts = np.array(counts)
    # log-uniform target in [2e4, 4e5], up to the rounding of the lattice
    assert counts.min() >= 1.2e4 and counts.max() <= 5e5
    assert np.log(counts).std() > 0.5


def test_generators_are_deterministic_per_seed():
    a, b = W.gelsight_contact(3), W.gelsight_contact(3)
    assert a["cfg"] == b["cfg"] and np.array_equal(a["poses"], b["poses"])
    assert not np.array_equal(W.gelsight_contact(4)["poses"], a["poses"])
    c, d = W.batch_contact(11, steps=10), W.batch_contact(11, steps=10)
    assert c["cfg"] == d["cfg"] and np.array_equal(c["poses"], d["poses"])
    small = W.small_sphere_contact(seed=2)["cfg"]
    x1 = W.random_particle_state(5, small)
    x2 = W.random_particle_state(5, small)
    assert all(np.array_equal(p, q) for p, q in zip(x1, x2))
