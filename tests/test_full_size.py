"""Parity at the benchmark's full size: the 1.6M-particle GelSight press
(200 x 200 x 40 lattice, 256 x 256 x 64 grid, FP32, 8-node blocks), in the
launch configuration the benchmark times, for each of the five indenter
families.

The whole press is beyond the oracle, so the checks are
* sampled outputs the oracle computes one by one: one substep of sampled
  particles (under the indenter, near the top face, in the bulk), each from
  a small oracle run holding every particle whose stencil can reach the
  sample's nodes, taken from the GPU's own state before the substep;
* properties that hold at any size: the mass and momentum that P2G puts on
  the grid (the transfer weights sum to one and their first moment about the
  particle vanishes, so the affine and stress terms carry no net momentum),
  the depth map against the particles' own top layer, and the tactile image
  against the oracle's renderer on the GPU's depth map.
"""
import numpy as np
import pytest

from paper_2301_08343_amd import workloads as W

from _local_oracle import local_oracle_step, samples, soa_to_aos

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SUBSTEPS_BEFORE = 1200  # of 2000: the indenter is well into the gel


def to_np(t):
    return t.detach().cpu().double().numpy()


@pytest.fixture(scope="module", params=[0, 1, 2, 3, 4],
                ids=["sphere", "cylinder", "cone", "edge", "textured_plate"])
def press(request):
    """The press of one indenter family (seed = family), run on the GPU to
    SUBSTEPS_BEFORE substeps."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_08343_amd.sim import Sim
    wl = W.gelsight_contact(seed=request.param, steps=2000)
    print(f"full-size press: {wl['name']}, {SUBSTEPS_BEFORE} substeps", flush=True)
    sim = Sim(wl["cfg"], wl["poses"][0], precision="f32", tile=8)
    sim.run(wl["poses"][1:SUBSTEPS_BEFORE + 1], wl["dt"])
    sim.sync()
    return wl, sim


def test_sampled_particles_match_oracle_after_one_substep(oracle_lib, press):
    wl, sim = press
    cfg, poses, dt = wl["cfg"], wl["poses"], wl["dt"]
    k = SUBSTEPS_BEFORE
    x, v, C, F = soa_to_aos(*(to_np(t) for t in sim.read_particles()))
    sim.step(poses[k + 1], dt)
    x1, v1, C1, F1 = soa_to_aos(*(to_np(t) for t in sim.read_particles()))
    assert np.abs(sim.force()[2]) > 0, "the indenter should be in contact"
    picks = samples(cfg, x, poses[k])
    assert len(picks) >= 40
    ref = [local_oracle_step(oracle_lib, cfg, x, v, C, F, p, poses[k], poses[k + 1], dt) for p in picks]
    # FP32 kernels against the FP64 oracle from the same FP32-valued state,
    # to the bounds of the injected-state FP32 phase test (scales: the
    # sample's largest |v| and |C|). The largest term is the FP32 stress:
    # its ~1e-6 relative rounding, times the stress impulse that dominates
    # A = m C - dt V0 (4/dx^2) tau near the indenter, moves C by ~0.1 % of
    # the largest gradient.
    v_max = max(np.abs(r[1]).max() for r in ref)
    c_max = max(np.abs(r[2]).max() for r in ref)
    tol = dict(x=1e-8, v=1e-3 * v_max, F=2e-4, C=2e-3 * c_max)
    worst = dict(x=0.0, v=0.0, F=0.0, C=0.0)
    moved = 0
    for p, (xo, vo, Co, Fo) in zip(picks, ref):
        for key, a, b in (("x", x1[p], xo), ("v", v1[p], vo), ("F", F1[p], Fo), ("C", C1[p], Co)):
            worst[key] = max(worst[key], float(np.abs(a - b).max()))
        moved += np.abs(vo).max() > 0.1 * v_max
    print("largest error / bound:", {k: f"{worst[k]:.3g} / {tol[k]:.3g}" for k in tol}, flush=True)
    for key in tol:
        assert worst[key] <= tol[key], (key, worst[key], tol[key])
    assert moved >= 8  # the sample includes particles the indenter is driving


def test_p2g_conserves_mass_and_momentum(press):
    wl, sim = press
    cfg, dt = wl["cfg"], wl["dt"]
    x, v, _, _ = soa_to_aos(*(to_np(t) for t in sim.read_particles()))
    h = cfg["block_size"][0] / cfg["n"][0]
    m = cfg["rho"] * h ** 3
    sim.p2g(dt)
    M, P = sim.read_grid(0)
    M, P = to_np(M), to_np(P)
    assert abs(M.sum() - m * len(x)) <= 1e-6 * m * len(x)
    mom = m * v.sum(axis=0)
    scale = m * np.abs(v).sum()
    assert scale > 0
    # FP32 P2G rounds each of the 27 N contributions to a 2^-28 share of
    # m dx / dt (fixed point): a random-walk bound of ten times its spread
    quantum = m * cfg["dx"] / dt / 2.0 ** 28
    atol = 1e-6 * scale + 10 * np.sqrt(27 * len(x)) * quantum
    np.testing.assert_allclose(P.sum(axis=1), mom, rtol=0, atol=atol)
    # finish the substep so the handle is back between substeps
    k = SUBSTEPS_BEFORE + 1
    sim.grid_update(wl["poses"][k + 1], dt)
    sim.g2p(dt)
    sim.sync()


def test_heightmap_and_image_at_full_size(oracle_lib, press):
    wl, sim = press
    cfg = wl["cfg"]
    n0, n1, n2 = cfg["n"]
    x, _, _, _ = soa_to_aos(*(to_np(t) for t in sim.read_particles()))
    H = to_np(sim.heightmap())
    assert H.shape == (n1, n0)
    ztop = x[n0 * n1 * (n2 - 1):, 2].reshape(n1, n0)
    np.testing.assert_allclose(H, ztop, rtol=0, atol=2e-9)
    assert H.min() < W.top_z(cfg) - 0.2e-3  # the press (0.29-0.72 mm deep by now) shows in the map
    rp = wl["render"]
    img_g = to_np(sim.render(rp))
    img_o = oracle_lib.render_height(cfg, H, rp)
    assert img_g.shape == img_o.shape == (rp["h"], rp["w"], 3)
    # FP32 resampling and differences of the same map: ~3e-5 expected
    assert np.abs(img_g - img_o).max() <= 3e-4
