"""Batched contacts: each contact of a batch advanced by the batched, graph-
replayed kernels matches the same contact run alone, small contacts match the
FP64 oracle, and the tuner's choices round-trip through its cache file."""
import json
import math
import os

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


def to_np(t):
    return t.detach().cpu().double().numpy()


def tiny_contact(seed, steps, shape=W.SPHERE):
    """A 16 x 16 x 6 corotated block at 0.25 mm pressed by a sphere."""
    rng = W.SplitMix64(0x71 + seed)
    h = 0.25e-3
    n = (16, 16, 6)
    pad = 5
    cfg = W._contact(block_origin=(pad * h, pad * h, 3 * h), block_size=(n[0] * h, n[1] * h, n[2] * h), n=n,
                     grid_origin=(0, 0, 0), dx=h, gn=(n[0] + 2 * pad, n[1] + 2 * pad, n[2] + 10),
                     E=rng.uniform(0.1e6, 0.3e6), nu=rng.uniform(0.40, 0.48), rho=1000.0, model=W.COROTATED,
                     shape=shape, sp=[1.5e-3], seed=seed)
    cx, cy = W.block_center_xy(cfg)
    depth = 0.4e-3
    tilt = W.quat_axis_angle((1.0, 0.3, 0.0), math.radians(4.0))
    poses = W.press_trajectory((cx + rng.uniform(-0.5e-3, 0.5e-3), cy, W.top_z(cfg)), tilt, depth, steps)
    lam = cfg["E"] * cfg["nu"] / ((1 + cfg["nu"]) * (1 - 2 * cfg["nu"]))
    mu = cfg["E"] / (2 * (1 + cfg["nu"]))
    dt = 0.45 * h / math.sqrt((lam + 2 * mu) / cfg["rho"])
    return dict(cfg=cfg, poses=poses, dt=dt)


def test_batch_contacts_match_their_solo_runs(gpu):
    Batch, Sim = gpu
    S = 120
    contacts = [W.batch_contact(seed, steps=S) for seed in range(4)]
    batch = Batch(contacts, S)
    batch.run(S)  # two graph replays of 50 substeps + 20 direct
    assert batch.substeps_done() == S
    batch.sync()
    tuning = batch.tuning()
    for i, c in enumerate(contacts):
        solo = Sim(c["cfg"], c["poses"][0], precision="f32", tile=tuning[i][0])
        solo.run(c["poses"][1:S + 1], c["dt"])
        xs = to_np(solo.read_particles()[0])
        xb = to_np(batch.contact(i).read_particles()[0])
        hs = to_np(solo.heightmap())
        hb = to_np(batch.contact(i).heightmap())
        diff = np.abs(xs - xb).max()
        print(f"contact {i}: N = {solo.N}, tile {tuning[i][0]}, wg {tuning[i][1]}, max |dx| = {diff:.3e} m")
        assert diff <= 2e-9
        assert np.abs(hs - hb).max() <= 2e-9
        assert np.abs(hb - W.top_z(c["cfg"])).max() > 1e-6  # the indenter deformed the surface


def test_batch_graph_and_direct_launches_agree(gpu):
    Batch, _ = gpu
    S = 104
    contacts = [W.batch_contact(seed, steps=S) for seed in (5, 6)]
    a = Batch(contacts, S, use_graph=True)
    b = Batch(contacts, S, use_graph=False)
    a.run(50)
    a.run(54)
    b.run(S)
    a.sync()
    b.sync()
    for i in range(2):
        xa = to_np(a.contact(i).read_particles()[0])
        xb = to_np(b.contact(i).read_particles()[0])
        assert np.array_equal(xa, xb)


def test_small_batch_matches_oracle(oracle_lib, gpu):
    Batch, _ = gpu
    S = 150
    contacts = [tiny_contact(s, S) for s in range(3)]
    batch = Batch(contacts, S)
    batch.run(S)
    batch.sync()
    for i, c in enumerate(contacts):
        orc = oracle_lib.OracleSim(c["cfg"], c["poses"][0])
        orc.run(c["poses"], c["dt"], 0, S)
        xo = orc.particles()[0]
        xb = to_np(batch.contact(i).read_particles()[0]).T
        err = np.abs(xb - xo).max()
        print(f"tiny contact {i}: max |dx| = {err:.3e} m")
        assert err <= 1e-5 * c["cfg"]["block_size"][0]
        assert np.abs(to_np(batch.contact(i).heightmap()) - orc.heightmap()).max() <= 0.1e-6


def test_drawn_batch_matches_oracle(oracle_lib, gpu):
    """Contacts drawn by the uneven batch's generator (seeds covering the five
    indenter families: lattice spacing, thickness, E, nu, corotated law, tilt,
    depth and time step as drawn), cut to 32 x 32 particles laterally, pressed
    to their drawn depth in 400 substeps in one batch, FP32 with the FP64
    polar gate, against the FP64 oracle: positions within 1e-5 of the cut
    block's width and depth maps within 0.1 um."""
    Batch, _ = gpu
    S = 400
    seeds = [0, 1, 2, 3, 6]  # textured plate, edge, sphere, cylinder, cone
    contacts = [W.batch_contact(s, steps=S, max_lateral=32) for s in seeds]
    assert sorted(c["cfg"]["shape"] for c in contacts) == [0, 1, 2, 3, 4]
    batch = Batch(contacts, S)
    batch.run(S)
    batch.sync()
    for i, c in enumerate(contacts):
        print(f"drawn contact {c['name']}: n = {c['cfg']['n']}, h = {c['cfg']['dx'] * 1e3:.3f} mm", flush=True)
        orc = oracle_lib.OracleSim(c["cfg"], c["poses"][0])
        orc.run(c["poses"], c["dt"], 0, S)
        xo = orc.particles()[0]
        Ho = orc.heightmap()
        xb = to_np(batch.contact(i).read_particles()[0]).T
        Hb = to_np(batch.contact(i).heightmap())
        err, err_h = np.abs(xb - xo).max(), np.abs(Hb - Ho).max()
        print(f"  max |dx| = {err:.3e} m, max |dH| = {err_h:.3e} m, indent {W.top_z(c['cfg']) - Ho.min():.3e} m")
        assert W.top_z(c["cfg"]) - Ho.min() > 0.1e-3  # the contact engaged
        assert err <= 1e-5 * c["cfg"]["block_size"][0]
        assert err_h <= 0.1e-6


SETTINGS = [(t, w, q) for t in (4, 8) for w in (64, 128, 256) for q in (1, 2)]


def test_tuner_sweeps_every_setting_and_reuses_its_cache(gpu, tmp_path):
    """Per (material model, size class) the tuner times all 12 settings
    (tile 4/8 x workgroup 64/128/256 x 1/2 blocks per workgroup), keeps the
    fastest, records every candidate in the cache, and a second batch reuses
    the cached choices without timing."""
    Batch, _ = gpu
    S = 240  # the tuner advances 200 substeps into the press before it times
    contacts = [W.batch_contact(seed, steps=S) for seed in (7, 8, 9)]
    neo = dict(W.batch_contact(7, steps=S))
    neo["cfg"] = dict(neo["cfg"], model=W.NEOHOOKEAN)
    contacts.append(neo)  # same size class as seed 7, other material model: its own entry
    path = str(tmp_path / "tune.json")
    a = Batch(contacts, S, tune_cache=path, tune=True)
    ta = a.tuning()
    data = json.load(open(path))
    classes = {(c["cfg"]["model"], int(math.floor(math.log2(W.lattice_count(c["cfg"]))))) for c in contacts}
    assert {(e["model"], e["log2n"]) for e in data["entries"]} == classes
    for e in data["entries"]:
        assert e["precision"] == "f32"
        cands = e["candidates"]
        assert sorted(tuple(c[:3]) for c in cands) == sorted(SETTINGS)
        assert all(c[3] > 0 for c in cands)
        best = min(cands, key=lambda c: c[3])
        assert (e["tile"], e["wg"], e["ipw"]) == tuple(best[:3])
        print(f"class model {e['model']} log2n {e['log2n']}: chose B{e['tile']} wg{e['wg']} ipw{e['ipw']} "
              f"{e['us_per_substep']:.1f} us; slowest {max(c[3] for c in cands):.1f} us", flush=True)
    # the per-class choices stand unless the whole batch ran faster with the
    # default everywhere
    us_tuned, us_default = a.tuning_check()
    print(f"whole batch: {us_tuned:.1f} us per substep tuned, {us_default:.1f} default", flush=True)
    assert us_tuned > 0 and us_default > 0
    for i, c in enumerate(contacts):
        cls = (c["cfg"]["model"], int(math.floor(math.log2(W.lattice_count(c["cfg"])))))
        e = next(e for e in data["entries"] if (e["model"], e["log2n"]) == cls)
        want = (e["tile"], e["wg"], e["ipw"]) if us_tuned <= us_default else (8, 256, 1)
        assert tuple(ta[i][:3]) == want
    b = Batch(contacts, S, tune_cache=path, tune=False)
    assert [t[:3] for t in b.tuning()] == [
        (e["tile"], e["wg"], e["ipw"]) for e in (next(e for e in data["entries"] if (e["model"], e["log2n"]) == (
            c["cfg"]["model"], int(math.floor(math.log2(W.lattice_count(c["cfg"])))))) for c in contacts)]
    assert b.tuning_check() == (0.0, 0.0)  # read from the cache, not timed
    a.run(S)
    b.run(S)
    for i in range(len(contacts)):
        assert np.array_equal(to_np(a.contact(i).read_particles()[0]), to_np(b.contact(i).read_particles()[0]))


@pytest.mark.parametrize("setting", [(4, 64, 2), (8, 64, 1), (8, 128, 2), (4, 256, 1)],
                         ids=lambda s: f"B{s[0]}_wg{s[1]}_ipw{s[2]}")
def test_every_tuner_setting_gives_the_same_substeps(gpu, tmp_path, setting):
    """A setting forced through the cache runs the same substeps bit for bit
    as the default launch of the same tile (the work per block does not
    depend on the workgroup size or on how many blocks a workgroup takes)."""
    Batch, _ = gpu
    S = 60
    contacts = [W.batch_contact(seed, steps=S) for seed in (3, 4)]
    tile, wg, ipw = setting
    path = str(tmp_path / "forced.json")
    ref_path = str(tmp_path / "ref.json")
    entries = []
    for c in contacts:
        cls = int(math.floor(math.log2(W.lattice_count(c["cfg"]))))
        entries.append({"arch": "", "precision": "f32", "model": c["cfg"]["model"], "log2n": cls})
    import torch as _t
    arch = _t.cuda.get_device_properties(0).gcnArchName.split(":")[0]

    def write(p, t, w, q):
        with open(p, "w") as f:
            json.dump({"entries": [dict(e, arch=arch, tile=t, wg=w, ipw=q, us_per_substep=1.0, candidates=[])
                                   for e in entries]}, f)

    write(path, tile, wg, ipw)
    write(ref_path, tile, 256, 1)
    a = Batch(contacts, S, tune_cache=path, tune=False)
    assert all(tuple(t[:3]) == setting for t in a.tuning())
    b = Batch(contacts, S, tune_cache=ref_path, tune=False)
    assert all(tuple(t[:3]) == (tile, 256, 1) for t in b.tuning())
    a.run(S)
    b.run(S)
    a.sync()
    b.sync()
    for i in range(len(contacts)):
        xa = to_np(a.contact(i).read_particles()[0])
        xb = to_np(b.contact(i).read_particles()[0])
        assert np.array_equal(xa, xb)
        assert np.abs(to_np(a.contact(i).heightmap()) - W.top_z(contacts[i]["cfg"])).max() > 1e-6
