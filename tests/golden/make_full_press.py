"""Write the FP64 oracle's end state of the whole 1.6M-particle GelSight press.

For each indenter family (seed = family: sphere, flat punch, cone, edge,
textured plate) the oracle runs the 200 x 200 x 40 lattice in the
256 x 256 x 64 grid at 0.1 mm through all 2000 substeps of 2 us (Sec. III-A,
Eqs. 1-11, the depth map of Sec. III-B) and stores

* H      the 200 x 200 depth map after the last substep (m, grid frame),
* idx    a seeded sample of particle indices (lattice order, x fastest):
         4096 drawn over the whole block and 4096 from the top ten layers
         within 4 mm (xy) of the indenter's axis,
* x      those particles' positions after the last substep (m),
* force  the contact force on the indenter in the last substep (N).

Only the oracle and the seeded workload generator are used. One seed takes
~20-25 minutes on one core; seeds run one process each:

    python tests/golden/make_full_press.py 0 1 2 3 4
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Process

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STEPS = 2000
N_UNIFORM = 4096
N_CONTACT = 4096


def fixture_path(seed: int) -> str:
    return os.path.join(HERE, f"full_press_seed{seed}.npz")


def sample_indices(wl, seed: int) -> np.ndarray:
    cfg = wl["cfg"]
    n0, n1, n2 = cfg["n"]
    N = n0 * n1 * n2
    rng = np.random.default_rng(1000 + seed)
    uni = rng.choice(N, size=N_UNIFORM, replace=False)
    h = cfg["block_size"][0] / n0
    i = np.arange(n0)
    j = np.arange(n1)
    X = cfg["block_origin"][0] + (i + 0.5) * h
    Y = cfg["block_origin"][1] + (j + 0.5) * h
    cx, cy = wl["poses"][0][0], wl["poses"][0][1]
    near = (X[None, :] - cx) ** 2 + (Y[:, None] - cy) ** 2 <= (4e-3) ** 2
    jj, ii = np.nonzero(near)
    cand = np.concatenate([(k * n1 + jj) * n0 + ii for k in range(n2 - 10, n2)])
    con = rng.choice(cand, size=min(N_CONTACT, len(cand)), replace=False)
    return np.unique(np.concatenate([uni, con])).astype(np.int64)


def run(seed: int) -> None:
    import oracle
    from paper_2301_08343_amd import workloads as W
    wl = W.gelsight_contact(seed=seed, steps=STEPS)
    sim = oracle.OracleSim(wl["cfg"], wl["poses"][0])
    t0 = time.time()
    for k in range(STEPS):
        st = sim.step(wl["poses"][k + 1], wl["dt"])
        if st != 0:
            raise RuntimeError(f"seed {seed}: oracle substep {k} failed with status {st}")
        if (k + 1) % 100 == 0:
            print(f"seed {seed} ({wl['name']}): {k + 1}/{STEPS} substeps, {time.time() - t0:.0f} s",
                  flush=True)
    idx = sample_indices(wl, seed)
    x = sim.particles()[0]
    np.savez_compressed(fixture_path(seed), H=sim.heightmap(), idx=idx, x=x[idx],
                        force=sim.force(), seed=np.int64(seed), steps=np.int64(STEPS))
    print(f"seed {seed}: wrote {fixture_path(seed)} after {time.time() - t0:.0f} s", flush=True)


def main(argv) -> None:
    import oracle
    oracle.build(force=False)
    seeds = [int(a) for a in argv] or [0, 1, 2, 3, 4]
    procs = [Process(target=run, args=(s,)) for s in seeds]
    for p in procs:
        p.start()
    for p in procs:
        p.join()
    bad = [s for s, p in zip(seeds, procs) if p.exitcode != 0]
    if bad:
        raise SystemExit(f"seeds failed: {bad}")


if __name__ == "__main__":
    main(sys.argv[1:])
