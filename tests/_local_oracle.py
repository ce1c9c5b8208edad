"""Sampled one-substep checks against the oracle for runs too large for it:
each sampled particle is advanced by a small oracle run over the particles
that can reach its grid nodes (test helper, not collected)."""
import numpy as np

from paper_2301_08343_amd import workloads as W


def soa_to_aos(x, v, C, F):
    n = x.shape[1]
    return x.T.copy(), v.T.copy(), C.T.reshape(n, 3, 3).copy(), F.T.reshape(n, 3, 3).copy()


def samples(cfg, x, pose):
    """Particle indices: 16 near the top face under the indenter, 16 near
    the top face anywhere, 16 in the bulk; all at least 10 layers above the
    bonded bottom layer and far from the grid walls."""
    n0, n1, n2 = cfg["n"]
    rng = W.SplitMix64(2024)
    lay = lambda i, j, k: i + n0 * (j + n1 * k)
    picks = []
    r = np.hypot(x[:, 0] - pose[0], x[:, 1] - pose[1])
    top = np.arange(lay(0, 0, n2 - 4), n0 * n1 * n2)
    under = top[np.argsort(r[top])[:400]]
    picks += [int(under[rng.randint(len(under))]) for _ in range(16)]
    picks += [lay(rng.randint(n0), rng.randint(n1), n2 - 1 - rng.randint(3)) for _ in range(16)]
    picks += [lay(rng.randint(n0), rng.randint(n1), 10 + rng.randint(n2 - 14)) for _ in range(16)]
    return sorted(set(picks))


def local_oracle_step(oracle_lib, cfg, x, v, C, F, p, pose0, pose1, dt):
    """The sampled particle p after one substep, from an oracle run over the
    particles whose stencil base lies within 3 nodes of p's on every axis (a
    superset of those that reach p's 27 nodes), on the part of the grid their
    stencils cover (the same nodes, so the same contact decisions)."""
    dx = cfg["dx"]
    go = np.array(cfg["grid_origin"])
    base = np.floor((x - go) / dx - 0.5).astype(np.int64)
    near = np.flatnonzero(np.abs(base - base[p]).max(axis=1) <= 3)
    lo = base[near].min(axis=0) - 1
    hi = base[near].max(axis=0) + 3
    assert (lo >= 3).all() and (hi <= np.array(cfg["gn"]) - 4).all(), "sample too close to a grid wall"
    assert lo[2] > cfg["floor_node"], "sample too close to the held floor"
    h = cfg["block_size"][0] / cfg["n"][0]
    sub = dict(cfg, block_origin=tuple(go + lo * dx), block_size=(len(near) * h, h, h), n=(len(near), 1, 1),
               grid_origin=tuple(go + lo * dx), gn=tuple(int(g) for g in hi - lo + 1),
               n_fixed_layers=0, floor_node=-1, wall_nodes=0)
    orc = oracle_lib.OracleSim(sub, pose0)
    orc.set_particles(x[near], v[near], C[near], F[near])
    assert orc.step(pose1, dt) == 0
    xo, vo, Co, Fo = orc.particles()
    k = int(np.flatnonzero(near == p)[0])
    return xo[k], vo[k], Co[k], Fo[k]
