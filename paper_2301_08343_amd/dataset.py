"""Training data of the tactile surrogate, produced by the batched MPM.

A sample is one GelSight-sized contact (indenter family, shape parameters,
position and depth drawn from its seed) solved at lattice spacing h:
  input  x[res][res][2]: the penetration of the indenter at its final pose
         into the undeformed top face (the gap clamped to [-GAP_CLIP, 0]:
         the elastomer only feels the indenter where they touch), and the
         press depth broadcast, both in mm;
  target y[res][res][3]: the top surface's displacement (ux, uy, uz) after
         the press, in units of Y_UNIT.
Both fields are cell means over SUB x SUB points, so an edge or a texture
finer than a cell enters as its covered fraction rather than as an aliased
point sample, and the cell mean of the penetration is also the contact term
the network's output adds in FP32 (Net.contact_residual).
All of it is computed by the library (gap field kernel, batched substeps,
displacement resampling kernel); this module only batches the calls.
"""
from __future__ import annotations

import time

import torch

from . import workloads as W
from .batch import Batch
from .sim import indenter_gap

GAP_CLIP = 2e-3   # m: the input is the penetration, clamped to [-GAP_CLIP, 0]
X_UNIT = 1e-3     # inputs in mm
Y_UNIT = 1e-4     # targets in 0.1 mm
RES = 64
SUB = 4           # each input and target cell is the mean of SUB x SUB points
H_DATA = 0.2e-3   # lattice spacing of the training solves


def contacts_for(seeds, h=H_DATA, full=True):
    """Contacts of the given seeds; full=False leaves out the trajectories
    (enough for the surrogate inputs; solve() rebuilds them)."""
    return [W.gelsight_contact_at(int(s), h, full) for s in seeds]


def _full(c):
    return c if c["poses"] is not None else W.gelsight_contact_at(c["seed"], c["h"], True)


def inputs(contacts, res=RES, device="cuda") -> torch.Tensor:
    """[n][res][res][2] float32 surrogate inputs (gap, depth) in mm."""
    gap = indenter_gap([c["cfg"] for c in contacts], [c["end_pose"] for c in contacts], res, -GAP_CLIP, 0.0,
                       device, sub=SUB)
    x = torch.empty(len(contacts), res, res, 2, dtype=torch.float32, device=device)
    x[..., 0] = gap / X_UNIT
    x[..., 1] = torch.tensor([c["depth"] / X_UNIT for c in contacts], dtype=torch.float32,
                             device=device).view(-1, 1, 1)
    return x


def solve(contacts, res=RES, tune_cache=None, device="cuda") -> torch.Tensor:
    """Run every contact's full press with the batched MPM and return the
    [n][res][res][3] top-surface displacement in Y_UNIT (float32)."""
    contacts = [_full(c) for c in contacts]
    steps = contacts[0]["steps"]
    if any(c["steps"] != steps for c in contacts):
        raise ValueError("contacts of one batch must share their substep count")
    b = Batch(contacts, steps, tune_cache=tune_cache, device=device)
    try:
        b.run(steps)
        u = b.surface_displacement(res, SUB)
    finally:
        b.close()
    return u / Y_UNIT


def generate(seeds, res=RES, h=H_DATA, batch=128, device="cuda", log=print):
    """(x, y) device tensors for the given seeds, solved `batch` at a time."""
    seeds = list(seeds)
    xs, ys = [], []
    t0 = time.perf_counter()
    for k in range(0, len(seeds), batch):
        cs = contacts_for(seeds[k:k + batch], h)
        xs.append(inputs(cs, res, device))
        ys.append(solve(cs, res, device=device))
        if log:
            done = k + len(cs)
            el = time.perf_counter() - t0
            ps = sum(c["particles"] * c["steps"] for c in cs)
            log(f"data: {done}/{len(seeds)} samples, {el:.1f} s, last batch {ps:.3e} particle-substeps")
    return torch.cat(xs), torch.cat(ys)

