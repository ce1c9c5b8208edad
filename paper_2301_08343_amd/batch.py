"""Batch: many independent contacts advanced together by libtacchi's batched
kernels (argument marshalling only)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import native as N
from .sim import Sim


class Batch:
    """`contacts` are workload dicts (cfg, poses [S+1][7], dt); all run FP32.
    With use_graph the batch runs on its own non-default stream so that runs
    of substeps are captured and replayed as a HIP graph."""

    def __init__(self, contacts, substeps: int, tune_cache: str | None = None, tune: bool = False,
                 use_graph: bool = True, device="cuda"):
        n = len(contacts)
        self.contacts = contacts
        self.device = torch.device(device)
        self.substeps = substeps
        cfgs = (N.Config * n)()
        traj = (N.Pose * (n * (substeps + 1)))()
        dts = (ctypes.c_double * n)()
        for i, c in enumerate(contacts):
            cfgs[i] = N.make_config(c["cfg"], c["poses"][0], N.F32, 0)
            poses = np.asarray(c["poses"])
            for k in range(substeps + 1):
                p = poses[min(k, len(poses) - 1)]
                traj[i * (substeps + 1) + k] = N.make_pose(p)
            dts[i] = c["dt"]
        L = N.lib()
        nbytes = L.tacchi_batch_workspace_bytes(cfgs, n, substeps)
        if nbytes == 0:
            raise N.TacchiError(N.E_ARG, L.tacchi_last_error().decode())
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._raw = raw
        ptr = raw.data_ptr() + ((-raw.data_ptr()) % 256)
        self.stream = torch.cuda.Stream(self.device) if use_graph else torch.cuda.default_stream(self.device)
        h = ctypes.c_void_p()
        sptr = self.stream.cuda_stream if use_graph else 0
        N.check(L.tacchi_batch_create(cfgs, n, traj, dts, substeps,
                                      tune_cache.encode() if tune_cache else None, 1 if tune else 0,
                                      ctypes.c_void_p(ptr), nbytes, ctypes.c_void_p(sptr), ctypes.byref(h)))
        self._h = h
        self.n = n
        self._views = [Sim.borrowed(L.tacchi_batch_contact(h, i), contacts[i]["cfg"], N.F32, self.device,
                                    self.stream) for i in range(n)]

    def run(self, substeps: int):
        N.check(N.lib().tacchi_batch_run(self._h, substeps))

    def contact(self, i: int) -> Sim:
        return self._views[i]

    def tuning(self):
        """Per contact (tile B, workgroup size, grid blocks per workgroup, tuned us per substep)."""
        t = (ctypes.c_int32 * self.n)()
        w = (ctypes.c_int32 * self.n)()
        q = (ctypes.c_int32 * self.n)()
        us = (ctypes.c_double * self.n)()
        N.check(N.lib().tacchi_batch_tuning(self._h, t, w, q, us))
        return [(t[i], w[i], q[i], us[i]) for i in range(self.n)]

    def tuning_check(self):
        """(whole-batch us per substep with the tuned choices, with the default
        everywhere); zeros when the batch was not tuned."""
        a, b = ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().tacchi_batch_tuning_check(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def substeps_done(self) -> int:
        return int(N.lib().tacchi_batch_substeps_done(self._h))

    def sync(self):
        N.check(N.lib().tacchi_batch_sync(self._h))

    def surface_displacement(self, res: int, sub: int = 1) -> torch.Tensor:
        """[n][res][res][3] top-surface displacements (m, float32, mean of
        sub x sub points per cell); synchronises."""
        out = torch.empty(self.n, res, res, 3, dtype=torch.float32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        N.check(N.lib().tacchi_batch_surface_displacement(self._h, res, sub, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def close(self):
        if getattr(self, "_h", None):
            for v in self._views:
                v._h = None
            N.lib().tacchi_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
