"""Sim: one elastomer contact simulated by libtacchi on the current GPU.

PyTorch supplies the device memory (one workspace tensor, output tensors)
and the HIP stream; all computation happens in the library's kernels.
"""
from __future__ import annotations

import ctypes
import json

import numpy as np
import torch

from . import native as N


class Sim:
    def __init__(self, cfg: dict, pose0, precision: str = "f64", tile: int = 0, device="cuda"):
        self.cfg = cfg
        self.precision = N.F64 if precision == "f64" else N.F32
        self.dtype = torch.float64 if self.precision == N.F64 else torch.float32
        self.device = torch.device(device)
        self._c = N.make_config(cfg, pose0, self.precision, tile)
        L = N.lib()
        nbytes = L.tacchi_workspace_bytes(ctypes.byref(self._c))
        if nbytes == 0:
            raise N.TacchiError(N.E_ARG, L.tacchi_last_error().decode())
        self.ws_bytes = nbytes
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        shift = (-raw.data_ptr()) % 256
        self._raw = raw
        self._ws_ptr = raw.data_ptr() + shift
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        N.check(L.tacchi_create(ctypes.byref(self._c), ctypes.c_void_p(self._ws_ptr), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.N = int(L.tacchi_num_particles(h))
        self.n = tuple(cfg["n"])

    @classmethod
    def borrowed(cls, handle, cfg: dict, precision: int, device, stream):
        """View of a handle owned elsewhere (a batch contact): read-out only."""
        self = cls.__new__(cls)
        self.cfg = cfg
        self.precision = precision
        self.dtype = torch.float64 if precision == N.F64 else torch.float32
        self.device = torch.device(device)
        self.stream = stream
        self._h = ctypes.c_void_p(handle)
        self._owned = False
        self.N = int(N.lib().tacchi_num_particles(self._h))
        self.n = tuple(cfg["n"])
        return self

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owned", True):
                N.lib().tacchi_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------ stepping
    def step(self, pose_end, dt: float):
        N.check(N.lib().tacchi_step(self._h, ctypes.byref(N.make_pose(pose_end)), dt))

    def run(self, poses, dt: float):
        arr = N.make_poses(poses)
        N.check(N.lib().tacchi_run(self._h, arr, len(poses), dt))

    STICKY, COULOMB = 0, 1

    def set_contact(self, model: int, mu: float = 0.0):
        """Contact model from the next substep: Sim.STICKY (no-slip, the
        default) or Sim.COULOMB with friction coefficient mu."""
        N.check(N.lib().tacchi_set_contact(self._h, int(model), float(mu)))

    def set_indenter_points(self, xyz, mass: float):
        """Represent the indenter by points [n][3] (indenter frame, metres) of
        `mass` kg each; an empty array returns to the shape's contact."""
        pts = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        n = pts.shape[0]
        nbytes = int(N.lib().tacchi_points_workspace_bytes(self._h, n)) if n > 0 else 0
        ws, ptr = None, 0
        if nbytes:
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
        N.check(N.lib().tacchi_set_indenter_points(self._h, pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                   n, float(mass), ctypes.c_void_p(ptr), nbytes))
        # the points and per-node indenter mass live here until the next call
        self._points_ws = ws

    def run_until_force(self, poses, dt: float, fz_limit: float) -> int:
        """Substeps to poses[0], poses[1], ... until the z contact force on the
        indenter reaches fz_limit [N] (tested on the device after every
        substep); returns the number of substeps that ran."""
        arr = N.make_poses(poses)
        done = ctypes.c_int32(0)
        N.check(N.lib().tacchi_run_until_force(self._h, arr, len(poses), dt, fz_limit, ctypes.byref(done)))
        return int(done.value)

    def p2g(self, dt: float):
        N.check(N.lib().tacchi_p2g(self._h, dt))

    def grid_update(self, pose_end, dt: float):
        N.check(N.lib().tacchi_grid_update(self._h, ctypes.byref(N.make_pose(pose_end)), dt))

    def g2p(self, dt: float):
        N.check(N.lib().tacchi_g2p(self._h, dt))

    def sync(self):
        N.check(N.lib().tacchi_sync(self._h))

    # ------------------------------------------------------------ outputs
    def _empty(self, *shape, dtype=None):
        return torch.empty(*shape, dtype=dtype or self.dtype, device=self.device)

    def heightmap(self) -> torch.Tensor:
        out = self._empty(self.n[1], self.n[0])
        N.check(N.lib().tacchi_heightmap(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def surface_displacement(self, res: int, sub: int = 1) -> torch.Tensor:
        """Top-surface displacement over res x res cells (mean of sub x sub
        points per cell), [res][res][3] (m, float32)."""
        out = self._empty(res, res, 3, dtype=torch.float32)
        N.check(N.lib().tacchi_surface_displacement(self._h, res, sub, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def markers(self, xy) -> torch.Tensor:
        """Displacement [n][3] (m, simulation precision) of the top surface at
        marker positions xy [n][2] (world metres on the undeformed top face)."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
        out = self._empty(xy.shape[0], 3)
        N.check(N.lib().tacchi_markers(self._h, xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), xy.shape[0],
                                       ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def render(self, rp: dict) -> torch.Tensor:
        out = self._empty(rp["h"], rp["w"], 3, dtype=torch.float32)
        r = N.make_render(rp)
        N.check(N.lib().tacchi_render(self._h, ctypes.byref(r), ctypes.c_void_p(out.data_ptr()),
                                      rp["h"], rp["w"], 1))
        return out

    def read_particles(self):
        """(x[3][N], v[3][N], C[9][N], F[9][N]) device tensors, SI units."""
        x, v = self._empty(3, self.N), self._empty(3, self.N)
        C, F = self._empty(9, self.N), self._empty(9, self.N)
        N.check(N.lib().tacchi_read_particles(self._h, *(ctypes.c_void_p(t.data_ptr()) for t in (x, v, C, F)), 1))
        return x, v, C, F

    def write_particles(self, x, v, C, F):
        ts = [torch.as_tensor(a, dtype=self.dtype).to(self.device).contiguous() for a in (x, v, C, F)]
        assert ts[0].shape == (3, self.N) and ts[1].shape == (3, self.N)
        assert ts[2].shape == (9, self.N) and ts[3].shape == (9, self.N)
        N.check(N.lib().tacchi_write_particles(self._h, *(ctypes.c_void_p(t.data_ptr()) for t in ts), 1))
        self.stream.synchronize()

    # ------------------------------------------------------------ checkpoints
    def save_checkpoint(self, path) -> None:
        """Write what the press needs to continue to an .npz file: the
        particle state (x, v, C, F as read_particles returns it, SI units),
        the indenter pose reached by the last substep, the configuration and
        the precision. The contact model and a point-cloud indenter are set
        on the handle by their own calls and are not part of the file."""
        x, v, C, F = (t.double().cpu().numpy() for t in self.read_particles())
        cfg = json.dumps(self.cfg, default=lambda o: o.item() if hasattr(o, "item") else list(o))
        np.savez(path, x=x, v=v, C=C, F=F, pose=self.pose(), cfg=np.array(cfg),
                 precision=np.array("f64" if self.precision == N.F64 else "f32"))

    @classmethod
    def from_checkpoint(cls, path, tile: int = 0, device="cuda"):
        """A simulator that continues the press saved by save_checkpoint: the
        same configuration and precision, the indenter at the saved pose and
        the saved particle state."""
        with np.load(path, allow_pickle=False) as d:
            cfg = json.loads(str(d["cfg"]))
            cfg = {k: tuple(v) if isinstance(v, list) else v for k, v in cfg.items()}
            sim = cls(cfg, d["pose"], precision=str(d["precision"]), tile=tile, device=device)
            sim.write_particles(d["x"], d["v"], d["C"], d["F"])
        return sim

    def read_grid(self, which: int):
        g = self.cfg["gn"]
        n = g[0] * g[1] * g[2]
        M = self._empty(n)
        vec = self._empty(3, n)
        N.check(N.lib().tacchi_read_grid(self._h, which, ctypes.c_void_p(M.data_ptr()),
                                         ctypes.c_void_p(vec.data_ptr()), 1))
        return M, vec

    def force(self) -> np.ndarray:
        f = (ctypes.c_double * 3)()
        N.check(N.lib().tacchi_indenter_force(self._h, f))
        return np.array(list(f))

    def timing_enable(self, classes=()):
        mask = 0
        for c in classes:
            mask |= 1 << N.KERNEL_CLASSES.index(c)
        N.check(N.lib().tacchi_timing_enable(self._h, mask))

    def timing_read(self, reset=True) -> dict:
        ms = (ctypes.c_double * N.NUM_KERNEL_CLASSES)()
        cnt = (ctypes.c_int64 * N.NUM_KERNEL_CLASSES)()
        N.check(N.lib().tacchi_timing_read(self._h, ms, cnt, 1 if reset else 0))
        return {name: (ms[k], cnt[k]) for k, name in enumerate(N.KERNEL_CLASSES)}

    def polar_fallbacks(self) -> int:
        c = ctypes.c_uint64()
        N.check(N.lib().tacchi_polar_fallbacks(self._h, ctypes.byref(c)))
        return int(c.value)

    def pose(self) -> np.ndarray:
        p = N.Pose()
        N.check(N.lib().tacchi_get_pose(self._h, ctypes.byref(p)))
        return np.array(list(p.pos) + list(p.quat))


def aos_to_soa(x, v, C, F):
    """Oracle AoS arrays ([N][3], [N][3], [N][3][3], [N][3][3]) to the ABI's SoA."""
    n = len(x)
    return (np.ascontiguousarray(np.asarray(x).T), np.ascontiguousarray(np.asarray(v).T),
            np.ascontiguousarray(np.asarray(C).reshape(n, 9).T), np.ascontiguousarray(np.asarray(F).reshape(n, 9).T))


def indenter_gap(cfgs, poses, res: int, lo: float = -2e-3, hi: float = 2e-3, device="cuda",
                 sub: int = 1) -> torch.Tensor:
    """Gap fields [n][res][res] (m, float32) of each config's indenter at the
    given pose over its block's undeformed top face, clamped to [lo, hi], each
    cell the mean of sub x sub points (hi = 0: the penetration field)."""
    n = len(cfgs)
    carr = (N.Config * n)()
    parr = (N.Pose * n)()
    for k in range(n):
        carr[k] = N.make_config(cfgs[k], poses[k], N.F32, 0)
        parr[k] = N.make_pose(poses[k])
    out = torch.empty(n, res, res, dtype=torch.float32, device=device)
    nbytes = int(N.lib().tacchi_indenter_gap_workspace_bytes(n))
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    N.check(N.lib().tacchi_indenter_gap(carr, parr, n, res, sub, lo, hi, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(ptr), nbytes,
                                        ctypes.c_void_p(torch.cuda.current_stream(out.device).cuda_stream)))
    return out
