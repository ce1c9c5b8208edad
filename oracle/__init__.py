"""CPU FP64 oracle for the tactile MLS-MPM path -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It wraps the plain C oracle (oracle.c) through ctypes and
shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DEFAULT_LIB = os.path.join(_HERE, "liboracle.so")
# The planted-mistake tests point this at a build of a mutated copy of
# oracle.c, to show that the pins catch the mistake.
LIB_PATH = os.environ.get("TACCHI_ORACLE_LIB") or _DEFAULT_LIB
SOURCES = [os.path.join(_HERE, "oracle.c")]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall", "-Wextra",
          "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE FP64: no contraction, no fast-math)."""
    if LIB_PATH != _DEFAULT_LIB:
        return LIB_PATH  # a mutated build, used as given
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *SOURCES, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcConfig(ctypes.Structure):
    _fields_ = [("block_origin", ctypes.c_double * 3), ("block_size", ctypes.c_double * 3),
                ("n", ctypes.c_int32 * 3), ("grid_origin", ctypes.c_double * 3),
                ("dx", ctypes.c_double), ("gn", ctypes.c_int32 * 3),
                ("E", ctypes.c_double), ("nu", ctypes.c_double), ("rho", ctypes.c_double),
                ("model", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("sp", ctypes.c_double * 8), ("seed", ctypes.c_uint64),
                ("gravity", ctypes.c_double * 3), ("n_fixed_layers", ctypes.c_int32),
                ("floor_node", ctypes.c_int32), ("wall_nodes", ctypes.c_int32)]


class OrcRender(ctypes.Structure):
    _fields_ = [("ka_ia", ctypes.c_double), ("kd", ctypes.c_double), ("ks", ctypes.c_double),
                ("alpha", ctypes.c_double), ("light_elev_deg", ctypes.c_double),
                ("light_azim_deg", ctypes.c_double * 3), ("pitch", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(OrcConfig), _dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_num_particles.restype = ctypes.c_int64
        L.orc_num_particles.argtypes = [ctypes.c_void_p]
        L.orc_num_nodes.restype = ctypes.c_int64
        L.orc_num_nodes.argtypes = [ctypes.c_void_p]
        for name in ("orc_get_particles", "orc_set_particles"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
        for name in ("orc_get_pose", "orc_set_pose"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp]
        for name in ("orc_p2g", "orc_g2p"):
            getattr(L, name).argtypes = [ctypes.c_void_p, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_int
        for name in ("orc_grid_update", "orc_step"):
            getattr(L, name).argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_int
        L.orc_get_grid.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_force.argtypes = [ctypes.c_void_p, _dp]
        L.orc_set_contact.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.orc_set_contact.restype = None
        L.orc_set_indenter_points.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int64, ctypes.c_double]
        L.orc_set_indenter_points.restype = ctypes.c_int
        L.orc_indenter_mass.argtypes = [ctypes.c_void_p, _dp]
        L.orc_indenter_mass.restype = None
        L.orc_heightmap.argtypes = [ctypes.c_void_p, _dp]
        L.orc_render.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcRender), ctypes.c_int32,
                                 ctypes.c_int32, _dp]
        L.orc_render_height.argtypes = [ctypes.POINTER(OrcConfig), _dp, ctypes.POINTER(OrcRender),
                                        ctypes.c_int32, ctypes.c_int32, _dp]
        L.orc_bspline.restype = ctypes.c_double
        L.orc_bspline.argtypes = [ctypes.c_double]
        L.orc_lame.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_stress.restype = ctypes.c_int
        L.orc_stress.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_polar.restype = ctypes.c_int
        L.orc_polar.argtypes = [_dp, _dp, _dp]
        L.orc_phi.restype = ctypes.c_double
        L.orc_phi.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64, _dp]
        L.orc_indenter_velocity.argtypes = [_dp, _dp, ctypes.c_double, _dp, _dp]
        L.orc_lowest_point.restype = ctypes.c_double
        L.orc_lowest_point.argtypes = [ctypes.c_int, _dp, ctypes.c_uint64, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_noise2.restype = ctypes.c_double
        L.orc_noise2.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def make_config(cfg: dict) -> OrcConfig:
    c = OrcConfig()
    c.block_origin[:] = cfg["block_origin"]
    c.block_size[:] = cfg["block_size"]
    c.n[:] = cfg["n"]
    c.grid_origin[:] = cfg["grid_origin"]
    c.dx = cfg["dx"]
    c.gn[:] = cfg["gn"]
    c.E, c.nu, c.rho = cfg["E"], cfg["nu"], cfg["rho"]
    c.model = cfg["model"]
    c.shape = cfg["shape"]
    c.sp[:] = cfg["sp"]
    c.seed = cfg["seed"]
    c.gravity[:] = cfg["gravity"]
    c.n_fixed_layers = cfg["n_fixed_layers"]
    c.floor_node = cfg["floor_node"]
    c.wall_nodes = cfg["wall_nodes"]
    return c


def make_render(rp: dict) -> OrcRender:
    r = OrcRender()
    r.ka_ia, r.kd, r.ks, r.alpha = rp["ka_ia"], rp["kd"], rp["ks"], rp["alpha"]
    r.light_elev_deg = rp["light_elev_deg"]
    r.light_azim_deg[:] = rp["light_azim_deg"]
    r.pitch = rp["pitch"]
    return r


class OracleSim:
    """One elastomer contact simulated by the FP64 oracle."""

    def __init__(self, cfg: dict, pose0):
        self.cfg = cfg
        self._c = make_config(cfg)
        p0 = np.ascontiguousarray(pose0, dtype=np.float64)
        self._h = lib().orc_create(ctypes.byref(self._c), _ptr(p0))
        if not self._h:
            raise MemoryError("orc_create failed")
        self.N = lib().orc_num_particles(self._h)
        self.nn = lib().orc_num_nodes(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def particles(self):
        x = np.zeros((self.N, 3)); v = np.zeros((self.N, 3))
        C = np.zeros((self.N, 3, 3)); F = np.zeros((self.N, 3, 3))
        lib().orc_get_particles(self._h, _ptr(x), _ptr(v), _ptr(C), _ptr(F))
        return x, v, C, F

    def set_particles(self, x, v, C, F):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, v, C, F)]
        lib().orc_set_particles(self._h, *[_ptr(a) for a in arrs])

    def pose(self):
        p = np.zeros(7)
        lib().orc_get_pose(self._h, _ptr(p))
        return p

    def set_pose(self, pose):
        p = np.ascontiguousarray(pose, dtype=np.float64)
        lib().orc_set_pose(self._h, _ptr(p))

    def p2g(self, dt):
        return lib().orc_p2g(self._h, dt)

    def grid_update(self, pose_end, dt):
        p = np.ascontiguousarray(pose_end, dtype=np.float64)
        return lib().orc_grid_update(self._h, _ptr(p), dt)

    def g2p(self, dt):
        return lib().orc_g2p(self._h, dt)

    def step(self, pose_end, dt):
        p = np.ascontiguousarray(pose_end, dtype=np.float64)
        return lib().orc_step(self._h, _ptr(p), dt)

    def run(self, poses, dt, start=0, stop=None):
        """Advance through poses[start+1 .. stop] (pose k -> k+1 per substep)."""
        stop = len(poses) - 1 if stop is None else stop
        for k in range(start, stop):
            st = self.step(poses[k + 1], dt)
            if st != 0:
                raise RuntimeError(f"oracle step {k} failed with status {st}")

    def run_until_force(self, poses, dt, fz_limit, start=0, stop=None):
        """Sec. III-C's terminal condition on the contact force: advance
        through poses[start+1 ..] one substep at a time and stop after the
        first substep whose contact force on the indenter has a z component
        >= fz_limit; returns the number of substeps run."""
        stop = len(poses) - 1 if stop is None else stop
        done = 0
        for k in range(start, stop):
            st = self.step(poses[k + 1], dt)
            if st != 0:
                raise RuntimeError(f"oracle step {k} failed with status {st}")
            done += 1
            if self.force()[2] >= fz_limit:
                break
        return done

    def grid(self):
        M = np.zeros(self.nn); P = np.zeros((self.nn, 3)); V = np.zeros((self.nn, 3))
        lib().orc_get_grid(self._h, _ptr(M), _ptr(P), _ptr(V))
        return M, P, V

    def set_contact(self, model: int, mu: float = 0.0):
        """0: no-slip contact (default); 1: Coulomb friction with coefficient mu."""
        lib().orc_set_contact(self._h, int(model), float(mu))

    def set_indenter_points(self, xyz, mass: float):
        """The indenter as particles: points [n][3] in the indenter frame, mass each."""
        pts = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        assert lib().orc_set_indenter_points(self._h, _ptr(pts), pts.shape[0], float(mass)) == 0

    def indenter_mass(self):
        """Indenter mass per grid node (node order x fastest) of the last grid update."""
        out = np.zeros(self.nn)
        lib().orc_indenter_mass(self._h, _ptr(out))
        return out

    def force(self):
        f = np.zeros(3)
        lib().orc_force(self._h, _ptr(f))
        return f

    def heightmap(self):
        n = self.cfg["n"]
        H = np.zeros((n[1], n[0]))
        lib().orc_heightmap(self._h, _ptr(H))
        return H

    def render(self, rp: dict):
        r = make_render(rp)
        out = np.zeros((rp["h"], rp["w"], 3))
        lib().orc_render(self._h, ctypes.byref(r), rp["h"], rp["w"], _ptr(out))
        return out


def render_height(cfg: dict, H, rp: dict):
    c = make_config(cfg)
    r = make_render(rp)
    Hc = np.ascontiguousarray(H, dtype=np.float64)
    out = np.zeros((rp["h"], rp["w"], 3))
    lib().orc_render_height(ctypes.byref(c), _ptr(Hc), ctypes.byref(r), rp["h"], rp["w"], _ptr(out))
    return out


def bspline(r: float) -> float:
    return lib().orc_bspline(r)


def lame(E, nu):
    mu = ctypes.c_double(); lam = ctypes.c_double()
    lib().orc_lame(E, nu, ctypes.byref(mu), ctypes.byref(lam))
    return mu.value, lam.value


def stress(model: int, mu: float, lam: float, F):
    Fc = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    tau = np.zeros(9)
    st = lib().orc_stress(model, mu, lam, _ptr(Fc), _ptr(tau))
    return st, tau.reshape(3, 3)


def polar(F):
    Fc = np.ascontiguousarray(F, dtype=np.float64).reshape(9)
    R = np.zeros(9); S = np.zeros(9)
    st = lib().orc_polar(_ptr(Fc), _ptr(R), _ptr(S))
    return st, R.reshape(3, 3), S.reshape(3, 3)


def phi(shape: int, sp, seed: int, p_local):
    spc = np.ascontiguousarray(list(sp) + [0.0] * (8 - len(sp)), dtype=np.float64)
    pc = np.ascontiguousarray(p_local, dtype=np.float64)
    return lib().orc_phi(shape, _ptr(spc), seed, _ptr(pc))


def indenter_velocity(pose0, pose1, dt, X):
    a = np.ascontiguousarray(pose0, dtype=np.float64)
    b = np.ascontiguousarray(pose1, dtype=np.float64)
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    v = np.zeros(3)
    lib().orc_indenter_velocity(_ptr(a), _ptr(b), dt, _ptr(Xc), _ptr(v))
    return v


def noise2(seed: int, x: float, y: float) -> float:
    return lib().orc_noise2(seed, x, y)


def lowest_point(shape: int, sp, seed: int, pose, x, y, zlo, zhi, nscan=20000):
    spc = np.ascontiguousarray(list(sp) + [0.0] * (8 - len(sp)), dtype=np.float64)
    pc = np.ascontiguousarray(pose, dtype=np.float64)
    return lib().orc_lowest_point(shape, _ptr(spc), seed, _ptr(pc), x, y, zlo, zhi, nscan)


def indenter_gap(cfg: dict, pose, res: int, lo: float, hi: float, nscan: int = 20000, sub: int = 1):
    """[res][res] gap z_ind - z_top over a res x res partition of the block's
    top face (z_top = top face of the undeformed block), where z_ind is the
    indenter's lowest point on a vertical, clamped to [lo, hi]; each cell is
    the mean over sub x sub points at (c + (q + 1/2)/sub) * width / res."""
    ox, oy, oz = cfg["block_origin"]
    wx, wy, wz = cfg["block_size"]
    ztop = oz + wz
    out = np.zeros((res, res))
    for r in range(res):
        for c in range(res):
            acc = 0.0
            for qy in range(sub):
                for qx in range(sub):
                    x = ox + (c + (qx + 0.5) / sub) * wx / res
                    y = oy + (r + (qy + 0.5) / sub) * wy / res
                    z = lowest_point(cfg["shape"], cfg["sp"], cfg["seed"], pose, x, y, ztop + lo, ztop + hi, nscan)
                    acc += min(max(z - ztop, lo), hi)
            out[r, c] = acc / (sub * sub)
    return out


def markers(cfg: dict, x, xy):
    """[n][3] displacement of the top surface at marker positions xy [n][2]
    (world metres on the undeformed top face). Sec. VI: a marker moves with
    the surface particles at its position; here the displacement x - X is
    interpolated bilinearly between the four top-layer particles around the
    point (particle i at (i + 1/2) h), a point on the half-cell rim outside
    the outermost particle centres taking the edge value."""
    n0, n1, n2 = cfg["n"]
    h = [cfg["block_size"][a] / cfg["n"][a] for a in range(3)]
    o = cfg["block_origin"]
    top = np.asarray(x, dtype=np.float64).reshape(n2, n1, n0, 3)[n2 - 1]
    ii, jj = np.meshgrid(np.arange(n0), np.arange(n1), indexing="xy")
    rest = np.stack([o[0] + (ii + 0.5) * h[0], o[1] + (jj + 0.5) * h[1],
                     np.full(ii.shape, o[2] + (n2 - 0.5) * h[2])], axis=-1)
    u = top - rest  # [n1][n0][3]
    out = []
    for px, py in np.asarray(xy, dtype=np.float64).reshape(-1, 2):
        if not (o[0] <= px <= o[0] + cfg["block_size"][0] and o[1] <= py <= o[1] + cfg["block_size"][1]):
            raise ValueError("marker outside the top face")
        si = min(max((px - o[0]) / h[0] - 0.5, 0.0), n0 - 1.0)
        sj = min(max((py - o[1]) / h[1] - 0.5, 0.0), n1 - 1.0)
        i0 = min(int(np.floor(si)), n0 - 2)
        j0 = min(int(np.floor(sj)), n1 - 2)
        tx, ty = si - i0, sj - j0
        out.append((1 - tx) * (1 - ty) * u[j0, i0] + tx * (1 - ty) * u[j0, i0 + 1]
                   + (1 - tx) * ty * u[j0 + 1, i0] + tx * ty * u[j0 + 1, i0 + 1])
    return np.array(out)


def surface_displacement(cfg: dict, x, res: int, sub: int = 1):
    """[res][res][3] displacement of the top surface over a res x res
    partition of the top face: each cell the mean over sub x sub points at
    (c + (q + 1/2)/sub) * width / res of the bilinear interpolation of the
    top-layer particles' displacements x - X (x: [N][3] in lattice order
    i + n0 (j + n1 k), X the cell-centred rest lattice), each point clamped
    to the outermost particles."""
    n0, n1, n2 = cfg["n"]
    h = [cfg["block_size"][a] / cfg["n"][a] for a in range(3)]
    o = cfg["block_origin"]
    top = np.asarray(x, dtype=np.float64).reshape(n2, n1, n0, 3)[n2 - 1]
    ii, jj = np.meshgrid(np.arange(n0), np.arange(n1), indexing="xy")
    rest = np.stack([o[0] + (ii + 0.5) * h[0], o[1] + (jj + 0.5) * h[1],
                     np.full(ii.shape, o[2] + (n2 - 0.5) * h[2])], axis=-1)
    u = top - rest  # [n1][n0][3]
    out = np.zeros((res, res, 3))
    for r in range(res):
        for c in range(res):
            for qy in range(sub):
                for qx in range(sub):
                    si = min(max((c + (qx + 0.5) / sub) * n0 / res - 0.5, 0.0), n0 - 1.0)
                    sj = min(max((r + (qy + 0.5) / sub) * n1 / res - 0.5, 0.0), n1 - 1.0)
                    i0 = min(int(np.floor(si)), n0 - 2)
                    j0 = min(int(np.floor(sj)), n1 - 2)
                    tx, ty = si - i0, sj - j0
                    out[r, c] += ((1 - tx) * (1 - ty) * u[j0, i0] + tx * (1 - ty) * u[j0, i0 + 1]
                                  + (1 - tx) * ty * u[j0 + 1, i0] + tx * ty * u[j0 + 1, i0 + 1])
            out[r, c] /= sub * sub
    return out
