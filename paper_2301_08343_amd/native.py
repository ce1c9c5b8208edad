"""ctypes binding of libtacchi.so (argument marshalling only).

Every step of the simulation runs in the HIP library; this module only turns
Python values into the C structs of include/tacchi.h, hands over device
pointers of torch tensors and the current HIP stream, and raises on error
statuses. It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtacchi.so")

OK, E_ARG, E_WORKSPACE, E_DEVICE, E_UNSTABLE, E_OUT_OF_GRID, E_STATE = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_WORKSPACE", -3: "E_DEVICE", -4: "E_UNSTABLE",
                -5: "E_OUT_OF_GRID", -6: "E_STATE"}

# every entry point declared in include/tacchi.h
EXPORTS = (
    "tacchi_workspace_bytes", "tacchi_create", "tacchi_step", "tacchi_run", "tacchi_p2g",
    "tacchi_grid_update", "tacchi_g2p", "tacchi_read_grid", "tacchi_heightmap", "tacchi_render",
    "tacchi_read_particles", "tacchi_write_particles", "tacchi_indenter_force", "tacchi_get_pose",
    "tacchi_num_particles", "tacchi_sync", "tacchi_destroy", "tacchi_last_error",
    "tacchi_timing_enable", "tacchi_timing_read", "tacchi_polar_fallbacks",
    "tacchi_batch_workspace_bytes", "tacchi_batch_create", "tacchi_batch_run", "tacchi_batch_contact",
    "tacchi_batch_tuning", "tacchi_batch_substeps_done", "tacchi_batch_sync", "tacchi_batch_destroy",
    "tacchi_surface_displacement", "tacchi_indenter_gap", "tacchi_batch_surface_displacement", "tacchi_markers",
    "tacchi_run_until_force", "tacchi_set_contact", "tacchi_set_indenter_points",
    "tacchi_points_workspace_bytes", "tacchi_indenter_gap_workspace_bytes",
    "tacchi_indenter_gap_noalloc", "tacchi_indenter_gap_noalloc_max", "tacchi_batch_tuning_check",
)
NUM_KERNEL_CLASSES = 6
KERNEL_CLASSES = ("bin", "p2g", "grid", "g2p", "heightmap", "render")


class TacchiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Block(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("size", ctypes.c_double * 3), ("n", ctypes.c_int32 * 3)]


class Grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("dx", ctypes.c_double), ("n", ctypes.c_int32 * 3)]


class Material(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double), ("rho", ctypes.c_double),
                ("model", ctypes.c_int32)]


class Indenter(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("p", ctypes.c_double * 8), ("seed", ctypes.c_uint64)]


class Pose(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("quat", ctypes.c_double * 4)]


class Config(ctypes.Structure):
    _fields_ = [("block", Block), ("grid", Grid), ("mat", Material), ("ind", Indenter),
                ("pose0", Pose), ("gravity", ctypes.c_double * 3), ("n_fixed_layers", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tile", ctypes.c_int32)]


class RenderParams(ctypes.Structure):
    _fields_ = [("ka_ia", ctypes.c_double), ("kd", ctypes.c_double), ("ks", ctypes.c_double),
                ("alpha", ctypes.c_double), ("light_elev_deg", ctypes.c_double),
                ("light_azim_deg", ctypes.c_double * 3), ("pitch", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        L.tacchi_workspace_bytes.restype = ctypes.c_size_t
        L.tacchi_workspace_bytes.argtypes = [ctypes.POINTER(Config)]
        L.tacchi_create.restype = ctypes.c_int32
        L.tacchi_create.argtypes = [ctypes.POINTER(Config), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.tacchi_step.restype = ctypes.c_int32
        L.tacchi_step.argtypes = [_vp, ctypes.POINTER(Pose), ctypes.c_double]
        L.tacchi_run.restype = ctypes.c_int32
        L.tacchi_run.argtypes = [_vp, ctypes.POINTER(Pose), ctypes.c_int32, ctypes.c_double]
        L.tacchi_p2g.restype = ctypes.c_int32
        L.tacchi_p2g.argtypes = [_vp, ctypes.c_double]
        L.tacchi_grid_update.restype = ctypes.c_int32
        L.tacchi_grid_update.argtypes = [_vp, ctypes.POINTER(Pose), ctypes.c_double]
        L.tacchi_g2p.restype = ctypes.c_int32
        L.tacchi_g2p.argtypes = [_vp, ctypes.c_double]
        L.tacchi_read_grid.restype = ctypes.c_int32
        L.tacchi_read_grid.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32]
        L.tacchi_heightmap.restype = ctypes.c_int32
        L.tacchi_heightmap.argtypes = [_vp, _vp, ctypes.c_int32]
        L.tacchi_render.restype = ctypes.c_int32
        L.tacchi_render.argtypes = [_vp, ctypes.POINTER(RenderParams), _vp, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32]
        L.tacchi_read_particles.restype = ctypes.c_int32
        L.tacchi_read_particles.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32]
        L.tacchi_write_particles.restype = ctypes.c_int32
        L.tacchi_write_particles.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32]
        L.tacchi_indenter_force.restype = ctypes.c_int32
        L.tacchi_indenter_force.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
        L.tacchi_get_pose.restype = ctypes.c_int32
        L.tacchi_get_pose.argtypes = [_vp, ctypes.POINTER(Pose)]
        L.tacchi_num_particles.restype = ctypes.c_int64
        L.tacchi_num_particles.argtypes = [_vp]
        L.tacchi_sync.restype = ctypes.c_int32
        L.tacchi_sync.argtypes = [_vp]
        L.tacchi_destroy.restype = None
        L.tacchi_destroy.argtypes = [_vp]
        L.tacchi_timing_enable.restype = ctypes.c_int32
        L.tacchi_timing_enable.argtypes = [_vp, ctypes.c_uint32]
        L.tacchi_timing_read.restype = ctypes.c_int32
        L.tacchi_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.c_int32]
        L.tacchi_polar_fallbacks.restype = ctypes.c_int32
        L.tacchi_polar_fallbacks.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint64)]
        L.tacchi_batch_workspace_bytes.restype = ctypes.c_size_t
        L.tacchi_batch_workspace_bytes.argtypes = [ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_int32]
        L.tacchi_batch_create.restype = ctypes.c_int32
        L.tacchi_batch_create.argtypes = [ctypes.POINTER(Config), ctypes.c_int32, ctypes.POINTER(Pose),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_char_p,
                                          ctypes.c_int32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
        L.tacchi_batch_run.restype = ctypes.c_int32
        L.tacchi_batch_run.argtypes = [_vp, ctypes.c_int32]
        L.tacchi_batch_contact.restype = _vp
        L.tacchi_batch_contact.argtypes = [_vp, ctypes.c_int32]
        L.tacchi_batch_tuning.restype = ctypes.c_int32
        L.tacchi_batch_tuning.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
        L.tacchi_batch_tuning_check.restype = ctypes.c_int32
        L.tacchi_batch_tuning_check.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.tacchi_batch_substeps_done.restype = ctypes.c_int64
        L.tacchi_batch_substeps_done.argtypes = [_vp]
        L.tacchi_batch_sync.restype = ctypes.c_int32
        L.tacchi_batch_sync.argtypes = [_vp]
        L.tacchi_batch_destroy.restype = None
        L.tacchi_batch_destroy.argtypes = [_vp]
        L.tacchi_surface_displacement.restype = ctypes.c_int32
        L.tacchi_surface_displacement.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32]
        L.tacchi_set_indenter_points.restype = ctypes.c_int32
        L.tacchi_set_indenter_points.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                                 ctypes.c_double, _vp, ctypes.c_size_t]
        L.tacchi_points_workspace_bytes.restype = ctypes.c_size_t
        L.tacchi_points_workspace_bytes.argtypes = [_vp, ctypes.c_int32]
        L.tacchi_indenter_gap_workspace_bytes.restype = ctypes.c_size_t
        L.tacchi_indenter_gap_workspace_bytes.argtypes = [ctypes.c_int32]
        L.tacchi_indenter_gap_noalloc_max.restype = ctypes.c_int32
        L.tacchi_indenter_gap_noalloc_max.argtypes = []
        L.tacchi_indenter_gap_noalloc.restype = ctypes.c_int32
        L.tacchi_indenter_gap_noalloc.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(Pose), ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                  _vp, _vp]
        L.tacchi_set_contact.restype = ctypes.c_int32
        L.tacchi_set_contact.argtypes = [_vp, ctypes.c_int32, ctypes.c_double]
        L.tacchi_run_until_force.restype = ctypes.c_int32
        L.tacchi_run_until_force.argtypes = [_vp, ctypes.POINTER(Pose), ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]
        L.tacchi_markers.restype = ctypes.c_int32
        L.tacchi_markers.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _vp, ctypes.c_int32]
        L.tacchi_indenter_gap.restype = ctypes.c_int32
        L.tacchi_indenter_gap.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(Pose), ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _vp,
                                          _vp, ctypes.c_size_t, _vp]
        L.tacchi_batch_surface_displacement.restype = ctypes.c_int32
        L.tacchi_batch_surface_displacement.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32]
        L.tacchi_last_error.restype = ctypes.c_char_p
        L.tacchi_last_error.argtypes = []
        _lib = L
    return _lib


# every entry point declared in include/tsg.h, with its argument types
_i32, _i64, _sz, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
_TSG_SIGS = {
    "tsg_pack_k": (_i32, [_i32, _i32]),
    "tsg_pack_weights": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp]),
    "tsg_conv": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _i32, _i32, _i32, _vp, _i32, _i32,
                        _vp, _i32, _i32, _vp, _vp]),
    "tsg_wgrad_scratch_bytes": (_sz, [_i32, _i32, _i32, _i32, _i32, _i32]),
    "tsg_conv_wgrad": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _vp,
                              _vp, _vp, _sz, _vp]),
    "tsg_head_scratch_bytes": (_sz, [_i32, _i32]),
    "tsg_conv_wgrad_f32": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _sz,
                                  _vp]),
    "tsg_head_dgrad": (_i32, [_vp, _i32, _i32, _vp, _i32, _vp, _i32, _i32, _vp, _i32, _i32, _vp]),
    "tsg_avgpool2": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp]),
    "tsg_avgpool2_bwd": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _vp]),
    "tsg_upsample2": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp]),
    "tsg_upsample2_bwd": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp]),
    "tsg_avgpool2_bwd_dgelu": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _i32, _vp, _i32, _i32,
                                      _vp]),
    "tsg_upsample2_bwd_dgelu": (_i32, [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _i32,
                                       _vp]),
    "tsg_add_inplace": (_i32, [_vp, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _vp]),
    "tsg_dgelu": (_i32, [_vp, _i32, _i32, _vp, _i32, _i32, _i32, _i32, _vp]),
    "tsg_mse": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp, _vp]),
    "tsg_adamw": (_i32, [_vp, _vp, _vp, _vp, _i64, _f32, _f32, _f32, _f32, _f32, _i32, _vp]),
    "tsg_to_bf16": (_i32, [_vp, _i32, _i32, _vp, _i32, _vp]),
    "tsg_nn_dist": (_i32, [_vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp]),
    "tsg_features": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, _f32, _vp, _vp]),
    "tsg_channel_mse": (_i32, [_vp, _vp, _i32, _i32, _i32, _i32, _vp, _vp]),
    "tsg_augment": (_i32, [_vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp]),
    "tsg_contact_residual": (_i32, [_vp, _vp, _i64, _f32, _vp]),
    "tsg_last_error": (ctypes.c_char_p, []),
}
TSG_EXPORTS = tuple(_TSG_SIGS)
_tsg = None


class TsgError(RuntimeError):
    pass


def tsg():
    """The library with the surrogate kernels' argument types set."""
    global _tsg
    if _tsg is None:
        L = lib()
        for name, (res, args) in _TSG_SIGS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _tsg = L
    return _tsg


def tsg_call(name: str, *args):
    """Call a tsg_* entry point and raise on a non-zero status."""
    st = getattr(tsg(), name)(*args)
    if st != 0:
        raise TsgError(f"{name}: {tsg().tsg_last_error().decode()} (status {st})")


def check(status: int):
    if status != OK:
        raise TacchiError(status, lib().tacchi_last_error().decode())


def make_pose(p) -> Pose:
    out = Pose()
    out.pos[:] = [float(v) for v in p[:3]]
    out.quat[:] = [float(v) for v in p[3:7]]
    return out


def make_poses(poses):
    arr = (Pose * len(poses))()
    for k, p in enumerate(poses):
        arr[k].pos[:] = [float(v) for v in p[:3]]
        arr[k].quat[:] = [float(v) for v in p[3:7]]
    return arr


def make_config(cfg: dict, pose0, precision: int = F64, tile: int = 0) -> Config:
    c = Config()
    c.block.origin[:] = cfg["block_origin"]
    c.block.size[:] = cfg["block_size"]
    c.block.n[:] = cfg["n"]
    c.grid.origin[:] = cfg["grid_origin"]
    c.grid.dx = cfg["dx"]
    c.grid.n[:] = cfg["gn"]
    c.mat.E, c.mat.nu, c.mat.rho, c.mat.model = cfg["E"], cfg["nu"], cfg["rho"], cfg["model"]
    c.ind.shape = cfg["shape"]
    c.ind.p[:] = cfg["sp"]
    c.ind.seed = cfg["seed"]
    c.pose0 = make_pose(pose0)
    c.gravity[:] = cfg["gravity"]
    c.n_fixed_layers = cfg["n_fixed_layers"]
    c.precision = precision
    c.tile = tile
    return c


def make_render(rp: dict) -> RenderParams:
    r = RenderParams()
    r.ka_ia, r.kd, r.ks, r.alpha = rp["ka_ia"], rp["kd"], rp["ks"], rp["alpha"]
    r.light_elev_deg = rp["light_elev_deg"]
    r.light_azim_deg[:] = rp["light_azim_deg"]
    r.pitch = rp["pitch"]
    return r
