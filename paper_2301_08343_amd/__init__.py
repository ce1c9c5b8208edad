"""MI355X-native tactile elastomer simulator (explicit MLS-MPM, depth map, Phong render).

The compute path is libtacchi.so (HIP, gfx950) behind the C ABI of
include/tacchi.h; `Sim` is a thin binding over it.
"""
from . import workloads  # noqa: F401  (no GPU or library needed)

__all__ = ["workloads", "Sim"]


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    raise AttributeError(name)
