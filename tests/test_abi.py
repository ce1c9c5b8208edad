"""The C ABI library loads on the CPU, exports every entry point that
include/tacchi.h declares, and its host-side validation rejects bad
configurations (no device call is made by these)."""
import ctypes
import os
import re

import pytest

from paper_2301_08343_amd import native as N
from paper_2301_08343_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b((?:tacchi|tsg)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = N.lib()
    decl = declared_entry_points()
    assert "tacchi_create" in decl and "tacchi_step" in decl
    for name in decl:
        assert hasattr(L, name), name
    assert set(N.EXPORTS) <= set(decl)


def _bytes(cfg, pose0, **kw):
    c = N.make_config(cfg, pose0, **kw)
    return N.lib().tacchi_workspace_bytes(ctypes.byref(c)), N.lib().tacchi_last_error().decode()


def test_workspace_sizes():
    wl = W.small_sphere_contact()
    b64, _ = _bytes(wl["cfg"], wl["poses"][0], precision=N.F64)
    b32, _ = _bytes(wl["cfg"], wl["poses"][0], precision=N.F32)
    assert b64 > b32 > 0
    g = W.gelsight_contact(0)
    b, _ = _bytes(g["cfg"], g["poses"][0], precision=N.F32)
    # 1.6M particles in 208 x 208 x 48 tiled slots x 24 scalars, two bin lists of
    # 8192 blocks x 1280 entries, 8192 P2G tiles of 10^3 nodes and the
    # 4.2M-node velocity grid, 4 scalars per node
    assert 208 * 208 * 48 * 96 + 2 * 8192 * 1280 * 4 + 8192 * 1000 * 16 + 256 * 256 * 64 * 16 <= b < 6e8


@pytest.mark.parametrize("mutate,msg", [
    (lambda c: c.update(nu=0.5), "nu"),
    (lambda c: c.update(E=0.0), "E > 0"),
    (lambda c: c.update(block_origin=(1e-3, 4e-3, 1.5e-3)), "margin"),
    (lambda c: c.update(block_origin=(4e-3, 4e-3, 1.6e-3)), "node plane"),
    (lambda c: c.update(n_fixed_layers=0), "n_fixed_layers"),
    (lambda c: c.update(dx=0.4e-3, gn=(80, 80, 20)), "lattice spacing"),
    (lambda c: c.update(shape=9), "shape"),
    (lambda c: c.update(sp=(0.0,) * 8), "radius"),
    (lambda c: c.update(gn=(64, 64, 70000)), "65536"),
    (lambda c: c.update(gn=(1024, 1024, 1024)), "too many grid nodes"),
])
def test_config_validation(mutate, msg):
    wl = W.small_sphere_contact()
    cfg = dict(wl["cfg"])
    mutate(cfg)
    b, err = _bytes(cfg, wl["poses"][0])
    assert b == 0 and msg in err


def test_bad_tile_and_workspace_rejected():
    wl = W.small_sphere_contact()
    b, err = _bytes(wl["cfg"], wl["poses"][0], tile=5)
    assert b == 0 and "tile" in err
    c = N.make_config(wl["cfg"], wl["poses"][0])
    h = ctypes.c_void_p()
    st = N.lib().tacchi_create(ctypes.byref(c), None, 0, None, ctypes.byref(h))
    assert st == N.E_WORKSPACE and not h.value
    st = N.lib().tacchi_create(ctypes.byref(c), ctypes.c_void_p(0x1000 + 8), 1 << 30, None, ctypes.byref(h))
    assert st == N.E_WORKSPACE and "aligned" in N.lib().tacchi_last_error().decode()
    st = N.lib().tacchi_create(ctypes.byref(c), ctypes.c_void_p(0x1000), 16, None, ctypes.byref(h))
    assert st == N.E_WORKSPACE and "small" in N.lib().tacchi_last_error().decode()
