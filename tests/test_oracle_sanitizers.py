"""The C oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer.

A child process loads an instrumented build of oracle.c (the sanitizer
runtime preloaded, halting at the first report) and runs the oracle's pins
against it; the five long pins (Hertz, friction, force-terminated press,
particle indenter: minutes under instrumentation) are replaced by short runs
of the same code paths. CPU only: the HIP library is not involved.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")

LONG_PINS = "hertz or coulomb or run_until_force or test_particle_indenter"

SHORT_RUNS = r"""
import numpy as np
import oracle
from paper_2301_08343_amd import workloads as W
wl = W.small_sphere_contact(seed=1, steps=1000)
poses, dt = wl["poses"].copy(), wl["dt"]
poses[:, 2] -= 0.4e-3  # start in contact
# Coulomb contact, sliding
s = oracle.OracleSim(wl["cfg"], poses[0])
s.set_contact(1, 0.3)
slide = poses.copy()
slide[:, 0] += np.linspace(0.0, 0.2e-3, len(slide))
s.run(slide, dt, 0, 15)
# the indenter as points
s = oracle.OracleSim(wl["cfg"], poses[0])
m = wl["cfg"]["rho"] * (wl["cfg"]["block_size"][0] / wl["cfg"]["n"][0]) ** 3
s.set_indenter_points(W.sphere_points(wl["cfg"]["sp"][0], 3000, 0.5e-3, 0), 10 * m)
s.run(poses, dt, 0, 15)
assert s.indenter_mass().sum() > 0
# force-terminated press
s = oracle.OracleSim(wl["cfg"], poses[0])
n = s.run_until_force(poses, dt, 1e-4, 0, 30)
assert 1 <= n <= 30
print("short runs ok", n)
"""


def _runtime(lib: str) -> str | None:
    p = subprocess.run(["gcc", f"-print-file-name={lib}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_oracle_pins_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                           "-I", ORACLE_DIR, os.path.join(ORACLE_DIR, "oracle.c"), "-o", so, "-lm"])
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, TACCHI_ORACLE_LIB=so, PYTHONDONTWRITEBYTECODE="1",
               LD_PRELOAD=asan + (" " + pre if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x",
                        "-q", "-m", "not gpu", "-k", f"not ({LONG_PINS})", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout
    r = subprocess.run([sys.executable, "-c", SHORT_RUNS], cwd=ROOT, env=dict(env, PYTHONPATH=ROOT),
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "short runs ok" in r.stdout
