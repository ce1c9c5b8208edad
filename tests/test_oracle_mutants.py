"""Planted mistakes in the oracle: each one must fail a pin.

Every case below copies oracle.c (or the network's reference,
oracle/surrogate.py), plants one plausible mistake (a dropped term, a wrong
sign, constant or index, a transposed operand, an off-by-one boundary),
builds or loads the copy and runs the pin tests named for it against that
copy in a child process; the case passes when a pin fails.
This is what makes the pins a check of the oracle rather than of
themselves. CPU only; nothing here touches the HIP library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
SURROGATE_PY = os.path.join(ROOT, "oracle", "surrogate.py")
ORACLE_PY = os.path.join(ROOT, "oracle", "__init__.py")

# (name, text in oracle.c, replacement, pins expected to catch it (pytest -k))
MUTANTS = [
    ("bspline_centre_coefficient",
     "if (a < 0.5) return 0.75 - a * a;", "if (a < 0.5) return 0.75 - 0.5 * a * a;", "bspline_moments"),
    ("bspline_outer_square_dropped",
     "return 0.5 * (1.5 - a) * (1.5 - a);", "return 0.5 * (1.5 - a);", "bspline_moments"),
    ("stencil_base_off_by_half",
     "double b = floor(xi - 0.5);", "double b = floor(xi);", "p2g_mass_and_linear_momentum"),
    ("lattice_not_cell_centred",
     "(idx[a] + 0.5) * s->h[a];", "idx[a] * s->h[a];", "symmetric_press"),
    ("apic_affine_term_without_mass",
     "s->m * vp[r] + s->m * Cd", "s->m * vp[r] + Cd", "angular_momentum"),
    ("stress_term_sign",
     "double me = -dt * Dinv * wt", "double me = dt * Dinv * wt", "energy_gradient"),
    ("p2g_stress_scale_1_over_dx2",
     "Dinv = 4.0 / (dx * dx);\n    memset(s->M", "Dinv = 1.0 / (dx * dx);\n    memset(s->M", "energy_gradient"),
    ("g2p_velocity_gradient_scale_dropped",
     "Cn[k] = Dinv * B[k];", "Cn[k] = B[k];", "affine_field_reproduction"),
    ("g2p_velocity_gradient_transposed",
     "B[r * 3 + cc] += wt * Vq[r] * d[cc];", "B[cc * 3 + r] += wt * Vq[r] * d[cc];", "affine_field_reproduction"),
    ("deformation_update_order",
     "mat_mul(G, Fp, Fn);", "mat_mul(Fp, G, Fn);", "deformation_gradient_follows"),
    ("neo_hookean_volume_term",
     "(r == c ? lambda * lnJ : 0.0)", "(r == c ? lambda * (J - 1.0) : 0.0)", "textbook_energy"),
    ("corotated_missing_Ft",
     "mat_mul(D, Ft, DFt);", "memcpy(DFt, D, sizeof D);", "textbook_energy"),
    ("lame_lambda_denominator",
     "(1.0 - 2.0 * nu)", "(1.0 - nu)", "lame_parameters"),
    ("polar_reflection_not_removed",
     "if (mat_det(F) < 0.0) sig[kmin] = -sig[kmin];", "", "polar_decomposition"),
    ("gravity_dropped",
     "/ s->M[q] + dt * s->cfg.gravity[r];", "/ s->M[q];", "free_fall"),
    ("advection_with_old_velocity",
     "vp[r] = vn[r];\n            xp[r] = xp[r] + dt * vn[r];",
     "xp[r] = xp[r] + dt * vp[r];\n            vp[r] = vn[r];", "free_fall"),
    ("rigid_velocity_cross_sign",
     "om[1] * r[2] - om[2] * r[1];", "om[2] * r[1] - om[1] * r[2];", "rigid_motion_of_the_pose"),
    ("quaternion_matrix_sign",
     "R[1] = 2 * (x * y - w * z);", "R[1] = 2 * (x * y + w * z);", "rotated_sphere"),
    ("contact_force_sign",
     "s->force[r] += s->M[q] * (V[r] - after[r]) / dt;", "s->force[r] += s->M[q] * (after[r] - V[r]) / dt;",
     "run_until_force"),
    ("floor_off_by_one",
     "if (c <= s->cfg.floor_node)", "if (c < s->cfg.floor_node)", "walls_and_floor"),
    ("wall_keeps_outward_velocity",
     "if (idx[r] < wall && V[r] < 0.0)", "if (idx[r] < wall && V[r] > 0.0)", "walls_and_floor"),
    ("bonded_layers_off_by_one",
     "p / layer_size < s->cfg.n_fixed_layers", "p / layer_size <= s->cfg.n_fixed_layers", "free_fall"),
    ("coulomb_friction_sign",
     "1.0 + s->friction * un / tn", "1.0 - s->friction * un / tn", "friction_law"),
    ("particle_indenter_blend_mass",
     "/ (s->M[q] + s->MI[q]);", "/ s->M[q];", "particle_indenter"),
    ("heightmap_transposed",
     "H[(int64_t)j * n0 + i] = s->x[p * 3 + 2];", "H[(int64_t)i * n1 + j] = s->x[p * 3 + 2];", "heightmap_rows"),
    ("render_normal_sign",
     "double N[3] = {gx / nrm, gy / nrm, -1.0 / nrm};", "double N[3] = {-gx / nrm, -gy / nrm, -1.0 / nrm};",
     "render_plane"),
    ("render_central_difference_step",
     "/ (2.0 * r);\n            double gy", "/ r;\n            double gy", "render_plane"),
    ("contact_normal_sign",
     "g[k] = (phi_world(s, s->pose, a) - phi_world(s, s->pose, b)) / (2.0 * eps);",
     "g[k] = (phi_world(s, s->pose, b) - phi_world(s, s->pose, a)) / (2.0 * eps);", "does_not_pull"),
    ("coulomb_never_separates", "if (un >= 0.0) {", "if (un >= 1e300) {", "does_not_pull"),
    ("noise_cubic_fade",
     "double u = fx * fx * fx * (fx * (fx * 6.0 - 15.0) + 10.0);", "double u = fx * fx * (3.0 - 2.0 * fx);",
     "gradient_noise"),
    ("indenter_scatter_weight",
     "+= w[0][a] * w[1][b] * w[2][c] * s->imass;", "+= w[0][a] * w[1][b] * s->imass;", "placed_by_the_pose"),
    ("indenter_points_rotation_transposed",
     "X[r] = s->pose[r] + R[r * 3 + 0] * l[0] + R[r * 3 + 1] * l[1] + R[r * 3 + 2] * l[2];",
     "X[r] = s->pose[r] + R[0 * 3 + r] * l[0] + R[1 * 3 + r] * l[1] + R[2 * 3 + r] * l[2];", "placed_by_the_pose"),
    ("contact_at_end_pose",
     "} else if (s->cfg.shape >= 0 && phi_world(s, s->pose, X) <= 0.0) {",
     "} else if (s->cfg.shape >= 0 && phi_world(s, pose_end, X) <= 0.0) {", "start_pose"),
    ("empty_node_keeps_velocity",
     "                    V[0] = V[1] = V[2] = 0.0;\n                    continue;",
     "                    continue;", "empty_nodes"),
]


def _run_mutant(tmpdir: str, name: str, old: str, new: str, select: str):
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once in oracle.c"
    d = os.path.join(tmpdir, name)
    os.makedirs(d, exist_ok=True)
    c_path, so_path = os.path.join(d, "oracle.c"), os.path.join(d, "liboracle.so")
    with open(c_path, "w") as f:
        f.write(src.replace(old, new))
    # the copy includes oracle.h from the oracle's own folder
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
                           "-I", os.path.dirname(ORACLE_C), c_path, "-o", so_path, "-lm"])
    env = dict(os.environ, TACCHI_ORACLE_LIB=so_path, PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-m", "not gpu", "-k", select, "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    workers = min(8, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m), MUTANTS))
    survivors = [(name, out) for name, rc, out in results if rc != 1]
    # rc 1: tests ran and one failed; 0 would mean the mistake went unnoticed,
    # anything else that the selection or the build is broken
    assert not survivors, "planted mistakes not caught by the pins:\n" + "\n".join(
        f"{n}:\n{o}" for n, o in survivors)


@pytest.mark.parametrize("name,old,new,select", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutation_text_is_unique(name, old, new, select):
    assert open(ORACLE_C).read().count(old) == 1


# the network's reference: (name, text in surrogate.py, replacement, pins (pytest -k))
SURROGATE_MUTANTS = [
    ("tap_offsets_transposed", "(t // 3 - 1, t % 3 - 1)", "(t % 3 - 1, t // 3 - 1)", "conv_matches"),
    ("conv_shift_sign", "_shifted(x, dh, dw) @ w[:, t, :].T", "_shifted(x, -dh, -dw) @ w[:, t, :].T", "conv_matches"),
    ("dx_shift_sign", "dx += _shifted(gout @ w[:, t, :], -dh, -dw_)", "dx += _shifted(gout @ w[:, t, :], dh, dw_)",
     "conv_backward"),
    ("bias_grad_mean", "gout.sum(axis=(0, 1, 2))", "gout.mean(axis=(0, 1, 2))", "conv_backward"),
    ("gelu_grad_density_term", " + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)", "", "gelu_closed"),
    ("gelu_scale", "return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))", "return 0.5 * z * (1.0 + erf(z / 2.0))",
     "gelu_closed"),
    ("avgpool_backward_factor", "/ 4.0", "/ 2.0", "adjoint"),
    ("upsample_backward_mean", "g.reshape(n, H // 2, 2, W // 2, 2, c).sum(axis=(2, 4))",
     "g.reshape(n, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4))", "adjoint"),
    ("mse_gradient_factor", "2.0 * e / e.size", "e / e.size", "central_differences"),
    ("adamw_no_bias_correction", "mh = m / (1.0 - b1 ** step)", "mh = m", "adamw"),
    ("adamw_decay_dropped", "+ wd * p)", ")", "adamw"),
    ("adamw_eps_inside_sqrt", "(np.sqrt(vh) + eps)", "np.sqrt(vh + eps)", "adamw"),
    ("nearest_last_index_on_ties", "idx = np.argmin(d2, axis=1)",
     "idx = d2.shape[1] - 1 - np.argmin(d2[:, ::-1], axis=1)", "ties"),
    ("skip_concat_order", "np.concatenate([up, skips[l]], axis=-1)", "np.concatenate([skips[l], up], axis=-1)",
     "match_torch_autograd"),
    ("backward_split_swapped", "g_up, g_skip[l] = g[..., :c], g[..., c:]", "g_skip[l], g_up = g[..., :c], g[..., c:]",
     "central_differences"),
    ("pool_before_skip", "        skips.append(h)\n        h = S(avgpool2(h))",
     "        h = S(avgpool2(h))\n        skips.append(upsample2(h))", "match_torch_autograd"),
    ("he_init_std", "math.sqrt(2.0 / (ci * t))", "math.sqrt(1.0 / (ci * t))", "he_normal"),
    ("bf16_round_half_up", "(u + 0x7FFF + ((u >> 16) & 1))", "(u + 0x8000)", "bf16_rounding"),
    ("decoder_input_channels", '(f"dec{l}a", 2 * c, c, 9)', '(f"dec{l}a", c, c, 9)', "parameter_count"),
    ("contact_residual_side", "contact_residual * np.minimum(x[..., 0], 0.0)",
     "contact_residual * np.maximum(x[..., 0], 0.0)", "match_torch_autograd"),
]

# loads the mutated copy as oracle.surrogate before pytest imports the pins
_SURROGATE_DRIVER = """
import importlib.util, sys
sys.path.insert(0, sys.argv[1])
import oracle
spec = importlib.util.spec_from_file_location("oracle.surrogate", sys.argv[2])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle.surrogate"] = mod
spec.loader.exec_module(mod)
oracle.surrogate = mod
import pytest
sys.exit(pytest.main(sys.argv[3:]))
"""


def _run_surrogate_mutant(tmpdir: str, name: str, old: str, new: str, select: str):
    src = open(SURROGATE_PY).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once in surrogate.py"
    path = os.path.join(tmpdir, f"surrogate_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    r = subprocess.run([sys.executable, "-c", _SURROGATE_DRIVER, ROOT, path,
                        os.path.join(ROOT, "tests", "test_surrogate_oracle.py"), "-x", "-q", "-m", "not gpu",
                        "-k", select, "-p", "no:cacheprovider"],
                       cwd=ROOT, env=dict(os.environ, PYTHONDONTWRITEBYTECODE="1"),
                       capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_planted_mistake_in_the_network_reference_fails_a_pin(tmp_path):
    workers = min(6, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda m: _run_surrogate_mutant(str(tmp_path), *m), SURROGATE_MUTANTS))
    survivors = [(name, out) for name, rc, out in results if rc != 1]
    assert not survivors, "planted mistakes not caught by the pins:\n" + "\n".join(
        f"{n}:\n{o}" for n, o in survivors)


@pytest.mark.parametrize("name,old,new,select", SURROGATE_MUTANTS, ids=[m[0] for m in SURROGATE_MUTANTS])
def test_network_mutation_text_is_unique(name, old, new, select):
    assert open(SURROGATE_PY).read().count(old) == 1


# the oracle's Python side (depth-map resampling, markers, gap field):
# (name, text in oracle/__init__.py, replacement, pins (pytest -k))
PACKAGE_MUTANTS = [
    ("marker_rim_offset", "si = min(max((px - o[0]) / h[0] - 0.5, 0.0), n0 - 1.0)",
     "si = min(max((px - o[0]) / h[0], 0.0), n0 - 1.0)", "markers_reproduce"),
    ("marker_bilinear_corner", "out.append((1 - tx) * (1 - ty) * u[j0, i0] + tx * (1 - ty) * u[j0, i0 + 1]",
     "out.append((1 - tx) * (1 - ty) * u[j0, i0] + tx * (1 - ty) * u[j0 + 1, i0]", "markers_reproduce"),
    ("displacement_mean_divisor", "out[r, c] /= sub * sub", "out[r, c] /= sub", "surface_displacement"),
    ("displacement_subpoint_offset", "si = min(max((c + (qx + 0.5) / sub) * n0 / res - 0.5, 0.0), n0 - 1.0)",
     "si = min(max((c + qx / sub) * n0 / res - 0.5, 0.0), n0 - 1.0)", "surface_displacement"),
    ("gap_subpoints_ignored", "x = ox + (c + (qx + 0.5) / sub) * wx / res",
     "x = ox + (c + 0.5) * wx / res", "upright_sphere"),
    ("gap_upper_clamp_dropped", "acc += min(max(z - ztop, lo), hi)", "acc += max(z - ztop, lo)",
     "upright_sphere"),
    ("force_limit_strict", "if self.force()[2] >= fz_limit:", "if self.force()[2] > fz_limit:",
     "run_until_force"),
]

# loads the mutated copy as the oracle package (its C library as built)
_PACKAGE_DRIVER = """
import importlib.util, os, sys
sys.path.insert(0, sys.argv[1])
spec = importlib.util.spec_from_file_location("oracle", sys.argv[2],
                                              submodule_search_locations=[os.path.join(sys.argv[1], "oracle")])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle"] = mod
spec.loader.exec_module(mod)
import pytest
sys.exit(pytest.main(sys.argv[3:]))
"""


def _run_package_mutant(tmpdir: str, name: str, old: str, new: str, select: str):
    src = open(ORACLE_PY).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once in oracle/__init__.py"
    path = os.path.join(tmpdir, f"oracle_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    import oracle
    lib = oracle.build(force=False)
    r = subprocess.run([sys.executable, "-c", _PACKAGE_DRIVER, ROOT, path,
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x", "-q", "-m", "not gpu",
                        "-k", select, "-p", "no:cacheprovider"],
                       cwd=ROOT, env=dict(os.environ, PYTHONDONTWRITEBYTECODE="1", TACCHI_ORACLE_LIB=lib),
                       capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_every_planted_mistake_in_the_oracle_package_fails_a_pin(tmp_path):
    with cf.ThreadPoolExecutor(min(6, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda m: _run_package_mutant(str(tmp_path), *m), PACKAGE_MUTANTS))
    survivors = [(name, out) for name, rc, out in results if rc != 1]
    assert not survivors, "planted mistakes not caught by the pins:\n" + "\n".join(
        f"{n}:\n{o}" for n, o in survivors)


@pytest.mark.parametrize("name,old,new,select", PACKAGE_MUTANTS, ids=[m[0] for m in PACKAGE_MUTANTS])
def test_package_mutation_text_is_unique(name, old, new, select):
    assert open(ORACLE_PY).read().count(old) == 1
