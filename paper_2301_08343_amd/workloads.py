"""Seeded synthetic contact workloads for the tactile MLS-MPM path.

This module holds no simulation arithmetic. It only draws what defines a
contact -- elastomer block and particle lattice, background grid, material,
indenter family and parameters, the indenter pose trajectory, time step -- from
a counter-based generator, and returns plain Python/numpy values. The CPU
oracle and the HIP library each marshal these values into their own structs.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), written from its published definition.

Shapes and sizes follow the paper's workload (Sec. IV-B: a 20 x 20 x 4 mm
GelSight elastomer, E = 1.45e5, nu = 0.45; Sec. IV-A: indentation depths up to
about 1 mm) with the project's synthetic analytic indenters standing in for the
3D-printed indenter set, which is not available.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1

# indenter families (shape codes shared by both C ABIs)
SPHERE, CYLINDER, CONE, EDGE, TEXTURED_PLATE = 0, 1, 2, 3, 4
NO_INDENTER = -1
SHAPE_NAMES = {SPHERE: "sphere", CYLINDER: "cylinder", CONE: "cone", EDGE: "edge",
               TEXTURED_PLATE: "textured_plate", NO_INDENTER: "none"}

NEOHOOKEAN, COROTATED = 0, 1


class SplitMix64:
    """SplitMix64 stream: state advances by the golden-ratio increment and each
    output is the state passed through the two xor-shift-multiply rounds."""

    GAMMA = 0x9E3779B97F4A7C15

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + self.GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        """53-bit uniform double in [lo, hi)."""
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / 9007199254740992.0))

    def randint(self, n: int) -> int:
        return self.next_u64() % n


def quat_axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    s = math.sin(0.5 * angle)
    return np.array([math.cos(0.5 * angle), axis[0] * s, axis[1] * s, axis[2] * s])


IDENTITY_QUAT = np.array([1.0, 0.0, 0.0, 0.0])


def default_render(pitch: float, h: int, w: int) -> dict:
    """Project-chosen Phong constants (the sensor's own constants are not
    available): ambient 0.1, diffuse 0.6, specular 0.2, shininess 8, three
    distant lights (red, green, blue) at azimuth 0/120/240 degrees and 30 degrees
    elevation on the camera side."""
    return dict(ka_ia=0.1, kd=0.6, ks=0.2, alpha=8.0, light_elev_deg=30.0,
                light_azim_deg=(0.0, 120.0, 240.0), pitch=pitch, h=h, w=w)


def _contact(block_origin, block_size, n, grid_origin, dx, gn, E, nu, rho, model,
             shape, sp, seed, n_fixed_layers=1, gravity=(0.0, 0.0, 0.0)):
    return dict(block_origin=tuple(float(v) for v in block_origin),
                block_size=tuple(float(v) for v in block_size),
                n=tuple(int(v) for v in n),
                grid_origin=tuple(float(v) for v in grid_origin), dx=float(dx),
                gn=tuple(int(v) for v in gn),
                E=float(E), nu=float(nu), rho=float(rho), model=int(model),
                shape=int(shape), sp=tuple(float(v) for v in sp) + (0.0,) * (8 - len(sp)),
                seed=int(seed) & MASK64, gravity=tuple(float(v) for v in gravity),
                n_fixed_layers=int(n_fixed_layers),
                floor_node=int(round((block_origin[2] - grid_origin[2]) / dx)),
                wall_nodes=3)


def top_z(cfg) -> float:
    return cfg["block_origin"][2] + cfg["block_size"][2]


def block_center_xy(cfg):
    return (cfg["block_origin"][0] + 0.5 * cfg["block_size"][0],
            cfg["block_origin"][1] + 0.5 * cfg["block_size"][1])


def press_trajectory(start_pos, quat, depth, steps):
    """Indenter tip moving straight down at constant speed from `start_pos`
    (tip touching the top face) to `depth` below it; returns [steps+1][7] poses
    (x, y, z, qw, qx, qy, qz)."""
    poses = np.zeros((steps + 1, 7))
    k = np.arange(steps + 1, dtype=np.float64)
    poses[:, 0] = start_pos[0]
    poses[:, 1] = start_pos[1]
    poses[:, 2] = start_pos[2] - depth * k / steps
    poses[:, 3:] = quat
    return poses


def draw_indenter(rng: SplitMix64, family: int):
    """Indenter parameters per family, in the indenter frame whose origin is the
    lowest point of the shape (tip) and whose +z points away from the gel.

    sphere: sp = (R,)            R in [2, 5] mm
    cylinder (flat punch): (r,)  r in [1, 4] mm
    cone: (half_angle, tip_r)    half-angle in [30, 60] deg, tip radius 0.2 mm
    edge (90-degree wedge along the indenter y axis): (pi/4, 0.2 mm)
    textured plate: (half_width, amplitude, wavelength): square punch of
        half-width in [3, 6] mm whose bottom face carries 50 um gradient noise
        of 1 mm wavelength.
    """
    if family == SPHERE:
        return [rng.uniform(2e-3, 5e-3)]
    if family == CYLINDER:
        return [rng.uniform(1e-3, 4e-3)]
    if family == CONE:
        return [math.radians(rng.uniform(30.0, 60.0)), 0.2e-3]
    if family == EDGE:
        return [math.pi / 4, 0.2e-3]
    if family == TEXTURED_PLATE:
        return [rng.uniform(3e-3, 6e-3), 50e-6, 1e-3]
    raise ValueError(family)


def small_sphere_contact(seed: int = 0, steps: int = 1000, jitter: bool = True):
    """The 18,432-particle FP64 parity workload: 24 x 24 x 4 mm block as a
    48 x 48 x 8 lattice (0.5 mm), grid 64 x 64 x 16 at 0.5 mm, neo-Hookean
    E = 0.15 MPa, nu = 0.45, rho = 1000, bottom layer fixed, dt = 1e-5 s, sphere
    R = 3 mm with xy jitter of +-3 mm pressed 0.5 mm at 50 mm/s over 1000 steps.
    Outputs a 48 x 48 height map and a 96 x 96 image at 0.25 mm pitch."""
    rng = SplitMix64(0x5AC0 + seed)
    dx = 0.5e-3
    cfg = _contact(block_origin=(4e-3, 4e-3, 1.5e-3), block_size=(24e-3, 24e-3, 4e-3),
                   n=(48, 48, 8), grid_origin=(0.0, 0.0, 0.0), dx=dx, gn=(64, 64, 16),
                   E=0.15e6, nu=0.45, rho=1000.0, model=NEOHOOKEAN,
                   shape=SPHERE, sp=[3e-3], seed=seed)
    cx, cy = block_center_xy(cfg)
    if jitter:
        cx += rng.uniform(-3e-3, 3e-3)
        cy += rng.uniform(-3e-3, 3e-3)
    dt = 1e-5
    depth = 0.05 * steps * dt  # 50 mm/s
    poses = press_trajectory((cx, cy, top_z(cfg)), IDENTITY_QUAT, depth, steps)
    return dict(name="sphere_18k_fp64", cfg=cfg, dt=dt, steps=steps, poses=poses,
                render=default_render(0.25e-3, 96, 96))


def sphere_points(radius: float, n: int, shell: float, seed: int = 0):
    """Point cloud of a sphere indenter for the particle-represented indenter
    (Sec. IV-B: objects enter as point clouds): n points uniform in the
    spherical shell of the given thickness under the surface, in the indenter
    frame (origin at the lowest point, +z up, centre at (0, 0, radius))."""
    rng = np.random.default_rng(0x5EED + seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r_in = max(radius - shell, 0.0)
    r = (r_in ** 3 + rng.uniform(0.0, 1.0, n) * (radius ** 3 - r_in ** 3)) ** (1.0 / 3.0)
    return d * r[:, None] + np.array([0.0, 0.0, radius])


def slide_contact(radius: float = 3e-3, depth: float = 0.3e-3, slide=(2e-3, 0.0), steps_press: int = 300,
                  steps_slide: int = 600, retract: int = 0, seed: int = 0):
    """Sliding over the 18,432-particle block of small_sphere_contact (no
    jitter): a sphere of the given radius pressed `depth` into the top face
    over steps_press substeps, then moved by `slide` (x, y) at that depth over
    steps_slide substeps, then (retract > 0) lifted back to its starting
    height over `retract` substeps. dt = 1e-5 s."""
    cfg = _contact(block_origin=(4e-3, 4e-3, 1.5e-3), block_size=(24e-3, 24e-3, 4e-3),
                   n=(48, 48, 8), grid_origin=(0.0, 0.0, 0.0), dx=0.5e-3, gn=(64, 64, 16),
                   E=0.15e6, nu=0.45, rho=1000.0, model=NEOHOOKEAN,
                   shape=SPHERE, sp=[radius], seed=seed)
    cx, cy = block_center_xy(cfg)
    cx -= 0.5 * slide[0]
    cy -= 0.5 * slide[1]
    z0 = top_z(cfg)
    poses = [press_trajectory((cx, cy, z0), IDENTITY_QUAT, depth, steps_press)]
    t = np.arange(1, steps_slide + 1, dtype=np.float64) / steps_slide
    sl = np.zeros((steps_slide, 7))
    sl[:, 0] = cx + slide[0] * t
    sl[:, 1] = cy + slide[1] * t
    sl[:, 2] = z0 - depth
    sl[:, 3:] = IDENTITY_QUAT
    poses.append(sl)
    if retract > 0:
        r = np.zeros((retract, 7))
        u = np.arange(1, retract + 1, dtype=np.float64) / retract
        r[:, 0] = cx + slide[0]
        r[:, 1] = cy + slide[1]
        r[:, 2] = z0 - depth * (1.0 - u)
        r[:, 3:] = IDENTITY_QUAT
        poses.append(r)
    poses = np.concatenate(poses)
    return dict(name="slide_18k", cfg=cfg, dt=1e-5, steps=len(poses) - 1, poses=poses,
                render=default_render(0.25e-3, 96, 96))


def gelsight_contact(seed: int = 0, steps: int = 2000, scale: int = 1):
    """The 1.6M-particle GelSight-sized workload: 20 x 20 x 4 mm block as a
    200 x 200 x 40 lattice (0.1 mm), grid 256 x 256 x 64 at 0.1 mm, neo-Hookean
    E = 0.15 MPa, nu = 0.45, dt = 2e-6 s; indenter family = seed mod 5 with
    xy jitter +-3 mm; depth uniform in [0.2, 1.5] mm reached over `steps`
    substeps; 200 x 200 height map, 480 x 640 image (31.25 um pitch).

    `scale` > 1 shrinks the block and grid laterally by that factor at the same
    spacing (a down-scaled block for oracle parity)."""
    rng = SplitMix64(0x6E15 + seed)
    dx = 0.1e-3
    family = seed % 5
    sp = draw_indenter(rng, family)
    nxy = 200 // scale
    gxy = 256 // scale if scale > 1 else 256
    if scale > 1:
        gxy = nxy + 2 * 14
    origin_xy = 0.5 * (gxy - 1) * dx - 0.5 * nxy * dx
    origin_xy = round(origin_xy / dx) * dx
    cfg = _contact(block_origin=(origin_xy, origin_xy, 0.3e-3),
                   block_size=(nxy * dx, nxy * dx, 4e-3), n=(nxy, nxy, 40),
                   grid_origin=(0.0, 0.0, 0.0), dx=dx, gn=(gxy, gxy, 64),
                   E=0.15e6, nu=0.45, rho=1000.0, model=NEOHOOKEAN,
                   shape=family, sp=sp, seed=seed)
    cx, cy = block_center_xy(cfg)
    jit = 3e-3 / scale
    cx += rng.uniform(-jit, jit)
    cy += rng.uniform(-jit, jit)
    depth = rng.uniform(0.2e-3, 1.5e-3)
    dt = 2e-6
    poses = press_trajectory((cx, cy, top_z(cfg)), IDENTITY_QUAT, depth, steps)
    h, w = (480, 640) if scale == 1 else (max(8, 480 // scale), max(8, 640 // scale))
    return dict(name=f"gelsight_{SHAPE_NAMES[family]}", cfg=cfg, dt=dt, steps=steps,
                poses=poses, depth=depth,
                render=default_render(nxy * dx / w, h, w))


def gelsight_contact_at(seed: int, h: float = 0.2e-3, full: bool = True):
    """The GelSight-sized contact of `seed` (the same indenter, position and
    depth draws as gelsight_contact) on a lattice of spacing h with grid
    spacing h: the 20 x 20 x 4 mm block in a 25.6 x 25.6 x 6.4 mm grid (at
    least 9 nodes taller than the block), bottom face 3 nodes above the grid
    floor, 2000 (0.1 mm / h) substeps of
    dt = 4 ms / substeps, so the press lasts 4 ms as at 0.1 mm. With
    full=False the trajectory is left out (poses = None); `end_pose` is the
    final pose either way."""
    rng = SplitMix64(0x6E15 + seed)
    family = seed % 5
    sp = draw_indenter(rng, family)
    nxy = int(round(20e-3 / h))
    nz = int(round(4e-3 / h))
    gxy = int(round(25.6e-3 / h))
    gz = max(int(round(6.4e-3 / h)), nz + 9)
    origin_xy = round((0.5 * (gxy - 1) * h - 0.5 * nxy * h) / h) * h
    cfg = _contact(block_origin=(origin_xy, origin_xy, 3 * h),
                   block_size=(nxy * h, nxy * h, nz * h), n=(nxy, nxy, nz),
                   grid_origin=(0.0, 0.0, 0.0), dx=h, gn=(gxy, gxy, gz),
                   E=0.15e6, nu=0.45, rho=1000.0, model=NEOHOOKEAN,
                   shape=family, sp=sp, seed=seed)
    cx, cy = block_center_xy(cfg)
    cx += rng.uniform(-3e-3, 3e-3)
    cy += rng.uniform(-3e-3, 3e-3)
    depth = rng.uniform(0.2e-3, 1.5e-3)
    steps = int(round(2000 * 0.1e-3 / h))
    dt = 4e-3 / steps
    start = (cx, cy, top_z(cfg))
    poses = press_trajectory(start, IDENTITY_QUAT, depth, steps) if full else None
    end = np.array([cx, cy, start[2] - depth * float(steps) / steps, *IDENTITY_QUAT])
    return dict(name=f"gelsight_{SHAPE_NAMES[family]}_h{h * 1e3:.2f}mm", cfg=cfg, dt=dt, steps=steps,
                poses=poses, end_pose=end, depth=depth, particles=nxy * nxy * nz, seed=seed, h=h)


def batch_contact(seed: int, steps: int = 2000, max_lateral: int = 0):
    """One contact of the uneven batch: particle count log-uniform in
    [2e4, 4e5]; block side L ~ U[10, 20] mm, thickness T ~ U[3, 5] mm,
    spacing h = (L^2 T / N)^(1/3) (redrawn until h is in [0.1, 0.3] mm);
    E ~ U[0.1, 0.3] MPa, nu ~ U[0.40, 0.48]; fixed-corotated material;
    indenter family and depth as in the GelSight workload plus a tilt of up to
    5 degrees about a random horizontal axis; dt = 0.45 dx / c_p.

    max_lateral > 0 keeps every draw (h, thickness, material, indenter, tilt,
    depth, time step) but cuts the block to at most that many particles per
    lateral axis, with the grid margin and xy jitter sized to the cut block:
    the same contact at a size a single-core solver finishes quickly."""
    rng = SplitMix64(0xBA7C + seed)
    while True:
        N = math.exp(rng.uniform(math.log(2e4), math.log(4e5)))
        L = rng.uniform(10e-3, 20e-3)
        T = rng.uniform(3e-3, 5e-3)
        h = (L * L * T / N) ** (1.0 / 3.0)
        if 0.1e-3 <= h <= 0.3e-3:
            break
    nxy = max(8, int(round(L / h)))
    if max_lateral > 0:
        nxy = min(nxy, max_lateral)
    nz = max(4, int(round(T / h)))
    dx = h
    margin = max(6, int(math.ceil(0.12 * nxy)))
    gxy = nxy + 2 * margin
    gz = nz + 3 + max(6, int(math.ceil(0.25 * nz)))
    E = rng.uniform(0.1e6, 0.3e6)
    nu = rng.uniform(0.40, 0.48)
    rho = 1000.0
    family = rng.randint(5)
    sp = draw_indenter(rng, family)
    cfg = _contact(block_origin=(margin * dx, margin * dx, 3 * dx),
                   block_size=(nxy * dx, nxy * dx, nz * dx), n=(nxy, nxy, nz),
                   grid_origin=(0.0, 0.0, 0.0), dx=dx, gn=(gxy, gxy, gz),
                   E=E, nu=nu, rho=rho, model=COROTATED, shape=family, sp=sp, seed=seed)
    cx, cy = block_center_xy(cfg)
    jit = min(3e-3, 0.15 * nxy * dx)
    cx += rng.uniform(-jit, jit)
    cy += rng.uniform(-jit, jit)
    tilt = math.radians(rng.uniform(-5.0, 5.0))
    az = rng.uniform(0.0, 2.0 * math.pi)
    quat = quat_axis_angle((math.cos(az), math.sin(az), 0.0), tilt)
    depth = rng.uniform(0.2e-3, min(1.5e-3, 0.35 * nz * dx))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    cp = math.sqrt((lam + 2 * mu) / rho)
    dt = 0.45 * dx / cp
    poses = press_trajectory((cx, cy, top_z(cfg)), quat, depth, steps)
    return dict(name=f"batch_{seed}_{SHAPE_NAMES[family]}", cfg=cfg, dt=dt, steps=steps,
                poses=poses, depth=depth, particles=nxy * nxy * nz)


def lattice_count(cfg) -> int:
    n = cfg["n"]
    return n[0] * n[1] * n[2]


def random_particle_state(seed: int, cfg, vel_scale=0.05, c_scale=50.0, f_scale=0.05,
                          pos_jitter=0.3):
    """Random (x, v, C, F) around the rest lattice for single-substep parity
    cases, in [N][3], [N][3], [N][3][3], [N][3][3] float64 layout. Positions are
    jittered by up to `pos_jitter` lattice spacings."""
    rng = SplitMix64(0xC0FFEE + seed)
    n = cfg["n"]
    N = n[0] * n[1] * n[2]
    u = np.array([rng.uniform(-1.0, 1.0) for _ in range(N * 24)]).reshape(N, 24)
    hh = np.array(cfg["block_size"]) / np.array(n)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    idx = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
    x = np.array(cfg["block_origin"]) + (idx + 0.5) * hh + pos_jitter * hh * u[:, 0:3]
    v = vel_scale * u[:, 3:6]
    C = c_scale * u[:, 6:15].reshape(N, 3, 3)
    F = np.eye(3)[None] + f_scale * u[:, 15:24].reshape(N, 3, 3)
    return x, v, C, F
