/*
 * tacchi.h -- C ABI of the MI355X (gfx950) tactile elastomer simulator.
 *
 * The library simulates an optical tactile sensor's elastomer pressed by a
 * rigid indenter with the explicit MLS-MPM substep of the Tacchi paper
 * (Sec. III-A, Eqs. 1-11) and turns the deformed top surface into a depth map
 * and a Phong-shaded tactile image (Sec. III-B, Eqs. 12-14). The calls follow
 * the paper's statement of the problem (Sec. III-C, Fig. 3): the elastomer is
 * a particle block with Young's modulus and Poisson's ratio (Sec. III-D,
 * Sec. IV-B); each simulation step the host simulator supplies the indenter
 * pose; the outputs are the depth map and the tactile image.
 *
 * Conventions shared by every call
 *  - SI units (m, s, kg, Pa). World frame; the sensor looks along +z at the
 *    elastomer from below, the indenter comes from +z.
 *  - Memory: the caller owns all device memory. `tacchi_workspace_bytes`
 *    sizes one device buffer; `tacchi_create` carves every array out of it
 *    (256-byte aligned base required) and allocates no device memory. The
 *    workspace must outlive the handle. Host-side inputs are copied.
 *  - Streams: every device operation of a handle is enqueued on the HIP
 *    stream given at creation (NULL = the legacy default stream).
 *    Calls are asynchronous unless stated otherwise.
 *  - Errors: no exception crosses the ABI. Each call returns a tacchi_status;
 *    the message of the last failure on the calling thread is in
 *    `tacchi_last_error()`. Device-side faults (non-finite state, inverted
 *    elements under neo-Hookean, particles leaving the grid) set a device
 *    error word that is reported by the next synchronising call
 *    (`tacchi_sync`, `tacchi_heightmap`, `tacchi_render`, `tacchi_read_*`,
 *    `tacchi_indenter_force`); the handle keeps working but its state is
 *    then undefined until rewritten with `tacchi_write_particles`. A grid
 *    block that collects more than 2.5x its rest particle count (a local
 *    compression below J = 0.4) is reported as E_UNSTABLE.
 *  - Particle p of the lattice (i, j, k), i fastest, is p = i + n0*(j + n1*k);
 *    k = 0 is the bottom layer (bonded to the sensor), k = n2-1 the contact
 *    surface. Particle arrays are structure-of-arrays in the simulation
 *    precision: x[3][N], v[3][N], C[9][N], F[9][N] (row-major 3x3, entry
 *    (r, c) at [3r+c][N]).
 *  - A handle is not thread-safe; separate handles are independent.
 */
#ifndef TACCHI_H
#define TACCHI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tacchi_status;
enum {
    TACCHI_OK = 0,
    TACCHI_E_ARG = -1,          /* invalid argument or configuration */
    TACCHI_E_WORKSPACE = -2,    /* workspace missing, too small or misaligned */
    TACCHI_E_DEVICE = -3,       /* a HIP call failed */
    TACCHI_E_UNSTABLE = -4,     /* non-finite state, J <= 0 (neo-Hookean), dt above the CFL limit */
    TACCHI_E_OUT_OF_GRID = -5,  /* a particle's 3x3x3 stencil left the grid */
    TACCHI_E_STATE = -6         /* call not valid in the handle's current state */
};

enum { TACCHI_F64 = 0, TACCHI_F32 = 1 };
enum { TACCHI_NEOHOOKEAN = 0, TACCHI_COROTATED = 1 };
enum { TACCHI_NO_INDENTER = -1, TACCHI_SPHERE = 0, TACCHI_CYLINDER = 1, TACCHI_CONE = 2,
       TACCHI_EDGE = 3, TACCHI_TEXTURED_PLATE = 4 };

/* Elastomer block sampled by a cell-centred particle lattice: particle
 * (i, j, k) rests at origin + ((i, j, k) + 1/2) * size / n. */
typedef struct { double origin[3], size[3]; int32_t n[3]; } tacchi_block;
/* Background grid: node (a, b, c) at origin + (a, b, c) * dx, n nodes per axis
 * (7 to 65536 per axis, at most 2^29 nodes once rounded up to whole blocks;
 * dx >= the lattice spacing; at least 3 nodes of margin around the block,
 * whose bottom face lies on a node plane). */
typedef struct { double origin[3]; double dx; int32_t n[3]; } tacchi_grid;
/* Hyperelastic material: E [Pa], nu, rho [kg/m^3], model TACCHI_NEOHOOKEAN or
 * TACCHI_COROTATED. */
typedef struct { double E, nu, rho; int32_t model; } tacchi_material;
/* Rigid indenter, described in its own frame (lowest point at the origin,
 * +z away from the gel):
 *   SPHERE          p[0] = radius
 *   CYLINDER        p[0] = radius of a flat circular punch
 *   CONE            p[0] = half-angle [rad], p[1] = tip rounding radius
 *   EDGE            p[0] = half-angle [rad], p[1] = tip rounding radius;
 *                   a wedge whose edge runs along the indenter y axis
 *   TEXTURED_PLATE  p[0] = half-width of a square punch, p[1] = amplitude,
 *                   p[2] = wavelength of the gradient noise on its bottom face
 *                   (noise lattice hashed from `seed`) */
typedef struct { int32_t shape; double p[8]; uint64_t seed; } tacchi_indenter;
/* Indenter pose: position of the indenter-frame origin and unit quaternion
 * (w, x, y, z) rotating indenter-frame vectors into the world frame. */
typedef struct { double pos[3], quat[4]; } tacchi_pose;

typedef struct {
    tacchi_block block;
    tacchi_grid grid;
    tacchi_material mat;
    tacchi_indenter ind;
    tacchi_pose pose0;          /* indenter pose at t = 0 */
    double gravity[3];          /* m/s^2 */
    int32_t n_fixed_layers;     /* bottom lattice layers held at v = 0 (Eq. 10), >= 1 */
    int32_t precision;          /* TACCHI_F64 or TACCHI_F32 */
    int32_t tile;               /* grid block edge in nodes: 4 or 8; 0 picks 8 */
} tacchi_config;

/* Phong shading constants (Eq. 12): ambient ka*ia, diffuse kd, specular ks,
 * shininess alpha; three distant lights (red, green, blue channel) at
 * elevation light_elev_deg toward the camera and azimuths light_azim_deg;
 * pitch = metres per pixel (the r of Eq. 14). */
typedef struct {
    double ka_ia, kd, ks, alpha, light_elev_deg, light_azim_deg[3], pitch;
} tacchi_render_params;

typedef struct tacchi_sim tacchi_sim;   /* opaque, host memory owned by the library */

/* Bytes of device workspace a handle for `cfg` needs (0 if cfg is invalid;
 * the reason is then in tacchi_last_error()). */
size_t tacchi_workspace_bytes(const tacchi_config *cfg);

/* Validate `cfg` (Sec. III-D guidelines: the grid encloses the block with at
 * least 3 nodes of margin on every side; the bottom face lies on a node plane;
 * dx >= lattice spacing; n_fixed_layers >= 1; E > 0; 0 <= nu < 0.5; rho > 0),
 * carve the workspace and initialise the particles (Eq. 1: rest lattice,
 * v = 0, C = 0, F = I). `hip_stream` is a hipStream_t (may be NULL).
 * Errors: E_ARG, E_WORKSPACE, E_DEVICE. */
tacchi_status tacchi_create(const tacchi_config *cfg, void *dev_ws, size_t ws_bytes,
                            void *hip_stream, tacchi_sim **out);

/* One explicit substep from the current indenter pose to `pose_end` over dt
 * (Sec. III-A: particle-to-grid Eqs. 2-5, grid velocity Eq. 6 with the rigid
 * indenter contact, grid-to-particle Eqs. 7-9, special cases Eq. 10 and
 * advection Eq. 11). Sorting particles into grid blocks is part of the step.
 * Asynchronous. Errors: E_ARG (dt <= 0), E_UNSTABLE (dt * c_p / dx > 1 with
 * c_p = sqrt((lambda + 2 mu)/rho)), E_DEVICE. */
tacchi_status tacchi_step(tacchi_sim *sim, const tacchi_pose *pose_end, double dt);

/* `n` substeps of size dt; substep s ends at poses[s]. Asynchronous. */
tacchi_status tacchi_run(tacchi_sim *sim, const tacchi_pose *poses, int32_t n, double dt);

/* Contact model of the indenter (beyond the paper, whose contact is
 * no-slip and which leaves surface friction to future work, Sec. VI):
 * TACCHI_CONTACT_STICKY (the default) gives every grid node inside the
 * indenter the rigid velocity; TACCHI_CONTACT_COULOMB with coefficient
 * mu >= 0 (+inf allowed) splits a contact node's velocity relative to the
 * indenter along the outward normal n (central differences of the shape's
 * signed distance, step 1e-3 dx): a node moving apart keeps its velocity,
 * an approaching one loses its normal component and its tangential
 * component shrinks by mu times the normal speed, stopping where it is
 * smaller (stick). Takes effect from the next substep; TACCHI_E_ARG for an
 * unknown model or a negative or NaN mu. */
enum { TACCHI_CONTACT_STICKY = 0, TACCHI_CONTACT_COULOMB = 1 };
tacchi_status tacchi_set_contact(tacchi_sim *sim, int32_t model, double mu);

/* The indenter as particles (Eq. 10: the particles representing the indenter
 * take its velocity; Sec. IV-B: objects enter as point clouds, whose density
 * the paper varies): n points xyz[k] in the indenter frame (metres, host
 * memory, copied), each of mass `mass` [kg]. Every substep the points are
 * placed rigidly at the pose of the substep's start and scatter their mass to
 * the grid with the weights of Eq. 2 (points whose 3x3x3 nodes leave the grid
 * are ignored); their momentum there is that mass times the indenter's rigid
 * velocity at the node (APIC with the rigid body's velocity gradient is exact
 * for it), and a grid node carrying indenter mass M_I takes the velocity
 * (M V + M_I v_indenter)/(M + M_I) in place of the shape's contact; the
 * contact force is still the gel's momentum change. n = 0 returns to the
 * shape's contact (tacchi_set_contact); dev_ws may then be NULL.
 * The points and an FP64 indenter mass per grid node live in dev_ws, device
 * memory owned by the caller: 256-byte aligned, at least
 * tacchi_points_workspace_bytes(sim, n) bytes, kept alive (and not used
 * otherwise) until the next tacchi_set_indenter_points or tacchi_destroy.
 * Errors: E_ARG (NULL, n outside [0, 2^24], bad mass or coordinate),
 * E_WORKSPACE (workspace missing, misaligned or too small), E_STATE (inside a
 * substep). Must be called between substeps. Synchronises. */
size_t tacchi_points_workspace_bytes(const tacchi_sim *sim, int32_t n);
tacchi_status tacchi_set_indenter_points(tacchi_sim *sim, const double *xyz, int32_t n, double mass,
                                         void *dev_ws, size_t ws_bytes);

/* The scripted press with a terminal condition on the contact force
 * (Sec. III-C: the simulation ends when a terminal condition is met): runs
 * substeps as tacchi_run does, poses[s] ending substep s, until the z
 * component of the contact force on the indenter (tacchi_indenter_force)
 * after a substep is >= fz_limit [N] (+inf: never; -inf: after the first
 * substep; NaN is rejected), or until all n substeps have run. The
 * test is made on the device after every substep, so the n substeps are
 * queued without a host round trip per substep; once the limit is reached
 * the remaining queued substeps do nothing. *steps_done receives the number
 * of substeps that ran (the stopping one included); the simulation is left
 * after that substep, at pose poses[*steps_done - 1], ready for further
 * steps. Must be called between substeps (not after tacchi_p2g or
 * tacchi_grid_update). Synchronises; reports the device error word. */
tacchi_status tacchi_run_until_force(tacchi_sim *sim, const tacchi_pose *poses, int32_t n, double dt,
                                     double fz_limit, int32_t *steps_done);

/* The three phases of tacchi_step, for callers that inspect the grid:
 * tacchi_p2g (sort + particle-to-grid), tacchi_grid_update (grid velocity and
 * contact toward `pose_end`), tacchi_g2p (grid-to-particle; commits
 * `pose_end` as the current pose). They must be called in this order;
 * otherwise E_STATE. */
tacchi_status tacchi_p2g(tacchi_sim *sim, double dt);
tacchi_status tacchi_grid_update(tacchi_sim *sim, const tacchi_pose *pose_end, double dt);
tacchi_status tacchi_g2p(tacchi_sim *sim, double dt);

/* Dense copy of the grid in node order (a fastest): after tacchi_p2g,
 * which = 0 gives node mass M[n] and momentum P[3][n] (kg, kg m/s); after
 * tacchi_grid_update, which = 1 gives M[n] unset and velocity V[3][n] (m/s).
 * Buffers are in the simulation precision, on device if on_device != 0.
 * Synchronises. */
tacchi_status tacchi_read_grid(tacchi_sim *sim, int32_t which, void *M, void *vec,
                               int32_t on_device);

/* Depth map of the contact surface (Sec. III-B): out[j][i] = world z of
 * top-layer particle (i, j, n2-1), n1 x n0 values in the simulation
 * precision. Synchronises (and reports the device error word). */
tacchi_status tacchi_heightmap(tacchi_sim *sim, void *out, int32_t out_on_device);

/* Tactile image (Sec. III-B, Eqs. 12-14): an h x w crop centred on the top
 * face at `pitch` m/pixel; the depth map is resampled bilinearly at the pixel
 * centres (rest coordinates), normals come from central differences
 * [-1, 0, 1]/(2 pitch) with replicated borders, each channel is lit by its
 * light with Phong's model (dot products clamped at 0, specular only where
 * the light faces the surface, result clamped to [0, 1]). rgb is float32
 * [h][w][3]. Synchronises. */
tacchi_status tacchi_render(tacchi_sim *sim, const tacchi_render_params *rp, float *rgb,
                            int32_t h, int32_t w, int32_t out_on_device);

/* Displacement field of the contact surface (the depth map of Sec. III-B
 * extended to all three components): out[r][c][a] (metres, float32,
 * res x res x 3) is the mean displacement x - X of the top face over cell
 * (c, r) of a res x res partition of the block's top face, taken over
 * sub x sub points spread evenly in the cell (at (c + (q + 1/2)/sub) L/res,
 * q = 0 .. sub-1, per axis; sub = 1 is the cell centre), each interpolated
 * bilinearly between the top-layer particles' displacements (particle i at
 * (i + 1/2) h; clamped at the border). 1 <= res <= 4096, 1 <= sub <= 16.
 * With out_on_device != 0 the call is asynchronous on the simulation's
 * stream; otherwise the kernel writes into the handle's pinned host staging
 * buffer (no device memory is allocated), and the call synchronises and
 * reports the device error word. */
tacchi_status tacchi_surface_displacement(tacchi_sim *sim, int32_t res, int32_t sub, float *out,
                                          int32_t out_on_device);

/* Markers (Sec. VI: marker motion is simulated by recording the motion of
 * the surface particles at the markers' positions): for n marker positions
 * xy[k] = (x, y) on the undeformed top face (world metres, host memory,
 * copied; each must lie on the face, else TACCHI_E_ARG), out[k][a] is the
 * displacement x - X of the top surface at that point (metres, simulation
 * precision, n x 3): bilinear between the four surrounding top-layer
 * particles (particle i at (i + 1/2) h), a point on the half-cell rim outside
 * the outermost particle centres taking the edge value. 1 <= n <= 2^24.
 * With out_on_device != 0 out is device memory. The marker coordinates (and
 * a host output) pass through the handle's pinned host staging buffer, which
 * the kernel reads and writes directly: no device memory is allocated. The
 * call synchronises either way and reports the device error word. */
tacchi_status tacchi_markers(tacchi_sim *sim, const double *xy, int32_t n, void *out, int32_t out_on_device);

/* Gap field of an indenter over the undeformed top face, the geometric input
 * of the learned surrogate: for n configurations and poses (indenter frame ->
 * world, as in tacchi_step), out[k][r][c] (metres, float32, device memory)
 * is the mean over the sub x sub points of cell (c, r) of block k's top face
 * (placed as in tacchi_surface_displacement) of the clamped gap
 * clamp(z_ind - z_top, lo, hi), where z_top = block.origin[2] +
 * block.size[2] and z_ind is the lowest point of the indenter's solid (the
 * inside test of Eq. 10's rigid body) on the vertical through the point (no
 * indenter up to z_top + hi: hi). With hi = 0 this is the penetration of the
 * indenter into the undeformed face. z_ind is found by sampling the inside
 * test at 512 heights from z_top + lo to z_top + hi and bisecting the first
 * crossing 40 times. lo < hi, hi - lo <= 1 m. The n query descriptors are
 * copied into dev_ws, device memory owned by the caller (256-byte aligned,
 * at least tacchi_indenter_gap_workspace_bytes(n) bytes). Runs on
 * hip_stream and synchronises it. Errors: E_ARG, E_WORKSPACE (workspace
 * missing, misaligned or too small), E_DEVICE. */
size_t tacchi_indenter_gap_workspace_bytes(int32_t n);
tacchi_status tacchi_indenter_gap(const tacchi_config *cfgs, const tacchi_pose *poses, int32_t n,
                                  int32_t res, int32_t sub, double lo, double hi, float *out,
                                  void *dev_ws, size_t ws_bytes, void *hip_stream);

/* tacchi_indenter_gap for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same gap field, computed by the same kernel from the same
 * arguments, with the n query descriptors kept in a fixed device array of the
 * library instead of a caller workspace. Nothing is allocated: the array comes
 * with the library's code object, one copy per GPU, held until the process
 * ends; its address on a GPU is looked up on the first call there (with that
 * GPU current). n <= tacchi_indenter_gap_noalloc_max() (2048), else E_ARG.
 * hip_stream must belong to the current GPU. Every call on a GPU uses that
 * GPU's one array, so calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller; the call synchronises
 * hip_stream before it returns. Errors as tacchi_indenter_gap (no
 * E_WORKSPACE). */
int32_t tacchi_indenter_gap_noalloc_max(void);
tacchi_status tacchi_indenter_gap_noalloc(const tacchi_config *cfgs, const tacchi_pose *poses, int32_t n,
                                          int32_t res, int32_t sub, double lo, double hi, float *out,
                                          void *hip_stream);

/* Particle state in SoA layout (see the conventions); any pointer may be
 * NULL to skip that array. Synchronises. */
tacchi_status tacchi_read_particles(tacchi_sim *sim, void *x, void *v, void *C, void *F,
                                    int32_t on_device);
/* Overwrite the particle state (all four arrays required); used to restore a
 * checkpoint or inject a state. Clears the device error word. */
tacchi_status tacchi_write_particles(tacchi_sim *sim, const void *x, const void *v,
                                     const void *C, const void *F, int32_t on_device);

/* Reaction force [N] on the indenter over the last substep: sum over contact
 * nodes of M (V_before - V_indenter) / dt. Synchronises. */
tacchi_status tacchi_indenter_force(tacchi_sim *sim, double f[3]);

/* Current indenter pose (host copy, no sync). */
tacchi_status tacchi_get_pose(const tacchi_sim *sim, tacchi_pose *pose);

/* Fixed-corotated model in FP32: the polar factor of F is computed in FP32
 * by a scaled Newton iteration and recomputed in FP64 where the Frobenius
 * condition number |F| |adj F| / |det F| exceeds 1e6, det F <= 0 or the FP32
 * iteration does not converge. *count receives the number of such FP64
 * recomputations since creation (always 0 in FP64 mode, where every polar
 * factor is computed in FP64). Synchronises. */
tacchi_status tacchi_polar_fallbacks(tacchi_sim *sim, uint64_t *count);

/* Number of particles N of the handle. */
int64_t tacchi_num_particles(const tacchi_sim *sim);

/* Drain the handle's stream and report the device error word:
 * E_UNSTABLE, E_OUT_OF_GRID or OK. */
tacchi_status tacchi_sync(tacchi_sim *sim);

/* Kernel timing with HIP events on the handle's stream. Kernel classes:
 * 0 binning of all particles (after creation or a state write), 1 P2G,
 * 2 grid update, 3 G2P (which also bins the particles for the next
 * substep), 4 depth map, 5 render. tacchi_timing_enable brackets every later
 * launch of the classes set in `class_mask` (bit k = class k; 0 disables)
 * with a pair of events; tacchi_timing_read synchronises and returns, per
 * class, the summed elapsed milliseconds and the launch count since the last
 * reset (reset != 0 clears them afterwards). ms and counts hold
 * TACCHI_NUM_KERNEL_CLASSES entries. */
#define TACCHI_NUM_KERNEL_CLASSES 6
tacchi_status tacchi_timing_enable(tacchi_sim *sim, uint32_t class_mask);
tacchi_status tacchi_timing_read(tacchi_sim *sim, double *ms, int64_t *counts, int32_t reset);

/* Release the handle (host memory only; the workspace stays the caller's). */
void tacchi_destroy(tacchi_sim *sim);

/* ---------------------------------------------------------------------------
 * Batched contacts: many independent elastomer contacts (each its own block,
 * grid, material, indenter and dt) advanced together, one kernel launch per
 * phase of a substep for all of them, with runs of substeps captured once as
 * a HIP graph and replayed. Contacts must be FP32 (precision TACCHI_F32).
 * Indenter trajectories are given up front: traj[i][k] is contact i's pose
 * after k substeps (k = 0..substeps); past the last entry the final pose is
 * held. A tuner picks, per (material model, log2(N) class), the grid block
 * edge B in {4, 8}, the workgroup size in {64, 128, 256} (grid update and G2P;
 * P2G at B = 8 keeps 512 threads) and the work items (grid blocks) per
 * workgroup in {1, 2}, by timing 20 substeps of each setting on up to 8 of
 * the class's contacts launched together, after advancing them
 * 200 substeps into their own presses; the per-class choices are then kept
 * only if the whole batch runs at least as fast with them as with the default
 * everywhere (tacchi_batch_tuning_check). Choices and the time of every
 * candidate are cached in the JSON file `tune_cache` (keyed by GPU
 * architecture, precision, material model and class; read if present,
 * extended when `tune` != 0; NULL disables the file). Without a cached or
 * tuned choice a contact uses B = 8, 256 threads, one block per workgroup.
 * The batch owns one single-contact handle per contact for read-out.
 * ------------------------------------------------------------------------- */
typedef struct tacchi_batch tacchi_batch;   /* opaque, host memory owned by the library */

/* Device workspace bytes for a batch (0 on invalid input, reason in
 * tacchi_last_error()). */
size_t tacchi_batch_workspace_bytes(const tacchi_config *cfgs, int32_t n, int32_t substeps);

/* Validate and initialise all contacts (as tacchi_create), tabulate their
 * indenters ([n][substeps+1] poses, dt[n] per contact, each within its CFL
 * limit), tune, and set up the launch groups. `hip_stream` must be a
 * non-default stream for graph replay (with NULL every substep is launched
 * directly). Synchronises. Errors: E_ARG, E_WORKSPACE, E_UNSTABLE (CFL),
 * E_DEVICE. */
tacchi_status tacchi_batch_create(const tacchi_config *cfgs, int32_t n, const tacchi_pose *traj,
                                  const double *dt, int32_t substeps, const char *tune_cache,
                                  int32_t tune, void *dev_ws, size_t ws_bytes, void *hip_stream,
                                  tacchi_batch **out);

/* Advance every contact by `substeps` substeps (asynchronous). */
tacchi_status tacchi_batch_run(tacchi_batch *batch, int32_t substeps);

/* Handle of contact i for read-out calls (tacchi_heightmap, tacchi_render,
 * tacchi_read_particles, tacchi_indenter_force, tacchi_sync). It belongs to
 * the batch: do not step, write or destroy it. NULL if i is out of range. */
tacchi_sim *tacchi_batch_contact(tacchi_batch *batch, int32_t i);

/* Per-contact tuning choice: grid block edge, workgroup size, grid blocks per
 * workgroup and the measured microseconds per substep of the tuning run (0 if
 * the choice was a default); any pointer may be NULL, arrays hold n entries. */
tacchi_status tacchi_batch_tuning(const tacchi_batch *batch, int32_t *tile, int32_t *wg, int32_t *ipw,
                                  double *us_per_substep);

/* The tuner's whole-batch check (batch created with tune != 0): microseconds
 * per substep of the whole batch with the per-class choices and with the
 * default setting for every contact, each timed over 20 substeps after
 * advancing 200 into the presses; the batch keeps the choices only when they
 * are not slower. Both 0 when the batch was not tuned. */
tacchi_status tacchi_batch_tuning_check(const tacchi_batch *batch, double *us_tuned, double *us_default);

/* Substeps advanced so far. */
int64_t tacchi_batch_substeps_done(const tacchi_batch *batch);

/* Drain the stream and report the first contact's device error, if any. */
tacchi_status tacchi_batch_sync(tacchi_batch *batch);

/* tacchi_surface_displacement of every contact: out is [n][res][res][3].
 * Synchronises and reports device errors. */
tacchi_status tacchi_batch_surface_displacement(tacchi_batch *batch, int32_t res, int32_t sub, float *out,
                                                int32_t out_on_device);

/* Release the batch and its contact handles (host memory only). */
void tacchi_batch_destroy(tacchi_batch *batch);

/* Message of the last failing call on this thread ("" if none). */
const char *tacchi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TACCHI_H */
