/*
 * Tacchi MLS-MPM oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the explicit
 * MLS-MPM substep of Sec. III-A (Eqs. 1-11) with a rigid-indenter inside test
 * applied on the grid, plus the depth map and Phong shading of Sec. III-B
 * (Eqs. 12-14). Only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the HIP library never links, includes or calls it,
 * and the two share no source.
 *
 * Conventions: SI units, world frame. Particle p of the lattice (i, j, k),
 * i fastest, is p = i + n0*(j + n1*k). Arrays are AoS: x[p][3], v[p][3],
 * C[p][3][3], F[p][3][3] (row-major matrices). Grid node (a, b, c) is
 * q = a + g0*(b + g1*c) at X = grid_origin + (a, b, c)*dx.
 *
 * Poses are 7 doubles: tip position (x, y, z) and unit quaternion
 * (w, x, y, z) mapping the indenter frame to the world frame.
 */
#ifndef TACCHI_ORACLE_H
#define TACCHI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_UNSTABLE = -4, ORC_E_OUT_OF_GRID = -5 };

typedef struct {
    double block_origin[3];
    double block_size[3];
    int32_t n[3];
    double grid_origin[3];
    double dx;
    int32_t gn[3];
    double E, nu, rho;
    int32_t model;          /* 0 neo-Hookean, 1 fixed corotated */
    int32_t shape;          /* -1 none, 0 sphere, 1 cylinder, 2 cone, 3 edge, 4 textured plate */
    double sp[8];
    uint64_t seed;
    double gravity[3];
    int32_t n_fixed_layers; /* particles in lattice layers k < this keep v = 0 (Eq. 10) */
    int32_t floor_node;     /* nodes with iz <= floor_node are held at rest; -1 none */
    int32_t wall_nodes;     /* nodes within this many of a face drop outward velocity; 0 none */
} orc_config;

typedef struct {
    double ka_ia, kd, ks, alpha;
    double light_elev_deg, light_azim_deg[3];
    double pitch;           /* m per pixel */
} orc_render_params;

typedef struct orc_sim orc_sim;

orc_sim *orc_create(const orc_config *cfg, const double pose0[7]);
void orc_destroy(orc_sim *s);
int64_t orc_num_particles(const orc_sim *s);
int64_t orc_num_nodes(const orc_sim *s);

void orc_get_particles(const orc_sim *s, double *x, double *v, double *C, double *F);
void orc_set_particles(orc_sim *s, const double *x, const double *v, const double *C,
                       const double *F);
void orc_get_pose(const orc_sim *s, double pose[7]);
void orc_set_pose(orc_sim *s, const double pose[7]);

/* The three phases of one substep, and the whole substep. */
int orc_p2g(orc_sim *s, double dt);
int orc_grid_update(orc_sim *s, const double pose_end[7], double dt);
int orc_g2p(orc_sim *s, double dt);
int orc_step(orc_sim *s, const double pose_end[7], double dt);

void orc_get_grid(const orc_sim *s, double *M, double *P, double *V); /* [n], [n][3], [n][3] */
void orc_force(const orc_sim *s, double f[3]);
/* Contact model from the next grid update: 0 no-slip (default), 1 Coulomb
 * friction with coefficient mu (see orc_grid_update). */
void orc_set_contact(orc_sim *s, int model, double mu);
/* Particle indenter: n points (indenter frame, [n][3]) of mass `mass` each;
 * n = 0 returns to the implicit solid. orc_indenter_mass copies the
 * indenter's mass per grid node of the last grid update. */
int orc_set_indenter_points(orc_sim *s, const double *xyz, int64_t n, double mass);
void orc_indenter_mass(const orc_sim *s, double *out);

void orc_heightmap(const orc_sim *s, double *H);                      /* [n1][n0] */
void orc_render(const orc_sim *s, const orc_render_params *rp, int32_t h, int32_t w,
                double *rgb);                                         /* [h][w][3] */
void orc_render_height(const orc_config *cfg, const double *H, const orc_render_params *rp,
                       int32_t h, int32_t w, double *rgb);

/* Building blocks, exposed for the pins. */
double orc_bspline(double r);
void orc_lame(double E, double nu, double *mu, double *lambda);
int orc_stress(int model, double mu, double lambda, const double F[9], double tau[9]);
int orc_polar(const double F[9], double R[9], double S[9]);
double orc_phi(int shape, const double sp[8], uint64_t seed, const double p_local[3]);
double orc_lowest_point(int shape, const double sp[8], uint64_t seed, const double pose[7], double x, double y,
                        double zlo, double zhi, int nscan);
void orc_indenter_velocity(const double pose0[7], const double pose1[7], double dt,
                           const double X[3], double v[3]);
double orc_noise2(uint64_t seed, double x, double y);

#ifdef __cplusplus
}
#endif
#endif
