/*
 * Tacchi MLS-MPM oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain FP64 C, single thread, no blocking, fusion or reordering: each phase
 * follows the paper's order of operations so a reader can check it against
 * Sec. III-A (Eqs. 1-11) and Sec. III-B (Eqs. 12-14) by eye.
 *
 * Readings of the paper used here (the paper leaves these open):
 *  - w_ip is the tensor product of 1D quadratic B-splines N(x_p - X_i)/dx
 *    (Eq. 2 and its prose); the 3x3x3 node set of a particle starts at
 *    base = floor(x/dx - 1/2).
 *  - Eq. 4 carries m_p on the affine term: w m_p (v_p + C_p (X_i - x_p)).
 *  - S_p of Eq. 5 is the Kirchhoff stress tau = P(F) F^T of the chosen
 *    hyperelastic model, so the stress term is -dt V0 (4/dx^2) tau (X_i - x_p).
 *  - Eq. 8 sums the grid velocities V_i (the printed v_p^(k+1) would make
 *    C vanish identically): C = (4/dx^2) sum_i w V_i (X_i - x_p)^T.
 *  - The rigid indenter is an implicit solid phi <= 0 applied on the grid:
 *    nodes inside take the rigid indenter velocity (no-slip), replacing the
 *    paper's indenter particles of Eq. 10 (same single-velocity-field effect).
 *  - The bottom lattice layers keep v = 0 (Eq. 10); grid nodes at or below
 *    the block's bottom node plane are held at rest; nodes within
 *    `wall_nodes` of a grid face lose their outward velocity component.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

struct orc_sim {
    orc_config cfg;
    int64_t N, nn;
    double h[3];          /* lattice spacing per axis */
    double m, V0;         /* particle mass and initial volume */
    double mu, lambda;
    double *x, *v, *C, *F;
    double *M, *P, *V;
    double pose[7];       /* indenter pose at the start of the current substep */
    double force[3];
    int status;
    int contact;          /* 0 no-slip, 1 Coulomb friction */
    double friction;      /* Coulomb coefficient */
    double *ipts;         /* particle indenter: points in the indenter frame [ni][3] */
    int64_t ni;
    double imass;         /* mass per indenter point */
    double *MI;           /* indenter mass per node of the last grid update */
};

/* ---------------------------------------------------------------- small 3x3 helpers */

static void mat_mul(const double A[9], const double B[9], double out[9])
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
            t[r * 3 + c] = s;
        }
    memcpy(out, t, sizeof t);
}

static void mat_transpose(const double A[9], double out[9])
{
    double t[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) t[r * 3 + c] = A[c * 3 + r];
    memcpy(out, t, sizeof t);
}

static double mat_det(const double A[9])
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void quat_to_matrix(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ---------------------------------------------------------------- interpolation */

/* 1D quadratic B-spline kernel N(r), r in grid units (Eq. 2 prose: "quadratic
 * B-Spline"); the 3D weight is the product over the three axes. */
double orc_bspline(double r)
{
    double a = fabs(r);
    if (a < 0.5) return 0.75 - a * a;
    if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
    return 0.0;
}

/* ---------------------------------------------------------------- material */

void orc_lame(double E, double nu, double *mu, double *lambda)
{
    *mu = E / (2.0 * (1.0 + nu));
    *lambda = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations:
 * A = Q diag(d) Q^T. */
static void sym_eig(const double A_in[9], double d[3], double Q[9])
{
    double A[9];
    memcpy(A, A_in, sizeof A);
    for (int i = 0; i < 9; ++i) Q[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-40 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[p * 3 + q];
                if (apq == 0.0) continue;
                double theta = (A[q * 3 + q] - A[p * 3 + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k * 3 + p], akq = A[k * 3 + q];
                    A[k * 3 + p] = c * akp - s * akq;
                    A[k * 3 + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p * 3 + k], aqk = A[q * 3 + k];
                    A[p * 3 + k] = c * apk - s * aqk;
                    A[q * 3 + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double qkp = Q[k * 3 + p], qkq = Q[k * 3 + q];
                    Q[k * 3 + p] = c * qkp - s * qkq;
                    Q[k * 3 + q] = s * qkp + c * qkq;
                }
            }
    }
    d[0] = A[0]; d[1] = A[4]; d[2] = A[8];
}

/* Polar decomposition F = R S with det R = +1 from the eigen-decomposition of
 * F^T F: S = Q diag(sigma) Q^T, R = F Q diag(1/sigma) Q^T; when det F < 0 the
 * smallest sigma takes the minus sign so that R stays a proper rotation. */
int orc_polar(const double F[9], double R[9], double S[9])
{
    double Ft[9], FtF[9], d[3], Q[9];
    mat_transpose(F, Ft);
    mat_mul(Ft, F, FtF);
    sym_eig(FtF, d, Q);
    double sig[3];
    int kmin = 0;
    for (int k = 0; k < 3; ++k) {
        sig[k] = sqrt(d[k] > 0.0 ? d[k] : 0.0);
        if (sig[k] < sig[kmin]) kmin = k;
    }
    if (mat_det(F) < 0.0) sig[kmin] = -sig[kmin];
    for (int k = 0; k < 3; ++k)
        if (sig[k] == 0.0) return ORC_E_UNSTABLE;
    double Dq[9], Dinv[9], Qt[9];
    mat_transpose(Q, Qt);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Dq[r * 3 + c] = Q[r * 3 + c] * sig[c];
            Dinv[r * 3 + c] = Q[r * 3 + c] / sig[c];
        }
    mat_mul(Dq, Qt, S);
    double FQ[9];
    mat_mul(F, Dinv, FQ);
    mat_mul(FQ, Qt, R);
    return ORC_OK;
}

/* Kirchhoff stress tau = P(F) F^T (the S_p of Eq. 5 under the reading above).
 *  neo-Hookean (Psi = mu/2 (tr F^T F - 3) - mu ln J + lambda/2 (ln J)^2):
 *      tau = mu (F F^T - I) + lambda ln(J) I
 *  fixed corotated (Psi = mu |F - R|^2 + lambda/2 (J - 1)^2):
 *      tau = 2 mu (F - R) F^T + lambda (J - 1) J I */
int orc_stress(int model, double mu, double lambda, const double F[9], double tau[9])
{
    double J = mat_det(F);
    double Ft[9];
    mat_transpose(F, Ft);
    if (!isfinite(J)) return ORC_E_UNSTABLE;
    if (model == 0) {
        if (J <= 0.0) return ORC_E_UNSTABLE;
        double FFt[9];
        mat_mul(F, Ft, FFt);
        double lnJ = log(J);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                tau[r * 3 + c] = mu * (FFt[r * 3 + c] - (r == c ? 1.0 : 0.0)) +
                                 (r == c ? lambda * lnJ : 0.0);
        return ORC_OK;
    }
    double R[9], S[9], D[9], DFt[9];
    if (orc_polar(F, R, S) != ORC_OK) return ORC_E_UNSTABLE;
    for (int k = 0; k < 9; ++k) D[k] = F[k] - R[k];
    mat_mul(D, Ft, DFt);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            tau[r * 3 + c] = 2.0 * mu * DFt[r * 3 + c] + (r == c ? lambda * (J - 1.0) * J : 0.0);
    return ORC_OK;
}

/* ---------------------------------------------------------------- indenter */

/* Counter-based hash for the noise lattice: one SplitMix64 output step
 * (Steele et al. 2014) applied to a key built from the seed and the lattice
 * corner. */
static uint64_t corner_hash(uint64_t seed, int64_t ix, int64_t iy)
{
    uint64_t z = seed + (uint64_t)ix * 0x9E3779B97F4A7C15ULL + (uint64_t)iy * 0xD1B54A32D192ED03ULL;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* 2D gradient noise (Perlin, "Improving Noise", 2002: quintic fade) with the
 * eight gradients (+-1, 0), (0, +-1), (+-1, +-1) picked by the corner hash. */
double orc_noise2(uint64_t seed, double x, double y)
{
    static const double G[8][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
    double fx0 = floor(x), fy0 = floor(y);
    int64_t X0 = (int64_t)fx0, Y0 = (int64_t)fy0;
    double fx = x - fx0, fy = y - fy0;
    double n[2][2];
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            const double *g = G[corner_hash(seed, X0 + a, Y0 + b) >> 61];
            n[b][a] = g[0] * (fx - a) + g[1] * (fy - b);
        }
    double u = fx * fx * fx * (fx * (fx * 6.0 - 15.0) + 10.0);
    double w = fy * fy * fy * (fy * (fy * 6.0 - 15.0) + 10.0);
    double top = n[0][0] + u * (n[0][1] - n[0][0]);
    double bot = n[1][0] + u * (n[1][1] - n[1][0]);
    return top + w * (bot - top);
}

/* Rounded cone/wedge in a 2D section (rho, z) with the tip at the origin, axis
 * +z, half-angle th, tip radius rt: the sharp cone with apex at (0, rt)
 * inflated by rt. */
static double rounded_cone(double rho, double z, double th, double rt)
{
    double qz = z - rt;
    double s = rho * sin(th) + qz * cos(th);
    double d = (s <= 0.0) ? sqrt(rho * rho + qz * qz) : rho * cos(th) - qz * sin(th);
    return d - rt;
}

/* Indenter solid as an implicit function of a point in the indenter frame
 * (tip at the origin, +z away from the gel); phi <= 0 is inside. */
double orc_phi(int shape, const double sp[8], uint64_t seed, const double p[3])
{
    double x = p[0], y = p[1], z = p[2];
    switch (shape) {
    case 0: { /* sphere of radius sp[0] resting on its lowest point */
        double dz = z - sp[0];
        return sqrt(x * x + y * y + dz * dz) - sp[0];
    }
    case 1: { /* flat cylindrical punch of radius sp[0], bottom face z = 0 */
        double dr = sqrt(x * x + y * y) - sp[0], dz = -z;
        double inside = fmax(dr, dz) < 0.0 ? fmax(dr, dz) : 0.0;
        double ox = dr > 0.0 ? dr : 0.0, oz = dz > 0.0 ? dz : 0.0;
        return inside + sqrt(ox * ox + oz * oz);
    }
    case 2: /* cone, half-angle sp[0], tip radius sp[1] */
        return rounded_cone(sqrt(x * x + y * y), z, sp[0], sp[1]);
    case 3: /* straight edge along the indenter y axis */
        return rounded_cone(fabs(x), z, sp[0], sp[1]);
    case 4: { /* square plate, half-width sp[0], bottom face z = sp[1] n(x/sp[2], y/sp[2]) */
        double surf = sp[1] * orc_noise2(seed, x / sp[2], y / sp[2]);
        return fmax(fmax(fabs(x) - sp[0], fabs(y) - sp[0]), surf - z);
    }
    default:
        return 1.0;
    }
}

/* Rigid indenter velocity at X over [t_k, t_k + dt] from the poses at both
 * ends: translation of the tip plus omega x (X - tip), omega from the relative
 * rotation q1 q0^-1 (shortest arc). */
void orc_indenter_velocity(const double pose0[7], const double pose1[7], double dt,
                           const double X[3], double v[3])
{
    const double *a = pose0 + 3, *b = pose1 + 3; /* w x y z */
    /* q = b * conj(a) */
    double aw = a[0], ax = -a[1], ay = -a[2], az = -a[3];
    double qw = b[0] * aw - b[1] * ax - b[2] * ay - b[3] * az;
    double qx = b[0] * ax + b[1] * aw + b[2] * az - b[3] * ay;
    double qy = b[0] * ay - b[1] * az + b[2] * aw + b[3] * ax;
    double qz = b[0] * az + b[1] * ay - b[2] * ax + b[3] * aw;
    if (qw < 0) { qw = -qw; qx = -qx; qy = -qy; qz = -qz; }
    double sn = sqrt(qx * qx + qy * qy + qz * qz);
    double om[3] = {0, 0, 0};
    if (sn > 0.0) {
        double ang = 2.0 * atan2(sn, qw);
        om[0] = qx / sn * ang / dt; om[1] = qy / sn * ang / dt; om[2] = qz / sn * ang / dt;
    }
    double r[3] = {X[0] - pose0[0], X[1] - pose0[1], X[2] - pose0[2]};
    v[0] = (pose1[0] - pose0[0]) / dt + om[1] * r[2] - om[2] * r[1];
    v[1] = (pose1[1] - pose0[1]) / dt + om[2] * r[0] - om[0] * r[2];
    v[2] = (pose1[2] - pose0[2]) / dt + om[0] * r[1] - om[1] * r[0];
}

static double phi_world(const orc_sim *s, const double pose[7], const double X[3])
{
    double R[9];
    quat_to_matrix(pose + 3, R);
    double r[3] = {X[0] - pose[0], X[1] - pose[1], X[2] - pose[2]};
    double pl[3];
    for (int i = 0; i < 3; ++i) pl[i] = R[0 * 3 + i] * r[0] + R[1 * 3 + i] * r[1] + R[2 * 3 + i] * r[2];
    return orc_phi(s->cfg.shape, s->cfg.sp, s->cfg.seed, pl);
}

/* Lowest point of the posed indenter on the vertical line through (x, y):
 * the line is scanned upward from zlo in nscan equal steps up to zhi and the
 * first step that lands inside is bisected until the bracket stops shrinking.
 * Returns zlo when zlo is already inside and zhi + (zhi - zlo) when the line
 * stays outside up to zhi. */
double orc_lowest_point(int shape, const double sp[8], uint64_t seed, const double pose[7], double x, double y,
                        double zlo, double zhi, int nscan)
{
    double R[9];
    quat_to_matrix(pose + 3, R);
    double r[3], pl[3];
    r[0] = x - pose[0];
    r[1] = y - pose[1];
#define ORC_INSIDE(zz, res)                                                                            \
    do {                                                                                               \
        r[2] = (zz) - pose[2];                                                                         \
        for (int i_ = 0; i_ < 3; ++i_) pl[i_] = R[0 * 3 + i_] * r[0] + R[1 * 3 + i_] * r[1] + R[2 * 3 + i_] * r[2]; \
        (res) = orc_phi(shape, sp, seed, pl) <= 0.0;                                                   \
    } while (0)
    int in;
    ORC_INSIDE(zlo, in);
    if (in) return zlo;
    double a = zlo;
    for (int k = 1; k <= nscan; ++k) {
        double b = zlo + (zhi - zlo) * (double)k / (double)nscan;
        ORC_INSIDE(b, in);
        if (in) {
            for (;;) {
                double m = 0.5 * (a + b);
                if (m <= a || m >= b) break;
                ORC_INSIDE(m, in);
                if (in) b = m; else a = m;
            }
            return b;
        }
        a = b;
    }
#undef ORC_INSIDE
    return zhi + (zhi - zlo);
}

/* ---------------------------------------------------------------- lifecycle */

/* Initialization (Eq. 1 and the prose around it): particles on the
 * cell-centred lattice of the block, v = 0, F = I, C = 0; m = rho h^3 and
 * V0 = h^3 per particle. */
orc_sim *orc_create(const orc_config *cfg, const double pose0[7])
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->cfg = *cfg;
    s->N = (int64_t)cfg->n[0] * cfg->n[1] * cfg->n[2];
    s->nn = (int64_t)cfg->gn[0] * cfg->gn[1] * cfg->gn[2];
    for (int a = 0; a < 3; ++a) s->h[a] = cfg->block_size[a] / cfg->n[a];
    s->V0 = s->h[0] * s->h[1] * s->h[2];
    s->m = cfg->rho * s->V0;
    orc_lame(cfg->E, cfg->nu, &s->mu, &s->lambda);
    s->x = (double *)calloc((size_t)s->N * 3, sizeof(double));
    s->v = (double *)calloc((size_t)s->N * 3, sizeof(double));
    s->C = (double *)calloc((size_t)s->N * 9, sizeof(double));
    s->F = (double *)calloc((size_t)s->N * 9, sizeof(double));
    s->M = (double *)calloc((size_t)s->nn, sizeof(double));
    s->P = (double *)calloc((size_t)s->nn * 3, sizeof(double));
    s->V = (double *)calloc((size_t)s->nn * 3, sizeof(double));
    if (!s->x || !s->v || !s->C || !s->F || !s->M || !s->P || !s->V) {
        orc_destroy(s);
        return NULL;
    }
    for (int k = 0; k < cfg->n[2]; ++k)
        for (int j = 0; j < cfg->n[1]; ++j)
            for (int i = 0; i < cfg->n[0]; ++i) {
                int64_t p = i + (int64_t)cfg->n[0] * (j + (int64_t)cfg->n[1] * k);
                int idx[3] = {i, j, k};
                for (int a = 0; a < 3; ++a)
                    s->x[p * 3 + a] = cfg->block_origin[a] + (idx[a] + 0.5) * s->h[a];
                s->F[p * 9 + 0] = s->F[p * 9 + 4] = s->F[p * 9 + 8] = 1.0;
            }
    memcpy(s->pose, pose0, sizeof s->pose);
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->x); free(s->v); free(s->C); free(s->F);
    free(s->M); free(s->P); free(s->V);
    free(s->ipts); free(s->MI);
    free(s);
}

int64_t orc_num_particles(const orc_sim *s) { return s->N; }
int64_t orc_num_nodes(const orc_sim *s) { return s->nn; }

void orc_get_particles(const orc_sim *s, double *x, double *v, double *C, double *F)
{
    if (x) memcpy(x, s->x, (size_t)s->N * 3 * sizeof(double));
    if (v) memcpy(v, s->v, (size_t)s->N * 3 * sizeof(double));
    if (C) memcpy(C, s->C, (size_t)s->N * 9 * sizeof(double));
    if (F) memcpy(F, s->F, (size_t)s->N * 9 * sizeof(double));
}

void orc_set_particles(orc_sim *s, const double *x, const double *v, const double *C,
                       const double *F)
{
    if (x) memcpy(s->x, x, (size_t)s->N * 3 * sizeof(double));
    if (v) memcpy(s->v, v, (size_t)s->N * 3 * sizeof(double));
    if (C) memcpy(s->C, C, (size_t)s->N * 9 * sizeof(double));
    if (F) memcpy(s->F, F, (size_t)s->N * 9 * sizeof(double));
}

void orc_get_pose(const orc_sim *s, double pose[7]) { memcpy(pose, s->pose, sizeof s->pose); }
void orc_set_pose(orc_sim *s, const double pose[7]) { memcpy(s->pose, pose, sizeof s->pose); }

/* Stencil of particle p: base node and the 3 weights per axis. Returns 0 when
 * the 3x3x3 node set lies inside the grid. */
static int stencil(const orc_sim *s, const double xp[3], int64_t base[3], double w[3][3])
{
    for (int a = 0; a < 3; ++a) {
        double xi = (xp[a] - s->cfg.grid_origin[a]) / s->cfg.dx;
        if (!isfinite(xi)) return ORC_E_UNSTABLE;
        double b = floor(xi - 0.5);
        if (b < 0.0 || b + 2.0 > (double)(s->cfg.gn[a] - 1)) return ORC_E_OUT_OF_GRID;
        base[a] = (int64_t)b;
        for (int o = 0; o < 3; ++o) w[a][o] = orc_bspline(xi - (double)(base[a] + o));
    }
    return ORC_OK;
}

static int64_t node_index(const orc_sim *s, int64_t a, int64_t b, int64_t c)
{
    return a + (int64_t)s->cfg.gn[0] * (b + (int64_t)s->cfg.gn[1] * c);
}

/* ---------------------------------------------------------------- particle-to-grid */

/* Eqs. 2-5: clear the grid, then for every particle scatter mass w m_p (Eq. 2)
 * and momentum w (m_p v_p + m_p C_p (X_i - x_p)) (Eq. 4) minus
 * dt w V0 (4/dx^2) tau_p (X_i - x_p) (Eq. 5) to its 3x3x3 nodes. */
int orc_p2g(orc_sim *s, double dt)
{
    int status = ORC_OK;
    const double dx = s->cfg.dx, Dinv = 4.0 / (dx * dx);
    memset(s->M, 0, (size_t)s->nn * sizeof(double));
    memset(s->P, 0, (size_t)s->nn * 3 * sizeof(double));
    for (int64_t p = 0; p < s->N; ++p) {
        const double *xp = s->x + p * 3, *vp = s->v + p * 3, *Cp = s->C + p * 9, *Fp = s->F + p * 9;
        int64_t base[3];
        double w[3][3];
        int st = stencil(s, xp, base, w);
        if (st != ORC_OK) { status = st; continue; }
        double tau[9];
        st = orc_stress(s->cfg.model, s->mu, s->lambda, Fp, tau);
        if (st != ORC_OK) { status = st; continue; }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    int64_t q = node_index(s, base[0] + a, base[1] + b, base[2] + c);
                    double X[3] = {s->cfg.grid_origin[0] + (base[0] + a) * dx,
                                   s->cfg.grid_origin[1] + (base[1] + b) * dx,
                                   s->cfg.grid_origin[2] + (base[2] + c) * dx};
                    double d[3] = {X[0] - xp[0], X[1] - xp[1], X[2] - xp[2]};
                    double wt = w[0][a] * w[1][b] * w[2][c];
                    s->M[q] += wt * s->m;
                    for (int r = 0; r < 3; ++r) {
                        double Cd = Cp[r * 3 + 0] * d[0] + Cp[r * 3 + 1] * d[1] + Cp[r * 3 + 2] * d[2];
                        double td = tau[r * 3 + 0] * d[0] + tau[r * 3 + 1] * d[1] + tau[r * 3 + 2] * d[2];
                        double mm = wt * (s->m * vp[r] + s->m * Cd);        /* Eq. 4 */
                        double me = -dt * Dinv * wt * s->V0 * td;           /* Eq. 5 */
                        s->P[q * 3 + r] += mm + me;                         /* Eq. 3 */
                    }
                }
    }
    return status;
}

/* ---------------------------------------------------------------- grid update */

void orc_set_contact(orc_sim *s, int model, double mu)
{
    s->contact = model;
    s->friction = mu;
}

/* The indenter as particles (Eq. 10's set I, the object's point cloud):
 * n points in the indenter frame, each of mass `mass`; n = 0 returns to the
 * implicit solid. */
int orc_set_indenter_points(orc_sim *s, const double *xyz, int64_t n, double mass)
{
    free(s->ipts);
    s->ipts = NULL;
    s->ni = 0;
    if (n <= 0) return ORC_OK;
    s->ipts = (double *)malloc((size_t)n * 3 * sizeof(double));
    if (!s->MI) s->MI = (double *)calloc((size_t)s->nn, sizeof(double));
    if (!s->ipts || !s->MI) return ORC_E_ARG;
    memcpy(s->ipts, xyz, (size_t)n * 3 * sizeof(double));
    s->ni = n;
    s->imass = mass;
    return ORC_OK;
}

void orc_indenter_mass(const orc_sim *s, double *out)
{
    for (int64_t q = 0; q < s->nn; ++q) out[q] = s->MI ? s->MI[q] : 0.0;
}

/* Mass of the particle indenter on the grid: every point placed rigidly at
 * the pose of the substep's start scatters w m_I to its 3x3x3 nodes (the
 * weights of Eq. 2); points whose nodes leave the grid are ignored. */
static void scatter_indenter(orc_sim *s)
{
    double R[9];
    quat_to_matrix(s->pose + 3, R);
    memset(s->MI, 0, (size_t)s->nn * sizeof(double));
    for (int64_t k = 0; k < s->ni; ++k) {
        const double *l = s->ipts + k * 3;
        double X[3], w[3][3];
        int64_t base[3];
        for (int r = 0; r < 3; ++r) X[r] = s->pose[r] + R[r * 3 + 0] * l[0] + R[r * 3 + 1] * l[1] + R[r * 3 + 2] * l[2];
        if (stencil(s, X, base, w) != ORC_OK) continue;
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a)
                    s->MI[node_index(s, base[0] + a, base[1] + b, base[2] + c)] += w[0][a] * w[1][b] * w[2][c] * s->imass;
    }
}

/* Outward unit normal of the posed indenter at world point X: the gradient
 * of its signed distance by central differences of step eps along the world
 * axes. Returns 0 where the gradient vanishes. */
static int contact_normal(const orc_sim *s, const double X[3], double eps, double n[3])
{
    double g[3], norm = 0.0;
    for (int k = 0; k < 3; ++k) {
        double a[3] = {X[0], X[1], X[2]}, b[3] = {X[0], X[1], X[2]};
        a[k] += eps;
        b[k] -= eps;
        g[k] = (phi_world(s, s->pose, a) - phi_world(s, s->pose, b)) / (2.0 * eps);
        norm += g[k] * g[k];
    }
    norm = sqrt(norm);
    if (!(norm > 1e-12)) return 0;
    for (int k = 0; k < 3; ++k) n[k] = g[k] / norm;
    return 1;
}

/* Eq. 6 plus gravity, then the rigid-indenter contact (Eq. 10's indenter
 * case, applied at the nodes inside the indenter at the start pose), the
 * held floor and the grid walls. The contact reaction on the indenter is
 * sum M (V_before - V_after) / dt over the contact nodes. No-slip contact
 * gives a contact node the indenter's velocity. Coulomb contact (friction is
 * left to future work in the paper) takes the node's velocity relative to the
 * indenter, u = V - v_ind, and the outward normal n: if u.n >= 0 the node
 * moves apart and keeps V; otherwise the normal part of u is removed and the
 * tangential part u_t scaled by max(0, 1 - mu |u.n| / |u_t|) (zero if u_t is
 * zero), i.e. sliding against a friction bounded by mu times the normal
 * impulse, or sticking. */
int orc_grid_update(orc_sim *s, const double pose_end[7], double dt)
{
    const double dx = s->cfg.dx;
    const int wall = s->cfg.wall_nodes;
    s->force[0] = s->force[1] = s->force[2] = 0.0;
    if (s->ni > 0) scatter_indenter(s);
    for (int64_t c = 0; c < s->cfg.gn[2]; ++c)
        for (int64_t b = 0; b < s->cfg.gn[1]; ++b)
            for (int64_t a = 0; a < s->cfg.gn[0]; ++a) {
                int64_t q = node_index(s, a, b, c);
                double *V = s->V + q * 3;
                if (!(s->M[q] > 0.0)) {
                    V[0] = V[1] = V[2] = 0.0;
                    continue;
                }
                for (int r = 0; r < 3; ++r) V[r] = s->P[q * 3 + r] / s->M[q] + dt * s->cfg.gravity[r];
                double X[3] = {s->cfg.grid_origin[0] + a * dx, s->cfg.grid_origin[1] + b * dx,
                               s->cfg.grid_origin[2] + c * dx};
                if (s->ni > 0) {
                    /* particle indenter: its points move with the rigid velocity
                     * (Eq. 10), so their momentum on node i is M_I v_ind(X_i) (APIC
                     * with the rigid body's velocity gradient is exact for it), and
                     * the node's velocity is that of the summed momentum */
                    if (s->MI[q] > 0.0) {
                        double vi[3];
                        orc_indenter_velocity(s->pose, pose_end, dt, X, vi);
                        for (int r = 0; r < 3; ++r) {
                            const double after = (s->M[q] * V[r] + s->MI[q] * vi[r]) / (s->M[q] + s->MI[q]);
                            s->force[r] += s->M[q] * (V[r] - after) / dt;
                            V[r] = after;
                        }
                    }
                } else if (s->cfg.shape >= 0 && phi_world(s, s->pose, X) <= 0.0) {
                    double vi[3], after[3] = {0.0, 0.0, 0.0}, n[3];
                    orc_indenter_velocity(s->pose, pose_end, dt, X, vi);
                    for (int r = 0; r < 3; ++r) after[r] = vi[r];
                    if (s->contact == 1 && contact_normal(s, X, 1e-3 * dx, n)) {
                        double u[3], un = 0.0;
                        for (int r = 0; r < 3; ++r) {
                            u[r] = V[r] - vi[r];
                            un += u[r] * n[r];
                        }
                        if (un >= 0.0) {
                            for (int r = 0; r < 3; ++r) after[r] = V[r];
                        } else {
                            double ut[3], tn = 0.0;
                            for (int r = 0; r < 3; ++r) {
                                ut[r] = u[r] - un * n[r];
                                tn += ut[r] * ut[r];
                            }
                            tn = sqrt(tn);
                            double k = tn > 0.0 ? 1.0 + s->friction * un / tn : 0.0;
                            if (k < 0.0) k = 0.0;
                            for (int r = 0; r < 3; ++r) after[r] = vi[r] + k * ut[r];
                        }
                    }
                    for (int r = 0; r < 3; ++r) {
                        s->force[r] += s->M[q] * (V[r] - after[r]) / dt;
                        V[r] = after[r];
                    }
                }
                if (c <= s->cfg.floor_node) V[0] = V[1] = V[2] = 0.0;
                int64_t idx[3] = {a, b, c};
                for (int r = 0; r < 3; ++r) {
                    if (idx[r] < wall && V[r] < 0.0) V[r] = 0.0;
                    if (idx[r] > s->cfg.gn[r] - 1 - wall && V[r] > 0.0) V[r] = 0.0;
                }
            }
    return ORC_OK;
}

/* ---------------------------------------------------------------- grid-to-particle */

/* Eqs. 7-9 (with the V_i reading of Eq. 8), Eq. 10's bottom-layer case and
 * the advection of Eq. 11. */
int orc_g2p(orc_sim *s, double dt)
{
    int status = ORC_OK;
    const double dx = s->cfg.dx, Dinv = 4.0 / (dx * dx);
    const int64_t layer_size = (int64_t)s->cfg.n[0] * s->cfg.n[1];
    for (int64_t p = 0; p < s->N; ++p) {
        double *xp = s->x + p * 3, *vp = s->v + p * 3, *Cp = s->C + p * 9, *Fp = s->F + p * 9;
        int64_t base[3];
        double w[3][3];
        int st = stencil(s, xp, base, w);
        if (st != ORC_OK) { status = st; continue; }
        double vn[3] = {0, 0, 0}, B[9] = {0};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    int64_t q = node_index(s, base[0] + a, base[1] + b, base[2] + c);
                    double X[3] = {s->cfg.grid_origin[0] + (base[0] + a) * dx,
                                   s->cfg.grid_origin[1] + (base[1] + b) * dx,
                                   s->cfg.grid_origin[2] + (base[2] + c) * dx};
                    double d[3] = {X[0] - xp[0], X[1] - xp[1], X[2] - xp[2]};
                    double wt = w[0][a] * w[1][b] * w[2][c];
                    const double *Vq = s->V + q * 3;
                    for (int r = 0; r < 3; ++r) {
                        vn[r] += wt * Vq[r];                                  /* Eq. 7 */
                        for (int cc = 0; cc < 3; ++cc) B[r * 3 + cc] += wt * Vq[r] * d[cc];
                    }
                }
        double Cn[9], G[9], Fn[9];
        for (int k = 0; k < 9; ++k) Cn[k] = Dinv * B[k];                      /* Eq. 8 */
        for (int k = 0; k < 9; ++k) G[k] = (k % 4 == 0 ? 1.0 : 0.0) + dt * Cn[k];
        mat_mul(G, Fp, Fn);                                                   /* Eq. 9 */
        if (p / layer_size < s->cfg.n_fixed_layers) vn[0] = vn[1] = vn[2] = 0.0; /* Eq. 10 */
        for (int r = 0; r < 3; ++r) {
            vp[r] = vn[r];
            xp[r] = xp[r] + dt * vn[r];                                       /* Eq. 11 */
        }
        memcpy(Cp, Cn, sizeof Cn);
        memcpy(Fp, Fn, sizeof Fn);
        if (!isfinite(xp[0] + xp[1] + xp[2])) status = ORC_E_UNSTABLE;
    }
    return status;
}

int orc_step(orc_sim *s, const double pose_end[7], double dt)
{
    int st = orc_p2g(s, dt);
    int st2 = orc_grid_update(s, pose_end, dt);
    int st3 = orc_g2p(s, dt);
    memcpy(s->pose, pose_end, sizeof s->pose);
    if (st != ORC_OK) return st;
    if (st2 != ORC_OK) return st2;
    return st3;
}

void orc_get_grid(const orc_sim *s, double *M, double *P, double *V)
{
    if (M) memcpy(M, s->M, (size_t)s->nn * sizeof(double));
    if (P) memcpy(P, s->P, (size_t)s->nn * 3 * sizeof(double));
    if (V) memcpy(V, s->V, (size_t)s->nn * 3 * sizeof(double));
}

void orc_force(const orc_sim *s, double f[3])
{
    f[0] = s->force[0]; f[1] = s->force[1]; f[2] = s->force[2];
}

/* ---------------------------------------------------------------- depth map and image */

/* Surface depth map (Sec. III-B): the z of each top-layer particle, indexed
 * by its lattice position (i, j). */
void orc_heightmap(const orc_sim *s, double *H)
{
    const int n0 = s->cfg.n[0], n1 = s->cfg.n[1], k = s->cfg.n[2] - 1;
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n0; ++i) {
            int64_t p = i + (int64_t)n0 * (j + (int64_t)n1 * k);
            H[(int64_t)j * n0 + i] = s->x[p * 3 + 2];
        }
}

/* Tactile image (Sec. III-B, Eqs. 12-14): the depth map is resampled
 * bilinearly at the pixel centres of an h x w crop centred on the block's top
 * face (rest coordinates, pitch r), the normal is (dH/dx, dH/dy, -1)
 * normalised with central differences [-1, 0, 1]/(2r) (replicated border),
 * and each RGB channel is lit by its own distant light with the Phong model:
 * ka ia + kd max(L.N, 0) + ks max(R.V, 0)^alpha (specular only where L.N > 0),
 * R = 2 (L.N) N - L, V = (0, 0, -1) toward the camera below the gel, clamped
 * to [0, 1]. */
void orc_render_height(const orc_config *cfg, const double *H, const orc_render_params *rp,
                       int32_t h, int32_t w, double *rgb)
{
    const int n0 = cfg->n[0], n1 = cfg->n[1];
    const double hx = cfg->block_size[0] / n0, hy = cfg->block_size[1] / n1;
    const double cx = cfg->block_origin[0] + 0.5 * cfg->block_size[0];
    const double cy = cfg->block_origin[1] + 0.5 * cfg->block_size[1];
    const double r = rp->pitch;
    double *img = (double *)malloc((size_t)h * w * sizeof(double));
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            double X = cx + (u - 0.5 * (w - 1)) * r, Y = cy + (v - 0.5 * (h - 1)) * r;
            double sx = (X - (cfg->block_origin[0] + 0.5 * hx)) / hx;
            double sy = (Y - (cfg->block_origin[1] + 0.5 * hy)) / hy;
            double fi = floor(sx), fj = floor(sy);
            if (fi < 0) fi = 0;
            if (fi > n0 - 2) fi = n0 - 2;
            if (fj < 0) fj = 0;
            if (fj > n1 - 2) fj = n1 - 2;
            double tx = sx - fi, ty = sy - fj;
            if (tx < 0) tx = 0;
            if (tx > 1) tx = 1;
            if (ty < 0) ty = 0;
            if (ty > 1) ty = 1;
            int i0 = (int)fi, j0 = (int)fj;
            double h00 = H[(int64_t)j0 * n0 + i0], h10 = H[(int64_t)j0 * n0 + i0 + 1];
            double h01 = H[(int64_t)(j0 + 1) * n0 + i0], h11 = H[(int64_t)(j0 + 1) * n0 + i0 + 1];
            img[(int64_t)v * w + u] = (1 - ty) * ((1 - tx) * h00 + tx * h10) + ty * ((1 - tx) * h01 + tx * h11);
        }
    const double el = rp->light_elev_deg * M_PI / 180.0;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            int ul = u > 0 ? u - 1 : 0, ur = u < w - 1 ? u + 1 : w - 1;
            int vd = v > 0 ? v - 1 : 0, vu = v < h - 1 ? v + 1 : h - 1;
            double gx = (img[(int64_t)v * w + ur] - img[(int64_t)v * w + ul]) / (2.0 * r);
            double gy = (img[(int64_t)vu * w + u] - img[(int64_t)vd * w + u]) / (2.0 * r);
            double nrm = sqrt(gx * gx + gy * gy + 1.0);
            double N[3] = {gx / nrm, gy / nrm, -1.0 / nrm};
            const double V[3] = {0.0, 0.0, -1.0};
            for (int ch = 0; ch < 3; ++ch) {
                double az = rp->light_azim_deg[ch] * M_PI / 180.0;
                double L[3] = {cos(el) * cos(az), cos(el) * sin(az), -sin(el)};
                double LN = L[0] * N[0] + L[1] * N[1] + L[2] * N[2];
                double I = rp->ka_ia;
                if (LN > 0.0) {
                    I += rp->kd * LN;
                    double R[3] = {2 * LN * N[0] - L[0], 2 * LN * N[1] - L[1], 2 * LN * N[2] - L[2]};
                    double RV = R[0] * V[0] + R[1] * V[1] + R[2] * V[2];
                    if (RV > 0.0) I += rp->ks * pow(RV, rp->alpha);
                }
                if (I < 0.0) I = 0.0;
                if (I > 1.0) I = 1.0;
                rgb[((int64_t)v * w + u) * 3 + ch] = I;
            }
        }
    free(img);
}

void orc_render(const orc_sim *s, const orc_render_params *rp, int32_t h, int32_t w, double *rgb)
{
    double *H = (double *)malloc((size_t)s->cfg.n[0] * s->cfg.n[1] * sizeof(double));
    orc_heightmap(s, H);
    orc_render_height(&s->cfg, H, rp, h, w, rgb);
    free(H);
}
