// Host side of libtacchi: configuration checks, workspace carving, per-step
// indenter kinematics and kernel launches on the caller's HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tacchi.h"
#include "sim_kernels.hpp"

using namespace tacchi;

namespace {

thread_local std::string g_last_error;

tacchi_status fail(tacchi_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define TC_HIP(expr)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(TACCHI_E_DEVICE, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define TC_LAUNCHED()                                                                            \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess)                                                                    \
            return fail(TACCHI_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;

// Sizes and material constants derived from a validated configuration.
struct Derived {
    int64_t N = 0;
    int n[3] = {0, 0, 0};
    int g[3] = {0, 0, 0};
    int B = 8;
    int nb[3] = {0, 0, 0};
    int nblk = 0;
    int64_t nodes = 0;
    double dx = 0, h[3] = {0, 0, 0}, m = 0, V0 = 0, mu = 0, lambda = 0, cp = 0;
    double xr[3] = {0, 0, 0};
    int floor_node = 0;
    size_t es = 8;
    int ts[3] = {0, 0, 0};   // lattice tile shift (see SimDev)
    int nt[3] = {0, 0, 0};   // lattice tiles per axis
    int64_t Ns = 0;          // particle slots
    int cap = 0;             // bin-list entries per grid block
};

struct Layout {
    size_t u, v, H, A, cnt[2], perm[2], tiles, V, err, force, fallback, stop, hmap, total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(const Derived &d)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    const size_t Ns = (size_t)d.Ns, es = d.es;
    L.u = take(3 * Ns * es);
    L.v = take(3 * Ns * es);
    L.H = take(9 * Ns * es);
    L.A = take(9 * Ns * es);
    for (int k = 0; k < 2; ++k) {
        L.cnt[k] = take((size_t)d.nblk * 4);
        L.perm[k] = take((size_t)d.nblk * d.cap * 4);
    }
    const size_t tb = (size_t)d.B + 3;
    L.tiles = take((size_t)d.nblk * tb * tb * tb * 4 * es);
    L.V = take((size_t)d.nodes * 3 * es);
    L.err = take(64);
    L.force = take(64);
    L.fallback = take(64);
    L.stop = take(64);
    L.hmap = take((size_t)d.n[0] * d.n[1] * es);
    L.total = o;
    return L;
}

tacchi_status check_indenter(const tacchi_indenter &ind)
{
    switch (ind.shape) {
    case TACCHI_NO_INDENTER:
        return TACCHI_OK;
    case TACCHI_SPHERE:
    case TACCHI_CYLINDER:
        if (!(ind.p[0] > 0)) return fail(TACCHI_E_ARG, "indenter radius must be > 0");
        return TACCHI_OK;
    case TACCHI_CONE:
    case TACCHI_EDGE:
        if (!(ind.p[0] > 0 && ind.p[0] < 0.5 * kPi)) return fail(TACCHI_E_ARG, "half-angle must be in (0, pi/2)");
        if (!(ind.p[1] >= 0)) return fail(TACCHI_E_ARG, "tip radius must be >= 0");
        return TACCHI_OK;
    case TACCHI_TEXTURED_PLATE:
        if (!(ind.p[0] > 0 && ind.p[2] > 0 && ind.p[1] >= 0))
            return fail(TACCHI_E_ARG, "plate needs half-width > 0, amplitude >= 0, wavelength > 0");
        return TACCHI_OK;
    default:
        return fail(TACCHI_E_ARG, "unknown indenter shape");
    }
}

tacchi_status derive(const tacchi_config *c, Derived *d)
{
    if (!c) return fail(TACCHI_E_ARG, "config is NULL");
    if (c->precision != TACCHI_F64 && c->precision != TACCHI_F32) return fail(TACCHI_E_ARG, "bad precision");
    if (c->mat.model != TACCHI_NEOHOOKEAN && c->mat.model != TACCHI_COROTATED)
        return fail(TACCHI_E_ARG, "bad material model");
    if (c->tile != 0 && c->tile != 4 && c->tile != 8) return fail(TACCHI_E_ARG, "tile must be 0, 4 or 8");
    if (!(c->mat.E > 0) || !(c->mat.nu >= 0 && c->mat.nu < 0.5) || !(c->mat.rho > 0))
        return fail(TACCHI_E_ARG, "material needs E > 0, 0 <= nu < 0.5, rho > 0");
    if (!(c->grid.dx > 0)) return fail(TACCHI_E_ARG, "grid dx must be > 0");
    const double dx = c->grid.dx;
    int64_t N = 1, nodes = 1;
    for (int a = 0; a < 3; ++a) {
        if (c->block.n[a] < 2) return fail(TACCHI_E_ARG, "lattice needs >= 2 particles per axis");
        if (c->grid.n[a] < 7) return fail(TACCHI_E_ARG, "grid needs >= 7 nodes per axis");
        if (c->grid.n[a] > (1 << 16)) return fail(TACCHI_E_ARG, "grid needs <= 65536 nodes per axis");
        if (!(c->block.size[a] > 0)) return fail(TACCHI_E_ARG, "block size must be > 0");
        N *= c->block.n[a];
        nodes *= c->grid.n[a];
        d->h[a] = c->block.size[a] / c->block.n[a];
        if (dx < d->h[a] * (1 - 1e-9)) return fail(TACCHI_E_ARG, "grid spacing must be >= lattice spacing");
        const double lo = (c->block.origin[a] - c->grid.origin[a]) / dx;
        const double hi = (c->block.origin[a] + c->block.size[a] - c->grid.origin[a]) / dx;
        if (lo < 3 - 1e-9 || hi > (c->grid.n[a] - 1 - 3) + 1e-9)
            return fail(TACCHI_E_ARG, "grid must enclose the block with >= 3 nodes of margin on every side");
        d->n[a] = c->block.n[a];
        d->g[a] = c->grid.n[a];
        d->xr[a] = lo + 0.5 * d->h[a] / dx;
    }
    if (N >= (int64_t)1 << 31) return fail(TACCHI_E_ARG, "too many particles (limit 2^31 - 1)");
    const double z0 = (c->block.origin[2] - c->grid.origin[2]) / dx;
    if (std::fabs(z0 - std::round(z0)) > 1e-6) return fail(TACCHI_E_ARG, "block bottom face must lie on a grid node plane");
    if (c->n_fixed_layers < 1 || c->n_fixed_layers > c->block.n[2])
        return fail(TACCHI_E_ARG, "n_fixed_layers must be in [1, n2]");
    tacchi_status st = check_indenter(c->ind);
    if (st != TACCHI_OK) return st;
    const double *q = c->pose0.quat;
    if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 0)) return fail(TACCHI_E_ARG, "pose0 quaternion is zero");
    d->N = N;
    d->dx = dx;
    d->B = c->tile == 0 ? 8 : c->tile;
    int64_t nblk = 1;
    for (int a = 0; a < 3; ++a) {
        d->nb[a] = (d->g[a] + d->B - 1) / d->B;
        nblk *= d->nb[a];
    }
    // node indices (and four values per node) stay within 32-bit arithmetic
    if (nblk * d->B * d->B * d->B >= (int64_t)1 << 29)
        return fail(TACCHI_E_ARG, "too many grid nodes (limit 2^29 after rounding up to whole blocks)");
    d->nblk = (int)nblk;
    d->nodes = nblk * d->B * d->B * d->B;
    d->V0 = d->h[0] * d->h[1] * d->h[2];
    d->m = c->mat.rho * d->V0;
    d->mu = c->mat.E / (2 * (1 + c->mat.nu));
    d->lambda = c->mat.E * c->mat.nu / ((1 + c->mat.nu) * (1 - 2 * c->mat.nu));
    d->cp = std::sqrt((d->lambda + 2 * d->mu) / c->mat.rho);
    d->floor_node = (int)std::lround(z0);
    d->es = c->precision == TACCHI_F64 ? 8 : 4;
    // particle tiles aligned with the grid blocks at rest
    d->Ns = 1;
    double ppc = 1.0;
    for (int a = 0; a < 3; ++a) {
        const long cell0 = (long)std::floor(d->xr[a]);  // grid cell of lattice index 0 at rest
        d->ts[a] = (int)(((cell0 % d->B) + d->B) % d->B);
        d->nt[a] = (d->n[a] + d->ts[a] + d->B - 1) / d->B;
        d->Ns *= (int64_t)d->nt[a] * d->B;
        ppc *= dx / d->h[a];
    }
    if (d->Ns >= (int64_t)1 << 31) return fail(TACCHI_E_ARG, "too many particle slots (limit 2^31 - 1)");
    // bin capacity: 2.5x the rest particle count of a block (a block's
    // particles would need to be compressed to J < 0.4 to overflow it)
    const double c0 = 2.5 * ppc * d->B * d->B * d->B;
    d->cap = (int)(std::ceil(std::max(64.0, c0) / 64.0) * 64.0);
    (void)nodes;
    return TACCHI_OK;
}

void quat_normalise(const double q[4], double out[4])
{
    const double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) out[k] = q[k] / n;
}

void quat_matrix(const double qin[4], double R[9])
{
    double q[4];
    quat_normalise(qin, q);
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

// Angular velocity of the rigid rotation taking q0 to q1 over dt (shortest arc).
void angular_velocity(const double q0in[4], const double q1in[4], double dt, double om[3])
{
    double a[4], b[4];
    quat_normalise(q0in, a);
    quat_normalise(q1in, b);
    // r = b * conj(a)
    const double rw = b[0] * a[0] + b[1] * a[1] + b[2] * a[2] + b[3] * a[3];
    const double rx = -b[0] * a[1] + b[1] * a[0] - b[2] * a[3] + b[3] * a[2];
    const double ry = -b[0] * a[2] + b[1] * a[3] + b[2] * a[0] - b[3] * a[1];
    const double rz = -b[0] * a[3] - b[1] * a[2] + b[2] * a[1] + b[3] * a[0];
    double s = rw < 0 ? -1.0 : 1.0;
    const double vx = s * rx, vy = s * ry, vz = s * rz, w = s * rw;
    const double vn = std::sqrt(vx * vx + vy * vy + vz * vz);
    if (vn == 0.0) {
        om[0] = om[1] = om[2] = 0.0;
        return;
    }
    const double ang = 2.0 * std::atan2(vn, w);
    om[0] = vx / vn * ang / dt;
    om[1] = vy / vn * ang / dt;
    om[2] = vz / vn * ang / dt;
}

template <typename T>
IndenterDev<T> make_indenter(const tacchi_config &cfg, const double pose0[7], const double pose1[7], double dt)
{
    IndenterDev<T> I{};
    const tacchi_indenter &ind = cfg.ind;
    I.shape = ind.shape;
    I.seed = ind.seed;
    for (int k = 0; k < 4; ++k) I.p[k] = T(0);
    if (ind.shape == TACCHI_CONE || ind.shape == TACCHI_EDGE) {
        I.p[0] = T(std::sin(ind.p[0]));
        I.p[1] = T(std::cos(ind.p[0]));
        I.p[2] = T(ind.p[1]);
    } else {
        for (int k = 0; k < 3; ++k) I.p[k] = T(ind.p[k]);
    }
    // every solid lies above its tip plane z = 0 of the indenter frame; the
    // plate's textured face reaches down to -2 amplitudes (|noise| <= 2: a
    // blend of corner terms g.d with |g|, |d| <= sqrt 2). A 1 nm margin keeps
    // the test clear of rounding, so it only skips points that the full
    // signed distance puts outside.
    I.zmin = T(-(ind.shape == TACCHI_TEXTURED_PLATE ? 2.0 * ind.p[1] : 0.0) - 1e-9);
    const double dx = cfg.grid.dx;
    I.dx = T(dx);
    double R[9], om[3];
    quat_matrix(pose0 + 3, R);
    angular_velocity(pose0 + 3, pose1 + 3, dt, om);
    for (int k = 0; k < 9; ++k) I.R[k] = T(R[k]);
    for (int a = 0; a < 3; ++a) {
        I.tip[a] = T((pose0[a] - cfg.grid.origin[a]) / dx);
        I.vc[a] = T((pose1[a] - pose0[a]) / dt / dx);
        I.om[a] = T(om[a]);
    }
    return I;
}

}  // namespace

struct tacchi_sim {
    tacchi_config cfg;
    Derived d;
    Layout L;
    int device = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    double pose[7];
    double pending[7];
    int phase = 0;        // 0: ready for P2G, 1: P2G done, 2: grid updated
    int parity = 0;       // which bin buffers hold the current substep's lists
    bool stop_armed = false;  // substep kernels honour the stop flag (tacchi_run_until_force)
    int contact_model = TACCHI_CONTACT_STICKY;
    double friction = 0.0;    // Coulomb coefficient (TACCHI_CONTACT_COULOMB)
    // particle indenter (tacchi_set_indenter_points): device buffers owned by the handle
    double *ipts = nullptr;   // [ni][3] points, indenter frame [m]
    int ni = 0;
    double imass = 0.0;       // mass per point [kg]
    double *MI = nullptr;     // indenter mass per grid node
    double plo[3], phi_[3];   // bounding box of the points, indenter frame [m]
    double dtA = 0.0;     // dt the stored affine matrices were formed with
    double dt_phase = 0.0;
    SimDev<float> sf;
    SimDev<double> sd;
    void *stage = nullptr;  // pinned host staging for host-side arguments
    size_t stage_bytes = 0;
    int64_t g2p_count = 0;    // G2P launches so far (every kSortEvery-th sorts the bin lists)
    // kernel timing (see tacchi_timing_enable)
    uint32_t timing_mask = 0;
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<Pending> timed;
    std::vector<hipEvent_t> event_pool;
    double timing_ms[TACCHI_NUM_KERNEL_CLASSES] = {0};
    int64_t timing_n[TACCHI_NUM_KERNEL_CLASSES] = {0};
};

namespace {

enum { KC_BIN = 0, KC_P2G = 1, KC_GRID = 2, KC_G2P = 3, KC_HEIGHT = 4, KC_RENDER = 5 };

hipEvent_t pool_event(tacchi_sim *s)
{
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one kernel launch with events when its class is being timed.
struct KernelTimer {
    tacchi_sim *s;
    int cls;
    hipEvent_t a = nullptr;
    KernelTimer(tacchi_sim *s_, int cls_) : s(s_), cls(cls_)
    {
        if (s->timing_mask & (1u << cls)) {
            a = pool_event(s);
            if (a) (void)hipEventRecord(a, s->stream);
        }
    }
    ~KernelTimer()
    {
        if (!a) return;
        hipEvent_t b = pool_event(s);
        if (!b) return;
        (void)hipEventRecord(b, s->stream);
        s->timed.push_back({cls, a, b});
    }
};

// The box of grid blocks that hold the particles at rest: blocks lo[a] ..
// lo[a] + n[a] - 1 per axis (block_key of the first and last lattice
// position).
void rest_block_box(const Derived &d, int lo[3], int n[3])
{
    for (int a = 0; a < 3; ++a) {
        const auto blk = [&](double x) {
            const int cell = std::min(std::max((int)std::floor(x), 0), d.g[a] - 1);
            return std::min(cell / d.B, d.nb[a] - 1);
        };
        lo[a] = blk(d.xr[a]);
        n[a] = blk(d.xr[a] + (d.n[a] - 1) * d.h[a] / d.dx) - lo[a] + 1;
    }
}

template <typename T>
SimDev<T> make_simdev(tacchi_sim *s)
{
    const Derived &d = s->d;
    const Layout &L = s->L;
    SimDev<T> S{};
    S.N = d.N;
    S.Ns = d.Ns;
    S.n0 = d.n[0]; S.n1 = d.n[1]; S.n2 = d.n[2];
    S.g0 = d.g[0]; S.g1 = d.g[1]; S.g2 = d.g[2];
    S.nb0 = d.nb[0]; S.nb1 = d.nb[1]; S.nb2 = d.nb[2];
    S.nblk = d.nblk;
    // the blocks that hold the particles at rest are dispatched first
    {
        int lo[3], n[3];
        rest_block_box(d, lo, n);
        S.bx0 = lo[0]; S.by0 = lo[1]; S.bz0 = lo[2];
        S.bxn = n[0]; S.byn = n[1]; S.bzn = n[2];
        S.box_chunk = 3 * n[0];
        int hl[3], hn[3];
        for (int a = 0; a < 3; ++a) {
            hl[a] = std::max(lo[a] - 1, 0);
            hn[a] = std::min(lo[a] + n[a] + 1, d.nb[a]) - hl[a];
        }
        S.hx0 = hl[0]; S.hy0 = hl[1]; S.hz0 = hl[2];
        S.hxn = hn[0]; S.hyn = hn[1]; S.hzn = hn[2];
        S.halo_chunk = 3 * hn[0];
    }
    S.ts0 = d.ts[0]; S.ts1 = d.ts[1]; S.ts2 = d.ts[2];
    S.nt0 = d.nt[0]; S.nt1 = d.nt[1]; S.nt2 = d.nt[2];
    S.div_nt0 = make_fastdiv((uint32_t)d.nt[0]);
    S.div_nt1 = make_fastdiv((uint32_t)d.nt[1]);
    S.div_n0 = make_fastdiv((uint32_t)d.n[0]);
    S.div_n1 = make_fastdiv((uint32_t)d.n[1]);
    S.cap = d.cap;
    for (int a = 0; a < 3; ++a) {
        S.xr[a] = T(d.xr[a]);
        S.hr[a] = T(d.h[a] / d.dx);
        S.grav[a] = T(s->cfg.gravity[a] / d.dx);
    }
    S.m = T(d.m);
    // FP32 grid nodes lighter than 2^-22 particle masses (64 units of the
    // fixed-point P2G accumulator) are treated as empty: their P/M carries
    // quantisation error of up to 1/64 cell per substep, and the weight they
    // carry into any particle is below 27 * 2^-22, so the velocity error they
    // would pass on stays under 2^-21 cells per substep.
    S.m_floor = sizeof(T) == 4 ? T(d.m * 2.384185791015625e-07) : T(0);
    S.vcoef = T(d.V0 * 4.0 / (d.dx * d.dx));
    S.mu = T(d.mu);
    S.lambda = T(d.lambda);
    S.floor_node = d.floor_node;
    S.wall = 3;
    S.n_fixed = s->cfg.n_fixed_layers;
    char *w = s->ws;
    S.u = (T *)(w + L.u);
    S.v = (T *)(w + L.v);
    S.H = (T *)(w + L.H);
    S.A = (T *)(w + L.A);
    S.cnt_cur = (int *)(w + L.cnt[s->parity]);
    S.cnt_next = (int *)(w + L.cnt[s->parity ^ 1]);
    S.perm_cur = (int *)(w + L.perm[s->parity]);
    S.perm_next = (int *)(w + L.perm[s->parity ^ 1]);
    S.tiles = (T *)(w + L.tiles);
    S.V = (T *)(w + L.V);
    S.err = (int *)(w + L.err);
    S.force = (double *)(w + L.force);
    S.fallback = (unsigned int *)(w + L.fallback);
    S.stop = s->stop_armed ? (const int *)(w + L.stop) : nullptr;
    return S;
}

unsigned grid1d(int64_t n) { return (unsigned)((n + kWG - 1) / kWG); }

template <typename T>
SimDev<T> &sdev(tacchi_sim *s);
template <>
SimDev<float> &sdev<float>(tacchi_sim *s) { return s->sf; }
template <>
SimDev<double> &sdev<double>(tacchi_sim *s) { return s->sd; }

template <typename T>
tacchi_status zero_bytes(tacchi_sim *s, void *p, size_t bytes)
{
    // fill kernel (not hipMemsetAsync) so the sequence stays safe to capture
    const int64_t n = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_fill<int>, dim3(grid1d(n)), dim3(kWG), 0, s->stream, (int *)p, n, 0);
    TC_LAUNCHED();
    return TACCHI_OK;
}

template <typename T>
tacchi_status launch_bin(tacchi_sim *s)
{
    SimDev<T> &S = sdev<T>(s);
    tacchi_status st = zero_bytes<T>(s, S.cnt_cur, (size_t)S.nblk * 4);
    if (st) return st;
    KernelTimer t(s, KC_BIN);
    if (s->d.B == 4)
        hipLaunchKernelGGL((k_bin<T, 4>), dim3(grid1d(S.Ns)), dim3(kWG), 0, s->stream, S);
    else
        hipLaunchKernelGGL((k_bin<T, 8>), dim3(grid1d(S.Ns)), dim3(kWG), 0, s->stream, S);
    TC_LAUNCHED();
    return TACCHI_OK;
}

// Accumulator units of P2G: FP32 tiles count one particle mass and one
// momentum unit m/dt as 2^28 (fixed point, see TileAcc); FP64 accumulates in
// SI/grid units directly.
struct P2GScales {
    double mscale, pscale, munit, punit;
};

P2GScales p2g_scales(const tacchi_sim *s, double dt)
{
    if (s->cfg.precision == TACCHI_F64) return {1.0, 1.0, 1.0, 1.0};
    const double one = kFixedUnits;
    const double m = s->d.m;
    return {one / m, one * dt / m, m / one, m / (one * dt)};
}

template <typename T, int B, bool FIX>
void launch_p2g_model(tacchi_sim *s, T fix, const P2GScales &k)
{
    SimDev<T> &S = sdev<T>(s);
    if (s->cfg.mat.model == TACCHI_NEOHOOKEAN)
        hipLaunchKernelGGL((k_p2g<T, B, FIX, 0>), dim3(S.nblk), dim3(kP2GWG), 0, s->stream, S, fix, T(k.mscale),
                           T(k.pscale), T(k.munit), T(k.punit));
    else
        hipLaunchKernelGGL((k_p2g<T, B, FIX, 1>), dim3(S.nblk), dim3(kP2GWG), 0, s->stream, S, fix, T(k.mscale),
                           T(k.pscale), T(k.munit), T(k.punit));
}

template <typename T, int B>
void launch_p2g_b(tacchi_sim *s, bool fix_dt, T fix, const P2GScales &k)
{
    if (fix_dt)
        launch_p2g_model<T, B, true>(s, fix, k);
    else
        launch_p2g_model<T, B, false>(s, fix, k);
}

template <typename T>
tacchi_status do_p2g(tacchi_sim *s, double dt)
{
    (void)sdev<T>(s);
    const bool fix_dt = dt != s->dtA;
    const T fix = T((dt - s->dtA) * s->d.V0 * 4.0 / (s->d.dx * s->d.dx));
    const P2GScales k = p2g_scales(s, dt);
    KernelTimer t(s, KC_P2G);
    if (s->d.B == 4)
        launch_p2g_b<T, 4>(s, fix_dt, fix, k);
    else
        launch_p2g_b<T, 8>(s, fix_dt, fix, k);
    TC_LAUNCHED();
    return TACCHI_OK;
}

template <typename T>
tacchi_status do_grid(tacchi_sim *s, const double pose_end[7], double dt)
{
    SimDev<T> &S = sdev<T>(s);
    IndenterDev<double> I = make_indenter<double>(s->cfg, s->pose, pose_end, dt);
    I.mu = s->friction;
    I.eps = 1e-3 * s->d.dx;
    const int contact = s->ni > 0 ? CONTACT_PARTICLES
                                  : (s->contact_model == TACCHI_CONTACT_COULOMB ? CONTACT_COULOMB : CONTACT_STICKY);
    KernelTimer t(s, KC_GRID);
    if (contact == CONTACT_PARTICLES) {
        // the points' mass on the grid at the substep's start pose, within the
        // node box of their stencils (the points' bounding box at that pose,
        // one node of slack for rounding); the grid update reads MI only there
        double R[9];
        quat_matrix(s->pose + 3, R);
        const int gdim[3] = {S.g0, S.g1, S.g2};
        int64_t nbox = 1;
        for (int a = 0; a < 3; ++a) {
            double lo = 1e300, hi = -1e300;
            for (int c = 0; c < 8; ++c) {
                const double l[3] = {(c & 1) ? s->phi_[0] : s->plo[0], (c & 2) ? s->phi_[1] : s->plo[1],
                                     (c & 4) ? s->phi_[2] : s->plo[2]};
                const double w = s->pose[a] + R[3 * a] * l[0] + R[3 * a + 1] * l[1] + R[3 * a + 2] * l[2];
                lo = std::min(lo, w);
                hi = std::max(hi, w);
            }
            const double glo = std::floor((lo - s->cfg.grid.origin[a]) / s->d.dx - 0.5) - 1.0;
            const double ghi = std::floor((hi - s->cfg.grid.origin[a]) / s->d.dx - 0.5) + 3.0;
            I.blo[a] = (int)std::max(0.0, std::min(glo, (double)gdim[a]));
            I.bhi[a] = (int)std::max(-1.0, std::min(ghi, (double)(gdim[a] - 1)));
            nbox *= std::max(0, I.bhi[a] - I.blo[a] + 1);
        }
        I.MI = s->MI;
        if (nbox > 0) {
            hipLaunchKernelGGL(k_clear_box, dim3(grid1d(nbox)), dim3(kWG), 0, s->stream, s->MI, S.g0, S.g1, I.blo[0],
                               I.blo[1], I.blo[2], I.bhi[0] - I.blo[0] + 1, I.bhi[1] - I.blo[1] + 1, nbox);
            hipLaunchKernelGGL(k_indenter_scatter, dim3(grid1d(s->ni)), dim3(kWG), 0, s->stream, s->ipts, s->ni, I,
                               S.g0, S.g1, S.g2, s->imass, s->MI);
        }
    }
    const dim3 g(S.nblk), b(kWG);
    if (s->d.B == 4) {
        if (contact == CONTACT_PARTICLES)
            hipLaunchKernelGGL((k_grid<T, 4, CONTACT_PARTICLES>), g, b, 0, s->stream, S, I, T(dt));
        else if (contact == CONTACT_COULOMB)
            hipLaunchKernelGGL((k_grid<T, 4, CONTACT_COULOMB>), g, b, 0, s->stream, S, I, T(dt));
        else
            hipLaunchKernelGGL((k_grid<T, 4, CONTACT_STICKY>), g, b, 0, s->stream, S, I, T(dt));
    } else {
        if (contact == CONTACT_PARTICLES)
            hipLaunchKernelGGL((k_grid<T, 8, CONTACT_PARTICLES>), g, b, 0, s->stream, S, I, T(dt));
        else if (contact == CONTACT_COULOMB)
            hipLaunchKernelGGL((k_grid<T, 8, CONTACT_COULOMB>), g, b, 0, s->stream, S, I, T(dt));
        else
            hipLaunchKernelGGL((k_grid<T, 8, CONTACT_STICKY>), g, b, 0, s->stream, S, I, T(dt));
    }
    TC_LAUNCHED();
    return TACCHI_OK;
}

template <typename T, bool SORT>
void launch_g2p(tacchi_sim *s, SimDev<T> &S, T dt, T coef)
{
    const bool neo = s->cfg.mat.model == TACCHI_NEOHOOKEAN;
    if (s->d.B == 4) {
        if (neo)
            hipLaunchKernelGGL((k_g2p<T, 4, 0, SORT>), dim3(S.nblk), dim3(kWG), 0, s->stream, S, dt, coef);
        else
            hipLaunchKernelGGL((k_g2p<T, 4, 1, SORT>), dim3(S.nblk), dim3(kWG), 0, s->stream, S, dt, coef);
    } else {
        if (neo)
            hipLaunchKernelGGL((k_g2p<T, 8, 0, SORT>), dim3(S.nblk), dim3(kWG), 0, s->stream, S, dt, coef);
        else
            hipLaunchKernelGGL((k_g2p<T, 8, 1, SORT>), dim3(S.nblk), dim3(kWG), 0, s->stream, S, dt, coef);
    }
}

template <typename T>
tacchi_status do_g2p(tacchi_sim *s, double dt)
{
    SimDev<T> &S = sdev<T>(s);
    const T coef = T(dt * s->d.V0 * 4.0 / (s->d.dx * s->d.dx));
    KernelTimer t(s, KC_G2P);
    // every kSortEvery-th G2P first sorts the bin lists by slot
    if (s->g2p_count++ % kSortEvery == kSortEvery - 1)
        launch_g2p<T, true>(s, S, T(dt), coef);
    else
        launch_g2p<T, false>(s, S, T(dt), coef);
    TC_LAUNCHED();
    return TACCHI_OK;
}

tacchi_status set_device(tacchi_sim *s)
{
    int cur = -1;
    TC_HIP(hipGetDevice(&cur));
    if (cur != s->device) TC_HIP(hipSetDevice(s->device));
    return TACCHI_OK;
}

tacchi_status check_dt(tacchi_sim *s, double dt)
{
    if (!(dt > 0) || !std::isfinite(dt)) return fail(TACCHI_E_ARG, "dt must be finite and > 0");
    const double cfl = dt * s->d.cp / s->d.dx;
    if (cfl > 1.0) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "dt above the CFL limit: dt*c_p/dx = %.4g > 1", cfl);
        return fail(TACCHI_E_UNSTABLE, buf);
    }
    return TACCHI_OK;
}

tacchi_status read_error_word(tacchi_sim *s)
{
    int h_err = 0;
    TC_HIP(hipMemcpyAsync(&h_err, s->ws + s->L.err, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    TC_HIP(hipStreamSynchronize(s->stream));
    if (h_err & ERR_OUT_OF_GRID) return fail(TACCHI_E_OUT_OF_GRID, "a particle's stencil left the grid");
    if (h_err & ERR_CAPACITY)
        return fail(TACCHI_E_UNSTABLE, "a grid block collected more particles than its bin capacity "
                                       "(local compression below J = 0.4)");
    if (h_err & ERR_INVERTED) return fail(TACCHI_E_UNSTABLE, "an element inverted (J <= 0) under neo-Hookean");
    if (h_err & ERR_NONFINITE) return fail(TACCHI_E_UNSTABLE, "non-finite particle state");
    return TACCHI_OK;
}

tacchi_status staging(tacchi_sim *s, size_t bytes, void **out)
{
    if (bytes > s->stage_bytes) {
        if (s->stage) TC_HIP(hipHostFree(s->stage));
        s->stage = nullptr;
        s->stage_bytes = 0;
        TC_HIP(hipHostMalloc(&s->stage, bytes, hipHostMallocDefault));
        s->stage_bytes = bytes;
    }
    *out = s->stage;
    return TACCHI_OK;
}

template <typename T>
tacchi_status init_state(tacchi_sim *s)
{
    SimDev<T> &S = sdev<T>(s);
    hipLaunchKernelGGL(k_init_particles<T>, dim3(grid1d(S.Ns)), dim3(kWG), 0, s->stream, S);
    TC_LAUNCHED();
    tacchi_status st = zero_bytes<T>(s, S.V, (size_t)s->d.nodes * 3 * sizeof(T));
    if (st) return st;
    st = zero_bytes<T>(s, S.err, 64);
    if (st) return st;
    st = zero_bytes<T>(s, S.force, 64);
    if (st) return st;
    st = zero_bytes<T>(s, S.fallback, 64);
    if (st) return st;
    return launch_bin<T>(s);
}

template <typename T>
tacchi_status read_particles_t(tacchi_sim *s, void *x, void *v, void *C, void *F, int on_device)
{
    SimDev<T> &S = sdev<T>(s);
    const size_t N = (size_t)S.N;
    void *dst[4] = {x, v, C, F};
    const size_t cnt[4] = {3 * N, 3 * N, 9 * N, 9 * N};
    T *tgt[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t offs[4] = {0, 0, 0, 0}, total = 0;
    for (int k = 0; k < 4; ++k) {
        offs[k] = total;
        if (dst[k]) total += cnt[k] * sizeof(T);
    }
    void *stage = nullptr;
    if (!on_device && total) {
        tacchi_status st = staging(s, total, &stage);
        if (st) return st;
    }
    for (int k = 0; k < 4; ++k)
        if (dst[k]) tgt[k] = on_device ? (T *)dst[k] : (T *)((char *)stage + offs[k]);
    const T dtA_coef = T(s->dtA * s->d.V0 * 4.0 / (s->d.dx * s->d.dx));
    const double *o = s->cfg.grid.origin;
    const bool neo = s->cfg.mat.model == TACCHI_NEOHOOKEAN;
    const dim3 g(grid1d(S.N)), blk(kWG);
    if (s->d.B == 4 && neo)
        hipLaunchKernelGGL((k_read_particles<T, 4, 0>), g, blk, 0, s->stream, S, T(o[0]), T(o[1]), T(o[2]),
                           T(s->d.dx), dtA_coef, tgt[0], tgt[1], tgt[2], tgt[3]);
    else if (s->d.B == 4)
        hipLaunchKernelGGL((k_read_particles<T, 4, 1>), g, blk, 0, s->stream, S, T(o[0]), T(o[1]), T(o[2]),
                           T(s->d.dx), dtA_coef, tgt[0], tgt[1], tgt[2], tgt[3]);
    else if (neo)
        hipLaunchKernelGGL((k_read_particles<T, 8, 0>), g, blk, 0, s->stream, S, T(o[0]), T(o[1]), T(o[2]),
                           T(s->d.dx), dtA_coef, tgt[0], tgt[1], tgt[2], tgt[3]);
    else
        hipLaunchKernelGGL((k_read_particles<T, 8, 1>), g, blk, 0, s->stream, S, T(o[0]), T(o[1]), T(o[2]),
                           T(s->d.dx), dtA_coef, tgt[0], tgt[1], tgt[2], tgt[3]);
    TC_LAUNCHED();
    TC_HIP(hipStreamSynchronize(s->stream));
    if (!on_device)
        for (int k = 0; k < 4; ++k)
            if (dst[k]) std::memcpy(dst[k], (char *)stage + offs[k], cnt[k] * sizeof(T));
    return read_error_word(s);
}

template <typename T>
tacchi_status write_particles_t(tacchi_sim *s, const void *x, const void *v, const void *C, const void *F,
                                int on_device)
{
    SimDev<T> &S = sdev<T>(s);
    const size_t N = (size_t)S.N;
    const void *src[4] = {x, v, C, F};
    const size_t cnt[4] = {3 * N, 3 * N, 9 * N, 9 * N};
    const T *in[4];
    if (on_device) {
        for (int k = 0; k < 4; ++k) in[k] = (const T *)src[k];
    } else {
        void *stage = nullptr;
        tacchi_status st = staging(s, 24 * N * sizeof(T), &stage);
        if (st) return st;
        TC_HIP(hipStreamSynchronize(s->stream));  // staging may still feed an earlier write
        size_t o = 0;
        for (int k = 0; k < 4; ++k) {
            std::memcpy((char *)stage + o, src[k], cnt[k] * sizeof(T));
            in[k] = (const T *)((char *)stage + o);
            o += cnt[k] * sizeof(T);
        }
    }
    const double *o = s->cfg.grid.origin;
    if (s->d.B == 4)
        hipLaunchKernelGGL((k_write_particles<T, 4>), dim3(grid1d(S.N)), dim3(kWG), 0, s->stream, S, T(o[0]),
                           T(o[1]), T(o[2]), T(1.0 / s->d.dx), in[0], in[1], in[2], in[3]);
    else
        hipLaunchKernelGGL((k_write_particles<T, 8>), dim3(grid1d(S.N)), dim3(kWG), 0, s->stream, S, T(o[0]),
                           T(o[1]), T(o[2]), T(1.0 / s->d.dx), in[0], in[1], in[2], in[3]);
    TC_LAUNCHED();
    tacchi_status st = zero_bytes<T>(s, S.err, 64);
    if (st) return st;
    s->dtA = 0.0;
    st = launch_bin<T>(s);
    if (st) return st;
    if (!on_device) TC_HIP(hipStreamSynchronize(s->stream));
    return TACCHI_OK;
}

template <typename T>
tacchi_status heightmap_t(tacchi_sim *s, void *out, int on_device, bool relative)
{
    SimDev<T> &S = sdev<T>(s);
    T *hm = (T *)(s->ws + s->L.hmap);
    const int nxy = s->d.n[0] * s->d.n[1];
    // relative maps hold only dx * u_z (the rest height is a constant that
    // drops out of the image's normals), which keeps FP32 differences exact
    const T zoff = relative ? T(0) : T(s->cfg.grid.origin[2]);
    SimDev<T> Sr = S;
    if (relative) Sr.xr[2] = T(0), Sr.hr[2] = T(0);
    {
        KernelTimer t(s, KC_HEIGHT);
        if (s->d.B == 4)
            hipLaunchKernelGGL((k_heightmap<T, 4>), dim3(grid1d(nxy)), dim3(kWG), 0, s->stream, Sr, zoff,
                               T(s->d.dx), hm);
        else
            hipLaunchKernelGGL((k_heightmap<T, 8>), dim3(grid1d(nxy)), dim3(kWG), 0, s->stream, Sr, zoff,
                               T(s->d.dx), hm);
    }
    TC_LAUNCHED();
    if (out) {
        TC_HIP(hipMemcpyAsync(out, hm, nxy * sizeof(T), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                              s->stream));
    }
    return TACCHI_OK;
}

template <typename T>
tacchi_status surface_disp_t(tacchi_sim *s, int res, int sub, float *out)
{
    SimDev<T> &S = sdev<T>(s);
    if (s->d.B == 4)
        hipLaunchKernelGGL((k_surface_disp<T, 4>), dim3(grid1d((int64_t)res * res)), dim3(kWG), 0, s->stream, S,
                           T(s->d.dx), res, sub, out);
    else
        hipLaunchKernelGGL((k_surface_disp<T, 8>), dim3(grid1d((int64_t)res * res)), dim3(kWG), 0, s->stream, S,
                           T(s->d.dx), res, sub, out);
    TC_LAUNCHED();
    return TACCHI_OK;
}

template <typename T>
tacchi_status markers_t(tacchi_sim *s, const std::vector<double> &q, int n, void *out, int on_device)
{
    SimDev<T> &S = sdev<T>(s);
    // the marker coordinates (and a host output) live in the handle's pinned
    // host staging buffer, which the kernel reads and writes directly: no
    // device memory is allocated
    const size_t qbytes = q.size() * sizeof(T), obytes = (size_t)n * 3 * sizeof(T);
    const size_t off = (qbytes + 255) & ~(size_t)255;
    void *stage = nullptr;
    TC_HIP(hipStreamSynchronize(s->stream));  // the staging buffer may still feed an earlier call
    tacchi_status st = staging(s, off + (on_device ? 0 : obytes), &stage);
    if (st) return st;
    T *dq = (T *)stage, *dout = on_device ? (T *)out : (T *)((char *)stage + off);
    for (size_t k = 0; k < q.size(); ++k) dq[k] = T(q[k]);
    if (s->d.B == 4)
        hipLaunchKernelGGL((k_markers<T, 4>), dim3(grid1d(n)), dim3(kWG), 0, s->stream, S, dq, n, T(s->d.dx), dout);
    else
        hipLaunchKernelGGL((k_markers<T, 8>), dim3(grid1d(n)), dim3(kWG), 0, s->stream, S, dq, n, T(s->d.dx), dout);
    hipError_t e = hipGetLastError();
    const hipError_t es = hipStreamSynchronize(s->stream);
    if (e != hipSuccess || es != hipSuccess)
        return fail(TACCHI_E_DEVICE, std::string("tacchi_markers: ") + hipGetErrorString(e != hipSuccess ? e : es));
    if (!on_device) std::memcpy(out, dout, obytes);
    return read_error_word(s);
}

// One vertical gap query: the indenter at a pose above a block's top face.
struct GapDev {
    IndenterDev<double> I;  // shape, parameters and orientation (indenter frame -> world)
    double pos[3];          // indenter origin, world metres
    double x0, y0, wx, wy;  // top face origin and extent
    double ztop;            // undeformed top face height
};

// Clipped gap at one point: (lowest z of the indenter on the vertical through
// (x, y)) - ztop, clamped to [lo, hi]. The inside test is sampled upward
// from ztop + lo to ztop + hi in 512 steps; the first sample inside is refined by 40
// bisections.
__device__ double gap_at(const GapDev &g, double x, double y, double lo, double hi)
{
    const double r0 = x - g.pos[0], r1 = y - g.pos[1];
    auto inside = [&](double z) {
        const double r2 = z - g.pos[2];
        const double px = g.I.R[0] * r0 + g.I.R[3] * r1 + g.I.R[6] * r2;
        const double py = g.I.R[1] * r0 + g.I.R[4] * r1 + g.I.R[7] * r2;
        const double pz = g.I.R[2] * r0 + g.I.R[5] * r1 + g.I.R[8] * r2;
        return indenter_phi<double>(g.I, px, py, pz) <= 0.0;
    };
    constexpr int kSamples = 512;
    const double zlo = g.ztop + lo, step = (hi - lo) / kSamples;
    double gap = hi;
    if (inside(zlo)) {
        gap = lo;
    } else {
        double a = zlo;
        for (int s = 1; s <= kSamples; ++s) {
            const double b = zlo + s * step;
            if (inside(b)) {
                double lo = a, hi = b;
                for (int it = 0; it < 40; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (inside(mid))
                        hi = mid;
                    else
                        lo = mid;
                }
                gap = hi - g.ztop;
                break;
            }
            a = b;
        }
    }
    return gap;
}

// out[k][r][c] = mean of gap_at over sub x sub points spread evenly inside
// cell (c, r) of the res x res partition of block k's top face (sub = 1: the
// cell centre).
__global__ void __launch_bounds__(kWG) k_indenter_gap(const GapDev *q, int n, int res, int sub, double lo, double hi,
                                                      float *out)
{
    const int64_t idx = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (idx >= (int64_t)n * res * res) return;
    const int k = (int)(idx / ((int64_t)res * res));
    const int rem = (int)(idx - (int64_t)k * res * res);
    const int r = rem / res, c = rem - r * res;
    const GapDev &g = q[k];
    double acc = 0.0;
    for (int qy = 0; qy < sub; ++qy)
        for (int qx = 0; qx < sub; ++qx) {
            const double x = g.x0 + (c + (qx + 0.5) / sub) * g.wx / res;
            const double y = g.y0 + (r + (qy + 0.5) / sub) * g.wy / res;
            acc += gap_at(g, x, y, lo, hi);
        }
    out[idx] = (float)(acc / (sub * sub));
}

template <typename T>
tacchi_status render_t(tacchi_sim *s, const tacchi_render_params *rp, float *rgb, int h, int w, int on_device)
{
    tacchi_status st = heightmap_t<T>(s, nullptr, 1, true);
    if (st) return st;
    RenderDev<T> R{};
    const tacchi_config &c = s->cfg;
    R.n0 = s->d.n[0];
    R.n1 = s->d.n[1];
    R.h = h;
    R.w = w;
    R.hx = T(s->d.h[0]);
    R.hy = T(s->d.h[1]);
    R.x0 = T(c.block.origin[0] + 0.5 * s->d.h[0]);
    R.y0 = T(c.block.origin[1] + 0.5 * s->d.h[1]);
    R.cx = T(c.block.origin[0] + 0.5 * c.block.size[0]);
    R.cy = T(c.block.origin[1] + 0.5 * c.block.size[1]);
    R.pitch = T(rp->pitch);
    R.ka = T(rp->ka_ia);
    R.kd = T(rp->kd);
    R.ks = T(rp->ks);
    R.alpha = T(rp->alpha);
    const double el = rp->light_elev_deg * kPi / 180.0;
    for (int ch = 0; ch < 3; ++ch) {
        const double az = rp->light_azim_deg[ch] * kPi / 180.0;
        R.L[ch][0] = T(std::cos(el) * std::cos(az));
        R.L[ch][1] = T(std::cos(el) * std::sin(az));
        R.L[ch][2] = T(-std::sin(el));
    }
    float *dst = rgb;
    void *stage = nullptr;
    const size_t bytes = (size_t)h * w * 3 * sizeof(float);
    if (!on_device) {
        st = staging(s, bytes, &stage);
        if (st) return st;
        dst = (float *)stage;
    }
    {
        KernelTimer t(s, KC_RENDER);
        hipLaunchKernelGGL(k_render<T>, dim3(grid1d((int64_t)h * w)), dim3(kWG), 0, s->stream,
                           (const T *)(s->ws + s->L.hmap), R, dst);
    }
    TC_LAUNCHED();
    TC_HIP(hipStreamSynchronize(s->stream));
    if (!on_device) std::memcpy(rgb, stage, bytes);
    return read_error_word(s);
}

template <typename T>
tacchi_status read_grid_t(tacchi_sim *s, int which, void *M, void *vec, int on_device)
{
    SimDev<T> &S = sdev<T>(s);
    const int64_t n = (int64_t)S.g0 * S.g1 * S.g2;
    T *m_out = (T *)M, *v_out = (T *)vec;
    void *stage = nullptr;
    if (!on_device) {
        tacchi_status st = staging(s, (size_t)n * 4 * sizeof(T), &stage);
        if (st) return st;
        m_out = M ? (T *)stage : nullptr;
        v_out = (T *)stage + n;
    }
    if (s->d.B == 4)
        hipLaunchKernelGGL((k_read_grid<T, 4>), dim3(grid1d(n)), dim3(kWG), 0, s->stream, S, which, T(s->d.dx),
                           m_out, v_out);
    else
        hipLaunchKernelGGL((k_read_grid<T, 8>), dim3(grid1d(n)), dim3(kWG), 0, s->stream, S, which, T(s->d.dx),
                           m_out, v_out);
    TC_LAUNCHED();
    TC_HIP(hipStreamSynchronize(s->stream));
    if (!on_device) {
        if (M && which == 0) std::memcpy(M, stage, n * sizeof(T));
        std::memcpy(vec, (T *)stage + n, 3 * n * sizeof(T));
    }
    return TACCHI_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char *tacchi_last_error(void) { return g_last_error.c_str(); }

size_t tacchi_workspace_bytes(const tacchi_config *cfg)
{
    Derived d;
    if (derive(cfg, &d) != TACCHI_OK) return 0;
    return make_layout(d).total;
}

tacchi_status tacchi_create(const tacchi_config *cfg, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            tacchi_sim **out)
{
    if (!out) return fail(TACCHI_E_ARG, "out is NULL");
    *out = nullptr;
    Derived d;
    tacchi_status st = derive(cfg, &d);
    if (st) return st;
    Layout L = make_layout(d);
    if (!dev_ws) return fail(TACCHI_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(TACCHI_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(TACCHI_E_WORKSPACE, "workspace too small");
    tacchi_sim *s = new (std::nothrow) tacchi_sim();
    if (!s) return fail(TACCHI_E_ARG, "out of host memory");
    s->cfg = *cfg;
    s->d = d;
    s->L = L;
    s->ws = (char *)dev_ws;
    s->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(TACCHI_E_DEVICE, "hipGetDevice failed");
    }
    std::memcpy(s->pose, cfg->pose0.pos, 3 * sizeof(double));
    std::memcpy(s->pose + 3, cfg->pose0.quat, 4 * sizeof(double));
    s->sf = make_simdev<float>(s);
    s->sd = make_simdev<double>(s);
    st = cfg->precision == TACCHI_F64 ? init_state<double>(s) : init_state<float>(s);
    if (st) {
        delete s;
        return st;
    }
    *out = s;
    return TACCHI_OK;
}

tacchi_status tacchi_p2g(tacchi_sim *s, double dt)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    if (s->phase != 0) return fail(TACCHI_E_STATE, "tacchi_p2g called out of order");
    tacchi_status st = check_dt(s, dt);
    if (st) return st;
    st = set_device(s);
    if (st) return st;
    st = s->cfg.precision == TACCHI_F64 ? do_p2g<double>(s, dt) : do_p2g<float>(s, dt);
    if (st) return st;
    s->phase = 1;
    s->dt_phase = dt;
    return TACCHI_OK;
}

tacchi_status tacchi_grid_update(tacchi_sim *s, const tacchi_pose *pose_end, double dt)
{
    if (!s || !pose_end) return fail(TACCHI_E_ARG, "NULL argument");
    if (s->phase != 1) return fail(TACCHI_E_STATE, "tacchi_grid_update called out of order");
    if (dt != s->dt_phase) return fail(TACCHI_E_ARG, "dt differs from the one given to tacchi_p2g");
    const double *q = pose_end->quat;
    if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 0)) return fail(TACCHI_E_ARG, "zero quaternion");
    tacchi_status st = set_device(s);
    if (st) return st;
    double pe[7];
    std::memcpy(pe, pose_end->pos, 3 * sizeof(double));
    std::memcpy(pe + 3, pose_end->quat, 4 * sizeof(double));
    st = s->cfg.precision == TACCHI_F64 ? do_grid<double>(s, pe, dt) : do_grid<float>(s, pe, dt);
    if (st) return st;
    std::memcpy(s->pending, pe, sizeof pe);
    s->phase = 2;
    return TACCHI_OK;
}

tacchi_status tacchi_g2p(tacchi_sim *s, double dt)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    if (s->phase != 2) return fail(TACCHI_E_STATE, "tacchi_g2p called out of order");
    if (dt != s->dt_phase) return fail(TACCHI_E_ARG, "dt differs from the one given to tacchi_p2g");
    tacchi_status st = set_device(s);
    if (st) return st;
    st = s->cfg.precision == TACCHI_F64 ? do_g2p<double>(s, dt) : do_g2p<float>(s, dt);
    if (st) return st;
    // the bin lists written by G2P become the current ones
    s->parity ^= 1;
    s->sf = make_simdev<float>(s);
    s->sd = make_simdev<double>(s);
    std::memcpy(s->pose, s->pending, sizeof s->pose);
    s->dtA = dt;
    s->phase = 0;
    return TACCHI_OK;
}

tacchi_status tacchi_step(tacchi_sim *s, const tacchi_pose *pose_end, double dt)
{
    tacchi_status st = tacchi_p2g(s, dt);
    if (st) return st;
    st = tacchi_grid_update(s, pose_end, dt);
    if (st) return st;
    return tacchi_g2p(s, dt);
}

tacchi_status tacchi_run(tacchi_sim *s, const tacchi_pose *poses, int32_t n, double dt)
{
    if (!s || (!poses && n > 0) || n < 0) return fail(TACCHI_E_ARG, "bad arguments to tacchi_run");
    for (int32_t k = 0; k < n; ++k) {
        tacchi_status st = tacchi_step(s, poses + k, dt);
        if (st) return st;
    }
    return TACCHI_OK;
}


size_t tacchi_points_workspace_bytes(const tacchi_sim *s, int32_t n)
{
    if (!s || n < 1) return 0;
    const size_t nn = (size_t)s->d.g[0] * s->d.g[1] * s->d.g[2];
    return align256(nn * sizeof(double)) + align256((size_t)n * 3 * sizeof(double));
}

tacchi_status tacchi_set_indenter_points(tacchi_sim *s, const double *xyz, int32_t n, double mass, void *dev_ws,
                                         size_t ws_bytes)
{
    if (!s || (n > 0 && !xyz)) return fail(TACCHI_E_ARG, "NULL argument");
    if (n < 0 || n > (1 << 24)) return fail(TACCHI_E_ARG, "point count must be in [0, 2^24]");
    if (!(mass >= 0.0) || !std::isfinite(mass)) return fail(TACCHI_E_ARG, "mass per point must be finite and >= 0");
    if (s->phase != 0) return fail(TACCHI_E_STATE, "tacchi_set_indenter_points called inside a substep");
    for (int64_t k = 0; k < 3 * (int64_t)n; ++k)
        if (!std::isfinite(xyz[k])) return fail(TACCHI_E_ARG, "non-finite point coordinate");
    tacchi_status st = set_device(s);
    if (st) return st;
    if (n > 0 && (!dev_ws || ((uintptr_t)dev_ws & 255) || ws_bytes < tacchi_points_workspace_bytes(s, n)))
        return fail(TACCHI_E_WORKSPACE, "indenter points need a 256-byte aligned device workspace of "
                                        "tacchi_points_workspace_bytes(sim, n) bytes");
    TC_HIP(hipStreamSynchronize(s->stream));
    s->ipts = nullptr;
    s->MI = nullptr;
    s->ni = 0;
    if (n == 0) return TACCHI_OK;
    const size_t nn = (size_t)s->d.g[0] * s->d.g[1] * s->d.g[2];
    s->MI = (double *)dev_ws;
    s->ipts = (double *)((char *)dev_ws + align256(nn * sizeof(double)));
    for (int a = 0; a < 3; ++a) {
        s->plo[a] = 1e300;
        s->phi_[a] = -1e300;
    }
    for (int64_t k = 0; k < n; ++k)
        for (int a = 0; a < 3; ++a) {
            s->plo[a] = std::min(s->plo[a], xyz[3 * k + a]);
            s->phi_[a] = std::max(s->phi_[a], xyz[3 * k + a]);
        }
    // spatial (Morton) order at the grid spacing, so that the scatter's
    // workgroups get compact groups of points
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffULL;
        v = (v | v << 16) & 0x1f0000ff0000ffULL;
        v = (v | v << 8) & 0x100f00f00f00f00fULL;
        v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
        v = (v | v << 2) & 0x1249249249249249ULL;
        return v;
    };
    std::vector<std::pair<uint64_t, int>> order((size_t)n);
    for (int k = 0; k < n; ++k) {
        uint64_t c[3];
        for (int a = 0; a < 3; ++a)
            c[a] = (uint64_t)std::min(std::max((xyz[3 * k + a] - s->plo[a]) / s->d.dx, 0.0), 2097151.0);
        order[k] = {spread(c[0]) | spread(c[1]) << 1 | spread(c[2]) << 2, k};
    }
    std::sort(order.begin(), order.end());
    std::vector<double> sorted((size_t)n * 3);
    for (int k = 0; k < n; ++k)
        for (int a = 0; a < 3; ++a) sorted[3 * (size_t)k + a] = xyz[3 * (size_t)order[k].second + a];
    // the order pays off once a fair share (1/8, measured at 10^5 points on
    // the GelSight sphere) of the groups of kWG consecutive points are dense
    // enough for the scatter's LDS tile (the kernel's own test, taken at the
    // rest orientation); a sparse cloud keeps the given order, whose
    // scattered groups spread the direct atomics over many nodes
    int64_t groups = 0, dense = 0;
    for (int g = 0; g < n; g += kWG) {
        const int cnt = std::min(kWG, n - g);
        int64_t nodes = 1;
        bool fits = true;
        for (int a = 0; a < 3; ++a) {
            double lo = 1e300, hi = -1e300;
            for (int k = g; k < g + cnt; ++k) {
                lo = std::min(lo, sorted[3 * (size_t)k + a]);
                hi = std::max(hi, sorted[3 * (size_t)k + a]);
            }
            const int e = (int)(std::floor(hi / s->d.dx) - std::floor(lo / s->d.dx)) + 3;
            fits = fits && e <= kScatterEdge;
            nodes *= e;
        }
        ++groups;
        dense += fits && 2 * nodes <= 27 * (int64_t)cnt;
    }
    const double *up = 8 * dense >= groups ? sorted.data() : xyz;
    TC_HIP(hipMemcpy(s->ipts, up, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice));
    s->ni = n;
    s->imass = mass;
    return TACCHI_OK;
}

tacchi_status tacchi_set_contact(tacchi_sim *s, int32_t model, double mu)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    if (model != TACCHI_CONTACT_STICKY && model != TACCHI_CONTACT_COULOMB) return fail(TACCHI_E_ARG, "unknown contact model");
    if (std::isnan(mu) || mu < 0.0) return fail(TACCHI_E_ARG, "friction coefficient must be >= 0");
    s->contact_model = model;
    s->friction = model == TACCHI_CONTACT_COULOMB ? mu : 0.0;
    return TACCHI_OK;
}

tacchi_status tacchi_run_until_force(tacchi_sim *s, const tacchi_pose *poses, int32_t n, double dt, double fz_limit,
                                     int32_t *steps_done)
{
    if (!s || !poses || !steps_done || n < 1) return fail(TACCHI_E_ARG, "bad arguments to tacchi_run_until_force");
    if (std::isnan(fz_limit)) return fail(TACCHI_E_ARG, "fz_limit is NaN");
    if (s->phase != 0) return fail(TACCHI_E_STATE, "tacchi_run_until_force called inside a substep");
    *steps_done = 0;
    tacchi_status st = set_device(s);
    if (st) return st;
    int *flag = (int *)(s->ws + s->L.stop);
    hipLaunchKernelGGL(k_fill<int>, dim3(1), dim3(kWG), 0, s->stream, flag, (int64_t)2, 0);
    TC_LAUNCHED();
    const double *force = (const double *)(s->ws + s->L.force);
    const int parity0 = s->parity;
    s->stop_armed = true;
    s->sf = make_simdev<float>(s);
    s->sd = make_simdev<double>(s);
    int launched = 0;
    for (; launched < n; ++launched) {
        st = tacchi_step(s, poses + launched, dt);
        if (st) break;
        hipLaunchKernelGGL(k_stop_check, dim3(1), dim3(64), 0, s->stream, flag, force, fz_limit);
        if (hipGetLastError() != hipSuccess) {
            st = fail(TACCHI_E_DEVICE, "tacchi_run_until_force: launch failed");
            break;
        }
    }
    int h[2] = {0, 0};
    const hipError_t e = hipMemcpyAsync(h, flag, sizeof h, hipMemcpyDeviceToHost, s->stream);
    const hipError_t es = hipStreamSynchronize(s->stream);
    // the host advanced its bin-buffer parity and pose once per launched
    // substep; the device state is that of the substeps that ran
    const int done = (e == hipSuccess && es == hipSuccess) ? h[1] : launched;
    s->parity = parity0 ^ (done & 1);
    if (done > 0) {
        std::memcpy(s->pose, poses[done - 1].pos, 3 * sizeof(double));
        std::memcpy(s->pose + 3, poses[done - 1].quat, 4 * sizeof(double));
    }
    s->stop_armed = false;
    s->sf = make_simdev<float>(s);
    s->sd = make_simdev<double>(s);
    if (st) return st;
    if (e != hipSuccess || es != hipSuccess) return fail(TACCHI_E_DEVICE, "tacchi_run_until_force: readback failed");
    *steps_done = done;
    return read_error_word(s);
}

tacchi_status tacchi_read_grid(tacchi_sim *s, int32_t which, void *M, void *vec, int32_t on_device)
{
    if (!s || !vec) return fail(TACCHI_E_ARG, "NULL argument");
    if (which != 0 && which != 1) return fail(TACCHI_E_ARG, "which must be 0 or 1");
    if ((which == 0 && s->phase != 1) || (which == 1 && s->phase != 2))
        return fail(TACCHI_E_STATE, "grid contents not available in this phase");
    tacchi_status st = set_device(s);
    if (st) return st;
    return s->cfg.precision == TACCHI_F64 ? read_grid_t<double>(s, which, M, vec, on_device)
                                          : read_grid_t<float>(s, which, M, vec, on_device);
}

tacchi_status tacchi_heightmap(tacchi_sim *s, void *out, int32_t on_device)
{
    if (!s || !out) return fail(TACCHI_E_ARG, "NULL argument");
    tacchi_status st = set_device(s);
    if (st) return st;
    st = s->cfg.precision == TACCHI_F64 ? heightmap_t<double>(s, out, on_device, false)
                                        : heightmap_t<float>(s, out, on_device, false);
    if (st) return st;
    return read_error_word(s);
}

tacchi_status tacchi_surface_displacement(tacchi_sim *s, int32_t res, int32_t sub, float *out, int32_t on_device)
{
    if (!s || !out) return fail(TACCHI_E_ARG, "NULL argument");
    if (res < 1 || res > 4096) return fail(TACCHI_E_ARG, "res must be in [1, 4096]");
    if (sub < 1 || sub > 16) return fail(TACCHI_E_ARG, "sub must be in [1, 16]");
    if (s->d.n[0] < 2 || s->d.n[1] < 2) return fail(TACCHI_E_ARG, "the top layer needs at least 2 x 2 particles");
    tacchi_status st = set_device(s);
    if (st) return st;
    if (on_device)
        return s->cfg.precision == TACCHI_F64 ? surface_disp_t<double>(s, res, sub, out)
                                              : surface_disp_t<float>(s, res, sub, out);
    // a host output is written by the kernel into the handle's pinned host
    // staging buffer and copied out: no device memory is allocated
    const size_t bytes = (size_t)res * res * 3 * sizeof(float);
    TC_HIP(hipStreamSynchronize(s->stream));  // the staging buffer may still feed an earlier call
    void *stage = nullptr;
    st = staging(s, bytes, &stage);
    if (st) return st;
    st = s->cfg.precision == TACCHI_F64 ? surface_disp_t<double>(s, res, sub, (float *)stage)
                                        : surface_disp_t<float>(s, res, sub, (float *)stage);
    const hipError_t es = hipStreamSynchronize(s->stream);
    if (st) return st;
    if (es != hipSuccess) return fail(TACCHI_E_DEVICE, "tacchi_surface_displacement: kernel failed");
    std::memcpy(out, stage, bytes);
    return read_error_word(s);
}

tacchi_status tacchi_markers(tacchi_sim *s, const double *xy, int32_t n, void *out, int32_t on_device)
{
    if (!s || !xy || !out) return fail(TACCHI_E_ARG, "NULL argument");
    if (n < 1 || n > (1 << 24)) return fail(TACCHI_E_ARG, "marker count must be in [1, 2^24]");
    if (s->d.n[0] < 2 || s->d.n[1] < 2) return fail(TACCHI_E_ARG, "the top layer needs at least 2 x 2 particles");
    const tacchi_block &bk = s->cfg.block;
    const double hx = bk.size[0] / bk.n[0], hy = bk.size[1] / bk.n[1];
    std::vector<double> q((size_t)n * 2);
    for (int k = 0; k < n; ++k) {
        const double x = xy[2 * k], y = xy[2 * k + 1];
        if (!(x >= bk.origin[0] && x <= bk.origin[0] + bk.size[0] && y >= bk.origin[1] &&
              y <= bk.origin[1] + bk.size[1]))
            return fail(TACCHI_E_ARG, "a marker lies outside the top face");
        // fractional lattice coordinates; the half-cell rims outside the
        // outermost particle centres take the edge value
        q[2 * k] = std::min(std::max((x - bk.origin[0]) / hx - 0.5, 0.0), (double)(bk.n[0] - 1));
        q[2 * k + 1] = std::min(std::max((y - bk.origin[1]) / hy - 0.5, 0.0), (double)(bk.n[1] - 1));
    }
    tacchi_status st = set_device(s);
    if (st) return st;
    return s->cfg.precision == TACCHI_F64 ? markers_t<double>(s, q, n, out, on_device)
                                          : markers_t<float>(s, q, n, out, on_device);
}

size_t tacchi_indenter_gap_workspace_bytes(int32_t n)
{
    return n < 1 ? 0 : (size_t)n * sizeof(GapDev);
}

}  // extern "C"

namespace {

// Validated query descriptors of a gap-field call.
tacchi_status gap_queries(const tacchi_config *cfgs, const tacchi_pose *poses, int32_t n, int32_t res, int32_t sub,
                          double lo, double hi, const float *out, const char *who, std::vector<GapDev> &q)
{
    if (!cfgs || !poses || !out || n < 1 || res < 1 || res > 4096 || sub < 1 || sub > 16 || !(hi > lo) ||
        !std::isfinite(lo) || !std::isfinite(hi) || hi - lo > 1.0)
        return fail(TACCHI_E_ARG, std::string(who) + ": bad arguments");
    q.resize((size_t)n);
    for (int k = 0; k < n; ++k) {
        const tacchi_config &c = cfgs[k];
        if (c.ind.shape < TACCHI_SPHERE || c.ind.shape > TACCHI_TEXTURED_PLATE)
            return fail(TACCHI_E_ARG, "unknown indenter shape");
        double pose[7];
        for (int a = 0; a < 3; ++a) pose[a] = poses[k].pos[a];
        for (int a = 0; a < 4; ++a) pose[3 + a] = poses[k].quat[a];
        const double qn = std::sqrt(pose[3] * pose[3] + pose[4] * pose[4] + pose[5] * pose[5] + pose[6] * pose[6]);
        if (!(qn > 0.5) || !(qn < 2.0)) return fail(TACCHI_E_ARG, "pose quaternion is not unit");
        q[k].I = make_indenter<double>(c, pose, pose, 1.0);
        for (int a = 0; a < 3; ++a) q[k].pos[a] = pose[a];
        q[k].x0 = c.block.origin[0];
        q[k].y0 = c.block.origin[1];
        q[k].wx = c.block.size[0];
        q[k].wy = c.block.size[1];
        q[k].ztop = c.block.origin[2] + c.block.size[2];
    }
    return TACCHI_OK;
}

// Copies the descriptors to dq (device memory) and runs the gap kernel on st;
// synchronises (q is pageable host memory read by the copy).
tacchi_status gap_run(const std::vector<GapDev> &q, GapDev *dq, int32_t res, int32_t sub, double lo, double hi,
                      float *out, hipStream_t st, const char *who)
{
    const int n = (int)q.size();
    hipError_t e = hipMemcpyAsync(dq, q.data(), q.size() * sizeof(GapDev), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_indenter_gap, dim3(grid1d((int64_t)n * res * res)), dim3(kWG), 0, st, dq, n, res, sub,
                           lo, hi, out);
        e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(st);
    if (e != hipSuccess || es != hipSuccess)
        return fail(TACCHI_E_DEVICE, std::string(who) + ": " + hipGetErrorString(e != hipSuccess ? e : es));
    return TACCHI_OK;
}

// Query descriptors of tacchi_indenter_gap_noalloc: a fixed array in device
// memory that comes with the library's code object, one copy on each GPU the
// library runs on, held until the process ends. Host code never uses its name
// as an address (that is a host-side stand-in): the device address of each
// GPU's copy is looked up once, with that GPU current, and kept.
constexpr int kGapNoAllocMax = 2048;
static __device__ __align__(256) unsigned char scratch[kGapNoAllocMax * sizeof(GapDev)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

tacchi_status gap_scratch(void **out)
{
    int dev = -1;
    TC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TACCHI_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TACCHI_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TACCHI_OK;
}

}  // namespace

extern "C" {

tacchi_status tacchi_indenter_gap(const tacchi_config *cfgs, const tacchi_pose *poses, int32_t n, int32_t res,
                                  int32_t sub, double lo, double hi, float *out, void *dev_ws, size_t ws_bytes,
                                  void *hip_stream)
{
    std::vector<GapDev> q;
    tacchi_status st = gap_queries(cfgs, poses, n, res, sub, lo, hi, out, "tacchi_indenter_gap", q);
    if (st) return st;
    if (!dev_ws || ((uintptr_t)dev_ws & 255) || ws_bytes < tacchi_indenter_gap_workspace_bytes(n))
        return fail(TACCHI_E_WORKSPACE, "tacchi_indenter_gap: workspace missing, misaligned or smaller than "
                                        "tacchi_indenter_gap_workspace_bytes(n)");
    return gap_run(q, (GapDev *)dev_ws, res, sub, lo, hi, out, (hipStream_t)hip_stream, "tacchi_indenter_gap");
}

int32_t tacchi_indenter_gap_noalloc_max(void)
{
    return kGapNoAllocMax;
}

tacchi_status tacchi_indenter_gap_noalloc(const tacchi_config *cfgs, const tacchi_pose *poses, int32_t n,
                                          int32_t res, int32_t sub, double lo, double hi, float *out,
                                          void *hip_stream)
{
    if (n > kGapNoAllocMax)
        return fail(TACCHI_E_ARG, "tacchi_indenter_gap_noalloc: more queries than "
                                  "tacchi_indenter_gap_noalloc_max() (" + std::to_string(kGapNoAllocMax) + ")");
    std::vector<GapDev> q;
    tacchi_status st = gap_queries(cfgs, poses, n, res, sub, lo, hi, out, "tacchi_indenter_gap_noalloc", q);
    if (st) return st;
    void *dq = nullptr;
    st = gap_scratch(&dq);
    if (st) return st;
    return gap_run(q, (GapDev *)dq, res, sub, lo, hi, out, (hipStream_t)hip_stream, "tacchi_indenter_gap_noalloc");
}

tacchi_status tacchi_render(tacchi_sim *s, const tacchi_render_params *rp, float *rgb, int32_t h, int32_t w,
                            int32_t on_device)
{
    if (!s || !rp || !rgb) return fail(TACCHI_E_ARG, "NULL argument");
    if (h < 1 || w < 1 || !(rp->pitch > 0)) return fail(TACCHI_E_ARG, "image size and pitch must be positive");
    tacchi_status st = set_device(s);
    if (st) return st;
    return s->cfg.precision == TACCHI_F64 ? render_t<double>(s, rp, rgb, h, w, on_device)
                                          : render_t<float>(s, rp, rgb, h, w, on_device);
}

tacchi_status tacchi_read_particles(tacchi_sim *s, void *x, void *v, void *C, void *F, int32_t on_device)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    tacchi_status st = set_device(s);
    if (st) return st;
    return s->cfg.precision == TACCHI_F64 ? read_particles_t<double>(s, x, v, C, F, on_device)
                                          : read_particles_t<float>(s, x, v, C, F, on_device);
}

tacchi_status tacchi_write_particles(tacchi_sim *s, const void *x, const void *v, const void *C, const void *F,
                                     int32_t on_device)
{
    if (!s || !x || !v || !C || !F) return fail(TACCHI_E_ARG, "all four particle arrays are required");
    if (s->phase != 0) return fail(TACCHI_E_STATE, "cannot write particles in the middle of a substep");
    tacchi_status st = set_device(s);
    if (st) return st;
    return s->cfg.precision == TACCHI_F64 ? write_particles_t<double>(s, x, v, C, F, on_device)
                                          : write_particles_t<float>(s, x, v, C, F, on_device);
}

tacchi_status tacchi_indenter_force(tacchi_sim *s, double f[3])
{
    if (!s || !f) return fail(TACCHI_E_ARG, "NULL argument");
    tacchi_status st = set_device(s);
    if (st) return st;
    TC_HIP(hipMemcpyAsync(f, s->ws + s->L.force, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    return read_error_word(s);
}

tacchi_status tacchi_polar_fallbacks(tacchi_sim *s, uint64_t *count)
{
    if (!s || !count) return fail(TACCHI_E_ARG, "NULL argument");
    tacchi_status st = set_device(s);
    if (st) return st;
    unsigned int c = 0;
    TC_HIP(hipMemcpyAsync(&c, s->ws + s->L.fallback, sizeof c, hipMemcpyDeviceToHost, s->stream));
    TC_HIP(hipStreamSynchronize(s->stream));
    *count = c;
    return TACCHI_OK;
}

tacchi_status tacchi_get_pose(const tacchi_sim *s, tacchi_pose *pose)
{
    if (!s || !pose) return fail(TACCHI_E_ARG, "NULL argument");
    std::memcpy(pose->pos, s->pose, 3 * sizeof(double));
    std::memcpy(pose->quat, s->pose + 3, 4 * sizeof(double));
    return TACCHI_OK;
}

int64_t tacchi_num_particles(const tacchi_sim *s) { return s ? s->d.N : 0; }

tacchi_status tacchi_sync(tacchi_sim *s)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    tacchi_status st = set_device(s);
    if (st) return st;
    return read_error_word(s);
}

tacchi_status tacchi_timing_enable(tacchi_sim *s, uint32_t class_mask)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    if (class_mask >> TACCHI_NUM_KERNEL_CLASSES) return fail(TACCHI_E_ARG, "unknown kernel class in mask");
    s->timing_mask = class_mask;
    return TACCHI_OK;
}

tacchi_status tacchi_timing_read(tacchi_sim *s, double *ms, int64_t *counts, int32_t reset)
{
    if (!s) return fail(TACCHI_E_ARG, "sim is NULL");
    tacchi_status st = set_device(s);
    if (st) return st;
    TC_HIP(hipStreamSynchronize(s->stream));
    for (auto &p : s->timed) {
        float e = 0.0f;
        TC_HIP(hipEventElapsedTime(&e, p.a, p.b));
        s->timing_ms[p.cls] += e;
        s->timing_n[p.cls] += 1;
        s->event_pool.push_back(p.a);
        s->event_pool.push_back(p.b);
    }
    s->timed.clear();
    for (int k = 0; k < TACCHI_NUM_KERNEL_CLASSES; ++k) {
        if (ms) ms[k] = s->timing_ms[k];
        if (counts) counts[k] = s->timing_n[k];
        if (reset) {
            s->timing_ms[k] = 0.0;
            s->timing_n[k] = 0;
        }
    }
    return TACCHI_OK;
}

void tacchi_destroy(tacchi_sim *s)
{
    if (!s) return;
    if (s->stage) (void)hipHostFree(s->stage);
    for (auto &p : s->timed) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    delete s;
}

}  // extern "C"

#include "batch_host.hpp"
