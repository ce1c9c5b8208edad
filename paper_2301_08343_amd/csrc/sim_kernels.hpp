// MLS-MPM substep kernels for one elastomer contact (gfx950, wave64).
//
// Per substep (Sec. III-A): P2G into an LDS tile per grid block, stored per
// block (Eqs. 2-5); the grid update, which gathers the tiles covering each
// node and applies gravity, rigid-indenter contact, floor and walls (Eq. 6,
// Eq. 10); and G2P fused with the constitutive update and advection
// (Eqs. 7-11), which also bins each particle into its block's list for the
// next substep (the per-substep counting sort).
#pragma once
#include "device_common.hpp"

namespace tacchi {

// ---------------------------------------------------------------- binning

// Appends particle `slot` with block key `key` (< 0: none) to the bin lists,
// one atomic per run of equal keys in the wave. All 64 lanes must call it.
template <typename T>
__device__ __forceinline__ void bin_append(const SimDev<T> &S, int *cnt, int *perm, int key, uint32_t slot)
{
    const int pos = wave_run_slot(cnt, key);
    if (key >= 0) {
        if (pos < S.cap)
            perm[(int64_t)key * S.cap + pos] = (int)slot;
        else
            atomicOr(S.err, ERR_CAPACITY);
    }
}

// Bins every particle by its current position (after init or a state write);
// the counts must be zero.
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_bin(SimDev<T> S)
{
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    int key = -1, i, j, k;
    if (s < S.Ns && slot_lattice<T, B>(S, (uint32_t)s, i, j, k)) {
        T xr[3];
        rest_position(S, i, j, k, xr);
        const T uu[3] = {S.u[s], S.u[S.Ns + s], S.u[2 * S.Ns + s]};
        key = block_key<T, B>(S, xr, uu);
    }
    bin_append(S, S.cnt_cur, S.perm_cur, key, (uint32_t)s);
}

// ---------------------------------------------------------------- P2G

// LDS accumulation slot of one tile channel. FP64 adds natively
// (ds_add_f64). FP32 accumulates 64-bit fixed point with ds_add_u64: the
// contributions are pre-scaled so that one particle mass is 2^28 units and one
// momentum unit m/dt (a particle crossing a cell per substep) is 2^28 units,
// rounded to the nearest integer and summed exactly, so the sum does not
// depend on the order of the atomics; gfx950 also executes ds_add_u64 about
// 25x faster than ds_add_f32. Each contribution is below 2^31 units (checked
// per particle: 8 cells per substep, far beyond the CFL limit), so it converts
// with an FP32 round-to-nearest-even and one FP32 -> int32 instruction and is
// sign-extended into the 64-bit sum. Rounding (not truncation) keeps the
// quantisation error unbiased: truncation shrinks every contribution toward
// zero, a bias that a steady configuration repeats every substep.
template <typename T>
struct TileAcc;

template <>
struct TileAcc<double> {
    using Slot = double;
    static constexpr bool kFixed = false;
    __device__ static void add(Slot *s, double v) { atomicAdd(s, v); }
    __device__ static double value(Slot s) { return s; }
};

template <>
struct TileAcc<float> {
    using Slot = unsigned long long;
    static constexpr bool kFixed = true;
    __device__ static void add(Slot *s, float v) { atomicAdd(s, (unsigned long long)(long long)(int)rintf(v)); }
    __device__ static float value(Slot s) { return (float)(double)(long long)s; }
};

// Storage order of a block's (B+3)^3 P2G tile in global memory. Along each
// axis the tile coordinate t splits into three regions by the block whose
// node it is: t = 0 (the lower neighbour's last layer, 1 node), t = 1..B (the
// block's own nodes), t = B+1, B+2 (the upper neighbour's first two layers).
// The tile is stored region by region (z region, then y, then x), each region
// x-fastest, so the grid update of a neighbour reads one contiguous run per
// region instead of 1- or 2-node pieces of every row.
template <int B>
struct TileRegions {
    static constexpr int TB = B + 3;
    __host__ __device__ static int size(int r) { return r == 0 ? 1 : (r == 1 ? B : 2); }
    __host__ __device__ static int start(int r) { return r == 0 ? 0 : (r == 1 ? 1 : B + 1); }
    __host__ __device__ static int region(int t) { return t == 0 ? 0 : (t <= B ? 1 : 2); }
    __host__ __device__ static int slot(int rx, int ux, int ry, int uy, int rz, int uz)
    {
        const int sx = size(rx), sy = size(ry), sz = size(rz);
        return start(rz) * TB * TB + sz * start(ry) * TB + sz * sy * start(rx) + (uz * sy + uy) * sx + ux;
    }
    // slot of tile coordinates (x, y, z)
    __host__ __device__ static int slot_of(int x, int y, int z)
    {
        const int rx = region(x), ry = region(y), rz = region(z);
        return slot(rx, x - start(rx), ry, y - start(ry), rz, z - start(rz));
    }
    // tile coordinates of slot s (inverse of slot_of)
    __host__ __device__ static void coords(int s, int &x, int &y, int &z)
    {
        const int rz = s < TB * TB ? 0 : (s < (B + 1) * TB * TB ? 1 : 2);
        s -= start(rz) * TB * TB;
        const int sz = size(rz);
        const int ry = s < sz * TB ? 0 : (s < sz * (B + 1) * TB ? 1 : 2);
        s -= sz * start(ry) * TB;
        const int sy = size(ry);
        const int rx = s < sz * sy ? 0 : (s < sz * sy * (B + 1) ? 1 : 2);
        s -= sz * sy * start(rx);
        // region sizes are 1, B or 2: powers of two, so shifts and masks
        const int lx = lg(rx), ly = lg(ry);
        const int ux = s & ((1 << lx) - 1), q = s >> lx;
        x = start(rx) + ux;
        y = start(ry) + (q & ((1 << ly) - 1));
        z = start(rz) + (q >> ly);
    }
    __host__ __device__ static int lg(int r) { return r == 0 ? 0 : (r == 1 ? Log2B<B>::v : 1); }
};

constexpr double kFixedUnits = 268435456.0;     // 2^28 units per particle mass and per m/dt
constexpr float kFixedLimit = 2147483520.0f;     // largest float below 2^31: bound of a scaled contribution

// LDS layout of a P2G tile, four channels per node of the (B+3)^3 tile:
// row (y, z) holds channel 0 (plane 0) or 2 (plane 1) at x and channel 1 or
// 3 at HALF + x; plane 1 starts TLP slots after plane 0.
template <int B>
struct P2GTileLayout {
    static constexpr int TB = B + 3, HALF = B == 8 ? 12 : TB, RP = 2 * HALF, TLP = TB * TB * RP, SLOTS = 2 * TLP;
    __host__ __device__ static constexpr int at(int x, int y, int z, int ch)
    {
        return (ch >> 1) * TLP + (ch & 1) * HALF + (z * TB + y) * RP + x;
    }
};

// LDS layout of a G2P velocity tile, three components per node of the
// (B+3)^3 tile: row (y, z) holds component r at r TB + x.
template <int B>
struct G2PTileLayout {
    static constexpr int TB = B + 3, RP = B == 8 ? 40 : 3 * TB, SLOTS = TB * TB * RP;
    __host__ __device__ static constexpr int at(int x, int y, int z, int r) { return (z * TB + y) * RP + r * TB + x; }
};

// One workgroup per grid block: particles binned to the block scatter mass
// and momentum (Eqs. 2-5) into a (B+3)^3 LDS tile; the whole tile is then
// stored (plain stores, no global atomics) in the block's slot of the tile
// buffer, where the grid update gathers it. FIXDT rebuilds the stress part of
// A when the substep's dt differs from the dt A was formed with:
// A += (dt_A - dt) V0 (4/dx^2) tau. mscale/pscale scale mass and momentum
// into accumulator units (1 in FP64); munit/punit scale back.
template <typename T, int B, bool FIXDT, int MODEL, int WG>
__device__ __forceinline__ void p2g_block(const SimDev<T> &S, const int b, T fix_coef, T mscale, T pscale, T munit,
                                          T punit)
{
    using Acc = TileAcc<T>;
    using Slot = typename Acc::Slot;
    constexpr int TB = B + 3, TN = TB * TB * TB;
    // LDS layout: a row (y, z) of the tile holds two channels side by side,
    // channel 0 (or 2) at x and channel 1 (or 3) at HALF + x, and channels 2
    // and 3 follow in a second plane of TLP slots. For B = 8 a row is 24
    // 8-byte slots (48 banks): the four rows y..y+3 that a half wave of an
    // 8 x 8 particle patch touches then start 16 banks apart modulo 64 and
    // each 64-bit atomic is conflict free, where rows of 11 or 12 slots
    // conflict two-way; the two channels per row cost no extra LDS.
    using L = P2GTileLayout<B>;
    constexpr int HALF = L::HALF, TLP = L::TLP;
    __shared__ Slot tile[L::SLOTS];
    // a force-terminated run that has stopped skips its remaining substeps
    if (S.stop && *S.stop) return;
    // the next substep's bin counts start from zero; the force of the coming
    // grid update too
    if (threadIdx.x == 0) S.cnt_next[b] = 0;
    if (b == 0 && threadIdx.x < 3) S.force[threadIdx.x] = 0.0;
    // a block that overflowed its list keeps only `cap` entries (flagged).
    // The thread's first list entry is read together with the count
    // (speculatively: a list holds cap entries, those past the count are
    // never used) and that particle's state before the tile is cleared; the
    // barrier does not wait for global loads, so they overlap the clearing
    const int *plist = S.perm_cur + (int64_t)b * S.cap;
    const int pf = (int)threadIdx.x < S.cap ? plist[threadIdx.x] : 0;
    const int count = min(S.cnt_cur[b], S.cap);
    if (count == 0) return;
    const int64_t N = S.Ns;
    T fu[3], fv[3], fA[9];
    if ((int)threadIdx.x < count) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            fu[r] = S.u[r * N + pf];
            fv[r] = S.v[r * N + pf];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) fA[k] = S.A[k * N + pf];
    }
    for (int i = threadIdx.x; i < L::SLOTS; i += WG) tile[i] = Slot(0);
    __syncthreads();
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    // tile node (0,0,0) is grid node (lo - 1): a block's particles are those
    // whose cell lies in the block, so their stencil base is lo-1 .. lo+B-1
    const int lo0 = bx * B - 1, lo1 = by * B - 1, lo2 = bz * B - 1;
    const T m = S.m * mscale;
    bool first = true;
    for (int i = threadIdx.x; i < count; i += WG, first = false) {
        int p;
        T uu[3], Am[9], vp[3];
        if (first) {
            p = pf;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                uu[r] = fu[r];
                vp[r] = fv[r];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) Am[k] = fA[k];
        } else {
            p = plist[i];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                uu[r] = S.u[r * N + p];
                vp[r] = S.v[r * N + p];
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) Am[k] = S.A[k * N + p];
            // an empty use keeps A and v next to u: one memory round trip
            // for all of the particle's state
#pragma unroll
            for (int k = 0; k < 9; ++k) asm volatile("" ::"v"(Am[k]));
#pragma unroll
            for (int r = 0; r < 3; ++r) asm volatile("" ::"v"(vp[r]));
        }
        int li0, li1, li2;
        slot_lattice<T, B>(S, (uint32_t)p, li0, li1, li2);
        T xr[3];
        rest_position(S, li0, li1, li2, xr);
        if (!finite3(uu[0], uu[1], uu[2])) {
            atomicOr(S.err, ERR_NONFINITE);
            continue;
        }
        int base[3];
        T f[3];
        stencil_base(xr, uu, base, f);
        const int l0 = base[0] - lo0, l1 = base[1] - lo1, l2 = base[2] - lo2;
        if ((unsigned)l0 > (unsigned)B || (unsigned)l1 > (unsigned)B || (unsigned)l2 > (unsigned)B ||
            base[0] < 0 || base[1] < 0 || base[2] < 0 || base[0] > S.g0 - 3 || base[1] > S.g1 - 3 || base[2] > S.g2 - 3) {
            atomicOr(S.err, ERR_OUT_OF_GRID);
            continue;
        }
        T wx[3], wy[3], wz[3];
        bspline3(f[0], wx);
        bspline3(f[1], wy);
        bspline3(f[2], wz);
        if (FIXDT) {
            T Hm[9], tau[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) Hm[k] = S.H[k * N + p];
            if (!kirchhoff<T, MODEL>(S, Hm, tau)) {
                atomicOr(S.err, MODEL == 0 ? ERR_INVERTED : ERR_NONFINITE);
#pragma unroll
                for (int k = 0; k < 9; ++k) tau[k] = T(0);
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) Am[k] -= fix_coef * tau[k];
        }
        // momentum at node offset o: m v + A (o - f) = q + A o, in accumulator units
        T q[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            q[r] = pscale * (S.m * vp[r] - (Am[r * 3 + 0] * f[0] + Am[r * 3 + 1] * f[1] + Am[r * 3 + 2] * f[2]));
#pragma unroll
        for (int k = 0; k < 9; ++k) Am[k] *= pscale;
        if (Acc::kFixed) {
            T big = T(0);
#pragma unroll
            for (int r = 0; r < 3; ++r)
                big = fmax(big, fabs(q[r]) + T(2) * (fabs(Am[r * 3]) + fabs(Am[r * 3 + 1]) + fabs(Am[r * 3 + 2])));
            if (!(big < T(kFixedLimit))) {
                atomicOr(S.err, ERR_NONFINITE);
                continue;
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const T wab = wx[a] * wy[bb];
                T qa[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) qa[r] = q[r] + Am[r * 3 + 0] * T(a) + Am[r * 3 + 1] * T(bb);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T wt = wab * wz[c];
                    const int li = L::at(l0 + a, l1 + bb, l2 + c, 0);
                    Acc::add(&tile[li], wt * m);
                    Acc::add(&tile[HALF + li], wt * (qa[0] + Am[2] * T(c)));
                    Acc::add(&tile[TLP + li], wt * (qa[1] + Am[5] * T(c)));
                    Acc::add(&tile[TLP + HALF + li], wt * (qa[2] + Am[8] * T(c)));
                }
            }
    }
    __syncthreads();
    T *dst = S.tiles + (int64_t)b * TN * 4;
    // stored in region order (TileRegions): consecutive threads write
    // consecutive slots
    for (int si = threadIdx.x; si < TN; si += WG) {
        T *d = dst + 4 * si;
        int x, y, z;
        TileRegions<B>::coords(si, x, y, z);
        const int ls = L::at(x, y, z, 0);
        d[0] = Acc::value(tile[ls]) * munit;
        d[1] = Acc::value(tile[HALF + ls]) * punit;
        d[2] = Acc::value(tile[TLP + ls]) * punit;
        d[3] = Acc::value(tile[TLP + HALF + ls]) * punit;
    }
}

// 512 threads: the LDS tile allows three workgroups per CU, so a larger
// workgroup is what raises the resident waves (24 per CU) that hide the
// latency between the VALU work and the LDS atomics.
constexpr int kP2GWG = 512;

template <typename T, int B, bool FIXDT, int MODEL>
__global__ void __launch_bounds__(kP2GWG) k_p2g(SimDev<T> S, T fix_coef, T mscale, T pscale, T munit, T punit)
{
    p2g_block<T, B, FIXDT, MODEL, kP2GWG>(S, dispatch_block(S, (int)blockIdx.x), fix_coef, mscale, pscale, munit, punit);
}

// Mass and momentum of grid node (block (bx,by,bz), local (lx,ly,lz)): the sum,
// in a fixed order, of the tiles of the blocks whose (B+3)^3 tile covers it.
// Block c's tile spans nodes lo_c - 1 .. lo_c + B + 1, so along each axis the
// node is covered by its own block, by the lower neighbour when l <= 1 and by
// the upper neighbour when l = B-1. Blocks without particles wrote no tile.
// Bit (oz+1)*9 + (oy+1)*3 + (ox+1) of live27 is set when block (bx+ox,
// by+oy, bz+oz) lies in the grid and holds particles.
template <typename T>
__device__ __forceinline__ uint32_t live_mask(const SimDev<T> &S, int bx, int by, int bz)
{
    uint32_t m = 0;
    for (int t = 0; t < 27; ++t) {
        const int cx = bx + t % 3 - 1, cy = by + (t / 3) % 3 - 1, cz = bz + t / 9 - 1;
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < S.nb0 && cy < S.nb1 && cz < S.nb2 &&
            S.cnt_cur[(cz * S.nb1 + cy) * S.nb0 + cx] > 0)
            m |= 1u << t;
    }
    return m;
}

// Blocks whose (B+3)^3 tile covers local coordinate l of a block along one
// axis, as offsets in increasing order: (-1, 0) when l <= 1, (0, +1) when
// l = B-1, else (0) alone (two = false; o1 = o0 = 0). Block c's tile spans
// nodes lo_c - 1 .. lo_c + B + 1.
template <int B>
__host__ __device__ __forceinline__ void gather_cover(int l, int &o0, int &o1, bool &two)
{
    const int nb = l <= 1 ? -1 : (l == B - 1 ? 1 : 0);
    o0 = nb < 0 ? nb : 0;
    o1 = nb > 0 ? nb : 0;
    two = nb != 0;
}

template <typename T, int B>
__device__ __forceinline__ void gather_node(const SimDev<T> &S, int bx, int by, int bz, int lx, int ly, int lz,
                                            T out[4], uint32_t live27)
{
    constexpr int TB = B + 3, TN = TB * TB * TB;
    const int l[3] = {lx, ly, lz};
    int o[3][2];
    bool two[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) gather_cover<B>(l[a], o[a][0], o[a][1], two[a]);
    // all eight candidate loads are issued before the sum (one memory round
    // trip); a candidate that does not cover the node or wrote no tile reads
    // the node's own slot in its own block, in bounds, and is dropped
    const int64_t own = ((int64_t)((bz * S.nb1 + by) * S.nb0 + bx) * TN +
                         TileRegions<B>::slot_of(lx + 1, ly + 1, lz + 1)) * 4;
    T v[8][4];
    bool use[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
        const int ox = o[0][kx], oy = o[1][ky], oz = o[2][kz];
        const int cx = bx + ox, cy = by + oy, cz = bz + oz;
        const bool ok = (kx == 0 || two[0]) && (ky == 0 || two[1]) && (kz == 0 || two[2]) &&
                        ((live27 >> ((oz + 1) * 9 + (oy + 1) * 3 + (ox + 1))) & 1u);
        // slot of the node in block c's tile (tile origin lo_c - 1; the
        // offset -1/0/+1 selects region 2/1/0 along each axis)
        const int64_t at = ok ? ((int64_t)((cz * S.nb1 + cy) * S.nb0 + cx) * TN +
                                 TileRegions<B>::slot_of(lx - ox * B + 1, ly - oy * B + 1, lz - oz * B + 1)) * 4
                              : own;
        const T *src = S.tiles + at;
        v[k][0] = src[0];
        v[k][1] = src[1];
        v[k][2] = src[2];
        v[k][3] = src[3];
        use[k] = ok;
    }
    // summed in the fixed order z, then y, then x offset ascending
    out[0] = out[1] = out[2] = out[3] = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (use[k]) {
            out[0] += v[k][0];
            out[1] += v[k][1];
            out[2] += v[k][2];
            out[3] += v[k][3];
        }
}

// True when a G2P tile may read this block's velocities: one of the 27
// blocks around it (itself included) holds particles.
template <typename T>
__device__ __forceinline__ bool block_live(const SimDev<T> &S, int bx, int by, int bz)
{
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                const int cx = bx + ox, cy = by + oy, cz = bz + oz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= S.nb0 || cy >= S.nb1 || cz >= S.nb2) continue;
                if (S.cnt_cur[(cz * S.nb1 + cy) * S.nb0 + cx] > 0) return true;
            }
    return false;
}

// ---------------------------------------------------------------- grid update

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Outward unit normal of the indenter at the node r (metres from the
// indenter origin, world frame; p = R^T r in the indenter frame): the
// gradient of phi with respect to r by central differences of step I.eps
// along the world axes. False where the gradient vanishes.
__device__ __forceinline__ bool indenter_normal(const IndenterDev<double> &I, double px, double py, double pz,
                                                double n[3])
{
    double g[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // d p / d r_k is column k of R^T, i.e. row k of R
        const double cx = I.R[3 * k] * I.eps, cy = I.R[3 * k + 1] * I.eps, cz = I.R[3 * k + 2] * I.eps;
        g[k] = (indenter_phi<double>(I, px + cx, py + cy, pz + cz) - indenter_phi<double>(I, px - cx, py - cy, pz - cz)) /
               (2.0 * I.eps);
    }
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(gn > 1e-12)) return false;
    n[0] = g[0] / gn;
    n[1] = g[1] / gn;
    n[2] = g[2] / gn;
    return true;
}

// Velocity of a contact node (cells/s) under Coulomb friction against the
// rigid velocity w (beyond the paper, which leaves friction to future work):
// with the relative velocity split along the outward normal n, a node
// moving apart (vn >= 0) keeps its velocity; an approaching node loses its
// normal component and its tangential one shrinks by mu |vn| (to zero when
// the tangential speed is smaller: stick).
__device__ __forceinline__ void coulomb_contact(const double V[3], const double w[3], const double n[3], double mu,
                                                double out[3])
{
    const double vr[3] = {V[0] - w[0], V[1] - w[1], V[2] - w[2]};
    const double vn = vr[0] * n[0] + vr[1] * n[1] + vr[2] * n[2];
    if (vn >= 0.0) {
        out[0] = V[0]; out[1] = V[1]; out[2] = V[2];
        return;
    }
    const double vt[3] = {vr[0] - vn * n[0], vr[1] - vn * n[1], vr[2] - vn * n[2]};
    const double t = sqrt(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    const double k = t > 0.0 ? fmax(0.0, 1.0 + mu * vn / t) : 0.0;
    out[0] = w[0] + k * vt[0];
    out[1] = w[1] + k * vt[1];
    out[2] = w[2] + k * vt[2];
}

// One workgroup per grid block that a G2P tile may read (the block or one of
// its 26 neighbours has particles). Per node with mass above S.m_floor
// (0 in FP64; in FP32 2^-22 of a particle's mass, below which P/M is
// dominated by fixed-point quantisation and the node's weight in any particle
// is negligible): V = P/M + dt g (Eq. 6);
// inside the indenter V takes the rigid indenter velocity (sticky contact)
// or the Coulomb update (CONTACT_COULOMB), or, for an indenter represented
// by particles (CONTACT_PARTICLES), the velocity of the node's gel momentum
// plus the indenter points' momentum; the reaction M (V_before - V_after)/dt
// is summed into the force;
// floor nodes are held; wall nodes drop their outward component. The inside test and the
// rigid velocity are evaluated in FP64 in both precisions, so the discrete
// contact decision does not depend on the simulation precision.
constexpr int CONTACT_STICKY = 0, CONTACT_COULOMB = 1, CONTACT_PARTICLES = 2;

// Velocity of one grid node from its gathered mass and momentum mp (Eq. 6
// with the contact of Eq. 10, floor and walls; the rules above), in cells/s;
// a contact node adds its reaction M (V_before - V_after)/dt to f (in FP64).
template <typename T, int CONTACT>
__device__ __forceinline__ void node_velocity(const SimDev<T> &S, const IndenterDev<double> &I, int gx, int gy, int gz,
                                              const T mp[4], T dt, T inv_dt, T V[3], double f[3])
{
    const T m = mp[0];
    T V0 = T(0), V1 = T(0), V2 = T(0);
    if (m > S.m_floor && gx < S.g0 && gy < S.g1 && gz < S.g2) {
        const T im = T(1) / m;
        V0 = mp[1] * im + dt * S.grav[0];
        V1 = mp[2] * im + dt * S.grav[1];
        V2 = mp[3] * im + dt * S.grav[2];
        if (I.shape >= 0) {
            // node relative to the indenter origin, metres, then indenter frame
            const double r0 = ((double)gx - I.tip[0]) * I.dx, r1 = ((double)gy - I.tip[1]) * I.dx,
                         r2 = ((double)gz - I.tip[2]) * I.dx;
            const double px = I.R[0] * r0 + I.R[3] * r1 + I.R[6] * r2;
            const double py = I.R[1] * r0 + I.R[4] * r1 + I.R[7] * r2;
            const double pz = I.R[2] * r0 + I.R[5] * r1 + I.R[8] * r2;
            // particle indenter: the node is in contact where the points
            // scattered mass; else where the shape's signed distance is <= 0
            const double mi = CONTACT == CONTACT_PARTICLES && gx >= I.blo[0] && gx <= I.bhi[0] &&
                                      gy >= I.blo[1] && gy <= I.bhi[1] && gz >= I.blo[2] && gz <= I.bhi[2]
                                  ? I.MI[gx + (int64_t)S.g0 * (gy + (int64_t)S.g1 * gz)]
                                  : 0.0;
            // below the solid's lowest level the node is outside: the
            // signed distance (the plate's noise above all) is skipped
            if (CONTACT == CONTACT_PARTICLES ? mi > 0.0
                                             : (pz >= I.zmin && indenter_phi<double>(I, px, py, pz) <= 0.0)) {
                // rigid velocity v_c + omega x r, converted to cells/s
                const double ir = 1.0 / I.dx;
                const double wd[3] = {I.vc[0] + (I.om[1] * r2 - I.om[2] * r1) * ir,
                                      I.vc[1] + (I.om[2] * r0 - I.om[0] * r2) * ir,
                                      I.vc[2] + (I.om[0] * r1 - I.om[1] * r0) * ir};
                T w0 = T(wd[0]), w1 = T(wd[1]), w2 = T(wd[2]);
                double nrm[3];
                if (CONTACT == CONTACT_COULOMB && indenter_normal(I, px, py, pz, nrm)) {
                    const double Vd[3] = {(double)V0, (double)V1, (double)V2};
                    double Va[3];
                    coulomb_contact(Vd, wd, nrm, I.mu, Va);
                    w0 = T(Va[0]); w1 = T(Va[1]); w2 = T(Va[2]);
                }
                if (CONTACT == CONTACT_PARTICLES) {
                    // the points move with the rigid velocity (Eq. 10): their
                    // momentum on the node is mi w (APIC with the rigid velocity
                    // gradient is exact), and the node takes the velocity of
                    // the summed momentum
                    const double md = (double)m;
                    w0 = T((md * (double)V0 + mi * wd[0]) / (md + mi));
                    w1 = T((md * (double)V1 + mi * wd[1]) / (md + mi));
                    w2 = T((md * (double)V2 + mi * wd[2]) / (md + mi));
                }
                const T sc = m * T(I.dx) * inv_dt;
                f[0] += (double)(sc * (V0 - w0));
                f[1] += (double)(sc * (V1 - w1));
                f[2] += (double)(sc * (V2 - w2));
                V0 = w0; V1 = w1; V2 = w2;
            }
        }
        if (gz <= S.floor_node) V0 = V1 = V2 = T(0);
        if ((gx < S.wall && V0 < T(0)) || (gx > S.g0 - 1 - S.wall && V0 > T(0))) V0 = T(0);
        if ((gy < S.wall && V1 < T(0)) || (gy > S.g1 - 1 - S.wall && V1 > T(0))) V1 = T(0);
        if ((gz < S.wall && V2 < T(0)) || (gz > S.g2 - 1 - S.wall && V2 > T(0))) V2 = T(0);
    }
    V[0] = V0; V[1] = V1; V[2] = V2;
}

template <typename T, int B, int WG, int CONTACT = CONTACT_STICKY>
__device__ __forceinline__ void grid_block(const SimDev<T> &S, const int b, const IndenterDev<double> &I, T dt)
{
    constexpr int B3 = B * B * B;
    if (S.stop && *S.stop) return;
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    // particle counts of the 27 surrounding blocks, loaded once per workgroup
    __shared__ int nc27[27];
    if (threadIdx.x < 27) {
        const int t = threadIdx.x;
        const int cx = bx + t % 3 - 1, cy = by + (t / 3) % 3 - 1, cz = bz + t / 9 - 1;
        const bool in = cx >= 0 && cy >= 0 && cz >= 0 && cx < S.nb0 && cy < S.nb1 && cz < S.nb2;
        nc27[t] = in ? S.cnt_cur[(cz * S.nb1 + cy) * S.nb0 + cx] : 0;
    }
    __syncthreads();
    uint32_t live27 = 0;
#pragma unroll
    for (int t = 0; t < 27; ++t) live27 |= nc27[t] > 0 ? 1u << t : 0u;
    if (!live27) return;
    double f[3] = {0.0, 0.0, 0.0};
    const T inv_dt = T(1) / dt;
    for (int l = threadIdx.x; l < B3; l += WG) {
        const int lx = l % B, ly = (l / B) % B, lz = l / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        const int64_t addr = (int64_t)b * B3 + node_local<B>(lx, ly, lz);
        T mp[4], V[3];
        gather_node<T, B>(S, bx, by, bz, lx, ly, lz, mp, live27);
        node_velocity<T, CONTACT>(S, I, gx, gy, gz, mp, dt, inv_dt, V, f);
        T *vv = S.V + 3 * addr;
        vv[0] = V[0]; vv[1] = V[1]; vv[2] = V[2];
    }
    double fx = f[0], fy = f[1], fz = f[2];
    if (I.shape >= 0) {
        __shared__ double red[3][WG / 64];
        fx = wave_sum(fx); fy = wave_sum(fy); fz = wave_sum(fz);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { red[0][w] = fx; red[1][w] = fy; red[2][w] = fz; }
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int k = 0; k < WG / 64; ++k) s += red[threadIdx.x][k];
            if (s != 0.0) atomicAdd(&S.force[threadIdx.x], s);
        }
    }
}

// One instantiation per contact model: the no-slip kernel carries none of
// the Coulomb code (the normal's six extra shape evaluations would otherwise
// raise the register count of every grid update)
template <typename T, int B, int CONTACT>
__global__ void __launch_bounds__(kWG) k_grid(SimDev<T> S, IndenterDev<double> I, T dt)
{
    grid_block<T, B, kWG, CONTACT>(S, dispatch_halo_block(S, (int)blockIdx.x), I, dt);
}

// Zeroes MI over the node box lo..hi (inclusive; x fastest in MI).
__global__ void __launch_bounds__(kWG) k_clear_box(double *MI, int g0, int g1, int lo0, int lo1, int lo2, int nx,
                                                   int ny, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    const int x = (int)(i % nx);
    const int64_t t = i / nx;
    const int y = (int)(t % ny), z = (int)(t / ny);
    MI[(lo0 + x) + (int64_t)g0 * ((lo1 + y) + (int64_t)g1 * (lo2 + z))] = 0.0;
}

// Particle indenter: each point (indenter frame, metres) placed at the pose
// of the substep's start scatters w * mass to its 3x3x3 nodes (the weights
// of Eq. 2) in the dense node array MI (x fastest, cleared before); points
// whose nodes leave the grid are ignored. The points are stored in spatial
// (Morton) order, so a workgroup's points cover a small node box: their
// weights are summed in an LDS tile over that box (LDS FP64 atomics) and
// flushed with one global FP64 atomic per touched node, instead of 27 global
// atomics per point on nodes shared by ~100 points. A workgroup whose box
// exceeds the tile, or holds more than half as many nodes as its points have
// weights (a sparse cloud: the tile would save little), adds its points
// directly.
constexpr int kScatterEdge = 16;

// The (z, y) node offsets of step (cc, bc) of a point's scatter, rotated by
// the lane: neighbouring points of the spatially sorted cloud share most of
// their nodes, and same-address atomics of one wave serialise, so each lane
// starts at a different (z, y) row. Returns the offsets and w_z * w_y.
__device__ __forceinline__ void rotated_pair(int cc, int bc, const double (&w)[3][3], int &c, int &bb, double &wzy)
{
    const int lane = threadIdx.x & 63;
    c = cc + lane % 3;
    c = c >= 3 ? c - 3 : c;
    bb = bc + (lane / 3) % 3;
    bb = bb >= 3 ? bb - 3 : bb;
    const double wz = c == 0 ? w[2][0] : (c == 1 ? w[2][1] : w[2][2]);
    const double wy = bb == 0 ? w[1][0] : (bb == 1 ? w[1][1] : w[1][2]);
    wzy = wz * wy;
}

__global__ void __launch_bounds__(kWG) k_indenter_scatter(const double *pts, int n, IndenterDev<double> I, int g0,
                                                          int g1, int g2, double mass, double *MI)
{
    __shared__ double tile[kScatterEdge * kScatterEdge * kScatterEdge];
    __shared__ int bmin[3], bmax[3], nvalid;
    if (threadIdx.x < 3) {
        bmin[threadIdx.x] = 0x7fffffff;
        bmax[threadIdx.x] = -1;
    }
    if (threadIdx.x == 0) nvalid = 0;
    __syncthreads();
    const int k = blockIdx.x * kWG + threadIdx.x;
    const int gn[3] = {g0, g1, g2};
    int base[3] = {0, 0, 0};
    double w[3][3];
    bool ok = k < n;
    if (ok) {
        const double l0 = pts[3 * k], l1 = pts[3 * k + 1], l2 = pts[3 * k + 2];
        const double ir = 1.0 / I.dx;
        // grid coordinates: origin + R l (R indenter frame -> world, row-major)
        const double xg[3] = {I.tip[0] + (I.R[0] * l0 + I.R[1] * l1 + I.R[2] * l2) * ir,
                              I.tip[1] + (I.R[3] * l0 + I.R[4] * l1 + I.R[5] * l2) * ir,
                              I.tip[2] + (I.R[6] * l0 + I.R[7] * l1 + I.R[8] * l2) * ir};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double b = floor(xg[a] - 0.5);
            ok = ok && b >= 0.0 && b <= (double)(gn[a] - 3);
            base[a] = ok ? (int)b : 0;
            bspline3<double>(xg[a] - b, w[a]);
        }
    }
    if (ok) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            atomicMin(&bmin[a], base[a]);
            atomicMax(&bmax[a], base[a]);
        }
        atomicAdd(&nvalid, 1);
    }
    __syncthreads();
    if (bmax[0] < 0) return;  // no point of the workgroup in the grid
    const int ex = bmax[0] - bmin[0] + 3, ey = bmax[1] - bmin[1] + 3, ez = bmax[2] - bmin[2] + 3;
    if (ex <= kScatterEdge && ey <= kScatterEdge && ez <= kScatterEdge && 2 * ex * ey * ez <= 27 * nvalid) {
        const int ne = ex * ey * ez;
        for (int i = threadIdx.x; i < ne; i += kWG) tile[i] = 0.0;
        __syncthreads();
        if (ok)
            for (int cc = 0; cc < 3; ++cc)
                for (int bc = 0; bc < 3; ++bc) {
                    int c, bb;
                    double wzy;
                    rotated_pair(cc, bc, w, c, bb, wzy);
                    for (int a = 0; a < 3; ++a)
                        atomicAdd(&tile[((base[2] - bmin[2] + c) * ey + (base[1] - bmin[1] + bb)) * ex +
                                        (base[0] - bmin[0] + a)],
                                  w[0][a] * wzy * mass);
                }
        __syncthreads();
        for (int i = threadIdx.x; i < ne; i += kWG) {
            const double v = tile[i];
            if (v != 0.0) {
                const int x = i % ex, t = i / ex, y = t % ey, z = t / ey;
                atomicAdd(&MI[(bmin[0] + x) + (int64_t)g0 * ((bmin[1] + y) + (int64_t)g1 * (bmin[2] + z))], v);
            }
        }
    } else if (ok) {
        for (int cc = 0; cc < 3; ++cc)
            for (int bc = 0; bc < 3; ++bc) {
                int c, bb;
                double wzy;
                rotated_pair(cc, bc, w, c, bb, wzy);
                for (int a = 0; a < 3; ++a)
                    atomicAdd(&MI[(base[0] + a) + (int64_t)g0 * ((base[1] + bb) + (int64_t)g1 * (base[2] + c))],
                              w[0][a] * wzy * mass);
            }
    }
}

// ---------------------------------------------------------------- G2P

// Bin lists are filled by atomic appends, one run per wave and destination,
// so where many particles change blocks (under a wide indenter) a block's
// list breaks into short runs of slots from different lattice tiles, and the
// SoA loads and stores of G2P and P2G touch several times the cache lines of
// a contiguous run (measured: G2P 177 against 134 us under the textured
// plate). Every kSortEvery-th G2P sorts each list by slot first (bitonic sort
// in LDS); the appends of a sorted pass keep runs long for the next
// substeps. Sorting every substep cost the undisturbed presses ~20 us per G2P;
// every 4th, 8th and 16th substep measured alike (plate 107-110 us, sphere
// 80-85 us per G2P), the 16th slightly ahead.
constexpr int kSortMax = 2048;   // longer lists (more than 4 particles per cell) stay unsorted
constexpr int kSortEvery = 16;

// One workgroup per grid block: the block's (B+3)^3 velocity tile is staged
// in LDS; each particle gathers v and C (Eqs. 7-8, with the grid velocities
// in Eq. 8), updates F (Eq. 9), forms the stress and the affine momentum
// A = m C - dt V0 (4/dx^2) tau for the next P2G, applies the bonded bottom
// layers (Eq. 10), advects (Eq. 11) and appends itself to the bin list of
// the block holding its new stencil base.
template <typename T, int B, int MODEL, int WG, bool SORT = false>
__device__ __forceinline__ void g2p_block(const SimDev<T> &S, const int b, T dt, T stress_coef)
{
    constexpr int TB = B + 3, TN = TB * TB * TB;
    // LDS layout: row (y, z) holds the three velocity components side by
    // side (component r at r*TB + x). For B = 8 a row is 40 words: the eight
    // rows of an 8 x 8 particle patch then start on distinct multiples of 8
    // banks modulo 64 and every LDS read of the gather is conflict free,
    // where rows of 11 words conflict.
    using L = G2PTileLayout<B>;
    constexpr int RP = L::RP;
    __shared__ T tile[L::SLOTS];
    // the thread's first list entry is read with the count (speculatively,
    // as in P2G) and its particle's state behind the tile's staging loads:
    // the barrier does not wait for global loads, so the particle work
    // starts two memory round trips after the kernel instead of four
    if (S.stop && *S.stop) return;
    const int *plist = S.perm_cur + (int64_t)b * S.cap;
    __shared__ int lst[SORT ? kSortMax : 1];
    const int pf = !SORT && (int)threadIdx.x < S.cap ? plist[threadIdx.x] : 0;
    const int count = min(S.cnt_cur[b], S.cap);
    if (count == 0) return;
    const bool sorted = SORT && count <= kSortMax;
    int P = 1;
    if (sorted) {
        while (P < count) P <<= 1;
        for (int i = threadIdx.x; i < P; i += WG) lst[i] = i < count ? plist[i] : 0x7fffffff;
    }
    const int64_t N = S.Ns;
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    // tile node (0,0,0) is grid node (lo - 1): a block's particles are those
    // whose cell lies in the block, so their stencil base is lo-1 .. lo+B-1
    const int lo0 = bx * B - 1, lo1 = by * B - 1, lo2 = bz * B - 1;
    // every load of a thread's share of the tile is issued before the first
    // LDS write, so the staging costs one memory round trip, not one per node
    constexpr int NPT = (TN + WG - 1) / WG;
    T st[NPT][3];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int li = threadIdx.x + k * WG;
        const int x = li % TB, yz = li / TB, y = yz % TB, z = yz / TB;
        const int gx = lo0 + x, gy = lo1 + y, gz = lo2 + z;
        st[k][0] = st[k][1] = st[k][2] = T(0);
        if (li < TN && (unsigned)gx < (unsigned)S.g0 && (unsigned)gy < (unsigned)S.g1 &&
            (unsigned)gz < (unsigned)S.g2) {
            const T *src = S.V + 3 * node_addr<B>(S.nb0, S.nb1, gx, gy, gz);
            st[k][0] = src[0]; st[k][1] = src[1]; st[k][2] = src[2];
        }
    }
    T fu[3], fh[9];
    if (!SORT && (int)threadIdx.x < count) {
#pragma unroll
        for (int r = 0; r < 3; ++r) fu[r] = S.u[r * N + pf];
#pragma unroll
        for (int k = 0; k < 9; ++k) fh[k] = S.H[k * N + pf];
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int li = threadIdx.x + k * WG;
        if (li < TN) {
            const int x = li % TB, yz = li / TB;
            tile[L::at(x, yz, 0, 0)] = st[k][0];
            tile[L::at(x, yz, 0, 1)] = st[k][1];
            tile[L::at(x, yz, 0, 2)] = st[k][2];
        }
    }
    __syncthreads();
    // bitonic sort of the list by slot (padded to a power of two)
    if (sorted) {
        for (int k = 2; k <= P; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < (P >> 1); i += WG) {
                    const int a = 2 * i - (i & (j - 1)), c = a + j;
                    const int x = lst[a], y = lst[c];
                    if ((x > y) == ((a & k) == 0)) {
                        lst[a] = y;
                        lst[c] = x;
                    }
                }
                __syncthreads();
            }
    }
    for (int i0 = 0; i0 < count; i0 += WG) {
        const int i = i0 + threadIdx.x;
        int newkey = -1;
        int p = 0;
        if (i < count) {
            T uu[3], h[9];
            if (!SORT && i0 == 0) {
                p = pf;
#pragma unroll
                for (int r = 0; r < 3; ++r) uu[r] = fu[r];
#pragma unroll
                for (int k = 0; k < 9; ++k) h[k] = fh[k];
            } else {
                p = sorted ? lst[i] : plist[i];
#pragma unroll
                for (int r = 0; r < 3; ++r) uu[r] = S.u[r * N + p];
                // H is loaded with u, before the stores below: the compiler
                // cannot move loads across stores to other arrays, and the
                // stores would otherwise add a second memory round trip; an
                // empty use keeps the loads here instead of sunk to the F update
#pragma unroll
                for (int k = 0; k < 9; ++k) h[k] = S.H[k * N + p];
#pragma unroll
                for (int k = 0; k < 9; ++k) asm volatile("" ::"v"(h[k]));
            }
            int li0, li1, li2;
            slot_lattice<T, B>(S, (uint32_t)p, li0, li1, li2);
            T xr[3];
            rest_position(S, li0, li1, li2, xr);
            int base[3] = {0, 0, 0};
            T f[3];
            const bool fin = finite3(uu[0], uu[1], uu[2]);
            if (fin) stencil_base(xr, uu, base, f);
            const int l0 = base[0] - lo0, l1 = base[1] - lo1, l2 = base[2] - lo2;
            if (!fin) {
                atomicOr(S.err, ERR_NONFINITE);
                newkey = b;
            } else if ((unsigned)l0 > (unsigned)B || (unsigned)l1 > (unsigned)B || (unsigned)l2 > (unsigned)B ||
                       base[0] < 0 || base[1] < 0 || base[2] < 0 || base[0] > S.g0 - 3 || base[1] > S.g1 - 3 || base[2] > S.g2 - 3) {
                atomicOr(S.err, ERR_OUT_OF_GRID);
                newkey = b;
            } else {
                T wx[3], wy[3], wz[3];
                bspline3(f[0], wx);
                bspline3(f[1], wy);
                bspline3(f[2], wz);
                // velocities relative to the stencil centre keep the affine
                // sums well conditioned in FP32
                const int lc = L::at(l0 + 1, l1 + 1, l2 + 1, 0);
                const T vr[3] = {tile[lc], tile[TB + lc], tile[2 * TB + lc]};
                // The weights are a tensor product, so the sums over the 27
                // nodes of w D, w D a, w D b, w D c (D = V - vr, offsets a, b,
                // c along x, y, z) are taken one axis at a time: over c, then
                // b, then a.
                T sx[3], sy[3], sz[3], sr[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    T u[3], uy[3], uz[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        T t[3], tz[3];
#pragma unroll
                        for (int bb = 0; bb < 3; ++bb) {
                            const int li = L::at(l0 + a, l1 + bb, l2, r);
                            const T d0 = tile[li] - vr[r];
                            const T d1 = tile[li + TB * RP] - vr[r];
                            const T d2 = tile[li + 2 * TB * RP] - vr[r];
                            t[bb] = wz[0] * d0 + wz[1] * d1 + wz[2] * d2;
                            tz[bb] = wz[1] * d1 + T(2) * wz[2] * d2;
                        }
                        u[a] = wy[0] * t[0] + wy[1] * t[1] + wy[2] * t[2];
                        uy[a] = wy[1] * t[1] + T(2) * wy[2] * t[2];
                        uz[a] = wy[0] * tz[0] + wy[1] * tz[1] + wy[2] * tz[2];
                    }
                    sr[r] = wx[0] * u[0] + wx[1] * u[1] + wx[2] * u[2];
                    sx[r] = wx[1] * u[1] + T(2) * wx[2] * u[2];
                    sy[r] = wx[0] * uy[0] + wx[1] * uy[1] + wx[2] * uy[2];
                    sz[r] = wx[0] * uz[0] + wx[1] * uz[1] + wx[2] * uz[2];
                }
                // sum w V = sum w D + vr sum w, with sum w the product of the
                // per-axis weight sums
                const T wsum = (wx[0] + wx[1] + wx[2]) * (wy[0] + wy[1] + wy[2]) * (wz[0] + wz[1] + wz[2]);
                const T s0[3] = {sr[0] + vr[0] * wsum, sr[1] + vr[1] * wsum, sr[2] + vr[2] * wsum};
                // C = (4/dx^2) sum w V (X_i - x_p)^T, in 1/s with grid-unit offsets
                T Cm[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Cm[r * 3 + 0] = T(4) * (sx[r] - sr[r] * f[0]);
                    Cm[r * 3 + 1] = T(4) * (sy[r] - sr[r] * f[1]);
                    Cm[r * 3 + 2] = T(4) * (sz[r] - sr[r] * f[2]);
                }
                T vn[3] = {s0[0], s0[1], s0[2]};
                if (li2 < S.n_fixed) vn[0] = vn[1] = vn[2] = T(0);
    #pragma unroll
                for (int r = 0; r < 3; ++r) {
                    S.v[r * N + p] = vn[r];
                    uu[r] += dt * vn[r];
                    S.u[r * N + p] = uu[r];
                }
                // F <- (I + dt C) F, i.e. H <- H + dt (C + C H), one column at a time
                T Hn[9];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T h0 = h[0 * 3 + c], h1 = h[1 * 3 + c], h2 = h[2 * 3 + c];
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const T hrc = r == 0 ? h0 : (r == 1 ? h1 : h2);
                        Hn[r * 3 + c] = hrc + dt * (Cm[r * 3 + c] + Cm[r * 3 + 0] * h0 + Cm[r * 3 + 1] * h1 +
                                                    Cm[r * 3 + 2] * h2);
                    }
                }
#pragma unroll
                for (int k = 0; k < 9; ++k) S.H[k * N + p] = Hn[k];
                T tau[9];
                if (!kirchhoff<T, MODEL>(S, Hn, tau)) {
                    atomicOr(S.err, MODEL == 0 ? ERR_INVERTED : ERR_NONFINITE);
#pragma unroll
                    for (int k = 0; k < 9; ++k) tau[k] = T(0);
                }
#pragma unroll
                for (int k = 0; k < 9; ++k) S.A[k * N + p] = S.m * Cm[k] - stress_coef * tau[k];
                newkey = block_key<T, B>(S, xr, uu);
            }
        }
        bin_append(S, S.cnt_next, S.perm_next, newkey, (uint32_t)p);
    }
}

template <typename T, int B, int MODEL, bool SORT>
__global__ void __launch_bounds__(kWG) k_g2p(SimDev<T> S, T dt, T stress_coef)
{
    g2p_block<T, B, MODEL, kWG, SORT>(S, dispatch_block(S, (int)blockIdx.x), dt, stress_coef);
}


// ---------------------------------------------------------------- outputs

// out[j][i] = world z of top-layer particle (i, j).
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_heightmap(SimDev<T> S, T origin_z, T dx, T *out)
{
    const int idx = blockIdx.x * kWG + threadIdx.x;
    if (idx >= S.n0 * S.n1) return;
    const int j = idx / S.n0, i = idx - j * S.n0;
    const uint32_t s = lattice_slot<T, B>(S, i, j, S.n2 - 1);
    const T zr = S.xr[2] + T(S.n2 - 1) * S.hr[2];
    out[idx] = origin_z + dx * (zr + S.u[2 * S.Ns + s]);
}

// Displacement of the top surface over a res x res partition of the block's
// top face: out[(r res + c) 3 + a] (metres, FP32) is the mean, over sub x sub
// points spread evenly inside cell (c, r) (at ((c + (q + 1/2)/sub) L / res),
// q = 0 .. sub-1, per axis), of the displacement interpolated bilinearly
// between the top-layer particles (particle i sits at (i + 1/2) h; clamped at
// the border). sub = 1 samples the cell centre.
// Displacement (grid units) of the top surface at fractional lattice
// coordinates (si, sj) of the top layer, si in [0, n0-1], sj in [0, n1-1]:
// bilinear in the four surrounding top-layer particles.
template <typename T, int B>
__device__ __forceinline__ void top_disp_at(const SimDev<T> &S, T si, T sj, T out[3])
{
    const int k = S.n2 - 1;
    int i0 = (int)tfloor<T>(si), j0 = (int)tfloor<T>(sj);
    i0 = i0 > S.n0 - 2 ? S.n0 - 2 : i0;
    j0 = j0 > S.n1 - 2 ? S.n1 - 2 : j0;
    const T tx = si - T(i0), ty = sj - T(j0);
    const uint32_t s00 = lattice_slot<T, B>(S, i0, j0, k), s10 = lattice_slot<T, B>(S, i0 + 1, j0, k);
    const uint32_t s01 = lattice_slot<T, B>(S, i0, j0 + 1, k), s11 = lattice_slot<T, B>(S, i0 + 1, j0 + 1, k);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T *u = S.u + (size_t)a * S.Ns;
        const T lo = u[s00] + tx * (u[s10] - u[s00]);
        const T hi = u[s01] + tx * (u[s11] - u[s01]);
        out[a] = lo + ty * (hi - lo);
    }
}

// Markers (surface points tracked through the press): q holds n fractional
// top-layer lattice coordinates (si, sj), already clamped; out [n][3] the
// displacement in metres.
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_markers(SimDev<T> S, const T *q, int n, T dx, T *out)
{
    const int idx = blockIdx.x * kWG + threadIdx.x;
    if (idx >= n) return;
    T d[3];
    top_disp_at<T, B>(S, q[2 * idx], q[2 * idx + 1], d);
#pragma unroll
    for (int a = 0; a < 3; ++a) out[(size_t)idx * 3 + a] = dx * d[a];
}

template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_surface_disp(SimDev<T> S, T dx, int res, int sub, float *out)
{
    const int idx = blockIdx.x * kWG + threadIdx.x;
    if (idx >= res * res) return;
    const int r = idx / res, c = idx - r * res;
    T acc[3] = {T(0), T(0), T(0)};
    for (int qy = 0; qy < sub; ++qy)
        for (int qx = 0; qx < sub; ++qx) {
            T si = (T(c) + (T(qx) + T(0.5)) / T(sub)) * T(S.n0) / T(res) - T(0.5);
            T sj = (T(r) + (T(qy) + T(0.5)) / T(sub)) * T(S.n1) / T(res) - T(0.5);
            si = si < T(0) ? T(0) : (si > T(S.n0 - 1) ? T(S.n0 - 1) : si);
            sj = sj < T(0) ? T(0) : (sj > T(S.n1 - 1) ? T(S.n1 - 1) : sj);
            T d[3];
            top_disp_at<T, B>(S, si, sj, d);
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[a] += d[a];
        }
    const T w = dx / T(sub * sub);
#pragma unroll
    for (int a = 0; a < 3; ++a) out[(size_t)idx * 3 + a] = (float)(w * acc[a]);
}

template <typename T>
struct RenderDev {
    int n0, n1, h, w;
    T x0, y0;          // world position of lattice column 0 / row 0
    T hx, hy;          // lattice spacing
    T cx, cy;          // image centre
    T pitch;
    T ka, kd, ks, alpha;
    T L[3][3];         // unit light directions (surface -> light)
};

template <typename T>
__device__ __forceinline__ T sample_height(const T *Hm, const RenderDev<T> &R, int u, int v)
{
    const T X = R.cx + (T(u) - T(0.5) * T(R.w - 1)) * R.pitch;
    const T Y = R.cy + (T(v) - T(0.5) * T(R.h - 1)) * R.pitch;
    const T sx = (X - R.x0) / R.hx, sy = (Y - R.y0) / R.hy;
    T fi = tfloor<T>(sx), fj = tfloor<T>(sy);
    fi = fi < T(0) ? T(0) : (fi > T(R.n0 - 2) ? T(R.n0 - 2) : fi);
    fj = fj < T(0) ? T(0) : (fj > T(R.n1 - 2) ? T(R.n1 - 2) : fj);
    T tx = sx - fi, ty = sy - fj;
    tx = tx < T(0) ? T(0) : (tx > T(1) ? T(1) : tx);
    ty = ty < T(0) ? T(0) : (ty > T(1) ? T(1) : ty);
    const int i0 = (int)fi, j0 = (int)fj;
    const T *r0 = Hm + (int64_t)j0 * R.n0 + i0;
    const T *r1 = r0 + R.n0;
    return (T(1) - ty) * ((T(1) - tx) * r0[0] + tx * r0[1]) + ty * ((T(1) - tx) * r1[0] + tx * r1[1]);
}

// Tactile image: bilinear resample of the depth map at the pixel and its four
// neighbours (replicated at the border), normal from central differences,
// Phong per channel with its own light (Eqs. 12-14).
template <typename T>
__global__ void __launch_bounds__(kWG) k_render(const T *Hm, RenderDev<T> R, float *rgb)
{
    const int idx = blockIdx.x * kWG + threadIdx.x;
    if (idx >= R.h * R.w) return;
    const int v = idx / R.w, u = idx - v * R.w;
    const int ul = u > 0 ? u - 1 : 0, ur = u < R.w - 1 ? u + 1 : R.w - 1;
    const int vd = v > 0 ? v - 1 : 0, vu = v < R.h - 1 ? v + 1 : R.h - 1;
    const T gx = (sample_height(Hm, R, ur, v) - sample_height(Hm, R, ul, v)) / (T(2) * R.pitch);
    const T gy = (sample_height(Hm, R, u, vu) - sample_height(Hm, R, u, vd)) / (T(2) * R.pitch);
    const T inv = T(1) / sqrt(gx * gx + gy * gy + T(1));
    const T N[3] = {gx * inv, gy * inv, -inv};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const T ln = R.L[ch][0] * N[0] + R.L[ch][1] * N[1] + R.L[ch][2] * N[2];
        T I = R.ka;
        if (ln > T(0)) {
            I += R.kd * ln;
            // reflected ray R = 2 (L.N) N - L; view direction (0, 0, -1)
            const T rv = -(T(2) * ln * N[2] - R.L[ch][2]);
            if (rv > T(0)) I += R.ks * pow(rv, R.alpha);
        }
        I = I < T(0) ? T(0) : (I > T(1) ? T(1) : I);
        rgb[(int64_t)idx * 3 + ch] = (float)I;
    }
}

// ---------------------------------------------------------------- state conversion

// Particle state in the ABI's order and units (SoA over p = i + n0 (j + n1 k)).
template <typename T, int B, int MODEL>
__global__ void __launch_bounds__(kWG) k_read_particles(SimDev<T> S, T ox, T oy, T oz, T dx, T dtA_coef,
                                                        T *x, T *v, T *C, T *F)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= S.N) return;
    const int64_t N = S.N, Ns = S.Ns;
    int i, j, k;
    api_lattice(S, (uint32_t)p, i, j, k);
    const int64_t s = lattice_slot<T, B>(S, i, j, k);
    T xr[3];
    rest_position(S, i, j, k, xr);
    if (x) {
        x[p] = ox + dx * (xr[0] + S.u[s]);
        x[N + p] = oy + dx * (xr[1] + S.u[Ns + s]);
        x[2 * N + p] = oz + dx * (xr[2] + S.u[2 * Ns + s]);
    }
    if (v)
        for (int r = 0; r < 3; ++r) v[r * N + p] = dx * S.v[r * Ns + s];
    T Hm[9];
    for (int q = 0; q < 9; ++q) Hm[q] = S.H[q * Ns + s];
    if (F)
        for (int q = 0; q < 9; ++q) F[q * N + p] = Hm[q] + ((q % 4 == 0) ? T(1) : T(0));
    if (C) {
        T tau[9];
        if (dtA_coef == T(0) || !kirchhoff<T, MODEL>(S, Hm, tau))
            for (int q = 0; q < 9; ++q) tau[q] = T(0);
        for (int q = 0; q < 9; ++q) C[q * N + p] = (S.A[q * Ns + s] + dtA_coef * tau[q]) / S.m;
    }
}

// Writes a state given in SI/world terms; A is stored as m C (the stress part
// is added by the next P2G, which sees dt_A = 0).
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_write_particles(SimDev<T> S, T ox, T oy, T oz, T inv_dx,
                                                         const T *x, const T *v, const T *C, const T *F)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= S.N) return;
    const int64_t N = S.N, Ns = S.Ns;
    int i, j, k;
    api_lattice(S, (uint32_t)p, i, j, k);
    const int64_t s = lattice_slot<T, B>(S, i, j, k);
    T xr[3];
    rest_position(S, i, j, k, xr);
    const T o[3] = {ox, oy, oz};
    for (int r = 0; r < 3; ++r) {
        S.u[r * Ns + s] = (x[r * N + p] - o[r]) * inv_dx - xr[r];
        S.v[r * Ns + s] = v[r * N + p] * inv_dx;
    }
    for (int q = 0; q < 9; ++q) {
        S.H[q * Ns + s] = F[q * N + p] - ((q % 4 == 0) ? T(1) : T(0));
        S.A[q * Ns + s] = S.m * C[q * N + p];
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_init_particles(SimDev<T> S)
{
    const int64_t s = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (s >= S.Ns) return;
    const int64_t Ns = S.Ns;
    for (int r = 0; r < 3; ++r) {
        S.u[r * Ns + s] = T(0);
        S.v[r * Ns + s] = T(0);
    }
    for (int q = 0; q < 9; ++q) {
        S.H[q * Ns + s] = T(0);
        S.A[q * Ns + s] = T(0);
    }
}

// After each substep of a force-terminated run (the terminal condition of
// Sec. III-C, on the contact force): flag[1] counts the substeps that ran,
// and flag[0] is raised once the z component of the contact force on the
// indenter reaches fz_limit, which makes the later substeps' kernels return
// at once. One thread.
__global__ void k_stop_check(int *flag, const double *force, double fz_limit)
{
    if (threadIdx.x == 0 && flag[0] == 0) {
        flag[1] += 1;
        if (force[2] >= fz_limit) flag[0] = 1;
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_fill(T *dst, int64_t n, T val)
{
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < n) dst[i] = val;
}

// Dense copy of the grid in node order (x fastest), momentum or velocity
// converted from grid units to SI by `scale` (= dx).
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_read_grid(SimDev<T> S, int which, T scale, T *M, T *vec)
{
    const int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int64_t n = (int64_t)S.g0 * S.g1 * S.g2;
    if (q >= n) return;
    const int gx = (int)(q % S.g0);
    const int64_t t = q / S.g0;
    const int gy = (int)(t % S.g1), gz = (int)(t / S.g1);
    const int64_t a = node_addr<B>(S.nb0, S.nb1, gx, gy, gz);
    T mp[4];
    constexpr int LB0 = Log2B<B>::v;
    const int bx = gx >> LB0, by = gy >> LB0, bz = gz >> LB0;
    gather_node<T, B>(S, bx, by, bz, gx & (B - 1), gy & (B - 1), gz & (B - 1), mp, live_mask(S, bx, by, bz));
    const T *src = which == 0 ? mp : S.V + 3 * a;
    if (M && which == 0) M[q] = src[0];
    // velocities exist only in blocks the last grid update visited (a block
    // or one of its seven lower neighbours holds particles); elsewhere V = 0
    constexpr int LB = Log2B<B>::v;
    const bool live = which == 0 || block_live(S, gx >> LB, gy >> LB, gz >> LB);
    for (int r = 0; r < 3; ++r) vec[r * n + q] = live ? scale * src[1 - which + r] : T(0);
}

}  // namespace tacchi
