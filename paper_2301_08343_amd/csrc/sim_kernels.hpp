// MLS-MPM substep kernels for one elastomer contact (gfx950, wave64).
//
// Per substep (Sec. III-A): block sort of the particles (histogram kept by
// the previous G2P -> scan -> scatter), P2G into an LDS tile per grid block
// flushed with one global atomic per tile node (Eqs. 2-5), the grid update
// fused with gravity, rigid-indenter contact, floor and walls (Eq. 6,
// Eq. 10), and G2P fused with the constitutive update and advection
// (Eqs. 7-11), which also bins each particle for the next substep.
#pragma once
#include "device_common.hpp"

namespace tacchi {

// ---------------------------------------------------------------- sort

// Exclusive scan of the per-block particle counts into offsets and scatter
// cursors; clears the counts for the next histogram and the force
// accumulator of the coming grid update. One workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan_bins(int *cnt, int *off, int *cursor, int nblk,
                                                    double *force)
{
    __shared__ int sh[1024];
    constexpr int IT = 8;
    const int tid = threadIdx.x;
    if (tid < 3 && force) force[tid] = 0.0;
    int carry = 0;
    for (int base = 0; base < nblk; base += 1024 * IT) {
        int vals[IT];
        int s = 0;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int idx = base + tid * IT + j;
            vals[j] = idx < nblk ? cnt[idx] : 0;
            s += vals[j];
        }
        sh[tid] = s;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int t = tid >= d ? sh[tid - d] : 0;
            __syncthreads();
            sh[tid] += t;
            __syncthreads();
        }
        int run = sh[tid] - s + carry;
#pragma unroll
        for (int j = 0; j < IT; ++j) {
            const int idx = base + tid * IT + j;
            if (idx < nblk) {
                off[idx] = run;
                cursor[idx] = run;
                cnt[idx] = 0;
            }
            run += vals[j];
        }
        carry += sh[1023];
        __syncthreads();
    }
    if (tid == 0) off[nblk] = carry;
}

// perm[cursor[key[p]]++] = p, one atomic per run of equal keys in a wave.
__global__ void __launch_bounds__(kWG) k_scatter(const int *key, int *cursor, int *perm, int64_t N)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    const int k = p < N ? key[p] : -1;
    const int slot = wave_run_slot(cursor, k);
    if (p < N) perm[slot] = (int)p;
}

// Block keys and histogram of the current positions (after init or a state
// write).
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_bin(SimDev<T> S)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    int k = -1;
    if (p < S.N) {
        T xr[3];
        rest_position(S, (uint32_t)p, xr);
        const T uu[3] = {S.u[p], S.u[S.N + p], S.u[2 * S.N + p]};
        k = block_key<T, B>(S, xr, uu);
        S.key[p] = k;
    }
    wave_run_slot(S.cnt, k);
}

// ---------------------------------------------------------------- P2G

// LDS accumulation slot of one tile channel. FP64 adds natively
// (ds_add_f64). FP32 accumulates 64-bit fixed point with ds_add_u64: the
// contributions are pre-scaled so that one particle mass is 2^40 units and one
// momentum unit m/dt (a particle crossing a cell per substep) is 2^40 units,
// converted to integers and summed exactly, so the sum does not depend on the
// order of the atomics; gfx950 also executes ds_add_u64 about 25x faster than
// ds_add_f32.
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
    __device__ static void add(Slot *s, float v) { atomicAdd(s, (unsigned long long)(long long)v); }
    __device__ static float value(Slot s) { return (float)(double)(long long)s; }
};

constexpr float kFixedOne = 1099511627776.0f;    // 2^40
constexpr float kFixedLimit = 3.6028797e16f;     // 2^55: largest accepted scaled contribution

// One workgroup per grid block: particles binned to the block scatter mass
// and momentum (Eqs. 2-5) into a (B+2)^3 LDS tile; the whole tile is then
// stored (plain stores, no global atomics) in the block's slot of the tile
// buffer, where the grid update gathers it. FIXDT rebuilds the stress part of
// A when the substep's dt differs from the dt A was formed with:
// A += (dt_A - dt) V0 (4/dx^2) tau. mscale/pscale scale mass and momentum
// into accumulator units (1 in FP64); munit/punit scale back.
template <typename T, int B, bool FIXDT, int MODEL>
__global__ void __launch_bounds__(kWG) k_p2g(SimDev<T> S, T fix_coef, T mscale, T pscale, T munit, T punit)
{
    using Acc = TileAcc<T>;
    using Slot = typename Acc::Slot;
    constexpr int TB = B + 2, TN = TB * TB * TB;
    __shared__ Slot tile[4 * TN];
    const int b = blockIdx.x;
    const int beg = S.off[b], end = S.off[b + 1];
    if (beg >= end) return;
    for (int i = threadIdx.x; i < 4 * TN; i += kWG) tile[i] = Slot(0);
    __syncthreads();
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    const int lo0 = bx * B, lo1 = by * B, lo2 = bz * B;
    const int64_t N = S.N;
    const T m = S.m * mscale;
    for (int i = beg + threadIdx.x; i < end; i += kWG) {
        const int p = S.perm[i];
        T xr[3];
        rest_position(S, (uint32_t)p, xr);
        const T uu[3] = {S.u[p], S.u[N + p], S.u[2 * N + p]};
        if (!finite3(uu[0], uu[1], uu[2])) {
            atomicOr(S.err, ERR_NONFINITE);
            continue;
        }
        int base[3];
        T f[3];
        stencil_base(xr, uu, base, f);
        const int l0 = base[0] - lo0, l1 = base[1] - lo1, l2 = base[2] - lo2;
        if ((unsigned)l0 >= (unsigned)B || (unsigned)l1 >= (unsigned)B || (unsigned)l2 >= (unsigned)B ||
            base[0] > S.g0 - 3 || base[1] > S.g1 - 3 || base[2] > S.g2 - 3) {
            atomicOr(S.err, ERR_OUT_OF_GRID);
            continue;
        }
        T wx[3], wy[3], wz[3];
        bspline3(f[0], wx);
        bspline3(f[1], wy);
        bspline3(f[2], wz);
        T Am[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Am[k] = S.A[k * N + p];
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
            q[r] = pscale * (S.m * S.v[r * N + p] - (Am[r * 3 + 0] * f[0] + Am[r * 3 + 1] * f[1] + Am[r * 3 + 2] * f[2]));
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
                    const int li = ((l2 + c) * TB + (l1 + bb)) * TB + (l0 + a);
                    Acc::add(&tile[li], wt * m);
                    Acc::add(&tile[TN + li], wt * (qa[0] + Am[2] * T(c)));
                    Acc::add(&tile[2 * TN + li], wt * (qa[1] + Am[5] * T(c)));
                    Acc::add(&tile[3 * TN + li], wt * (qa[2] + Am[8] * T(c)));
                }
            }
    }
    __syncthreads();
    T *dst = S.tiles + (int64_t)b * TN * 4;
    for (int li = threadIdx.x; li < TN; li += kWG) {
        T *d = dst + 4 * li;
        d[0] = Acc::value(tile[li]) * munit;
        d[1] = Acc::value(tile[TN + li]) * punit;
        d[2] = Acc::value(tile[2 * TN + li]) * punit;
        d[3] = Acc::value(tile[3 * TN + li]) * punit;
    }
}

// Mass and momentum of grid node (block (bx,by,bz), local (lx,ly,lz)): the sum,
// in a fixed order, of the tiles of the up-to-8 blocks whose (B+2)^3 tile
// covers it (the block itself and, where the node lies in the first two
// layers, its lower neighbours). Blocks without particles wrote no tile.
template <typename T, int B>
__device__ __forceinline__ void gather_node(const SimDev<T> &S, int bx, int by, int bz, int lx, int ly, int lz,
                                            T out[4])
{
    constexpr int TB = B + 2, TN = TB * TB * TB;
    out[0] = out[1] = out[2] = out[3] = T(0);
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
        if ((ox && lx > 1) || (oy && ly > 1) || (oz && lz > 1)) continue;
        const int cx = bx - ox, cy = by - oy, cz = bz - oz;
        if (cx < 0 || cy < 0 || cz < 0) continue;
        const int c = (cz * S.nb1 + cy) * S.nb0 + cx;
        if (S.off[c + 1] <= S.off[c]) continue;
        const int ti = ((lz + oz * B) * TB + (ly + oy * B)) * TB + (lx + ox * B);
        const T *src = S.tiles + ((int64_t)c * TN + ti) * 4;
        out[0] += src[0];
        out[1] += src[1];
        out[2] += src[2];
        out[3] += src[3];
    }
}

// ---------------------------------------------------------------- grid update

template <typename T>
__device__ __forceinline__ T wave_sum(T x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// One workgroup per grid block that can hold mass (the block or one of its
// seven lower neighbours has particles). Per node with mass above S.m_floor
// (0 in FP64; in FP32 2^-30 of a particle's mass, below which P/M is
// dominated by fixed-point quantisation and the node's weight in any particle
// is under FP32 resolution): V = P/M + dt g (Eq. 6);
// inside the indenter V takes the rigid indenter velocity (sticky contact;
// the reaction M (V_before - V_indenter)/dt is summed into the force);
// floor nodes are held; wall nodes drop their outward component. The inside test and the
// rigid velocity are evaluated in FP64 in both precisions, so the discrete
// contact decision does not depend on the simulation precision.
template <typename T, int B>
__global__ void __launch_bounds__(kWG) k_grid(SimDev<T> S, IndenterDev<double> I, T dt)
{
    constexpr int B3 = B * B * B;
    const int b = blockIdx.x;
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    bool live = false;
    for (int o = 0; o < 8; ++o) {
        const int cx = bx - (o & 1), cy = by - ((o >> 1) & 1), cz = bz - (o >> 2);
        if (cx < 0 || cy < 0 || cz < 0) continue;
        const int c = (cz * S.nb1 + cy) * S.nb0 + cx;
        if (S.off[c + 1] > S.off[c]) live = true;
    }
    if (!live) return;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    const T inv_dt = T(1) / dt;
    for (int l = threadIdx.x; l < B3; l += kWG) {
        const int lx = l % B, ly = (l / B) % B, lz = l / (B * B);
        const int gx = bx * B + lx, gy = by * B + ly, gz = bz * B + lz;
        const int64_t addr = (int64_t)b * B3 + l;
        T mp[4];
        gather_node<T, B>(S, bx, by, bz, lx, ly, lz, mp);
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
                if (indenter_phi<double>(I, px, py, pz) <= 0.0) {
                    // rigid velocity v_c + omega x r, converted to cells/s
                    const double ir = 1.0 / I.dx;
                    const T w0 = T(I.vc[0] + (I.om[1] * r2 - I.om[2] * r1) * ir);
                    const T w1 = T(I.vc[1] + (I.om[2] * r0 - I.om[0] * r2) * ir);
                    const T w2 = T(I.vc[2] + (I.om[0] * r1 - I.om[1] * r0) * ir);
                    const T s = m * T(I.dx) * inv_dt;
                    fx += (double)(s * (V0 - w0));
                    fy += (double)(s * (V1 - w1));
                    fz += (double)(s * (V2 - w2));
                    V0 = w0; V1 = w1; V2 = w2;
                }
            }
            if (gz <= S.floor_node) V0 = V1 = V2 = T(0);
            if ((gx < S.wall && V0 < T(0)) || (gx > S.g0 - 1 - S.wall && V0 > T(0))) V0 = T(0);
            if ((gy < S.wall && V1 < T(0)) || (gy > S.g1 - 1 - S.wall && V1 > T(0))) V1 = T(0);
            if ((gz < S.wall && V2 < T(0)) || (gz > S.g2 - 1 - S.wall && V2 > T(0))) V2 = T(0);
        }
        T *vv = S.V + 4 * addr;
        vv[0] = V0; vv[1] = V1; vv[2] = V2; vv[3] = T(0);
    }
    if (I.shape >= 0) {
        __shared__ double red[3][kWG / 64];
        fx = wave_sum(fx); fy = wave_sum(fy); fz = wave_sum(fz);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { red[0][w] = fx; red[1][w] = fy; red[2][w] = fz; }
        __syncthreads();
        if (threadIdx.x < 3) {
            double s = 0.0;
            for (int k = 0; k < kWG / 64; ++k) s += red[threadIdx.x][k];
            if (s != 0.0) atomicAdd(&S.force[threadIdx.x], s);
        }
    }
}

// ---------------------------------------------------------------- G2P

// One workgroup per grid block: the block's (B+2)^3 velocity tile is staged
// in LDS; each particle gathers v and C (Eqs. 7-8, with the grid velocities
// in Eq. 8), updates F (Eq. 9), forms the stress and the affine momentum
// A = m C - dt V0 (4/dx^2) tau for the next P2G, applies the bonded bottom
// layers (Eq. 10), advects (Eq. 11) and bins itself for the next substep.
template <typename T, int B, int MODEL>
__global__ void __launch_bounds__(kWG) k_g2p(SimDev<T> S, T dt, T stress_coef)
{
    constexpr int TB = B + 2, TN = TB * TB * TB;
    __shared__ T tile[3 * TN];
    const int b = blockIdx.x;
    const int beg = S.off[b], end = S.off[b + 1];
    if (beg >= end) return;
    const int bx = b % S.nb0, byz = b / S.nb0, by = byz % S.nb1, bz = byz / S.nb1;
    const int lo0 = bx * B, lo1 = by * B, lo2 = bz * B;
    for (int li = threadIdx.x; li < TN; li += kWG) {
        const int x = li % TB, yz = li / TB, y = yz % TB, z = yz / TB;
        const int gx = lo0 + x, gy = lo1 + y, gz = lo2 + z;
        T a0 = T(0), a1 = T(0), a2 = T(0);
        if (gx < S.g0 && gy < S.g1 && gz < S.g2) {
            const T *src = S.V + 4 * node_addr<B>(S.nb0, S.nb1, gx, gy, gz);
            a0 = src[0]; a1 = src[1]; a2 = src[2];
        }
        tile[li] = a0;
        tile[TN + li] = a1;
        tile[2 * TN + li] = a2;
    }
    __syncthreads();
    const int64_t N = S.N;
    for (int i0 = beg; i0 < end; i0 += kWG) {
        const int i = i0 + threadIdx.x;
        int newkey = -1;
        if (i < end) {
            const int p = S.perm[i];
            T xr[3];
            rest_position(S, (uint32_t)p, xr);
            T uu[3] = {S.u[p], S.u[N + p], S.u[2 * N + p]};
            int base[3] = {0, 0, 0};
            T f[3];
            const bool fin = finite3(uu[0], uu[1], uu[2]);
            if (fin) stencil_base(xr, uu, base, f);
            const int l0 = base[0] - lo0, l1 = base[1] - lo1, l2 = base[2] - lo2;
            if (!fin) {
                atomicOr(S.err, ERR_NONFINITE);
                newkey = S.key[p];
            } else if ((unsigned)l0 >= (unsigned)B || (unsigned)l1 >= (unsigned)B || (unsigned)l2 >= (unsigned)B ||
                base[0] > S.g0 - 3 || base[1] > S.g1 - 3 || base[2] > S.g2 - 3) {
                atomicOr(S.err, ERR_OUT_OF_GRID);
                newkey = S.key[p];
            } else {
                T wx[3], wy[3], wz[3];
                bspline3(f[0], wx);
                bspline3(f[1], wy);
                bspline3(f[2], wz);
                // velocities relative to the stencil centre keep the affine
                // sums well conditioned in FP32
                const int lc = ((l2 + 1) * TB + (l1 + 1)) * TB + (l0 + 1);
                const T vr[3] = {tile[lc], tile[TN + lc], tile[2 * TN + lc]};
                T s0[3] = {T(0), T(0), T(0)};       // sum w V
                T sx[3] = {T(0), T(0), T(0)};       // sum w (V - vr) a
                T sy[3] = {T(0), T(0), T(0)};
                T sz[3] = {T(0), T(0), T(0)};
                T sr[3] = {T(0), T(0), T(0)};       // sum w (V - vr)
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const T wt = wx[a] * wy[bb] * wz[c];
                            const int li = ((l2 + c) * TB + (l1 + bb)) * TB + (l0 + a);
                            const T Vn[3] = {tile[li], tile[TN + li], tile[2 * TN + li]};
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                const T wv = wt * Vn[r];
                                const T wd = wt * (Vn[r] - vr[r]);
                                s0[r] += wv;
                                sr[r] += wd;
                                sx[r] += wd * T(a);
                                sy[r] += wd * T(bb);
                                sz[r] += wd * T(c);
                            }
                        }
                // C = (4/dx^2) sum w V (X_i - x_p)^T, in 1/s with grid-unit offsets
                T Cm[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Cm[r * 3 + 0] = T(4) * (sx[r] - sr[r] * f[0]);
                    Cm[r * 3 + 1] = T(4) * (sy[r] - sr[r] * f[1]);
                    Cm[r * 3 + 2] = T(4) * (sz[r] - sr[r] * f[2]);
                }
                // F <- (I + dt C) F, i.e. H <- H + dt (C + C H)
                T Hm[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) Hm[k] = S.H[k * N + p];
                T Hn[9];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        Hn[r * 3 + c] = Hm[r * 3 + c] +
                                        dt * (Cm[r * 3 + c] + Cm[r * 3 + 0] * Hm[0 * 3 + c] +
                                              Cm[r * 3 + 1] * Hm[1 * 3 + c] + Cm[r * 3 + 2] * Hm[2 * 3 + c]);
                T tau[9];
                if (!kirchhoff<T, MODEL>(S, Hn, tau)) {
                    atomicOr(S.err, MODEL == 0 ? ERR_INVERTED : ERR_NONFINITE);
#pragma unroll
                    for (int k = 0; k < 9; ++k) tau[k] = T(0);
                }
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    S.H[k * N + p] = Hn[k];
                    S.A[k * N + p] = S.m * Cm[k] - stress_coef * tau[k];
                }
                T vn[3] = {s0[0], s0[1], s0[2]};
                if (p < S.fixed_count) vn[0] = vn[1] = vn[2] = T(0);
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    S.v[r * N + p] = vn[r];
                    uu[r] += dt * vn[r];
                    S.u[r * N + p] = uu[r];
                }
                newkey = block_key<T, B>(S, xr, uu);
                S.key[p] = newkey;
            }
        }
        wave_run_slot(S.cnt, newkey);
    }
}

// ---------------------------------------------------------------- outputs

// out[j][i] = world z of top-layer particle (i, j).
template <typename T>
__global__ void __launch_bounds__(kWG) k_heightmap(SimDev<T> S, T origin_z, T dx, T *out)
{
    const int idx = blockIdx.x * kWG + threadIdx.x;
    const int nxy = S.n0 * S.n1;
    if (idx >= nxy) return;
    const int64_t p = (int64_t)(S.n2 - 1) * nxy + idx;
    const T zr = S.xr[2] + T(S.n2 - 1) * S.hr[2];
    out[idx] = origin_z + dx * (zr + S.u[2 * S.N + p]);
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

template <typename T, int MODEL>
__global__ void __launch_bounds__(kWG) k_read_particles(SimDev<T> S, T ox, T oy, T oz, T dx, T dtA_coef,
                                                        T *x, T *v, T *C, T *F)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= S.N) return;
    const int64_t N = S.N;
    T xr[3];
    rest_position(S, (uint32_t)p, xr);
    if (x) {
        x[p] = ox + dx * (xr[0] + S.u[p]);
        x[N + p] = oy + dx * (xr[1] + S.u[N + p]);
        x[2 * N + p] = oz + dx * (xr[2] + S.u[2 * N + p]);
    }
    if (v)
        for (int r = 0; r < 3; ++r) v[r * N + p] = dx * S.v[r * N + p];
    T Hm[9];
    for (int k = 0; k < 9; ++k) Hm[k] = S.H[k * N + p];
    if (F)
        for (int k = 0; k < 9; ++k) F[k * N + p] = Hm[k] + ((k % 4 == 0) ? T(1) : T(0));
    if (C) {
        T tau[9];
        if (dtA_coef == T(0) || !kirchhoff<T, MODEL>(S, Hm, tau))
            for (int k = 0; k < 9; ++k) tau[k] = T(0);
        for (int k = 0; k < 9; ++k) C[k * N + p] = (S.A[k * N + p] + dtA_coef * tau[k]) / S.m;
    }
}

// Writes a state given in SI/world terms; A is stored as m C (the stress part
// is added by the next P2G, which sees dt_A = 0).
template <typename T>
__global__ void __launch_bounds__(kWG) k_write_particles(SimDev<T> S, T ox, T oy, T oz, T inv_dx,
                                                         const T *x, const T *v, const T *C, const T *F)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= S.N) return;
    const int64_t N = S.N;
    T xr[3];
    rest_position(S, (uint32_t)p, xr);
    const T o[3] = {ox, oy, oz};
    for (int r = 0; r < 3; ++r) {
        S.u[r * N + p] = (x[r * N + p] - o[r]) * inv_dx - xr[r];
        S.v[r * N + p] = v[r * N + p] * inv_dx;
    }
    for (int k = 0; k < 9; ++k) {
        S.H[k * N + p] = F[k * N + p] - ((k % 4 == 0) ? T(1) : T(0));
        S.A[k * N + p] = S.m * C[k * N + p];
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_init_particles(SimDev<T> S)
{
    const int64_t p = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= S.N) return;
    const int64_t N = S.N;
    for (int r = 0; r < 3; ++r) {
        S.u[r * N + p] = T(0);
        S.v[r * N + p] = T(0);
    }
    for (int k = 0; k < 9; ++k) {
        S.H[k * N + p] = T(0);
        S.A[k * N + p] = T(0);
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
    constexpr int LB0 = (B == 4) ? 2 : 3;
    gather_node<T, B>(S, gx >> LB0, gy >> LB0, gz >> LB0, gx & (B - 1), gy & (B - 1), gz & (B - 1), mp);
    const T *src = which == 0 ? mp : S.V + 4 * a;
    if (M && which == 0) M[q] = src[0];
    // velocities exist only in blocks the last grid update visited (a block
    // or one of its seven lower neighbours holds particles); elsewhere V = 0
    bool live = which == 0;
    constexpr int LB = (B == 4) ? 2 : 3;
    const int bx = gx >> LB, by = gy >> LB, bz = gz >> LB;
    for (int o = 0; o < 8 && !live; ++o) {
        const int cx = bx - (o & 1), cy = by - ((o >> 1) & 1), cz = bz - (o >> 2);
        if (cx < 0 || cy < 0 || cz < 0) continue;
        const int c = (cz * S.nb1 + cy) * S.nb0 + cx;
        if (S.off[c + 1] > S.off[c]) live = true;
    }
    for (int r = 0; r < 3; ++r) vec[r * n + q] = live ? scale * src[1 - which + r] : T(0);
}

}  // namespace tacchi
