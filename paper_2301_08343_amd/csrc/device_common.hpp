// Device-side building blocks shared by the tactile MPM kernels (gfx950).
//
// Internal representation (chosen for FP32 accuracy):
//  - lengths in grid units (cells of size dx); a particle stores its
//    displacement u from its rest lattice position, so the rest position is
//    recomputed exactly from the particle index and only the small u carries
//    rounding;
//  - velocities in cells/s;
//  - the deformation gradient as H = F - I, so F F^T - I = H + H^T + H H^T
//    and J - 1 = det(I + H) - 1 avoid cancellation near the rest state;
//  - the MLS-MPM affine momentum matrix A = m C - dt V0 (4/dx^2) tau instead
//    of C (Eqs. 4-5 fused), which P2G needs as is. C is recovered on read-out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tacchi {

constexpr int kWG = 256;

enum : int { ERR_NONFINITE = 1, ERR_INVERTED = 2, ERR_OUT_OF_GRID = 4, ERR_CAPACITY = 8 };

// Division by a runtime constant via a precomputed multiplier (round-up
// method of Granlund and Montgomery, 1994): valid for n < 2^31.
struct FastDiv {
    uint32_t d, mul, shift;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.shift = s;
    f.mul = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << s) - d)) / d + 1);
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    uint32_t t = __umulhi(n, f.mul);
    return (t + n) >> f.shift;
}

// Everything a kernel needs to know about one elastomer contact.
//
// Particle storage: the lattice is cut into tiles of B x B x B particles,
// shifted so that at rest each tile holds exactly the particles whose grid
// cell lies in one grid block; tiles are stored contiguously (B^3 slots each,
// slots outside the lattice stay unused). A grid block's particles are then
// one contiguous run of slots, which keeps the transfers' loads and stores
// coalesced.
//
// Binning: each grid block owns `cap` entries of a bin list; G2P appends each
// updated particle to the list of the block holding its new stencil base
// (a counting sort whose offsets are fixed), so the next substep's P2G and
// G2P find a block's particles without a global scan.
template <typename T>
struct SimDev {
    int64_t N;             // particles
    int64_t Ns;            // particle slots
    int n0, n1, n2;        // particle lattice
    int g0, g1, g2;        // grid nodes per axis
    int nb0, nb1, nb2;     // grid blocks per axis
    int nblk;
    int bx0, by0, bz0;     // first block of the box that holds the particles at rest
    int bxn, byn, bzn;     // its extent in blocks (dispatched first, box_first_block)
    int box_chunk;         // XCD chunk within that box
    int hx0, hy0, hz0;     // that box grown by one block (clamped to the grid): the grid
    int hxn, hyn, hzn;     // update's nodes there take the particles' halo, so it goes first
    int halo_chunk;
    int ts0, ts1, ts2;     // lattice index i lies in tile (i + ts) / B
    int nt0, nt1, nt2;     // tiles per axis
    FastDiv div_nt0, div_nt1, div_n0, div_n1;
    int cap;               // bin-list entries per grid block
    T xr[3];               // rest position of lattice particle (0,0,0), grid units
    T hr[3];               // lattice spacing / dx
    T m;                   // particle mass [kg]
    T m_floor;             // grid nodes lighter than this get V = 0 (see k_grid)
    T vcoef;               // V0 * 4 / dx^2 [m]
    T mu, lambda;          // Lame parameters [Pa]
    int floor_node, wall;
    int n_fixed;           // lattice layers k < n_fixed are bonded to the sensor
    T grav[3];             // gravity [cells/s^2]
    T *u, *v, *H, *A;      // SoA over slots: u[3][Ns], v[3][Ns], H[9][Ns], A[9][Ns]
    int *cnt_cur, *cnt_next;    // [nblk] particles per block (this / next substep)
    int *perm_cur, *perm_next;  // [nblk][cap] particle slots per block
    T *tiles;              // [blocks][(B+3)^3][4]: per-block P2G tiles of mass, momentum (kg, kg cells/s)
    T *V;                  // [nodes][4]: velocity (cells/s), 4th lane unused
    int *err;
    double *force;         // [3] contact reaction on the indenter [N]
    unsigned int *fallback;// count of FP64 polar recomputations
    const int *stop;       // force-terminated runs: while *stop != 0 the substep kernels do nothing (else null)
};

// Rigid indenter for one substep: shape, its pose at the start of the
// substep and its rigid velocity over the substep.
template <typename T>
struct IndenterDev {
    int shape;
    T p[4];
    uint64_t seed;
    T tip[3];              // indenter origin, grid units
    T R[9];                // indenter frame -> world (row-major)
    T vc[3];               // translation velocity [cells/s]
    T om[3];               // angular velocity [rad/s]
    T dx;                  // [m] converts grid units to metres for the shape
    T mu;                  // Coulomb friction coefficient (grid kernels instantiated with friction)
    T eps;                 // [m] step of the central differences giving the contact normal
    T zmin;                // [m] below this indenter-frame height a point is outside the solid
    const double *MI;      // particle indenter: its mass per grid node (x fastest), else null
    int blo[3], bhi[3];    // node box (inclusive) outside which MI is zero this substep
};

template <typename T> __device__ __forceinline__ T tfloor(T x);
template <> __device__ __forceinline__ float tfloor<float>(float x) { return floorf(x); }
template <> __device__ __forceinline__ double tfloor<double>(double x) { return floor(x); }

template <typename T>
__device__ __forceinline__ bool finite3(T a, T b, T c)
{
    return isfinite(a) && isfinite(b) && isfinite(c);
}

// Grid block of workgroup i in the per-block kernels. Workgroups are handed to
// the eight XCDs round robin (workgroup i to XCD i mod 8), and each XCD has its
// own L2. Here XCD x takes whole chunks of C consecutive blocks (chunks x,
// x + 8, x + 16, ...): three rows of blocks, so the tile and velocity halos
// that neighbouring blocks share along x and y are fetched into one L2. With
// three rows a round of 8 chunks (24 rows) does not tile a z layer of the
// GelSight grid (32 rows), so the XCDs rotate over the rows from layer to
// layer and none is left with the empty border rows only (chunks that tile
// the layer were measured 10-15 % slower than this). Blocks past the last
// whole round of 8 chunks keep their index. A bijection of [0, n).
__host__ __device__ __forceinline__ int xcd_block(int i, int n, int C)
{
    const int R = 8 * C;
    if (C <= 1 || i >= (n / R) * R) return i;
    const int x = i & 7, j = i >> 3;
    return ((j / C) * 8 + x) * C + (j % C);
}

// Block of dispatch index i for the per-block kernels: first the blocks of
// a box (x0..x0+xn-1, y0.., z0..; the blocks that hold the particles at
// rest) in the XCD-aware order of xcd_block, then every other block of the
// nb0 x nb1 x nb2 grid (the layers below and above the box, then per layer
// of the box the rows in front of and behind it, then the rest of its rows
// left and right of it). Workgroups of blocks that hold no particles exit at
// once, but each holds a slot for the round trip of its count; dispatched
// after the live ones they wait in the launch's tail instead of between
// them. A permutation of 0 .. nb0 nb1 nb2 - 1 for any box inside the grid
// (an empty box included); which workgroup takes a block changes no result.
__host__ __device__ __forceinline__ int box_first_block(int i, int nb0, int nb1, int nb2, int x0, int y0, int z0, int xn,
                                                        int yn, int zn, int C)
{
    const int nbox = xn * yn * zn;
    if (i < nbox) {
        const int k = xcd_block(i, nbox, C), t = k / xn;
        return (x0 + k % xn) + nb0 * ((y0 + t % yn) + nb1 * (z0 + t / yn));
    }
    int j = i - nbox;
    const int layer = nb0 * nb1;
    if (j < layer * z0) return j;
    j -= layer * z0;
    const int above = layer * (nb2 - z0 - zn);
    if (j < above) return layer * (z0 + zn) + j;
    j -= above;
    const int front = nb0 * y0, back = nb0 * (nb1 - y0 - yn), side = nb0 - xn;
    const int per_layer = front + back + yn * side;
    if (per_layer <= 0) return i;  // unreachable: the box layers then hold no other block
    const int z = z0 + j / per_layer;
    j %= per_layer;
    int x, y;
    if (j < front) {
        y = j / nb0;
        x = j % nb0;
    } else if (j < front + back) {
        j -= front;
        y = y0 + yn + j / nb0;
        x = j % nb0;
    } else {
        j -= front + back;
        y = y0 + j / side;
        x = j % side;
        if (x >= x0) x += xn;
    }
    return x + nb0 * (y + nb1 * z);
}

template <typename T>
__device__ __forceinline__ int dispatch_block(const SimDev<T> &S, int i)
{
    return box_first_block(i, S.nb0, S.nb1, S.nb2, S.bx0, S.by0, S.bz0, S.bxn, S.byn, S.bzn, S.box_chunk);
}

// The grid update's order: the particle box grown by one block first.
template <typename T>
__device__ __forceinline__ int dispatch_halo_block(const SimDev<T> &S, int i)
{
    return box_first_block(i, S.nb0, S.nb1, S.nb2, S.hx0, S.hy0, S.hz0, S.hxn, S.hyn, S.hzn, S.halo_chunk);
}

template <int B>
struct Log2B {
    static constexpr int v = (B == 4) ? 2 : 3;
};

// Lattice index (i, j, k) of a particle slot; false for unused slots.
template <typename T, int B>
__device__ __forceinline__ bool slot_lattice(const SimDev<T> &S, uint32_t slot, int &i, int &j, int &k)
{
    constexpr int LB = Log2B<B>::v;
    const uint32_t blk = slot >> (3 * LB), loc = slot & (B * B * B - 1);
    const uint32_t t1 = fdiv(blk, S.div_nt0);
    const int tx = (int)(blk - t1 * (uint32_t)S.nt0);
    const uint32_t tz = fdiv(t1, S.div_nt1);
    const int ty = (int)(t1 - tz * (uint32_t)S.nt1);
    i = tx * B + (int)(loc & (B - 1)) - S.ts0;
    j = ty * B + (int)((loc >> LB) & (B - 1)) - S.ts1;
    k = (int)tz * B + (int)(loc >> (2 * LB)) - S.ts2;
    return (unsigned)i < (unsigned)S.n0 && (unsigned)j < (unsigned)S.n1 && (unsigned)k < (unsigned)S.n2;
}

// Slot of lattice particle (i, j, k).
template <typename T, int B>
__device__ __forceinline__ uint32_t lattice_slot(const SimDev<T> &S, int i, int j, int k)
{
    constexpr int LB = Log2B<B>::v;
    const int a = i + S.ts0, b = j + S.ts1, c = k + S.ts2;
    const uint32_t tile = ((uint32_t)(c >> LB) * S.nt1 + (uint32_t)(b >> LB)) * S.nt0 + (uint32_t)(a >> LB);
    return (tile << (3 * LB)) + (uint32_t)((((c & (B - 1)) << LB) + (b & (B - 1))) << LB) + (uint32_t)(a & (B - 1));
}

// Lattice index of the API's particle order p = i + n0 (j + n1 k).
template <typename T>
__device__ __forceinline__ void api_lattice(const SimDev<T> &S, uint32_t p, int &i, int &j, int &k)
{
    const uint32_t q = fdiv(p, S.div_n0);
    i = (int)(p - q * (uint32_t)S.n0);
    const uint32_t kk = fdiv(q, S.div_n1);
    j = (int)(q - kk * (uint32_t)S.n1);
    k = (int)kk;
}

// Rest position (grid units) of lattice particle (i, j, k).
template <typename T>
__device__ __forceinline__ void rest_position(const SimDev<T> &S, int i, int j, int k, T xr[3])
{
    xr[0] = S.xr[0] + T(i) * S.hr[0];
    xr[1] = S.xr[1] + T(j) * S.hr[1];
    xr[2] = S.xr[2] + T(k) * S.hr[2];
}

// Quadratic B-spline weights of the three nodes base, base+1, base+2 of a
// particle at fractional offset f = x/dx - base in [0.5, 1.5).
template <typename T>
__device__ __forceinline__ void bspline3(T f, T w[3])
{
    T a = T(1.5) - f;
    T b = f - T(1);
    T c = f - T(0.5);
    w[0] = T(0.5) * a * a;
    w[1] = T(0.75) - b * b;
    w[2] = T(0.5) * c * c;
}

// Stencil base node and fractional offset of a particle with rest position
// xr and displacement uu (grid units). The offset is formed as
// (xr - base) + u, which is exact up to one rounding of the small result.
template <typename T>
__device__ __forceinline__ void stencil_base(const T xr[3], const T uu[3], int base[3], T f[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T s = xr[a] + uu[a];
        base[a] = (int)tfloor<T>(s - T(0.5));
        f[a] = (xr[a] - T(base[a])) + uu[a];
    }
}

// Position of node (lx, ly, lz) inside its block's B^3 run of the velocity
// grid. The G2P tile of a block reads the last layer of its lower neighbour
// and the first two layers of its upper neighbour along each axis, so each
// axis splits into the segments {0, 1}, {2 .. B-2}, {B-1}; the block's nodes
// are stored segment region by segment region (z, then y, then x), each
// region x-fastest, and a neighbour's share is a few contiguous runs.
template <int B>
__host__ __device__ __forceinline__ int node_local(int lx, int ly, int lz)
{
    auto seg = [](int l) { return l <= 1 ? 0 : (l <= B - 2 ? 1 : 2); };
    auto start = [](int r) { return r == 0 ? 0 : (r == 1 ? 2 : B - 1); };
    auto size = [](int r) { return r == 0 ? 2 : (r == 1 ? B - 3 : 1); };
    const int rx = seg(lx), ry = seg(ly), rz = seg(lz);
    const int sx = size(rx), sy = size(ry), sz = size(rz);
    return start(rz) * B * B + sz * start(ry) * B + sz * sy * start(rx) +
           ((lz - start(rz)) * sy + (ly - start(ry))) * sx + (lx - start(rx));
}

template <int B>
__host__ __device__ __forceinline__ int64_t node_addr(int nb0, int nb1, int x, int y, int z)
{
    constexpr int LB = Log2B<B>::v;
    int bx = x >> LB, by = y >> LB, bz = z >> LB;
    int lx = x & (B - 1), ly = y & (B - 1), lz = z & (B - 1);
    int64_t blk = ((int64_t)bz * nb1 + by) * nb0 + bx;
    return blk * (B * B * B) + node_local<B>(lx, ly, lz);
}

// Block key of a particle: the grid block holding the grid cell the particle
// lies in (floor(x/dx)). Binning by cell rather than by stencil base keeps
// particles that sit exactly at a cell centre -- every particle of a rest
// lattice with one particle per cell -- from flipping between blocks under
// rounding-level motion; the transfer tiles carry one extra lower layer for
// the stencil base (floor(x/dx - 1/2)) one below the cell. Out-of-grid or
// non-finite particles are flagged and clamped to a valid block (the
// transfer kernels then skip them).
template <typename T, int B>
__device__ __forceinline__ int block_key(const SimDev<T> &S, const T xr[3], const T uu[3])
{
    constexpr int LB = Log2B<B>::v;
    if (!finite3(uu[0], uu[1], uu[2])) {
        atomicOr(S.err, ERR_NONFINITE);
        return 0;
    }
    const int gn[3] = {S.g0, S.g1, S.g2};
    const int nb[3] = {S.nb0, S.nb1, S.nb2};
    int blk[3];
    bool oog = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T s = xr[a] + uu[a];
        const int base = (int)tfloor<T>(s - T(0.5));
        if (base < 0 || base > gn[a] - 3) oog = true;
        int cell = (int)tfloor<T>(s);
        cell = cell < 0 ? 0 : (cell > gn[a] - 1 ? gn[a] - 1 : cell);
        blk[a] = min(cell >> LB, nb[a] - 1);
    }
    if (oog) atomicOr(S.err, ERR_OUT_OF_GRID);
    return (blk[2] * S.nb1 + blk[1]) * S.nb0 + blk[0];
}

// Wave-level aggregation of counter increments: the lanes of one wave64 that
// carry the same key take one atomicAdd per distinct key (issued by the
// lowest such lane) and consecutive slots in lane order. Keys are handled one
// distinct value per iteration, so a wave whose particles straddle a block
// boundary costs a couple of atomics instead of one per lane. Lanes with
// key < 0 take no slot. All 64 lanes must execute this together.
__device__ __forceinline__ int wave_run_slot(int *counter, int key)
{
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long remaining = __ballot(key >= 0);
    int slot = 0;
    while (remaining) {
        const int leader = __ffsll((long long)remaining) - 1;
        const int k = __shfl(key, leader);
        const unsigned long long same = __ballot(key == k) & remaining;
        int base = 0;
        if (lane == leader) base = atomicAdd(&counter[k], __popcll(same));
        base = __shfl(base, leader);
        if ((same >> lane) & 1ull) slot = base + __popcll(same & below);
        remaining &= ~same;
    }
    return slot;
}

// ---------------------------------------------------------------- constitutive models

// Kirchhoff stress of the compressible neo-Hookean model,
// tau = mu (F F^T - I) + lambda ln(J) I, from H = F - I. Returns false when
// J <= 0 or the state is not finite.
template <typename T>
__device__ __forceinline__ bool tau_neohookean(const T H[9], T mu, T lambda, T tau[9])
{
    const T tr = H[0] + H[4] + H[8];
    const T m2 = (H[0] * H[4] - H[1] * H[3]) + (H[0] * H[8] - H[2] * H[6]) + (H[4] * H[8] - H[5] * H[7]);
    const T d3 = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                 H[2] * (H[3] * H[7] - H[4] * H[6]);
    const T Jm1 = tr + m2 + d3;
    if (!(Jm1 > T(-1))) return false;
    const T lnJ = log1p(Jm1);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T hh = H[r * 3 + 0] * H[c * 3 + 0] + H[r * 3 + 1] * H[c * 3 + 1] + H[r * 3 + 2] * H[c * 3 + 2];
            tau[r * 3 + c] = mu * (H[r * 3 + c] + H[c * 3 + r] + hh) + (r == c ? lambda * lnJ : T(0));
        }
    return true;
}

template <typename T>
__device__ __forceinline__ T det3(const T M[9])
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

template <typename T>
__device__ __forceinline__ void cofactor3(const T M[9], T C[9])
{
    C[0] = M[4] * M[8] - M[5] * M[7];
    C[1] = M[5] * M[6] - M[3] * M[8];
    C[2] = M[3] * M[7] - M[4] * M[6];
    C[3] = M[2] * M[7] - M[1] * M[8];
    C[4] = M[0] * M[8] - M[2] * M[6];
    C[5] = M[1] * M[6] - M[0] * M[7];
    C[6] = M[1] * M[5] - M[2] * M[4];
    C[7] = M[2] * M[3] - M[0] * M[5];
    C[8] = M[0] * M[4] - M[1] * M[3];
}

template <typename T>
__device__ __forceinline__ T frob2(const T M[9])
{
    T s = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) s += M[k] * M[k];
    return s;
}

// Orthogonal polar factor by Higham's scaled Newton iteration
// X <- (g X + X^{-T}/g)/2 with g = sqrt(|X^{-1}|_F / |X|_F)
// (N. J. Higham, "Computing the polar decomposition -- with applications",
// SIAM J. Sci. Stat. Comput. 7, 1986). Returns false if it did not converge.
template <typename T>
__device__ __forceinline__ bool polar_newton(const T F[9], T R[9], T tol, int maxit)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = F[k];
    for (int it = 0; it < maxit; ++it) {
        T C[9];
        cofactor3(R, C);
        const T d = R[0] * C[0] + R[1] * C[1] + R[2] * C[2];
        if (!(fabs(d) > T(0))) return false;
        const T nx = frob2(R), ni = frob2(C) / (d * d);
        const T g = sqrt(sqrt(ni / nx));
        const T a = T(0.5) * g, b = T(0.5) / (g * d);
        T diff = T(0);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            T nk = a * R[k] + b * C[k];
            diff += (nk - R[k]) * (nk - R[k]);
            R[k] = nk;
        }
        if (diff <= tol * tol) return true;
    }
    return false;
}

// FP64 polar decomposition that also handles det F <= 0: the orthogonal
// factor U of F is made a proper rotation by reflecting it across the
// direction e of the smallest eigenvalue of S = U^T F (found by power
// iteration on adj(S), whose dominant eigenvector is e):
// R = U (I - 2 e e^T), so that F = R S' with S' = (I - 2 e e^T) S.
__device__ inline bool polar_f64_proper(const double F[9], double R[9])
{
    double U[9];
    if (!polar_newton<double>(F, U, 1e-13, 60)) return false;
    if (det3(U) > 0.0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = U[k];
        return true;
    }
    double S[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            S[r * 3 + c] = U[0 * 3 + r] * F[0 * 3 + c] + U[1 * 3 + r] * F[1 * 3 + c] + U[2 * 3 + r] * F[2 * 3 + c];
    double Cs[9];
    cofactor3(S, Cs);  // adj(S) = cof(S)^T; S symmetric so cof(S) is too
    int best = 0;
    double bn = -1.0;
    for (int c = 0; c < 3; ++c) {
        double n = Cs[c] * Cs[c] + Cs[3 + c] * Cs[3 + c] + Cs[6 + c] * Cs[6 + c];
        if (n > bn) { bn = n; best = c; }
    }
    double e[3] = {Cs[best], Cs[3 + best], Cs[6 + best]};
    for (int it = 0; it < 50; ++it) {
        double n = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (!(n > 0.0)) return false;
        double y[3];
        for (int r = 0; r < 3; ++r) y[r] = (Cs[r * 3 + 0] * e[0] + Cs[r * 3 + 1] * e[1] + Cs[r * 3 + 2] * e[2]) / n;
        e[0] = y[0]; e[1] = y[1]; e[2] = y[2];
    }
    double n = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int r = 0; r < 3; ++r) e[r] /= n;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double Ue = U[r * 3 + 0] * e[0] + U[r * 3 + 1] * e[1] + U[r * 3 + 2] * e[2];
            R[r * 3 + c] = U[r * 3 + c] - 2.0 * Ue * e[c];
        }
    return true;
}

// Kirchhoff stress of the fixed-corotated model,
// tau = 2 mu (F - R) F^T + lambda (J - 1) J I. The polar factor is computed
// in T; when the Frobenius condition number |F| |adj F| / |det F| exceeds 1e6,
// det F <= 0, or the iteration fails, it is recomputed in FP64 (counted in
// *fallback).
template <typename T>
__device__ __forceinline__ bool tau_corotated(const T H[9], T mu, T lambda, T tau[9],
                                              unsigned int *fallback)
{
    T F[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) F[k] = H[k] + ((k % 4 == 0) ? T(1) : T(0));
    T C[9];
    cofactor3(F, C);
    const T J = F[0] * C[0] + F[1] * C[1] + F[2] * C[2];
    if (!isfinite(J)) return false;
    T R[9];
    bool ok = false;
    if (sizeof(T) == 4 && J > T(0)) {
        const T kappa2 = frob2(F) * frob2(C) / (J * J);
        if (kappa2 <= T(1e12)) ok = polar_newton<T>(F, R, T(2e-6), 30);
    }
    if (!ok) {
        double Fd[9], Rd[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Fd[k] = (double)F[k];
        if (!polar_f64_proper(Fd, Rd)) return false;
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = (T)Rd[k];
        if (sizeof(T) == 4) atomicAdd(fallback, 1u);
    }
    // F - R formed as H + (I - R) to keep the small difference accurate
    T D[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) D[k] = H[k] + (((k % 4 == 0) ? T(1) : T(0)) - R[k]);
    const T lj = lambda * (J - T(1)) * J;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            tau[r * 3 + c] = T(2) * mu * (D[r * 3 + 0] * F[c * 3 + 0] + D[r * 3 + 1] * F[c * 3 + 1] +
                                          D[r * 3 + 2] * F[c * 3 + 2]) +
                             (r == c ? lj : T(0));
    return true;
}

template <typename T, int MODEL>
__device__ __forceinline__ bool kirchhoff(const SimDev<T> &S, const T H[9], T tau[9])
{
    if (MODEL == 0) return tau_neohookean<T>(H, S.mu, S.lambda, tau);
    return tau_corotated<T>(H, S.mu, S.lambda, tau, S.fallback);
}

// ---------------------------------------------------------------- indenter

__device__ __forceinline__ uint64_t lattice_hash(uint64_t seed, int64_t ix, int64_t iy)
{
    // one SplitMix64 output step (Steele, Lea and Flood, 2014) of a key built
    // from the seed and the lattice corner
    uint64_t z = seed + (uint64_t)ix * 0x9E3779B97F4A7C15ull + (uint64_t)iy * 0xD1B54A32D192ED03ull;
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// 2D gradient noise with quintic fade (Perlin 2002), gradients from the
// eight directions (1,0),(1,1),(0,1),(-1,1),(-1,0),(-1,-1),(0,-1),(1,-1)
// indexed by the top three bits of the lattice hash.
template <typename T>
__device__ inline T gradient_noise(uint64_t seed, T x, T y)
{
    const T fx0 = tfloor<T>(x), fy0 = tfloor<T>(y);
    const int64_t X0 = (int64_t)fx0, Y0 = (int64_t)fy0;
    const T fx = x - fx0, fy = y - fy0;
    T n[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int a = c & 1, b = c >> 1;
        const int g = (int)(lattice_hash(seed, X0 + a, Y0 + b) >> 61);
        const int gxi = (g == 0 || g == 1 || g == 7) ? 1 : ((g >= 3 && g <= 5) ? -1 : 0);
        const int gyi = (g >= 1 && g <= 3) ? 1 : ((g >= 5) ? -1 : 0);
        n[c] = T(gxi) * (fx - T(a)) + T(gyi) * (fy - T(b));
    }
    const T u = fx * fx * fx * (fx * (fx * T(6) - T(15)) + T(10));
    const T w = fy * fy * fy * (fy * (fy * T(6) - T(15)) + T(10));
    const T lo = n[0] + u * (n[1] - n[0]);
    const T hi = n[2] + u * (n[3] - n[2]);
    return lo + w * (hi - lo);
}

template <typename T>
__device__ __forceinline__ T rounded_cone_phi(T rho, T z, T th_sin, T th_cos, T rt)
{
    // cone of half-angle th with apex at (0, rt) inflated by rt
    const T qz = z - rt;
    const T s = rho * th_sin + qz * th_cos;
    const T d = (s <= T(0)) ? sqrt(rho * rho + qz * qz) : (rho * th_cos - qz * th_sin);
    return d - rt;
}

// Inside test of the indenter (<= 0 inside) at a point given in the indenter
// frame in metres. For CONE/EDGE p[0], p[1] hold sin and cos of the
// half-angle and p[2] the tip radius (precomputed on the host).
template <typename T>
__device__ __forceinline__ T indenter_phi(const IndenterDev<T> &I, T x, T y, T z)
{
    switch (I.shape) {
    case 0: {
        const T dz = z - I.p[0];
        return sqrt(x * x + y * y + dz * dz) - I.p[0];
    }
    case 1: {
        const T dr = sqrt(x * x + y * y) - I.p[0], dz = -z;
        const T mx = dr > dz ? dr : dz;
        const T ox = dr > T(0) ? dr : T(0), oz = dz > T(0) ? dz : T(0);
        return (mx < T(0) ? mx : T(0)) + sqrt(ox * ox + oz * oz);
    }
    case 2:
        return rounded_cone_phi<T>(sqrt(x * x + y * y), z, I.p[0], I.p[1], I.p[2]);
    case 3:
        return rounded_cone_phi<T>(fabs(x), z, I.p[0], I.p[1], I.p[2]);
    case 4: {
        const T surf = I.p[1] * gradient_noise<T>(I.seed, x / I.p[2], y / I.p[2]);
        const T ex = fabs(x) - I.p[0], ey = fabs(y) - I.p[0], ez = surf - z;
        T mx = ex > ey ? ex : ey;
        return mx > ez ? mx : ez;
    }
    default:
        return T(1);
    }
}

}  // namespace tacchi
