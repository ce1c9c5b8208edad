// Host-side check of the index arithmetic the MPM kernels share (compiled
// from the same headers, run on the CPU): the XCD-aware block order is a
// permutation of the blocks for every block count and chunk size the
// library uses, and so is the box-first dispatch order for every box; the velocity grid's node layout is a bijection; the P2G and
// G2P LDS tile layouts keep every channel of every tile node inside the
// tile and apart from every other; every tile node the scatter or gather
// can touch lies in the tile; and the grid update's gather finds, for every
// node of a block, exactly the neighbouring tiles that cover it, at slots
// inside those tiles that hold that node. Prints "ok" and exits 0, or
// prints the first failure and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2301_08343_amd/csrc/sim_kernels.hpp"

using namespace tacchi;

static int fails = 0;
#define CHECK(cond, ...)                        \
    do {                                        \
        if (!(cond)) {                          \
            if (fails++ < 5) {                  \
                std::printf("FAIL %s: ", #cond); \
                std::printf(__VA_ARGS__);       \
                std::printf("\n");              \
            }                                   \
        }                                       \
    } while (0)

static void check_xcd_block()
{
    for (int nb0 = 1; nb0 <= 40; ++nb0) {
        const int C = 3 * nb0;  // the library's chunk: three rows of blocks
        const int counts[] = {1, 7, 8, 9, 8 * C - 1, 8 * C, 8 * C + 1, 16 * C + 5, 8192, nb0 * nb0 * 5 + 3};
        for (int n : counts) {
            std::vector<int> seen(n, 0);
            for (int i = 0; i < n; ++i) {
                const int b = xcd_block(i, n, C);
                CHECK(b >= 0 && b < n, "n=%d C=%d i=%d -> %d", n, C, i, b);
                if (b >= 0 && b < n) seen[b]++;
            }
            for (int b = 0; b < n; ++b) CHECK(seen[b] == 1, "n=%d C=%d block %d taken %d times", n, C, b, seen[b]);
        }
    }
}

// The box-first dispatch order is a permutation of the grid's blocks for
// boxes anywhere inside grids of several shapes, the whole grid, one block
// and an empty box included, and it takes the box's blocks first.
static void check_box_first()
{
    const int grids[][3] = {{32, 32, 8}, {7, 5, 3}, {1, 1, 1}, {4, 9, 2}, {13, 1, 6}};
    for (const auto &g : grids) {
        const int nb0 = g[0], nb1 = g[1], nb2 = g[2], n = nb0 * nb1 * nb2;
        std::vector<int> boxes;  // x0, y0, z0, xn, yn, zn
        for (int x0 = 0; x0 < nb0; x0 += (nb0 > 6 ? 3 : 1))
            for (int xn = 0; x0 + xn <= nb0; xn += (nb0 > 6 ? 5 : 1))
                for (int y0 = 0; y0 < nb1; y0 += (nb1 > 6 ? 4 : 1))
                    for (int yn = 1; y0 + yn <= nb1; yn += (nb1 > 6 ? 7 : 1))
                        for (int z0 = 0; z0 < nb2; ++z0)
                            for (int zn = 1; z0 + zn <= nb2; zn += 2) {
                                const int bx[6] = {x0, y0, z0, xn, yn, zn};
                                boxes.insert(boxes.end(), bx, bx + 6);
                            }
        const int full[6] = {0, 0, 0, nb0, nb1, nb2};
        boxes.insert(boxes.end(), full, full + 6);
        for (size_t q = 0; q < boxes.size(); q += 6) {
            const int *bx = &boxes[q];
            const int nbox = bx[3] * bx[4] * bx[5];
            std::vector<int> seen(n, 0);
            for (int i = 0; i < n; ++i) {
                const int b = box_first_block(i, nb0, nb1, nb2, bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], 3 * bx[3]);
                CHECK(b >= 0 && b < n, "grid %dx%dx%d box (%d,%d,%d)+(%d,%d,%d) i=%d -> %d", nb0, nb1, nb2, bx[0], bx[1],
                      bx[2], bx[3], bx[4], bx[5], i, b);
                if (b < 0 || b >= n) continue;
                seen[b]++;
                const int x = b % nb0, y = (b / nb0) % nb1, z = b / (nb0 * nb1);
                const bool in = x >= bx[0] && x < bx[0] + bx[3] && y >= bx[1] && y < bx[1] + bx[4] && z >= bx[2] &&
                                z < bx[2] + bx[5];
                CHECK(in == (i < nbox), "grid %dx%dx%d box (%d,%d,%d)+(%d,%d,%d): i=%d -> block %d inside=%d", nb0, nb1,
                      nb2, bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], i, b, (int)in);
            }
            for (int b = 0; b < n; ++b)
                CHECK(seen[b] == 1, "grid %dx%dx%d box (%d,%d,%d)+(%d,%d,%d): block %d taken %d times", nb0, nb1, nb2,
                      bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], b, seen[b]);
        }
    }
}

template <int B>
static void check_node_layout()
{
    std::vector<int> seen(B * B * B, 0);
    for (int z = 0; z < B; ++z)
        for (int y = 0; y < B; ++y)
            for (int x = 0; x < B; ++x) {
                const int l = node_local<B>(x, y, z);
                CHECK(l >= 0 && l < B * B * B, "B=%d (%d,%d,%d) -> %d", B, x, y, z, l);
                if (l >= 0 && l < B * B * B) seen[l]++;
            }
    for (int l = 0; l < B * B * B; ++l) CHECK(seen[l] == 1, "B=%d local %d taken %d times", B, l, seen[l]);
    const int nb[3] = {3, 2, 4};
    const int64_t total = (int64_t)nb[0] * nb[1] * nb[2] * B * B * B;
    std::vector<int> g(total, 0);
    for (int z = 0; z < nb[2] * B; ++z)
        for (int y = 0; y < nb[1] * B; ++y)
            for (int x = 0; x < nb[0] * B; ++x) {
                const int64_t a = node_addr<B>(nb[0], nb[1], x, y, z);
                CHECK(a >= 0 && a < total, "B=%d node (%d,%d,%d) -> %lld", B, x, y, z, (long long)a);
                if (a >= 0 && a < total) g[a]++;
            }
    for (int64_t a = 0; a < total; ++a) CHECK(g[a] == 1, "B=%d address %lld taken %d times", B, (long long)a, g[a]);
}

template <int B>
static void check_tiles()
{
    constexpr int TB = B + 3, TN = TB * TB * TB;
    // tile storage order: a bijection, inverted by coords
    std::vector<int> seen(TN, 0);
    for (int z = 0; z < TB; ++z)
        for (int y = 0; y < TB; ++y)
            for (int x = 0; x < TB; ++x) {
                const int s = TileRegions<B>::slot_of(x, y, z);
                CHECK(s >= 0 && s < TN, "B=%d tile (%d,%d,%d) -> %d", B, x, y, z, s);
                if (s < 0 || s >= TN) continue;
                seen[s]++;
                int a, b, c;
                TileRegions<B>::coords(s, a, b, c);
                CHECK(a == x && b == y && c == z, "B=%d slot %d -> (%d,%d,%d), not (%d,%d,%d)", B, s, a, b, c, x, y, z);
            }
    for (int s = 0; s < TN; ++s) CHECK(seen[s] == 1, "B=%d slot %d taken %d times", B, s, seen[s]);
    // LDS layouts: every (node, channel) inside the tile, no two alike
    using LP = P2GTileLayout<B>;
    using LG = G2PTileLayout<B>;
    std::vector<int> p2g(LP::SLOTS, 0), g2p(LG::SLOTS, 0);
    for (int z = 0; z < TB; ++z)
        for (int y = 0; y < TB; ++y)
            for (int x = 0; x < TB; ++x) {
                for (int ch = 0; ch < 4; ++ch) {
                    const int i = LP::at(x, y, z, ch);
                    CHECK(i >= 0 && i < LP::SLOTS, "B=%d P2G (%d,%d,%d) ch %d -> %d", B, x, y, z, ch, i);
                    if (i >= 0 && i < LP::SLOTS) p2g[i]++;
                }
                for (int r = 0; r < 3; ++r) {
                    const int i = LG::at(x, y, z, r);
                    CHECK(i >= 0 && i < LG::SLOTS, "B=%d G2P (%d,%d,%d) r %d -> %d", B, x, y, z, r, i);
                    if (i >= 0 && i < LG::SLOTS) g2p[i]++;
                }
            }
    for (int i = 0; i < LP::SLOTS; ++i) CHECK(p2g[i] <= 1, "B=%d P2G slot %d shared by %d", B, i, p2g[i]);
    for (int i = 0; i < LG::SLOTS; ++i) CHECK(g2p[i] <= 1, "B=%d G2P slot %d shared by %d", B, i, g2p[i]);
    // the transfers touch tile nodes base - lo + (0..2) for stencil bases the
    // kernels accept (0 <= base - lo <= B, lo = the block's first node - 1)
    for (int l = 0; l <= B; ++l)
        for (int o = 0; o < 3; ++o) CHECK(l + o >= 0 && l + o < TB, "B=%d stencil %d + %d leaves the tile", B, l, o);
    // gather: the tiles covering node l of block b along one axis are those
    // of blocks b + o whose span (lo_c - 1 .. lo_c + B + 1, lo_c = (b + o) B)
    // holds b B + l; gather_cover must name exactly those, and the tile
    // coordinate l - o B + 1 must lie in the tile
    for (int l = 0; l < B; ++l) {
        int o0, o1;
        bool two;
        gather_cover<B>(l, o0, o1, two);
        std::vector<int> want;
        for (int o = -1; o <= 1; ++o) {
            const int t = l - o * B + 1;
            if (t >= 0 && t < TB) want.push_back(o);
        }
        std::vector<int> got = {o0};
        if (two) got.push_back(o1);
        CHECK(got == want, "B=%d l=%d: gather takes %zu tiles, %zu cover the node", B, l, got.size(), want.size());
        for (int o : got) {
            const int t = l - o * B + 1;
            CHECK(t >= 0 && t < TB, "B=%d l=%d o=%d: tile coordinate %d", B, l, o, t);
        }
    }
}

int main()
{
    check_xcd_block();
    check_box_first();
    check_node_layout<4>();
    check_node_layout<8>();
    check_tiles<4>();
    check_tiles<8>();
    if (fails) {
        std::printf("%d failures\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
