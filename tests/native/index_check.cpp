// Host check of the library's own walk and neighbour-index arithmetic
// (su2_device.hpp) against plain coordinate arithmetic, for every walk mode
// and both addressing policies.  Built for the host only and run by
// tests/test_indexing.py; it needs no GPU.
//
// For each lattice shape and walk (plain order, every strip width, every
// split of the columns into row ranges):
//  - walk_cb is a bijection of [0, V/2) onto the checkerboard indices;
//  - site_of_cb gives coordinates of the right parity whose linear index
//    halves to cb;
//  - for every displacement d in {-1,0,1}^4 with |d|_1 <= 2 (all the staple
//    and plaquette needs), CbAddr::at and, where the lattice qualifies,
//    ColAddr::at (in bytes, < 2^32) equal the index computed from
//    ((x + d) mod N);
//  - xcd_tile is a bijection of [0, nblocks).
// Large lattices are checked on a strided sample of walk indices plus the
// first and last columns.
#include "su2_device.hpp"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace su2;

static long g_fail = 0;

static void fail(const char *what, const int32_t n[4], int tile, uint32_t i, int par)
{
    if (g_fail++ < 10)
        std::printf("FAIL %s: shape %dx%dx%dx%d tile %d index %u parity %d\n", what, n[0], n[1], n[2], n[3], tile,
                    i, par);
}

static uint32_t ref_cb(const int32_t n[4], const int32_t c[4], const int32_t d[4])
{
    int32_t w[4];
    for (int k = 0; k < 4; ++k)
        w[k] = ((c[k] + d[k]) % n[k] + n[k]) % n[k];
    return (uint32_t)(w[0] / 2) + (uint32_t)(n[0] / 2) * ((uint32_t)w[1] + (uint32_t)n[1] * ((uint32_t)w[2] + (uint32_t)n[2] * (uint32_t)w[3]));
}

static void check_index(const Geom &g, const int32_t n[4], int tile, bool col, uint32_t i, int par,
                        std::vector<uint8_t> *seen)
{
    const uint32_t cb = walk_cb(i, g.ord);
    if (cb >= g.half) {
        fail("walk out of range", n, tile, i, par);
        return;
    }
    if (seen) {
        if ((*seen)[cb])
            fail("walk not injective", n, tile, i, par);
        (*seen)[cb] = 1;
    }
    const Site s = site_of_cb(g, cb, par);
    const int32_t *c = s.c;
    if (((c[0] + c[1] + c[2] + c[3]) & 1) != par)
        fail("parity", n, tile, i, par);
    const uint32_t lin = (uint32_t)c[0] + (uint32_t)n[0] * ((uint32_t)c[1] + (uint32_t)n[1] * ((uint32_t)c[2] + (uint32_t)n[2] * (uint32_t)c[3]));
    if (lin != s.site || lin / 2 != cb)
        fail("site index", n, tile, i, par);
    CbAddr ca;
    ca.s = s;
    ca.cb = cb;
    ca.g = &g;
    ColAddr aa = {};
    if (col) {
        aa = col_addr_at(g, i & ~63u, i & 63u, par);
        if (aa.site() != s.site)
            fail("column site", n, tile, i, par);
    }
    int32_t d[4];
    for (d[0] = -1; d[0] <= 1; ++d[0])
        for (d[1] = -1; d[1] <= 1; ++d[1])
            for (d[2] = -1; d[2] <= 1; ++d[2])
                for (d[3] = -1; d[3] <= 1; ++d[3]) {
                    if (std::abs(d[0]) + std::abs(d[1]) + std::abs(d[2]) + std::abs(d[3]) > 2)
                        continue;
                    const uint32_t r = ref_cb(n, c, d);
                    if (ca.at(d[0], d[1], d[2], d[3]) != r)
                        fail("coordinate neighbour", n, tile, i, par);
                    if (col) {
                        const uint64_t b = aa.at(d[0], d[1], d[2], d[3]);
                        if (b != 16ull * r)
                            fail("column neighbour", n, tile, i, par);
                    }
                }
}

static void check_shape(const int32_t n[4], uint32_t stride)
{
    // plain order, the defaults, and the smallest, second-smallest and
    // largest divisors (strip widths of Nz, row splits of Ny)
    auto some_divisors = [stride](int m) {
        std::vector<int> d;
        for (int k = 1; k <= m; ++k)
            if (m % k == 0)
                d.push_back(k);
        if (stride != 1)
            return d; // sampled checks are cheap: every walk the API accepts
        std::vector<int> pick = {d[0]};
        if (d.size() > 1)
            pick.push_back(d[1]);
        if (d.size() > 3)
            pick.push_back(d[d.size() / 2]);
        if (d.size() > 2)
            pick.push_back(d.back());
        return pick;
    };
    std::vector<int> tiles = {-1, 0};
    for (int w : some_divisors(n[2]))
        tiles.push_back(w);
    std::vector<int> ysplits = {0};
    for (int sy : some_divisors(n[1]))
        ysplits.push_back(sy);
    int ncol = 0;
    for (int tile : tiles)
      for (int tile_y : ysplits) {
        const Geom g = make_geom(n, tile, tile_y);
        const bool col = col_addressing_ok(g);
        ncol += col;
        for (int par = 0; par < 2; ++par) {
            if (stride == 1) {
                std::vector<uint8_t> seen(g.half, 0);
                for (uint32_t i = 0; i < g.half; ++i)
                    check_index(g, n, tile, col, i, par, &seen);
                for (uint32_t cb = 0; cb < g.half; ++cb)
                    if (!seen[cb]) {
                        fail("walk not surjective", n, tile, cb, par);
                        break;
                    }
            } else {
                const uint32_t cols = g.ord.cols < 2048u ? g.ord.cols : 2048u;
                for (uint32_t i = 0; i < g.half; i += stride)
                    check_index(g, n, tile, col, i, par, nullptr);
                for (uint32_t i = 0; i < 2 * cols && i < g.half; ++i)
                    check_index(g, n, tile, col, i, par, nullptr);
                for (uint32_t i = g.half - 2 * cols; i < g.half; ++i)
                    check_index(g, n, tile, col, i, par, nullptr);
            }
        }
      }
    std::printf("ok %dx%dx%dx%d walks=%zu column-addressed=%d stride=%u\n", n[0], n[1], n[2], n[3],
                tiles.size() * ysplits.size(), ncol, stride);
}

int main()
{
    const int32_t full[][4] = {{8, 8, 8, 8},   {6, 4, 10, 8},  {2, 2, 2, 2},   {4, 6, 2, 12}, {10, 6, 4, 6},
                               {16, 32, 8, 4}, {32, 16, 8, 2}, {32, 16, 8, 4}, {16, 16, 16, 4}, {8, 8, 8, 4},
                               {16, 8, 8, 4},  {24, 16, 6, 6}, {8, 16, 4, 2}};
    for (const auto &n : full)
        check_shape(n, 1);
    // up to the largest the API accepts: V/2 = 2^28 (the last column-
    // addressed size: byte offsets of a plane just fit 32 bits), V/2 > 2^28
    // (coordinate addressing), and V just under 2^32 (the 32-bit site index)
    const int32_t big[][4] = {{16, 16, 16, 16}, {32, 32, 32, 4},    {48, 48, 48, 6},    {64, 64, 64, 8},
                              {64, 64, 64, 64}, {96, 96, 96, 96},   {128, 128, 128, 256}, {160, 160, 160, 160},
                              {256, 256, 256, 254}, {254, 256, 256, 256}};
    for (const auto &n : big)
        check_shape(n, 99991);
    for (uint32_t nb = 1; nb < 3000; nb += 7) {
        std::vector<uint8_t> hit(nb, 0);
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t t = xcd_tile(b, nb);
            if (t >= nb || hit[t]++) {
                const int32_t z[4] = {0, 0, 0, 0};
                fail("xcd_tile", z, 0, b, 0);
                break;
            }
        }
    }
    std::printf("%s (%ld failures)\n", g_fail ? "FAILED" : "PASSED", g_fail);
    return g_fail ? 1 : 0;
}
