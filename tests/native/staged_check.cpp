// Host check of the LDS-staged overrelaxation's index arithmetic
// (su2_staged.hpp), run by tests/test_indexing.py; it needs no GPU.
//
// For each class direction mu, lattice shape and slab plan, the check
// replays every block's schedule on a tag array standing in for its LDS:
// the prologue and each slice's loads write, at the element load_item
// names, the (direction, parity, checkerboard index) of the global link
// they read.  Before a slice's updates, every one of the 18 links of every
// site's staple, looked up with staged_link_index, must carry the tag of the
// link plain coordinate arithmetic gives for that staple term; every element
// index stays inside the plan's LDS; every site of the class is updated
// exactly once over all blocks.
#include "su2_staged.hpp"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace su2;

static long g_fail = 0;

struct Tag {
    int dir, par;
    uint32_t cb;
    bool operator==(const Tag &o) const { return dir == o.dir && par == o.par && cb == o.cb; }
};

static void fail(const char *what, int mu, const int32_t n[4], const StagePlan &p, long detail)
{
    if (g_fail++ < 20)
        std::printf("FAIL %s: mu %d shape %dx%dx%dx%d plan A=%u B=%u S=%u detail %ld\n", what, mu, n[0], n[1], n[2],
                    n[3], p.A, p.B, p.S, detail);
}

static Tag ref_link(const int32_t n[4], const int32_t c[4], int d, const int32_t e[4])
{
    int32_t w[4];
    for (int k = 0; k < 4; ++k)
        w[k] = ((c[k] + e[k]) % n[k] + n[k]) % n[k];
    const uint32_t site = (uint32_t)w[0] + (uint32_t)n[0] * ((uint32_t)w[1] + (uint32_t)n[1] * ((uint32_t)w[2] + (uint32_t)n[2] * (uint32_t)w[3]));
    return {d, (w[0] + w[1] + w[2] + w[3]) & 1, site / 2};
}

template <int MU>
static void check_plan(const int32_t n[4], const StagePlan &p, int par)
{
    using R = Roles<MU>;
    const Geom g = make_geom(n, 0, 0);
    const uint32_t total = array_shape<MU>(p, 4).base;
    if (array_shape<MU>(p, 3).base + array_shape<MU>(p, 3).count != total)
        fail("array sizes", MU, n, p, total);
    const int opp = par ^ 1;
    const uint32_t half = g.half;
    std::vector<uint8_t> updated(half, 0);
    std::vector<Tag> lds(total);
    const uint32_t nblocks = p.na * p.nb * p.ns;
    const uint32_t sites = p.A * p.B * p.nxh;
    if (load_count<MU>(p, 15u) != p.n_fresh)
        fail("n_fresh", MU, n, p, p.n_fresh);
    for (uint32_t blk = 0; blk < nblocks; ++blk) {
        const uint32_t j = xcd_tile(blk, nblocks);
        const uint32_t ia = j % p.na, ib = (j / p.na) % p.nb, is = j / (p.na * p.nb);
        const uint32_t y0 = ia * p.A, b0 = ib * p.B;
        const int32_t s0 = (int32_t)(is * p.S);
        for (auto &t : lds)
            t = {-1, -1, 0xffffffffu};
        auto stage = [&](uint32_t which, int32_t ss, int32_t sm) {
            const uint32_t cnt = load_count<MU>(p, which);
            for (uint32_t i = 0; i < cnt + 3; ++i) {
                LoadItem it;
                const bool ok = load_item<MU>(g, p, y0, b0, s0, which, ss, sm, opp, i, it);
                if (ok != (i < cnt)) {
                    fail("load_item range", MU, n, p, (long)i);
                    continue;
                }
                if (!ok)
                    continue;
                if (it.lds >= total || it.cb >= half) {
                    fail("load out of bounds", MU, n, p, (long)it.lds);
                    continue;
                }
                lds[it.lds] = {it.dir, it.parity, it.cb};
            }
        };
        stage(1u, s0 - 1, 0);
        stage(8u, 0, s0 - 1);
        stage(8u, 0, s0);
        // the slice loop's loads as the kernel forms them: decoded once
        // (load_base), then per slice (load_at); they must be load_item's
        std::vector<LoadBase> bases(p.n_fresh);
        for (uint32_t i = 0; i < p.n_fresh; ++i)
            if (!load_base<MU>(g, p, y0, b0, opp, i, bases[i]))
                fail("load_base range", MU, n, p, (long)i);
        for (int32_t sl = s0; sl < s0 + (int32_t)p.S; ++sl) {
            const SliceTerms terms = slice_terms<MU>(g, p, s0, sl);
            for (uint32_t i = 0; i < p.n_fresh; ++i) {
                LoadItem it;
                load_item<MU>(g, p, y0, b0, s0, 15u, sl, sl + 1, opp, i, it);
                uint32_t cb, li;
                load_at(bases[i], terms, cb, li);
                const int plane = (int)(bases[i].info & 0xffu);
                if (cb != it.cb || li != it.lds || plane != 2 * it.dir + it.parity)
                    fail("load_base/load_at differ from load_item", MU, n, p, (long)i);
            }
            stage(15u, sl, sl + 1);
            for (uint32_t u = 0; u < sites; ++u) {
                const uint32_t xh = u % p.nxh, row = u / p.nxh;
                const int32_t a = (int32_t)(row % p.A), b = (int32_t)(row / p.A);
                const uint32_t own_cb = xh + p.nxh * global_row<MU>(g, y0, b0, a, b, sl);
                // the site's coordinates, as the kernel forms them
                const uint32_t yc = y0 + (uint32_t)a, bc = b0 + (uint32_t)b, sc = (uint32_t)sl;
                const uint32_t xs = 2u * xh + ((yc + bc + sc + (uint32_t)par) & 1u);
                int32_t c[4];
                c[0] = (int32_t)xs;
                c[1] = (int32_t)yc;
                c[R::b] = (int32_t)bc;
                c[R::s] = (int32_t)sc;
                const uint32_t site = (uint32_t)c[0] + (uint32_t)n[0] * ((uint32_t)c[1] + (uint32_t)n[1] * ((uint32_t)c[2] + (uint32_t)n[2] * (uint32_t)c[3]));
                if (((c[0] + c[1] + c[2] + c[3]) & 1) != par || site / 2 != own_cb) {
                    fail("own site", MU, n, p, (long)u);
                    continue;
                }
                if (updated[own_cb]++)
                    fail("site updated twice", MU, n, p, (long)own_cb);
                // the 18 staple links
                for (int nu = 0; nu < 4; ++nu) {
                    if (nu == MU)
                        continue;
                    int32_t m[4] = {0, 0, 0, 0}, e[4] = {0, 0, 0, 0};
                    m[MU] = 1;
                    e[nu] = 1;
                    struct Term {
                        int d;
                        int32_t s[4];
                    } terms[6] = {
                        {nu, {m[0], m[1], m[2], m[3]}},
                        {MU, {e[0], e[1], e[2], e[3]}},
                        {nu, {0, 0, 0, 0}},
                        {nu, {m[0] - e[0], m[1] - e[1], m[2] - e[2], m[3] - e[3]}},
                        {MU, {-e[0], -e[1], -e[2], -e[3]}},
                        {nu, {-e[0], -e[1], -e[2], -e[3]}},
                    };
                    for (const Term &t : terms) {
                        // the displacement in the kernel's (x, y, b, s) order
                        const int32_t ex = t.s[0], ea = t.s[1], eb = t.s[R::b], es = t.s[R::s];
                        const uint32_t li =
                            staged_link_index<MU>(p, s0, sl, (uint32_t)n[0], xs, a, b, par, t.d, ex, ea, eb, es);
                        if (li >= total) {
                            fail("staple index out of LDS", MU, n, p, (long)li);
                            continue;
                        }
                        if (!(lds[li] == ref_link(n, c, t.d, t.s)))
                            fail("staple link", MU, n, p, (long)own_cb);
                    }
                }
            }
        }
    }
    for (uint32_t cb = 0; cb < half; ++cb)
        if (!updated[cb]) {
            fail("site not updated", MU, n, p, (long)cb);
            break;
        }
}

template <int MU>
static int check_shape(const int32_t n[4])
{
    // every plan the chooser could pick for a range of LDS limits and block
    // counts, plus hand-picked slabs
    int checked = 0;
    // 147424: 160 KB less the staged heat bath's compaction state (512
    // threads x 32 B + 32 B)
    const uint32_t limits[] = {16384, 49152, 65536, 131072, 147424, 163840};
    const uint32_t mins[] = {1, 8, 64, 256};
    for (uint32_t lb : {16u, 32u})
        for (uint32_t lim : limits)
            for (uint32_t mb : mins) {
                StagePlan p;
                if (!make_stage_plan<MU>(n, lb, lim, mb, p))
                    continue;
                if ((uint64_t)array_shape<MU>(p, 4).base * lb > lim)
                    fail("plan above its LDS limit", MU, n, p, lim);
                for (int par = 0; par < 2; ++par)
                    check_plan<MU>(n, p, par);
                ++checked;
            }
    return checked;
}

int main()
{
    const int32_t shapes[][4] = {{8, 8, 8, 8},    {16, 8, 8, 4},  {32, 16, 8, 8}, {16, 16, 16, 16}, {8, 12, 6, 10},
                                 {64, 16, 8, 16}, {32, 8, 16, 8}, {32, 16, 8, 4}, {16, 8, 8, 16},   {48, 12, 6, 6}};
    for (const auto &n : shapes) {
        const int c0 = check_shape<0>(n), c1 = check_shape<1>(n), c2 = check_shape<2>(n), c3 = check_shape<3>(n);
        std::printf("ok %dx%dx%dx%d plans checked %d %d %d %d\n", n[0], n[1], n[2], n[3], c0, c1, c2, c3);
    }
    // the plan the library takes at the benchmark's sizes (160 KB of LDS,
    // 256 slabs at least), its loads per update, checked in full at 64^4
    for (uint32_t lb : {16u, 32u}) {
        const int32_t n[4] = {64, 64, 64, 64};
        StagePlan p;
        if (make_stage_plan<0>(n, lb, 163840, 256, p)) {
            std::printf("64^4 link %u B, mu=x: A=%u B=%u S=%u slabs=%u LDS=%u fresh/slice=%u (%.2f loads per update)\n",
                        lb, p.A, p.B, p.S, p.na * p.nb * p.ns, p.lds_bytes, p.n_fresh,
                        (double)p.n_fresh / (p.A * p.B * p.nxh) + 1.0);
            for (int par = 0; par < 2; ++par)
                check_plan<0>(n, p, par);
        }
        StagePlan q;
        if (make_stage_plan<3>(n, lb, 163840, 256, q)) {
            for (int par = 0; par < 2; ++par)
                check_plan<3>(n, q, par);
        }
        // the staged heat bath's plans (its compaction state beside the ring)
        for (int par = 0; par < 2; ++par) {
            StagePlan h0, h3;
            if (make_stage_plan<0>(n, lb, 147424, 256, h0))
                check_plan<0>(n, h0, par);
            if (make_stage_plan<3>(n, lb, 147424, 256, h3))
                check_plan<3>(n, h3, par);
        }
        // a device that gives a block 64 KB
        StagePlan r;
        if (make_stage_plan<1>(n, lb, 65536, 256, r))
            check_plan<1>(n, r, 1);
        if (make_stage_plan<2>(n, lb, 65536, 256, r))
            check_plan<2>(n, r, 0);
    }
    std::printf("%s (%ld failures)\n", g_fail ? "FAILED" : "PASSED", g_fail);
    return g_fail ? 1 : 0;
}
