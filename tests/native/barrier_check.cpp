// Host check of the persistent sweep's barrier counter arithmetic
// (barrier_increment, barrier_passed in su2_device.hpp): G blocks arrive at
// a sequence of barriers in random orders, their additions applied one at a
// time as the device's atomic additions would be.  Checked:
//  - no block sees the barrier passed before the last block has arrived,
//    and every block sees it passed right after (whatever the order, the
//    word's value before the barrier, and which block comes last);
//  - bits 0-30 of the word return to 0 after every barrier and bit 31
//    flips once per barrier, so nothing needs resetting between barriers or
//    launches;
//  - with blocks that give up waiting and run ahead (arriving at later
//    barriers before earlier ones complete), the word still ends at bits
//    0-30 = 0 once every block has arrived at every barrier.
// Built for the host only and run by tests/test_indexing.py.
#include "su2_device.hpp"

#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

using namespace su2;

static long g_fail = 0;

static void fail(const char *what, uint32_t g, int barrier, uint32_t detail)
{
    if (g_fail++ < 10)
        std::printf("FAIL %s: grid %u barrier %d detail %u\n", what, g, barrier, detail);
}

int main()
{
    std::mt19937 rng(20041);
    for (uint32_t g : {1u, 2u, 8u, 16u, 64u, 768u, 1280u, 2048u}) {
        for (uint32_t start : {0u, 0x80000000u}) {
            uint32_t word = start;
            std::vector<uint32_t> order(g), old(g);
            for (uint32_t b = 0; b < g; ++b)
                order[b] = b;
            for (int bar = 0; bar < 41; ++bar) {
                std::shuffle(order.begin(), order.end(), rng);
                const uint32_t phase = word & 0x80000000u;
                for (uint32_t k = 0; k < g; ++k) {
                    const uint32_t b = order[k];
                    old[b] = word;
                    word += barrier_increment(b, g);
                    if (k + 1 < g) {
                        // nobody may pass yet: check the arrivals so far
                        // (all of them on small grids, a sample on large)
                        const uint32_t step = g > 64 ? 97u : 1u;
                        for (uint32_t j = 0; j <= k; j += step)
                            if (barrier_passed(word, old[order[j]]))
                                fail("passed early", g, bar, k);
                        if (barrier_passed(word, old[b]))
                            fail("passed early (last arrival so far)", g, bar, k);
                    }
                }
                for (uint32_t b = 0; b < g; ++b)
                    if (!barrier_passed(word, old[b]))
                        fail("not passed after the last arrival", g, bar, b);
                if ((word & 0x7fffffffu) != 0u)
                    fail("low bits not back to 0", g, bar, word);
                if ((word & 0x80000000u) == phase)
                    fail("phase did not flip", g, bar, word);
            }
        }
        // run-ahead: each block arrives at all barriers in its own order of
        // time, interleaved at random with the others (but in its own
        // sequence); the sum of every block's additions over 39 barriers
        uint32_t word = 0;
        std::vector<int> next(g, 0);
        std::vector<uint32_t> pending;
        for (uint32_t b = 0; b < g; ++b)
            for (int bar = 0; bar < 39; ++bar)
                pending.push_back(b);
        std::shuffle(pending.begin(), pending.end(), rng);
        for (uint32_t b : pending) {
            word += barrier_increment(b, g);
            ++next[b];
        }
        if ((word & 0x7fffffffu) != 0u || (word & 0x80000000u) == 0u)
            fail("run-ahead arrivals leave the word inconsistent", g, 39, word);
        std::printf("ok grid %u\n", g);
    }
    std::printf("%s (%ld failures)\n", g_fail ? "FAILED" : "PASSED", g_fail);
    return g_fail ? 1 : 0;
}
