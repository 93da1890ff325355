// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) on stdin and prints the
// four 32-bit outputs of PyTorch's header-only host Philox4x32-10 engine for
// that counter and key.  Used only to pin the oracle's own Philox.
// PyTorch's engine takes (seed, subsequence, offset) and forms
// counter = (offset lo, offset hi, subsequence lo, subsequence hi),
// key = (seed lo, seed hi).
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint64_t seed = k0 | (k1 << 32);
        uint64_t subseq = c2 | (c3 << 32);
        uint64_t offset = c0 | (c1 << 32);
        at::Philox4_32 eng(seed, subseq, offset);
        uint32_t r0 = eng(10), r1 = eng(10), r2 = eng(10), r3 = eng(10);
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
