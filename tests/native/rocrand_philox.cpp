// Prints Philox4x32-10 blocks computed by rocRAND's own engine (a library
// routine used here only as an independent check of the oracle's generator).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin; writes "o0 o1 o2 o3" (hex).
//
// rocRAND's engine keys with (seed low word, seed high word) and places the
// subsequence in counter words 2-3 and offset/4 in counter words 0-1, so the
// block for counter (c0,c1,c2,c3) and key (k0,k1) is the first output of the
// engine built with seed k1:k0 and subsequence c3:c2, advanced by 4*(c1:c0)
// outputs (in steps small enough not to overflow the 64-bit offset).
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long blocks = ((unsigned long long)c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine eng(seed, sub, 0);
        while (blocks > 0) {
            unsigned long long step = blocks < (1ull << 60) ? blocks : (1ull << 60);
            eng.discard(step * 4ull);
            blocks -= step;
        }
        unsigned o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
    }
    return 0;
}
