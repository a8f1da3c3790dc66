// Reads lines "c0 c1 c2 c3 k0 k1" (hex) and prints the Philox4x32-10 block
// produced by rocRAND's header-only engine for that key and counter.
// rocRAND maps (seed, subsequence, offset) onto key = seed, counter words
// (0,1) = offset / 4 and counter words (2,3) = subsequence.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long offset = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, subseq, offset, &st);
        unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
