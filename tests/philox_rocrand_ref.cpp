// Test-only reference program: evaluates Philox4x32-10 blocks through rocRAND's
// engine (an implementation independent of both the oracle and the GPU
// library).  Reads lines "c0 c1 c2 c3 k0 k1" (decimal u32) on stdin and prints
// the four output words of each block.
//
// rocRAND's engine keyed by seed = (k1 << 32) | k0, started at subsequence
// (c3 << 32) | c2 and offset 4 * ((c1 << 32) | c0), returns the four words of the
// block with counter (c0, c1, c2, c3) as its next four outputs.
#include <rocrand/rocrand_kernel.h>

#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_init(seed, sub, off, &st);
        unsigned w0 = rocrand(&st), w1 = rocrand(&st), w2 = rocrand(&st), w3 = rocrand(&st);
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
