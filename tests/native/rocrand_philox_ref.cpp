// Independent Philox4x32-10 values for pinning the oracle: rocRAND's engine, run on
// the host. Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four
// output words of the block with that counter and key.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = k0 | (k1 << 32);
        const unsigned long long subsequence = c2 | (c3 << 32);
        const unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        unsigned int w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
