// Prints Philox4x32-10 blocks computed by rocRAND's engine (an independent
// implementation) for counters/keys read from stdin: "c0 c1 c2 c3 k0 k1" per
// line -> "w0 w1 w2 w3".  Host-only use of the header.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned c[4], k[2];
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        const unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
        const unsigned long long subsequence = ((unsigned long long)c[3] << 32) | c[2];
        // counter words 0, 1 = c1 * 2^32 + c0 blocks of 4 outputs from the
        // start of the subsequence; advanced in pieces that fit 64 bits
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 4ull * c[0]);
        for (int q = 0; q < 4; ++q) eng.discard(4ull * ((unsigned long long)c[1] << 30));
        const unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
        std::printf("%u %u %u %u\n", w0, w1, w2, w3);
    }
    return 0;
}
