// Host-only driver of rocRAND's Philox4x32-10 engine, used to pin the CPU
// oracle's Philox implementation against an independent library one.
// Reads lines "key_lo key_hi c0 c1 c2 c3" (decimal) from stdin and prints the
// four 32-bit outputs of Philox4x32-10(counter = (c0,c1,c2,c3), key).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long kl, kh, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &kl, &kh, &c0, &c1, &c2, &c3) == 6) {
        // rocRAND: key = seed; counter words 2,3 = subsequence; words 0,1 += offset/4
        unsigned long long seed = kl | (kh << 32);
        unsigned long long subsequence = c2 | (c3 << 32);
        unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine e(seed, subsequence, offset);
        unsigned a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
