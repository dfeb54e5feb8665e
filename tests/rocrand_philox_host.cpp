// Runs rocRAND's Philox4x32-10 engine on the host to produce known-answer
// blocks for arbitrary (key, counter) pairs.  Used only by the test suite to
// pin the oracle's independent Philox implementation against a third-party
// library.  Reads lines "k0 k1 c0 c1 c2 c3" (decimal) and prints four words.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        // offset counts 32-bit outputs; each counter value yields four of them
        rocrand_device::philox4x32_10_engine eng(seed, subseq, 0);
        eng.discard(block * 4ull);
        unsigned r0 = eng.next(), r1 = eng.next(), r2 = eng.next(), r3 = eng.next();
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
