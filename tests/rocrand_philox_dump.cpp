// Independent Philox4x32-10 for the oracle's pin: prints rocRAND's open-source host/device engine
// output for the counters given on stdin ("ctr0 ctr1 ctr2 ctr3 key0 key1" in hex per line).
// The rocRAND engine takes key = (seed_lo32, seed_hi32) and counter words (x, y) from `offset`/4
// and (z, w) from `subsequence`, so a counter is reached with seed/subsequence/offset arithmetic.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdint>

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off4 = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        if (c1 >= (1u << 30)) { std::printf("unsupported\n"); continue; }
        rocrand_device::philox4x32_10_engine eng(seed, sub, 0);
        eng.discard(4ull * off4);               // counter words (x, y) += off4
        unsigned o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
    }
    return 0;
}
