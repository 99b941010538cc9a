// Independent Philox4x32-10 reference for the tests: rocRAND's header-only
// engine (the installed rocrand_philox4x32_10.h, a separate implementation
// from the oracle's), run on the host.  The engine starts from counter 0 and
// key = seed; a "subsequence" s adds to counter words 2..3 and an offset of
// 4*n outputs adds n to counter words 0..1, so (seed, s, 4n) reaches any
// (counter, key).  Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin and prints
// the four output words (hex) per line.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k1 << 32 | k0;
        unsigned long long sub = (unsigned long long)c3 << 32 | c2;
        unsigned long long n = (unsigned long long)c1 << 32 | c0;
        rocrand_device::philox4x32_10_engine eng(seed, sub, 0ull);
        // advance by n blocks of four outputs, in two steps so 4n cannot overflow
        eng.discard(4ull * (n >> 2));
        eng.discard(4ull * (n >> 2));
        eng.discard(4ull * (n >> 2));
        eng.discard(4ull * (n >> 2));
        eng.discard(4ull * (n & 3ull));
        unsigned o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
    }
    return 0;
}
