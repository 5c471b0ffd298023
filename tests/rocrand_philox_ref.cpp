// Reference Philox4x32-10 values from rocRAND's engine (an implementation
// independent of the oracle).  Reads "c0 c1 c2 c3 seed" per line, prints the
// four output words.  The engine's counter is set through its public API:
// subsequence = (c3 << 32 | c2), offset = 4 * (c1 << 32 | c0).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned int c0, c1, c2, c3;
    unsigned long long seed;
    while (std::scanf("%u %u %u %u %llu", &c0, &c1, &c2, &c3, &seed) == 5) {
        unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = 4ull * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned int a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
