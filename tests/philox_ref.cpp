// Reference Philox-4x32-10 values from rocRAND's host-callable engine (a library routine),
// used only to pin the oracle's own Philox.  Reads lines "seed subsequence offset" on stdin and
// prints the next four 32-bit outputs of the engine for each.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        unsigned int a = e(), b = e(), c = e(), d = e();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
