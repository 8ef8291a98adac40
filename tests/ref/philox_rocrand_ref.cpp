// Test-only reference: prints Philox4x32-10 blocks computed by rocRAND's
// open-source engine (host path of rocrand_philox4x32_10.h), an implementation
// independent of the oracle's.  Input lines: seed path event; output: 4 words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned long long seed, path, event;
    while (std::scanf("%llu %llu %llu", &seed, &path, &event) == 3) {
        // counter = (offset/4 as 64 bits in x,y ; subsequence in z,w), key = seed
        rocrand_device::philox4x32_10_engine e(seed, event, 4ull * path);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
