// Independent Philox4x32-10 implementation used as a pin for the CPU checker:
// rocRAND's engine, driven so that its internal counter equals the requested
// (c0, c1, c2, c3): subsequence = c3:c2, offset = 4 * (c1:c0).
// Reads lines "c0 c1 c2 c3 k0 k1" (hex) on stdin, prints four hex words each.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long off = ((unsigned long long)c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0);
        e.discard(off * 4ull);
        uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
