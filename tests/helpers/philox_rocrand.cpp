// Independent reference for the oracle's Philox4x32-10: rocRAND's engine
// (an implementation of the same published generator).  Reads lines
// "c0 c1 c2 c3 k0 k1" on stdin, prints the four output words of one block.
// rocRAND counts (offset/4, subsequence) into the 128-bit counter, so the
// counter (c0, c1, c2, c3) is reached with offset = 4 (c0 + 2^32 c1) and
// subsequence = c2 + 2^32 c3 (valid for c1 < 2^30).
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_state_philox4x32_10 s;
        rocrand_init(seed, sub, off, &s);
        uint4 r = rocrand4(&s);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
