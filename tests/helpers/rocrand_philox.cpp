// Test helper: evaluates rocRAND's host-callable Philox4x32-10 for the
// (key, counter) pairs read from stdin, one "k0 k1 c0 c1 c2 c3" line each,
// and prints the four output lanes.  rocRAND maps seed -> key, subsequence ->
// counter words 2..3 and offset/4 -> counter words 0..1, so
// rocrand_init(k0 | k1<<32, c2 | c3<<32, 4*(c0 | c1<<32)) followed by four
// rocrand() calls yields lanes o0..o3 of the block at that counter (valid
// while c1 < 2^30).  Compiled with the host compiler only; no GPU needed.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main()
{
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%x %x %x %x %x %x", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        rocrand_state_philox4x32_10 st;
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long off = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
        rocrand_init(seed, sub, off, &st);
        unsigned o0 = rocrand(&st), o1 = rocrand(&st), o2 = rocrand(&st), o3 = rocrand(&st);
        std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
    }
    return 0;
}
