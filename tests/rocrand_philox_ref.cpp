// Prints Philox4x32-10 blocks computed by rocRAND's header-only engine on the
// host, for (counter, key) rows read from stdin as six hex words
// c0 c1 c2 c3 k0 k1.  An independent implementation of the generator
// (Salmon et al., SC'11) used to pin the oracle's own Philox.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        // advance the counter's low 64 bits by c0 + c1 * 2^32 blocks; discard()
        // counts 32-bit outputs (4 per block), so split the advance into
        // pieces that fit in 64 bits: 4*c0, then 16 pieces of c1 * 2^30
        rocrand_device::philox4x32_10_engine e(seed, subsequence, 4ull * c0);
        for (int i = 0; i < 16 && c1 != 0; ++i) e.discard((unsigned long long)c1 << 30);
        unsigned a = e.next(), b = e.next(), c = e.next(), d = e.next();
        std::printf("%08x %08x %08x %08x\n", a, b, c, d);
    }
    return 0;
}
