// Prints Philox4x32-10 blocks produced by rocRAND's own generator, used only to
// cross-check the oracle's Philox against an independent implementation.
// rocrand_init(seed, subsequence, offset): the key is the 64-bit seed split
// into (low, high) words, the subsequence fills counter words 2 and 3, and an
// offset of 4*n starts at counter words (0, 1) = n.
// Usage: probe <seed> <c0> <c1> <c2> <c3> <n_blocks>
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char** argv)
{
    if (argc != 7) return 2;
    unsigned long long seed = strtoull(argv[1], 0, 0);
    unsigned long long c0 = strtoull(argv[2], 0, 0), c1 = strtoull(argv[3], 0, 0);
    unsigned long long c2 = strtoull(argv[4], 0, 0), c3 = strtoull(argv[5], 0, 0);
    int n = atoi(argv[6]);
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, (c3 << 32) | c2, 4ull * ((c1 << 32) | c0), &st);
    for (int i = 0; i < 4 * n; ++i) printf("%u\n", rocrand(&st));
    return 0;
}
