// Reference Philox4x32-10 block from rocRAND's engine (host path only), used to pin
// the oracle's own implementation. Arguments: key0 key1 c0 c1 c2 c3.
// rocRAND maps seed -> key (low, high word), subsequence -> counter words 2-3 and
// offset/4 -> counter words 0-1, so one next4() right after seeding returns the
// block at exactly the requested counter.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>
#include <cstdlib>

int main(int argc, char **argv)
{
    if (argc != 7)
        return 2;
    unsigned long v[6];
    for (int i = 0; i < 6; ++i)
        v[i] = strtoul(argv[i + 1], nullptr, 0);
    unsigned long long seed = ((unsigned long long)v[1] << 32) | v[0];
    unsigned long long sub = ((unsigned long long)v[5] << 32) | v[4];
    unsigned long long blk = ((unsigned long long)v[3] << 32) | v[2];
    rocrand_device::philox4x32_10_engine e(seed, sub, 0);
    // offset in numbers = 4 * block; applied in pieces that fit in 64 bits
    const unsigned long long piece = 1ull << 60;
    while (blk > 0) {
        unsigned long long s = blk < piece ? blk : piece;
        e.discard(4ull * s);
        blk -= s;
    }
    uint4 r = e.next4();
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    return 0;
}
