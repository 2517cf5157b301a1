// Host-only pin for the oracle's Philox-4x32-10: evaluates the block function
// of rocRAND's philox4x32_10 engine (a library implementation of the same
// published generator) for (counter, key) pairs read from stdin, one per line
// as "c0 c1 c2 c3 k0 k1" in decimal, and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// The ten-round block function is a protected member of the engine; a derived
// class exposes it without touching the engine's counter bookkeeping.
struct philox_block : rocrand_device::philox4x32_10_engine {
    uint4 eval(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    unsigned int c[4], k[2];
    philox_block p;
    while (std::scanf("%u %u %u %u %u %u", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        uint4 r = p.eval(uint4{c[0], c[1], c[2], c[3]}, uint2{k[0], k[1]});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
