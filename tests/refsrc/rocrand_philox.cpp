// Host-side reference outputs of Philox4x32-10 taken from rocRAND's engine
// (an independent implementation of Salmon et al., SC'11).  Reads lines
// "c0 c1 c2 c3 k0 k1" (hex) from stdin and prints the four output words (hex).
// Built with "hipcc -x hip"; it makes no device call.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

// Exposes the engine's block function so that any 128-bit counter can be given.
struct philox_block : rocrand_device::philox4x32_10_engine {
    uint4 at(uint4 counter, uint2 key) { return ten_rounds(counter, key); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    philox_block e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr;
        ctr.x = c0; ctr.y = c1; ctr.z = c2; ctr.w = c3;
        uint2 key;
        key.x = k0; key.y = k1;
        uint4 v = e.at(ctr, key);
        std::printf("%08x %08x %08x %08x\n", v.x, v.y, v.z, v.w);
    }
    return 0;
}
