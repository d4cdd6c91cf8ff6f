// Prints Philox4x32-10 outputs computed by rocRAND's host-callable engine for counters
// and keys read from stdin (one "c0 c1 c2 c3 k0 k1" line each, hexadecimal).  Used by
// the test-suite as an independent library check of the oracle's Philox.  Host code
// only: no GPU call is made.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

// The engine's ten-round block function is protected; expose it for direct counters.
struct probe_engine : rocrand_device::philox4x32_10_engine
{
    uint4 block(uint4 counter, uint2 key) { return this->ten_rounds(counter, key); }
};

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    probe_engine eng;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
