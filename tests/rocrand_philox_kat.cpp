// rocrand_philox_kat.cpp -- test helper (not part of the library or the
// oracle): evaluates Philox4x32-10 with rocRAND's own implementation
// (philox4x32_10_engine from the ROCm headers, built for the host), as an
// independent known-answer source for the oracle's generator.
//
// stdin: lines "c0 c1 c2 c3 k0 k1" (hex words); stdout: "r0 r1 r2 r3".
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

// The engine keeps its ten-round block function protected; a derived class
// exposes it for raw (counter, key) evaluation.
struct RawPhilox : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main()
{
    RawPhilox p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const uint4 r = p.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
