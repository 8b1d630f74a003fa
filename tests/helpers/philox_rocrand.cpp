// Test helper: evaluates rocRAND's Philox4x32-10 block function on the host,
// as an implementation independent of the oracle's, to pin it.
// stdin : lines "c0 c1 c2 c3 k0 k1" (hex)   stdout: "r0 r1 r2 r3" (hex)
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

struct PhiloxBlock : rocrand_device::philox4x32_10_engine {
    static uint4 eval(uint4 ctr, uint2 key) {
        PhiloxBlock p;
        return p.ten_rounds(ctr, key);
    }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = PhiloxBlock::eval(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
