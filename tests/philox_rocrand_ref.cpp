// Test helper: evaluates rocRAND's Philox4x32-10 bijection on (counter, key)
// tuples read from stdin, one "c0 c1 c2 c3 k0 k1" line each, and prints the
// four output words.  Used only to pin the oracle's Philox implementation
// against an independent library implementation.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct philox_probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 ctr, uint2 key) { return this->ten_rounds(ctr, key); }
};

int main() {
    philox_probe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 ctr = {c0, c1, c2, c3};
        uint2 key = {k0, k1};
        uint4 o = p.run(ctr, key);
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
