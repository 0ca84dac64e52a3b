// Host-side reference for Philox4x32-10 taken from rocRAND's engine (an
// implementation independent of both the oracle and the HIP library).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) on stdin, prints the 4 output
// words per line.  Test infrastructure only.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return this->ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Engine e;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = e.rounds(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
