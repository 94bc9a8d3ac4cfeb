// Host-side reference words of rocRAND's Philox4x32-10 engine, used only to
// pin the oracle's Philox implementation.  Reads lines "c0 c1 c2 c3 k0 k1"
// (decimal uint32) from stdin and prints the four output words per line.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct PhiloxProbe : rocrand_device::philox4x32_10_engine {
    uint4 words(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    PhiloxProbe p;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
        uint2 k; k.x = k0; k.y = k1;
        uint4 r = p.words(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
