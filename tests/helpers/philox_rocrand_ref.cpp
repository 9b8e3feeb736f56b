// Test helper (host only): Philox4x32-10 from the rocRAND header, used as an
// independent reference for the oracle's and the GPU library's generators.
// Reads "c0 c1 c2 c3 k0 k1" hex lines on stdin, prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Engine e;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
