// Prints rocRAND's Philox4x32-10 block function for counters/keys read from
// stdin ("c0 c1 c2 c3 k0 k1" per line, decimal).  Host code only: it is the
// library cross-check for the oracle's own Philox implementation.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Block : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Block eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 o = eng.ten_rounds(c, k);
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
