// Cross-check driver: evaluates rocRAND's own Philox4x32-10, Threefry4x32-20
// and Threefry2x64-20 block functions on the host, for (key, counter) pairs
// read from stdin, so the test-suite can compare the oracle against an
// implementation it did not write.  Built host-only with hipcc; rocRAND is
// used through its public headers, nothing of it is copied here.
//
// Input lines:  P k0 k1 c0 c1 c2 c3        (32-bit words, decimal)
//               T k0 k1 k2 k3 c0 c1 c2 c3
//               S k0 k1 c0 c1              (64-bit words, decimal)
// Output: one line of decimal output words per input line.
#include <rocrand/rocrand_philox4x32_10.h>
#include <rocrand/rocrand_threefry2x64_20.h>
#include <rocrand/rocrand_threefry4x32_20.h>

#include <cstdio>

namespace {
// expose the block functions, which rocRAND keeps protected
struct PhiloxBlock : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
struct Tf4Block : rocrand_device::threefry4x32_20_engine {
    static uint4 block(uint4 c, uint4 k) { return threefry_rounds(c, k); }
};
struct Tf2Block : rocrand_device::threefry2x64_20_engine {
    static ulonglong2 block(ulonglong2 c, ulonglong2 k) { return threefry_rounds(c, k); }
};
} // namespace

int main() {
    char tag;
    PhiloxBlock ph;
    while (std::scanf(" %c", &tag) == 1) {
        if (tag == 'P') {
            unsigned k0, k1, c0, c1, c2, c3;
            if (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) != 6) return 2;
            uint4 r = ph.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
            std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
        } else if (tag == 'T') {
            unsigned k[4], c[4];
            if (std::scanf("%u %u %u %u %u %u %u %u", &k[0], &k[1], &k[2], &k[3], &c[0], &c[1],
                           &c[2], &c[3]) != 8)
                return 2;
            uint4 r = Tf4Block::block(uint4{c[0], c[1], c[2], c[3]}, uint4{k[0], k[1], k[2], k[3]});
            std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
        } else if (tag == 'S') {
            unsigned long long k0, k1, c0, c1;
            if (std::scanf("%llu %llu %llu %llu", &k0, &k1, &c0, &c1) != 4) return 2;
            ulonglong2 r = Tf2Block::block(ulonglong2{c0, c1}, ulonglong2{k0, k1});
            std::printf("%llu %llu\n", r.x, r.y);
        } else {
            return 3;
        }
    }
    return 0;
}
