// Cross-check driver: evaluates rocRAND's own Philox4x32-10, Threefry4x32-20
// and Threefry2x64-20 block functions on the host, for (key, counter) pairs
// read from stdin, so the test-suite can compare the oracle against an
// implementation it did not write.  Built host-only with hipcc; rocRAND is
// used through its public headers, nothing of it is copied here.
//
// Input lines:  P k0 k1 c0 c1 c2 c3        (32-bit words, decimal)
//               T k0 k1 k2 k3 c0 c1 c2 c3  (Threefry4x32, 20 rounds)
//               S k0 k1 c0 c1              (Threefry2x64, 20 rounds; 64-bit words)
//               U ... as T, V ... as S     (the same engines with 13 rounds)
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
// rocRAND's engine templates take the round count as a parameter
struct Tf4Block13 : rocrand_device::threefry_engine4_base<uint4, unsigned int, 13> {
    static uint4 block(uint4 c, uint4 k) { return threefry_rounds(c, k); }
};
struct Tf2Block13 : rocrand_device::threefry_engine2_base<ulonglong2, unsigned long long, 13> {
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
        } else if (tag == 'T' || tag == 'U') {
            unsigned k[4], c[4];
            if (std::scanf("%u %u %u %u %u %u %u %u", &k[0], &k[1], &k[2], &k[3], &c[0], &c[1],
                           &c[2], &c[3]) != 8)
                return 2;
            const uint4 cc{c[0], c[1], c[2], c[3]}, kk{k[0], k[1], k[2], k[3]};
            uint4 r = tag == 'T' ? Tf4Block::block(cc, kk) : Tf4Block13::block(cc, kk);
            std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
        } else if (tag == 'S' || tag == 'V') {
            unsigned long long k0, k1, c0, c1;
            if (std::scanf("%llu %llu %llu %llu", &k0, &k1, &c0, &c1) != 4) return 2;
            const ulonglong2 cc{c0, c1}, kk{k0, k1};
            ulonglong2 r = tag == 'S' ? Tf2Block::block(cc, kk) : Tf2Block13::block(cc, kk);
            std::printf("%llu %llu\n", r.x, r.y);
        } else {
            return 3;
        }
    }
    return 0;
}
