// Host check of the request-record helpers shared by the batched and served
// paths (host-only header): validation, integer-range bounds and the output
// alignment class.  Draws requests whose fields sit on and around every
// boundary the checks test (generator and distribution ids, the 32-bit seed
// limit of Philox2x32, the per-distribution sample limit, lo/hi order and
// extremes, pointer alignment) and writes one row per request for the
// test-suite to compare with its own model.  Built with the address and
// undefined-behaviour sanitizers by the test-suite.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../../paper_2310_19925_amd/csrc/orng_host.hpp"

int main(int argc, char **argv) {
    if (argc < 3) return 2;
    const unsigned long long n = std::strtoull(argv[1], nullptr, 10);
    FILE *f = std::fopen(argv[2], "wb");
    if (!f) return 2;
    std::mt19937_64 rng(19925);
    auto pick = [&](const uint64_t *v, size_t k) { return v[rng() % k]; };
    const uint64_t seeds[] = {0, 1, 0xFFFFFFFFull, 0x100000000ull, ~0ull};
    const uint64_t edges[] = {0, 1, 3, 1ull << 31, (1ull << 31) - 1, (1ull << 31) + 1,
                              1ull << 32, (1ull << 32) - 1, (1ull << 32) + 1, ~0ull};
    const int32_t bounds[] = {INT32_MIN, INT32_MIN + 1, -1, 0, 1, INT32_MAX - 1, INT32_MAX};
    for (unsigned long long i = 0; i < n; ++i) {
        orng_req_t r{};
        r.gen = (uint32_t)(rng() % 12);
        r.dist = (uint32_t)(rng() % 8);
        r.flags = (rng() % 16 == 0) ? 1u : 0u;
        r.seed = (rng() % 2) ? pick(seeds, 5) : rng();
        r.ctr = (uint32_t)rng();
        r.offset = (rng() % 2) ? pick(edges, 10) : rng() % 4096;
        r.n = (rng() % 2) ? pick(edges, 10) : rng() % 4096;
        if (rng() % 2 == 0 && r.offset <= (1ull << 32)) {  // end exactly at or next to a limit
            const uint64_t lim = (rng() % 2) ? (1ull << 31) : (1ull << 32);
            const uint64_t end = lim - 1 + rng() % 3;
            r.n = end >= r.offset ? end - r.offset : 0;
        }
        r.lo =(rng() % 2) ? bounds[rng() % 7] : (int32_t)(rng() % 2001) - 1000;
        r.hi = (rng() % 2) ? bounds[rng() % 7] : (int32_t)(rng() % 2001) - 1000;
        const uint64_t addr = (rng() % 8 == 0) ? 0 : 0x7f0000000000ull + (rng() % 64);
        r.out = reinterpret_cast<void *>(addr);
        const int rc = orng::validate_request(r);
        uint32_t lo = 0, rr = 0, delta = 0;
        orng::range_bounds(r, &lo, &rr);
        if (rc == ORNG_OK && r.n > 0) delta = orng::output_delta(r, r.out);
        const uint64_t row[13] = {r.gen,  r.dist, r.flags, r.seed, r.ctr,          r.offset,
                                  r.n,    addr,   (uint64_t)(uint32_t)r.lo,
                                  (uint64_t)(uint32_t)r.hi, (uint64_t)(int64_t)rc, lo,
                                  ((uint64_t)rr << 32) | delta};
        if (std::fwrite(row, sizeof row, 1, f) != 1) return 2;
    }
    std::fclose(f);
    std::printf("OK %llu requests\n", n);
    return 0;
}
