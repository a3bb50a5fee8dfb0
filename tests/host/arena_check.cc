// Host check of the server's arena allocator against a model: a granule map
// of the arena.  Every allocation must be the lowest free run that fits
// (first fit), lie inside the arena, not overlap a live range, and the used
// and peak byte counts must match the model after every step.  Built with
// the address and undefined-behaviour sanitizers by the test-suite.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2310_19925_amd/csrc/orng_arena.hpp"

static int fail(const char *what, unsigned long long step) {
    std::printf("FAIL %s at step %llu\n", what, step);
    return 1;
}

int main(int argc, char **argv) {
    const unsigned long long steps = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 200000;
    const uint64_t G = 256, granules = 4096;
    orng::Arena a;
    a.init(granules * G + 100);  // a ragged size is cut down to whole granules
    if (a.size() != granules * G) return fail("size", 0);
    std::vector<char> busy(granules, 0);
    struct Live { uint64_t off, bytes; };
    std::vector<Live> live;
    std::mt19937_64 rng(2310);
    uint64_t used = 0, peak = 0;
    for (unsigned long long s = 0; s < steps; ++s) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            // sizes from one byte to a quarter of the arena, skewed small
            const uint64_t bytes = 1 + (rng() % (1ull << (rng() % 19)));
            const uint64_t need = (bytes + G - 1) / G;
            // model: the lowest run of `need` free granules
            uint64_t first = granules, run = 0;
            for (uint64_t g = 0; g < granules; ++g) {
                run = busy[g] ? 0 : run + 1;
                if (run == need) { first = g + 1 - need; break; }
            }
            uint64_t off = ~0ull;
            const bool ok = a.alloc(bytes, &off);
            if (ok != (first < granules)) return fail("alloc success", s);
            if (!ok) continue;
            if (off != first * G) return fail("first fit", s);
            for (uint64_t g = first; g < first + need; ++g) busy[g] = 1;
            live.push_back({off, bytes});
            used += need * G;
            peak = std::max(peak, used);
        } else {
            const size_t k = rng() % live.size();
            const Live l = live[k];
            live[k] = live.back();
            live.pop_back();
            a.release(l.off, l.bytes);
            const uint64_t need = (l.bytes + G - 1) / G;
            for (uint64_t g = l.off / G; g < l.off / G + need; ++g) {
                if (!busy[g]) return fail("double free in model", s);
                busy[g] = 0;
            }
            used -= need * G;
        }
        if (a.used() != used) return fail("used bytes", s);
        if (a.peak() != peak) return fail("peak bytes", s);
    }
    // everything released: the arena is one free range again
    for (const Live &l : live) a.release(l.off, l.bytes);
    uint64_t off = 1;
    if (!a.alloc(granules * G, &off) || off != 0) return fail("coalescing", steps);
    std::printf("OK %llu steps\n", steps);
    return 0;
}
