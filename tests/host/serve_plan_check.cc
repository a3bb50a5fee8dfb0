// Host check of the serving loop's scheduling rules (host-only header):
//  - tiling: for random generators, span lengths, workgroup sizes and word
//    ranges anywhere in a stream, the tiles cover the range, start at or
//    before its first word, and none of them lies wholly past its end;
//  - step planning: random request sets, admitted over time, are planned
//    step by step until every tile is scheduled; every step must take a
//    prefix of the requests that still have tiles (admission order), at
//    least one tile and at most what is left of each, at most half a step per
//    request unless one tile is larger, and overshoot the step's budget by
//    less than one tile of its last pick; every tile is scheduled once.
// Built with the address and undefined-behaviour sanitizers by the test-suite.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2310_19925_amd/csrc/orng_serve_plan.hpp"

using namespace orng;

static int fail(const char *what, unsigned long long i) {
    std::printf("FAIL %s at %llu\n", what, i);
    return 1;
}

struct Req {
    uint64_t tiles_total, tiles_sched, tile_words;
};

int main(int argc, char **argv) {
    const unsigned long long rounds = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 2000;
    std::mt19937_64 rng(2310);
    // tiling
    for (unsigned long long i = 0; i < 200000; ++i) {
        const int gen = (int)(rng() % NGEN);
        const uint32_t unroll = tyche_like(gen) ? 64 : (uint32_t)(4 + rng() % 29);
        const uint32_t wg = 64u << (rng() % 3);
        const uint64_t p0 = rng() % (1ull << 32);
        const uint64_t room = (1ull << 32) - p0;
        const uint64_t nw = 1 + (rng() % 2 ? rng() % std::min<uint64_t>(room, 1ull << (rng() % 33))
                                           : rng() % room);
        if (nw > room) continue;
        const ReqTiling t = tile_request(gen, unroll, wg, p0, nw);
        const uint64_t span_words = span_blocks(gen, unroll) * 4, W = wg / 64;
        if (t.tile_words != span_words * W) return fail("tile size", i);
        const uint64_t start = t.first_span * span_words;
        const uint64_t end = start + t.tiles_total * t.tile_words;  // one past the last tile
        if (start > p0 || p0 - start >= span_words) return fail("first span", i);
        if (end < p0 + nw) return fail("tiles cover the range", i);
        if (t.tiles_total == 0 || end - t.tile_words >= p0 + nw) return fail("no empty tile", i);
    }
    // step planning
    unsigned long long steps_total = 0;
    for (unsigned long long rd = 0; rd < rounds; ++rd) {
        const uint64_t step_words = 1ull << (12 + rng() % 19);
        std::vector<Req> store;
        store.reserve(400);
        std::vector<Req *> active;
        uint64_t want_tiles = 0, got_tiles = 0;
        const size_t nreq = 1 + rng() % 300;
        size_t admitted = 0;
        for (int step = 0;; ++step) {
            // a few arrivals before each step
            for (size_t a = rng() % 6; a > 0 && admitted < nreq; --a, ++admitted) {
                Req r;
                r.tile_words = 2048ull << (rng() % 6);
                r.tiles_total = 1 + (rng() % (1ull << (rng() % 14)));
                r.tiles_sched = 0;
                store.push_back(r);
                active.push_back(&store.back());
                want_tiles += r.tiles_total;
            }
            bool any_left = false;
            for (Req *r : active) any_left |= r->tiles_total > r->tiles_sched;
            if (!any_left && admitted == nreq) break;
            if (step > 1000000) return fail("termination", rd);
            const uint64_t cap = std::max<uint64_t>(step_words / 2, 1);
            size_t next = 0;  // index into active of the next request expected to get tiles
            uint64_t words = 0, last_tw = 0;
            bool bad = false;
            std::vector<std::pair<Req *, uint64_t>> picks;
            plan_step(active, step_words, [&](Req *r, uint64_t k) { picks.push_back({r, k}); });
            for (auto &pk : picks) {
                Req *r = pk.first;
                const uint64_t k = pk.second, left = r->tiles_total - r->tiles_sched;
                // every request between the previous pick and this one has nothing left
                while (next < active.size() && active[next] != r) {
                    if (active[next]->tiles_total > active[next]->tiles_sched) bad = true;
                    ++next;
                }
                if (next == active.size()) return fail("pick outside the active list", rd);
                ++next;
                if (k < 1 || k > left) return fail("pick size", rd);
                if (k > 1 && k * r->tile_words > cap) return fail("half a step per request", rd);
                words += k * r->tile_words;
                last_tw = r->tile_words;
            }
            if (bad) return fail("admission order", rd);
            if (any_left && picks.empty()) return fail("progress", rd);
            if (!picks.empty() && words >= step_words + last_tw) return fail("budget", rd);
            // a step stops early only when its budget is spent
            if (words < step_words)
                for (size_t j = next; j < active.size(); ++j)
                    if (active[j]->tiles_total > active[j]->tiles_sched)
                        return fail("budget left unused", rd);
            for (auto &pk : picks) {
                pk.first->tiles_sched += pk.second;
                got_tiles += pk.second;
            }
            ++steps_total;
        }
        if (got_tiles != want_tiles) return fail("every tile once", rd);
        for (Req *r : active)
            if (r->tiles_sched != r->tiles_total) return fail("request finished", rd);
    }
    std::printf("OK %llu rounds %llu steps\n", rounds, steps_total);
    return 0;
}
