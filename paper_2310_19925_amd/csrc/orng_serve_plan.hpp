// Scheduling rules of the serving loop that need no device: how an admitted
// request is cut into step tiles, and how a step's word budget is shared out
// among the admitted requests.  Plain C++ with no HIP dependency, so that the
// rules can be built and checked on the host alone.
#pragma once

#include <stdint.h>

#include <algorithm>

#include "orng_host.hpp"

namespace orng {

constexpr uint32_t kServeWg = 128;  // threads per workgroup of a step: W = 2 spans per tile

// Blocks per lane for a served request of n stream words on a device with
// `cus` compute units: 4 for small requests, growing with the request to 32
// (long spans cut the per-span setup that dominates a saturated step).
inline uint32_t serve_unroll(uint64_t n, int cus) {
    const uint64_t words_per_unroll = (uint64_t)cus * kServeWg * 4;
    return (uint32_t)std::min<uint64_t>(32, std::max<uint64_t>(4, n / words_per_unroll));
}

// A request's tiling: spans of span_blocks(gen, unroll) blocks numbered in
// the stream's block space, W = wg / 64 consecutive spans per tile.
struct ReqTiling {
    uint64_t first_span;   // span of the request's first stream word
    uint64_t tiles_total;  // tiles that cover every span the request touches
    uint64_t tile_words;   // stream words of a whole tile
};

// Tiling of stream words p0 .. p0 + nw - 1 (nw > 0) of a generator.
inline ReqTiling tile_request(int gen, uint32_t unroll, uint32_t wg, uint64_t p0, uint64_t nw) {
    const uint64_t sbk = span_blocks(gen, unroll);
    const uint64_t W = wg / 64;
    const uint64_t fb = p0 / 4, lb = (p0 + nw - 1) / 4;
    ReqTiling t;
    t.first_span = fb / sbk;
    t.tiles_total = (lb / sbk - t.first_span + 1 + W - 1) / W;
    t.tile_words = sbk * 4 * W;
    return t;
}

// Share of the next step: the budget of step_words goes to the requests in
// admission order (`active`, pointers to records with tiles_total,
// tiles_sched and tile_words), each taking its remaining tiles up to half a
// step, and at least one tile, until the budget is spent; requests with no
// tiles left are passed over.  Results then complete in arrival order, so a
// loaded server frees arena space (and admits the next requests) as early as
// possible; under light load every ready request fits into one step.
// visit(request, tiles) is called for each pick, in order.  The words picked
// exceed step_words by less than one tile of the last pick.
template <class ReqPtrRange, class Visit>
void plan_step(const ReqPtrRange &active, uint64_t step_words, Visit visit) {
    uint64_t budget = step_words;
    const uint64_t cap = std::max<uint64_t>(step_words / 2, 1);
    for (auto *r : active) {
        if (!budget) break;
        const uint64_t left = r->tiles_total - r->tiles_sched;
        if (!left) continue;
        uint64_t k = std::max<uint64_t>(1, std::min(budget, cap) / r->tile_words);
        k = std::min(k, left);
        visit(r, k);
        budget -= std::min(budget, k * r->tile_words);
    }
}

}  // namespace orng
