// Parallel micro-streams for statistical testing of parallel streams (paper
// section 5.2, after the procedure it cites): particle p draws a micro-stream
// of `draws` words per iteration from its own stream, keyed as in the paper's
// example (seed = seed0 + p, counter = ctr0 + t); the micro-streams of an
// iteration are concatenated in particle order and the iterations follow one
// another:
//   out[(t * n_particles + p) * draws + k] = word k of stream (seed0 + p, ctr0 + t)
// Word k of a stream is the same word orng_fill returns at position k.
//
// One lane per particle forms its key schedule once (it depends only on the
// seed) and runs a chunk of iterations; the wave's micro-streams of an
// iteration are contiguous in the output and are stored through LDS.
// Iterations are cut into chunks so that a few thousand particles still fill
// the device with many workgroups.
#include "../../include/orng.h"
#include "orng_device.hpp"
#include "orng_internal.hpp"

#include <algorithm>

namespace orng {

struct PartArgs {
    uint32_t *out;
    uint64_t seed0;
    uint32_t n_particles, draws, ctr0, n_iters;
    uint32_t xblocks;       // workgroups across the particles
    uint32_t iters_per_wg;  // iterations per workgroup
};

// A wave's 64 particles own 64 * draws consecutive output words per
// iteration.  Each lane writes its micro-stream into the wave's LDS slice,
// then the wave stores the slice with `draws` instructions of 64 consecutive
// words (fully coalesced whatever draws is and however the slice is aligned).
// A wave executes its LDS operations in order, so a scheduling barrier is
// the only synchronization needed between writing and reading the slice.
// DT: the micro-stream length when fixed at compile time (3, the section 5.2
// shape: fully unrolled, the three LDS reads issued together), 0 for any.
template <int G, int DT>
__global__ __launch_bounds__(256) void k_particles(PartArgs a) {
    __shared__ uint32_t lds[256 * 16];
    const uint32_t xb = blockIdx.x % a.xblocks, tb = blockIdx.x / a.xblocks;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t pw0 = xb * 256 + wave * 64;  // first particle of the wave
    if (pw0 >= a.n_particles) return;           // whole wave past the end
    const uint32_t nvalid = std::min(64u, a.n_particles - pw0);
    const uint32_t p = pw0 + lane;
    const bool live = lane < nvalid;
    uint32_t *slice = lds + wave * 64 * 16;
    const uint32_t t0 = tb * a.iters_per_wg;
    const uint32_t t1 = std::min(a.n_iters, t0 + a.iters_per_wg);
    const KeySched ks = make_keysched(a.seed0 + (live ? p : pw0));
    const uint32_t D = DT ? DT : a.draws, nblk = (D + 3) / 4, nwords = nvalid * D;
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t ctr = a.ctr0 + t;
        if (live) {
            for (uint32_t b = 0; b < nblk; ++b) {
                uint32_t w[4];
                if constexpr (tyche_like(G)) {
                    // words 4b..4b+3 of the stream: outputs 0..3 of substream b
                    // (the first tile's layout, as in orng_fill)
                    TycheT<G == G_TYCHE_I> st;
                    st.seed(ks, b, ctr);
                    st.next4(w);
                } else {
                    counter_block<G>(b, ctr, ks, w);
                }
#pragma unroll
                for (uint32_t k = 0; k < 4; ++k)
                    if (4 * b + k < D) slice[lane * D + 4 * b + k] = w[k];
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t *o = a.out + ((uint64_t)t * a.n_particles + pw0) * D;
        if constexpr (DT != 0) {
            uint32_t v[DT];
#pragma unroll
            for (int i = 0; i < DT; ++i) v[i] = slice[lane + 64 * i];
#pragma unroll
            for (int i = 0; i < DT; ++i)
                if (lane + 64 * i < nwords) o[lane + 64 * i] = v[i];
        } else {
            for (uint32_t j = lane; j < nwords; j += 64) o[j] = slice[j];
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace orng

using namespace orng;

extern "C" int orng_particle_streams(int gen, uint64_t seed0, uint32_t n_particles,
                                     uint32_t draws, uint32_t ctr0, uint32_t n_iters,
                                     void *d_out, void *stream) {
    if (gen < ORNG_PHILOX4X32_10 || gen > ORNG_PHILOX2X32 || draws < 1 || draws > 16)
        return ORNG_EINVAL;
    if (n_iters && (uint64_t)ctr0 + n_iters - 1 > 0xFFFFFFFFull) return ORNG_ERANGE;
    if (n_particles && seed0 + (n_particles - 1) < seed0) return ORNG_ERANGE;
    if (n_particles && !seed_ok(gen, seed0 + (n_particles - 1))) return ORNG_ERANGE;
    if (!n_particles || !n_iters) return ORNG_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 3u)) return ORNG_EINVAL;
    PartArgs a;
    a.out = static_cast<uint32_t *>(d_out);
    a.seed0 = seed0;
    a.n_particles = n_particles;
    a.draws = draws;
    a.ctr0 = ctr0;
    a.n_iters = n_iters;
    a.xblocks = (n_particles + 255) / 256;
    // about 64K workgroups in all, at least one iteration each
    const uint64_t want_tb = std::max<uint64_t>(1, 65536 / a.xblocks);
    a.iters_per_wg = (uint32_t)std::max<uint64_t>(1, (n_iters + want_tb - 1) / want_tb);
    const uint64_t tblocks = (n_iters + a.iters_per_wg - 1) / a.iters_per_wg;
    const uint64_t grid = tblocks * a.xblocks;
    if (grid > 0x7FFFFFFFull) return ORNG_ERANGE;
    void *kern = nullptr;
#define ORNG_PK(G) (draws == 3 ? reinterpret_cast<void *>(&k_particles<G, 3>) \
                               : reinterpret_cast<void *>(&k_particles<G, 0>))
    switch (gen) {
    case G_PHILOX: kern = ORNG_PK(G_PHILOX); break;
    case G_TF4X32: kern = ORNG_PK(G_TF4X32); break;
    case G_TF2X64: kern = ORNG_PK(G_TF2X64); break;
    case G_SQUARES: kern = ORNG_PK(G_SQUARES); break;
    case G_TF4X32_13: kern = ORNG_PK(G_TF4X32_13); break;
    case G_TF2X64_13: kern = ORNG_PK(G_TF2X64_13); break;
    case G_TYCHE_I: kern = ORNG_PK(G_TYCHE_I); break;
    case G_SQUARES64: kern = ORNG_PK(G_SQUARES64); break;
    case G_PHILOX2X32: kern = ORNG_PK(G_PHILOX2X32); break;
    default: kern = ORNG_PK(G_TYCHE); break;
    }
#undef ORNG_PK
    void *args[] = {&a};
    const hipError_t e = hipLaunchKernel(kern, dim3((uint32_t)grid), dim3(256), args, 0,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    return ORNG_OK;
}
