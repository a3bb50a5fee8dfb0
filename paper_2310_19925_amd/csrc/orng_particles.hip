// Parallel micro-streams for statistical testing of parallel streams (paper
// section 5.2, after the procedure it cites): particle p draws a micro-stream
// of `draws` words per iteration from its own stream, keyed as in the paper's
// example (seed = seed0 + p, counter = ctr0 + t); the micro-streams of an
// iteration are concatenated in particle order and the iterations follow one
// another:
//   out[(t * n_particles + p) * draws + k] = word k of stream (seed0 + p, ctr0 + t)
// Word k of a stream is the same word orng_fill returns at position k.
//
// Two schedules:
// - flat (Philox4x32, both Threefry4x32 forms and Squares64; micro-streams of
//   at most four words, at least 1024 particles, a 16-byte aligned output):
//   workgroup w makes the 1024 (iteration, particle) slots 1024 w .. 1024 w +
//   1023 of the output order, four per thread, each with its own key
//   schedule, and stores its 4096 * draws contiguous bytes in 16-byte chunks
//   (short-lived workgroups of independent slots, where the lane schedule
//   keeps long-lived lanes with a key schedule each).  Measured against the
//   lane schedule on 16,000 x 3 x 22,369 words, the
//   flat one is 17-18% faster for the Threefry4x32 forms and 2% for Philox4x32
//   and Squares64, and 2-7% slower for the other generators (the same kernel
//   built for them), which keep the lane schedule.
// - lane per particle (any other shape): a lane forms its key schedule once
//   (it depends only on the seed) and runs a chunk of iterations; the wave's
//   micro-streams of an iteration are contiguous in the output and are stored
//   through LDS.  Iterations are cut into chunks so that a few thousand
//   particles still fill the device with many workgroups.
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
    uint32_t n_wgs;         // workgroups with work (the grid may hold a few more)
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
    const uint32_t b = flat_block();
    if (b >= a.n_wgs) return;  // beyond the last workgroup of a two-row grid
    const uint32_t xb = b % a.xblocks, tb = b / a.xblocks;
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

struct FlatArgs {
    uint32_t *out;          // 16-byte aligned
    uint64_t seed0;
    uint32_t n_particles;   // >= FLAT_SLOTS
    uint32_t ctr0;
    uint32_t n_full;        // workgroups with FLAT_SLOTS slots; one more holds the tail
    uint32_t tail;          // slots of the last workgroup when n_iters * n_particles
                            // is not a multiple of FLAT_SLOTS (0 otherwise)
};

constexpr uint32_t FLAT_SLOTS = 1024;  // slots per workgroup (256 threads, four each)

// Slot j of a workgroup whose first slot is (iteration t0, particle p0):
// its DT words into the workgroup's LDS staging area.
template <int G, int DT>
__device__ __forceinline__ void flat_slot(const FlatArgs &a, uint32_t t0, uint32_t p0, uint32_t j,
                                          uint32_t *lds) {
    // p0 < n_particles and j < 1024 <= n_particles: at most one wrap
    uint32_t p = p0 + j, t = t0;
    if (p >= a.n_particles) { p -= a.n_particles; ++t; }
    const uint32_t ctr = a.ctr0 + t;
    const KeySched ks = make_keysched(a.seed0 + p);
    uint32_t w[4];
    counter_block<G>(0, ctr, ks, w);
#pragma unroll
    for (int k = 0; k < DT; ++k) lds[j * DT + k] = w[k];
}

template <int G, int DT>
__global__ __launch_bounds__(256) void k_particles_flat(FlatArgs a) {
    static_assert(DT >= 1 && DT <= 4, "one block of four words per slot");
    static_assert(!tyche_like(G), "counter-based generators only");
    __shared__ __align__(16) uint32_t lds[FLAT_SLOTS * DT];
    const uint32_t b = flat_block();
    if (b > a.n_full || (b == a.n_full && a.tail == 0)) return;  // past the last workgroup
    const uint64_t s0 = (uint64_t)b * FLAT_SLOTS;
    // the slot count from two 32-bit kernel arguments: a clamp of the 64-bit
    // remainder (n_slots - s0 against FLAT_SLOTS) compiled to a select on a
    // stale scalar condition code with this toolchain and gave the last
    // workgroup FLAT_SLOTS slots
    const uint32_t ns = b < a.n_full ? FLAT_SLOTS : a.tail;
    // s0 = t0 * n_particles + p0 (uniform: one scalar division per workgroup)
    const uint64_t t0 = s0 / a.n_particles;
    const uint32_t p0 = (uint32_t)(s0 - t0 * a.n_particles);
    if (ns == FLAT_SLOTS) {
        // every workgroup but the last: the four slots of a thread are
        // independent and unconditional, so their rounds interleave
#pragma unroll
        for (uint32_t q = 0; q < FLAT_SLOTS / 256; ++q)
            flat_slot<G, DT>(a, (uint32_t)t0, p0, threadIdx.x + 256u * q, lds);
    } else {
        for (uint32_t j = threadIdx.x; j < ns; j += 256)
            flat_slot<G, DT>(a, (uint32_t)t0, p0, j, lds);
    }
    __syncthreads();
    const uint32_t nw = ns * DT;
    uint32_t *o = a.out + s0 * DT;
#pragma unroll
    for (uint32_t r = 0; r < DT; ++r) {
        const uint32_t c = 4u * (threadIdx.x + 256u * r);  // first word of this chunk
        if (c + 4 <= nw) {
            *reinterpret_cast<uint4 *>(o + c) = *reinterpret_cast<const uint4 *>(lds + c);
        } else {
            for (uint32_t k = c; k < nw; ++k) o[k] = lds[k];  // the last workgroup's tail
        }
    }
}

}  // namespace orng

using namespace orng;

// The flat schedule's kernel for a generator that takes it, else nullptr.
template <int DT>
static void *flat_kernel(int gen) {
    switch (gen) {
    case G_PHILOX: return reinterpret_cast<void *>(&k_particles_flat<G_PHILOX, DT>);
    case G_TF4X32: return reinterpret_cast<void *>(&k_particles_flat<G_TF4X32, DT>);
    case G_TF4X32_13: return reinterpret_cast<void *>(&k_particles_flat<G_TF4X32_13, DT>);
    case G_SQUARES64: return reinterpret_cast<void *>(&k_particles_flat<G_SQUARES64, DT>);
    default: return nullptr;
    }
}

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
    const uint64_t n_slots = (uint64_t)n_particles * n_iters;
    const uint64_t flat_grid = (n_slots + FLAT_SLOTS - 1) / FLAT_SLOTS;
    void *flat = draws == 1 ? flat_kernel<1>(gen)
               : draws == 2 ? flat_kernel<2>(gen)
               : draws == 3 ? flat_kernel<3>(gen)
               : draws == 4 ? flat_kernel<4>(gen) : nullptr;
    // (the flat kernel's p0 + j stays below 2^32 only when n_particles does not
    // come within FLAT_SLOTS of it)
    if (flat && n_particles >= FLAT_SLOTS && n_particles <= 0xFFFFFFFFu - FLAT_SLOTS &&
        flat_grid <= 0xFFFF0000ull &&
        (reinterpret_cast<uintptr_t>(d_out) & 15u) == 0) {
        FlatArgs f;
        f.out = static_cast<uint32_t *>(d_out);
        f.seed0 = seed0;
        f.n_particles = n_particles;
        f.n_full = (uint32_t)(n_slots / FLAT_SLOTS);
        f.tail = (uint32_t)(n_slots % FLAT_SLOTS);
        f.ctr0 = ctr0;
        void *args[] = {&f};
        const Grid2 g = grid_2d(flat_grid);
        const hipError_t e = hipLaunchKernel(flat, dim3(g.x, g.y), dim3(256), args, 0,
                                             static_cast<hipStream_t>(stream));
        if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
        return ORNG_OK;
    }
    PartArgs a;
    a.out = static_cast<uint32_t *>(d_out);
    a.seed0 = seed0;
    a.n_particles = n_particles;
    a.draws = draws;
    a.ctr0 = ctr0;
    a.n_iters = n_iters;
    a.xblocks = blocks_for(n_particles, 256);
    // about 64K workgroups in all, at least one iteration each
    const uint64_t want_tb = std::max<uint64_t>(1, 65536 / a.xblocks);
    a.iters_per_wg = (uint32_t)std::max<uint64_t>(1, (n_iters + want_tb - 1) / want_tb);
    const uint64_t tblocks = (n_iters + a.iters_per_wg - 1) / a.iters_per_wg;
    const uint64_t grid = tblocks * a.xblocks;
    if (grid > 0xFFFF0000ull) return ORNG_ERANGE;
    a.n_wgs = (uint32_t)grid;
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
    const Grid2 g = grid_2d(grid);
    const hipError_t e = hipLaunchKernel(kern, dim3(g.x, g.y), dim3(256), args, 0,
                                         static_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    return ORNG_OK;
}
