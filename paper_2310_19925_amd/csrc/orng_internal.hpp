// Internal declarations shared by the library's translation units (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "orng_device.hpp"

namespace orng {

// Launch knobs.  0 means "choose automatically".
struct LaunchCfg {
    uint32_t wg_size;   // threads per workgroup (multiple of 64, <= 512)
    uint32_t unroll;    // blocks per lane per span (U); span = 64*U blocks
    uint32_t max_wgs;   // cap on workgroups (grid-stride beyond it)
    uint32_t nontemporal;  // 1: nontemporal stores, 2: normal stores, 0: auto
};

// Tuned launch parameters of one (generator, distribution) pair.
struct Tuned {
    uint32_t wg_size;      // fill: threads per workgroup
    uint32_t unroll;       // fill: blocks per lane per span
    uint32_t max_wgs;      // fill: grid cap (0: one wave per span)
    uint32_t nontemporal;  // fill: 1 nontemporal, 2 ordinary stores
    uint32_t b_wg_size;    // batched: threads per workgroup
    uint32_t b_unroll;     // batched: blocks per lane per tile
    uint32_t b_chunk;      // batched: tiles claimed per queue access
    uint32_t b_wgs_per_cu; // batched: persistent workgroups per CU
};
Tuned tuned_fill(int gen, int dist);
void set_tuned(int gen, int dist, const Tuned &t);
// launch row of the integer-range fill (wg_size, unroll, max_wgs used)
Tuned tuned_range(int gen);
void set_tuned_range(int gen, const Tuned &t);
int load_tune_cache(const char *path);
int save_tune_cache(const char *path);

// Current launch configuration (thread-safe copy).
LaunchCfg launch_cfg();
void set_launch_cfg(const LaunchCfg &c);

// Per-thread last HIP error.
void set_hip_error(hipError_t e);
int last_hip_error();

// Launchers; arguments already validated.  Return hipError_t.  launch_fill
// takes offset and per_stream in stream words (positions).
hipError_t launch_fill(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                       uint64_t offset, uint64_t per_stream, void *out, hipStream_t s);
hipError_t launch_walk(uint64_t seed, uint32_t ctr0, uint32_t n, uint32_t dim, uint64_t step0,
                       uint32_t n_steps, float sigma, float *pos, double *msd,
                       uint32_t msd_every, hipStream_t s);

int device_cu_count();

}  // namespace orng
