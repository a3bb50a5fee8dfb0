// Internal declarations shared by the library's translation units (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "orng_device.hpp"

namespace orng {

constexpr uint64_t PERIOD = 1ull << 32;

// Launch knobs.  0 means "choose automatically".
struct LaunchCfg {
    uint32_t wg_size;   // threads per workgroup (multiple of 64, <= 512)
    uint32_t unroll;    // blocks per lane per span (U); span = 64*U blocks
    uint32_t max_wgs;   // cap on workgroups (grid-stride beyond it)
    uint32_t nontemporal;  // 1: nontemporal stores, 2: normal stores, 0: auto
};

KeySched make_keysched(uint64_t seed);

// Current launch configuration (thread-safe copy).
LaunchCfg launch_cfg();
void set_launch_cfg(const LaunchCfg &c);

// Per-thread last HIP error.
void set_hip_error(hipError_t e);
int last_hip_error();

// Launchers; arguments already validated.  Return hipError_t.
hipError_t launch_fill(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                       uint64_t offset, uint64_t per_stream, void *out, hipStream_t s);
hipError_t launch_walk(uint64_t seed, uint32_t ctr0, uint32_t n, uint32_t dim, uint64_t step0,
                       uint32_t n_steps, float sigma, float *pos, double *msd,
                       uint32_t msd_every, hipStream_t s);

int device_cu_count();

}  // namespace orng
