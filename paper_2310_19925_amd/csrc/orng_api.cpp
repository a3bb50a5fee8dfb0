// C-ABI entry points: argument validation, error mapping, launch knobs.
#include <cmath>
#include <mutex>

#include "../../include/orng.h"
#include "orng_internal.hpp"

namespace orng {

static std::mutex g_cfg_mu;
static LaunchCfg g_cfg = {0, 0, 0, 0};
static thread_local int t_last_hip = 0;

LaunchCfg launch_cfg() {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    return g_cfg;
}

void set_launch_cfg(const LaunchCfg &c) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    g_cfg = c;
}

void set_hip_error(hipError_t e) { t_last_hip = (int)e; }
int last_hip_error() { return t_last_hip; }

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

static int hip_status(hipError_t e) {
    if (e == hipSuccess) return ORNG_OK;
    set_hip_error(e);
    return ORNG_EHIP;
}

static bool valid_gen(int g) { return g >= ORNG_PHILOX4X32_10 && g <= ORNG_PHILOX2X32; }
static bool valid_dist(int d) { return d >= ORNG_U32 && d <= ORNG_F64_NORMAL; }

}  // namespace orng

using namespace orng;

extern "C" {

int orng_fill(int gen, int dist, uint64_t seed, uint32_t ctr, uint64_t offset, uint64_t n,
              void *d_out, void *stream) {
    if (!valid_gen(gen) || !valid_dist(dist) || !seed_ok(gen, seed)) return ORNG_EINVAL;
    const uint64_t k = words_per_sample(dist), lim = sample_limit(dist);
    if (offset > lim || n > lim - offset) return ORNG_ERANGE;
    if (n == 0) return ORNG_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (4 * k - 1))) return ORNG_EINVAL;
    return hip_status(launch_fill(gen, dist, seed, ctr, 1, offset * k, n * k, d_out,
                                  static_cast<hipStream_t>(stream)));
}

int orng_fill_multi(int gen, int dist, uint64_t seed, uint32_t ctr0, uint32_t n_streams,
                    uint64_t offset, uint64_t per_stream, void *d_out, void *stream) {
    if (!valid_gen(gen) || !valid_dist(dist) || !seed_ok(gen, seed)) return ORNG_EINVAL;
    const uint64_t k = words_per_sample(dist), lim = sample_limit(dist);
    if (offset > lim || per_stream > lim - offset) return ORNG_ERANGE;
    if (n_streams && (uint64_t)ctr0 + n_streams - 1 > 0xFFFFFFFFull) return ORNG_ERANGE;
    if (n_streams == 0 || per_stream == 0) return ORNG_OK;
    if (!d_out || (reinterpret_cast<uintptr_t>(d_out) & (4 * k - 1))) return ORNG_EINVAL;
    return hip_status(launch_fill(gen, dist, seed, ctr0, n_streams, offset * k, per_stream * k,
                                  d_out, static_cast<hipStream_t>(stream)));
}

int orng_brownian(uint64_t seed, uint32_t ctr0, uint32_t n_particles, uint32_t dim,
                  uint64_t step0, uint32_t n_steps, float dt, float D, float *d_pos,
                  double *d_msd, uint32_t msd_every, void *stream) {
    if (dim < 1 || dim > 3) return ORNG_EINVAL;
    if (!(dt >= 0.0f) || !(D >= 0.0f) || !std::isfinite(dt) || !std::isfinite(D))
        return ORNG_EINVAL;
    if (step0 > PERIOD || (step0 + n_steps) * (uint64_t)dim > PERIOD) return ORNG_ERANGE;
    if (n_particles && (uint64_t)ctr0 + n_particles - 1 > 0xFFFFFFFFull) return ORNG_ERANGE;
    if (n_particles == 0 || n_steps == 0) return ORNG_OK;
    if (!d_pos || (reinterpret_cast<uintptr_t>(d_pos) & 3u)) return ORNG_EINVAL;
    if (d_msd && (reinterpret_cast<uintptr_t>(d_msd) & 7u)) return ORNG_EINVAL;
    const float sigma = (float)std::sqrt(2.0 * (double)D * (double)dt);
    return hip_status(launch_walk(seed, ctr0, n_particles, dim, step0, n_steps, sigma, d_pos,
                                  d_msd, msd_every, static_cast<hipStream_t>(stream)));
}

int orng_set_launch(const orng_launch_t *cfg) {
    LaunchCfg c = {0, 0, 0, 0};
    if (cfg) {
        if (cfg->wg_size && (cfg->wg_size % 64 || cfg->wg_size > 512)) return ORNG_EINVAL;
        if (cfg->unroll > 64) return ORNG_EINVAL;
        if (cfg->nontemporal > 2) return ORNG_EINVAL;
        c.wg_size = cfg->wg_size;
        c.unroll = cfg->unroll;
        c.max_wgs = cfg->max_wgs;
        c.nontemporal = cfg->nontemporal;
    }
    set_launch_cfg(c);
    return ORNG_OK;
}

int orng_get_launch(orng_launch_t *cfg) {
    if (!cfg) return ORNG_EINVAL;
    const LaunchCfg c = launch_cfg();
    cfg->wg_size = c.wg_size;
    cfg->unroll = c.unroll;
    cfg->max_wgs = c.max_wgs;
    cfg->nontemporal = c.nontemporal;
    return ORNG_OK;
}

const char *orng_strerror(int status) {
    switch (status) {
    case ORNG_OK: return "ok";
    case ORNG_EINVAL: return "invalid argument";
    case ORNG_ERANGE: return "position or counter out of range";
    case ORNG_ENOMEM: return "request exceeds available memory";
    case ORNG_EAGAIN: return "resources temporarily exhausted";
    case ORNG_EBUSY: return "result not ready";
    case ORNG_EHIP: return "HIP runtime error";
    case ORNG_ENOENT: return "no such ticket or object";
    default: return "unknown status";
    }
}

int orng_last_hip_error(void) { return last_hip_error(); }

int orng_version(void) { return 0x000100; }

}  // extern "C"
