// The paper's 2-D Brownian dynamics example (section 4, Fig. 1; the GPU
// benchmark of section 5.1): every particle is one stream, seeded by its id
// and counted by the step, so a step needs no state besides the particle.
//
// The model: each velocity component relaxes at the rate c = gamma / mass and
// takes a uniform kick on [-sqrt(dt), sqrt(dt)); the position integrates the
// velocity.  Per step this library evaluates it as, for each component d of
// (x, y), with u_d the double made from words 2d, 2d+1 of Philox stream
// (pid, step0 + s):
//   v_d <- a v_d + (u_d - 1/2) w        a = 1 - c dt,  w = 2 sqrt(dt)
//   x_d <- x_d + v_d dt
// a and w are formed once on the host; every operation is one IEEE float64
// operation (the build turns contraction off).  u - 1/2 is exact, so the kick
// is (2u - 1) sqrt(dt) rounded once.
// The paper launches one kernel per step and loads and stores the particle
// each time; here a launch runs steps_per_launch steps with the particle in
// registers (0: all steps in one launch).  Results are the same for every
// value, since each step's randoms depend only on (pid, step).
#include "../../include/orng.h"
#include "orng_device.hpp"
#include "orng_internal.hpp"

#include <algorithm>
#include <cmath>

namespace orng {

struct Bd2Args {
    double *x, *y, *vx, *vy;
    uint64_t pid0;
    uint32_t n, step0, n_steps, pad;
    double dt, decay, kick;  // dt, a = 1 - c dt, w = 2 sqrt(dt)
};

__global__ __launch_bounds__(256) void k_bd2(Bd2Args a) {
    const uint64_t i64 = (uint64_t)flat_block() * blockDim.x + threadIdx.x;
    if (i64 >= a.n) return;
    const uint32_t i = (uint32_t)i64;
    const uint64_t pid = a.pid0 + i;
    const uint32_t klo = (uint32_t)pid, khi = (uint32_t)(pid >> 32);
    double pos[2] = {a.x[i], a.y[i]}, vel[2] = {a.vx[i], a.vy[i]};
    for (uint32_t s = 0; s < a.n_steps; ++s) {
        uint32_t w[4];
        philox_block0_lanekey(a.step0 + s, klo, khi, w);
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const double kick = (u01_f64(w[2 * d], w[2 * d + 1]) - 0.5) * a.kick;
            vel[d] = a.decay * vel[d] + kick;
            pos[d] = pos[d] + vel[d] * a.dt;
        }
    }
    a.x[i] = pos[0];
    a.y[i] = pos[1];
    a.vx[i] = vel[0];
    a.vy[i] = vel[1];
}

}  // namespace orng

using namespace orng;

extern "C" int orng_bd2(uint64_t pid0, uint32_t n, uint32_t step0, uint32_t n_steps, double dt,
                        double gamma_over_m, double *x, double *y, double *vx, double *vy,
                        uint32_t steps_per_launch, void *stream) {
    if (!std::isfinite(dt) || dt < 0.0 || !std::isfinite(gamma_over_m)) return ORNG_EINVAL;
    if (n_steps && (uint64_t)step0 + n_steps - 1 > 0xFFFFFFFFull) return ORNG_ERANGE;
    if (n && pid0 + (n - 1) < pid0) return ORNG_ERANGE;
    if (!n || !n_steps) return ORNG_OK;
    for (const double *p : {x, y, vx, vy})
        if (!p || (reinterpret_cast<uintptr_t>(p) & 7u)) return ORNG_EINVAL;
    Bd2Args a;
    a.x = x;
    a.y = y;
    a.vx = vx;
    a.vy = vy;
    a.pid0 = pid0;
    a.n = n;
    a.pad = 0;
    a.dt = dt;
    a.decay = 1.0 - gamma_over_m * dt;
    a.kick = 2.0 * std::sqrt(dt);
    const uint32_t per = steps_per_launch ? steps_per_launch : n_steps;
    const Grid2 grid = grid_2d(blocks_for(n, 256));
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (uint32_t done = 0; done < n_steps; done += std::min(per, n_steps - done)) {
        a.step0 = step0 + done;
        a.n_steps = std::min(per, n_steps - done);
        hipLaunchKernelGGL(k_bd2, dim3(grid.x, grid.y), dim3(256), 0, s, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) { set_hip_error(e); return ORNG_EHIP; }
    }
    return ORNG_OK;
}
