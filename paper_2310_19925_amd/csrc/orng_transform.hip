// Element-wise Box-Muller transform of caller-supplied words: the same
// float32 functions the F32_NORMAL fills use, exposed for users who bring
// their own random bits (and used by the test-suite to check the normal path
// on every argument its logarithm and quarter-turn sine/cosine can take).
#include "../../include/orng.h"
#include "orng_internal.hpp"

namespace orng {

__global__ __launch_bounds__(256) void k_normal_pairs(const uint32_t *x0, const uint32_t *x1,
                                                      uint64_t n, float *z0, float *z1) {
    const uint64_t i = (uint64_t)flat_block() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float a, b;
    normal_pair(x0[i], x1[i], a, b);
    z0[i] = a;
    z1[i] = b;
}

}  // namespace orng

extern "C" int orng_normal_pairs(const uint32_t *d_x0, const uint32_t *d_x1, uint64_t n,
                                 float *d_z0, float *d_z1, void *stream) {
    if (n == 0) return ORNG_OK;
    const void *ptrs[] = {d_x0, d_x1, d_z0, d_z1};
    for (const void *p : ptrs)
        if (!p || (reinterpret_cast<uintptr_t>(p) & 3u)) return ORNG_EINVAL;
    if (n > (1ull << 40)) return ORNG_ERANGE;
    const orng::Grid2 g = orng::grid_2d((n + 255) / 256);
    orng::k_normal_pairs<<<dim3(g.x, g.y), dim3(256), 0, static_cast<hipStream_t>(stream)>>>(
        d_x0, d_x1, n, d_z0, d_z1);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        orng::set_hip_error(e);
        return ORNG_EHIP;
    }
    return ORNG_OK;
}
