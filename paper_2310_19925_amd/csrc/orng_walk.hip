// Fused Brownian walk: one lane per particle, all steps in registers.
//
// The paper's benchmark (section 4, Fig. 1; section 5.1) advances many
// independent particles with one kernel launch per step, each thread building
// its generator from (particle id, step) and loading/storing the particle
// every step.  Here the whole walk is one launch: particle i owns the Philox
// stream (seed, ctr0 + i); global step g uses normal samples dim*g .. dim*g +
// dim - 1 of that stream; each coordinate is updated as
// x = fmaf(sigma, normal, x), sigma = float(sqrt(2 D dt)).  One Philox block
// yields four normals, so three blocks cover four 3-D steps.  Positions are
// read once and written once (12 bytes per particle for the 3-D case); the
// only other memory traffic is the optional mean-squared-displacement
// snapshot, a workgroup reduction plus one float64 atomic per workgroup.
#include "orng_internal.hpp"

namespace orng {

struct WalkArgs {
    KeySched ks;
    float *pos;          // SoA [dim][n]
    double *msd;         // nullable: sums of |x|^2 per snapshot
    uint64_t q0, q1;     // normal-sample range [dim*step0, dim*(step0+n_steps))
    uint32_t n;
    uint32_t ctr0;
    uint32_t msd_every;  // 0: no snapshots
    uint32_t dim;
    float sigma;
};

// Sum of v over the workgroup, atomically added to *dst by thread 0.
__device__ void wg_sum_add(double v, double *dst) {
    __shared__ double part[8];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const uint32_t wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63u) == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w) t += part[w];
        unsafeAtomicAdd(dst, t);
    }
    __syncthreads();
}

template <int DIM>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < a.n;
    float x[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[d] = live ? a.pos[(uint64_t)d * a.n + i] : 0.0f;
    const uint32_t ctr = a.ctr0 + i;
    const uint64_t step0 = a.q0 / DIM;
    // blocks of four normals covering [q0, q1)
    const uint64_t bfirst = a.q0 / 4, blast = (a.q1 - 1) / 4;
    for (uint64_t b = bfirst; b <= blast; ++b) {
        uint32_t w[4];
        philox_block((uint32_t)b, ctr, a.ks, w);
        float g[4];
        normal_pair(w[0], w[1], g[0], g[1]);
        normal_pair(w[2], w[3], g[2], g[3]);
        const bool inner = b * 4 >= a.q0 && b * 4 + 4 <= a.q1;
        const uint32_t d0 = (uint32_t)((b * 4) % DIM);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t q = b * 4 + (uint64_t)j;
            if (!inner && (q < a.q0 || q >= a.q1)) continue;
            const uint32_t d = (d0 + (uint32_t)j) % DIM;  // wave-uniform
#pragma unroll
            for (int e = 0; e < DIM; ++e)
                if ((uint32_t)e == d) x[e] = fmaf(a.sigma, g[j], x[e]);
            if (a.msd_every && d == DIM - 1) {
                const uint64_t done = q / DIM + 1 - step0;  // local steps completed
                if (done % a.msd_every == 0) {
                    double r2 = 0.0;
#pragma unroll
                    for (int e = 0; e < DIM; ++e) r2 += (double)x[e] * (double)x[e];
                    wg_sum_add(live ? r2 : 0.0, a.msd + (done / a.msd_every - 1));
                }
            }
        }
    }
    if (live) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) a.pos[(uint64_t)d * a.n + i] = x[d];
    }
}

__global__ void k_zero_f64(double *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

hipError_t launch_walk(uint64_t seed, uint32_t ctr0, uint32_t n, uint32_t dim, uint64_t step0,
                       uint32_t n_steps, float sigma, float *pos, double *msd,
                       uint32_t msd_every, hipStream_t s) {
    if (n == 0 || n_steps == 0) return hipSuccess;
    WalkArgs a;
    a.ks = make_keysched(seed);
    a.pos = pos;
    a.msd = msd;
    a.q0 = (uint64_t)dim * step0;
    a.q1 = (uint64_t)dim * (step0 + n_steps);
    a.n = n;
    a.ctr0 = ctr0;
    a.msd_every = msd ? msd_every : 0;
    a.dim = dim;
    a.sigma = sigma;
    if (a.msd_every) {
        const uint32_t nsnap = n_steps / a.msd_every;
        if (nsnap == 0) {
            a.msd_every = 0;
        } else {
            k_zero_f64<<<(nsnap + 255) / 256, 256, 0, s>>>(msd, nsnap);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    const uint32_t wg = 256;
    const uint32_t grid = (n + wg - 1) / wg;
    void *args[] = {&a};
    void *k = dim == 1 ? reinterpret_cast<void *>(&k_walk<1>)
            : dim == 2 ? reinterpret_cast<void *>(&k_walk<2>)
                       : reinterpret_cast<void *>(&k_walk<3>);
    return hipLaunchKernel(k, dim3(grid), dim3(wg), args, 0, s);
}

}  // namespace orng
