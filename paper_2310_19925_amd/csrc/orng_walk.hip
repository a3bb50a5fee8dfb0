// Fused Brownian walk: one lane per particle, all steps in registers.
//
// The paper's benchmark (section 4, Fig. 1; section 5.1) advances many
// independent particles with one kernel launch per step, each thread building
// its generator from (particle id, step) and loading/storing the particle
// every step.  Here the whole walk is one launch: particle i owns the Philox
// stream (seed, ctr0 + i); global step g uses normal samples dim*g .. dim*g +
// dim - 1 of that stream; each coordinate is updated as
// x = fmaf(sigma, normal, x), sigma = float(sqrt(2 D dt)).  One Philox block
// yields four normals, so three blocks cover four 3-D steps (a group).  Positions are
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

// Normal sample q of this lane's stream (one Philox block, one pair).
__device__ __forceinline__ float normal_at(uint64_t q, uint32_t ctr, const KeySched &ks) {
    uint32_t w[4];
    philox_block((uint32_t)(q >> 2), ctr, ks, w);
    const uint32_t h = (uint32_t)(q >> 1) & 1u;
    float z0, z1;
    normal_pair(h ? w[2] : w[0], h ? w[3] : w[1], z0, z1);
    return (q & 1) ? z1 : z0;
}

// Per-step bookkeeping shared by both loops: count local steps and take an
// MSD snapshot after every msd_every of them (uniform across the grid).
template <int DIM>
__device__ __forceinline__ void after_step(const WalkArgs &a, const float x[DIM], bool live,
                                           uint32_t &done, uint32_t &next_snap) {
    ++done;
    if (a.msd_every && done == next_snap) {
        double r2 = 0.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) r2 += (double)x[e] * (double)x[e];
        wg_sum_add(live ? r2 : 0.0, a.msd + (done / a.msd_every - 1));
        next_snap += a.msd_every;
    }
}

// Steps are processed in groups that start on a Philox block boundary:
// GB blocks (4*GB normals) feed GS = 4*GB/DIM whole steps, so inside a group
// every normal's coordinate is a compile-time constant.  Steps before the
// first group boundary and after the last are done one at a time.
template <int DIM>
__global__ __launch_bounds__(256) void k_walk(WalkArgs a) {
    constexpr uint32_t GB = DIM == 3 ? 3 : 1;   // Philox blocks per group
    constexpr uint32_t GS = 4 * GB / DIM;       // steps per group
    const uint64_t i64 = (uint64_t)flat_block() * blockDim.x + threadIdx.x;
    if ((uint64_t)flat_block() * blockDim.x >= a.n) return;  // a whole workgroup past the end
    const uint32_t i = (uint32_t)i64;
    const bool live = i64 < a.n;
    float x[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) x[d] = live ? a.pos[(uint64_t)d * a.n + i] : 0.0f;
    const uint32_t ctr = a.ctr0 + i;
    const uint64_t g0 = a.q0 / DIM, g1 = a.q1 / DIM;  // global steps [g0, g1)
    uint64_t ga = (g0 + GS - 1) / GS * GS;             // first group-aligned step
    if (ga > g1) ga = g1;
    const uint64_t gb = ga + (g1 - ga) / GS * GS;      // end of whole groups
    uint32_t done = 0, next_snap = a.msd_every;
    // head: single steps
    for (uint64_t g = g0; g < ga; ++g) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            x[d] = fmaf(a.sigma, normal_at(DIM * g + d, ctr, a.ks), x[d]);
        after_step<DIM>(a, x, live, done, next_snap);
    }
    // whole groups
    for (uint64_t g = ga; g < gb; g += GS) {
        const uint64_t b0 = DIM * g / 4;
        float nrm[4 * GB];
#pragma unroll
        for (uint32_t k = 0; k < GB; ++k) {
            uint32_t w[4];
            philox_block((uint32_t)(b0 + k), ctr, a.ks, w);
            normal_pair(w[0], w[1], nrm[4 * k + 0], nrm[4 * k + 1]);
            normal_pair(w[2], w[3], nrm[4 * k + 2], nrm[4 * k + 3]);
        }
#pragma unroll
        for (uint32_t s = 0; s < GS; ++s) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) x[d] = fmaf(a.sigma, nrm[DIM * s + d], x[d]);
            after_step<DIM>(a, x, live, done, next_snap);
        }
    }
    // tail: single steps
    for (uint64_t g = gb; g < g1; ++g) {
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            x[d] = fmaf(a.sigma, normal_at(DIM * g + d, ctr, a.ks), x[d]);
        after_step<DIM>(a, x, live, done, next_snap);
    }
    if (live) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) a.pos[(uint64_t)d * a.n + i] = x[d];
    }
}

__global__ void k_zero_f64(double *p, uint32_t n) {
    const uint64_t i = (uint64_t)flat_block() * blockDim.x + threadIdx.x;
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
            const Grid2 gz = grid_2d(blocks_for(nsnap, 256));
            k_zero_f64<<<dim3(gz.x, gz.y), 256, 0, s>>>(msd, nsnap);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    const uint32_t wg = 256;
    const Grid2 grid = grid_2d(blocks_for(n, wg));
    void *args[] = {&a};
    void *k = dim == 1 ? reinterpret_cast<void *>(&k_walk<1>)
            : dim == 2 ? reinterpret_cast<void *>(&k_walk<2>)
                       : reinterpret_cast<void *>(&k_walk<3>);
    return hipLaunchKernel(k, dim3(grid.x, grid.y), dim3(wg), args, 0, s);
}

}  // namespace orng
