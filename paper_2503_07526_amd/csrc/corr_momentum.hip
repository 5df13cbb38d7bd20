// corr_momentum.hip -- partial momentum densities of the mass-flux correction
// of the thermal conductivity (Section "Viscosity and thermal conductivity"):
// j_s = (1/V) sum over the atoms i of species s of m_s v(i), for every species.
//
// HBM-bound reduction: per atom three velocity components (12 or 24 bytes)
// and a one-byte species id (the ids are stored as bytes at create).  Each
// thread sums its atoms (grid-stride, fixed order; four consecutive atoms per
// 16-byte load when the layout allows) per species and component in double,
// the block reduces its 3 x n_species sums by wave shuffles and then across
// waves in a fixed order, and a final kernel (one wave per channel) adds the
// block sums in a fixed order and scales them by m_s / V, so the result does
// not depend on timing.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

constexpr int kMomThreads = 256;
constexpr int kMomAtomsPerThread = 8; // atoms per thread before the grid is capped
constexpr int kMomMaxBlocks = 1024;
constexpr int kMomSums = 3 * kMomMaxSpecies;

// Four consecutive values of a component (16-byte loads; the caller checks
// the alignment).  Every input byte is read once per push, so the loads are
// non-temporal (streamed past the caches: the massflux step 0.0769 against
// 0.0781 ms).
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void load4(const float *p, int64_t q, double (&o)[4])
{
    const nt_f4 f = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p) + q);
    o[0] = f[0];
    o[1] = f[1];
    o[2] = f[2];
    o[3] = f[3];
}

__device__ __forceinline__ void load4(const double *p, int64_t q, double (&o)[4])
{
    const nt_d2 f = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p) + 2 * q);
    const nt_d2 g = __builtin_nontemporal_load(reinterpret_cast<const nt_d2 *>(p) + 2 * q + 1);
    o[0] = f[0];
    o[1] = f[1];
    o[2] = g[0];
    o[3] = g[1];
}

__device__ __forceinline__ void add_atom(double (&acc)[kMomSums], int ns, int sp, double vx,
                                         double vy, double vz)
{
#pragma unroll
    for (int s = 0; s < kMomMaxSpecies; ++s) {
        if (s < ns) {
            const bool hit = sp == s;
            acc[3 * s + 0] += hit ? vx : 0.0;
            acc[3 * s + 1] += hit ? vy : 0.0;
            acc[3 * s + 2] += hit ? vz : 0.0;
        }
    }
}

template <typename T> __global__ __launch_bounds__(kMomThreads) void momentum_partial_kernel(MomentumArgs a)
{
    if (a.stamps && threadIdx.x == 0) stamp_start(a.stamps, blockIdx.x);
    const T *v = static_cast<const T *>(a.vel);
    const int64_t n = a.n_atoms;
    const int ns = a.n_species;
    double acc[kMomSums];
#pragma unroll
    for (int q = 0; q < kMomSums; ++q) acc[q] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.vec4) {
        // four consecutive atoms per step: n is a multiple of 4 and every
        // component starts 16-byte aligned
        const uint32_t *sp4 = reinterpret_cast<const uint32_t *>(a.species);
        for (int64_t q = first; q < n / 4; q += stride) {
            const uint32_t ids = __builtin_nontemporal_load(sp4 + q);
            double x[4], y[4], z[4];
            load4(v, q, x);
            load4(v + n, q, y);
            load4(v + 2 * n, q, z);
#pragma unroll
            for (int e = 0; e < 4; ++e) add_atom(acc, ns, (int)((ids >> (8 * e)) & 0xffu), x[e], y[e], z[e]);
        }
    } else {
        for (int64_t i = first; i < n; i += stride)
            add_atom(acc, ns, a.species[i], (double)v[i], (double)v[n + i], (double)v[2 * n + i]);
    }
    // wave sums (lane 0 ends with the wave's sum), then waves in order
    __shared__ double wsum[kMomThreads / 64][kMomSums];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kMomSums; ++q) {
        if (q < 3 * ns) {
            double x = acc[q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
            if (lane == 0) wsum[wave][q] = x;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 3 * ns) {
        double x = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) x += wsum[w][threadIdx.x];
        a.partial[(size_t)blockIdx.x * kMomSums + threadIdx.x] = x;
    }
}

// One wave per channel (block q): lane l adds the block sums l, l + 64, ...
// in order, then the wave adds its lanes by shuffles in a fixed order.
template <typename T> __global__ __launch_bounds__(64) void momentum_final_kernel(MomentumArgs a)
{
    const int q = blockIdx.x;
    const int nch = 3 * a.n_species;
    const int lane = threadIdx.x;
    double x = 0.0;
#pragma unroll 4
    for (int b = lane; b < a.n_blocks; b += 64) x += a.partial[(size_t)b * kMomSums + q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane != 0) return;
    if (a.stamps) stamp_end(a.stamps, (unsigned)q);
    T *out = static_cast<T *>(a.out);
    const T j = (T)(x * a.scale[q / 3]);
    if (a.pair) {
        const T *xin = static_cast<const T *>(a.vel) + 3 * a.n_atoms;
        out[q] = xin[q];
        out[nch + q] = j;
    } else {
        out[q] = j;
    }
}

} // namespace

int momentum_blocks(int64_t n_atoms)
{
    const int64_t per_block = (int64_t)kMomThreads * kMomAtomsPerThread;
    int64_t b = (n_atoms + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > kMomMaxBlocks) b = kMomMaxBlocks;
    return (int)b;
}

hipError_t launch_momentum(const MomentumArgs &a, hipStream_t st)
{
    if (a.n_species < 1 || a.n_species > kMomMaxSpecies || a.n_atoms < 1 || a.n_blocks < 1 ||
        a.n_blocks > kMomMaxBlocks)
        return hipErrorInvalidValue;
    if (a.dbl) {
        hipLaunchKernelGGL(momentum_partial_kernel<double>, dim3((unsigned)a.n_blocks),
                           dim3(kMomThreads), 0, st, a);
    } else {
        hipLaunchKernelGGL(momentum_partial_kernel<float>, dim3((unsigned)a.n_blocks),
                           dim3(kMomThreads), 0, st, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid((unsigned)(3 * a.n_species));
    if (a.dbl)
        hipLaunchKernelGGL(momentum_final_kernel<double>, grid, dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(momentum_final_kernel<float>, grid, dim3(64), 0, st, a);
    return hipGetLastError();
}

} // namespace corr
