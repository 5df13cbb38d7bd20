// corr_rhok.hip -- k-space density n(k) = sum_j exp(i k.r_j), k = 2 pi n / L
// (Section "Currents", Eq. k-density), the producer of a k-density group.
//
// Pass 1 (rhok_partial_kernel): block (kc, ab) owns a chunk of up to 256
// k-vectors (one per thread) and a contiguous range of atoms.  The range is
// walked in tiles of TA atoms: each thread first builds the power tables
// exp(2 pi i n x_j / L), n = 0..nmax, for one atom and each axis (base phase
// from a double sincospi, powers by double recurrence, rounded once to
// float) into LDS; after a barrier every thread accumulates
// X^nx * (Y^ny * Z^nz) of its own k-vector over the tile's atoms (negative
// components use the conjugate entry).  The tile sum is kept in float and
// added to a per-thread double accumulator, and the block writes one double
// partial per k.  Pass 2 (rhok_final_kernel) adds the partials of all atom
// blocks in a fixed order and stores n(k) in the group's sample precision,
// so the result is bitwise reproducible and uses no floating-point atomics.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

constexpr int kRhokThreads = 256;

__global__ __launch_bounds__(kRhokThreads) void rhok_partial_kernel(RhokArgs a, int tile_atoms)
{
    extern __shared__ float2 tab[]; // [tile_atoms][3][nmax+1]
    const int nn = a.nmax + 1;
    const int q = blockIdx.x * kRhokThreads + threadIdx.x; // sorted k index
    const bool active = q < a.nk;
    int ax = 0, ay = 0, az = 0;
    float sx = 1.f, sy = 1.f, sz = 1.f;
    if (active) {
        const int nx = a.kq[3 * q + 0], ny = a.kq[3 * q + 1], nz = a.kq[3 * q + 2];
        ax = nx < 0 ? -nx : nx; sx = nx < 0 ? -1.f : 1.f;
        ay = ny < 0 ? -ny : ny; sy = ny < 0 ? -1.f : 1.f;
        az = nz < 0 ? -nz : nz; sz = nz < 0 ? -1.f : 1.f;
    }
    const int64_t a_begin = (int64_t)blockIdx.y * a.atoms_per_block;
    int64_t a_end = a_begin + a.atoms_per_block;
    if (a_end > a.n_atoms) a_end = a.n_atoms;

    double accr = 0.0, acci = 0.0;
    for (int64_t t0 = a_begin; t0 < a_end; t0 += tile_atoms) {
        const int nt = (int)((a_end - t0) < tile_atoms ? (a_end - t0) : tile_atoms);
        __syncthreads();
        for (int j = threadIdx.x; j < nt; j += kRhokThreads) {
            const int64_t atom = t0 + j;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double f = (double)a.pos[(int64_t)d * a.n_atoms + atom] * a.inv_box;
                double sn, cs;
                sincospi(2.0 * f, &sn, &cs);
                float2 *row = tab + ((size_t)j * 3 + d) * nn;
                double pr = 1.0, pi = 0.0;
                row[0] = make_float2(1.f, 0.f);
                for (int n = 1; n < nn; ++n) {
                    const double r = pr * cs - pi * sn;
                    const double i = pr * sn + pi * cs;
                    pr = r;
                    pi = i;
                    row[n] = make_float2((float)pr, (float)pi);
                }
            }
        }
        __syncthreads();
        if (active) {
            float tr = 0.f, ti = 0.f;
            for (int j = 0; j < nt; ++j) {
                const float2 *base = tab + (size_t)j * 3 * nn;
                const float2 X = base[ax];
                const float2 Y = base[nn + ay];
                const float2 Z = base[2 * nn + az];
                const float xr = X.x, xi = sx * X.y;
                const float yr = Y.x, yi = sy * Y.y;
                const float zr = Z.x, zi = sz * Z.y;
                const float wr = __builtin_fmaf(yr, zr, -yi * zi);
                const float wi = __builtin_fmaf(yr, zi, yi * zr);
                tr = __builtin_fmaf(xr, wr, __builtin_fmaf(-xi, wi, tr));
                ti = __builtin_fmaf(xr, wi, __builtin_fmaf(xi, wr, ti));
            }
            accr += (double)tr;
            acci += (double)ti;
        }
    }
    if (active) {
        double *dst = a.partial + ((size_t)blockIdx.y * a.nk + q) * 2;
        dst[0] = accr;
        dst[1] = acci;
    }
}

__global__ void rhok_final_kernel(RhokArgs a)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.nk) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < a.n_atom_blocks; ++b) {
        const double *src = a.partial + ((size_t)b * a.nk + q) * 2;
        sr += src[0];
        si += src[1];
    }
    const int o = a.kperm[q];
    if (a.out_double)
        static_cast<double2 *>(a.out)[o] = make_double2(sr, si);
    else
        static_cast<float2 *>(a.out)[o] = make_float2((float)sr, (float)si);
}

int rhok_tile_atoms(int nmax)
{
    // Keep the table within 64 KiB of LDS.
    const size_t per_atom = (size_t)3 * (nmax + 1) * sizeof(float2);
    int ta = 256;
    while (ta > 32 && (size_t)ta * per_atom > 64 * 1024) ta /= 2;
    return ta;
}

hipError_t launch_rhok(const RhokArgs &a, hipStream_t st)
{
    const int ta = rhok_tile_atoms(a.nmax);
    const size_t lds = (size_t)ta * 3 * (a.nmax + 1) * sizeof(float2);
    dim3 grid((unsigned)a.n_chunks, (unsigned)a.n_atom_blocks);
    hipLaunchKernelGGL(rhok_partial_kernel, grid, dim3(kRhokThreads), lds, st, a, ta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rhok_final_kernel, dim3((unsigned)((a.nk + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

} // namespace corr
