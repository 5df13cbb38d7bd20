// corr_rhok.hip -- k-space density n(k) = sum_j exp(i k.r_j), k = 2 pi n / L
// (Section "Currents", Eq. k-density), the producer of a k-density group.
//
// The k-vectors are grouped on the host into segments: up to kSegWidth
// k-vectors that share (n_y, n_z) and have n_x in [nx0, nx0 + kSegWidth).  For
// one atom, exp(i k.r) = X^{n_x} * W with W = Y^{n_y} Z^{n_z}, so a thread
// owning a segment forms W once per atom and then needs one complex
// multiply-add per k-vector of the segment.
//
// Pass 1 (rhok_partial_kernel): block (chunk, atom-block) = one thread per
// segment (up to 1024 segments per chunk) over a contiguous range of atoms,
// walked in tiles of TA atoms.  For each tile the block first builds, for
// every atom and axis, the powers exp(2 pi i n x / L) for n in [-nmax,
// nmax (+ kSegWidth - 1 for x)] in LDS (base phase from a double sincospi,
// powers by a double recurrence, each rounded once to float; negative powers
// are the conjugates).  Each thread then accumulates its segment over the
// tile's atoms in float, adds the tile sums to double accumulators and
// finally writes double partials.  Pass 2 (rhok_final_kernel) adds the
// partials of all atom blocks in a fixed order and scatters n(k) to the
// caller's k order in the group's sample precision.  No floating-point
// atomics: the result is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

// LDS entries per atom: X over [-nmax, nmax + kSegWidth - 1], Y and Z over
// [-nmax, nmax].
__host__ __device__ inline int tab_x(int nmax) { return 2 * nmax + kSegWidth; }
__host__ __device__ inline int tab_yz(int nmax) { return 2 * nmax + 1; }
__host__ __device__ inline int tab_atom(int nmax) { return tab_x(nmax) + 2 * tab_yz(nmax); }

__global__ __launch_bounds__(1024) void rhok_partial_kernel(RhokArgs a, int tile_atoms)
{
    if (a.stamps && threadIdx.x == 0) stamp_start(a.stamps, blockIdx.x + gridDim.x * blockIdx.y);
    extern __shared__ float2 tab[]; // [tile_atoms][tab_atom]
    const int nmax = a.nmax;
    const int TX = tab_x(nmax), TYZ = tab_yz(nmax), TA = tab_atom(nmax);
    const int seg = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = seg < a.n_seg;
    int ix = 0, iy = 0, iz = 0;
    if (active) {
        ix = a.seg_nx0[seg] + nmax;            // X index of the segment's first n_x
        iy = TX + a.seg_ny[seg] + nmax;        // Y entry
        iz = TX + TYZ + a.seg_nz[seg] + nmax;  // Z entry
    }
    const int64_t a_begin = (int64_t)blockIdx.y * a.atoms_per_block;
    int64_t a_end = a_begin + a.atoms_per_block;
    if (a_end > a.n_atoms) a_end = a.n_atoms;

    double accr[kSegWidth], acci[kSegWidth];
#pragma unroll
    for (int i = 0; i < kSegWidth; ++i) accr[i] = acci[i] = 0.0;

    for (int64_t t0 = a_begin; t0 < a_end; t0 += tile_atoms) {
        const int nt = (int)((a_end - t0) < tile_atoms ? (a_end - t0) : tile_atoms);
        __syncthreads();
        // one (atom, axis) power table per thread
        for (int task = threadIdx.x; task < 3 * nt; task += blockDim.x) {
            const int j = task / 3, d = task - 3 * (task / 3);
            const double f = (double)a.pos[(int64_t)d * a.n_atoms + t0 + j] * a.inv_box;
            double sn, cs;
            sincospi(2.0 * f, &sn, &cs);
            float2 *row = tab + (size_t)j * TA + (d == 0 ? 0 : d == 1 ? TX : TX + TYZ);
            const int hi = d == 0 ? nmax + kSegWidth - 1 : nmax;
            double pr = 1.0, pi = 0.0;
            row[nmax] = make_float2(1.f, 0.f);
            for (int n = 1; n <= hi; ++n) {
                const double r = pr * cs - pi * sn;
                const double i = pr * sn + pi * cs;
                pr = r;
                pi = i;
                row[nmax + n] = make_float2((float)pr, (float)pi);
                if (n <= nmax) row[nmax - n] = make_float2((float)pr, -(float)pi);
            }
        }
        __syncthreads();
        if (active) {
            float tr[kSegWidth], ti[kSegWidth];
#pragma unroll
            for (int i = 0; i < kSegWidth; ++i) tr[i] = ti[i] = 0.f;
            for (int j = 0; j < nt; ++j) {
                const float2 *base = tab + (size_t)j * TA;
                const float2 Y = base[iy];
                const float2 Z = base[iz];
                const float wr = __builtin_fmaf(Y.x, Z.x, -Y.y * Z.y);
                const float wi = __builtin_fmaf(Y.x, Z.y, Y.y * Z.x);
#pragma unroll
                for (int i = 0; i < kSegWidth; ++i) {
                    const float2 X = base[ix + i];
                    tr[i] = __builtin_fmaf(X.x, wr, __builtin_fmaf(-X.y, wi, tr[i]));
                    ti[i] = __builtin_fmaf(X.x, wi, __builtin_fmaf(X.y, wr, ti[i]));
                }
            }
#pragma unroll
            for (int i = 0; i < kSegWidth; ++i) {
                accr[i] += (double)tr[i];
                acci[i] += (double)ti[i];
            }
        }
    }
    if (active) {
        // partial[slot][atom block] so that one slot's partials are contiguous
#pragma unroll
        for (int i = 0; i < kSegWidth; ++i) {
            const size_t slot = (size_t)seg * kSegWidth + i;
            double *dst = a.partial + (slot * a.n_atom_blocks + blockIdx.y) * 2;
            dst[0] = accr[i];
            dst[1] = acci[i];
        }
    }
}

// One wave per slot: lane l adds atom blocks l, l+64, ... in order, then a
// fixed-order wave reduction.
__global__ __launch_bounds__(256) void rhok_final_kernel(RhokArgs a)
{
    const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); // slot
    const int lane = threadIdx.x & 63;
    const int n_slots = a.n_seg * kSegWidth;
    if (q >= n_slots) return; // whole wave
    const int o = a.slot_out[q];
    if (o < 0) return; // whole wave
    double sr = 0.0, si = 0.0;
    const double *src = a.partial + (size_t)q * a.n_atom_blocks * 2;
    for (int b = lane; b < a.n_atom_blocks; b += 64) {
        sr += src[2 * b];
        si += src[2 * b + 1];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sr += __shfl_down(sr, off, 64);
        si += __shfl_down(si, off, 64);
    }
    if (lane != 0) return;
    if (a.stamps) stamp_end(a.stamps, (unsigned)q);
    if (a.out_double)
        static_cast<double2 *>(a.out)[o] = make_double2(sr, si);
    else
        static_cast<float2 *>(a.out)[o] = make_float2((float)sr, (float)si);
}

} // namespace

int rhok_tile_atoms(int nmax)
{
    // Keep the tables within 64 KiB of LDS.
    const size_t per_atom = (size_t)tab_atom(nmax) * sizeof(float2);
    int ta = 128;
    while (ta > 8 && (size_t)ta * per_atom > 64 * 1024) ta /= 2;
    return ta;
}

int rhok_block_threads(int n_seg)
{
    int t = ((n_seg + 63) / 64) * 64;
    return t > 1024 ? 1024 : (t < 64 ? 64 : t);
}

hipError_t launch_rhok(const RhokArgs &a, hipStream_t st)
{
    const int ta = rhok_tile_atoms(a.nmax);
    const size_t lds = (size_t)ta * tab_atom(a.nmax) * sizeof(float2);
    const int threads = rhok_block_threads(a.n_seg);
    const unsigned chunks = (unsigned)((a.n_seg + threads - 1) / threads);
    hipLaunchKernelGGL(rhok_partial_kernel, dim3(chunks, (unsigned)a.n_atom_blocks),
                       dim3(threads), lds, st, a, ta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n_slots = a.n_seg * kSegWidth;
    hipLaunchKernelGGL(rhok_final_kernel, dim3((unsigned)((n_slots + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

} // namespace corr
