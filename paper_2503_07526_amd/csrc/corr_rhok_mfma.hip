// corr_rhok_mfma.hip -- k-space density n(k) = sum_j exp(i k.r_j) (Section
// "Currents", Eq. k-density) as a dense contraction on the matrix cores.
//
// With X = exp(2 pi i x/L), Y, Z likewise, exp(i k.r) = (X^{n_x} Y^{n_y}) Z^{n_z}
// and Z^{-n} = conj(Z^{n}).  With P = X^{n_x} Y^{n_y} and z = Z^{|n_z|} the four
// real sums over the atoms
//     A1 = sum Re P Re z,  A2 = sum Im P Im z,  A3 = sum Re P Im z,  A4 = sum Im P Re z
// give n(k) = (A1 - A2) + i (A3 + A4) for n_z >= 0 and (A1 + A2) + i (A4 - A3)
// for n_z < 0.  Each sum is a real matrix product over the atoms between M =
// the distinct (n_x, n_y) pairs of the k-set (16-row tiles) and N = |n_z| in
// [0, 15] (one 16-column tile).  Per atom only one complex product P per pair
// is formed on the vector units; z comes from a table.
//
// Precision: the operands are at most 1 in magnitude.  Each real operand v is
// split into v_hi = fp16(v) and v_lo = fp16(v - v_hi) (about 22 significant
// bits together) and a real product is a_hi b_hi + a_hi b_lo + a_lo b_hi (the
// dropped a_lo b_lo is below 2^-22), i.e. three fp16 matrix products with
// fp32 accumulation per sum, twelve per tile and K-step
// (v_mfma_f32_16x16x16_f16).  The fp32 accumulators are added to double
// accumulators after every tile of kMfmaTileAtoms atoms and the blocks write
// double partials, reduced over the atom blocks in a fixed order as in the
// vector-unit producer (corr_rhok.hip), so the result is reproducible.
//
// Operand layout of v_mfma_f32_16x16x16_f16 (checked on the device): lane l
// holds A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16] for j < 4 and receives
// D[4(l/16)+v][l%16] for v < 4; K runs over 16 atoms.
//
// Work split: block (chunk, atom block); each wave of a block owns one M tile
// and all waves share the tile's LDS tables: X and Y powers as float2
// [2 nmax + 1][kTabStride] (a row per power, atoms along the row, so a lane's
// four atoms are two 16-byte reads; the row stride is padded so that the 16
// rows a K-step reads start in different banks) and the split |n_z| powers
// already in B-fragment order.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaTileAtoms = 64; // atoms per LDS tile (4 K-steps of 16)
constexpr int kMfmaKSteps = kMfmaTileAtoms / 16;
constexpr int kTabStride = kMfmaTileAtoms + 2; // float2 per table row (4-bank shift)
constexpr int kMfmaMaxWaves = 16;  // waves per block (one M tile each)
constexpr int kMfmaCols = 16;      // |n_z| = 0 .. 15
// B fragments in LDS: [K-step][part: re hi, re lo, im hi, im lo][atom quad][column]
constexpr int kBParts = 4;
constexpr int kBHalves = kMfmaKSteps * kBParts * 4 * kMfmaCols * 4;

__device__ __forceinline__ float4_t mfma(half4_t a, half4_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int bfrag_index(int ks, int part, int quad, int col)
{
    return ((ks * kBParts + part) * 4 + quad) * kMfmaCols + col; // in half4 units
}

__global__ __launch_bounds__(kMfmaMaxWaves * 64) void rhok_mfma_kernel(RhokMfmaArgs a)
{
    extern __shared__ float2 lds[];
    const int nn = 2 * a.nmax + 1;
    float2 *tabx = lds;                        // [nn][kTabStride]
    float2 *taby = tabx + nn * kTabStride;     // [nn][kTabStride]
    half4_t *bfr = reinterpret_cast<half4_t *>(taby + nn * kTabStride);
    _Float16 *bh = reinterpret_cast<_Float16 *>(bfr);

    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15; // A row / B column within the tile
    const int kq = lane >> 4;  // atom quad of the K-step
    const int mt = blockIdx.x * waves + wave;
    const bool active = mt < a.n_mtiles; // wave-uniform
    const int pm_row = mt * 16 + col;
    const int ax = active ? a.pair_nx[pm_row] + a.nmax : a.nmax;
    const int ay = active ? a.pair_ny[pm_row] + a.nmax : a.nmax;
    // the lane's X and Y rows at its first atom, 16-byte aligned
    const float4 *xrow = reinterpret_cast<const float4 *>(tabx + ax * kTabStride + kq * 4);
    const float4 *yrow = reinterpret_cast<const float4 *>(taby + ay * kTabStride + kq * 4);
    const half4_t *bl = bfr + kq * kMfmaCols + col;

    double acc[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][v] = 0.0;

    const int64_t a_begin = (int64_t)blockIdx.y * a.atoms_per_block;
    int64_t a_end = a_begin + a.atoms_per_block;
    if (a_end > a.n_atoms) a_end = a.n_atoms;

    for (int64_t t0 = a_begin; t0 < a_end; t0 += kMfmaTileAtoms) {
        const int nt = (int)((a_end - t0) < kMfmaTileAtoms ? (a_end - t0) : kMfmaTileAtoms);
        __syncthreads();
        // Tables: task (axis d, atom j), d uniform per wave.  Base phase from a
        // double sincospi, powers by a double recurrence, rounded once.  Atoms
        // past the end of the range get zero entries (no contribution).
        for (int task = threadIdx.x; task < 3 * kMfmaTileAtoms; task += blockDim.x) {
            const int d = task / kMfmaTileAtoms, j = task - d * kMfmaTileAtoms;
            const bool live = j < nt;
            double sn = 0.0, cs = 1.0;
            if (live) {
                const double f = (double)a.pos[(int64_t)d * a.n_atoms + t0 + j] * a.inv_box;
                sincospi(2.0 * f, &sn, &cs);
            }
            if (d < 2) {
                float2 *colp = (d == 0 ? tabx : taby) + j;
                if (!live) {
                    for (int n = 0; n < nn; ++n) colp[n * kTabStride] = make_float2(0.f, 0.f);
                    continue;
                }
                double pr = 1.0, pi = 0.0;
                colp[a.nmax * kTabStride] = make_float2(1.f, 0.f);
                for (int n = 1; n <= a.nmax; ++n) {
                    const double r = pr * cs - pi * sn;
                    const double i = pr * sn + pi * cs;
                    pr = r;
                    pi = i;
                    colp[(a.nmax + n) * kTabStride] = make_float2((float)pr, (float)pi);
                    colp[(a.nmax - n) * kTabStride] = make_float2((float)pr, -(float)pi);
                }
            } else {
                // Z^{c}, c = |n_z| in [0, 15], split into fp16 hi/lo, stored at
                // half j%4 of the fragment of (K-step, quad, column c)
                const int ks = j >> 4, quad = (j >> 2) & 3, h = j & 3;
                double pr = live ? 1.0 : 0.0, pi = 0.0;
                for (int c = 0; c < kMfmaCols; ++c) {
                    if (c > 0) {
                        const double r = pr * cs - pi * sn;
                        const double i = pr * sn + pi * cs;
                        pr = r;
                        pi = i;
                    }
                    const float zr = c <= a.nmax ? (float)pr : 0.f;
                    const float zi = c <= a.nmax ? (float)pi : 0.f;
                    const _Float16 rh = (_Float16)zr, ih = (_Float16)zi;
                    const _Float16 rl = (_Float16)(zr - (float)rh), il = (_Float16)(zi - (float)ih);
                    bh[bfrag_index(ks, 0, quad, c) * 4 + h] = rh;
                    bh[bfrag_index(ks, 1, quad, c) * 4 + h] = rl;
                    bh[bfrag_index(ks, 2, quad, c) * 4 + h] = ih;
                    bh[bfrag_index(ks, 3, quad, c) * 4 + h] = il;
                }
            }
        }
        __syncthreads();
        if (!active) continue;
        float4_t s1 = {0.f, 0.f, 0.f, 0.f}, s2 = s1, s3 = s1, s4 = s1;
        // all four K-steps: the entries of atoms past nt are zero
#pragma unroll
        for (int ks = 0; ks < kMfmaKSteps; ++ks) {
            const half4_t zrh = bl[bfrag_index(ks, 0, 0, 0)];
            const half4_t zrl = bl[bfrag_index(ks, 1, 0, 0)];
            const half4_t zih = bl[bfrag_index(ks, 2, 0, 0)];
            const half4_t zil = bl[bfrag_index(ks, 3, 0, 0)];
            const float4 x01 = xrow[ks * 8], x23 = xrow[ks * 8 + 1];
            const float4 y01 = yrow[ks * 8], y23 = yrow[ks * 8 + 1];
            const float xr[4] = {x01.x, x01.z, x23.x, x23.z}, xi[4] = {x01.y, x01.w, x23.y, x23.w};
            const float yr[4] = {y01.x, y01.z, y23.x, y23.z}, yi[4] = {y01.y, y01.w, y23.y, y23.w};
            half4_t prh, prl, pih, pil;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float pr = __builtin_fmaf(xr[q], yr[q], -xi[q] * yi[q]);
                const float pi = __builtin_fmaf(xr[q], yi[q], xi[q] * yr[q]);
                const _Float16 rh = (_Float16)pr, ih = (_Float16)pi;
                prh[q] = rh;
                pih[q] = ih;
                prl[q] = (_Float16)(pr - (float)rh);
                pil[q] = (_Float16)(pi - (float)ih);
            }
            // interleaved so that dependent products on one sum are apart
            s1 = mfma(prh, zrh, s1);
            s2 = mfma(pih, zih, s2);
            s3 = mfma(prh, zih, s3);
            s4 = mfma(pih, zrh, s4);
            s1 = mfma(prh, zrl, s1);
            s2 = mfma(pih, zil, s2);
            s3 = mfma(prh, zil, s3);
            s4 = mfma(pih, zrl, s4);
            s1 = mfma(prl, zrh, s1);
            s2 = mfma(pil, zih, s2);
            s3 = mfma(prl, zih, s3);
            s4 = mfma(pil, zrh, s4);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            acc[0][v] += (double)s1[v];
            acc[1][v] += (double)s2[v];
            acc[2][v] += (double)s3[v];
            acc[3][v] += (double)s4[v];
        }
    }
    if (!active) return;
    // Row pm = pair, column col = |n_z|: only slots that are k-vectors of the
    // group are stored, in partial[k][atom block].
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int pm = mt * 16 + kq * 4 + v;
        const int32_t *sk = a.slot_k + ((size_t)pm * kMfmaCols + col) * 2;
        const int kp = sk[0], km = sk[1];
        if (kp >= 0) {
            double *dst = a.partial + ((size_t)kp * a.n_atom_blocks + blockIdx.y) * 2;
            dst[0] = acc[0][v] - acc[1][v];
            dst[1] = acc[2][v] + acc[3][v];
        }
        if (km >= 0) {
            double *dst = a.partial + ((size_t)km * a.n_atom_blocks + blockIdx.y) * 2;
            dst[0] = acc[0][v] + acc[1][v];
            dst[1] = acc[3][v] - acc[2][v];
        }
    }
}

// One wave per k-vector: sum the partials of its slot over the atom blocks in
// a fixed order and store n(k) at the caller's index.  A k-vector listed
// twice reads the partials stored under its first index.
__global__ __launch_bounds__(256) void rhok_mfma_final_kernel(RhokMfmaArgs a)
{
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= a.nk) return; // whole wave
    const size_t row = (size_t)a.k_src[k];
    const double *src = a.partial + row * a.n_atom_blocks * 2;
    double sr = 0.0, si = 0.0;
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
    if (a.out_double)
        static_cast<double2 *>(a.out)[k] = make_double2(sr, si);
    else
        static_cast<float2 *>(a.out)[k] = make_float2((float)sr, (float)si);
}

} // namespace

int rhok_mfma_cols() { return kMfmaCols; }
int rhok_mfma_max_nmax() { return kMfmaCols - 1; }

hipError_t launch_rhok_mfma(const RhokMfmaArgs &a, hipStream_t st)
{
    if (a.nmax > kMfmaCols - 1 || a.n_mtiles < 1) return hipErrorInvalidValue;
    const int nn = 2 * a.nmax + 1;
    const size_t lds = (size_t)2 * nn * kTabStride * sizeof(float2) +
                       (size_t)kBHalves * sizeof(_Float16);
    // waves per block: the M tiles dealt evenly over the fewest blocks
    const int chunks = (a.n_mtiles + kMfmaMaxWaves - 1) / kMfmaMaxWaves;
    const int waves = (a.n_mtiles + chunks - 1) / chunks;
    hipLaunchKernelGGL(rhok_mfma_kernel, dim3((unsigned)chunks, (unsigned)a.n_atom_blocks),
                       dim3(waves * 64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rhok_mfma_final_kernel, dim3((unsigned)((a.nk + 3) / 4)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

} // namespace corr
