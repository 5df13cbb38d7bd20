// corr_reduce.hip -- readout support (Algorithm 2): per-(level, lag) sums of
// the accumulators over a channel range, in double precision, in a fixed
// order (block partials, then partials in block order), plus a gather of the
// accumulators of a channel slice.  A compensated accumulator is read as
// value - compensation, evaluated in double; a one-level window in the
// block-deferred form adds the products of its pending pushes.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

// Products of the pushes that a one-level window in the block-deferred form
// (corr_window.hip) has staged but not yet folded into lag L = e: its lag
// block j = L / wlpb has folded every block q with kWindowT q + j <= S, so the
// pushes after f = kWindowT floor((S - j) / kWindowT) are pending.  Summed in
// double in push order; pushes s <= L have no lagged value and add nothing.
__device__ double2 window_pending(const ReduceArgs &a, int e, int64_t c)
{
    const int L = e;
    const int j = L / a.wlpb;
    const int64_t S = a.n_push;
    const int64_t f = S >= j ? ((S - j) / kWindowT) * kWindowT : 0;
    const int64_t s1 = f + 1 > (int64_t)L + 1 ? f + 1 : (int64_t)L + 1;
    if (s1 > S) return make_double2(0.0, 0.0);
    const int64_t tile = c / a.tw;
    const int64_t lane = c - tile * a.tw;
    const char *tb = a.state + tile * a.tile_bytes;
    const int p0 = a.p0;
    int sx = (int)((s1 - 1) % p0);
    int sy = (int)((s1 - L - 1) % p0);
    double re = 0.0, im = 0.0;
    if (a.kind >= K_CF32_F64) {
        const float2 *ring = reinterpret_cast<const float2 *>(tb) + lane;
        for (int64_t s = s1; s <= S; ++s) {
            const float2 x = ring[(size_t)sx * a.tw];
            const float2 y = ring[(size_t)sy * a.tw];
            re += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
            im += (double)x.y * (double)y.x - (double)x.x * (double)y.y;
            sx = sx + 1 == p0 ? 0 : sx + 1;
            sy = sy + 1 == p0 ? 0 : sy + 1;
        }
    } else {
        const float *ring = reinterpret_cast<const float *>(tb) + lane;
        for (int64_t s = s1; s <= S; ++s) {
            re += (double)ring[(size_t)sx * a.tw] * (double)ring[(size_t)sy * a.tw];
            sx = sx + 1 == p0 ? 0 : sx + 1;
            sy = sy + 1 == p0 ? 0 : sy + 1;
        }
    }
    return make_double2(re, im);
}

__device__ __forceinline__ double2 stored_acc(const ReduceArgs &a, int e, int64_t c)
{
    const int64_t tile = c / a.tw;
    const int64_t lane = c - tile * a.tw;
    const char *tb = a.state + tile * a.tile_bytes;
    switch (a.kind) {
    case K_F32_F64:
    case K_F64_F64:
        return make_double2(reinterpret_cast<const double *>(tb + a.hi_off[e])[lane], 0.0);
    case K_F32_KAHAN: {
        const float h = reinterpret_cast<const float *>(tb + a.hi_off[e])[lane];
        const float l = reinterpret_cast<const float *>(tb + a.lo_off[e])[lane];
        return make_double2((double)h - (double)l, 0.0);
    }
    case K_F32_F32:
        return make_double2((double)reinterpret_cast<const float *>(tb + a.hi_off[e])[lane], 0.0);
    case K_CF32_F64:
    case K_CF64_F64:
        return reinterpret_cast<const double2 *>(tb + a.hi_off[e])[lane];
    case K_CF32_KAHAN: {
        const float2 h = reinterpret_cast<const float2 *>(tb + a.hi_off[e])[lane];
        const float2 l = reinterpret_cast<const float2 *>(tb + a.lo_off[e])[lane];
        return make_double2((double)h.x - (double)l.x, (double)h.y - (double)l.y);
    }
    default: {
        const float2 h = reinterpret_cast<const float2 *>(tb + a.hi_off[e])[lane];
        return make_double2((double)h.x, (double)h.y);
    }
    }
}

__device__ __forceinline__ double2 read_acc(const ReduceArgs &a, int e, int64_t c)
{
    double2 v = stored_acc(a, e, c);
    if (a.wlpb > 0) {
        const double2 w = window_pending(a, e, c);
        v.x += w.x;
        v.y += w.y;
    }
    return v;
}

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void reduce_partial_kernel(ReduceArgs a)
{
    __shared__ double sr[kRedThreads];
    __shared__ double si[kRedThreads];
    const int e = blockIdx.y;
    const int64_t n = a.ch_end - a.ch_begin;
    const int64_t per = (n + a.blocks_per_entry - 1) / a.blocks_per_entry;
    const int64_t b0 = a.ch_begin + (int64_t)blockIdx.x * per;
    int64_t b1 = b0 + per;
    if (b1 > a.ch_end) b1 = a.ch_end;
    double ar = 0.0, ai = 0.0;
    for (int64_t c = b0 + threadIdx.x; c < b1; c += kRedThreads) {
        const double2 v = read_acc(a, e, c);
        ar += v.x;
        ai += v.y;
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *dst = a.partial + ((size_t)e * a.blocks_per_entry + blockIdx.x) * 2;
        dst[0] = sr[0];
        dst[1] = si[0];
    }
}

__global__ void reduce_final_kernel(ReduceArgs a)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_entries) return;
    double r = 0.0, i = 0.0;
    for (int b = 0; b < a.blocks_per_entry; ++b) {
        r += a.partial[((size_t)e * a.blocks_per_entry + b) * 2 + 0];
        i += a.partial[((size_t)e * a.blocks_per_entry + b) * 2 + 1];
    }
    a.out[2 * e + 0] = r;
    a.out[2 * e + 1] = i;
}

// out[(c - ch_begin) * n_entries + e][2] for c in [ch_begin, ch_end).
__global__ void gather_kernel(ReduceArgs a)
{
    const int64_t n = (a.ch_end - a.ch_begin) * a.n_entries;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = a.ch_begin + i / a.n_entries;
        const int e = (int)(i % a.n_entries);
        const double2 v = read_acc(a, e, c);
        a.out[2 * i + 0] = v.x;
        a.out[2 * i + 1] = v.y;
    }
}

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st)
{
    dim3 grid((unsigned)a.blocks_per_entry, (unsigned)a.n_entries);
    hipLaunchKernelGGL(reduce_partial_kernel, grid, dim3(kRedThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_final_kernel, dim3((unsigned)((a.n_entries + 63) / 64)), dim3(64), 0,
                       st, a);
    return hipGetLastError();
}

hipError_t launch_gather(const ReduceArgs &a, hipStream_t st)
{
    const int64_t n = (a.ch_end - a.ch_begin) * a.n_entries;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

} // namespace corr
