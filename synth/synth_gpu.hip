// synth_gpu.hip -- seeded synthetic inputs generated on the GPU.
//
// Same definitions as synth_cpu.c, bit for bit (SplitMix64 output function on
// a counter, Irwin-Hall innovations of twelve 20-bit midpoint uniforms, OU
// recursion x_{t+1} = fma(a, x_t, round(b * xi))).  Used by the benchmark and
// the large-size tests to produce inputs directly in device memory.  Holds
// none of the correlator's arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int32_t xi_num(uint64_t key, uint64_t step, uint64_t channel)
{
    int32_t s = 0;
    const uint64_t base = (step << 32) | (channel << 2);
#pragma unroll
    for (uint64_t w = 0; w < 4; ++w) {
        uint64_t r = mix64(key + (base | w) * kGamma);
        s += (int32_t)(r & 0xFFFFF);
        s += (int32_t)((r >> 20) & 0xFFFFF);
        s += (int32_t)((r >> 40) & 0xFFFFF);
    }
    return s + 6 - 6 * (1 << 20);
}

// out[s][n] for s in [0, n_steps): channel c = i, coefficients a[c/comps].
__global__ void ou_f32_kernel(uint64_t key, int64_t n, int comps, const float* __restrict__ a,
                              const float* __restrict__ b, float sigma, int64_t t_begin,
                              int64_t n_steps, float* __restrict__ state, float* __restrict__ out,
                              int64_t out_stride)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float ac = a[i / comps];
    float bc = b[i / comps];
    float x = state[i];
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t t = t_begin + s;
        float xi = (float)xi_num(key, (uint64_t)t, (uint64_t)i) * 0x1p-20f;
        if (t == 0)
            x = __fmul_rn(sigma, xi);
        else
            x = __builtin_fmaf(ac, x, __fmul_rn(bc, xi));
        out[s * out_stride + i] = x;
    }
    state[i] = x;
}

__global__ void ou_f64_kernel(uint64_t key, int64_t n, int comps, const double* __restrict__ a,
                              const double* __restrict__ b, double sigma, int64_t t_begin,
                              int64_t n_steps, double* __restrict__ state,
                              double* __restrict__ out, int64_t out_stride)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double ac = a[i / comps];
    double bc = b[i / comps];
    double x = state[i];
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t t = t_begin + s;
        double xi = (double)xi_num(key, (uint64_t)t, (uint64_t)i) * 0x1p-20;
        if (t == 0)
            x = __dmul_rn(sigma, xi);
        else
            x = __builtin_fma(ac, x, __dmul_rn(bc, xi));
        out[s * out_stride + i] = x;
    }
    state[i] = x;
}

__global__ void positions_kernel(uint64_t key, int64_t n3, const float* __restrict__ r0, float a_d,
                                 float b_d, float sigma_d, int64_t t_begin, int64_t n_steps,
                                 float* __restrict__ d_state, float* __restrict__ out,
                                 int64_t out_stride)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n3) return;
    float d = d_state[c];
    const float base = r0[c];
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t t = t_begin + s;
        float xi = (float)xi_num(key, (uint64_t)t, (uint64_t)c) * 0x1p-20f;
        if (t == 0)
            d = __fmul_rn(sigma_d, xi);
        else
            d = __builtin_fmaf(a_d, d, __fmul_rn(b_d, xi));
        out[s * out_stride + c] = __fadd_rn(base, d);
    }
    d_state[c] = d;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

// All pointers are device pointers; `stream` is a hipStream_t (may be NULL).
// out_stride is the element distance between consecutive steps in `out`.
// Returns 0 on success, else the hipError_t of the launch.
int synth_gpu_ou_f32(uint64_t key, int64_t n, int comps, const float* a, const float* b,
                     float sigma, int64_t t_begin, int64_t n_steps, float* state, float* out,
                     int64_t out_stride, void* stream)
{
    if (n <= 0 || n_steps <= 0) return 0;
    hipLaunchKernelGGL(ou_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, key,
                       n, comps, a, b, sigma, t_begin, n_steps, state, out, out_stride);
    return (int)hipGetLastError();
}

int synth_gpu_ou_f64(uint64_t key, int64_t n, int comps, const double* a, const double* b,
                     double sigma, int64_t t_begin, int64_t n_steps, double* state, double* out,
                     int64_t out_stride, void* stream)
{
    if (n <= 0 || n_steps <= 0) return 0;
    hipLaunchKernelGGL(ou_f64_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, key,
                       n, comps, a, b, sigma, t_begin, n_steps, state, out, out_stride);
    return (int)hipGetLastError();
}

int synth_gpu_positions(uint64_t key, int64_t n_atoms, const float* r0, float a_d, float b_d,
                        float sigma_d, int64_t t_begin, int64_t n_steps, float* d_state,
                        float* out, int64_t out_stride, void* stream)
{
    int64_t n3 = 3 * n_atoms;
    if (n3 <= 0 || n_steps <= 0) return 0;
    hipLaunchKernelGGL(positions_kernel, dim3(blocks_for(n3)), dim3(256), 0, (hipStream_t)stream,
                       key, n3, r0, a_d, b_d, sigma_d, t_begin, n_steps, d_state, out, out_stride);
    return (int)hipGetLastError();
}

}  // extern "C"
