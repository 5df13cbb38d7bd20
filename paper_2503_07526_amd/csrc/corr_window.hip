// corr_window.hip -- block-deferred form of a long one-level window.
//
// A one-level group with p points (Algorithm 1 with b = 1: lags 0..p-1 of the
// raw series) costs p products per channel per push, and updating all p
// accumulators on every push moves every accumulator row through HBM once per
// push.  The sums are linear, so the products of kWindowT consecutive pushes
// can be added in one pass: each push only stages its sample in a ring of
// P0 = p + 2 kWindowT slots (written by the fold kernel of the push), and the lag
// range is cut into kWindowT lag blocks of lpb = ceil(p / kWindowT) lags.  At
// push kWindowT q + j, lag block j folds block q (pushes kWindowT (q-1) + 1 ..
// kWindowT q) of every channel: the kWindowT x lpb products x_s conj(x_{s-L})
// are summed in registers and added once to the stored accumulators.  Every
// push therefore does the same work (p products per channel, 1/kWindowT of the
// accumulator rows), and each accumulator row is read and written once per
// kWindowT pushes.
//
// Ring: value v (1-based) sits in slot (v - 1) mod P0; the fold kernel of
// push v writes it there (no separate staging launch).  When lag block j
// folds block q at push kWindowT q + j, the oldest value it reads is
// kWindowT (q - 1) + 1 - (p - 1), and the slots still hold every value from
// kWindowT q + j - P0 + 1 on, which is older for every j < kWindowT.  Values
// before the first push (v <= 0) map to slots that have not been written
// yet and read as the zeros the state is created with, so the products of
// lags longer than the series add nothing, as the counts max(0, S - L) say.
//
// A readout adds, for lag L of lag block j, the products of the pushes after
// the last block that lag block folded (at most 2 kWindowT - 2 of them) on the
// fly from the ring, without writing state (corr_reduce.hip).
//
// Threads: a wave holds 64 consecutive channels (one per lane) and a
// sub-block of LB consecutive lags of lag block j (LB = 8, or 4 when the
// grid would be small); the waves of a block (and blockIdx.y) cover the
// sub-blocks.  The block first copies the values its waves read into LDS,
// once each: the kWindowT new values of the folded block and the
// kWindowT + (lags of the block) - 1 lagged values, as rows of 64 channels
// (the waves' lagged ranges overlap, and every wave reads the same new
// values; read straight from the ring, each value was loaded about 18 times
// per push for the 4-lag waves of a long window).  Each lane then keeps LB
// partial sums and a sliding window of LB - 1 + U lagged values in registers:
// per U pushes it reads U new and U lagged values from LDS and does U x LB
// products.  Two windows of one kind and length can share a launch, the
// second's channel blocks after the first's (a few thousand channels alone
// hold only about one wave per SIMD).
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

// Sample type S, accumulator element A, partial-sum precision PT, planes NP.
template <int K> struct WK;
template <> struct WK<K_F32_F64>    { using S = float;  using A = double;  using PT = double; static constexpr int NP = 1; };
template <> struct WK<K_F32_KAHAN>  { using S = float;  using A = float;   using PT = float;  static constexpr int NP = 2; };
template <> struct WK<K_F32_F32>    { using S = float;  using A = float;   using PT = float;  static constexpr int NP = 1; };
template <> struct WK<K_CF32_F64>   { using S = float2; using A = double2; using PT = double; static constexpr int NP = 1; };
template <> struct WK<K_CF32_KAHAN> { using S = float2; using A = float2;  using PT = float;  static constexpr int NP = 2; };
template <> struct WK<K_CF32_F32>   { using S = float2; using A = float2;  using PT = float;  static constexpr int NP = 1; };

// Partial sum of one lag: (re, im); real kinds use re only.
template <typename PT> struct Part { PT re, im; };

// part += x * conj(y) in the partial-sum precision (single-precision
// products are exact in double).
__device__ __forceinline__ void mac(Part<float> &p, float x, float y) { p.re = __builtin_fmaf(x, y, p.re); }
__device__ __forceinline__ void mac(Part<double> &p, float x, float y)
{
    p.re = __builtin_fma((double)x, (double)y, p.re);
}
__device__ __forceinline__ void mac(Part<float> &p, float2 x, float2 y)
{
    p.re = __builtin_fmaf(x.x, y.x, __builtin_fmaf(x.y, y.y, p.re));
    p.im = __builtin_fmaf(x.y, y.x, __builtin_fmaf(-x.x, y.y, p.im));
}
__device__ __forceinline__ void mac(Part<double> &p, float2 x, float2 y)
{
    const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
    p.re = __builtin_fma(xr, yr, __builtin_fma(xi, yi, p.re));
    p.im = __builtin_fma(xi, yr, __builtin_fma(-xr, yi, p.im));
}

// Add a partial sum to a stored accumulator element (compensated kinds: one
// Kahan step per component, true value h - c).
__device__ __forceinline__ void kahan(float &h, float &c, float v)
{
    const float y = v - c;
    const float t = h + y;
    c = (t - h) - y;
    h = t;
}
template <int K> struct Fold;
template <> struct Fold<K_F32_F64> {
    static __device__ __forceinline__ void add(double &h, double &, const Part<double> &p) { h += p.re; }
};
template <> struct Fold<K_F32_KAHAN> {
    static __device__ __forceinline__ void add(float &h, float &c, const Part<float> &p) { kahan(h, c, p.re); }
};
template <> struct Fold<K_F32_F32> {
    static __device__ __forceinline__ void add(float &h, float &, const Part<float> &p) { h += p.re; }
};
template <> struct Fold<K_CF32_F64> {
    static __device__ __forceinline__ void add(double2 &h, double2 &, const Part<double> &p)
    {
        h.x += p.re;
        h.y += p.im;
    }
};
template <> struct Fold<K_CF32_KAHAN> {
    static __device__ __forceinline__ void add(float2 &h, float2 &c, const Part<float> &p)
    {
        kahan(h.x, c.x, p.re);
        kahan(h.y, c.y, p.im);
    }
};
template <> struct Fold<K_CF32_F32> {
    static __device__ __forceinline__ void add(float2 &h, float2 &, const Part<float> &p)
    {
        h.x += p.re;
        h.y += p.im;
    }
};

// Streaming loads and stores of accumulator elements (touched once per
// kWindowT pushes); the complex types go through clang vector types.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float nt_load(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double nt_load(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float2 nt_load(const float2 *p)
{
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 nt_load(const double2 *p)
{
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void nt_store(float v, float *p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(double v, double *p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(float2 v, float2 *p)
{
    __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v *>(p));
}
__device__ __forceinline__ void nt_store(double2 v, double2 *p)
{
    __builtin_nontemporal_store(d2v{v.x, v.y}, reinterpret_cast<d2v *>(p));
}

// Pushes per register window step.
constexpr int kWinU = 8;

__device__ __forceinline__ int wrap_slot(int64_t v, int p0)
{
    // slot of value v (1-based; v may be <= 0): (v - 1) mod p0 in [0, p0)
    int64_t r = (v - 1) % p0;
    if (r < 0) r += p0;
    return (int)r;
}

// Blocks x < x1 fold window g0, the others window g1 (two windows of one
// kind and length share a launch; a single window passes itself twice).
template <int K, int LB>
__global__ __launch_bounds__(512) void window_fold_kernel(GroupArgs g0, GroupArgs g1, int x1,
                                                          const int64_t *step, int lpb, int subs_per_block)
{
    using S = typename WK<K>::S;
    using A = typename WK<K>::A;
    using PT = typename WK<K>::PT;
    constexpr int NP = WK<K>::NP;
    constexpr int U = kWinU;
    constexpr int T = kWindowT;
    extern __shared__ __align__(16) unsigned char win_lds[];
    S *const rows = reinterpret_cast<S *>(win_lds); // [row][64 channels]

    // Push P = *step + 1: its sample goes to ring slot (P - 1) mod p0 (the
    // first wave of each channel group's y = 0 block writes it; the blocks of
    // this launch that need value P read it from the input instead, and none
    // reads that slot for an older value: the oldest value folded is newer
    // than P - p0).  Then lag block j folds block q.
    const int64_t P = *step + 1;
    const bool second = (int)blockIdx.x >= x1; // uniform over the block
    const int tw = second ? g1.tw : g0.tw;
    const int p0 = second ? g1.p0 : g0.p0;
    const int np = second ? g1.p : g0.p;
    const int64_t n_ch = second ? g1.n_ch : g0.n_ch;
    const int64_t tile_bytes = second ? g1.tile_bytes : g0.tile_bytes;
    char *const state = second ? g1.state : g0.state;
    const S *const samples = static_cast<const S *>(second ? g1.samples : g0.samples);
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t ch = (int64_t)((int)blockIdx.x - (second ? x1 : 0)) * 64 + lane;
    const int64_t tile = ch / tw;
    const int tl = (int)(ch - tile * tw);
    char *tb = state + tile * tile_bytes;
    S *const ring = reinterpret_cast<S *>(tb) + tl;
    // channels past the end of the group (the padded tail) hold zeros
    const S xP = ch < n_ch ? samples[ch] : S{};
    if (blockIdx.y == 0 && wave == 0) ring[(size_t)wrap_slot(P, p0) * tw] = xP;

    const int j = (int)(P % T);
    const int64_t q = P / T;
    if (q < 1) return;
    const int nwaves = (int)(blockDim.x >> 6);
    const int lag_end = min((j + 1) * lpb, np);
    const int Lb0 = j * lpb + (int)blockIdx.y * subs_per_block * LB; // the block's first lag
    if (Lb0 >= lag_end) return; // whole block
    const int L0 = Lb0 + wave * LB;

    // Rows 0 .. T-1: the new values s0 .. s0 + T - 1.  Rows T .. : the lagged
    // values from v_lo = s0 - Lb0 - (span - 1) on, span = the block's lags
    // (some past lag_end in the last block: read, never used).
    const int64_t s0 = (q - 1) * T + 1;
    const int span = nwaves * LB;
    const int64_t v_lo = s0 - Lb0 - (span - 1);
    const int n_rows = 2 * T + span - 1;
    for (int r = wave; r < n_rows; r += nwaves) {
        const int64_t v = r < T ? s0 + r : v_lo + (r - T);
        rows[(size_t)r * 64 + lane] = v == P ? xP : ring[(size_t)wrap_slot(v, p0) * tw];
    }
    __syncthreads();
    if (L0 >= lag_end) return; // this wave's lags are past the lag block
    const int nl = min(LB, lag_end - L0);

    // Lagged value s0 + i - L0 - l (push s0 + i, lag L0 + l) sits in row
    // wb + i - l with wb = T + span - 1 - wave LB; the window W[LB - 1 + u]
    // holds the value of row wb + i + u.
    const int wb = T + span - 1 - wave * LB;
    S W[LB - 1 + U];
#pragma unroll
    for (int k = 0; k < LB - 1; ++k) W[k] = rows[(size_t)(wb - (LB - 1) + k) * 64 + lane];
    Part<PT> part[LB];
#pragma unroll
    for (int l = 0; l < LB; ++l) part[l] = Part<PT>{PT(0), PT(0)};
#pragma unroll 1
    for (int i = 0; i < T; i += U) {
        S N[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            N[u] = rows[(size_t)(i + u) * 64 + lane];
            W[LB - 1 + u] = rows[(size_t)(wb + i + u) * 64 + lane];
        }
        // push s = s0 + i + u, lag L0 + l: lagged value s - L0 - l = W[LB - 1 + u - l]
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int l = 0; l < LB; ++l) mac(part[l], N[u], W[LB - 1 + u - l]);
#pragma unroll
        for (int k = 0; k < LB - 1; ++k) W[k] = W[k + U];
    }

    A *hi = reinterpret_cast<A *>(tb + (int64_t)p0 * tw * (int64_t)sizeof(S)) + tl;
    A *lo = hi + (size_t)np * tw;
#pragma unroll
    for (int l = 0; l < LB; ++l) {
        if (l < nl) {
            const size_t r = (size_t)(L0 + l) * tw;
            A h = nt_load(&hi[r]);
            A c{};
            if constexpr (NP == 2) c = nt_load(&lo[r]);
            Fold<K>::add(h, c, part[l]);
            nt_store(h, &hi[r]);
            if constexpr (NP == 2) nt_store(c, &lo[r]);
        }
    }
}

// Waves of the eight-lag form from which it is preferred (4 per SIMD of a
// 256-CU device).
constexpr int64_t kWindowWideWaves = 4096;

struct WindowShape {
    int lpb, subs_per_block;
    unsigned grid_x, grid_y, block;
};

// LDS rows of one block: 2 kWindowT + (waves) LB - 1 rows of 64 samples, at
// most kWinLdsBytes so that two blocks share a CU.
constexpr size_t kWinLdsBytes = 80 * 1024;

size_t window_lds_bytes(const GroupArgs &g, int lb, int subs_per_block)
{
    const size_t sb = g.kind == K_CF32_F64 || g.kind == K_CF32_KAHAN || g.kind == K_CF32_F32 ? 8 : 4;
    return (size_t)(2 * kWindowT + subs_per_block * lb - 1) * 64 * sb;
}

WindowShape window_shape(const GroupArgs &g, int lb)
{
    WindowShape w{};
    w.lpb = (g.p + kWindowT - 1) / kWindowT;
    const int n_sub = (w.lpb + lb - 1) / lb;
    int cap = 8; // at most 8 waves per block, and the block's rows within kWinLdsBytes
    while (cap > 1 && window_lds_bytes(g, lb, cap) > kWinLdsBytes) --cap;
    const int by = (n_sub + cap - 1) / cap;
    w.subs_per_block = (n_sub + by - 1) / by;
    w.grid_x = (unsigned)(g.n_tiles * g.tw / 64);
    w.grid_y = (unsigned)by;
    w.block = (unsigned)(64 * w.subs_per_block);
    return w;
}

// The kernel of kind K with LB lags per wave, allowed kWinLdsBytes of LDS
// (above the 64 KiB default; set once per kernel, no stream operation).
template <int K, int LB> const void *window_kernel()
{
    const void *fn = reinterpret_cast<const void *>(&window_fold_kernel<K, LB>);
    static const hipError_t set =
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWinLdsBytes);
    return set == hipSuccess ? fn : nullptr;
}

// One launch of window g0 and, when g1 is given (same kind and length), of
// window g1 in the blocks after g0's.
template <int LB>
hipError_t launch_fold_lb(const GroupArgs &g0, const GroupArgs *g1, const int64_t *step, hipStream_t st)
{
    const WindowShape w = window_shape(g0, LB);
    const unsigned x1 = w.grid_x;
    const unsigned gx = x1 + (g1 ? window_shape(*g1, LB).grid_x : 0u);
    const dim3 grid(gx, w.grid_y), block(w.block);
    const size_t lds = window_lds_bytes(g0, LB, w.subs_per_block);
    if (lds > kWinLdsBytes) return hipErrorInvalidValue;
    const void *fn = nullptr;
    switch (g0.kind) {
    case K_F32_F64: fn = window_kernel<K_F32_F64, LB>(); break;
    case K_F32_KAHAN: fn = window_kernel<K_F32_KAHAN, LB>(); break;
    case K_F32_F32: fn = window_kernel<K_F32_F32, LB>(); break;
    case K_CF32_F64: fn = window_kernel<K_CF32_F64, LB>(); break;
    case K_CF32_KAHAN: fn = window_kernel<K_CF32_KAHAN, LB>(); break;
    case K_CF32_F32: fn = window_kernel<K_CF32_F32, LB>(); break;
    default: return hipErrorInvalidValue;
    }
    if (!fn) return hipErrorInvalidValue;
    GroupArgs ga = g0, gb = g1 ? *g1 : g0;
    int xs = (int)x1;
    const int64_t *sp = step;
    int lpb = w.lpb, spb = w.subs_per_block;
    void *args[] = {&ga, &gb, &xs, &sp, &lpb, &spb};
    return hipLaunchKernel(fn, grid, block, args, lds, st);
}

bool window_fold_valid(const GroupArgs &g)
{
    return g.levels == 1 && g.deferred && !g.pair && g.tw % 64 == 0 && g.p0 == g.p + 2 * kWindowT;
}

// Eight lags per wave reuse each loaded value more; four give twice the waves,
// which wins while the grid holds fewer than four waves per SIMD (a few
// thousand channels, the k-space groups of long windows).
hipError_t launch_fold(const GroupArgs &g0, const GroupArgs *g1, const int64_t *step, hipStream_t st)
{
    const WindowShape w8 = window_shape(g0, 8);
    const unsigned gx = w8.grid_x + (g1 ? window_shape(*g1, 8).grid_x : 0u);
    const int64_t waves8 = (int64_t)gx * w8.grid_y * w8.subs_per_block;
    if (waves8 < kWindowWideWaves) return launch_fold_lb<4>(g0, g1, step, st);
    return launch_fold_lb<8>(g0, g1, step, st);
}

} // namespace

bool window_deferred_supported(int kind)
{
    return kind == K_F32_F64 || kind == K_F32_KAHAN || kind == K_F32_F32 || kind == K_CF32_F64 ||
           kind == K_CF32_KAHAN || kind == K_CF32_F32;
}

int window_lags_per_block(int p) { return (p + kWindowT - 1) / kWindowT; }

hipError_t launch_window_fold(const GroupArgs &g, const int64_t *step, hipStream_t st)
{
    if (!window_fold_valid(g)) return hipErrorInvalidValue;
    return launch_fold(g, nullptr, step, st);
}

bool window_folds_share_launch(const GroupArgs &a, const GroupArgs &b)
{
    // the same kernel and block shape: kind (sample and accumulator types) and
    // length (lags per lag block, LDS rows)
    return a.kind == b.kind && a.p == b.p;
}

hipError_t launch_window_fold2(const GroupArgs &a, const GroupArgs &b, const int64_t *step, hipStream_t st)
{
    if (!window_fold_valid(a) || !window_fold_valid(b) || !window_folds_share_launch(a, b))
        return hipErrorInvalidValue;
    return launch_fold(a, &b, step, st);
}

} // namespace corr
