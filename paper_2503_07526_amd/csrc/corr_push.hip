// corr_push.hip -- per-step correlator update on gfx950.
//
// One push is Algorithm 1 of the paper's Appendix D called with block index
// 1 for every channel: write the newest sample into the level-0 ring,
// accumulate x * conj(ring[lag L]) for L = 0..min(S, p)-1, and, every m^k
// pushes, average the last m values of level k-1 into level k and
// accumulate lags floor(p/m)..p-1 there.  All channels of a group receive the
// same number of pushes, so the ring cursors, fill levels and counts of the
// algorithm are the same for every channel and follow from the push index
// alone: level k has received S_k = floor(S / m^k) values, its newest value
// sits in slot (S_k - 1) mod p, and lag L of level k has count
// max(0, S_k - L).  No per-channel integer state exists; the averaging
// accumulator of Algorithm 1 is replaced by the last m ring values of the
// level above (p > m, so they are always still in the ring).
//
// Threads own channels (one to four consecutive channels each); a block owns
// a tile of the state laid out structure-of-arrays (corr_internal.h), so the
// lanes of a wave read and write whole consecutive cache lines of every ring
// and accumulator row.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

// Whole-vector loads and stores of N consecutive elements (N * sizeof(T) is
// 4..64 bytes and naturally aligned by the tile layout): moved as a vector of
// dwords so that each lane issues 16-byte memory instructions.
template <typename T, int N>
__device__ __forceinline__ void vload(const T *p, T (&out)[N])
{
    constexpr int W = (int)(sizeof(T) * N / 4);
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    const V v = *reinterpret_cast<const V *>(p);
    __builtin_memcpy(&out[0], &v, sizeof(T) * N);
}

template <typename T, int N>
__device__ __forceinline__ void vstore(T *p, const T (&in)[N])
{
    constexpr int W = (int)(sizeof(T) * N / 4);
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    V v;
    __builtin_memcpy(&v, &in[0], sizeof(T) * N);
    *reinterpret_cast<V *>(p) = v;
}

// The same, non-temporal: for the accumulator rows of a group whose state is
// larger than the last-level cache, which a push reads and writes once and no
// later push touches before the whole state has streamed past the caches
// (the plain 3e6-channel push 267 against 294 us: the ring, which the next
// p - 1 pushes read again and which keeps ordinary loads, then stays cached).
// A smaller group keeps its accumulators cached from push to push.
template <typename T, int N>
__device__ __forceinline__ void vload_nt(const T *p, T (&out)[N])
{
    constexpr int W = (int)(sizeof(T) * N / 4);
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    __builtin_memcpy(&out[0], &v, sizeof(T) * N);
}

template <typename T, int N>
__device__ __forceinline__ void vstore_nt(T *p, const T (&in)[N])
{
    constexpr int W = (int)(sizeof(T) * N / 4);
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    V v;
    __builtin_memcpy(&v, &in[0], sizeof(T) * N);
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}

// A group whose state is above this size streams its accumulator rows (the
// device's last-level cache holds 256 MB).  The choice is a template argument
// of the kernel: a branch between the two forms of the same load lets the
// compiler merge them and drop the non-temporal hint.
constexpr int64_t kStreamAccBytes = (int64_t)256 << 20;
static bool stream_acc(const GroupArgs &g) { return g.n_tiles * g.tile_bytes > kStreamAccBytes; }

// ---------------------------------------------------------------- kinds
template <int K> struct KT;
template <> struct KT<K_F32_F64>    { using S = float;   using A = double;  static constexpr int NP = 1; };
template <> struct KT<K_F32_KAHAN>  { using S = float;   using A = float;   static constexpr int NP = 2; };
template <> struct KT<K_F32_F32>    { using S = float;   using A = float;   static constexpr int NP = 1; };
template <> struct KT<K_F64_F64>    { using S = double;  using A = double;  static constexpr int NP = 1; };
template <> struct KT<K_CF32_F64>   { using S = float2;  using A = double2; static constexpr int NP = 1; };
template <> struct KT<K_CF32_KAHAN> { using S = float2;  using A = float2;  static constexpr int NP = 2; };
template <> struct KT<K_CF32_F32>   { using S = float2;  using A = float2;  static constexpr int NP = 1; };
template <> struct KT<K_CF64_F64>   { using S = double2; using A = double2; static constexpr int NP = 1; };

// Sample arithmetic used by the block average (sum in push order, then / m).
__device__ __forceinline__ float sadd(float a, float b) { return a + b; }
__device__ __forceinline__ double sadd(double a, double b) { return a + b; }
__device__ __forceinline__ float2 sadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float sdiv(float a, int m) { return a / (float)m; }
__device__ __forceinline__ double sdiv(double a, int m) { return a / (double)m; }
__device__ __forceinline__ float2 sdiv(float2 a, int m) { return make_float2(a.x / (float)m, a.y / (float)m); }
__device__ __forceinline__ double2 sdiv(double2 a, int m) { return make_double2(a.x / (double)m, a.y / (double)m); }
template <typename S> __device__ __forceinline__ S szero();
template <> __device__ __forceinline__ float szero<float>() { return 0.0f; }
template <> __device__ __forceinline__ double szero<double>() { return 0.0; }
template <> __device__ __forceinline__ float2 szero<float2>() { return make_float2(0.0f, 0.0f); }
template <> __device__ __forceinline__ double2 szero<double2>() { return make_double2(0.0, 0.0); }

// sum += x * conj(r) in the accumulator precision of kind K.  The compensated
// form is Kahan summation with the product folded into the first step:
// y = x*r - c (one rounding), t = h + y, c = (t - h) - y, h = t; the true sum is
// h - c.
template <int K> struct Acc;
template <> struct Acc<K_F32_F64> {
    static __device__ __forceinline__ void add(double &h, double &, float x, float r)
    { h = __builtin_fma((double)x, (double)r, h); }
};
template <> struct Acc<K_F32_KAHAN> {
    static __device__ __forceinline__ void add(float &h, float &c, float x, float r)
    {
        float y = __builtin_fmaf(x, r, -c);
        float t = h + y;
        c = (t - h) - y;
        h = t;
    }
};
template <> struct Acc<K_F32_F32> {
    static __device__ __forceinline__ void add(float &h, float &, float x, float r)
    { h = __builtin_fmaf(x, r, h); }
};
template <> struct Acc<K_F64_F64> {
    static __device__ __forceinline__ void add(double &h, double &, double x, double r)
    { h = __builtin_fma(x, r, h); }
};
template <> struct Acc<K_CF32_F64> {
    static __device__ __forceinline__ void add(double2 &h, double2 &, float2 x, float2 r)
    {
        const double xr = x.x, xi = x.y, rr = r.x, ri = r.y;
        h.x = __builtin_fma(xr, rr, __builtin_fma(xi, ri, h.x));
        h.y = __builtin_fma(xi, rr, __builtin_fma(-xr, ri, h.y));
    }
};
template <> struct Acc<K_CF32_KAHAN> {
    static __device__ __forceinline__ void add(float2 &h, float2 &c, float2 x, float2 r)
    {
        float yr = __builtin_fmaf(x.x, r.x, __builtin_fmaf(x.y, r.y, -c.x));
        float yi = __builtin_fmaf(x.y, r.x, __builtin_fmaf(-x.x, r.y, -c.y));
        float tr = h.x + yr;
        float ti = h.y + yi;
        c.x = (tr - h.x) - yr;
        c.y = (ti - h.y) - yi;
        h.x = tr;
        h.y = ti;
    }
};
template <> struct Acc<K_CF32_F32> {
    static __device__ __forceinline__ void add(float2 &h, float2 &, float2 x, float2 r)
    {
        h.x = __builtin_fmaf(x.x, r.x, __builtin_fmaf(x.y, r.y, h.x));
        h.y = __builtin_fmaf(x.y, r.x, __builtin_fmaf(-x.x, r.y, h.y));
    }
};
template <> struct Acc<K_CF64_F64> {
    static __device__ __forceinline__ void add(double2 &h, double2 &, double2 x, double2 r)
    {
        h.x = __builtin_fma(x.x, r.x, __builtin_fma(x.y, r.y, h.x));
        h.y = __builtin_fma(x.y, r.x, __builtin_fma(-x.x, r.y, h.y));
    }
};

// NJ consecutive lags [L0, L0 + NJ) of one level, branch-free: all loads of
// the chunk are issued before any arithmetic so that each lane has many
// independent memory requests in flight.  Lag L reads ring slot
// (slot - L) mod p of the lagged series; lag 0 takes the newest lagged value
// y0 from registers (y0 = x for an autocorrelation).
template <int K, int CPT, int NJ, bool NTA>
__device__ __forceinline__ void lag_chunk(const typename KT<K>::S (&x)[CPT],
                                          const typename KT<K>::S (&y0)[CPT],
                                          const typename KT<K>::S *ring, typename KT<K>::A *hi,
                                          typename KT<K>::A *lo, int slot, int p, int L0,
                                          int row_base, int tw, int lane_off)
{
    using S = typename KT<K>::S;
    using A = typename KT<K>::A;
    constexpr int NP = KT<K>::NP;
    S r[NJ][CPT];
    A h[NJ][CPT];
    A c[NJ][CPT];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        int sl = slot - (L0 + j);
        if (sl < 0) sl += p;
        vload<S, CPT>(ring + (size_t)sl * tw + lane_off, r[j]);
        const size_t ro = (size_t)(L0 + j - row_base) * tw + lane_off;
        if constexpr (NTA) {
            vload_nt<A, CPT>(hi + ro, h[j]);
            if constexpr (NP == 2) vload_nt<A, CPT>(lo + ro, c[j]);
        } else {
            vload<A, CPT>(hi + ro, h[j]);
            if constexpr (NP == 2) vload<A, CPT>(lo + ro, c[j]);
        }
    }
    if (L0 == 0) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) r[0][i] = y0[i];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) Acc<K>::add(h[j][i], c[j][i], x[i], r[j][i]);
        const size_t ro = (size_t)(L0 + j - row_base) * tw + lane_off;
        if constexpr (NTA) {
            vstore_nt<A, CPT>(hi + ro, h[j]);
            if constexpr (NP == 2) vstore_nt<A, CPT>(lo + ro, c[j]);
        } else {
            vstore<A, CPT>(hi + ro, h[j]);
            if constexpr (NP == 2) vstore<A, CPT>(lo + ro, c[j]);
        }
    }
}

// Lag loop of one level: lags [l_begin, l_end), accumulator row L - row_base.
// Full chunks of LCH lags, then chunks of 4, then single lags.
template <int K, int CPT, int LCH, bool NTA>
__device__ __forceinline__ void lag_loop(const typename KT<K>::S (&x)[CPT],
                                         const typename KT<K>::S (&y0)[CPT],
                                         const typename KT<K>::S *ring, typename KT<K>::A *hi,
                                         typename KT<K>::A *lo, int slot, int p, int l_begin,
                                         int l_end, int row_base, int tw, int lane_off)
{
    int L = l_begin;
#pragma unroll 1
    for (; L + LCH <= l_end; L += LCH)
        lag_chunk<K, CPT, LCH, NTA>(x, y0, ring, hi, lo, slot, p, L, row_base, tw, lane_off);
    if constexpr (LCH > 4) {
#pragma unroll 1
        for (; L + 4 <= l_end; L += 4)
            lag_chunk<K, CPT, 4, NTA>(x, y0, ring, hi, lo, slot, p, L, row_base, tw, lane_off);
    }
#pragma unroll 1
    for (; L < l_end; ++L)
        lag_chunk<K, CPT, 1, NTA>(x, y0, ring, hi, lo, slot, p, L, row_base, tw, lane_off);
}

// One push of one tile of one group.  s = 1-based push index.  PAIR: the
// group correlates (x, y) pairs (its own launches; the batched kernel only
// instantiates the autocorrelation form).  [lag_lo, lag_hi) restricts the
// level-0 lags this call adds; head: the call also writes the ring slots and
// runs the cascade (one head call per tile and push; the level-0 lags of a
// push never read the slot it writes, so the calls are independent).
template <int K, int CPT, int LCH, bool PAIR = false, bool NTA = false>
__device__ __forceinline__ void push_tile(const GroupArgs &g, int64_t tile, int64_t s,
                                          int lag_lo = 0, int lag_hi = 1 << 30, bool head = true)
{
    using S = typename KT<K>::S;
    using A = typename KT<K>::A;
    const int tw = g.tw;
    const int p = g.p;
    const int m = g.m;
    const int lane_off = (int)threadIdx.x * CPT;
    const int64_t ch0 = tile * (int64_t)tw + lane_off;

    // Samples of this push; channels past the end of the group read as 0 (the
    // state of the padded tail is allocated and never read out).  Pair
    // groups: x then y planes; otherwise y is x.
    S x[CPT], y[CPT];
    const S *src = static_cast<const S *>(g.samples);
#pragma unroll
    for (int i = 0; i < CPT; ++i) x[i] = (ch0 + i < g.n_ch) ? src[ch0 + i] : szero<S>();
#pragma unroll
    for (int i = 0; i < CPT; ++i)
        y[i] = PAIR ? ((ch0 + i < g.n_ch) ? src[g.n_ch + ch0 + i] : szero<S>()) : x[i];

    char *tb = g.state + tile * g.tile_bytes;
    const int64_t rowS = (int64_t)tw * (int64_t)sizeof(S);
    constexpr int rings = PAIR ? 2 : 1;

    if (g.deferred) {
        // Block-deferred group (or window): only stage the sample in the
        // level-0 ring of p0 slots; the flush pass folds a block of pushes at
        // once.
        S *ring = reinterpret_cast<S *>(tb);
        const int slot = (int)((s - 1) % g.p0);
        vstore<S, CPT>(ring + (size_t)slot * tw + lane_off, x);
        return;
    }

    // Level 0: ring write(s) and lags 0..min(s, p)-1.
    {
        S *ring = reinterpret_cast<S *>(tb);
        A *hi = reinterpret_cast<A *>(tb + (int64_t)rings * p * rowS);
        A *lo = hi + (size_t)p * tw;
        const int slot = (int)((s - 1) % p);
        if (head) {
            vstore<S, CPT>(ring + (size_t)slot * tw + lane_off, y);
            if constexpr (PAIR) vstore<S, CPT>(ring + (size_t)(p + slot) * tw + lane_off, x);
        }
        const int nlag = (int)(s < p ? s : p);
        const int l_end = lag_hi < nlag ? lag_hi : nlag;
        if (lag_lo < l_end)
            lag_loop<K, CPT, LCH, NTA>(x, y, ring, hi, lo, slot, p, lag_lo, l_end, 0, tw, lane_off);
    }
    if (!head) return;

    // Cascade: level k receives a value when m^k divides s.
    int kmax = 0;
    {
        int64_t q = s;
        while (kmax < g.levels - 1 && q % m == 0) {
            q /= m;
            ++kmax;
        }
    }
    // vprev: the newest value of level k-1 (y series; x series of pairs in vprevx)
    S vprev[CPT], vprevx[CPT];
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
        vprev[i] = y[i];
        vprevx[i] = x[i];
    }
    int64_t s_prev = s;
    const char *lvl_prev = tb;
    const int lag0 = g.lag0;
    const int nlk = p - lag0;
    // Mean of the last m values of one ring of level k-1, summed oldest first
    // (the newest is in registers).
    auto block_mean = [&](const S *ringp, int slotp, const S (&newest)[CPT], S (&v)[CPT]) {
        int sl = slotp - (m - 1);
        if (sl < 0) sl += p;
        vload<S, CPT>(ringp + (size_t)sl * tw + lane_off, v);
#pragma unroll 1
        for (int j = m - 2; j >= 1; --j) {
            int sj = slotp - j;
            if (sj < 0) sj += p;
            S t[CPT];
            vload<S, CPT>(ringp + (size_t)sj * tw + lane_off, t);
#pragma unroll
            for (int i = 0; i < CPT; ++i) v[i] = sadd(v[i], t[i]);
        }
#pragma unroll
        for (int i = 0; i < CPT; ++i) v[i] = sdiv(sadd(v[i], newest[i]), m);
    };
#pragma unroll 1
    for (int k = 1; k <= kmax; ++k) {
        const S *ringp = reinterpret_cast<const S *>(lvl_prev);
        const int slotp = (int)((s_prev - 1) % p);
        S v[CPT], vx[CPT];
        block_mean(ringp, slotp, vprev, v);
        if constexpr (PAIR)
            block_mean(ringp + (size_t)p * tw, slotp, vprevx, vx);
        else {
#pragma unroll
            for (int i = 0; i < CPT; ++i) vx[i] = v[i];
        }
        char *lvl = tb + g.lvl0_bytes + (int64_t)(k - 1) * g.lvlk_bytes;
        S *ring = reinterpret_cast<S *>(lvl);
        A *hi = reinterpret_cast<A *>(lvl + (int64_t)rings * p * rowS);
        A *lo = hi + (size_t)nlk * tw;
        const int64_t sk = s_prev / m;
        const int slot = (int)((sk - 1) % p);
        vstore<S, CPT>(ring + (size_t)slot * tw + lane_off, v);
        if constexpr (PAIR) vstore<S, CPT>(ring + (size_t)(p + slot) * tw + lane_off, vx);
        const int nl = (int)(sk < p ? sk : p);
        if (nl > lag0) lag_loop<K, CPT, LCH, NTA>(vx, v, ring, hi, lo, slot, p, lag0, nl, lag0, tw, lane_off);
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            vprev[i] = v[i];
            vprevx[i] = vx[i];
        }
        s_prev = sk;
        lvl_prev = lvl;
    }
}

template <int CPT, int LCH>
__device__ __forceinline__ void dispatch_tile(const GroupArgs &g, int64_t tile, int64_t s)
{
    switch (g.kind) {
    case K_F32_F64: push_tile<K_F32_F64, CPT, LCH>(g, tile, s); break;
    case K_F32_KAHAN: push_tile<K_F32_KAHAN, CPT, LCH>(g, tile, s); break;
    case K_F32_F32: push_tile<K_F32_F32, CPT, LCH>(g, tile, s); break;
    case K_F64_F64: push_tile<K_F64_F64, CPT, LCH>(g, tile, s); break;
    case K_CF32_F64: push_tile<K_CF32_F64, CPT, LCH>(g, tile, s); break;
    case K_CF32_KAHAN: push_tile<K_CF32_KAHAN, CPT, LCH>(g, tile, s); break;
    case K_CF32_F32: push_tile<K_CF32_F32, CPT, LCH>(g, tile, s); break;
    default: push_tile<K_CF64_F64, CPT, LCH>(g, tile, s); break;
    }
}

// Batched form: every group of the context in one launch.  Blocks stride over
// the concatenated tile space of all groups (a persistent grid when
// gridDim.x is smaller than the number of tiles).  Every kind is compiled
// into this kernel, so its register budget is that of the widest (complex
// double samples); it has no occupancy bound, which would make those spill.
template <int CPT, int LCH>
__global__ __launch_bounds__(256) void push_batched_kernel(PushArgs a)
{
    const int64_t s = *a.step + 1;
#pragma unroll 1
    for (int64_t t = blockIdx.x; t < a.total_tiles; t += gridDim.x) {
        int gi = 0;
        while (gi + 1 < a.n_groups && t >= a.g[gi + 1].tile_first) ++gi;
        // Copy the group's arguments with constant indices (keeps them in
        // scalar registers instead of a private copy of the whole table).
        GroupArgs g;
        switch (gi) {
        case 0: g = a.g[0]; break;
        case 1: g = a.g[1]; break;
        case 2: g = a.g[2]; break;
        case 3: g = a.g[3]; break;
        case 4: g = a.g[4]; break;
        case 5: g = a.g[5]; break;
        case 6: g = a.g[6]; break;
        default: g = a.g[7]; break;
        }
        dispatch_tile<CPT, LCH>(g, t - g.tile_first, s);
    }
}

// Plain form: one group per launch, one block per tile, kind fixed at compile
// time (NTA: accumulator rows streamed, for groups larger than the cache).
template <int K, int CPT, int LCH, bool PAIR, bool NTA>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void push_group_kernel(GroupArgs g, const int64_t *step)
{
    const int64_t s = *step + 1;
    push_tile<K, CPT, LCH, PAIR, NTA>(g, (int64_t)blockIdx.x, s);
}

// Group with few tiles: the level-0 lags of a push split over blockIdx.y
// (lags_per_block each), so that more than one block per tile works on it;
// block y = 0 also writes the ring slots and runs the cascade.
template <int K, int CPT, int LCH>
__global__ __launch_bounds__(256) void push_split_kernel(GroupArgs g, const int64_t *step, int lags_per_block)
{
    const int64_t s = *step + 1;
    const int lo = (int)blockIdx.y * lags_per_block;
    push_tile<K, CPT, LCH>(g, (int64_t)blockIdx.x, s, lo, lo + lags_per_block, blockIdx.y == 0);
}

// One-level group with a long window: one push, with the lag range split
// over blockIdx.y (lags [y * lags_per_block, ...)) so that the grid has
// enough blocks when there are few channels.  Lag L >= 1 reads ring slot
// (slot - L) mod p, never the slot this push writes (that would be lag p), so
// the chunks are independent; chunk 0 writes the new sample.
template <int K, int CPT, int LCH, bool PAIR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void push_window_kernel(GroupArgs g, const int64_t *step, int lags_per_block)
{
    using S = typename KT<K>::S;
    using A = typename KT<K>::A;
    const int64_t s = *step + 1;
    const int64_t tile = blockIdx.x;
    const int tw = g.tw, p = g.p;
    const int lane_off = (int)threadIdx.x * CPT;
    const int64_t ch0 = tile * (int64_t)tw + lane_off;
    S x[CPT], y[CPT];
    const S *src = static_cast<const S *>(g.samples);
#pragma unroll
    for (int i = 0; i < CPT; ++i) x[i] = (ch0 + i < g.n_ch) ? src[ch0 + i] : szero<S>();
#pragma unroll
    for (int i = 0; i < CPT; ++i)
        y[i] = PAIR ? ((ch0 + i < g.n_ch) ? src[g.n_ch + ch0 + i] : szero<S>()) : x[i];
    char *tb = g.state + tile * g.tile_bytes;
    const int64_t rowS = (int64_t)tw * (int64_t)sizeof(S);
    constexpr int rings = PAIR ? 2 : 1;
    S *ring = reinterpret_cast<S *>(tb);
    A *hi = reinterpret_cast<A *>(tb + (int64_t)rings * p * rowS);
    A *lo = hi + (size_t)p * tw;
    const int slot = (int)((s - 1) % p);
    if (blockIdx.y == 0) {
        vstore<S, CPT>(ring + (size_t)slot * tw + lane_off, y);
        if constexpr (PAIR) vstore<S, CPT>(ring + (size_t)(p + slot) * tw + lane_off, x);
    }
    const int nlag = (int)(s < p ? s : p);
    const int l_begin = (int)blockIdx.y * lags_per_block;
    const int l_end = l_begin + lags_per_block < nlag ? l_begin + lags_per_block : nlag;
    if (l_begin < l_end)
        lag_loop<K, CPT, LCH, false>(x, y, ring, hi, lo, slot, p, l_begin, l_end, 0, tw, lane_off);
}

// Last kernel of a push S = *step + 1: tile group S mod T of every
// block-deferred group has folded block S / T (its flush ran earlier in this
// push), then the counter advances.  After the folds of every tile group
// (a catch-up, or a block folded from a stored history) the record is that
// block for all tile groups, and the counter advances by the pushes the
// launch stands for (a whole history block when no group needs per-push
// work, else 0: those pushes ended with their own end kernels).
__global__ void push_end_kernel(PushEndArgs a)
{
    if (blockIdx.x != 0) return;
    if (a.stamps && stamp_sampled(a.stamps)) {
        // the lanes take the slots of both stamp records in turn; the earliest
        // start and the latest end give the push's span of each class
        __shared__ unsigned long long lo[64], hi[64];
        for (int r = 0; r < a.n_stamps; ++r) {
            FoldStamps &st = a.stamps[r];
            const int l = threadIdx.x;
            if (l < 64) {
                unsigned long long s0 = ~0ull, e0 = 0;
                for (int q = l; q < kStampSlots; q += 64) {
                    const unsigned long long a0 = st.slot[q].start, b0 = st.slot[q].end;
                    s0 = a0 < s0 ? a0 : s0;
                    e0 = b0 > e0 ? b0 : e0;
                    st.slot[q].start = ~0ull;
                    st.slot[q].end = 0;
                }
                lo[l] = s0;
                hi[l] = e0;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                unsigned long long s0 = ~0ull, e0 = 0;
                for (int q = 0; q < 64; ++q) {
                    s0 = lo[q] < s0 ? lo[q] : s0;
                    e0 = hi[q] > e0 ? hi[q] : e0;
                }
                if (e0 > s0) {
                    st.total += e0 - s0;
                    st.count += 1;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x != 0) return;
    const int64_t S = *a.step + 1;
    for (int i = 0; i < a.n_flushed; ++i) {
        const int T = a.defer_t[i];
        if (a.commit_block >= 1) {
            // every tile group folded block commit_block
            for (int j = 0; j < T; ++j)
                if (a.flushed[i][j] < a.commit_block) a.flushed[i][j] = a.commit_block;
        } else {
            const int j = (int)(S % T);
            const int64_t q = S / T;
            if (q >= 1 && a.flushed[i][j] < q) a.flushed[i][j] = q;
        }
    }
    *a.step += a.advance;
    if (a.step2) *a.step2 += a.advance;
}

// ------------------------------------------------------------ host launchers
template <int CPT, int LCH>
static hipError_t launch_batched_t(const PushArgs &a, int grid, int block, hipStream_t st)
{
    hipLaunchKernelGGL((push_batched_kernel<CPT, LCH>), dim3(grid), dim3(block), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_push_batched(const PushArgs &a, int cpt, int lch, int grid, int block,
                               hipStream_t st)
{
    if (cpt == 1 && lch == 16) return launch_batched_t<1, 16>(a, grid, block, st);
    if (cpt == 1 && lch == 8) return launch_batched_t<1, 8>(a, grid, block, st);
    if (cpt == 2 && lch == 8) return launch_batched_t<2, 8>(a, grid, block, st);
    if (cpt == 2 && lch == 4) return launch_batched_t<2, 4>(a, grid, block, st);
    if (cpt == 4 && lch == 4) return launch_batched_t<4, 4>(a, grid, block, st);
    if (cpt == 4 && lch == 8) return launch_batched_t<4, 8>(a, grid, block, st);
    return hipErrorInvalidValue;
}

template <int CPT, int LCH, bool PAIR, bool NTA>
static hipError_t launch_group_t(const GroupArgs &g, const int64_t *step, int block,
                                 hipStream_t st)
{
    const dim3 grid((unsigned)g.n_tiles);
    switch (g.kind) {
    case K_F32_F64: hipLaunchKernelGGL((push_group_kernel<K_F32_F64, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_F32_KAHAN: hipLaunchKernelGGL((push_group_kernel<K_F32_KAHAN, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_F32_F32: hipLaunchKernelGGL((push_group_kernel<K_F32_F32, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_F64_F64: hipLaunchKernelGGL((push_group_kernel<K_F64_F64, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_CF32_F64: hipLaunchKernelGGL((push_group_kernel<K_CF32_F64, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_CF32_KAHAN: hipLaunchKernelGGL((push_group_kernel<K_CF32_KAHAN, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    case K_CF32_F32: hipLaunchKernelGGL((push_group_kernel<K_CF32_F32, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    default: hipLaunchKernelGGL((push_group_kernel<K_CF64_F64, CPT, LCH, PAIR, NTA>), grid, dim3(block), 0, st, g, step); break;
    }
    return hipGetLastError();
}

template <bool PAIR, bool NTA>
static hipError_t launch_push_group_p(const GroupArgs &g, const int64_t *step, int cpt, int lch,
                                      int block, hipStream_t st)
{
    if (cpt == 1 && lch == 16) return launch_group_t<1, 16, PAIR, NTA>(g, step, block, st);
    if (cpt == 1 && lch == 8) return launch_group_t<1, 8, PAIR, NTA>(g, step, block, st);
    if (cpt == 2 && lch == 8) return launch_group_t<2, 8, PAIR, NTA>(g, step, block, st);
    if (cpt == 2 && lch == 4) return launch_group_t<2, 4, PAIR, NTA>(g, step, block, st);
    if (cpt == 4 && lch == 4) return launch_group_t<4, 4, PAIR, NTA>(g, step, block, st);
    if (cpt == 4 && lch == 8) return launch_group_t<4, 8, PAIR, NTA>(g, step, block, st);
    return hipErrorInvalidValue;
}

hipError_t launch_push_group(const GroupArgs &g, const int64_t *step, int cpt, int lch, int block,
                             hipStream_t st)
{
    // pair groups keep cached accumulators (one form each)
    if (g.pair) return launch_push_group_p<true, false>(g, step, cpt, lch, block, st);
    return stream_acc(g) ? launch_push_group_p<false, true>(g, step, cpt, lch, block, st)
                         : launch_push_group_p<false, false>(g, step, cpt, lch, block, st);
}

template <int CPT, int LCH, bool PAIR>
static hipError_t launch_window_t(const GroupArgs &g, const int64_t *step, int block,
                                  int lags_per_block, hipStream_t st)
{
    const dim3 grid((unsigned)g.n_tiles, (unsigned)((g.p + lags_per_block - 1) / lags_per_block));
    switch (g.kind) {
    case K_F32_F64: hipLaunchKernelGGL((push_window_kernel<K_F32_F64, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F32_KAHAN: hipLaunchKernelGGL((push_window_kernel<K_F32_KAHAN, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F32_F32: hipLaunchKernelGGL((push_window_kernel<K_F32_F32, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F64_F64: hipLaunchKernelGGL((push_window_kernel<K_F64_F64, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_F64: hipLaunchKernelGGL((push_window_kernel<K_CF32_F64, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_KAHAN: hipLaunchKernelGGL((push_window_kernel<K_CF32_KAHAN, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_F32: hipLaunchKernelGGL((push_window_kernel<K_CF32_F32, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    default: hipLaunchKernelGGL((push_window_kernel<K_CF64_F64, CPT, LCH, PAIR>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    }
    return hipGetLastError();
}

template <bool PAIR>
static hipError_t launch_push_window_p(const GroupArgs &g, const int64_t *step, int cpt, int lch,
                                       int block, int lags_per_block, hipStream_t st)
{
    if (cpt == 1 && lch == 16) return launch_window_t<1, 16, PAIR>(g, step, block, lags_per_block, st);
    if (cpt == 1 && lch == 8) return launch_window_t<1, 8, PAIR>(g, step, block, lags_per_block, st);
    if (cpt == 2 && lch == 8) return launch_window_t<2, 8, PAIR>(g, step, block, lags_per_block, st);
    if (cpt == 2 && lch == 4) return launch_window_t<2, 4, PAIR>(g, step, block, lags_per_block, st);
    if (cpt == 4 && lch == 4) return launch_window_t<4, 4, PAIR>(g, step, block, lags_per_block, st);
    if (cpt == 4 && lch == 8) return launch_window_t<4, 8, PAIR>(g, step, block, lags_per_block, st);
    return hipErrorInvalidValue;
}

template <int CPT, int LCH>
static hipError_t launch_split_t(const GroupArgs &g, const int64_t *step, int block,
                                 int lags_per_block, hipStream_t st)
{
    const dim3 grid((unsigned)g.n_tiles, (unsigned)((g.p + lags_per_block - 1) / lags_per_block));
    switch (g.kind) {
    case K_F32_F64: hipLaunchKernelGGL((push_split_kernel<K_F32_F64, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F32_KAHAN: hipLaunchKernelGGL((push_split_kernel<K_F32_KAHAN, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F32_F32: hipLaunchKernelGGL((push_split_kernel<K_F32_F32, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_F64_F64: hipLaunchKernelGGL((push_split_kernel<K_F64_F64, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_F64: hipLaunchKernelGGL((push_split_kernel<K_CF32_F64, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_KAHAN: hipLaunchKernelGGL((push_split_kernel<K_CF32_KAHAN, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    case K_CF32_F32: hipLaunchKernelGGL((push_split_kernel<K_CF32_F32, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    default: hipLaunchKernelGGL((push_split_kernel<K_CF64_F64, CPT, LCH>), grid, dim3(block), 0, st, g, step, lags_per_block); break;
    }
    return hipGetLastError();
}

hipError_t launch_push_split(const GroupArgs &g, const int64_t *step, int cpt, int lch, int block,
                             int lags_per_block, hipStream_t st)
{
    if (lags_per_block < 1 || g.pair || g.deferred) return hipErrorInvalidValue;
    // a block holds lags_per_block lags: longer lag chunks would never run
    if (lch > 8 && lags_per_block <= 8) lch = 8;
    if (cpt == 1 && lch == 8) return launch_split_t<1, 8>(g, step, block, lags_per_block, st);
    if (cpt == 2 && lch == 8) return launch_split_t<2, 8>(g, step, block, lags_per_block, st);
    if (cpt == 2 && lch == 4) return launch_split_t<2, 4>(g, step, block, lags_per_block, st);
    if (cpt == 4 && lch == 4) return launch_split_t<4, 4>(g, step, block, lags_per_block, st);
    if (cpt == 4 && lch == 8) return launch_split_t<4, 8>(g, step, block, lags_per_block, st);
    return hipErrorInvalidValue;
}

hipError_t launch_push_window(const GroupArgs &g, const int64_t *step, int cpt, int lch,
                              int block, int lags_per_block, hipStream_t st)
{
    if (lags_per_block < 1 || g.levels != 1) return hipErrorInvalidValue;
    return g.pair ? launch_push_window_p<true>(g, step, cpt, lch, block, lags_per_block, st)
                  : launch_push_window_p<false>(g, step, cpt, lch, block, lags_per_block, st);
}

hipError_t launch_push_end(const PushEndArgs &a, hipStream_t st)
{
    if (a.n_flushed < 0 || a.n_flushed > kMaxGroups || a.n_stamps < 0 || a.n_stamps > 2)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(push_end_kernel, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

} // namespace corr
