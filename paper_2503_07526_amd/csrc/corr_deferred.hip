// corr_deferred.hip -- block-deferred form of the multiple-tau update.
//
// Algorithm 1 of the paper's Appendix D adds, at every push, the products of
// the newest value with the p lagged values of each level that receives a
// value.  The sums it builds are linear, so the products of T consecutive
// pushes can be added in one pass: on every push the sample is only written
// into a level-0 ring ("staging", 2 samples of traffic per channel), and once
// per block of T pushes (T a power of m) one flush pass per channel walks the
// T values of the block in order, adds each one's lag products to per-lag
// partial sums held in registers, forms the level-1 block means on the fly,
// and repeats level by level with the new values of the level above -- the
// same products, block means and counts as T single pushes, with the partial
// sums added to the stored accumulators once per flush.  The stored state
// after a flush is that of Algorithm 1 after the same pushes, up to the
// grouping of the floating-point sums.
//
// Staggering: the tiles are split into kFlushGroups groups and group j folds
// block q (pushes T(q-1)+1 .. Tq) at push Tq + j, so every push flushes about
// 1/kFlushGroups of the channels and the per-push cost is flat.  The level-0
// ring therefore holds P0 = 2T + p slots: the block being folded, up to T - 1
// pushes staged after it, and the p values before the block that its lags
// reach back to.  Each group's last folded block is kept in a device array
// (and mirrored on the host) so that a flush is never applied twice.
//
// State is touched once per flush and not again for T pushes, so the flush
// streams it with non-temporal loads and stores.
//
// A readout between flushes first lets every group catch up to the last
// complete block, then folds the pushes after it the same way without
// writing any state (so a readout never changes later results) and reduces
// the resulting per-channel accumulators over 64-channel chunks and then
// over chunks in a fixed order (the group mean does not depend on the tile
// width).
//
// Replay of a stored history: when whole blocks of pushes are given at once,
// every tile group folds a block in one pass with the level-0 values of the
// block read straight from the caller's history (no staging write and read);
// only the block's last p - 1 values are written to the ring, the ones later
// folds and readouts look back to.  The products, block means and sums are
// those of the staged fold, in the same order.
//
// Supported here: single-precision real samples, m = 2, p = 16, T = 256 or
// 128 (the group's defer_t).  Levels 0 and 1 are folded together, streamed
// through chunks of 64 pushes (levels01); from level 2 on the cascade takes
// the T / 4 level-2 values at once.  Levels k <= log2 T receive T / 2^k new
// values per flush (compile-time counts); deeper levels receive at most one.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

template <int K> struct RK;
template <> struct RK<K_F32_F64>   { using S = float;  using A = double; using PT = double; static constexpr int NP = 1; };
template <> struct RK<K_F32_KAHAN> { using S = float;  using A = float;  using PT = float;  static constexpr int NP = 2; };
template <> struct RK<K_F32_F32>   { using S = float;  using A = float;  using PT = float;  static constexpr int NP = 1; };

// part += x * r in the partial-sum precision (products of single-precision
// samples are exact in double).
__device__ __forceinline__ void pmac(double &pt, float x, float r) { pt = __builtin_fma((double)x, (double)r, pt); }
__device__ __forceinline__ void pmac(float &pt, float x, float r) { pt = __builtin_fmaf(x, r, pt); }

// Fold a partial sum into a stored accumulator (compensated: Kahan step on
// the partial, true value = h - c).
template <int K> struct Fold;
template <> struct Fold<K_F32_F64> {
    static __device__ __forceinline__ void add(double &h, double &, double pt) { h += pt; }
    static __device__ __forceinline__ double value(double h, double) { return h; }
};
template <> struct Fold<K_F32_F32> {
    static __device__ __forceinline__ void add(float &h, float &, float pt) { h += pt; }
    static __device__ __forceinline__ double value(float h, float) { return (double)h; }
};
template <> struct Fold<K_F32_KAHAN> {
    static __device__ __forceinline__ void add(float &h, float &c, float pt)
    {
        float y = pt - c;
        float t = h + y;
        c = (t - h) - y;
        h = t;
    }
    static __device__ __forceinline__ double value(float h, float c) { return (double)h - (double)c; }
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

struct Ctx {
    const DeferredArgs *a;
    int64_t f;       // pushes already folded (multiple of T)
    int r;           // pushes folded by this pass
    char *tb;        // tile base
    int lane;        // channel within the tile
    bool valid;      // channel < n_ch
    bool reduce_me;  // channel in [ch_begin, ch_end)
    int64_t ch;      // global channel index
};

// Accumulator rows of level k: value rows start at acc; compensation rows
// follow nl rows later.
template <int K, int P>
__device__ __forceinline__ typename RK<K>::A *acc_rows(const Ctx &cx, int k, int &nl)
{
    using S = typename RK<K>::S;
    using A = typename RK<K>::A;
    const GroupArgs &g = cx.a->g;
    const int tw = g.tw;
    if (k == 0) {
        nl = P;
        return reinterpret_cast<A *>(cx.tb + (int64_t)g.p0 * tw * (int64_t)sizeof(S));
    }
    nl = P - P / 2;
    char *lvl = cx.tb + g.lvl0_bytes + (int64_t)(k - 1) * g.lvlk_bytes;
    return reinterpret_cast<A *>(lvl + (int64_t)P * tw * (int64_t)sizeof(S));
}

// Index of the first readout entry of level k after S pushes (entries are the
// (level, lag) pairs with a non-zero count, level-major, lag-minor).
template <int P>
__device__ __forceinline__ int entry_offset(int k, int64_t S)
{
    int off = 0;
    int64_t sk = S;
    for (int j = 0; j < k; ++j) {
        const int l0 = j == 0 ? 0 : P / 2;
        const int64_t hi = sk < P ? sk : P;
        if (hi > l0) off += (int)(hi - l0);
        sk >>= 1;
    }
    return off;
}

// Fold the level's partial sums into its accumulators.  Flush mode stores
// them; readout mode reduces value(h, c) over the block instead.
template <int K, int P, int NL, bool READ>
__device__ __forceinline__ void fold_level(Ctx &cx, int k, const typename RK<K>::PT (&part)[NL],
                                           bool any_pending)
{
    using A = typename RK<K>::A;
    constexpr int NP = RK<K>::NP;
    int nl;
    A *hi = acc_rows<K, P>(cx, k, nl);
    A *lo = hi + (size_t)nl * cx.a->g.tw;
    const int tw = cx.a->g.tw;
    if constexpr (!READ) {
        if (!any_pending) return;
        A h[NL], c[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            h[j] = __builtin_nontemporal_load(&hi[(size_t)j * tw + cx.lane]);
            if constexpr (NP == 2) c[j] = __builtin_nontemporal_load(&lo[(size_t)j * tw + cx.lane]); else c[j] = A(0);
        }
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            Fold<K>::add(h[j], c[j], (A)part[j]);
            __builtin_nontemporal_store(h[j], &hi[(size_t)j * tw + cx.lane]);
            if constexpr (NP == 2) __builtin_nontemporal_store(c[j], &lo[(size_t)j * tw + cx.lane]);
        }
    } else {
        const DeferredArgs &a = *cx.a;
        const int64_t S = cx.f + cx.r;
        int64_t sk = S >> k;
        const int l0 = k == 0 ? 0 : P / 2;
        const int hi_lag = (int)(sk < P ? sk : P); // lags [l0, hi_lag) have counts
        if (hi_lag <= l0) return;
        const int e0 = entry_offset<P>(k, S);
        const bool in_slice = cx.valid && cx.ch >= a.slice_begin && cx.ch < a.slice_end;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            const int L = l0 + j;
            if (L < hi_lag) {
                A h = hi[(size_t)j * tw + cx.lane];
                A c = A(0);
                if constexpr (NP == 2) c = lo[(size_t)j * tw + cx.lane];
                if (any_pending) Fold<K>::add(h, c, (A)part[j]);
                const double v = Fold<K>::value(h, c);
                const int e = e0 + j;
                if (in_slice) a.slice_out[(size_t)(cx.ch - a.slice_begin) * a.ne + e] = v;
                // Fixed-order sum over the wave's 64 consecutive channels (a
                // chunk aligned to 64 whatever the tile width).
                const double s = wave_sum(cx.reduce_me ? v : 0.0);
                if ((threadIdx.x & 63) == 0)
                    a.chunk_partial[(size_t)((cx.ch >> 6) - a.row_begin) * a.ne + e] = s;
            }
        }
    }
}

// Level 0: fold the r pending pushes (f, f + r] into the lag sums and form the
// level-1 block means.  out[q] = mean of new values 2q, 2q+1.  The pushes are
// taken in chunks of kL0Chunk with a sliding window of the P - 1 values
// before each chunk, so that only P - 1 + kL0Chunk ring values are live.
constexpr int kL0Chunk = 64;

template <int K, int P, int T, bool READ>
__device__ __forceinline__ void level0(Ctx &cx, typename RK<K>::S (&out)[T / 2])
{
    using S = typename RK<K>::S;
    using PT = typename RK<K>::PT;
    constexpr int C = T < kL0Chunk ? T : kL0Chunk;
    static_assert(T % C == 0 && C % 2 == 0, "chunks of whole pairs");
    const DeferredArgs &a = *cx.a;
    const GroupArgs &g = a.g;
    const int tw = g.tw;
    const int P0 = g.p0;
    const S *ring = reinterpret_cast<const S *>(cx.tb);
    const int64_t f = cx.f;
    const int r = cx.r;
    // W: old values f-P+2 .. f, then the chunk's new values (zeros beyond r);
    // value j sits in slot (j - 1) mod P0, and P - 1 + T < P0, so one modulo
    // and a wrap per row suffice
    S W[P - 1 + C];
    const int slot0 = (int)((f - (P - 2) - 1 + P0) % P0);
    auto row = [&](int i) -> S { // i-th value from f - P + 2
        int slot = slot0 + i;
        if (slot >= P0) slot -= P0;
        return __builtin_nontemporal_load(&ring[(size_t)slot * tw + cx.lane]);
    };
#pragma unroll
    for (int i = 0; i < P - 1; ++i) W[i] = row(i);
    PT part[P];
#pragma unroll
    for (int L = 0; L < P; ++L) part[L] = PT(0);
#pragma unroll
    for (int c0 = 0; c0 < T; c0 += C) {
        // keep the next chunk's loads after this chunk's products (otherwise
        // they are hoisted and every chunk's values are live at once)
        if (c0 > 0) asm volatile("" ::: "memory");
#pragma unroll
        for (int q = 0; q < C; ++q) W[P - 1 + q] = c0 + q < r ? row(P - 1 + c0 + q) : S(0);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            if (c0 + q < r) {
                const S x = W[P - 1 + q];
#pragma unroll
                for (int L = 0; L < P; ++L) pmac(part[L], x, W[P - 1 + q - L]);
            }
        }
#pragma unroll
        for (int q = 0; q < C / 2; ++q)
            out[c0 / 2 + q] = (W[P - 1 + 2 * q] + W[P + 2 * q]) / S(2);
#pragma unroll
        for (int i = 0; i < P - 1; ++i) W[i] = W[i + C];
    }
    fold_level<K, P, P, READ>(cx, 0, part, r > 0);
}

// Levels 0 and 1 together, for blocks of more than kL0Chunk pushes: the r
// pending pushes are taken in chunks of kL0Chunk; each chunk adds its level-0
// lag products, forms its kL0Chunk / 2 level-1 means, adds their level-1 lag
// products at once (sliding windows of the P - 1 older values of both levels
// stay in registers) and forms the level-2 means, which are collected in
// the thread's column of the LDS array out[T / 4][blockDim.x] for the cascade
// (in registers they would crowd out the windows).  Only the last P level-1
// values of the block are written to the level-1 ring (the earlier ones would
// be overwritten).
template <int K, int P, int T, bool READ, bool HIST>
__device__ __forceinline__ void levels01(Ctx &cx, typename RK<K>::S *out)
{
    using S = typename RK<K>::S;
    using PT = typename RK<K>::PT;
    constexpr int C = kL0Chunk;
    constexpr int C1 = C / 2;   // level-1 values per chunk
    constexpr int NL1 = P - P / 2;
    static_assert(T % C == 0 && C1 % 2 == 0, "chunks of whole pairs");
    const DeferredArgs &a = *cx.a;
    const GroupArgs &g = a.g;
    const int tw = g.tw;
    const int P0 = g.p0;
    const S *ring0 = reinterpret_cast<const S *>(cx.tb);
    S *ring1 = reinterpret_cast<S *>(cx.tb + g.lvl0_bytes);
    const int64_t f = cx.f;
    const int r = cx.r;
    const bool has1 = g.levels > 1;     // a one-level group has no level-1 state
    const int n1 = has1 ? r / 2 : 0;    // level-1 values of this pass
    const int64_t f1 = f >> 1;          // level-1 values already in the ring
    // level 0: value j in slot (j - 1) mod P0 (one modulo, then a wrap per row)
    const int slot0 = (int)((f - (P - 2) - 1 + P0) % P0);
    auto row0 = [&](int i) -> S {
        int slot = slot0 + i;
        if (slot >= P0) slot -= P0;
        return __builtin_nontemporal_load(&ring0[(size_t)slot * tw + cx.lane]);
    };
    // value i (0-based) of the block: staged in the ring, or from the history
    auto newval = [&](int i) -> S {
        if constexpr (HIST) {
            const S *row = reinterpret_cast<const S *>(a.hist + (int64_t)i * a.hist_stride);
            return cx.valid ? __builtin_nontemporal_load(&row[cx.ch]) : S(0);
        } else {
            return row0(P - 1 + i);
        }
    };
    S W0[P - 1 + C], W1[P - 1 + C1];
#pragma unroll
    for (int i = 0; i < P - 1; ++i) W0[i] = row0(i);
#pragma unroll
    for (int i = 0; i < P - 1; ++i) {
        const int64_t v = f1 - (P - 2) + i; // level-1 value number (1-based)
        const int slot = (int)((v - 1 + P) % P);
        W1[i] = has1 ? __builtin_nontemporal_load(&ring1[(size_t)slot * tw + cx.lane]) : S(0);
    }
    PT part0[P], part1[NL1];
#pragma unroll
    for (int L = 0; L < P; ++L) part0[L] = PT(0);
#pragma unroll
    for (int j = 0; j < NL1; ++j) part1[j] = PT(0);
    // one chunk at a time (a rolled loop: only one chunk's values are live)
#pragma unroll 1
    for (int c0 = 0; c0 < T; c0 += C) {
#pragma unroll
        for (int q = 0; q < C; ++q) W0[P - 1 + q] = c0 + q < r ? newval(c0 + q) : S(0);
#pragma unroll
        for (int q = 0; q < C; ++q) {
            if (c0 + q < r) {
                const S x = W0[P - 1 + q];
#pragma unroll
                for (int L = 0; L < P; ++L) pmac(part0[L], x, W0[P - 1 + q - L]);
            }
        }
        // level-1 values c0/2 + q of the block
        const int b1 = c0 / 2;
#pragma unroll
        for (int q = 0; q < C1; ++q)
            W1[P - 1 + q] = b1 + q < n1 ? (W0[P - 1 + 2 * q] + W0[P + 2 * q]) / S(2) : S(0);
#pragma unroll
        for (int q = 0; q < C1; ++q) {
            if (b1 + q < n1) {
                const S x = W1[P - 1 + q];
#pragma unroll
                for (int j = 0; j < NL1; ++j) pmac(part1[j], x, W1[P - 1 + q - (P / 2 + j)]);
            }
        }
        if constexpr (!READ) {
            // ring slots of the last P level-1 values of the block
#pragma unroll
            for (int q = 0; q < C1; ++q) {
                const int idx = b1 + q;
                if (idx < n1 && idx >= n1 - P) {
                    const int64_t v = f1 + 1 + idx;
                    const int slot = (int)((v - 1) % P);
                    __builtin_nontemporal_store(W1[P - 1 + q], &ring1[(size_t)slot * tw + cx.lane]);
                }
            }
        }
        // level-2 means of this chunk's level-1 pairs (f1 is even: pairs align)
#pragma unroll
        for (int q = 0; q < C1 / 2; ++q)
            out[(size_t)(b1 / 2 + q) * blockDim.x + threadIdx.x] =
                (W1[P - 1 + 2 * q] + W1[P + 2 * q]) / S(2);
#pragma unroll
        for (int i = 0; i < P - 1; ++i) {
            W0[i] = W0[i + C];
            W1[i] = W1[i + C1];
        }
    }
    if constexpr (HIST && !READ) {
        // the block's last P - 1 values (now W0[0 .. P-2]) go to their ring
        // slots: the next block's folds and the readouts look back to them
        S *ring0w = reinterpret_cast<S *>(cx.tb);
        const int slot_w = (int)((f + T - (P - 1)) % P0); // value f + T - P + 2
#pragma unroll
        for (int i = 0; i < P - 1; ++i) {
            int slot = slot_w + i;
            if (slot >= P0) slot -= P0;
            __builtin_nontemporal_store(W0[i], &ring0w[(size_t)slot * tw + cx.lane]);
        }
    }
    fold_level<K, P, P, READ>(cx, 0, part0, r > 0);
    if (has1) fold_level<K, P, NL1, READ>(cx, 1, part1, n1 > 0);
}

// Level k >= 1 receiving n_in <= N new values in[0..n_in) (level-k values
// f_k+1 .. f_k+n_in).  Adds lags P/2..P-1, writes the new ring slots (flush
// mode) and forms the level-(k+1) means (n_out of them).
template <int K, int P, int N, bool READ>
__device__ __forceinline__ void level_k(Ctx &cx, int k, const typename RK<K>::S (&in)[N],
                                        int n_in, typename RK<K>::S (&out)[(N >= 2 ? N / 2 : 1)],
                                        int &n_out)
{
    using S = typename RK<K>::S;
    using PT = typename RK<K>::PT;
    constexpr int NL = P - P / 2;
    const DeferredArgs &a = *cx.a;
    const GroupArgs &g = a.g;
    const int tw = g.tw;
    S *ring = reinterpret_cast<S *>(cx.tb + g.lvl0_bytes + (int64_t)(k - 1) * g.lvlk_bytes);
    const int64_t fk = cx.f >> k; // level-k values already in the ring
    S H[P - 1 + N];
#pragma unroll
    for (int i = 0; i < P - 1; ++i) {
        const int64_t v = fk - (P - 2) + i; // value number (1-based)
        const int slot = (int)((v - 1 + P) % P);
        H[i] = __builtin_nontemporal_load(&ring[(size_t)slot * tw + cx.lane]);
    }
#pragma unroll
    for (int q = 0; q < N; ++q) H[P - 1 + q] = q < n_in ? in[q] : S(0);
    PT part[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) part[j] = PT(0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
        if (q < n_in) {
            const S x = H[P - 1 + q];
#pragma unroll
            for (int j = 0; j < NL; ++j) pmac(part[j], x, H[P - 1 + q - (P / 2 + j)]);
        }
    }
    if constexpr (!READ) {
        // ring slots of the new values (only the last P of them survive)
#pragma unroll
        for (int q = 0; q < N; ++q) {
            if (q < n_in && q >= n_in - P) {
                const int64_t v = fk + 1 + q;
                const int slot = (int)((v - 1) % P);
                __builtin_nontemporal_store(H[P - 1 + q], &ring[(size_t)slot * tw + cx.lane]);
            }
        }
    }
    if constexpr (N >= 2) {
        // f_k is a multiple of N here, so new values pair up as (2q, 2q+1)
#pragma unroll
        for (int q = 0; q < N / 2; ++q) out[q] = (H[P - 1 + 2 * q] + H[P + 2 * q]) / S(2);
        n_out = n_in / 2;
    } else {
        n_out = 0;
        out[0] = S(0);
        if (n_in == 1 && ((fk + 1) & 1) == 0) {
            out[0] = (H[P - 2] + H[P - 1]) / S(2);
            n_out = 1;
        }
    }
    fold_level<K, P, NL, READ>(cx, k, part, n_in > 0);
}

// Levels k .. b-1 starting with N new values.
template <int K, int P, int N, bool READ>
__device__ __forceinline__ void cascade(Ctx &cx, int k, const typename RK<K>::S (&in)[N], int n_in)
{
    using S = typename RK<K>::S;
    const int b = cx.a->g.levels;
    if (k >= b) return;
    if constexpr (N >= 2) {
        S out[N / 2];
        int n_out;
        level_k<K, P, N, READ>(cx, k, in, n_in, out, n_out);
        cascade<K, P, N / 2, READ>(cx, k + 1, out, n_out);
    } else {
        S cur[1] = {in[0]};
        int n = n_in;
        for (int kk = k; kk < b; ++kk) {
            if (n == 0 && !READ) break;
            S nxt[1];
            int nn;
            level_k<K, P, 1, READ>(cx, kk, cur, n, nxt, nn);
            cur[0] = nxt[0];
            n = nn;
        }
    }
}

template <int K, int P, int T, int NT, bool READ, bool HIST>
__device__ __forceinline__ void deferred_pass(const DeferredArgs &a)
{
    const GroupArgs &g = a.g;
    // block = (tile slot, part of the tile); parts of blockDim.x channels
    const int parts = (g.tw + (int)blockDim.x - 1) / (int)blockDim.x;
    const int64_t slot = blockIdx.x / parts;
    const int part = (int)(blockIdx.x % parts);
    int64_t f;
    int r;
    int64_t tile;
    if constexpr (READ) {
        // Readout (all tile groups caught up): fold the pushes after the
        // last complete block without writing state, for the tiles that hold
        // the pass's chunk rows [row_begin, row_end).
        const int64_t S = *a.step;
        f = (S / T) * T;
        r = (int)(S - f);
        tile = (a.row_begin * 64) / g.tw + slot;
        if (tile >= g.n_tiles) return;
    } else {
        // Flush of tile group j, block q: scheduled at push T q + j
        // (fixed_group -1; the counter is advanced after this push), requested
        // for one tile group (fixed_group >= 0) or for every tile group
        // (fixed_group -2: the grid spans all tiles).  Skipped when that block
        // is already folded.
        int j;
        int64_t q;
        if (a.fixed_group == -2) {
            q = a.fixed_block;
            tile = slot;
            if (tile >= g.n_tiles) return;
            j = (int)(tile / a.tiles_per_group);
        } else {
            if (a.fixed_group >= 0) {
                j = a.fixed_group;
                q = a.fixed_block;
            } else {
                const int64_t S = *a.step + 1;
                j = (int)(S % T);
                q = S / T;
            }
            tile = (int64_t)j * a.tiles_per_group + slot;
            if (tile >= g.n_tiles || slot >= a.tiles_per_group) return;
        }
        if (q < 1 || a.flushed[j] >= q) return;
        f = (q - 1) * T;
        r = T;
    }
    {
        const int sub = part;
        // whole waves past the tile's end skip the pass (tw is a multiple of 64)
        if (sub * (int)blockDim.x + (int)(threadIdx.x & ~63u) >= g.tw) return;
        if constexpr (READ) {
            // and, in a readout, waves whose chunk row belongs to another pass
            const int64_t row = (tile * g.tw + sub * (int64_t)blockDim.x + (threadIdx.x & ~63u)) >> 6;
            if (row < a.row_begin || row >= a.row_end) return;
        }
        Ctx cx;
        cx.a = &a;
        cx.f = f;
        cx.r = r;
        cx.tb = g.state + tile * g.tile_bytes;
        cx.lane = sub * blockDim.x + threadIdx.x;
        cx.ch = tile * g.tw + cx.lane;
        cx.valid = cx.ch < g.n_ch;
        cx.reduce_me = cx.valid && cx.ch >= a.ch_begin && cx.ch < a.ch_end;
        if constexpr (T > kL0Chunk) {
            // levels 0 and 1 streamed chunk by chunk, then the cascade from
            // level 2 (f is a multiple of T, so level-1 pairs align); each
            // thread reads back only its own column of l2s
            using S = typename RK<K>::S;
            __shared__ S l2s[(T / 4) * NT];
            levels01<K, P, T, READ, HIST>(cx, l2s);
            S l2[T / 4];
#pragma unroll
            for (int q = 0; q < T / 4; ++q) l2[q] = l2s[(size_t)q * blockDim.x + threadIdx.x];
            cascade<K, P, T / 4, READ>(cx, 2, l2, (r / 2) / 2);
        } else {
            static_assert(!HIST, "history folds take blocks of more than kL0Chunk pushes");
            typename RK<K>::S l1[T / 2];
            level0<K, P, T, READ>(cx, l1);
            cascade<K, P, T / 2, READ>(cx, 1, l1, r / 2);
        }
    }
}

// The scheduled (or requested) flush, NT threads per block: at most two waves
// per SIMD, so that the register budget covers the whole block of pushes
// without spilling.  HIST: level 0 from a stored history.
template <int K, int P, int T, int NT, bool HIST>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void deferred_kernel(DeferredArgs a)
{
    // with timing, on the sampled pushes: earliest block start and latest
    // block end of the push's folds (device wall clock; no event between
    // kernels); the other pushes skip the closing barrier as well
    FoldStamps *st = a.stamps;
    const bool stamped = st && stamp_sampled(st);
    if (stamped && threadIdx.x == 0) stamp_start_now(st, blockIdx.x);
    deferred_pass<K, P, T, NT, false, HIST>(a);
    if (stamped) {
        __syncthreads();
        if (threadIdx.x == 0) stamp_end_now(st, blockIdx.x);
    }
}

// The readout pass (no state written).
template <int K, int P, int T>
__global__ __launch_bounds__(kFoldThreadsDefault) void deferred_read_kernel(DeferredArgs a)
{
    deferred_pass<K, P, T, kFoldThreadsDefault, true, false>(a);
}

// Column sums of rows [n_rows][ne] in a fixed order: groups of kColGroup rows
// (grid.y: group group_begin + blockIdx.y, whose rows are held from row
// row_begin on), then the groups in order.
constexpr int kColGroup = 1024;

__global__ void colsum_group_kernel(const double *rows, int64_t row_begin, int64_t n_rows, int ne,
                                    int64_t group_begin, double *groups)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int64_t grp = group_begin + blockIdx.y;
    const int64_t r0 = grp * kColGroup;
    int64_t r1 = r0 + kColGroup;
    if (r1 > n_rows) r1 = n_rows;
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += rows[(size_t)(r - row_begin) * ne + e];
    groups[(size_t)grp * ne + e] = s;
}

__global__ void colsum_final_kernel(const double *groups, int64_t n_groups, int ne, double *out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double s = 0.0;
    for (int64_t q = 0; q < n_groups; ++q) s += groups[(size_t)q * ne + e];
    out[e] = s;
}

// Record that tile group j folded block q (runs after the flush kernel).
__global__ void flush_commit_kernel(DeferredArgs a)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int T = a.g.defer_t;
    int j;
    int64_t q;
    if (a.fixed_group >= 0) {
        j = a.fixed_group;
        q = a.fixed_block;
    } else {
        const int64_t S = *a.step + 1;
        j = (int)(S % T);
        q = S / T;
    }
    if (q >= 1 && a.flushed[j] < q) a.flushed[j] = q;
}

template <int K, int P, int T, int NT, bool READ, bool HIST>
hipError_t launch_deferred_kpt(const DeferredArgs &a, hipStream_t st)
{
    const int block = a.g.tw < NT ? a.g.tw : NT;
    const int parts = (a.g.tw + block - 1) / block;
    // readout: the tiles that hold chunk rows [row_begin, row_end); every
    // tile group: all tiles; otherwise the tiles of one tile group
    const int64_t read_tiles = (a.row_end * 64 + a.g.tw - 1) / a.g.tw - (a.row_begin * 64) / a.g.tw;
    const int64_t tiles = READ ? read_tiles : a.fixed_group == -2 ? a.g.n_tiles : a.tiles_per_group;
    const int64_t grid = tiles * parts;
    if (grid < 1) return hipSuccess;
    if constexpr (READ)
        hipLaunchKernelGGL((deferred_read_kernel<K, P, T>), dim3((unsigned)grid), dim3(block), 0, st,
                           a);
    else
        hipLaunchKernelGGL((deferred_kernel<K, P, T, NT, HIST>), dim3((unsigned)grid), dim3(block),
                           0, st, a);
    return hipGetLastError();
}

// Instantiated block shapes: the staged fold with 64, 128 or 256 threads per
// block; the readout and the history fold with the default 128.
template <int K, int P, int T, bool READ, bool HIST>
hipError_t launch_deferred_nt(const DeferredArgs &a, hipStream_t st)
{
    if constexpr (READ || HIST) {
        return launch_deferred_kpt<K, P, T, kFoldThreadsDefault, READ, HIST>(a, st);
    } else {
        switch (a.threads) {
        case 64: return launch_deferred_kpt<K, P, T, 64, false, false>(a, st);
        case 256: return launch_deferred_kpt<K, P, T, 256, false, false>(a, st);
        default: return launch_deferred_kpt<K, P, T, 128, false, false>(a, st);
        }
    }
}

template <int K, bool READ, bool HIST>
hipError_t launch_deferred_k(const DeferredArgs &a, hipStream_t st)
{
    switch (a.g.defer_t) {
    case kDeferT: return launch_deferred_nt<K, 16, kDeferT, READ, HIST>(a, st);
    case kDeferTMin: return launch_deferred_nt<K, 16, kDeferTMin, READ, HIST>(a, st);
    default: return hipErrorInvalidValue;
    }
}

template <bool READ, bool HIST = false>
hipError_t launch_deferred_t(const DeferredArgs &a, hipStream_t st)
{
    if (a.g.p != 16) return hipErrorInvalidValue;
    if (HIST && (!a.hist || a.fixed_group != -2)) return hipErrorInvalidValue;
    switch (a.g.kind) {
    case K_F32_F64: return launch_deferred_k<K_F32_F64, READ, HIST>(a, st);
    case K_F32_KAHAN: return launch_deferred_k<K_F32_KAHAN, READ, HIST>(a, st);
    case K_F32_F32: return launch_deferred_k<K_F32_F32, READ, HIST>(a, st);
    default: return hipErrorInvalidValue;
    }
}

// Per-push staging of one block-deferred group: sample c -> level-0 ring slot
// (s - 1) mod p0 of its tile.  Each thread moves kStageVec consecutive
// channels (one 16-byte load and store) for kStageUnroll grid strides, all
// loads issued before the stores.
constexpr int kStageVec = 4;
constexpr int kStageUnroll = 4;

// The sample is read once, and its ring row is read again only by the fold
// of its subset: in the same push for one subset in T, up to T pushes (and
// hundreds of MB of traffic) later for the others.  So both streams are
// non-temporal: the staging of 6e7 channels took about 9 us less per push
// (the large step 0.244 against 0.253 ms).
typedef float stage_f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stage_kernel(GroupArgs g, const int64_t *step, int aligned)
{
    const int64_t s = *step + 1;
    const int slot = (int)((s - 1) % g.p0);
    const float *src = static_cast<const float *>(g.samples);
    const int64_t n = g.n_ch;
    const int64_t nvec = (n + kStageVec - 1) / kStageVec;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < nvec;
         v0 += stride * kStageUnroll) {
        float4 x[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            const int64_t c = v * kStageVec;
            if (v < nvec) {
                if (aligned && c + kStageVec <= n) {
                    const stage_f4 t = __builtin_nontemporal_load(reinterpret_cast<const stage_f4 *>(src + c));
                    x[u] = make_float4(t[0], t[1], t[2], t[3]);
                } else {
                    x[u].x = c + 0 < n ? src[c + 0] : 0.f;
                    x[u].y = c + 1 < n ? src[c + 1] : 0.f;
                    x[u].z = c + 2 < n ? src[c + 2] : 0.f;
                    x[u].w = c + 3 < n ? src[c + 3] : 0.f;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const int64_t v = v0 + u * stride;
            if (v < nvec) {
                const int64_t c = v * kStageVec;
                const int64_t tile = c / g.tw;
                const int64_t lane = c - tile * g.tw;
                float *ring = reinterpret_cast<float *>(g.state + tile * g.tile_bytes);
                __builtin_nontemporal_store(stage_f4{x[u].x, x[u].y, x[u].z, x[u].w},
                                            reinterpret_cast<stage_f4 *>(ring + (size_t)slot * g.tw + lane));
            }
        }
    }
}

} // namespace

hipError_t launch_stage(const GroupArgs &g, const int64_t *step, hipStream_t st)
{
    // single-precision samples only (the deferred form's kinds); 16-byte
    // vectors need a 16-byte aligned source
    const int aligned = ((uintptr_t)g.samples % 16) == 0;
    const int64_t nvec = (g.n_ch + kStageVec - 1) / kStageVec;
    int64_t blocks = (nvec + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(stage_kernel, dim3((unsigned)blocks), dim3(256), 0, st, g, step, aligned);
    return hipGetLastError();
}

bool deferred_supported(int kind, int p, int m)
{
    return m == 2 && p == 16 && (kind == K_F32_F64 || kind == K_F32_KAHAN || kind == K_F32_F32);
}

hipError_t launch_flush_fold(const DeferredArgs &a, hipStream_t st)
{
    return launch_deferred_t<false>(a, st);
}

hipError_t launch_history_fold(const DeferredArgs &a, hipStream_t st)
{
    return launch_deferred_t<false, true>(a, st);
}

hipError_t launch_flush_commit(const DeferredArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(flush_commit_kernel, dim3(1), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_flush(const DeferredArgs &a, hipStream_t st)
{
    hipError_t e = launch_flush_fold(a, st);
    if (e != hipSuccess) return e;
    return launch_flush_commit(a, st);
}

int64_t deferred_readout_rows(const GroupArgs &g) { return g.n_tiles * (int64_t)g.tw / 64; }

int64_t deferred_readout_groups(const GroupArgs &g)
{
    return (deferred_readout_rows(g) + kColGroup - 1) / kColGroup;
}

int64_t deferred_readout_group_rows() { return kColGroup; }

hipError_t launch_deferred_readout_pass(const DeferredArgs &a, double *groups, hipStream_t st)
{
    const int64_t n_rows = deferred_readout_rows(a.g);
    if (a.row_begin < 0 || a.row_begin % kColGroup != 0 || a.row_end <= a.row_begin ||
        (a.row_end != n_rows && a.row_end % kColGroup != 0) || a.row_end > n_rows)
        return hipErrorInvalidValue; // a pass holds whole groups of rows
    hipError_t e = launch_deferred_t<true>(a, st);
    if (e != hipSuccess) return e;
    const int64_t g0 = a.row_begin / kColGroup;
    const int64_t g1 = (a.row_end + kColGroup - 1) / kColGroup;
    const unsigned ex = (unsigned)((a.ne + 63) / 64);
    hipLaunchKernelGGL(colsum_group_kernel, dim3(ex, (unsigned)(g1 - g0)), dim3(64), 0, st,
                       a.chunk_partial, a.row_begin, n_rows, a.ne, g0, groups);
    return hipGetLastError();
}

hipError_t launch_deferred_readout_final(const DeferredArgs &a, const double *groups, double *sums,
                                         hipStream_t st)
{
    const unsigned ex = (unsigned)((a.ne + 63) / 64);
    hipLaunchKernelGGL(colsum_final_kernel, dim3(ex), dim3(64), 0, st, groups,
                       deferred_readout_groups(a.g), a.ne, sums);
    return hipGetLastError();
}

} // namespace corr
