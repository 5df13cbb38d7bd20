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
// Precision: the operands are at most 1 in magnitude (the phases; for the
// currents, the velocity components are first scaled by a power of two per
// atom block, so that the largest magnitude of each component over the
// block's atoms lies in [1/2, 1), and the block's double sums are scaled back
// exactly when stored).  Each real operand v is
// split into v_hi = fp16(v) and v_lo = fp16(v - v_hi) (about 22 significant
// bits together) and a real product is a_hi b_hi + a_hi b_lo + a_lo b_hi (the
// dropped a_lo b_lo is below 2^-22), i.e. three fp16 matrix products with
// fp32 accumulation per sum, twelve per K-step.  The fp32 accumulators are
// added to double accumulators after every kAccAtoms atoms (an fp32 partial
// sum of at most 256 terms of magnitude <= 1 each) and the blocks write double
// partials, reduced over the atom blocks in a fixed order as in the
// vector-unit producer (corr_rhok.hip), so the result is reproducible.  The tables start from e^{2 pi i x / L} in double (a 64-entry
// root table times a short Taylor series) and take the powers by a double
// recurrence, each power rounded once to float.
//
// Operand layout of the contraction (checked on the device): lane l holds
// A[l%16][a(l/16)+j] and B[a(l/16)+j][l%16] for j < a, a = atoms per lane,
// and receives D[4(l/16)+v][l%16] for v < 4.  Only the pairing of A and B
// along K matters for the sum, and it is the same for both operands.
//
// Work split: block (chunk, atom block); each contraction wave of a block
// owns one M tile and all waves share the tile's LDS tables: X and Y powers as float2
// [rows][Tile::stride] (a row per power that a pair of the k-set uses: n_x in
// [x_lo, x_lo + x_rows), n_y likewise; atoms along the row, so a lane's
// atoms are 16-byte reads; the row stride is padded so that the 16 rows a
// K-step reads start in different banks) and the split |n_z| powers already
// in B-fragment order.  The tables are double-buffered: builder waves build
// the next tile's tables while the contraction waves contract the current
// one, one barrier per tile, and the positions are loaded a tile ahead.
//
// That is the form of the current producer (three weight sets).  n(k) (one
// weight set) takes the couple form below (rhok_couple_kernel): rows of the
// products that a pair (n_x, n_y) and its mirror (n_x, -n_y) share, which
// forms fewer products per pair on the vector units.
#include <hip/hip_runtime.h>

#include "corr_kernels.h"

namespace corr {

namespace {

// The contraction instruction: K = 32 atoms per v_mfma_f32_16x16x32_f16 (lane
// l holds 8 consecutive atoms, 8(l/16) .. 8(l/16)+7, of A row l%16 and of B
// column l%16), or K = 16 with v_mfma_f32_16x16x16_f16 (4 atoms per lane).
constexpr bool kWideK = true;
constexpr int kAtomsPerLane = kWideK ? 8 : 4;
constexpr int kKStep = 4 * kAtomsPerLane; // atoms per K-step

typedef _Float16 halfv_t __attribute__((ext_vector_type(kAtomsPerLane)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaMaxWaves = 12;  // waves per block
constexpr int kMfmaCols = 16;      // |n_z| = 0 .. 15
constexpr int kRoots = 64;         // e^{2 pi i q / kRoots} table for the base phase
// LDS after the root table for the weight scales (three weight sets): the
// waves' maxima [waves][NW] as floats, in double2 units
template <int NW> struct ScaleSlots { static constexpr int n = NW == 1 ? 0 : 8; };
// B fragments in LDS: [K-step][part: re hi, re lo, im hi, im lo][atom group][column],
// each atom group's row of 16 columns padded by one fragment and each K-step
// by four, so that a Z builder wave's 2-byte writes of 64 consecutive atoms
// (two K-steps, four atom groups, eight atoms each) fall in 32 different
// banks (16 ks + 4 grp + h / 2 modulo 32) instead of four
constexpr int kBParts = 4;
constexpr int kBGrpStride = 16 + 1;                          // halfv per atom-group row
constexpr int kBPartStride = 4 * kBGrpStride;                // halfv per part
constexpr int kBKsStride = kBParts * kBPartStride + 4;       // halfv per K-step
// atoms whose products the fp32 matrix accumulators sum before they are added
// to the double accumulators (256: the promotion's 16 conversions and double
// adds per 128-atom tile halve; C(0) of 2048 k at 10^6 atoms moves by 2e-7)
constexpr int kAccAtoms = 256;

// The LDS tile of TA atoms: K-steps, table row stride (float2; TA + 2 shifts
// consecutive rows by 4 banks) and B fragments per B tile.  128-atom tiles
// meet half the block-wide barriers of 64-atom tiles (n(k) 130 -> 108 us,
// currents 366 -> 333 us at 10^6 atoms).  One weight set always takes them;
// three weight sets need NB packed B tiles and take them only when two
// buffers fit in the 160 KB of LDS (k-sets with few table rows), else 64.
template <int TA> struct Tile {
    static constexpr int atoms = TA;
    static constexpr int ksteps = atoms / kKStep;
    static constexpr int stride = atoms + 2;
    static constexpr int bfrags = ksteps * kBKsStride; // halfv per B tile
    static constexpr int acc_tiles = kAccAtoms / atoms;
};
constexpr size_t kLdsBytes = 160 * 1024; // LDS of a CU (and most one block may take)

// Table tasks per tile: (axis, power part, atom), ordered X parts, Y parts, Z
// parts.  With three weight sets the Z task carries about three times the work
// of an X or Y task (three products and splits per power), so its powers are
// split in two parts on separate threads; with 64-atom tiles the X and Y
// powers are split as well, so that six waves still have a task per thread.
// With 128-atom tiles (z_pairs) the Z tasks take two neighbouring atoms per
// lane instead (table_role): a Z wave's build is bound by the latency of its
// dependent double operations, not by their issue, so two interleaved atoms
// cost far less than two waves, and the two waves this frees let one SIMD
// carry two contraction waves and no build.
template <int NW, int TA> struct TableShape {
    static constexpr int xy_parts = NW == 3 && TA == 64 ? 2 : 1;
    static constexpr int z_parts = NW == 3 ? 2 : 1;
    static constexpr bool z_pairs = NW == 3 && TA == 128;
    static constexpr int tasks = (2 * xy_parts + z_parts) * TA;
    static constexpr int min_waves = z_pairs ? 8 : tasks / 64; // every task has its own thread
};

// The table role of wave `twave` (uniform over the wave): axis d, power part
// hf, and the atom of lane 0 (a lane builds atom j0 + lane, or with pairs the
// atoms j0 + 2 lane and j0 + 2 lane + 1).
struct TableRole {
    bool builder;
    bool pairs;
    int d, hf, j0;
};

template <int NW, int TA> __device__ __forceinline__ TableRole table_role(int twave)
{
    TableRole r{false, false, 0, 0, 0};
    if constexpr (TableShape<NW, TA>::z_pairs) {
        // waves w and w + 4 share a SIMD: waves 0 and 4 only contract; X on
        // 1, 2 and Y on 3, 7 (64 atoms each), the Z powers' halves on 5, 6
        switch (twave) {
        case 1: r = TableRole{true, false, 0, 0, 0}; break;
        case 2: r = TableRole{true, false, 0, 0, 64}; break;
        case 3: r = TableRole{true, false, 1, 0, 0}; break;
        case 7: r = TableRole{true, false, 1, 0, 64}; break;
        case 5: r = TableRole{true, true, 2, 0, 0}; break;
        case 6: r = TableRole{true, true, 2, 1, 0}; break;
        default: break;
        }
    } else {
        // task t = 64 twave + lane: unit u = t / TA of X parts, Y parts, Z parts
        constexpr int xyp = TableShape<NW, TA>::xy_parts;
        const int t = twave * 64;
        const int u = t / TA;
        r.builder = t < TableShape<NW, TA>::tasks;
        r.j0 = t - u * TA;
        r.d = u < 2 * xyp ? u / xyp : 2;
        r.hf = u < 2 * xyp ? u - r.d * xyp : u - 2 * xyp;
    }
    return r;
}

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4_t mfma(half8_t a, half8_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// (the K = 16 form, for kWideK = false)
[[maybe_unused]] __device__ __forceinline__ float4_t mfma(half4_t a, half4_t b, float4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int bfrag_index(int ks, int part, int grp, int col)
{
    return ks * kBKsStride + part * kBPartStride + grp * kBGrpStride + col; // in halfv_t units
}

// Two floats to two fp16 (round to nearest even), packed low | high.
__device__ __forceinline__ uint32_t pack_half2(float a, float b)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef _Float16 h2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, h2v));
}

// lo = fp16(a - hi.low) | fp16(b - hi.high) << 16, each from one fused
// mixed-precision operation (the fp16 source negated, times 1, plus the fp32
// value, rounded once to fp16).
__device__ __forceinline__ void lo_half2(uint32_t &lo, uint32_t hi, float a, float b)
{
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(hi), "v"(a));
    asm("v_fma_mixhi_f16 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "+v"(lo)
        : "v"(hi), "v"(b));
}

__device__ __forceinline__ void cmul(double &r, double &i, double br, double bi)
{
    const double t = r * br - i * bi;
    i = r * bi + i * br;
    r = t;
}

// e^{2 pi i f} in double: f = q / kRoots + u with q the nearest multiple and
// |u| <= 1 / (2 kRoots); e^{2 pi i q / kRoots} from the block's table, e^{2 pi i u}
// from its Taylor series (|2 pi u| < 0.05: the first omitted terms are below
// 1e-19 relative).
__device__ __forceinline__ void unit_phase(double f, const double2 *roots, double &c, double &s)
{
    const double t = (f - floor(f)) * kRoots; // exact scaling
    const double q = rint(t);
    const double th = (t - q) * (2.0 * 3.14159265358979323846 / kRoots);
    const double t2 = th * th;
    const double cu = 1.0 + t2 * (-1.0 / 2 + t2 * (1.0 / 24 + t2 * (-1.0 / 720 + t2 * (1.0 / 40320))));
    const double su = th * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 +
                                                                     t2 * (1.0 / 362880)))));
    const double2 w = roots[(int)q & (kRoots - 1)];
    c = w.x * cu - w.y * su;
    s = w.x * su + w.y * cu;
}

struct TileBufs {
    float2 *tabx;   // [nn][Tile::stride]
    float2 *taby;   // [nn][Tile::stride]
    halfv_t *bfr;   // [NW][Tile::bfrags]
};

// Build the tables of one tile.  The B fragments of the NW weight sets are
// packed by column: column s (nmax + 1) + n of B tile (column / 16) holds
// w_s Z^n (NB = ceil(NW (nmax + 1) / 16) tiles instead of NW).
// Task (axis d, power part hf, atom j) of a lane (d and hf uniform over the
// wave, so all control flow is uniform): with two parts, part 0 takes n = 0
// .. n1 and part 1 takes n = n1+1 .. nmax (n1 = nmax / 2) starting from its
// own e^{2 pi i n1 x / L} (both from unit_phase).  Powers
// by a double recurrence, each rounded once; X and Y rows for both signs, and
// for each weight set w the products w * Z^n split into fp16 hi/lo B
// fragments (NW = 1: w = 1; NW = 3: the atom's velocity components).  Atoms
// past the end (live == false) get zero entries, so they add nothing.
template <int NW, int TA>
__device__ __forceinline__ void build_tile(const TileBufs &tb, int d, int hf, int j, bool live, float x,
                                           const float (&w)[NW], const double (&wsc)[NW],
                                           double inv_box, int nmax, int2 xrows, int2 yrows,
                                           const double2 *roots)
{
    const int parts = d < 2 ? TableShape<NW, TA>::xy_parts : TableShape<NW, TA>::z_parts;
    const int n1 = parts == 1 ? nmax : nmax / 2;
    const int n_begin = hf == 0 ? 0 : n1 + 1, n_end = hf == 0 ? n1 : nmax;
    const double f = (double)x * inv_box;
    // every lane evaluates (x = 0 past the end); a dead lane's powers are zero
    double cs, sn, pr = live ? 1.0 : 0.0, pi = 0.0;
    unit_phase(f, roots, cs, sn);
    if (hf != 0) {
        unit_phase(f * n1, roots, pr, pi); // e^{i n1 theta}; n1 f is exact to 1 ulp
        pr = live ? pr : 0.0;
        pi = live ? pi : 0.0;
    }
    if (d < 2) {
        // rows lo .. hi of this axis; row of power m at zero + m * stride
        const int lo = d == 0 ? xrows.x : yrows.x;
        const int hi = lo + (d == 0 ? xrows.y : yrows.y) - 1;
        float2 *zero = (d == 0 ? tb.tabx : tb.taby) + j - lo * Tile<TA>::stride;
        if (hf == 0 && lo <= 0 && hi >= 0) zero[0] = make_float2((float)pr, 0.f);
        const int n_last = min(n_end, max(-lo, hi));
        auto put = [&](int n, double r, double i) {
            if (n >= lo && n <= hi) zero[n * Tile<TA>::stride] = make_float2((float)r, (float)i);
            if (-n >= lo && -n <= hi) zero[-n * Tile<TA>::stride] = make_float2((float)r, -(float)i);
        };
        // two interleaved recurrences, powers n and n + 1 each stepping by
        // the squared base: half the dependent chain of a single recurrence
        const int n0 = n_begin > 0 ? n_begin : 1;
        double ar = pr, ai = pi, c2r = cs, c2i = sn;
        cmul(ar, ai, cs, sn); // power n0
        double br = ar, bi = ai;
        cmul(br, bi, cs, sn);   // power n0 + 1
        cmul(c2r, c2i, cs, sn); // the base squared
        for (int n = n0; n <= n_last; n += 2) {
            put(n, ar, ai);
            if (n + 1 <= n_last) put(n + 1, br, bi);
            cmul(ar, ai, c2r, c2i);
            cmul(br, bi, c2r, c2i);
        }
    } else {
        const int ks = j / kKStep, g = (j % kKStep) / kAtomsPerLane, h = j % kAtomsPerLane;
        // the lane's entry of column 0, part 0 of B tile 0; columns and B
        // tiles add a uniform offset, the parts a constant one
        _Float16 *const lane_b =
            reinterpret_cast<_Float16 *>(tb.bfr) + bfrag_index(ks, 0, g, 0) * kAtomsPerLane + h;
        auto store_z = [&](int n) {
#pragma unroll
            for (int s = 0; s < NW; ++s) {
                const double wd = NW == 1 ? 1.0 : (double)w[s] * wsc[s];
                const float zr = (float)(pr * wd), zi = (float)(pi * wd);
                // hi of both parts in one packed conversion, lo by one
                // mixed-precision fma each (as for P in the contraction)
                const uint32_t hh = pack_half2(zr, zi);
                uint32_t ll;
                lo_half2(ll, hh, zr, zi);
                typedef _Float16 h2v __attribute__((ext_vector_type(2)));
                const h2v H = __builtin_bit_cast(h2v, hh), L = __builtin_bit_cast(h2v, ll);
                const _Float16 rh = H[0], ih = H[1], rl = L[0], il = L[1];
                // column s (nmax + 1) + n of the packed B tiles
                const int gc = s * (nmax + 1) + n, bt = gc / kMfmaCols, c = gc % kMfmaCols;
                _Float16 *const e = lane_b + (bt * Tile<TA>::bfrags + c) * kAtomsPerLane;
                e[0] = rh;
                e[kBPartStride * kAtomsPerLane] = rl;
                e[2 * kBPartStride * kAtomsPerLane] = ih;
                e[3 * kBPartStride * kAtomsPerLane] = il;
            }
        };
        if (n_begin == 0) store_z(0);
        for (int n = n_begin > 0 ? n_begin : 1; n <= n_end; ++n) {
            cmul(pr, pi, cs, sn);
            store_z(n);
        }
    }
}

// Z fragments of a 128-atom tile from one wave: lane l builds the neighbouring
// atoms 2 l and 2 l + 1 (the same atom group, h and h + 1), powers n_begin ..
// n_end of part hf (as in build_tile), the two atoms' recurrences interleaved,
// and writes each part of a power of both atoms as one 4-byte entry (the
// group's halves h, h + 1).  Atoms past the end (live false) get zero entries.
template <int NW, int TA>
__device__ __forceinline__ void build_z_pairs(const TileBufs &tb, int lane, int hf, const bool (&live)[2],
                                              const float (&x)[2], const float (&w)[2][NW],
                                              const double (&wsc)[NW], double inv_box, int nmax,
                                              const double2 *roots)
{
    static_assert(TA == 128, "a wave of atom pairs covers a 128-atom tile");
    const int n1 = nmax / 2;
    const int n_begin = hf == 0 ? 0 : n1 + 1, n_end = hf == 0 ? n1 : nmax;
    double cs[2], sn[2], pr[2], pi[2], wd[2][NW];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const double f = (double)x[e] * inv_box;
        unit_phase(f, roots, cs[e], sn[e]);
        pr[e] = live[e] ? 1.0 : 0.0;
        pi[e] = 0.0;
        if (hf != 0) {
            unit_phase(f * n1, roots, pr[e], pi[e]); // e^{i n1 theta}; n1 f is exact to 1 ulp
            pr[e] = live[e] ? pr[e] : 0.0;
            pi[e] = live[e] ? pi[e] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < NW; ++s) wd[e][s] = NW == 1 ? 1.0 : (double)w[e][s] * wsc[s];
    }
    const int j = 2 * lane;
    const int ks = j / kKStep, g = (j % kKStep) / kAtomsPerLane, h = j % kAtomsPerLane; // h even
    // the lane's entry (halves h, h + 1) of column 0, part 0 of B tile 0
    uint32_t *const lane_b =
        reinterpret_cast<uint32_t *>(tb.bfr) + bfrag_index(ks, 0, g, 0) * (kAtomsPerLane / 2) + h / 2;
    auto store_z = [&](int n) {
#pragma unroll
        for (int s = 0; s < NW; ++s) {
            const float zr0 = (float)(pr[0] * wd[0][s]), zr1 = (float)(pr[1] * wd[1][s]);
            const float zi0 = (float)(pi[0] * wd[0][s]), zi1 = (float)(pi[1] * wd[1][s]);
            // hi of both atoms in one packed conversion, lo by one
            // mixed-precision fma each (as for P in the contraction)
            const uint32_t hr = pack_half2(zr0, zr1), hi = pack_half2(zi0, zi1);
            uint32_t lr, li;
            lo_half2(lr, hr, zr0, zr1);
            lo_half2(li, hi, zi0, zi1);
            // column s (nmax + 1) + n of the packed B tiles
            const int gc = s * (nmax + 1) + n, bt = gc / kMfmaCols, c = gc % kMfmaCols;
            uint32_t *const e = lane_b + (bt * Tile<TA>::bfrags + c) * (kAtomsPerLane / 2);
            e[0] = hr;
            e[kBPartStride * (kAtomsPerLane / 2)] = lr;
            e[2 * kBPartStride * (kAtomsPerLane / 2)] = hi;
            e[3 * kBPartStride * (kAtomsPerLane / 2)] = li;
        }
    };
    if (n_begin == 0) store_z(0);
    for (int n = n_begin > 0 ? n_begin : 1; n <= n_end; ++n) {
#pragma unroll
        for (int e = 0; e < 2; ++e) cmul(pr[e], pi[e], cs[e], sn[e]);
        store_z(n);
    }
}

// Waves per block: one M tile per contraction wave.  With three weight sets a
// wave holds the accumulators of NB B tiles (about 200 registers for two), so
// blocks stay at two waves per SIMD.
template <int NW> struct MfmaShape {
    static constexpr int max_waves = NW == 1 ? kMfmaMaxWaves : 8;
};

template <int NW, int TA, int NB> __device__ __forceinline__ void rhok_mfma_body(const RhokMfmaArgs &a)
{
    if (a.stamps && threadIdx.x == 0) stamp_start(a.stamps, blockIdx.x + gridDim.x * blockIdx.y);
    extern __shared__ double2 lds_roots[]; // [kRoots], the scale slots, then two tile buffers
    const int nmax = a.nmax;
    const int2 xrows = make_int2(a.x_lo, a.x_rows), yrows = make_int2(a.y_lo, a.y_rows);
    // two tile buffers of buf_stride float2 each (a multiple of 2: 16-byte aligned)
    float2 *const buf0 = reinterpret_cast<float2 *>(lds_roots + kRoots + ScaleSlots<NW>::n);
    const int buf_stride =
        (a.x_rows + a.y_rows) * Tile<TA>::stride +
        NB * Tile<TA>::bfrags * (int)(sizeof(halfv_t) / sizeof(float2));
    auto tile_bufs = [&](int b) {
        TileBufs t;
        t.tabx = buf0 + b * buf_stride;
        t.taby = t.tabx + a.x_rows * Tile<TA>::stride;
        t.bfr = reinterpret_cast<halfv_t *>(t.taby + a.y_rows * Tile<TA>::stride);
        return t;
    };

    const int waves = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int col = lane & 15; // A row / B column within the tile
    const int grp = lane >> 4; // atom group of the K-step
    // the M tiles dealt evenly over the chunks (gridDim.x), one per wave from
    // wave 0; the waves past them only build tables
    const int per_chunk = (a.n_mtiles + (int)gridDim.x - 1) / (int)gridDim.x;
    const int mt = blockIdx.x * per_chunk + wave;
    const bool active = wave < per_chunk && mt < a.n_mtiles; // wave-uniform
    const int pm_row = mt * 16 + col;
    const int ax = active ? a.pair_nx[pm_row] - a.x_lo : 0; // table rows
    const int ay = active ? a.pair_ny[pm_row] - a.y_lo : 0;
    // the lane's X and Y rows at its first atom (16-byte aligned) per buffer
    const int xoff = ax * Tile<TA>::stride + grp * kAtomsPerLane;
    const int yoff = ay * Tile<TA>::stride + grp * kAtomsPerLane;
    const int boff = bfrag_index(0, 0, grp, col);

    for (int q = threadIdx.x; q < kRoots; q += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * q / kRoots, &sn, &cs);
        lds_roots[q] = make_double2(cs, sn);
    }
    // packed B columns past NW (nmax + 1) are never stored; keep them zero
    // (f runs over (buffer, B tile, K-step, part, group, column))
    const int ncols = NW * (nmax + 1);
    constexpr int kRowsPerTile = Tile<TA>::ksteps * kBParts * 4;
    for (int f = threadIdx.x; f < 2 * NB * kRowsPerTile * kMfmaCols; f += blockDim.x) {
        const int c = f % kMfmaCols, r = f / kMfmaCols;
        const int gq = r % 4, part = (r / 4) % kBParts, ks = (r / (4 * kBParts)) % Tile<TA>::ksteps;
        const int bt = (r / kRowsPerTile) % NB, b = r / (kRowsPerTile * NB);
        if (bt * kMfmaCols + c >= ncols)
            tile_bufs(b).bfr[bt * Tile<TA>::bfrags + bfrag_index(ks, part, gq, c)] = halfv_t{};
    }

    double acc[NB][4][4];
    float4_t sum[NB][4]; // products of the last Tile::acc_tiles tiles at most
#pragma unroll
    for (int w = 0; w < NB; ++w)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[w][s][v] = 0.0;
            sum[w][s] = float4_t{0.f, 0.f, 0.f, 0.f};
        }

    const int64_t a_begin = (int64_t)blockIdx.y * a.atoms_per_block;
    int64_t a_end = a_begin + a.atoms_per_block;
    if (a_end > a.n_atoms) a_end = a.n_atoms;
    const int n_tiles =
        a_end > a_begin ? (int)((a_end - a_begin + Tile<TA>::atoms - 1) / Tile<TA>::atoms) : 0;

    // Weight scales: 2^-e per weight set with e the binary exponent of the
    // largest |w| over the block's atoms (frexp: max |w| 2^-e in [1/2, 1)),
    // so that every split operand keeps its 22 bits relative to that maximum
    // in any velocity units; wunsc = 2^e restores the double sums.
    double wsc[NW], wunsc[NW];
#pragma unroll
    for (int s = 0; s < NW; ++s) wsc[s] = wunsc[s] = 1.0;
    if constexpr (NW > 1) {
        float *red = reinterpret_cast<float *>(lds_roots + kRoots); // [waves][NW]
        float mx[NW];
#pragma unroll
        for (int s = 0; s < NW; ++s) mx[s] = 0.f;
        for (int64_t at = a_begin + threadIdx.x; at < a_end; at += blockDim.x)
#pragma unroll
            for (int s = 0; s < NW; ++s) mx[s] = fmaxf(mx[s], fabsf(a.pos[(int64_t)(3 + s) * a.n_atoms + at]));
#pragma unroll
        for (int s = 0; s < NW; ++s)
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) mx[s] = fmaxf(mx[s], __shfl_xor(mx[s], off, 64));
        if (lane == 0)
#pragma unroll
            for (int s = 0; s < NW; ++s) red[wave * NW + s] = mx[s];
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NW; ++s) {
            float m = 0.f;
            for (int w2 = 0; w2 < waves; ++w2) m = fmaxf(m, red[w2 * NW + s]);
            if (m > 0.f) {
                int ex = 0;
                (void)frexpf(m, &ex);
                wsc[s] = ldexp(1.0, -ex);
                wunsc[s] = ldexp(1.0, ex);
            }
        }
    }

    // table role of this wave and its inputs, loaded one tile ahead of their
    // use; the Z tasks also load the weights.  The role is taken from a
    // wave-uniform copy of the wave index (the build's loops and branches then
    // stay scalar; `wave` itself stays a vector value, which measured 6%
    // faster in the contraction).
    const int twave = __builtin_amdgcn_readfirstlane(wave);
    const TableRole role = table_role<NW, TA>(twave);
    const bool builder = role.builder; // wave-uniform
    const int td = role.d;
    const bool weighted = NW > 1 && td == 2;
    // the lane's atoms of the tile: one, or two neighbours (Z pairs)
    auto atom_of = [&](int e) { return role.pairs ? role.j0 + 2 * lane + e : role.j0 + lane; };
    auto load_in = [&](int it, float (&x)[2], float (&w)[2][NW], bool (&lv)[2]) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t at = a_begin + (int64_t)it * Tile<TA>::atoms + atom_of(e);
            lv[e] = builder && (e == 0 || role.pairs) && it < n_tiles && at < a_end;
            x[e] = lv[e] ? a.pos[(int64_t)td * a.n_atoms + at] : 0.f;
#pragma unroll
            for (int s = 0; s < NW; ++s)
                w[e][s] = lv[e] && weighted ? a.pos[(int64_t)(3 + s) * a.n_atoms + at] : 1.f;
        }
    };
    auto build = [&](const TileBufs &tb, const float (&x)[2], const float (&w)[2][NW],
                     const bool (&lv)[2]) {
        if constexpr (TableShape<NW, TA>::z_pairs) {
            if (role.pairs) {
                build_z_pairs<NW, TA>(tb, lane, role.hf, lv, x, w, wsc, a.inv_box, nmax, lds_roots);
                return;
            }
        }
        build_tile<NW, TA>(tb, role.d, role.hf, atom_of(0), lv[0], x[0], w[0], wsc, a.inv_box, nmax,
                           xrows, yrows, lds_roots);
    };
    float x_cur[2], x_next[2], w_cur[2][NW], w_next[2][NW];
    bool live_cur[2], live_next[2];
    load_in(0, x_cur, w_cur, live_cur);
    load_in(1, x_next, w_next, live_next);
    __syncthreads(); // roots and zero columns
    if (builder) build(tile_bufs(0), x_cur, w_cur, live_cur);
    __syncthreads();

    for (int it = 0; it < n_tiles; ++it) {
        const TileBufs cur = tile_bufs(it & 1);
        // tables of the next tile into the other buffer; the inputs of the
        // tile after that are loaded after the build and moved up after this
        // tile's contraction, so that no wave waits for them: loaded before
        // the build, or moved up right after it, they cost every builder wave
        // a memory latency per tile (the loads are conditional, so a wait
        // for older ones waits for them too)
        const bool building = builder && it + 1 < n_tiles;
        float x_after[2] = {0.f, 0.f}, w_after[2][NW];
        bool live_after[2] = {false, false};
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int s = 0; s < NW; ++s) w_after[e][s] = 1.f;
        if (building) {
            build(tile_bufs((it + 1) & 1), x_next, w_next, live_next);
            load_in(it + 2, x_after, w_after, live_after);
        }
        if (active) {
            const float4 *xrow = reinterpret_cast<const float4 *>(cur.tabx + xoff);
            const float4 *yrow = reinterpret_cast<const float4 *>(cur.taby + yoff);
            // all K-steps of the tile: the entries of atoms past the end are zero
#pragma unroll
            for (int ks = 0; ks < Tile<TA>::ksteps; ++ks) {
                uint32_t wrh[kAtomsPerLane / 2], wrl[kAtomsPerLane / 2];
                uint32_t wih[kAtomsPerLane / 2], wil[kAtomsPerLane / 2];
#pragma unroll
                for (int q2 = 0; q2 < kAtomsPerLane / 2; ++q2) {
                    const float4 x = xrow[ks * (kKStep / 2) + q2];
                    const float4 y = yrow[ks * (kKStep / 2) + q2];
                    const float xr[2] = {x.x, x.z}, xi[2] = {x.y, x.w};
                    const float yr[2] = {y.x, y.z}, yi[2] = {y.y, y.w};
                    float pr[2], pi[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        pr[e] = __builtin_fmaf(xr[e], yr[e], -xi[e] * yi[e]);
                        pi[e] = __builtin_fmaf(xr[e], yi[e], xi[e] * yr[e]);
                    }
                    // hi = fp16(v) for both atoms in one packed conversion; lo =
                    // fp16(v - hi) by a mixed-precision fma that reads hi as fp16
                    // (one instruction per value, no round trip through fp32)
                    const uint32_t hr = pack_half2(pr[0], pr[1]);
                    const uint32_t hi = pack_half2(pi[0], pi[1]);
                    uint32_t lr, li;
                    lo_half2(lr, hr, pr[0], pr[1]);
                    lo_half2(li, hi, pi[0], pi[1]);
                    wrh[q2] = hr;
                    wrl[q2] = lr;
                    wih[q2] = hi;
                    wil[q2] = li;
                }
                typedef uint32_t wv_t __attribute__((ext_vector_type(kAtomsPerLane / 2)));
                wv_t vrh, vrl, vih, vil;
#pragma unroll
                for (int q2 = 0; q2 < kAtomsPerLane / 2; ++q2) {
                    vrh[q2] = wrh[q2];
                    vrl[q2] = wrl[q2];
                    vih[q2] = wih[q2];
                    vil[q2] = wil[q2];
                }
                const halfv_t prh = __builtin_bit_cast(halfv_t, vrh);
                const halfv_t prl = __builtin_bit_cast(halfv_t, vrl);
                const halfv_t pih = __builtin_bit_cast(halfv_t, vih);
                const halfv_t pil = __builtin_bit_cast(halfv_t, vil);
#pragma unroll
                for (int w = 0; w < NB; ++w) {
                    const halfv_t *bl = cur.bfr + w * Tile<TA>::bfrags + boff;
                    const halfv_t zrh = bl[bfrag_index(ks, 0, 0, 0)];
                    const halfv_t zrl = bl[bfrag_index(ks, 1, 0, 0)];
                    const halfv_t zih = bl[bfrag_index(ks, 2, 0, 0)];
                    const halfv_t zil = bl[bfrag_index(ks, 3, 0, 0)];
                    float4_t *sw = sum[w];
                    // interleaved so that dependent products on one sum are apart
                    sw[0] = mfma(prh, zrh, sw[0]);
                    sw[1] = mfma(pih, zih, sw[1]);
                    sw[2] = mfma(prh, zih, sw[2]);
                    sw[3] = mfma(pih, zrh, sw[3]);
                    sw[0] = mfma(prh, zrl, sw[0]);
                    sw[1] = mfma(pih, zil, sw[1]);
                    sw[2] = mfma(prh, zil, sw[2]);
                    sw[3] = mfma(pih, zrl, sw[3]);
                    sw[0] = mfma(prl, zrh, sw[0]);
                    sw[1] = mfma(pil, zih, sw[1]);
                    sw[2] = mfma(prl, zih, sw[2]);
                    sw[3] = mfma(pil, zrh, sw[3]);
                }
            }
            if ((it + 1) % Tile<TA>::acc_tiles == 0 || it + 1 == n_tiles) {
#pragma unroll
                for (int w = 0; w < NB; ++w)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[w][s][v] += (double)sum[w][s][v];
                        sum[w][s] = float4_t{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        if (building) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                x_next[e] = x_after[e];
#pragma unroll
                for (int s = 0; s < NW; ++s) w_next[e][s] = w_after[e][s];
                live_next[e] = live_after[e];
            }
        }
        __syncthreads(); // next buffer complete; this one free for the tile after
    }
    if (!active) return;
    // Row pm = pair; the lane's column of B tile w is packed column
    // 16 w + col = s (nmax + 1) + |n_z| of weight set s.  Only slots that are
    // k-vectors of the group are stored, in partial[k][weight set][atom block].
#pragma unroll
    for (int w = 0; w < NB; ++w) {
        const int gc = w * kMfmaCols + col;
        if (gc >= ncols) continue;
        const int s = gc / (nmax + 1), nz = gc - s * (nmax + 1);
        double un = wunsc[0]; // the set's scale back (a select: no indexed private array)
#pragma unroll
        for (int q = 1; q < NW; ++q) un = s == q ? wunsc[q] : un;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int pm = mt * 16 + grp * 4 + v;
            const int32_t *sk = a.slot_k + ((size_t)pm * kMfmaCols + nz) * 2;
            const int kp = sk[0], km = sk[1];
            if (kp >= 0) {
                double *dst = a.partial + (((size_t)kp * NW + s) * a.n_atom_blocks + blockIdx.y) * 2;
                dst[0] = (acc[w][0][v] - acc[w][1][v]) * un;
                dst[1] = (acc[w][2][v] + acc[w][3][v]) * un;
            }
            if (km >= 0) {
                double *dst = a.partial + (((size_t)km * NW + s) * a.n_atom_blocks + blockIdx.y) * 2;
                dst[0] = (acc[w][0][v] + acc[w][1][v]) * un;
                dst[1] = (acc[w][3][v] - acc[w][2][v]) * un;
            }
        }
    }
}

template <int NW, int TA, int NB> __global__ void rhok_mfma_kernel(RhokMfmaArgs a);


// Three weight sets (currents), NB packed B tiles.
#define CORR_CURRENT_KERNEL(TA, NB)                                                               \
    template <>                                                                                   \
    __global__ __launch_bounds__(MfmaShape<3>::max_waves * 64) void rhok_mfma_kernel<3, TA, NB>( \
        RhokMfmaArgs a)                                                                           \
    {                                                                                             \
        rhok_mfma_body<3, TA, NB>(a);                                                             \
    }
CORR_CURRENT_KERNEL(64, 1)
CORR_CURRENT_KERNEL(64, 2)
CORR_CURRENT_KERNEL(64, 3)
CORR_CURRENT_KERNEL(128, 1)
CORR_CURRENT_KERNEL(128, 2)
CORR_CURRENT_KERNEL(128, 3)
#undef CORR_CURRENT_KERNEL

// ---- One weight set (n(k)): rows of couples ------------------------------
//
// The k-set's (n_x, n_y) pairs come in couples (a, +|b|), (a, -|b|) that share
// X = X^a and Y = Y^|b| (Y^{-|b|} = conj Y^|b|).  With the four real products
//     u = Xr Yr,  v = Xi Yi,  w = Xi Yr,  t = Xr Yi
// per atom, P(a, +|b|) = (u - v) + i (t + w) and P(a, -|b|) = (u + v) + i (w - t).
// The contraction's rows are (couple, component): a tile of 16 rows holds 4
// couples, row 4c + q the component q (u, v, w, t) of couple c, and each row
// is summed against Re z and Im z (two sums, three split products each).
// Every sign combination of (n_y, n_z) follows at the end from these eight
// sums of a couple by additions in double (the sums are linear in the
// products).  Per row and atom: one product and its split (2.5 vector
// instructions) instead of a complex product and the split of both parts for
// each pair (7 per pair; 5 per pair here).  A lane's four accumulator values
// of a tile are the four components of one couple at one |n_z| (D row 4g + v),
// so the combination needs no data from other lanes.
//
// Tables: X and Y as separate real and imaginary planes of float
// [2][rows][kPlaneStride] (X: n_x in [x_lo, x_lo + x_rows); Y: |n_y| in
// [0, y_rows)), Z split in B-fragment order as for the pairs.  Waves: each
// contraction wave takes kCpTilesPerWave tiles; waves 0, 1 build the X planes
// and 2, 3 the Y planes besides their tiles; the block's last wave builds the
// Z fragments, two atoms per lane (two interleaved recurrences).
constexpr int kCpTilesPerWave = 2;
constexpr int kCpMaxCWaves = kMfmaMaxWaves - 1;
constexpr int kCpMinCWaves = 4;               // waves 0 .. 3 build X and Y
constexpr int kPlaneStride = 128 + 4;         // floats per plane row (128-atom tiles); +4 banks per row
// B fragments of the couple kernel: the pair kernels' layout with a padded
// atom-group row (17 halfv) and K-step (+8 halfv), so that the Z builder's
// 2-byte writes of 64 atoms spread over 32 banks instead of 4.
constexpr int kCpGrpStride = kMfmaCols + 1;
constexpr int kCpKsStride = kBParts * 4 * kCpGrpStride + 8;
constexpr int kCpBfrags = Tile<128>::ksteps * kCpKsStride; // halfv per buffer
__device__ __forceinline__ int cp_bfrag_index(int ks, int part, int grp, int col)
{
    return ks * kCpKsStride + (part * 4 + grp) * kCpGrpStride + col; // in halfv_t units
}

struct CpBufs {
    float *xp;      // [2][x_rows][kPlaneStride]: real plane, then imaginary plane
    float *yp;      // [2][y_rows][kPlaneStride]
    halfv_t *bfr;   // [kCpBfrags] (cp_bfrag_index)
};

// X (d = 0) or Y (d = 1) planes of atom j of the tile: powers n in
// [lo, lo + rows) by a double recurrence from e^{2 pi i x / L}, each rounded
// once to float; a dead lane (past the atoms) writes zeros.  lo, rows and d
// are uniform over the wave, so the loop and its conditions are scalar.
// (Shorter dependency chains, e^{n+4} = e^n e^4 four at a time, measured no
// faster.)
__device__ __forceinline__ void cp_build_planes(float *plane0, int rows, int lo, int j, bool live,
                                                float x, double inv_box, const double2 *roots)
{
    double cs, sn, pr = live ? 1.0 : 0.0, pi = 0.0;
    unit_phase((double)x * inv_box, roots, cs, sn);
    float *re = plane0 + j - lo * kPlaneStride; // power m at re + m * kPlaneStride
    float *im = re + rows * kPlaneStride;
    const int hi = lo + rows - 1;
    if (lo <= 0 && hi >= 0) {
        re[0] = (float)pr;
        im[0] = 0.f;
    }
    const int n_last = max(-lo, hi);
    for (int n = 1; n <= n_last; ++n) {
        cmul(pr, pi, cs, sn);
        const float fr = (float)pr, fi = (float)pi;
        if (n >= lo && n <= hi) {
            re[n * kPlaneStride] = fr;
            im[n * kPlaneStride] = fi;
        }
        if (-n >= lo && -n <= hi) {
            re[-n * kPlaneStride] = fr;
            im[-n * kPlaneStride] = -fi;
        }
    }
}

// Z fragments of atoms 2 lane and 2 lane + 1 of the tile (|n_z| = 0 .. nmax):
// the two atoms are neighbours in a B fragment, so each part of a power is
// one 4-byte write of both atoms' halves.
__device__ __forceinline__ void cp_build_z(halfv_t *bfr, int lane, const bool (&live)[2],
                                           const float (&z)[2], double inv_box, int nmax,
                                           const double2 *roots)
{
    double cs[2], sn[2], pr[2], pi[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        unit_phase((double)z[e] * inv_box, roots, cs[e], sn[e]);
        pr[e] = live[e] ? 1.0 : 0.0;
        pi[e] = 0.0;
    }
    const int j = 2 * lane;
    const int ks = j / kKStep, g = (j % kKStep) / kAtomsPerLane, h = j % kAtomsPerLane;
    // dword of the pair in part 0 of power 0; parts kPart dwords apart
    uint32_t *const b0 = reinterpret_cast<uint32_t *>(bfr) + cp_bfrag_index(ks, 0, g, 0) * (kAtomsPerLane / 2) + h / 2;
    constexpr int kPart = 4 * kCpGrpStride * (kAtomsPerLane / 2);
    auto store = [&](int n) {
        const float r0 = (float)pr[0], r1 = (float)pr[1], i0 = (float)pi[0], i1 = (float)pi[1];
        const uint32_t rh = pack_half2(r0, r1), ih = pack_half2(i0, i1);
        uint32_t rl, il;
        lo_half2(rl, rh, r0, r1);
        lo_half2(il, ih, i0, i1);
        uint32_t *b = b0 + n * (kAtomsPerLane / 2);
        b[0] = rh;
        b[kPart] = rl;
        b[2 * kPart] = ih;
        b[3 * kPart] = il;
    };
    store(0);
    for (int n = 1; n <= nmax; ++n) {
        cmul(pr[0], pi[0], cs[0], sn[0]);
        cmul(pr[1], pi[1], cs[1], sn[1]);
        store(n);
    }
}

//
// EARLY: the table builders load the inputs of the tile after next before their
// build and move them up right after it.  The builder waves then wait for those
// loads once per tile (the loads are conditional, so the wait covers them), and
// that wait leaves issue slots to a flush kernel running beside the producer:
// with a fork and join on every push the batched step took 0.198-0.203 ms this
// way against 0.211-0.218 with the loads after the build.  Alone, or with the
// two streams joined every few pushes, loading after the build and moving the
// inputs up after the contraction is faster (93.7 against 96.6 us alone).
template <bool EARLY>
__device__ __forceinline__ void rhok_couple_body(const RhokMfmaArgs &a)
{
    constexpr int TA = 128;
    if (a.stamps && threadIdx.x == 0) stamp_start(a.stamps, blockIdx.x + gridDim.x * blockIdx.y);
    extern __shared__ double2 lds_roots[]; // [kRoots], then two tile buffers
    const int nmax = a.nmax;
    const int plane_rows = 2 * (a.x_rows + a.y_rows);
    // buffer: X planes, Y planes, B fragments (float units; 16-byte aligned)
    const int buf_floats = plane_rows * kPlaneStride + kCpBfrags * (int)(sizeof(halfv_t) / sizeof(float));
    float *const buf0 = reinterpret_cast<float *>(lds_roots + kRoots);
    auto bufs = [&](int b) {
        CpBufs t;
        t.xp = buf0 + b * buf_floats;
        t.yp = t.xp + 2 * a.x_rows * kPlaneStride;
        t.bfr = reinterpret_cast<halfv_t *>(t.yp + 2 * a.y_rows * kPlaneStride);
        return t;
    };
    const int waves = blockDim.x >> 6;
    const int cwaves = waves - 1; // the last wave builds Z
    const int wave = threadIdx.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const int lane = threadIdx.x & 63;
    const int col = lane & 15; // A row / B column within the tile
    const int grp = lane >> 4; // atom group of the K-step; couple of the lane's D rows
    const int cq = col & 3;    // the lane's A row: component cq of couple col / 4
    int tile[kCpTilesPerWave];
    bool act[kCpTilesPerWave]; // wave-uniform
    int xoff[kCpTilesPerWave], yoff[kCpTilesPerWave];
#pragma unroll
    for (int t = 0; t < kCpTilesPerWave; ++t) {
        tile[t] = (blockIdx.x * cwaves + wave) * kCpTilesPerWave + t;
        act[t] = wave < cwaves && tile[t] < a.n_mtiles;
        const int gc = act[t] ? tile[t] * 4 + (col >> 2) : 0; // the lane's A-row couple
        const int ax = act[t] ? a.pair_nx[gc] - a.x_lo : 0;
        const int ay = act[t] ? a.pair_ny[gc] - a.y_lo : 0;
        // u = Xr Yr, v = Xi Yi, w = Xi Yr, t = Xr Yi
        const int xpl = cq == 0 || cq == 3 ? 0 : 1, ypl = cq == 0 || cq == 2 ? 0 : 1;
        xoff[t] = (xpl * a.x_rows + ax) * kPlaneStride + grp * kAtomsPerLane;
        yoff[t] = (ypl * a.y_rows + ay) * kPlaneStride + grp * kAtomsPerLane;
    }
    const int boff = grp * kCpGrpStride + col;

    for (int q = threadIdx.x; q < kRoots; q += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * q / kRoots, &sn, &cs);
        lds_roots[q] = make_double2(cs, sn);
    }
    // B columns above nmax are never stored; keep them zero
    for (int f = threadIdx.x; f < 2 * Tile<TA>::ksteps * kBParts * 4 * kMfmaCols; f += blockDim.x) {
        const int c = f % kMfmaCols, r = f / kMfmaCols; // r: (buffer, K-step, part, group)
        const int gq = r % 4, part = (r / 4) % kBParts, ks = (r / (4 * kBParts)) % Tile<TA>::ksteps;
        if (c > nmax) bufs(r / (4 * kBParts * Tile<TA>::ksteps)).bfr[cp_bfrag_index(ks, part, gq, c)] = halfv_t{};
    }

    double acc[kCpTilesPerWave][2][4];
    float4_t sum[kCpTilesPerWave][2];
#pragma unroll
    for (int t = 0; t < kCpTilesPerWave; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][s][v] = 0.0;
            sum[t][s] = float4_t{0.f, 0.f, 0.f, 0.f};
        }

    const int64_t a_begin = (int64_t)blockIdx.y * a.atoms_per_block;
    int64_t a_end = a_begin + a.atoms_per_block;
    if (a_end > a.n_atoms) a_end = a.n_atoms;
    const int n_tiles =
        a_end > a_begin ? (int)((a_end - a_begin + Tile<TA>::atoms - 1) / Tile<TA>::atoms) : 0;

    // builders: waves 0, 1 the X planes, 2, 3 the Y planes (atom 64 (w & 1) +
    // lane), the last wave the Z fragments (atoms 2 lane, 2 lane + 1)
    const bool zb = wv == waves - 1;
    const bool xyb = wv < 4;
    const int bd = wv >> 1;                 // X/Y builder: axis
    const int bj = (wv & 1) * 64 + lane;    // X/Y builder: atom of the tile
    auto load_in = [&](int it, float (&in)[2], bool (&lv)[2]) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int j = zb ? 2 * lane + e : bj;
            const int64_t at = a_begin + (int64_t)it * TA + j;
            lv[e] = (zb || (xyb && e == 0)) && it < n_tiles && at < a_end;
            in[e] = lv[e] ? a.pos[(int64_t)(zb ? 2 : bd) * a.n_atoms + at] : 0.f;
        }
    };
    auto build = [&](const CpBufs &tb, const float (&in)[2], const bool (&lv)[2]) {
        if (zb)
            cp_build_z(tb.bfr, lane, lv, in, a.inv_box, nmax, lds_roots);
        else if (xyb)
            cp_build_planes(bd == 0 ? tb.xp : tb.yp, bd == 0 ? a.x_rows : a.y_rows,
                            bd == 0 ? a.x_lo : a.y_lo, bj, lv[0], in[0], a.inv_box, lds_roots);
    };
    float in_cur[2], in_next[2];
    bool lv_cur[2], lv_next[2];
    load_in(0, in_cur, lv_cur);
    load_in(1, in_next, lv_next);
    __syncthreads(); // roots and zero columns
    build(bufs(0), in_cur, lv_cur);
    __syncthreads();

    for (int it = 0; it < n_tiles; ++it) {
        const CpBufs cur = bufs(it & 1);
        // tables of the next tile into the other buffer; the inputs of the
        // tile after that are loaded before (EARLY) or after the build and
        // move up right after the build (EARLY) or after this tile's
        // contraction
        const bool building = (zb || xyb) && it + 1 < n_tiles;
        float in_after[2] = {0.f, 0.f};
        bool lv_after[2] = {false, false};
        if (building) {
            if constexpr (EARLY) load_in(it + 2, in_after, lv_after);
            build(bufs((it + 1) & 1), in_next, lv_next);
            if constexpr (EARLY) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    in_next[e] = in_after[e];
                    lv_next[e] = lv_after[e];
                }
            } else {
                load_in(it + 2, in_after, lv_after);
            }
        }
        if (act[0]) {
            const halfv_t *bl = cur.bfr + boff;
            // all K-steps of the tile: the entries of atoms past the end are zero
#pragma unroll
            for (int ks = 0; ks < Tile<TA>::ksteps; ++ks) {
                const halfv_t zrh = bl[cp_bfrag_index(ks, 0, 0, 0)];
                const halfv_t zrl = bl[cp_bfrag_index(ks, 1, 0, 0)];
                const halfv_t zih = bl[cp_bfrag_index(ks, 2, 0, 0)];
                const halfv_t zil = bl[cp_bfrag_index(ks, 3, 0, 0)];
#pragma unroll
                for (int t = 0; t < kCpTilesPerWave; ++t) {
                    if (!act[t]) continue;
                    const float4 *xr = reinterpret_cast<const float4 *>(cur.xp + xoff[t] + ks * kKStep);
                    const float4 *yr = reinterpret_cast<const float4 *>(cur.yp + yoff[t] + ks * kKStep);
                    typedef uint32_t wv_t __attribute__((ext_vector_type(kAtomsPerLane / 2)));
                    wv_t vh, vl;
#pragma unroll
                    for (int q4 = 0; q4 < kAtomsPerLane / 4; ++q4) {
                        const float4 x = xr[q4], y = yr[q4];
                        const float c0 = x.x * y.x, c1 = x.y * y.y, c2 = x.z * y.z, c3 = x.w * y.w;
                        // hi = fp16(v) two atoms per packed conversion, lo = fp16(v - hi)
                        const uint32_t h01 = pack_half2(c0, c1), h23 = pack_half2(c2, c3);
                        uint32_t l01, l23;
                        lo_half2(l01, h01, c0, c1);
                        lo_half2(l23, h23, c2, c3);
                        vh[2 * q4] = h01;
                        vh[2 * q4 + 1] = h23;
                        vl[2 * q4] = l01;
                        vl[2 * q4 + 1] = l23;
                    }
                    const halfv_t ch = __builtin_bit_cast(halfv_t, vh);
                    const halfv_t cl = __builtin_bit_cast(halfv_t, vl);
                    float4_t *sw = sum[t];
                    sw[0] = mfma(ch, zrh, sw[0]);
                    sw[1] = mfma(ch, zih, sw[1]);
                    sw[0] = mfma(ch, zrl, sw[0]);
                    sw[1] = mfma(ch, zil, sw[1]);
                    sw[0] = mfma(cl, zrh, sw[0]);
                    sw[1] = mfma(cl, zih, sw[1]);
                }
            }
            if ((it + 1) % Tile<TA>::acc_tiles == 0 || it + 1 == n_tiles) {
#pragma unroll
                for (int t = 0; t < kCpTilesPerWave; ++t)
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[t][s][v] += (double)sum[t][s][v];
                        sum[t][s] = float4_t{0.f, 0.f, 0.f, 0.f};
                    }
            }
        }
        if (!EARLY && building) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                in_next[e] = in_after[e];
                lv_next[e] = lv_after[e];
            }
        }
        __syncthreads(); // next buffer complete; this one free for the tile after
    }
    // The lane's accumulator values v = 0..3 are the components u, v, w, t of
    // couple grp of the tile at |n_z| = col, against Re z (s = 0) and Im z (s
    // = 1).  Slots [couple][|n_z|][n_y < 0][n_z < 0] that are k-vectors of the
    // group are stored in partial[k][atom block].
#pragma unroll
    for (int t = 0; t < kCpTilesPerWave; ++t) {
        if (!act[t]) continue;
        const int gc = tile[t] * 4 + grp;
        const double ur = acc[t][0][0], vr = acc[t][0][1], wr = acc[t][0][2], tr = acc[t][0][3];
        const double ui = acc[t][1][0], vi = acc[t][1][1], wi = acc[t][1][2], ti = acc[t][1][3];
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
            // P = (u -+ v) + i (t + w  |  w - t): sums against Re z (R) and Im z (I)
            const double prR = sb ? ur + vr : ur - vr, prI = sb ? ui + vi : ui - vi;
            const double piR = sb ? wr - tr : tr + wr, piI = sb ? wi - ti : ti + wi;
#pragma unroll
            for (int sz = 0; sz < 2; ++sz) {
                const int k = a.slot_k[(((size_t)gc * kMfmaCols + col) * 2 + sb) * 2 + sz];
                if (k < 0) continue;
                double *dst = a.partial + ((size_t)k * a.n_atom_blocks + blockIdx.y) * 2;
                dst[0] = sz ? prR + piI : prR - piI; // Re P z or Re P conj(z)
                dst[1] = sz ? piR - prI : prI + piR; // Im
            }
        }
    }
}

// One weight set: at most 120 registers, so that a SIMD holding three of its
// waves (360 registers) keeps room for a wave of a flush kernel that runs
// beside it on another stream.
template <bool EARLY>
__global__ __launch_bounds__(kMfmaMaxWaves * 64) __attribute__((amdgpu_num_vgpr(60)))
void rhok_couple_kernel(RhokMfmaArgs a)
{
    rhok_couple_body<EARLY>(a);
}

// One wave per k-vector: sum the partials of its slot over the atom blocks in
// a fixed order and store the result at the caller's index (a k-vector listed
// twice reads the partials stored under its first index).  NW = 1: n(k).
// NW = 3: the current vector J(k), stored as its components on the k-vector's
// basis (khat, e1, e2) at channels 3k, 3k+1, 3k+2.
template <int NW>
__global__ __launch_bounds__(256) void rhok_mfma_final_kernel(RhokMfmaArgs a)
{
    const int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= a.nk) return; // whole wave
    const size_t row = (size_t)a.k_src[k];
    double sr[NW], si[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const double *src = a.partial + (row * NW + w) * a.n_atom_blocks * 2;
        double r = 0.0, i = 0.0;
        for (int b = lane; b < a.n_atom_blocks; b += 64) {
            r += src[2 * b];
            i += src[2 * b + 1];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            r += __shfl_down(r, off, 64);
            i += __shfl_down(i, off, 64);
        }
        sr[w] = r;
        si[w] = i;
    }
    if (lane != 0) return;
    if (a.stamps) stamp_end(a.stamps, (unsigned)k);
    if constexpr (NW == 1) {
        if (a.out_double)
            static_cast<double2 *>(a.out)[k] = make_double2(sr[0], si[0]);
        else
            static_cast<float2 *>(a.out)[k] = make_float2((float)sr[0], (float)si[0]);
    } else {
        const double *bas = a.basis + (size_t)k * 9;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double r = 0.0, i = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                r += bas[3 * c + w] * sr[w];
                i += bas[3 * c + w] * si[w];
            }
            if (a.out_double)
                static_cast<double2 *>(a.out)[3 * k + c] = make_double2(r, i);
            else
                static_cast<float2 *>(a.out)[3 * k + c] = make_float2((float)r, (float)i);
        }
    }
}

} // namespace

int rhok_mfma_cols() { return kMfmaCols; }
int rhok_mfma_max_nmax() { return kMfmaCols - 1; }

// Three weight sets: packed B tiles for components up to nmax.
static int current_btiles(int nmax) { return (3 * (nmax + 1) + kMfmaCols - 1) / kMfmaCols; }

template <int TA> static size_t lds_bytes(int table_rows, int nb)
{
    return (size_t)(kRoots + ScaleSlots<3>::n) * sizeof(double2) +
           2 * ((size_t)table_rows * Tile<TA>::stride * sizeof(float2) +
                (size_t)nb * Tile<TA>::bfrags * sizeof(halfv_t));
}

// Atoms per tile for a current k-set with table_rows X and Y rows.
static int tile_atoms(int table_rows, int nb)
{
    return lds_bytes<128>(table_rows, nb) <= kLdsBytes ? 128 : 64;
}

// One weight set: the root table and two buffers of X and Y planes (table_rows
// rows of both parts) and B fragments.
static size_t couple_lds_bytes(int table_rows)
{
    return (size_t)kRoots * sizeof(double2) +
           2 * ((size_t)2 * table_rows * kPlaneStride * sizeof(float) + (size_t)kCpBfrags * sizeof(halfv_t));
}

size_t rhok_mfma_lds_bytes(int table_rows, int nw, int nmax)
{
    if (nw == 1) return couple_lds_bytes(table_rows);
    const int nb = current_btiles(nmax);
    return tile_atoms(table_rows, nb) == 128 ? lds_bytes<128>(table_rows, nb)
                                             : lds_bytes<64>(table_rows, nb);
}

static const void *current_kernel(int ta, int nb)
{
    if (ta == 128)
        return nb == 1 ? reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 128, 1>)
               : nb == 2 ? reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 128, 2>)
                         : reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 128, 3>);
    return nb == 1 ? reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 64, 1>)
           : nb == 2 ? reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 64, 2>)
                     : reinterpret_cast<const void *>(&rhok_mfma_kernel<3, 64, 3>);
}

hipError_t rhok_mfma_prepare(int table_rows, int nw, int nmax)
{
    if (table_rows > 4 * kMfmaCols - 2 || (nw != 1 && nw != 3) || nmax > kMfmaCols - 1)
        return hipErrorInvalidValue;
    const size_t lds = rhok_mfma_lds_bytes(table_rows, nw, nmax);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    if (lds <= 64 * 1024) return hipSuccess;
    if (nw == 1) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&rhok_couple_kernel<false>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&rhok_couple_kernel<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    const void *fn = current_kernel(tile_atoms(table_rows, current_btiles(nmax)), current_btiles(nmax));
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

int rhok_mfma_chunks(int n_mtiles, int nw)
{
    // M tiles per block (one weight set: couple tiles, kCpTilesPerWave per
    // contraction wave, one more wave builds Z)
    const int maxt = nw == 3 ? MfmaShape<3>::max_waves : kCpMaxCWaves * kCpTilesPerWave;
    return (n_mtiles + maxt - 1) / maxt;
}

static hipError_t launch_couples(const RhokMfmaArgs &a, hipStream_t st)
{
    const int chunks = rhok_mfma_chunks(a.n_mtiles, 1);
    const int per_chunk = (a.n_mtiles + chunks - 1) / chunks;
    int cwaves = (per_chunk + kCpTilesPerWave - 1) / kCpTilesPerWave;
    if (cwaves < kCpMinCWaves) cwaves = kCpMinCWaves;
    const size_t lds = couple_lds_bytes(a.x_rows + a.y_rows);
    if (a.early_loads)
        hipLaunchKernelGGL(rhok_couple_kernel<true>, dim3((unsigned)chunks, (unsigned)a.n_atom_blocks),
                           dim3((cwaves + 1) * 64), lds, st, a);
    else
        hipLaunchKernelGGL(rhok_couple_kernel<false>, dim3((unsigned)chunks, (unsigned)a.n_atom_blocks),
                           dim3((cwaves + 1) * 64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rhok_mfma_final_kernel<1>, dim3((unsigned)((a.nk + 3) / 4)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

template <int TA, int NB> static hipError_t launch_currents(const RhokMfmaArgs &a, hipStream_t st)
{
    // waves per block: the M tiles dealt evenly over the fewest blocks, at
    // least one thread per table task
    const int chunks = rhok_mfma_chunks(a.n_mtiles, 3);
    int waves = (a.n_mtiles + chunks - 1) / chunks;
    if (waves < TableShape<3, TA>::min_waves) waves = TableShape<3, TA>::min_waves;
    const size_t lds = lds_bytes<TA>(a.x_rows + a.y_rows, NB);
    hipLaunchKernelGGL((rhok_mfma_kernel<3, TA, NB>), dim3((unsigned)chunks, (unsigned)a.n_atom_blocks),
                       dim3(waves * 64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rhok_mfma_final_kernel<3>, dim3((unsigned)((a.nk + 3) / 4)), dim3(256), 0,
                       st, a);
    return hipGetLastError();
}

hipError_t launch_rhok_mfma(const RhokMfmaArgs &a, hipStream_t st)
{
    if (a.nmax > kMfmaCols - 1 || a.n_mtiles < 1 || a.x_rows < 1 || a.y_rows < 1 ||
        a.x_rows + a.y_rows > 4 * kMfmaCols - 2)
        return hipErrorInvalidValue;
    const int rows = a.x_rows + a.y_rows;
    if (a.nw == 1) return launch_couples(a, st);
    if (a.nw != 3) return hipErrorInvalidValue;
    const int nb = current_btiles(a.nmax);
    if (tile_atoms(rows, nb) == 128)
        return nb == 1 ? launch_currents<128, 1>(a, st)
               : nb == 2 ? launch_currents<128, 2>(a, st) : launch_currents<128, 3>(a, st);
    return nb == 1 ? launch_currents<64, 1>(a, st)
           : nb == 2 ? launch_currents<64, 2>(a, st) : launch_currents<64, 3>(a, st);
}

} // namespace corr
