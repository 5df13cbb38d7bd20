// corr_internal.h -- layout and kernel-argument structures shared by the
// host runtime and the HIP kernels of the correlator library.
//
// State layout (per group, in one device allocation): channels are grouped
// in tiles of `tw` consecutive channels; tile t occupies `tile_bytes` bytes
// at state + t * tile_bytes.  Inside a tile, level 0 comes first, then
// levels 1..b-1, each laid out as
//     ring  [p][tw]          sample type S (ring slot r of every channel)
//     acc   [nl][tw]         accumulator plane(s), one row per lag
// where nl = p for level 0 and p - floor(p/m) for the coarser levels (they
// only ever accumulate lags floor(p/m)..p-1, Algorithm 1).  A compensated
// accumulator has two planes, value rows then compensation rows.  Every row
// is a multiple of 256 bytes, so wave-wide vector loads are whole cache
// lines and all planes stay aligned.
#ifndef CORR_INTERNAL_H
#define CORR_INTERNAL_H

#include <stdint.h>

namespace corr {

constexpr int kMaxGroups = 8;

// (sample dtype, accumulator) combinations; the kernels are specialised on it.
enum Kind : int32_t {
    K_F32_F64 = 0,   // float samples, double sums
    K_F32_KAHAN = 1, // float samples, compensated float sums
    K_F32_F32 = 2,   // float samples, plain float sums
    K_F64_F64 = 3,   // double samples, double sums
    K_CF32_F64 = 4,  // complex float samples, complex double sums
    K_CF32_KAHAN = 5,
    K_CF32_F32 = 6,
    K_CF64_F64 = 7,
    K_COUNT = 8
};

struct GroupArgs {
    const void *samples; // this push's samples (device), n_ch elements
    char *state;         // tile 0 of the group
    int64_t n_ch;        // channels
    int64_t n_tiles;     // tiles (ceil(n_ch / tw))
    int64_t tile_first;  // index of the group's first tile in the batched tile space
    int64_t tile_bytes;  // bytes per tile
    int64_t lvl0_bytes;  // bytes of level 0 inside a tile
    int64_t lvlk_bytes;  // bytes of each level >= 1 inside a tile
    int32_t kind;        // enum Kind
    int32_t p, m, levels;
    int32_t lag0;        // floor(p / m): first lag of levels >= 1
    int32_t tw;          // channels per tile
    int32_t s_bytes;     // bytes per sample
    int32_t a_bytes;     // bytes per accumulator plane element
    int32_t deferred;    // 1: block-deferred form (pushes only stage samples)
    int32_t p0;          // ring rows of level 0 (p; 2 T + p when block-deferred;
                         // 2 kWindowT + p for a block-deferred window)
    int32_t pair;        // 1: channels correlate (x, y): samples [2][n_ch], and each
                         // level holds the lagged y ring, then an x ring
    int32_t defer_t;     // block-deferred form: pushes per fold block T, else 0
};

// Pushes staged between two flushes of a block-deferred group: T = kDeferT by
// default, kDeferTMin when the state of the longer block would not fit.
constexpr int kDeferT = 256;
constexpr int kDeferTMin = 128;
// Pushes per block of the block-deferred one-level window (corr_window.hip).
constexpr int kWindowT = 64;
// Tile groups of a block-deferred group: T of them; tile group j folds block
// q (pushes (T (q-1), T q]) at push T q + j, so every push flushes one group;
// the level-0 ring keeps 2 T + p slots.  Arrays of tile groups hold
// kFlushGroups (the largest T) entries.
constexpr int kFlushGroups = kDeferT;
// Threads per block of the fold kernels (the scheduled flush takes 64, 128 or
// 256; a tile wider than a block is split over several blocks).
constexpr int kFoldThreadsDefault = 128;

// Device timestamps of a class of kernels of a push (timing only: record 0
// the scheduled folds, record 1 the producers): the earliest block start and
// the latest block end of this push's kernels of that class, in wall-clock
// ticks, and their running sum over pushes (the push's end kernel reduces the
// slots, adds the span and resets them).  Only the pushes whose index n
// (pushes completed before them: the device counter `step`) satisfies
// n % stride == 0 are stamped, so that one push in `stride` carries the cost
// of the stamps.  Blocks record into one of
// kStampSlots slots, each on its own 128-byte line, so that the stamps of a
// few thousand blocks do not queue on one address (on one line they delayed
// the end of the fold kernel by about 15 us, on 64 lines still by 4 us).
constexpr int kStampSlots = 256;
struct StampSlot {
    unsigned long long start, end;
    unsigned long long pad_[14];
};
struct FoldStamps {
    StampSlot slot[kStampSlots];
    unsigned long long total, count;
    const int64_t *step; // the context's device push counter
    long long stride;    // stamp the pushes with *step % stride == 0
    unsigned long long pad_[12];
};

// Record a block's start (or end) in its slot.
#if defined(__HIPCC__)
} // namespace corr
#include <hip/hip_runtime.h>
namespace corr {
__device__ __forceinline__ bool stamp_sampled(const FoldStamps *st)
{
    return *st->step % st->stride == 0;
}
// The stamps themselves, for a caller that has checked stamp_sampled.
__device__ __forceinline__ void stamp_start_now(FoldStamps *st, unsigned block)
{
    atomicMin(&st->slot[block % kStampSlots].start, (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void stamp_end_now(FoldStamps *st, unsigned block)
{
    atomicMax(&st->slot[block % kStampSlots].end, (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void stamp_start(FoldStamps *st, unsigned block)
{
    if (stamp_sampled(st)) stamp_start_now(st, block);
}
__device__ __forceinline__ void stamp_end(FoldStamps *st, unsigned block)
{
    if (stamp_sampled(st)) stamp_end_now(st, block);
}
#endif

// Flush / readout of a block-deferred group.
struct DeferredArgs {
    GroupArgs g;
    const int64_t *step;    // device push counter (a scheduled flush runs before
                            // the increment of its push, a readout after it)
    int64_t *flushed;       // [kFlushGroups] last block folded per tile group
    int64_t tiles_per_group;
    int32_t fixed_group;    // >= 0: fold block fixed_block of this tile group; -2: of
                            // every tile group that has not folded it; -1: the
                            // flush scheduled for the push being issued
    int32_t ne;             // readout: number of (level, lag) entries
    int64_t fixed_block;
    int64_t ch_begin, ch_end;       // readout: channels reduced
    int64_t slice_begin, slice_end; // readout: channels written to slice_out
    int64_t row_begin, row_end;     // readout: the 64-channel chunk rows of this pass
    double *chunk_partial;  // readout: [row_end - row_begin][ne] sums over 64-channel chunks
                            // (row r at r - row_begin)
    double *slice_out;      // readout: [(c - slice_begin) * ne + e]
    FoldStamps *stamps;     // scheduled flush with timing: block start / end stamps, else null
    // Fold straight from a stored history (fixed_group -2): row i (push
    // T (fixed_block - 1) + 1 + i) of the block holds the n_ch samples at
    // hist + i hist_stride bytes; null: the level-0 ring
    const char *hist;
    int64_t hist_stride;
    int32_t threads;        // threads per block of the fold kernel (64, 128 or 256)
    int32_t pad_;
};

struct PushArgs {
    GroupArgs g[kMaxGroups];
    int32_t n_groups;
    int32_t pad_;
    int64_t total_tiles;
    const int64_t *step; // device: pushes completed before this one
};

// Number of accumulator planes of a kind (2 for compensated sums).
inline int acc_planes(int kind) { return (kind == K_F32_KAHAN || kind == K_CF32_KAHAN) ? 2 : 1; }
inline bool kind_complex(int kind) { return kind >= K_CF32_F64; }
inline int kind_sample_bytes(int kind)
{
    switch (kind) {
    case K_F32_F64: case K_F32_KAHAN: case K_F32_F32: return 4;
    case K_F64_F64: case K_CF32_F64: case K_CF32_KAHAN: case K_CF32_F32: return 8;
    default: return 16;
    }
}
inline int kind_acc_bytes(int kind)
{
    switch (kind) {
    case K_F32_F64: case K_F64_F64: return 8;
    case K_F32_KAHAN: case K_F32_F32: return 4;
    case K_CF32_F64: case K_CF64_F64: return 16;
    default: return 8; // complex float planes
    }
}

// k-density producer: k-vectors are grouped in segments of up to kSegWidth
// vectors sharing (n_y, n_z) with n_x in [nx0, nx0 + kSegWidth).
constexpr int kSegWidth = 4;

struct RhokArgs {
    const float *pos;        // [3][n_atoms]
    int64_t n_atoms;
    const int32_t *seg_nx0;  // [n_seg]
    const int32_t *seg_ny;   // [n_seg]
    const int32_t *seg_nz;   // [n_seg]
    const int32_t *slot_out; // [n_seg * kSegWidth]: output k index of slot, or -1
    int32_t n_seg;
    int32_t nmax;            // max |n component|
    double inv_box;          // 1 / L
    double *partial;         // [n_atom_blocks][n_seg * kSegWidth][2] FP64 partial sums
    int32_t n_atom_blocks;
    int32_t atoms_per_block;
    void *out;               // [nk] complex samples (float2 or double2)
    int32_t out_double;      // 1: double2 output
    int32_t pad_;
    FoldStamps *stamps;      // timing: the push's producer stamps, else null
};

// k-density producer on the matrix cores: n(k) from real products over the
// atoms of P(n_x, n_y) = X^{n_x} Y^{n_y} (rows: the distinct (n_x, n_y) pairs
// of the k-set, padded to whole 16-row tiles) and Z^{|n_z|} (16 columns,
// |n_z| = 0 .. 15); the sign of n_z selects how the sums combine.
// Partial momentum densities of the mass-flux correction: channel 3s + a =
// scale[s] * sum over the atoms of species s of v_a (scale = m_s / V).
constexpr int kMomMaxSpecies = 8;
struct MomentumArgs {
    const void *vel;         // [3][n_atoms] velocities (float or double); pair: then
                             // [n_ch] x samples of the same type
    const uint8_t *species;  // [n_atoms] species ids in [0, n_species)
    int64_t n_atoms;
    int32_t n_species;       // 1 .. kMomMaxSpecies
    int32_t dbl;             // 1: double velocities and output
    double scale[kMomMaxSpecies];
    double *partial;         // [n_blocks][3 kMomMaxSpecies] block sums
    int32_t n_blocks;
    int32_t pair;            // 1: output [2][n_ch], x copied from the input
    int32_t vec4;            // 1: n_atoms % 4 == 0 and vel 16-byte aligned (4 atoms per load)
    int32_t pad_;
    void *out;               // [n_ch] densities, or [2][n_ch] (x, then densities)
    FoldStamps *stamps;      // timing: the push's producer stamps, else null
};

struct RhokMfmaArgs {
    const float *pos;        // [3][n_atoms] positions; currents: then [3][n_atoms] velocities
    int64_t n_atoms;
    // Rows.  nw == 3: the (n_x, n_y) pairs, 16 per M tile; nw == 1: the
    // couples (n_x, |n_y|), 4 per M tile.  Padding rows (x_lo, y_lo).
    const int32_t *pair_nx;  // [n_mtiles * 16 | 4]
    const int32_t *pair_ny;  // [n_mtiles * 16 | 4]
    const int32_t *slot_k;   // nw == 3: [pair][16 |n_z|][n_z < 0]; nw == 1:
                             // [couple][16 |n_z|][n_y < 0][n_z < 0]: k index
                             // stored for the slot, or -1
    const int32_t *k_src;    // [nk]: partial row that holds k's sum
    int32_t n_mtiles;
    int32_t nmax;            // max |n component|, at most 15
    int32_t x_lo, x_rows;    // table rows: n_x in [x_lo, x_lo + x_rows) over the rows
    int32_t y_lo, y_rows;    // n_y likewise (nw == 1: |n_y|, y_lo = 0)
    double inv_box;          // 1 / L
    double *partial;         // [nk][nw][n_atom_blocks][2] FP64 partial sums
    int32_t n_atom_blocks;
    int32_t atoms_per_block;
    void *out;               // [nk * nw] complex samples (float2 or double2)
    int32_t out_double;      // 1: double2 output
    int32_t nk;              // k-vectors
    int32_t nw;              // weight sets: 1 = n(k), 3 = current components
    int32_t early_loads;     // n(k): 1 when forked beside the flush with a join on every
                             // push (the table builders then load the next inputs
                             // before their build), else 0 (after it)
    const double *basis;     // nw == 3: [nk][3][3] rows khat, e1, e2
    FoldStamps *stamps;      // timing: the push's producer stamps, else null
};

// End of a push: record the scheduled flush of each block-deferred group,
// then advance the device push counter by `advance` (1 for a push).  With
// commit_block >= 1 the record is instead that every tile group of those
// groups has folded block commit_block (after folds of all tile groups).
struct PushEndArgs {
    int64_t *step;
    int64_t *step2;                    // a second counter advanced with step (the
                                       // producer chain's), or null
    int32_t n_flushed;                 // block-deferred groups
    int32_t advance;                   // pushes counted
    int64_t *flushed[kMaxGroups];      // their [kFlushGroups] last-folded arrays
    int32_t defer_t[kMaxGroups];       // their blocks T
    int64_t commit_block;
    FoldStamps *stamps;                // timing: the push's stamp records (folds, then
                                       // producers), else null
    int32_t n_stamps;                  // records reduced from stamps (1 or 2)
};

// Readout reduction arguments.
struct ReduceArgs {
    const char *state;
    int64_t tile_bytes;
    int32_t tw;
    int32_t kind;
    const int64_t *hi_off;  // [n_entries] byte offset inside a tile of the entry's row
    const int64_t *lo_off;  // [n_entries] compensation row offset (compensated kinds)
    int32_t n_entries;
    int32_t blocks_per_entry;
    int64_t ch_begin, ch_end;
    double *partial;        // [n_entries][blocks_per_entry][2]
    double *out;            // [n_entries][2]
    // One-level window in the block-deferred form (wlpb > 0): entry e is lag
    // e, lag block e / wlpb; the pushes it has not folded are added from the
    // level-0 ring of p0 rows.
    int32_t wlpb;
    int32_t p0;
    int64_t n_push;         // pushes completed
};

} // namespace corr

#endif
