// corr_kernels.h -- host-side launchers of the correlator's HIP kernels.
#ifndef CORR_KERNELS_H
#define CORR_KERNELS_H

#include <hip/hip_runtime.h>

#include "corr_internal.h"

namespace corr {

hipError_t launch_push_batched(const PushArgs &a, int cpt, int lch, int grid, int block,
                               hipStream_t st);
hipError_t launch_push_group(const GroupArgs &g, const int64_t *step, int cpt, int lch, int block,
                             hipStream_t st);
hipError_t launch_push_window(const GroupArgs &g, const int64_t *step, int cpt, int lch,
                              int block, int lags_per_block, hipStream_t st);
hipError_t launch_push_split(const GroupArgs &g, const int64_t *step, int cpt, int lch, int block,
                             int lags_per_block, hipStream_t st);
hipError_t launch_push_end(const PushEndArgs &a, hipStream_t st); // flush records + step counter
hipError_t launch_rhok(const RhokArgs &a, hipStream_t st);
int rhok_tile_atoms(int nmax);
int rhok_block_threads(int n_seg);
hipError_t launch_rhok_mfma(const RhokMfmaArgs &a, hipStream_t st);
int rhok_mfma_cols();        // |n_z| columns of the matrix-core producer
int rhok_mfma_max_nmax();    // largest |n component| it takes
hipError_t launch_momentum(const MomentumArgs &a, hipStream_t st); // partial + final kernels
int momentum_blocks(int64_t n_atoms); // blocks of the partial kernel (size of the partial buffer)
hipError_t rhok_mfma_prepare(int table_rows, int nw, int nmax); // once per context, before the first launch
int rhok_mfma_chunks(int n_mtiles, int nw); // blocks along the M tiles (grid.x)
hipError_t launch_reduce(const ReduceArgs &a, hipStream_t st);
bool deferred_supported(int kind, int p, int m);
hipError_t launch_stage(const GroupArgs &g, const int64_t *step, hipStream_t st);
hipError_t launch_flush(const DeferredArgs &a, hipStream_t st);        // fold + commit
hipError_t launch_flush_fold(const DeferredArgs &a, hipStream_t st);   // the fold kernel
// Fold of block a.fixed_block for every tile group (a.fixed_group == -2) with
// level 0 read from the history a.hist (a.hist_stride bytes per push).
hipError_t launch_history_fold(const DeferredArgs &a, hipStream_t st);
hipError_t launch_flush_commit(const DeferredArgs &a, hipStream_t st); // flag update
int64_t deferred_readout_rows(const GroupArgs &g);
int64_t deferred_readout_groups(const GroupArgs &g);
int64_t deferred_readout_group_rows(); // chunk rows per fixed-order column group
// Readout of the chunk rows [a.row_begin, a.row_end) (whole column groups, or
// up to the last row): per-row sums into a.chunk_partial, then the column
// groups of those rows into groups[group][ne].
hipError_t launch_deferred_readout_pass(const DeferredArgs &a, double *groups, hipStream_t st);
// Sum of every column group, in order, into sums[ne].
hipError_t launch_deferred_readout_final(const DeferredArgs &a, const double *groups, double *sums,
                                         hipStream_t st);
hipError_t launch_gather(const ReduceArgs &a, hipStream_t st);
bool window_deferred_supported(int kind);
int window_lags_per_block(int p);
hipError_t launch_window_fold(const GroupArgs &g, const int64_t *step, hipStream_t st);
// Two block-deferred windows of the same kind and length in one launch (the
// second's blocks after the first's): a small window alone keeps few waves
// per SIMD.
bool window_folds_share_launch(const GroupArgs &a, const GroupArgs &b);
hipError_t launch_window_fold2(const GroupArgs &a, const GroupArgs &b, const int64_t *step, hipStream_t st);

} // namespace corr

#endif
