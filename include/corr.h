/*
 * corr.h -- C ABI of the MI355X (gfx950) on-the-fly multiple-tau correlator.
 *
 * The library implements the per-step update of the multiple-tau correlator
 * of the DL_POLY 5 paper (Section 2.2; Appendix D, Algorithm 1), its readout
 * (Algorithm 2) and the Green-Kubo integrals for shear viscosity and thermal
 * conductivity (Section 2.3, Eqs. for viscosity and thermal conductivity),
 * for many independent channels at once on one GPU.  Channels are organised
 * in groups; every channel of a group shares the correlator parameters
 * (b blocks/levels, p points per level, averaging factor m, update interval
 * u) and the sample / accumulator precision.  A group can instead be fed
 * with atom data, in which case the library evaluates on every push, and
 * correlates, the k-space density n(k) = sum_j exp(i k.r_j) of its
 * k-vectors (Section "Currents", Eq. k-density), their longitudinal and
 * transverse currents (Eqs. long-current, trans-current), or the partial
 * momentum densities of the mass-flux correction (Section "Viscosity and
 * thermal conductivity").  A group can also correlate pairs of observables
 * (the x, y form of Algorithm 1).
 *
 * Conventions shared by every entry point:
 *  - every call returns int: CORR_OK (0) or a negative corr_status; no
 *    exception or longjmp crosses the ABI;
 *  - "device" pointers are HIP device allocations on the context's device,
 *    "host" pointers are ordinary host memory;
 *  - a context is bound to one device and one HIP stream (hipStream_t passed
 *    as void*, NULL = the null stream); all device work is issued on that
 *    stream in call order; a context is not thread-safe;
 *  - the context owns every device allocation it makes and frees it in
 *    corr_destroy;
 *  - on an error the message is available from corr_last_error(ctx) (or
 *    corr_last_error(NULL) for errors of corr_create).
 */
#ifndef CORR_H
#define CORR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct corr_ctx corr_ctx;

enum corr_status {
    CORR_OK = 0,
    CORR_E_INVALID = -1,     /* bad argument or descriptor                      */
    CORR_E_OOM = -2,         /* device allocation failed                         */
    CORR_E_DEVICE = -3,      /* a HIP call failed (message names it)             */
    CORR_E_STATE = -4,       /* call not valid in the context's current state    */
    CORR_E_UNSUPPORTED = -5  /* valid descriptor the library does not implement  */
};

/* Sample precision (complex types are interleaved re, im). */
enum corr_dtype { CORR_F32 = 1, CORR_F64 = 2, CORR_CF32 = 3, CORR_CF64 = 4 };

/* Per-lag accumulator: FP64; compensated (Kahan) FP32 value + compensation
 * planes; or plain FP32 (uncompensated, for precision comparisons only).
 * KAHAN_F32 and F32 require a single-precision sample dtype. */
enum corr_accum { CORR_ACC_F64 = 1, CORR_ACC_KAHAN_F32 = 2, CORR_ACC_F32 = 3 };

/* Where a group's samples come from on each push. */
enum corr_source {
    CORR_SRC_SAMPLES = 0, /* caller provides n_channels samples per push        */
    CORR_SRC_RHOK = 1,    /* caller provides positions; channels = k-vectors     */
    CORR_SRC_CURRENTS = 2, /* caller provides positions and velocities; three
                             channels per k-vector: the longitudinal current
                             khat . j and the transverse current on the basis
                             vectors e1, e2 (Section "Currents", Eqs.
                             long-current, trans-current): with J(k) =
                             sum_j v_j exp(i k.r_j), channel 3q = khat . J,
                             3q+1 = e1 . J, 3q+2 = e2 . J, where e1 = the
                             Cartesian axis least aligned with khat (the
                             first on ties) made orthogonal to khat and
                             normalised, e2 = khat x e1.  C_L is the
                             correlation of channel 3q, C_T the mean of
                             channels 3q+1 and 3q+2.  Components of n must
                             lie within +-15; n = 0 is rejected.  Any finite
                             velocities: each component is scaled by a
                             power of two per block of about 1000 atoms
                             before the fp16 split (see CORR_FLAG_RHOK_VALU),
                             so products keep about 22 bits relative to
                             the largest |v_alpha| of the block; J(k) must
                             stay within the float range for CF32 groups.  */
    CORR_SRC_MOMENTUM = 3 /* caller provides velocities; channels = the
                             partial momentum densities of the mass-flux
                             correction of the thermal conductivity (Section
                             "Viscosity and thermal conductivity"): channel
                             3s + alpha = (1/V) sum over the atoms i of
                             species s of m_s v_alpha(i), V = box^3, for
                             every species s.  Input (the group's real
                             dtype): velocities [3][n_atoms]; a pair group
                             appends [n_channels] x samples (e.g. the heat
                             flux component of each channel) and correlates
                             C(L) = <x(s) j(s - L)>, the densities being y.
                             The correlations are not divided by N.        */
};

/* corr_create flags. */
enum corr_flags {
    CORR_FLAG_GRAPH = 1u,     /* capture one push of all groups in a HIP graph    */
    CORR_FLAG_PER_GROUP = 2u, /* one kernel launch per group and push (the plain
                                 form) instead of one batched launch            */
    CORR_FLAG_TIMING = 4u,    /* bracket the update kernels of every push with
                                 HIP events (see corr_kernel_time)              */
    CORR_FLAG_DIRECT = 8u,    /* update every channel on every push (Algorithm 1
                                 step by step) even where the block-deferred
                                 form is available                              */
    CORR_FLAG_RHOK_VALU = 16u /* evaluate n(k) on the vector units for every
                                 k-density group; by default a group whose
                                 k-set has |n component| <= 15 is evaluated as
                                 a matrix product on the matrix cores (fp16
                                 hi/lo operand split, about 22 significant
                                 bits per product, fp32 tile sums added in
                                 fp64).  On either unit the phases are float
                                 (about 24 bits), so producer samples carry
                                 about 22-24 significant bits per atom term
                                 whatever the group dtype: a CF64 group gets
                                 the double sums of those terms, not
                                 double-precision phases                        */
};

typedef struct corr_group_desc {
    int64_t n_channels;     /* channels; CORR_SRC_RHOK: the number of k-vectors;
                               CORR_SRC_CURRENTS: 3 x the number of k-vectors;
                               CORR_SRC_MOMENTUM: 3 x n_species                */
    int32_t levels;         /* b >= 1 blocks                                       */
    int32_t points;         /* p >= 2 values per block                             */
    int32_t m;              /* averaging factor, 2 <= m < p                        */
    int32_t dtype;          /* enum corr_dtype (CORR_SRC_RHOK, CURRENTS: CF32 or
                               CF64; CORR_SRC_MOMENTUM: F32 or F64)              */
    int32_t accum;          /* enum corr_accum                                     */
    int32_t source;         /* enum corr_source                                    */
    int32_t update_every;   /* u >= 1: scales reported lag times only (Sec. 2.2)  */
    int32_t pair;           /* 0: each channel is correlated with itself; 1: each
                               channel correlates a pair of observables (x, y),
                               the x, y form of Algorithm 1 (Appendix D): both are
                               carried through the rings and the block means and
                               C(L) = <x(s) conj(y(s - L))>.  A push then brings
                               [2][n_channels] samples (all x, then all y);
                               CORR_SRC_MOMENTUM: x from the caller, y the
                               densities (see there).  CORR_SRC_SAMPLES and
                               CORR_SRC_MOMENTUM only; such groups always take
                               the per-step (direct) form                        */
    double dt;              /* simulation time step; lag time = L m^k u dt        */
    /* CORR_SRC_RHOK and CORR_SRC_CURRENTS (kvec) and CORR_SRC_MOMENTUM
       (n_atoms, box) only (ignored otherwise): */
    const int32_t *kvec;    /* host [n_k][3] integer n, k = 2 pi n / box, n_k =
                               n_channels (RHOK) or n_channels / 3 (CURRENTS);
                               copied during corr_create                          */
    int64_t n_atoms;        /* atoms per push: input float [3][n_atoms] positions,
                               CURRENTS: then [3][n_atoms] velocities;
                               MOMENTUM: [3][n_atoms] velocities (group dtype)    */
    double box;             /* cubic box edge L (also MOMENTUM: V = L^3)          */
    /* CORR_SRC_MOMENTUM only (ignored otherwise): */
    const int32_t *species; /* host [n_atoms] species of every atom, in
                               [0, n_species) (else CORR_E_INVALID); copied
                               during corr_create                                 */
    const double *masses;   /* host [n_species] mass of the atoms of each species
                               (finite; copied during corr_create)                */
    int32_t n_species;      /* 1..8; n_channels must be 3 n_species               */
    int32_t reserved;       /* 0                                                  */
} corr_group_desc;

/* Launch shape.  Channels are stored in tiles of tile_channels consecutive
 * channels (the state layout depends on it, so it is fixed at create); each
 * thread handles chans_per_thread consecutive channels of a tile; the batched
 * kernel runs grid_blocks blocks that stride over all tiles of all groups
 * (0 = one block per tile).  overlap_producers chooses which work of a push
 * is issued on a second stream (results are the same in every mode).  Zeros
 * everywhere select the library defaults (or the autotuner's cached
 * choice). */
typedef struct corr_tuning {
    int32_t tile_channels;    /* multiple of 64 * chans_per_thread, at most
                                 256 * chans_per_thread (256 threads per block) */
    int32_t chans_per_thread; /* 1, 2 or 4                                          */
    int32_t lag_chunk;        /* lags loaded per batch: 4, 8 or 16                  */
    int32_t grid_blocks;      /* 0 = one block per tile                              */
    int32_t overlap_producers; /* 0: everything on the context's stream:
                                  staging, producers, per-step updates, flush;
                                  1: producers on a forked stream, followed
                                  there by the per-step updates of every
                                  direct group when block-deferred groups are
                                  present (concurrently with their staging and
                                  flush), else by their own groups' updates
                                  (concurrently with the other updates);
                                  2: producers first, then the
                                  per-step updates on a forked stream,
                                  concurrently with the flush of the
                                  block-deferred groups                        */
    int32_t fold_block;        /* pushes per fold block T of block-deferred
                                  groups: 256 or 128; 0 = 256, or 128 when the
                                  state of 256 would not fit in the device's
                                  free memory (and the per-step form when
                                  neither fits)                                 */
    int32_t fold_threads;      /* threads per block of the scheduled fold
                                  kernel: 64, 128 or 256 (0 = 128)              */
} corr_tuning;

/*
 * Create a context for n_groups channel groups on HIP device `device`, whose
 * work is issued on `stream`.  A group is a set of correlators of one shape
 * (b blocks, p points, averaging m; section "Correlation functions at
 * runtime" and the appendix on general correlations: one correlator per
 * observable, each with its shift arrays, accumulators and correlation sums
 * per block); corr_create allocates that state for every channel, all of
 * it on the device.  Validates every descriptor (CORR_E_INVALID on
 * b < 1, p < 2, m < 2, m >= p, n_channels < 1, u < 1, an unknown dtype /
 * accumulator / source, a compensated or FP32 accumulator with a double
 * dtype, a k-density group without k-vectors, positions or a positive box),
 * allocates and zeroes all state (CORR_E_OOM on failure) and, with
 * CORR_FLAG_GRAPH, captures the push graph.  `tuning` may be NULL.
 * On success *out receives the context.
 */
int corr_create(const corr_group_desc *groups, int32_t n_groups, int32_t device, void *stream,
                uint32_t flags, const corr_tuning *tuning, corr_ctx **out);

/* Device buffer the library reads a group's samples from when corr_push is
 * given NULL for that group: the newly observed values that Algorithm 1
 * (appendix on general correlations) feeds to each correlator of the group,
 * n_channels elements of the group dtype, or for CORR_SRC_RHOK float
 * positions [3][n_atoms] (the atoms of Eq. k-density, section "Currents").
 * The library owns the buffer; *bytes receives its size.  The pointer is stable for the
 * life of the context (required by graph mode). */
int corr_input_buffer(corr_ctx *ctx, int32_t group, void **dev_ptr, size_t *bytes);

/* Replace a group's input buffer by caller-owned device memory of at least
 * the bytes corr_input_buffer reports (dev_ptr NULL restores the library's own
 * buffer).  The caller keeps it valid until it is unbound or the context is
 * destroyed.  In graph mode the push graph is captured again, so later
 * replays read the new buffer.  Synchronises the context's stream. */
int corr_bind_input(corr_ctx *ctx, int32_t group, void *dev_ptr, size_t bytes);

/*
 * One correlator update (Algorithm 1 applied with block index 1) of every
 * channel of every group.  samples: NULL (use every group's input buffer) or
 * a host array of n_groups device pointers, each NULL (use that group's input
 * buffer) or the group's samples for this step (layout as for
 * corr_input_buffer).  The pointers are only read by work issued on the
 * context's stream; they must stay valid until that work has run.  In graph
 * mode, a push whose pointers are all NULL (or equal to the input buffers)
 * replays the captured graph; any other pointer launches the same kernels
 * directly.
 */
int corr_push(corr_ctx *ctx, const void *const *samples);

/* Replay of a stored history (the paper's comparison of on-the-fly analysis
 * with replaying saved trajectories, Section "Benchmarks and Trade-offs"):
 * n_steps consecutive pushes in one call.  samples[g] is group g's device
 * history; row r (the input of push r) starts at samples[g] + r * strides[g]
 * bytes (strides NULL: rows packed, stride = the group's per-push input size,
 * see corr_input_buffer).  Equivalent to n_steps corr_push calls with those
 * pointers, in order, with the same results bit for bit.  Every group needs a
 * history (CORR_E_INVALID otherwise, or for a stride below the push size).
 * Work is issued on the context's stream; the rows must stay valid until it
 * has run.
 *  - Without CORR_FLAG_GRAPH, the block-deferred groups fold every whole
 *    block of T pushes that the history holds (after the pushes up to the
 *    next block boundary, which are single pushes) in one pass per block,
 *    reading the block's samples from the history instead of staging them
 *    (the fold's products, block means and sums are the same); the other
 *    groups are pushed row by row.
 *  - With CORR_FLAG_GRAPH, the n_steps single pushes are captured once as a
 *    graph and replayed; the few most recent (histories, strides, n_steps)
 *    keep their graphs, so repeated replays of the same buffers launch once.
 *    No timing events are recorded in these replays (the fold kernels' device
 *    stamps are kept). */
int corr_push_steps(corr_ctx *ctx, int32_t n_steps, const void *const *samples,
                    const int64_t *strides);

/* The update form of a group (chosen at corr_create): *form = 0 per-step
 * form (Algorithm 1 push by push), 1 block-deferred form, 2 block-deferred
 * one-level window, 3 per-step one-level window; *block = pushes per fold
 * block (T for form 1, 64 for form 2, else 0).  Either pointer may be NULL. */
int corr_group_form(const corr_ctx *ctx, int32_t group, int32_t *form, int32_t *block);

/* Number of pushes so far and the maximum number of readout points of a
 * group, p + (b - 1)(p - floor(p/m)) (Algorithm 2). */
int corr_query(const corr_ctx *ctx, int32_t group, int64_t *n_pushes, int32_t *n_out_max);

typedef struct corr_readout_opts {
    int64_t ch_begin, ch_end; /* channels averaged; [0, 0) = all channels          */
    double t_cut;             /* Green-Kubo cut-off time; <= 0 = last emitted lag   */
    int32_t gk_kind;          /* 0: raw integral of C; 1: shear viscosity
                                 V/(kB T) * integral (channels = the shear
                                 components); 2: thermal conductivity
                                 V/(3 kB T^2) * integral of q(t).q(0), the dot
                                 product taken as 3x the channel mean            */
    int32_t reserved;
    double volume, kB, temperature; /* used by gk_kind 1 and 2                     */
    int64_t slice_begin, slice_end; /* channels returned in c_per_channel          */
} corr_readout_opts;

/*
 * Readout (Algorithm 2) of one group, non-destructive: more pushes may
 * follow.  Synchronises the context's stream.  For every (level k, lag L)
 * with a non-zero count, in level-major lag-minor order, writes
 *   t[i]     = L m^k u dt,
 *   c[i]     = mean over the selected channels of sum/count (complex dtypes:
 *              c is [n_out][2] re, im; k-density groups are scaled by
 *              1/n_atoms, i.e. F(k,t) of Section "Currents"),
 *   count[i] = pushes that contributed, max(0, floor(S / m^k) - L),
 *   gk_running[i] = trapezoid integral of Re c from t[0] to t[i] times the
 *              gk_kind prefactor, and *gk_at_cut the same at opts->t_cut,
 * and, if c_per_channel is not NULL, the per-channel values for channels
 * [slice_begin, slice_end) as [slice][n_out] (complex: [slice][n_out][2]).
 * Output arrays are host memory of at least n_out_max entries (corr_query);
 * any of t, count, gk_running, gk_at_cut may be NULL.  opts may be NULL.
 */
int corr_finalize(corr_ctx *ctx, int32_t group, const corr_readout_opts *opts, int32_t *n_out,
                  double *t, double *c, int64_t *count, double *gk_running, double *gk_at_cut,
                  double *c_per_channel);

/*
 * corr_finalize for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight serving loops or harnesses that forbid
 * it).  Same arguments, results and errors as corr_finalize, bit for bit; it
 * allocates nothing: instead of the context's readout buffer (grown with
 * hipMalloc on demand) it uses a fixed 16 MiB device array that the library
 * holds once per GPU until the process ends.  Groups whose readout needs more
 * than that fail with CORR_E_UNSUPPORTED and a message naming the size (the
 * per-channel slice and, for direct-form groups, n_out x ceil(channels /
 * 4096) partial sums must fit; block-deferred groups are reduced in several
 * passes when their channels need more).  Every call on a GPU shares that
 * GPU's array: calls that overlap in time on one GPU (from several threads,
 * or on contexts whose streams run concurrently) race and must be serialised
 * by the caller.  Nothing in the array needs to start at zero; it keeps the
 * last call's contents.
 */
int corr_finalize_noalloc(corr_ctx *ctx, int32_t group, const corr_readout_opts *opts,
                          int32_t *n_out, double *t, double *c, int64_t *count, double *gk_running,
                          double *gk_at_cut, double *c_per_channel);

/* Wait for all work issued by the context. */
int corr_sync(corr_ctx *ctx);

/* Free every device allocation of the context (synchronises first). */
int corr_destroy(corr_ctx *ctx);

/* Message of the last failed call on ctx (NULL: of the last failed
 * corr_create on this thread).  Never NULL; owned by the library. */
const char *corr_last_error(const corr_ctx *ctx);

/* Device bytes of correlator state held by a group (ring and accumulator
 * planes, padded to whole tiles). */
int corr_state_bytes(const corr_ctx *ctx, int32_t group, int64_t *bytes);

/* With CORR_FLAG_TIMING: synchronise and return summed device times from HIP
 * events (created without a system-scope fence).  which = 0: per push, on the
 * context's stream, from before the staging / push kernel launch(es) to after
 * the flush launch(es) of that push, i.e. the correlator-update kernels of
 * the main stream (excluding a k-density branch forked with
 * overlap_producers = 1, including the per-step updates forked with
 * overlap_producers = 2, and excluding the push's end kernel); *n = timed
 * pushes.  which = 1: the fold kernel of the scheduled
 * flush of block-deferred groups only (one per push); *n = timed flushes.
 * which = 2: each k-density producer launch, on the stream it runs on (the
 * forked side stream when other groups share the context); *n = timed
 * launches.  which = 3: the scheduled fold kernels of block-deferred groups
 * timed by the kernels themselves on every push (the earliest block start to
 * the latest block end, device wall clock), so that no event sits between
 * the kernels of a push; *n = pushes with a fold launch.  which = 4: the
 * producers of a push timed the same way (first block start of the producer
 * kernel to the last end of its final reduction; several producer groups in
 * one span); *n = pushes with a producer.  In graph mode the which = 0
 * events bracket the whole graph replay and the which = 3 and 4 stamps are
 * kept; no other times are recorded.  reset != 0 clears the counters of
 * `which` after reading.  CORR_E_STATE without the flag.
 *
 * Block-deferred form: for groups of single-precision samples with p = 16 and
 * m = 2 (unless CORR_FLAG_DIRECT), a push stages the samples and flushes one
 * of 256 channel subsets: subset j adds the lag products of block q (pushes
 * 256(q-1)+1 .. 256q) level by level at push 256q + j -- the same products,
 * block means and counts as Algorithm 1, only the grouping of the
 * floating-point sums differs.  A readout first folds complete blocks a
 * subset has not folded yet (exactly what its scheduled flush would do), then
 * folds the pushes after the last block without modifying state.
 *
 * Block-deferred window: a group with one level (b = 1), p >= 512 points and
 * single-precision samples (real or complex, any accumulator; not pair
 * groups; unless CORR_FLAG_DIRECT) keeps a ring of p + 128 samples; a push
 * stages its sample and, at push 64q + j, adds the products of block q
 * (pushes 64(q-1)+1 .. 64q) to the lags of lag block j (lags j ceil(p/64)
 * .. (j+1) ceil(p/64) - 1).  A readout adds the products of the pushes each
 * lag block has not folded yet from the ring, without modifying state.
 * Other one-level groups with p >= 512 take a per-step window kernel that
 * splits the lag range over the grid. */
int corr_kernel_time(corr_ctx *ctx, int32_t which, double *ms_total, int64_t *n, int32_t reset);

/* With CORR_FLAG_TIMING: record the timing events (the three event kinds of
 * corr_kernel_time) and the device stamps (the two stamp kinds) only on pushes
 * whose index n (pushes completed before it) satisfies n % stride == 0, so
 * that the events (each one a completion signal between two kernels) and the
 * stamps (atomics of every block, reduced by the push's last kernel) slow the
 * other pushes down by nothing; the times and counts of corr_kernel_time then
 * cover those pushes only.  The stamps take the push index from the device
 * counter, so captured graphs and stored-history replays follow the stride
 * too (a block folded from a stored history is stamped when the counter at
 * its launch is a multiple of the stride).
 * stride >= 1 (default 1: every push); CORR_E_INVALID otherwise, CORR_E_STATE
 * without the flag.  Takes effect from the next push (synchronises the
 * context's stream). */
int corr_set_timing_stride(corr_ctx *ctx, int32_t stride);

/* Launch shape in use. */
int corr_get_tuning(const corr_ctx *ctx, corr_tuning *out);

/*
 * Autotuner: choose the launch shape for these groups on `device` by timing
 * trial contexts (same descriptors with at most max_trial_channels channels
 * per group, zero samples; all trial memory is freed before returning) over
 * whole flush periods for every candidate shape; then, with the fastest
 * shape, choose overlap_producers on trial contexts whose sample-fed groups
 * and producer atom counts are scaled by one factor so that the largest group
 * has at most 2^25 channels (the concurrent kernels keep their balance), and
 * return the result in *out.  The choice is cached in a text file of JSON lines (cache_path, or
 * NULL for $CORR_TUNE_CACHE, else $HOME/.cache/corr_gfx950_tune.jsonl, else
 * no cache) keyed by the device architecture, the flags and the group
 * descriptors; a cached entry is returned without timing unless force != 0.
 * corr_create with a NULL or all-zero tuning uses the cached entry for its
 * key when one exists.  Synchronises the device.
 */
int corr_autotune(const corr_group_desc *groups, int32_t n_groups, int32_t device, void *stream,
                  uint32_t flags, const char *cache_path, int64_t max_trial_channels,
                  int32_t force, corr_tuning *out);

#ifdef __cplusplus
}
#endif
#endif /* CORR_H */
