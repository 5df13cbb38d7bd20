// corr_runtime.cpp -- host side of the correlator library: the C ABI of
// include/corr.h, the state layout planner, push orchestration (batched or
// per-group launches, optional HIP graph), and the readout (Algorithm 2 of
// the paper's Appendix D) with the trapezoid Green-Kubo integrals (Section
// 2.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/corr.h"
#include "corr_kernels.h"
#include "corr_tune.h"

using namespace corr;

namespace {

thread_local std::string g_create_error;

// Readout scratch of corr_finalize_noalloc: a fixed device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: the device address of each GPU's copy is looked up once (in
// corr_create, with that device current) and kept in g_noalloc_ptr.
constexpr size_t kNoAllocBytes = (size_t)16 << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocDevices] = {};

// Device address of the current device's scratch array (looked up on first use).
hipError_t noalloc_scratch(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    *out = nullptr;
    if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
    if (!g_noalloc_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = ptr;
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}

// One-level groups with at least this many points take a window form: the
// block-deferred window (corr_window.hip) where the kind allows, else the
// per-step window kernel, which splits the lag range over the grid
// (kWindowLags lags per block).
constexpr int kWindowMinP = 512;
constexpr int kWindowLags = 256;

struct Group {
    corr_group_desc d{};
    int kind = 0;
    int p = 0, m = 0, b = 0, lag0 = 0, nlk = 0;
    int s_bytes = 0, a_bytes = 0, np = 1;
    bool deferred = false; // block-deferred form (stage per push, staggered flushes)
    int T = 0;             // block-deferred form: pushes per fold block
    bool wdef = false;     // one-level window in the block-deferred form (staged per
                           // push, one lag block folded per push)
    int p0 = 0;            // ring rows of level 0
    bool pair = false;     // channels correlate (x, y) pairs
    int64_t *d_flushed = nullptr;                // [kFlushGroups] blocks folded per tile group (T used)
    std::vector<int64_t> flushed;                // host mirror of d_flushed
    int64_t tiles_per_group = 0;
    int64_t n_ch = 0, n_tiles = 0, tile_bytes = 0, lvl0_bytes = 0, lvlk_bytes = 0;
    char *state = nullptr;
    void *input = nullptr;     // buffer read when a push passes NULL (own or bound)
    void *own_input = nullptr; // the library's own input allocation
    size_t input_bytes = 0;
    // k-density producer
    bool rhok = false;
    void *rhok_out = nullptr;
    int32_t *d_seg = nullptr; // seg_nx0 | seg_ny | seg_nz | slot_out
    double *d_partial = nullptr;
    RhokArgs rargs{};
    bool rhok_mfma = false;       // matrix-core producer (else rargs, vector units)
    int nw = 1;                   // producer weight sets: 1 n(k), 3 currents
    int32_t *d_mtab = nullptr;    // pair_nx | pair_ny | slot_k | k_src
    double *d_basis = nullptr;    // currents: [nk][3][3] khat, e1, e2
    RhokMfmaArgs margs{};
    // partial momentum density producer (output in rhok_out, block sums in
    // d_partial)
    bool mom = false;
    uint8_t *d_species = nullptr; // [n_atoms] (ids < 8 fit a byte)
    MomentumArgs mom_args{};
    bool produced() const { return rhok || mom; } // samples come from a producer
};

} // namespace

struct corr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    corr_tuning tuning{};
    std::vector<Group> groups;
    // push counters: d_step[0] for the main stream's kernels, d_step[1]
    // (d_step_side) for the kernels that run on the side stream when the
    // producers are forked (their per-step pushes); equal after every push,
    // except inside a captured run of pushes whose two chains are joined only
    // at its end
    int64_t *d_step = nullptr;
    int64_t *d_step_side = nullptr;
    int64_t n_push = 0;
    int32_t defer_t = 0;       // pushes per fold block of the block-deferred groups
    int32_t fold_threads = kFoldThreadsDefault;
    int32_t timing_stride = 1; // CORR_FLAG_TIMING: events on pushes with n_push % stride == 0
    FoldStamps *d_stamps = nullptr; // CORR_FLAG_TIMING: device stamps of the scheduled folds
    double stamp_khz = 0.0;         // wall-clock rate of the stamps
    PushArgs pargs{};
    int64_t total_tiles = 0;
    hipStream_t cap_stream = nullptr;
    // k-density groups run on a side stream (producer, then their own push
    // launch) forked from and joined to the main stream on every push (in a
    // captured corr_push_steps beside block-deferred groups: every
    // kChainSync pushes), so the ALU-bound producer overlaps the HBM-bound
    // push of the other groups.
    // main_set: per-step (direct) groups fed with samples; side_set: k-density
    // groups; deferred_set (below): block-deferred groups (staged per push).
    std::vector<int> main_set, side_set; // context group indices
    PushArgs pa_main{}, pa_side{}, pa_direct{}; // pa_direct: main_set + side_set
    hipStream_t side_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // graph mode: captured replays of corr_push_steps (n pushes from given
    // histories), most recent last
    struct StepsGraph {
        int32_t n = 0;
        std::vector<const void *> src;
        std::vector<int64_t> stride;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<StepsGraph> steps_graphs;
    std::vector<int> deferred_set; // context group indices in the block-deferred form
    // kernel timing (CORR_FLAG_TIMING): pool 0 per push, pool 1 per flush
    // fold, pool 2 per k-density producer launch
    struct EventPool {
        std::vector<hipEvent_t> start, end;
        size_t used = 0;
        double ms = 0.0;
        int64_t n = 0;
    } pools[3];
    // readout scratch (corr_finalize; grown on demand)
    void *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    // this device's fixed readout scratch (corr_finalize_noalloc)
    void *noalloc = nullptr;
    std::string err;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int set_err(corr_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_create_error = buf;
    return code;
}

int hip_err(corr_ctx *c, hipError_t e, const char *what)
{
    return set_err(c, e == hipErrorOutOfMemory ? CORR_E_OOM : CORR_E_DEVICE, "%s: %s (%d)", what,
                   hipGetErrorString(e), (int)e);
}

#define HIP_TRY(ctx, expr)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return hip_err((ctx), e_, #expr);                                  \
    } while (0)

int kind_of(int dtype, int accum)
{
    switch (dtype) {
    case CORR_F32:
        return accum == CORR_ACC_F64 ? K_F32_F64 : accum == CORR_ACC_KAHAN_F32 ? K_F32_KAHAN
                                                                                : K_F32_F32;
    case CORR_F64: return K_F64_F64;
    case CORR_CF32:
        return accum == CORR_ACC_F64 ? K_CF32_F64 : accum == CORR_ACC_KAHAN_F32 ? K_CF32_KAHAN
                                                                                 : K_CF32_F32;
    default: return K_CF64_F64;
    }
}

int validate(const corr_group_desc &g, int idx)
{
    auto bad = [&](const char *why) {
        return set_err(nullptr, CORR_E_INVALID, "group %d: %s", idx, why);
    };
    if (g.n_channels < 1) return bad("n_channels must be >= 1");
    if (g.levels < 1) return bad("levels (b) must be >= 1");
    if (g.points < 2) return bad("points (p) must be >= 2");
    if (g.m < 2) return bad("m must be >= 2");
    if (g.m >= g.points) return bad("m must be < p");
    if (g.update_every < 1) return bad("update_every must be >= 1");
    if (g.dtype < CORR_F32 || g.dtype > CORR_CF64) return bad("unknown dtype");
    if (g.accum < CORR_ACC_F64 || g.accum > CORR_ACC_F32) return bad("unknown accumulator");
    if (g.source != CORR_SRC_SAMPLES && g.source != CORR_SRC_RHOK &&
        g.source != CORR_SRC_CURRENTS && g.source != CORR_SRC_MOMENTUM)
        return bad("unknown source");
    if ((g.dtype == CORR_F64 || g.dtype == CORR_CF64) && g.accum != CORR_ACC_F64)
        return bad("double samples need double accumulators");
    if (g.pair != 0 && g.pair != 1) return bad("pair must be 0 or 1");
    if (g.pair && g.source != CORR_SRC_SAMPLES && g.source != CORR_SRC_MOMENTUM)
        return bad("pair groups take samples or momentum densities");
    if (g.source == CORR_SRC_MOMENTUM) {
        if (g.dtype != CORR_F32 && g.dtype != CORR_F64) return bad("momentum needs a real dtype");
        if (g.n_species < 1 || g.n_species > kMomMaxSpecies)
            return bad("momentum: n_species must be 1..8");
        if (g.n_channels != 3 * (int64_t)g.n_species)
            return bad("momentum: n_channels must be 3 x n_species");
        if (!g.species || !g.masses) return bad("momentum group without species or masses");
        if (g.n_atoms < 1) return bad("momentum group needs n_atoms >= 1");
        if (!(g.box > 0.0)) return bad("momentum group needs box > 0");
        for (int s = 0; s < g.n_species; ++s)
            if (!std::isfinite(g.masses[s])) return bad("momentum: masses must be finite");
        for (int64_t i = 0; i < g.n_atoms; ++i)
            if (g.species[i] < 0 || g.species[i] >= g.n_species)
                return bad("momentum: species id out of range");
    }
    if (g.source == CORR_SRC_RHOK) {
        if (g.dtype != CORR_CF32 && g.dtype != CORR_CF64) return bad("k-density needs a complex dtype");
        if (!g.kvec) return bad("k-density group without k-vectors");
        if (g.n_atoms < 1) return bad("k-density group needs n_atoms >= 1");
        if (!(g.box > 0.0)) return bad("k-density group needs box > 0");
        for (int64_t q = 0; q < g.n_channels; ++q)
            for (int d = 0; d < 3; ++d)
                if (g.kvec[3 * q + d] > 64 || g.kvec[3 * q + d] < -64)
                    return set_err(nullptr, CORR_E_UNSUPPORTED,
                                   "group %d: k-vector components beyond +-64", idx);
    }
    if (g.source == CORR_SRC_CURRENTS) {
        if (g.dtype != CORR_CF32 && g.dtype != CORR_CF64) return bad("currents need a complex dtype");
        if (g.n_channels % 3 != 0) return bad("currents: n_channels must be 3 x k-vectors");
        if (!g.kvec) return bad("currents group without k-vectors");
        if (g.n_atoms < 1) return bad("currents group needs n_atoms >= 1");
        if (!(g.box > 0.0)) return bad("currents group needs box > 0");
        for (int64_t q = 0; q < g.n_channels / 3; ++q) {
            const int32_t *n = g.kvec + 3 * q;
            if (n[0] == 0 && n[1] == 0 && n[2] == 0) return bad("currents: zero k-vector");
            for (int d = 0; d < 3; ++d)
                if (n[d] > 15 || n[d] < -15)
                    return set_err(nullptr, CORR_E_UNSUPPORTED,
                                   "group %d: currents need k-vector components within +-15", idx);
        }
    }
    if (g.points > 16384) return set_err(nullptr, CORR_E_UNSUPPORTED, "group %d: p > 16384", idx);
    if (g.levels > 40) return set_err(nullptr, CORR_E_UNSUPPORTED, "group %d: b > 40", idx);
    return CORR_OK;
}

// Push kernels are compiled for at most this many threads per block.
constexpr int kMaxBlock = 256;

int validate_tuning(const corr_tuning &t)
{
    const int cpt = t.chans_per_thread, lch = t.lag_chunk;
    const bool pair_ok = (cpt == 1 && (lch == 16 || lch == 8)) || (cpt == 2 && (lch == 8 || lch == 4)) ||
                         (cpt == 4 && (lch == 4 || lch == 8));
    if (!pair_ok)
        return set_err(nullptr, CORR_E_INVALID, "tuning: unsupported (chans_per_thread, lag_chunk) = (%d, %d)",
                       cpt, lch);
    if (t.tile_channels < 64 || t.tile_channels > 4096 || t.tile_channels % (64 * cpt) != 0 ||
        t.tile_channels / cpt > kMaxBlock)
        return set_err(nullptr, CORR_E_INVALID, "tuning: tile_channels %d invalid for %d channels/thread",
                       t.tile_channels, cpt);
    if (t.grid_blocks < 0) return set_err(nullptr, CORR_E_INVALID, "tuning: grid_blocks < 0");
    if (t.overlap_producers < 0 || t.overlap_producers > 2)
        return set_err(nullptr, CORR_E_INVALID, "tuning: overlap_producers must be 0, 1 or 2");
    if (t.fold_block != 0 && t.fold_block != kDeferT && t.fold_block != kDeferTMin)
        return set_err(nullptr, CORR_E_INVALID, "tuning: fold_block must be 0, %d or %d", kDeferTMin,
                       kDeferT);
    if (t.fold_threads != 0 && t.fold_threads != 64 && t.fold_threads != 128 && t.fold_threads != 256)
        return set_err(nullptr, CORR_E_INVALID, "tuning: fold_threads must be 0, 64, 128 or 256");
    return CORR_OK;
}

void free_group(Group &g)
{
    if (g.state) (void)hipFree(g.state);
    if (g.own_input) (void)hipFree(g.own_input);
    if (g.rhok_out) (void)hipFree(g.rhok_out);
    if (g.d_seg) (void)hipFree(g.d_seg);
    if (g.d_partial) (void)hipFree(g.d_partial);
    if (g.d_mtab) (void)hipFree(g.d_mtab);
    if (g.d_basis) (void)hipFree(g.d_basis);
    if (g.d_species) (void)hipFree(g.d_species);
    if (g.d_flushed) (void)hipFree(g.d_flushed);
    g = Group{};
}

void free_ctx(corr_ctx *c)
{
    if (!c) return;
    DeviceGuard dg(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    for (auto &sg : c->steps_graphs) {
        if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
        if (sg.graph) (void)hipGraphDestroy(sg.graph);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (auto &g : c->groups) free_group(g);
    if (c->d_step) (void)hipFree(c->d_step);
    if (c->d_stamps) (void)hipFree(c->d_stamps);
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    for (auto &pl : c->pools) {
        for (auto e : pl.start) (void)hipEventDestroy(e);
        for (auto e : pl.end) (void)hipEventDestroy(e);
    }
    delete c;
}

constexpr size_t kEventPool = 1024;

// Fold the elapsed times of all recorded event pairs of a pool into its total.
int fold_events(corr_ctx *c, int which)
{
    auto &pl = c->pools[which];
    if (pl.used == 0) return CORR_OK;
    HIP_TRY(c, hipEventSynchronize(pl.end[pl.used - 1]));
    for (size_t i = 0; i < pl.used; ++i) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, pl.start[i], pl.end[i]));
        pl.ms += (double)ms;
    }
    pl.n += (int64_t)pl.used;
    pl.used = 0;
    return CORR_OK;
}

// Next free event pair of a pool (folds the pool when it is full).
int next_events(corr_ctx *c, int which, hipEvent_t *a, hipEvent_t *b)
{
    auto &pl = c->pools[which];
    if (pl.used == kEventPool) {
        int rc = fold_events(c, which);
        if (rc != CORR_OK) return rc;
    }
    if (pl.used == pl.start.size()) {
        // timing only: no system-scope fence on record (no cache writeback
        // between the bracketed kernels and their neighbours)
        hipEvent_t e0, e1;
        HIP_TRY(c, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
        HIP_TRY(c, hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
        pl.start.push_back(e0);
        pl.end.push_back(e1);
    }
    *a = pl.start[pl.used];
    *b = pl.end[pl.used];
    pl.used += 1;
    return CORR_OK;
}

DeferredArgs deferred_args(const corr_ctx *c, int i)
{
    const Group &g = c->groups[(size_t)i];
    DeferredArgs da{};
    da.g = c->pargs.g[(size_t)i];
    da.step = c->d_step;
    da.flushed = g.d_flushed;
    da.tiles_per_group = g.tiles_per_group;
    da.fixed_group = -1;
    da.threads = c->fold_threads;
    return da;
}

// Scheduled flush of every block-deferred group for the push being issued
// (tile group S mod kDeferT folds block S / kDeferT if not done yet); with
// events, f0/f1 bracket the fold kernels.  The flush is recorded as done by
// the push's last kernel (push_end).
int launch_flushes(corr_ctx *c, hipStream_t st, hipEvent_t f0, hipEvent_t f1)
{
    if (f0) HIP_TRY(c, hipEventRecord(f0, st));
    for (int i : c->deferred_set) {
        DeferredArgs da = deferred_args(c, i);
        da.stamps = c->d_stamps; // the catch-up flushes of a readout carry none
        HIP_TRY(c, launch_flush_fold(da, st));
    }
    if (f1) HIP_TRY(c, hipEventRecord(f1, st));
    return CORR_OK;
}

// Host mirror of the scheduled flush of push S (after it was issued).
void mirror_flushes(corr_ctx *c, int64_t S)
{
    for (int i : c->deferred_set) {
        Group &g = c->groups[(size_t)i];
        const int j = (int)(S % g.T);
        const int64_t q = S / g.T;
        if (q >= 1 && g.flushed[(size_t)j] < q) g.flushed[(size_t)j] = q;
    }
}

// Before a readout: fold every complete block a tile group has not folded yet
// (at most one per group: a block is scheduled within T - 1 pushes).
int catch_up_flushes(corr_ctx *c, int gi)
{
    Group &g = c->groups[(size_t)gi];
    const int64_t qn = c->n_push / g.T;
    for (int j = 0; j < g.T; ++j) {
        while (g.flushed[(size_t)j] < qn) {
            DeferredArgs da = deferred_args(c, gi);
            da.fixed_group = j;
            da.fixed_block = g.flushed[(size_t)j] + 1;
            HIP_TRY(c, launch_flush(da, c->stream));
            g.flushed[(size_t)j] += 1;
        }
    }
    return CORR_OK;
}

bool is_window(const GroupArgs &g) { return g.levels == 1 && g.p >= kWindowMinP && !g.deferred; }

// One-level window in the block-deferred form: the push kernels stage the
// sample (their deferred branch), then one lag block is folded.
bool is_window_deferred(const GroupArgs &g) { return g.levels == 1 && g.deferred && g.p >= kWindowMinP; }

// Per-step groups of fewer than kSplitMaxTiles tiles (a few thousand
// channels: the k-space groups) would keep only a few CUs busy in the batched
// kernel; their level-0 lags are split over kSplitLags-lag blocks instead
// (in every issue order: with the producers forked at the start of the push
// the batched workload's step goes from 0.2125 to 0.208 ms).
constexpr int64_t kSplitMaxTiles = 64;
constexpr int kSplitLags = 8;

bool is_split(const GroupArgs &g)
{
    return !g.pair && !g.deferred && g.n_tiles < kSplitMaxTiles && g.p >= 2 * kSplitLags &&
           !is_window(g);
}

// Push kernel launch(es) for the groups of one set (batched: one launch;
// per-group form: one launch per group; long one-level windows: one window
// launch each), all reading the push counter of the set's arguments.
int launch_set(corr_ctx *c, const PushArgs &base, const std::vector<int> &idx,
               const std::vector<const void *> &resolved, hipStream_t st)
{
    PushArgs a = base;
    for (size_t j = 0; j < idx.size(); ++j) a.g[j].samples = resolved[(size_t)idx[j]];
    const int cpt = c->tuning.chans_per_thread, lch = c->tuning.lag_chunk;
    const int block = c->tuning.tile_channels / cpt;
    {
        // take the window and pair groups out of the batched / per-group launch
        PushArgs rest = a;
        int n = 0;
        int64_t tf = 0;
        // block-deferred windows: the fold kernel also stages the push's
        // sample; two windows of one kind and length share a launch (not in
        // the per-group form)
        int pending = -1;
        for (int i = 0; i < a.n_groups; ++i) {
            if (!is_window_deferred(a.g[i])) continue;
            if (pending >= 0 && !(c->flags & CORR_FLAG_PER_GROUP) &&
                window_folds_share_launch(a.g[pending], a.g[i])) {
                HIP_TRY(c, launch_window_fold2(a.g[pending], a.g[i], base.step, st));
                pending = -1;
                continue;
            }
            if (pending >= 0) HIP_TRY(c, launch_window_fold(a.g[pending], base.step, st));
            pending = i;
        }
        if (pending >= 0) HIP_TRY(c, launch_window_fold(a.g[pending], base.step, st));
        for (int i = 0; i < a.n_groups; ++i) {
            if (is_window_deferred(a.g[i])) continue;
            if (is_window(a.g[i])) {
                HIP_TRY(c, launch_push_window(a.g[i], base.step, cpt, lch, block, kWindowLags, st));
                continue;
            }
            if (a.g[i].pair) { // pair groups have their own kernels
                HIP_TRY(c, launch_push_group(a.g[i], base.step, cpt, lch, block, st));
                continue;
            }
            if (!(c->flags & CORR_FLAG_PER_GROUP) && is_split(a.g[i])) {
                HIP_TRY(c, launch_push_split(a.g[i], base.step, cpt, lch, block, kSplitLags, st));
                continue;
            }
            rest.g[n] = a.g[i];
            rest.g[n].tile_first = tf;
            tf += a.g[i].n_tiles;
            ++n;
        }
        if (n == 0) return CORR_OK;
        rest.n_groups = n;
        rest.total_tiles = tf;
        a = rest;
    }
    if (c->flags & CORR_FLAG_PER_GROUP) {
        for (int i = 0; i < a.n_groups; ++i)
            HIP_TRY(c, launch_push_group(a.g[i], base.step, cpt, lch, block, st));
    } else {
        int64_t grid = c->tuning.grid_blocks > 0 ? c->tuning.grid_blocks : a.total_tiles;
        grid = std::min<int64_t>(grid, a.total_tiles);
        grid = std::min<int64_t>(grid, 0x7fffffff);
        HIP_TRY(c, launch_push_batched(a, cpt, lch, (int)grid, block, st));
    }
    return CORR_OK;
}

// Issue one push of every group on stream `st` with the given per-group
// sample pointers (already resolved, never NULL).  Order on the main stream:
// staging of block-deferred groups, the producers, the per-step push of the
// other groups, the flush of the block-deferred groups, the push end (flush
// records and step counter).  overlap_producers = 1 forks the producers onto
// the side stream at the start of the push (before the staging), followed
// there by the per-step push of every direct group
// when block-deferred groups keep the main stream busy with their flush, else
// by the push of the producers' groups only (the sample-fed groups then run on
// the main stream beside them); 2 keeps the producers on the main stream and
// forks the per-step pushes, which then run beside the flush.
//
// chained: a push inside a captured run whose two chains are forked and
// joined around a few pushes at a time (the caller does both; it requires the
// producers forked beside block-deferred groups).  Each chain then ends the
// push with its own end kernel and counter: the main stream staging, flush and
// end (d_step, flush records, fold stamps), the side stream the producers,
// the per-step pushes and an end (d_step_side, producer stamps).  No push
// waits for the other stream's work of the push before (the per-push fork
// and join each left the chip idle for a few microseconds).
int issue_push(corr_ctx *c, const void *const *src, hipStream_t st, bool with_flush,
               bool skip_deferred = false, bool chained = false)
{
    // skip_deferred: the block-deferred groups take no part in this push (a
    // replay folds their block straight from the history instead)
    static const std::vector<int> none;
    const std::vector<int> &dset = skip_deferred ? none : c->deferred_set;
    if (skip_deferred) with_flush = false;
    const size_t ng = c->groups.size();
    std::vector<const void *> resolved(ng);
    for (size_t i = 0; i < ng; ++i)
        resolved[i] = c->groups[i].produced() ? c->groups[i].rhok_out : src[i];
    // Events are only recorded on direct launches, never while capturing, on
    // one push in timing_stride.
    const bool timed = (c->flags & CORR_FLAG_TIMING) && st == c->stream &&
                       c->n_push % c->timing_stride == 0;
    const bool fork = c->tuning.overlap_producers == 1 && !c->side_set.empty() &&
                      (!c->main_set.empty() || !dset.empty());
    const bool fork_updates = c->tuning.overlap_producers == 2 && with_flush && !dset.empty() &&
                              (!c->main_set.empty() || !c->side_set.empty());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        int rc = next_events(c, 0, &e0, &e1);
        if (rc != CORR_OK) return rc;
        HIP_TRY(c, hipEventRecord(e0, st));
    }
    if (chained && !(fork && with_flush && !dset.empty() && !timed))
        return set_err(c, CORR_E_STATE, "chained push without forked producers beside a flush");
    if (fork && !chained) {
        // forked before the staging: the producers start at once and hold
        // their CUs before the staging and the flush fill the rest (forked
        // after the staging, the flush's small blocks took the chip first and
        // the producer branch became the longer one: 0.228 vs 0.210 ms)
        HIP_TRY(c, hipEventRecord(c->ev_fork, st));
        HIP_TRY(c, hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
    }
    for (int i : dset) {
        GroupArgs ga = c->pargs.g[(size_t)i];
        ga.samples = resolved[(size_t)i];
        HIP_TRY(c, launch_stage(ga, c->d_step, st));
    }
    hipStream_t pst = fork ? c->side_stream : st;
    for (int i : c->side_set) {
        const Group &g = c->groups[(size_t)i];
        hipEvent_t r0 = nullptr, r1 = nullptr;
        if (timed) {
            int rc = next_events(c, 2, &r0, &r1);
            if (rc != CORR_OK) return rc;
            HIP_TRY(c, hipEventRecord(r0, pst));
        }
        FoldStamps *pst_stamps = c->d_stamps ? c->d_stamps + 1 : nullptr;
        if (g.mom) {
            MomentumArgs ma = g.mom_args;
            ma.vel = src[i];
            ma.vec4 = g.d.n_atoms % 4 == 0 && reinterpret_cast<uintptr_t>(src[i]) % 16 == 0;
            ma.stamps = pst_stamps;
            HIP_TRY(c, launch_momentum(ma, pst));
        } else if (g.rhok_mfma) {
            RhokMfmaArgs ma = g.margs;
            ma.pos = static_cast<const float *>(src[i]);
            ma.stamps = pst_stamps;
            ma.early_loads = fork && !chained ? 1 : 0; // beside the flush, joined every push
            HIP_TRY(c, launch_rhok_mfma(ma, pst));
        } else {
            RhokArgs ra = g.rargs;
            ra.pos = static_cast<const float *>(src[i]);
            ra.stamps = pst_stamps;
            HIP_TRY(c, launch_rhok(ra, pst));
        }
        if (timed) HIP_TRY(c, hipEventRecord(r1, pst));
    }
    if (fork && !dset.empty()) {
        // the per-step push of every direct group, sample-fed ones included,
        // in one launch after the producers: the main stream keeps only the
        // staging and the flush of the block-deferred groups
        std::vector<int> idx(c->main_set);
        idx.insert(idx.end(), c->side_set.begin(), c->side_set.end());
        int rc = launch_set(c, c->pa_direct, idx, resolved, pst);
        if (rc != CORR_OK) return rc;
        if (chained) {
            PushEndArgs se{};
            se.step = c->d_step_side;
            se.advance = 1;
            se.stamps = c->d_stamps ? c->d_stamps + 1 : nullptr;
            se.n_stamps = 1;
            HIP_TRY(c, launch_push_end(se, pst));
        } else {
            HIP_TRY(c, hipEventRecord(c->ev_join, pst));
        }
    } else if (fork) {
        // no flush to overlap: the sample-fed groups run beside the producers
        int rc = launch_set(c, c->pa_side, c->side_set, resolved, pst);
        if (rc != CORR_OK) return rc;
        HIP_TRY(c, hipEventRecord(c->ev_join, pst));
        rc = launch_set(c, c->pa_main, c->main_set, resolved, st);
        if (rc != CORR_OK) return rc;
    } else {
        std::vector<int> idx(c->main_set);
        idx.insert(idx.end(), c->side_set.begin(), c->side_set.end());
        if (!idx.empty()) {
            hipStream_t ust = st;
            if (fork_updates) {
                HIP_TRY(c, hipEventRecord(c->ev_fork, st));
                HIP_TRY(c, hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
                ust = c->side_stream;
            }
            int rc = launch_set(c, c->pa_direct, idx, resolved, ust);
            if (rc != CORR_OK) return rc;
            if (fork_updates) HIP_TRY(c, hipEventRecord(c->ev_join, ust));
        }
    }
    if (with_flush && !dset.empty()) {
        hipEvent_t f0 = nullptr, f1 = nullptr;
        if (timed) {
            int rc = next_events(c, 1, &f0, &f1);
            if (rc != CORR_OK) return rc;
        }
        int rc = launch_flushes(c, st, f0, f1);
        if (rc != CORR_OK) return rc;
    }
    if (fork_updates) HIP_TRY(c, hipStreamWaitEvent(st, c->ev_join, 0));
    if (timed) HIP_TRY(c, hipEventRecord(e1, st));
    if (fork && !chained) HIP_TRY(c, hipStreamWaitEvent(st, c->ev_join, 0));
    PushEndArgs pe{};
    pe.step = c->d_step;
    pe.step2 = chained ? nullptr : c->d_step_side;
    pe.advance = 1;
    if (with_flush)
        for (int i : dset) {
            pe.defer_t[pe.n_flushed] = c->groups[(size_t)i].T;
            pe.flushed[pe.n_flushed++] = c->groups[(size_t)i].d_flushed;
        }
    pe.stamps = c->d_stamps; // timing: adds this push's fold (and producer) spans
    pe.n_stamps = chained ? 1 : 2;
    HIP_TRY(c, launch_push_end(pe, st));
    return CORR_OK;
}

// Capture one push of every group (reading the current input buffers) into a
// graph, with or without the flush of the block-deferred groups.
int capture_one(corr_ctx *c, bool with_flush, hipGraph_t *g_out, hipGraphExec_t *x_out)
{
    std::vector<const void *> src(c->groups.size());
    for (size_t i = 0; i < c->groups.size(); ++i) src[i] = c->groups[i].input;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = issue_push(c, src.data(), c->cap_stream, with_flush);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc != CORR_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return hip_err(c, ec, "hipStreamEndCapture");
    *g_out = graph;
    HIP_TRY(c, hipGraphInstantiate(x_out, graph, nullptr, nullptr, 0));
    return CORR_OK;
}

// (Re)capture the push graphs.
int capture_graph(corr_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    return capture_one(c, !c->deferred_set.empty(), &c->graph, &c->gexec);
}

int ensure_scratch(corr_ctx *c, size_t bytes)
{
    if (c->scratch_bytes >= bytes) return CORR_OK;
    if (c->d_scratch) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        (void)hipFree(c->d_scratch);
        c->d_scratch = nullptr;
        c->scratch_bytes = 0;
    }
    HIP_TRY(c, hipMalloc(&c->d_scratch, bytes));
    c->scratch_bytes = bytes;
    return CORR_OK;
}

struct Entry {
    int level, lag;
    int64_t count;
    int64_t hi_off, lo_off;
};

} // namespace

extern "C" {

const char *corr_last_error(const corr_ctx *ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

int corr_create(const corr_group_desc *groups, int32_t n_groups, int32_t device, void *stream,
                uint32_t flags, const corr_tuning *tuning, corr_ctx **out)
{
    g_create_error.clear();
    if (!out) return set_err(nullptr, CORR_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!groups || n_groups < 1) return set_err(nullptr, CORR_E_INVALID, "need at least one group");
    if (n_groups > kMaxGroups)
        return set_err(nullptr, CORR_E_UNSUPPORTED, "at most %d groups per context", kMaxGroups);
    if (flags & ~(uint32_t)(CORR_FLAG_GRAPH | CORR_FLAG_PER_GROUP | CORR_FLAG_TIMING |
                            CORR_FLAG_DIRECT | CORR_FLAG_RHOK_VALU))
        return set_err(nullptr, CORR_E_INVALID, "unknown flags 0x%x", flags);
    for (int i = 0; i < n_groups; ++i) {
        int rc = validate(groups[i], i);
        if (rc != CORR_OK) return rc;
    }
    // Default launch shape: 512-channel tiles, 2 channels per thread (256-thread
    // blocks), 8 lags per load batch, a persistent grid of 8 blocks per CU,
    // producers on the context's stream.
    corr_tuning tn{512, 2, 8, 2048, 0, 0, 0};
    const bool given = tuning && (tuning->tile_channels || tuning->chans_per_thread ||
                                  tuning->lag_chunk || tuning->grid_blocks ||
                                  tuning->overlap_producers || tuning->fold_block ||
                                  tuning->fold_threads);
    if (!given) {
        // the autotuner's cached choice for these groups, if any
        corr_tuning cached{};
        if (tune_cache_lookup(tune_cache_path(nullptr), tune_key(groups, n_groups, flags, device),
                              &cached) &&
            validate_tuning(cached) == CORR_OK)
            tn = cached;
        g_create_error.clear();
    }
    if (given) {
        tn = *tuning;
        if (!tn.chans_per_thread) tn.chans_per_thread = 2;
        if (!tn.lag_chunk) tn.lag_chunk = tn.chans_per_thread == 1 ? 16 : tn.chans_per_thread == 2 ? 8 : 4;
        if (!tn.tile_channels) tn.tile_channels = 256 * tn.chans_per_thread;
    }
    {
        int rc = validate_tuning(tn);
        if (rc != CORR_OK) return rc;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_err(nullptr, CORR_E_DEVICE, "device %d not available (%d devices)", device, ndev);

    corr_ctx *c = new (std::nothrow) corr_ctx();
    if (!c) return set_err(nullptr, CORR_E_OOM, "host allocation failed");
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->flags = flags;
    c->tuning = tn;
    c->fold_threads = tn.fold_threads ? tn.fold_threads : kFoldThreadsDefault;
    DeviceGuard dg(device);

    auto fail = [&](int rc) {
        g_create_error = c->err;
        free_ctx(c);
        return rc;
    };
#define CREATE_HIP(expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(hip_err(c, e_, #expr));                                \
    } while (0)

    const int tw = tn.tile_channels;
    // Block length of the block-deferred groups: the tuning's, else the
    // longest whose state fits in the device's free memory (each step down
    // shortens the level-0 ring of 2 T + p rows), else the per-step form.
    bool fold_ok = !(flags & CORR_FLAG_DIRECT);
    {
        auto folds = [&](const corr_group_desc &d) {
            return d.source == CORR_SRC_SAMPLES && !d.pair &&
                   deferred_supported(kind_of(d.dtype, d.accum), d.points, d.m);
        };
        // device bytes of the context's groups with fold block T (0: the
        // per-step form for the foldable groups)
        auto ctx_bytes = [&](int T) {
            double total = 0.0;
            for (int i = 0; i < n_groups; ++i) {
                const corr_group_desc &d = groups[i];
                const int kind = kind_of(d.dtype, d.accum);
                const int64_t n_tiles = (d.n_channels + tw - 1) / tw;
                const int64_t rowS = (int64_t)tw * kind_sample_bytes(kind);
                const int64_t rowA = (int64_t)tw * kind_acc_bytes(kind);
                const int np = acc_planes(kind), nlk = d.points - d.points / d.m;
                const bool def = T > 0 && folds(d);
                const bool win = !def && d.levels == 1 && d.points >= kWindowMinP && !d.pair &&
                                 !(flags & CORR_FLAG_DIRECT) && window_deferred_supported(kind);
                const int64_t p0 = def ? 2 * T + d.points : win ? 2 * kWindowT + d.points : d.points;
                const int rings = d.pair ? 2 : 1;
                const int64_t tile = rings * p0 * rowS + np * (int64_t)d.points * rowA +
                                     (int64_t)(d.levels - 1) * (rings * d.points * rowS + np * nlk * rowA);
                total += (double)n_tiles * (double)tile;
                total += (double)(d.pair ? 2 : 1) * (double)d.n_channels * kind_sample_bytes(kind);
            }
            return total;
        };
        bool any_fold = false;
        for (int i = 0; i < n_groups; ++i) any_fold = any_fold || folds(groups[i]);
        c->defer_t = tn.fold_block ? tn.fold_block : kDeferT;
        if (fold_ok && any_fold && tn.fold_block == 0) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && total_b > 0) {
                // keep a margin for the runtime and the caller's next buffers
                const double avail = (double)free_b - std::max(1.0 * (1 << 30), 0.01 * (double)total_b);
                if (ctx_bytes(kDeferT) > avail) {
                    if (ctx_bytes(kDeferTMin) <= avail)
                        c->defer_t = kDeferTMin;
                    else if (ctx_bytes(0) <= avail)
                        fold_ok = false; // only the per-step form fits
                }
            }
        }
    }
    c->groups.resize((size_t)n_groups);
    int64_t tile_first = 0;
    for (int i = 0; i < n_groups; ++i) {
        Group &g = c->groups[(size_t)i];
        g.d = groups[i];
        g.d.kvec = nullptr;
        g.d.species = nullptr;
        g.d.masses = nullptr;
        g.kind = kind_of(g.d.dtype, g.d.accum);
        g.p = g.d.points;
        g.m = g.d.m;
        g.b = g.d.levels;
        g.lag0 = g.p / g.m;
        g.nlk = g.p - g.lag0;
        g.s_bytes = kind_sample_bytes(g.kind);
        g.a_bytes = kind_acc_bytes(g.kind);
        g.np = acc_planes(g.kind);
        g.n_ch = g.d.n_channels;
        g.n_tiles = (g.n_ch + tw - 1) / tw;
        const int64_t rowS = (int64_t)tw * g.s_bytes;
        const int64_t rowA = (int64_t)tw * g.a_bytes;
        g.pair = g.d.pair != 0;
        g.deferred = fold_ok && g.d.source == CORR_SRC_SAMPLES && !g.pair &&
                     deferred_supported(g.kind, g.p, g.m);
        g.T = g.deferred ? c->defer_t : 0;
        g.wdef = !(flags & CORR_FLAG_DIRECT) && !g.deferred && !g.pair && g.b == 1 &&
                 g.p >= kWindowMinP && window_deferred_supported(g.kind);
        g.p0 = g.deferred ? 2 * g.T + g.p : g.wdef ? 2 * kWindowT + g.p : g.p;
        // pair groups: each level holds the lagged y ring, then an x ring
        const int rings = g.pair ? 2 : 1;
        g.lvl0_bytes = rings * g.p0 * rowS + (int64_t)g.np * g.p * rowA;
        g.lvlk_bytes = rings * g.p * rowS + (int64_t)g.np * g.nlk * rowA;
        g.tile_bytes = g.lvl0_bytes + (int64_t)(g.b - 1) * g.lvlk_bytes;
        const size_t state_bytes = (size_t)g.n_tiles * (size_t)g.tile_bytes;
        CREATE_HIP(hipMalloc(&g.state, state_bytes));
        CREATE_HIP(hipMemsetAsync(g.state, 0, state_bytes, c->stream));
        if (g.deferred) {
            g.tiles_per_group = (g.n_tiles + g.T - 1) / g.T;
            g.flushed.assign((size_t)g.T, 0);
            CREATE_HIP(hipMalloc(&g.d_flushed, kFlushGroups * sizeof(int64_t)));
            CREATE_HIP(hipMemsetAsync(g.d_flushed, 0, kFlushGroups * sizeof(int64_t), c->stream));
        }

        g.rhok = g.d.source == CORR_SRC_RHOK || g.d.source == CORR_SRC_CURRENTS;
        if (g.rhok) {
            g.nw = g.d.source == CORR_SRC_CURRENTS ? 3 : 1;
            // positions [3][N]; currents: then velocities [3][N]
            g.input_bytes = (size_t)(g.nw == 3 ? 6 : 3) * (size_t)g.d.n_atoms * sizeof(float);
            const int nk = (int)(g.n_ch / g.nw);
            const int32_t *kv = groups[i].kvec;
            int nmax = 0;
            for (int q = 0; q < nk; ++q)
                for (int d = 0; d < 3; ++d) nmax = std::max(nmax, std::abs(kv[3 * q + d]));
            CREATE_HIP(hipMalloc(&g.rhok_out, (size_t)g.n_ch * g.s_bytes));
            CREATE_HIP(hipMemsetAsync(g.rhok_out, 0, (size_t)g.n_ch * g.s_bytes, c->stream));
            // Matrix-core form: rows = distinct (n_x, n_y), columns = |n_z|
            // (the only form for currents; validation keeps their components
            // within its range).
            g.rhok_mfma = g.nw == 3 ||
                          (!(flags & CORR_FLAG_RHOK_VALU) && nmax <= rhok_mfma_max_nmax());
            // Atom blocks of about 1000 atoms or more; the vector-unit
            // producer takes up to 512.
            int n_ab = (int)std::max<int64_t>(1, std::min<int64_t>(512, g.d.n_atoms / 1024));
            if (g.rhok_mfma) {
                // Rows of the contraction.  Currents: the distinct (n_x, n_y)
                // pairs, 16 per M tile, slots [pair][|n_z|][n_z < 0].  n(k):
                // the couples (n_x, |n_y|), 4 per M tile (one row per
                // component of the products they share), slots
                // [couple][|n_z|][n_y < 0][n_z < 0].
                const bool couples = g.nw == 1;
                const int per_tile = couples ? 4 : 16;
                const int n_signs = couples ? 4 : 2;
                std::map<std::pair<int, int>, int> pair_ix;
                auto row_key = [&](int q) {
                    return std::make_pair(kv[3 * q], couples ? std::abs(kv[3 * q + 1]) : kv[3 * q + 1]);
                };
                for (int q = 0; q < nk; ++q) pair_ix.emplace(row_key(q), 0);
                const int n_pairs = (int)pair_ix.size();
                const int n_mtiles = (n_pairs + per_tile - 1) / per_tile;
                // The matrix-core producer runs fastest with one block per
                // compute unit (its double-buffered LDS tables and one wave
                // per M tile fill a CU): CUs / M-tile chunks atom blocks.
                int n_cu = 0;
                CREATE_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device));
                const int per_cu = std::max(1, n_cu / rhok_mfma_chunks(n_mtiles, g.nw));
                n_ab = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(512, per_cu),
                                                                   g.d.n_atoms / 1024));
                const int ncol = rhok_mfma_cols();
                // table rows: the n_x and n_y (couples: |n_y|) ranges of the
                // rows (padding rows take the first row of each)
                int x_lo = kv[0], x_hi = kv[0], y_lo = row_key(0).second, y_hi = y_lo;
                for (int q = 0; q < nk; ++q) {
                    x_lo = std::min(x_lo, kv[3 * q]);
                    x_hi = std::max(x_hi, kv[3 * q]);
                    y_lo = std::min(y_lo, row_key(q).second);
                    y_hi = std::max(y_hi, row_key(q).second);
                }
                if (couples) y_lo = 0; // Y planes hold |n_y| = 0 .. y_hi
                std::vector<int32_t> pnx((size_t)n_mtiles * per_tile, x_lo), pny((size_t)n_mtiles * per_tile, y_lo);
                int u = 0;
                for (auto &e : pair_ix) {
                    e.second = u;
                    pnx[(size_t)u] = e.first.first;
                    pny[(size_t)u] = e.first.second;
                    ++u;
                }
                std::vector<int32_t> slot_k((size_t)n_mtiles * per_tile * ncol * n_signs, -1),
                    k_src((size_t)nk);
                for (int q = 0; q < nk; ++q) {
                    const int pm = pair_ix[row_key(q)];
                    const int nz = kv[3 * q + 2];
                    const int sign = couples ? (kv[3 * q + 1] < 0 ? 2 : 0) + (nz < 0 ? 1 : 0) : (nz < 0 ? 1 : 0);
                    const size_t slot = ((size_t)pm * ncol + std::abs(nz)) * n_signs + sign;
                    if (slot_k[slot] < 0) slot_k[slot] = q; // first listing of a k-vector
                    k_src[(size_t)q] = slot_k[slot];
                }
                std::vector<int32_t> packed;
                packed.insert(packed.end(), pnx.begin(), pnx.end());
                packed.insert(packed.end(), pny.begin(), pny.end());
                packed.insert(packed.end(), slot_k.begin(), slot_k.end());
                packed.insert(packed.end(), k_src.begin(), k_src.end());
                CREATE_HIP(hipMalloc(&g.d_mtab, packed.size() * sizeof(int32_t)));
                CREATE_HIP(hipMemcpy(g.d_mtab, packed.data(), packed.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice));
                CREATE_HIP(hipMalloc(&g.d_partial, (size_t)n_ab * nk * g.nw * 2 * sizeof(double)));
                CREATE_HIP(rhok_mfma_prepare((x_hi - x_lo + 1) + (y_hi - y_lo + 1), g.nw, nmax));
                if (g.nw == 3) {
                    // basis of each k-vector: khat, then e1 = the Cartesian axis
                    // least aligned with khat, made orthogonal to it and
                    // normalised, then e2 = khat x e1
                    std::vector<double> bas((size_t)nk * 9);
                    for (int q = 0; q < nk; ++q) {
                        double kh[3], e1[3], e2[3];
                        const double len = std::sqrt((double)kv[3 * q] * kv[3 * q] +
                                                     (double)kv[3 * q + 1] * kv[3 * q + 1] +
                                                     (double)kv[3 * q + 2] * kv[3 * q + 2]);
                        int ax = 0;
                        for (int d = 0; d < 3; ++d) kh[d] = kv[3 * q + d] / len;
                        for (int d = 1; d < 3; ++d)
                            if (std::fabs(kh[d]) < std::fabs(kh[ax])) ax = d;
                        double nrm = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            e1[d] = (d == ax ? 1.0 : 0.0) - kh[ax] * kh[d];
                            nrm += e1[d] * e1[d];
                        }
                        nrm = std::sqrt(nrm);
                        for (int d = 0; d < 3; ++d) e1[d] /= nrm;
                        e2[0] = kh[1] * e1[2] - kh[2] * e1[1];
                        e2[1] = kh[2] * e1[0] - kh[0] * e1[2];
                        e2[2] = kh[0] * e1[1] - kh[1] * e1[0];
                        for (int d = 0; d < 3; ++d) {
                            bas[(size_t)q * 9 + d] = kh[d];
                            bas[(size_t)q * 9 + 3 + d] = e1[d];
                            bas[(size_t)q * 9 + 6 + d] = e2[d];
                        }
                    }
                    CREATE_HIP(hipMalloc(&g.d_basis, bas.size() * sizeof(double)));
                    CREATE_HIP(hipMemcpy(g.d_basis, bas.data(), bas.size() * sizeof(double),
                                         hipMemcpyHostToDevice));
                }
                RhokMfmaArgs &r = g.margs;
                r.pos = nullptr;
                r.n_atoms = g.d.n_atoms;
                r.pair_nx = g.d_mtab;
                r.pair_ny = r.pair_nx + pnx.size();
                r.slot_k = r.pair_ny + pny.size();
                r.k_src = r.slot_k + slot_k.size();
                r.n_mtiles = n_mtiles;
                r.nmax = nmax;
                r.x_lo = x_lo;
                r.x_rows = x_hi - x_lo + 1;
                r.y_lo = y_lo;
                r.y_rows = y_hi - y_lo + 1;
                r.inv_box = 1.0 / g.d.box;
                r.partial = g.d_partial;
                r.n_atom_blocks = n_ab;
                r.atoms_per_block = (int32_t)((g.d.n_atoms + n_ab - 1) / n_ab);
                r.out = g.rhok_out;
                r.out_double = g.d.dtype == CORR_CF64 ? 1 : 0;
                r.nk = nk;
                r.nw = g.nw;
                r.basis = g.d_basis;
            } else {
                // Segments: k-vectors sharing (n_y, n_z) with n_x in a window of
                // kSegWidth, rows ordered by (n_z, n_y).
                std::vector<int> order((size_t)nk);
                for (int q = 0; q < nk; ++q) order[(size_t)q] = q;
                std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
                    for (int d = 2; d >= 0; --d)
                        if (kv[3 * x + d] != kv[3 * y + d]) return kv[3 * x + d] < kv[3 * y + d];
                    return false;
                });
                std::vector<int32_t> s_nx0, s_ny, s_nz, s_out;
                for (size_t u = 0; u < order.size();) {
                    const int k0 = order[u];
                    const int nx0 = kv[3 * k0], ny = kv[3 * k0 + 1], nz = kv[3 * k0 + 2];
                    int slots[kSegWidth];
                    for (int w = 0; w < kSegWidth; ++w) slots[w] = -1;
                    while (u < order.size()) {
                        const int kq = order[u];
                        const int w = kv[3 * kq] - nx0;
                        if (kv[3 * kq + 1] != ny || kv[3 * kq + 2] != nz || w >= kSegWidth ||
                            slots[w] >= 0)
                            break;
                        slots[w] = kq;
                        ++u;
                    }
                    s_nx0.push_back(nx0);
                    s_ny.push_back(ny);
                    s_nz.push_back(nz);
                    for (int w = 0; w < kSegWidth; ++w) s_out.push_back(slots[w]);
                }
                const int n_seg = (int)s_nx0.size();
                std::vector<int32_t> packed;
                packed.insert(packed.end(), s_nx0.begin(), s_nx0.end());
                packed.insert(packed.end(), s_ny.begin(), s_ny.end());
                packed.insert(packed.end(), s_nz.begin(), s_nz.end());
                packed.insert(packed.end(), s_out.begin(), s_out.end());
                CREATE_HIP(hipMalloc(&g.d_seg, packed.size() * sizeof(int32_t)));
                CREATE_HIP(hipMemcpy(g.d_seg, packed.data(), packed.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice));
                CREATE_HIP(hipMalloc(&g.d_partial,
                                     (size_t)n_ab * n_seg * kSegWidth * 2 * sizeof(double)));
                RhokArgs &r = g.rargs;
                r.pos = nullptr;
                r.n_atoms = g.d.n_atoms;
                r.seg_nx0 = g.d_seg;
                r.seg_ny = g.d_seg + n_seg;
                r.seg_nz = g.d_seg + 2 * n_seg;
                r.slot_out = g.d_seg + 3 * n_seg;
                r.n_seg = n_seg;
                r.nmax = nmax;
                r.inv_box = 1.0 / g.d.box;
                r.partial = g.d_partial;
                r.n_atom_blocks = n_ab;
                r.atoms_per_block = (int32_t)((g.d.n_atoms + n_ab - 1) / n_ab);
                r.out = g.rhok_out;
                r.out_double = g.d.dtype == CORR_CF64 ? 1 : 0;
            }
        } else if (g.d.source == CORR_SRC_MOMENTUM) {
            g.mom = true;
            // velocities [3][N] in the group's dtype; pair: then the x samples
            g.input_bytes = (size_t)(3 * g.d.n_atoms + (g.pair ? g.n_ch : 0)) * g.s_bytes;
            CREATE_HIP(hipMalloc(&g.rhok_out, (size_t)(g.pair ? 2 : 1) * g.n_ch * g.s_bytes));
            CREATE_HIP(hipMemsetAsync(g.rhok_out, 0, (size_t)(g.pair ? 2 : 1) * g.n_ch * g.s_bytes,
                                      c->stream));
            {
                std::vector<uint8_t> ids((size_t)g.d.n_atoms);
                for (int64_t a = 0; a < g.d.n_atoms; ++a) ids[(size_t)a] = (uint8_t)groups[i].species[a];
                CREATE_HIP(hipMalloc(&g.d_species, ids.size()));
                CREATE_HIP(hipMemcpy(g.d_species, ids.data(), ids.size(), hipMemcpyHostToDevice));
            }
            MomentumArgs &ma = g.mom_args;
            ma.vel = nullptr;
            ma.species = g.d_species;
            ma.n_atoms = g.d.n_atoms;
            ma.n_species = g.d.n_species;
            ma.dbl = g.d.dtype == CORR_F64 ? 1 : 0;
            const double volume = g.d.box * g.d.box * g.d.box;
            for (int s = 0; s < g.d.n_species; ++s) ma.scale[s] = groups[i].masses[s] / volume;
            ma.n_blocks = momentum_blocks(g.d.n_atoms);
            CREATE_HIP(hipMalloc(&g.d_partial,
                                 (size_t)ma.n_blocks * 3 * kMomMaxSpecies * sizeof(double)));
            ma.partial = g.d_partial;
            ma.pair = g.pair ? 1 : 0;
            ma.out = g.rhok_out;
        } else {
            g.input_bytes = (size_t)(g.pair ? 2 : 1) * (size_t)g.n_ch * g.s_bytes;
        }
        CREATE_HIP(hipMalloc(&g.own_input, g.input_bytes));
        CREATE_HIP(hipMemsetAsync(g.own_input, 0, g.input_bytes, c->stream));
        g.input = g.own_input;

        GroupArgs &ga = c->pargs.g[i];
        ga.samples = nullptr;
        ga.state = g.state;
        ga.n_ch = g.n_ch;
        ga.n_tiles = g.n_tiles;
        ga.tile_first = tile_first;
        ga.tile_bytes = g.tile_bytes;
        ga.lvl0_bytes = g.lvl0_bytes;
        ga.lvlk_bytes = g.lvlk_bytes;
        ga.kind = g.kind;
        ga.p = g.p;
        ga.m = g.m;
        ga.levels = g.b;
        ga.lag0 = g.lag0;
        ga.tw = tw;
        ga.s_bytes = g.s_bytes;
        ga.a_bytes = g.a_bytes;
        ga.deferred = (g.deferred || g.wdef) ? 1 : 0;
        ga.p0 = g.p0;
        ga.pair = g.pair ? 1 : 0;
        ga.defer_t = g.T;
        if (g.deferred) c->deferred_set.push_back(i);
        tile_first += g.n_tiles;
    }
    c->pargs.n_groups = n_groups;
    c->pargs.total_tiles = tile_first;
    c->total_tiles = tile_first;
    for (int i = 0; i < n_groups; ++i) {
        const Group &g = c->groups[(size_t)i];
        if (g.produced())
            c->side_set.push_back(i);
        else if (!g.deferred)
            c->main_set.push_back(i);
    }
    {
        std::vector<int> both(c->main_set);
        both.insert(both.end(), c->side_set.begin(), c->side_set.end());
        const std::vector<int> *sets[3] = {&c->main_set, &c->side_set, &both};
        PushArgs *pas[3] = {&c->pa_main, &c->pa_side, &c->pa_direct};
        for (int pass = 0; pass < 3; ++pass) {
            const std::vector<int> &idx = *sets[pass];
            PushArgs &pa = *pas[pass];
            pa = c->pargs;
            int64_t tf = 0;
            for (size_t j = 0; j < idx.size(); ++j) {
                pa.g[j] = c->pargs.g[(size_t)idx[j]];
                pa.g[j].tile_first = tf;
                tf += pa.g[j].n_tiles;
            }
            pa.n_groups = (int32_t)idx.size();
            pa.total_tiles = tf;
        }
    }
    const bool direct_groups = !c->main_set.empty() || !c->side_set.empty();
    if ((!c->side_set.empty() && (!c->main_set.empty() || !c->deferred_set.empty())) ||
        (!c->deferred_set.empty() && direct_groups)) {
        CREATE_HIP(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
        CREATE_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        CREATE_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    CREATE_HIP(hipMalloc(&c->d_step, 2 * sizeof(int64_t)));
    CREATE_HIP(hipMemsetAsync(c->d_step, 0, 2 * sizeof(int64_t), c->stream));
    c->d_step_side = c->d_step + 1;
    CREATE_HIP(noalloc_scratch(device, &c->noalloc));
    if (flags & CORR_FLAG_TIMING) {
        int khz = 0;
        CREATE_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
        c->stamp_khz = khz > 0 ? (double)khz : 0.0;
        std::vector<FoldStamps> init(2);
        for (size_t k = 0; k < init.size(); ++k) {
            FoldStamps &r = init[k];
            r = FoldStamps{};
            for (auto &sl : r.slot) sl.start = ~0ull;
            r.step = k == 0 ? c->d_step : c->d_step_side; // folds / producers
            r.stride = 1;
        }
        CREATE_HIP(hipMalloc(&c->d_stamps, 2 * sizeof(FoldStamps)));
        CREATE_HIP(hipMemcpy(c->d_stamps, init.data(), 2 * sizeof(FoldStamps), hipMemcpyHostToDevice));
    }
    c->pargs.step = c->d_step;
    c->pa_main.step = c->d_step;
    c->pa_side.step = c->d_step_side; // the sets that run on the side stream
    c->pa_direct.step = c->d_step_side;
    CREATE_HIP(hipStreamSynchronize(c->stream));

    if (flags & CORR_FLAG_GRAPH) {
        CREATE_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        int rc = capture_graph(c);
        if (rc != CORR_OK) return fail(rc);
    }
#undef CREATE_HIP
    *out = c;
    return CORR_OK;
}

int corr_input_buffer(corr_ctx *ctx, int32_t group, void **dev_ptr, size_t *bytes)
{
    if (!ctx) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size())
        return set_err(ctx, CORR_E_INVALID, "group %d out of range", group);
    if (dev_ptr) *dev_ptr = ctx->groups[(size_t)group].input;
    if (bytes) *bytes = ctx->groups[(size_t)group].input_bytes;
    return CORR_OK;
}

int corr_bind_input(corr_ctx *ctx, int32_t group, void *dev_ptr, size_t bytes)
{
    if (!ctx) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size())
        return set_err(ctx, CORR_E_INVALID, "group %d out of range", group);
    Group &g = ctx->groups[(size_t)group];
    if (dev_ptr && bytes < g.input_bytes)
        return set_err(ctx, CORR_E_INVALID, "bound buffer has %zu bytes, group needs %zu", bytes,
                       g.input_bytes);
    DeviceGuard dg(ctx->device);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    g.input = dev_ptr ? dev_ptr : g.own_input;
    if (ctx->flags & CORR_FLAG_GRAPH) return capture_graph(ctx);
    return CORR_OK;
}

int corr_push(corr_ctx *ctx, const void *const *samples)
{
    if (!ctx) return CORR_E_INVALID;
    DeviceGuard dg(ctx->device);
    const size_t ng = ctx->groups.size();
    std::vector<const void *> src(ng);
    bool all_default = true;
    for (size_t i = 0; i < ng; ++i) {
        const void *p = samples ? samples[i] : nullptr;
        if (!p) p = ctx->groups[i].input;
        if (p != ctx->groups[i].input) all_default = false;
        src[i] = p;
    }
    const bool with_flush = !ctx->deferred_set.empty();
    if (ctx->gexec && all_default) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if ((ctx->flags & CORR_FLAG_TIMING) && ctx->n_push % ctx->timing_stride == 0) {
            int rc = next_events(ctx, 0, &e0, &e1);
            if (rc != CORR_OK) return rc;
            HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
        }
        HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
        if (e1) HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
    } else {
        int rc = issue_push(ctx, src.data(), ctx->stream, with_flush);
        if (rc != CORR_OK) return rc;
    }
    ctx->n_push += 1;
    mirror_flushes(ctx, ctx->n_push);
    return CORR_OK;
}

// Chained pushes of a captured run meet (join and fork again) after every
// kChainSync pushes.  Unprofiled, meeting every 4 to 32 pushes or only at the
// end of the run gave the same batched step within 2% (0.175-0.179 ms); under
// kernel tracing, where the graph's kernels are submitted more slowly and
// stream by stream, long chains ran one after the other (0.250 ms, the fold
// 80 us alone) and chains of 4 pushes still overlapped (0.187 ms).
constexpr int32_t kChainSync = 4;

int corr_push_steps(corr_ctx *ctx, int32_t n_steps, const void *const *samples,
                    const int64_t *strides)
{
    if (!ctx || !samples || n_steps < 0) return CORR_E_INVALID;
    DeviceGuard dg(ctx->device);
    const size_t ng = ctx->groups.size();
    std::vector<int64_t> stride(ng);
    for (size_t i = 0; i < ng; ++i) {
        if (!samples[i]) return set_err(ctx, CORR_E_INVALID, "push_steps: group %d has no history", (int)i);
        stride[i] = strides ? strides[i] : (int64_t)ctx->groups[i].input_bytes;
        if (stride[i] < (int64_t)ctx->groups[i].input_bytes)
            return set_err(ctx, CORR_E_INVALID, "push_steps: stride of group %d below its push size",
                           (int)i);
    }
    const bool with_flush = !ctx->deferred_set.empty();
    std::vector<const void *> src(ng);
    auto row = [&](int32_t r) {
        for (size_t i = 0; i < ng; ++i)
            src[i] = static_cast<const char *>(samples[i]) + (int64_t)r * stride[i];
    };
    auto one_push = [&](int32_t r) -> int {
        row(r);
        int rc = issue_push(ctx, src.data(), ctx->stream, with_flush);
        if (rc != CORR_OK) return rc;
        ctx->n_push += 1;
        mirror_flushes(ctx, ctx->n_push);
        return CORR_OK;
    };
    if (n_steps == 0) return CORR_OK;

    if (ctx->flags & CORR_FLAG_GRAPH) {
        // Graph mode: the n pushes as one captured graph (the same kernels as
        // single pushes; they take their schedule from the device counters,
        // so a graph replays correctly at any push count), kept for the next
        // call with the same histories and length.  With the producers forked
        // beside block-deferred groups the two streams form two chains forked
        // and joined around every kChainSync pushes (chained pushes).
        std::vector<const void *> base(samples, samples + ng);
        auto &cache = ctx->steps_graphs;
        size_t hit = cache.size();
        for (size_t k = 0; k < cache.size(); ++k)
            if (cache[k].n == n_steps && cache[k].src == base && cache[k].stride == stride) hit = k;
        if (hit == cache.size()) {
            corr_ctx::StepsGraph sg;
            sg.n = n_steps;
            sg.src = base;
            sg.stride = stride;
            const bool chained = ctx->tuning.overlap_producers == 1 && !ctx->side_set.empty() &&
                                 with_flush;
            HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = CORR_OK;
            auto cap = [&](hipError_t e, const char *what) {
                if (rc == CORR_OK && e != hipSuccess) rc = hip_err(ctx, e, what);
            };
            if (chained) {
                cap(hipEventRecord(ctx->ev_fork, ctx->cap_stream), "hipEventRecord");
                cap(hipStreamWaitEvent(ctx->side_stream, ctx->ev_fork, 0), "hipStreamWaitEvent");
            }
            for (int32_t r = 0; r < n_steps && rc == CORR_OK; ++r) {
                row(r);
                rc = issue_push(ctx, src.data(), ctx->cap_stream, with_flush, false, chained);
                if (chained && rc == CORR_OK && (r + 1) % kChainSync == 0 && r + 1 < n_steps) {
                    cap(hipEventRecord(ctx->ev_join, ctx->side_stream), "hipEventRecord");
                    cap(hipStreamWaitEvent(ctx->cap_stream, ctx->ev_join, 0), "hipStreamWaitEvent");
                    cap(hipEventRecord(ctx->ev_fork, ctx->cap_stream), "hipEventRecord");
                    cap(hipStreamWaitEvent(ctx->side_stream, ctx->ev_fork, 0), "hipStreamWaitEvent");
                }
            }
            if (chained) {
                // joined even after an error: the capture must end with the
                // side stream back in the main one
                const int rc0 = rc;
                rc = CORR_OK;
                cap(hipEventRecord(ctx->ev_join, ctx->side_stream), "hipEventRecord");
                cap(hipStreamWaitEvent(ctx->cap_stream, ctx->ev_join, 0), "hipStreamWaitEvent");
                if (rc0 != CORR_OK) rc = rc0;
            }
            const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &sg.graph);
            if (rc != CORR_OK || ec != hipSuccess) {
                if (sg.graph) (void)hipGraphDestroy(sg.graph);
                return rc != CORR_OK ? rc : hip_err(ctx, ec, "hipStreamEndCapture");
            }
            const hipError_t ei = hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0);
            if (ei != hipSuccess) {
                (void)hipGraphDestroy(sg.graph);
                return hip_err(ctx, ei, "hipGraphInstantiate");
            }
            if (cache.size() >= 4) { // keep the most recent few
                (void)hipGraphExecDestroy(cache.front().exec);
                (void)hipGraphDestroy(cache.front().graph);
                cache.erase(cache.begin());
            }
            cache.push_back(std::move(sg));
            hit = cache.size() - 1;
        }
        HIP_TRY(ctx, hipGraphLaunch(cache[hit].exec, ctx->stream));
        for (int32_t r = 0; r < n_steps; ++r) {
            ctx->n_push += 1;
            mirror_flushes(ctx, ctx->n_push);
        }
        return CORR_OK;
    }

    int32_t r = 0;
    const int T = ctx->defer_t;
    if (!ctx->deferred_set.empty() && n_steps >= T) {
        // Block-deferred groups fold whole blocks of the history directly.
        // Up to the next block boundary the pushes are single pushes.
        while (r < n_steps && ctx->n_push % T != 0) {
            int rc = one_push(r++);
            if (rc != CORR_OK) return rc;
        }
        const bool others = !ctx->main_set.empty() || !ctx->side_set.empty();
        int64_t q = ctx->n_push / T; // blocks that end at or before the current push
        bool behind = false;          // some tile group has not folded block q yet
        for (int i : ctx->deferred_set)
            for (int64_t f : ctx->groups[(size_t)i].flushed) behind = behind || f < q;
        if (n_steps - r >= T && q >= 1 && behind) {
            // every tile group folds block q now (their scheduled folds would
            // come during the next T - 1 pushes)
            for (int i : ctx->deferred_set) {
                DeferredArgs da = deferred_args(ctx, i);
                da.fixed_group = -2;
                da.fixed_block = q;
                HIP_TRY(ctx, launch_flush_fold(da, ctx->stream));
            }
            PushEndArgs pe{};
            pe.step = ctx->d_step;
            pe.step2 = ctx->d_step_side;
            pe.advance = 0;
            pe.commit_block = q;
            for (int i : ctx->deferred_set) {
                pe.defer_t[pe.n_flushed] = ctx->groups[(size_t)i].T;
                pe.flushed[pe.n_flushed++] = ctx->groups[(size_t)i].d_flushed;
            }
            HIP_TRY(ctx, launch_push_end(pe, ctx->stream));
            for (int i : ctx->deferred_set) {
                Group &g = ctx->groups[(size_t)i];
                for (int j = 0; j < g.T; ++j) g.flushed[(size_t)j] = std::max(g.flushed[(size_t)j], q);
            }
        }
        while (n_steps - r >= T) {
            // the other groups' pushes of the block, one by one
            if (others)
                for (int k = 0; k < T; ++k) {
                    row(r + k);
                    int rc = issue_push(ctx, src.data(), ctx->stream, false, true);
                    if (rc != CORR_OK) return rc;
                    ctx->n_push += 1;
                }
            // block q + 1 of every block-deferred group, read from the history
            for (int i : ctx->deferred_set) {
                DeferredArgs da = deferred_args(ctx, i);
                da.fixed_group = -2;
                da.fixed_block = q + 1;
                da.hist = static_cast<const char *>(samples[(size_t)i]) + (int64_t)r * stride[(size_t)i];
                da.hist_stride = stride[(size_t)i];
                da.stamps = ctx->d_stamps;
                HIP_TRY(ctx, launch_history_fold(da, ctx->stream));
            }
            PushEndArgs pe{};
            pe.step = ctx->d_step;
            pe.step2 = ctx->d_step_side;
            pe.advance = others ? 0 : T; // the other groups' pushes advanced the counter
            pe.commit_block = q + 1;
            pe.stamps = ctx->d_stamps;
            pe.n_stamps = 2;
            for (int i : ctx->deferred_set) {
                pe.defer_t[pe.n_flushed] = ctx->groups[(size_t)i].T;
                pe.flushed[pe.n_flushed++] = ctx->groups[(size_t)i].d_flushed;
            }
            HIP_TRY(ctx, launch_push_end(pe, ctx->stream));
            q += 1;
            r += T;
            if (!others) ctx->n_push += T;
            for (int i : ctx->deferred_set) {
                Group &g = ctx->groups[(size_t)i];
                for (int j = 0; j < g.T; ++j) g.flushed[(size_t)j] = std::max(g.flushed[(size_t)j], q);
            }
        }
    }
    while (r < n_steps) {
        int rc = one_push(r++);
        if (rc != CORR_OK) return rc;
    }
    return CORR_OK;
}

int corr_group_form(const corr_ctx *ctx, int32_t group, int32_t *form, int32_t *block)
{
    if (!ctx) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size()) return CORR_E_INVALID;
    const Group &g = ctx->groups[(size_t)group];
    const bool win = g.b == 1 && g.p >= kWindowMinP;
    const int f = g.deferred ? 1 : g.wdef ? 2 : win ? 3 : 0;
    if (form) *form = f;
    if (block) *block = g.deferred ? g.T : g.wdef ? kWindowT : 0;
    return CORR_OK;
}

int corr_query(const corr_ctx *ctx, int32_t group, int64_t *n_pushes, int32_t *n_out_max)
{
    if (!ctx) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size()) return CORR_E_INVALID;
    const Group &g = ctx->groups[(size_t)group];
    if (n_pushes) *n_pushes = ctx->n_push;
    if (n_out_max) *n_out_max = g.p + (g.b - 1) * g.nlk;
    return CORR_OK;
}

int corr_state_bytes(const corr_ctx *ctx, int32_t group, int64_t *bytes)
{
    if (!ctx || !bytes) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size()) return CORR_E_INVALID;
    const Group &g = ctx->groups[(size_t)group];
    *bytes = g.n_tiles * g.tile_bytes;
    return CORR_OK;
}

int corr_kernel_time(corr_ctx *ctx, int32_t which, double *ms_total, int64_t *n, int32_t reset)
{
    if (!ctx) return CORR_E_INVALID;
    if (which < 0 || which > 4) return set_err(ctx, CORR_E_INVALID, "which must be 0 .. 4");
    if (!(ctx->flags & CORR_FLAG_TIMING))
        return set_err(ctx, CORR_E_STATE, "context created without CORR_FLAG_TIMING");
    DeviceGuard dg(ctx->device);
    if (which >= 3) {
        // device stamps of the folds (3) or the producers (4), every push
        FoldStamps *rec = ctx->d_stamps + (which - 3);
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        unsigned long long tc[2] = {0, 0}; // total, count
        HIP_TRY(ctx, hipMemcpy(tc, &rec->total, sizeof(tc), hipMemcpyDeviceToHost));
        if (ms_total) *ms_total = ctx->stamp_khz > 0 ? (double)tc[0] / ctx->stamp_khz : 0.0;
        if (n) *n = (int64_t)tc[1];
        if (reset) {
            const unsigned long long zero[2] = {0, 0};
            HIP_TRY(ctx, hipMemcpy(&rec->total, zero, sizeof(zero), hipMemcpyHostToDevice));
        }
        return CORR_OK;
    }
    int rc = fold_events(ctx, which);
    if (rc != CORR_OK) return rc;
    auto &pl = ctx->pools[which];
    if (ms_total) *ms_total = pl.ms;
    if (n) *n = pl.n;
    if (reset) {
        pl.ms = 0.0;
        pl.n = 0;
    }
    return CORR_OK;
}

int corr_set_timing_stride(corr_ctx *ctx, int32_t stride)
{
    if (!ctx) return CORR_E_INVALID;
    if (stride < 1) return set_err(ctx, CORR_E_INVALID, "timing stride must be >= 1");
    if (!(ctx->flags & CORR_FLAG_TIMING))
        return set_err(ctx, CORR_E_STATE, "timing stride without CORR_FLAG_TIMING");
    // the device stamps read their stride next to the push counter (so that
    // captured graphs follow it too), ordered after the pushes already issued
    const long long st = stride;
    for (int r = 0; r < 2; ++r)
        HIP_TRY(ctx, hipMemcpyAsync(&ctx->d_stamps[r].stride, &st, sizeof(st), hipMemcpyHostToDevice,
                                    ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->timing_stride = stride;
    return CORR_OK;
}

int corr_get_tuning(const corr_ctx *ctx, corr_tuning *out)
{
    if (!ctx || !out) return CORR_E_INVALID;
    *out = ctx->tuning;
    return CORR_OK;
}

int corr_sync(corr_ctx *ctx)
{
    if (!ctx) return CORR_E_INVALID;
    DeviceGuard dg(ctx->device);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return CORR_OK;
}

int corr_destroy(corr_ctx *ctx)
{
    if (!ctx) return CORR_E_INVALID;
    free_ctx(ctx);
    return CORR_OK;
}

} // extern "C"

namespace {

// Scratch of one readout: the context's own buffer (grown with hipMalloc) or,
// for corr_finalize_noalloc, the device's fixed array.
int readout_scratch(corr_ctx *ctx, bool noalloc, size_t bytes, char **out)
{
    if (noalloc) {
        if (bytes > kNoAllocBytes)
            return set_err(ctx, CORR_E_UNSUPPORTED,
                           "readout needs %zu bytes of scratch; corr_finalize_noalloc has %zu",
                           bytes, kNoAllocBytes);
        *out = static_cast<char *>(ctx->noalloc);
        return CORR_OK;
    }
    int rc = ensure_scratch(ctx, bytes);
    if (rc != CORR_OK) return rc;
    *out = static_cast<char *>(ctx->d_scratch);
    return CORR_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

int finalize_impl(corr_ctx *ctx, int32_t group, const corr_readout_opts *opts, int32_t *n_out,
                  double *t, double *c, int64_t *count, double *gk_running, double *gk_at_cut,
                  double *c_per_channel, bool noalloc)
{
    if (!ctx) return CORR_E_INVALID;
    if (group < 0 || group >= (int)ctx->groups.size())
        return set_err(ctx, CORR_E_INVALID, "group %d out of range", group);
    if (!n_out || !c) return set_err(ctx, CORR_E_INVALID, "n_out and c are required");
    DeviceGuard dg(ctx->device);
    const Group &g = ctx->groups[(size_t)group];
    corr_readout_opts o{};
    if (opts) o = *opts;
    int64_t cb = o.ch_begin, ce = o.ch_end;
    if (cb == 0 && ce == 0) ce = g.n_ch;
    if (cb < 0 || ce > g.n_ch || cb >= ce)
        return set_err(ctx, CORR_E_INVALID, "channel range [%lld, %lld) invalid", (long long)cb,
                       (long long)ce);
    const bool want_slice = c_per_channel != nullptr;
    int64_t sb = o.slice_begin, se = o.slice_end;
    if (want_slice && (sb < 0 || se > g.n_ch || sb >= se))
        return set_err(ctx, CORR_E_INVALID, "slice [%lld, %lld) invalid", (long long)sb,
                       (long long)se);
    if (o.gk_kind < 0 || o.gk_kind > 2) return set_err(ctx, CORR_E_INVALID, "gk_kind must be 0, 1 or 2");
    if (o.gk_kind != 0 && !(o.volume > 0 && o.kB > 0 && o.temperature > 0))
        return set_err(ctx, CORR_E_INVALID, "Green-Kubo prefactor needs volume, kB, temperature > 0");

    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t S = ctx->n_push;
    const int tw = ctx->tuning.tile_channels;
    const int64_t rowS = (int64_t)tw * g.s_bytes;
    const int64_t rowA = (int64_t)tw * g.a_bytes;

    // Entries with non-zero count, Algorithm 2 order.
    std::vector<Entry> ent;
    {
        int64_t Sk = S;
        for (int k = 0; k < g.b && Sk > 0; ++k) {
            const int l0 = k == 0 ? 0 : g.lag0;
            const int nl = k == 0 ? g.p : g.nlk;
            const int64_t lvl = k == 0 ? 0 : g.lvl0_bytes + (int64_t)(k - 1) * g.lvlk_bytes;
            for (int L = l0; L < g.p; ++L) {
                const int64_t cnt = Sk - L;
                if (cnt <= 0) continue;
                Entry e;
                e.level = k;
                e.lag = L;
                e.count = cnt;
                const int ring_rows = (g.pair ? 2 : 1) * (k == 0 ? g.p0 : g.p);
                e.hi_off = lvl + (int64_t)ring_rows * rowS + (int64_t)(L - l0) * rowA;
                e.lo_off = e.hi_off + (int64_t)nl * rowA;
                ent.push_back(e);
            }
            Sk /= g.m;
        }
    }
    const int ne = (int)ent.size();
    *n_out = ne;
    if (ne == 0) {
        if (gk_at_cut) *gk_at_cut = 0.0;
        return CORR_OK;
    }
    const int64_t nsel = ce - cb;
    const int bpe = (int)std::max<int64_t>(1, std::min<int64_t>(256, (nsel + 4095) / 4096));
    const int64_t n_slice = want_slice ? (se - sb) : 0;
    std::vector<double> sums((size_t)ne * 2);
    std::vector<double> slice;
    if (g.deferred) {
        // Block-deferred group: fold pending complete blocks (the scheduled
        // flush would produce the same state), then fold the pushes after the
        // last block on the fly (no state is written) and reduce.
        const GroupArgs &ga = ctx->pargs.g[(size_t)group];
        // Per-chunk sums are reduced in passes over whole column groups of
        // rows; corr_finalize takes all rows in one pass, the no-alloc
        // readout as many groups per pass as its fixed scratch holds (the
        // same sums in the same order either way).
        const int64_t n_rows = deferred_readout_rows(ga);
        const int64_t n_cg = deferred_readout_groups(ga);
        const int64_t cg_rows = deferred_readout_group_rows();
        const size_t gr_bytes = round256((size_t)n_cg * ne * sizeof(double));
        const size_t s_bytes = round256((size_t)ne * sizeof(double));
        const size_t sl_bytes = round256((size_t)std::max<int64_t>(n_slice, 1) * ne * sizeof(double));
        const size_t fixed = gr_bytes + s_bytes + sl_bytes;
        const size_t cg_bytes = (size_t)cg_rows * ne * sizeof(double);
        int64_t cg_per_pass = n_cg;
        if (noalloc) {
            if (fixed + std::min<size_t>(cg_bytes, (size_t)n_rows * ne * sizeof(double)) > kNoAllocBytes)
                return set_err(ctx, CORR_E_UNSUPPORTED,
                               "readout needs more than the %zu bytes of scratch of "
                               "corr_finalize_noalloc (%d entries, slice of %lld channels)",
                               kNoAllocBytes, ne, (long long)n_slice);
            cg_per_pass = std::max<int64_t>(1, std::min<int64_t>(n_cg, (int64_t)((kNoAllocBytes - fixed) / cg_bytes)));
        }
        const size_t tp_bytes =
            round256((size_t)std::min<int64_t>(n_rows, cg_per_pass * cg_rows) * ne * sizeof(double));
        char *sc = nullptr;
        {
            int rc = readout_scratch(ctx, noalloc, tp_bytes + fixed, &sc);
            if (rc != CORR_OK) return rc;
            rc = catch_up_flushes(ctx, group);
            if (rc != CORR_OK) return rc;
        }
        DeferredArgs da{};
        da.g = ctx->pargs.g[(size_t)group];
        da.step = ctx->d_step;
        da.ne = ne;
        da.ch_begin = cb;
        da.ch_end = ce;
        da.slice_begin = want_slice ? sb : 0;
        da.slice_end = want_slice ? se : 0;
        da.chunk_partial = reinterpret_cast<double *>(sc);
        double *d_groups = reinterpret_cast<double *>(sc + tp_bytes);
        double *d_sums = reinterpret_cast<double *>(sc + tp_bytes + gr_bytes);
        da.slice_out = reinterpret_cast<double *>(sc + tp_bytes + gr_bytes + s_bytes);
        for (int64_t g0 = 0; g0 < n_cg; g0 += cg_per_pass) {
            const int64_t g1 = std::min(n_cg, g0 + cg_per_pass);
            da.row_begin = g0 * cg_rows;
            da.row_end = std::min(n_rows, g1 * cg_rows);
            HIP_TRY(ctx, launch_deferred_readout_pass(da, d_groups, ctx->stream));
        }
        HIP_TRY(ctx, launch_deferred_readout_final(da, d_groups, d_sums, ctx->stream));
        std::vector<double> re((size_t)ne);
        HIP_TRY(ctx, hipMemcpyAsync(re.data(), d_sums, (size_t)ne * sizeof(double),
                                    hipMemcpyDeviceToHost, ctx->stream));
        std::vector<double> sl;
        if (want_slice) {
            sl.resize((size_t)n_slice * ne);
            HIP_TRY(ctx, hipMemcpyAsync(sl.data(), da.slice_out, (size_t)n_slice * ne * sizeof(double),
                                        hipMemcpyDeviceToHost, ctx->stream));
        }
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        for (int i = 0; i < ne; ++i) {
            sums[(size_t)2 * i] = re[(size_t)i];
            sums[(size_t)2 * i + 1] = 0.0;
        }
        if (want_slice) {
            slice.assign((size_t)n_slice * ne * 2, 0.0);
            for (size_t i = 0; i < sl.size(); ++i) slice[2 * i] = sl[i];
        }
    } else {
    // scratch: offsets (2 * ne int64), partial (ne * bpe * 2 doubles), sums (ne * 2 doubles),
    // slice (n_slice * ne * 2 doubles)
    const size_t off_bytes = (size_t)2 * ne * sizeof(int64_t);
    const size_t part_bytes = (size_t)ne * bpe * 2 * sizeof(double);
    const size_t sum_bytes = (size_t)ne * 2 * sizeof(double);
    const size_t slice_bytes = (size_t)n_slice * ne * 2 * sizeof(double);
    const size_t total = off_bytes + part_bytes + sum_bytes + std::max(slice_bytes, (size_t)16);
    char *sc = nullptr;
    {
        int rc = readout_scratch(ctx, noalloc, total, &sc);
        if (rc != CORR_OK) return rc;
    }
    int64_t *d_off = reinterpret_cast<int64_t *>(sc);
    double *d_part = reinterpret_cast<double *>(sc + off_bytes);
    double *d_sum = reinterpret_cast<double *>(sc + off_bytes + part_bytes);
    double *d_slice = reinterpret_cast<double *>(sc + off_bytes + part_bytes + sum_bytes);
    std::vector<int64_t> offs((size_t)2 * ne);
    for (int i = 0; i < ne; ++i) {
        offs[(size_t)i] = ent[(size_t)i].hi_off;
        offs[(size_t)ne + i] = ent[(size_t)i].lo_off;
    }
    HIP_TRY(ctx, hipMemcpyAsync(d_off, offs.data(), off_bytes, hipMemcpyHostToDevice, ctx->stream));
    ReduceArgs ra{};
    ra.state = g.state;
    ra.tile_bytes = g.tile_bytes;
    ra.tw = tw;
    ra.kind = g.kind;
    ra.hi_off = d_off;
    ra.lo_off = d_off + ne;
    ra.n_entries = ne;
    ra.blocks_per_entry = bpe;
    ra.ch_begin = cb;
    ra.ch_end = ce;
    ra.partial = d_part;
    ra.out = d_sum;
    ra.wlpb = g.wdef ? window_lags_per_block(g.p) : 0;
    ra.p0 = g.p0;
    ra.n_push = S;
    HIP_TRY(ctx, launch_reduce(ra, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(sums.data(), d_sum, sum_bytes, hipMemcpyDeviceToHost, ctx->stream));
    if (want_slice) {
        ReduceArgs rs = ra;
        rs.ch_begin = sb;
        rs.ch_end = se;
        rs.out = d_slice;
        HIP_TRY(ctx, launch_gather(rs, ctx->stream));
        slice.resize((size_t)n_slice * ne * 2);
        HIP_TRY(ctx, hipMemcpyAsync(slice.data(), d_slice, slice_bytes, hipMemcpyDeviceToHost,
                                    ctx->stream));
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }

    const bool cplx = kind_complex(g.kind);
    // F(k,t) = <n n*> / N; currents likewise per atom
    const double norm = g.rhok ? 1.0 / (double)g.d.n_atoms : 1.0;
    const double tunit = (double)g.d.update_every * g.d.dt;
    std::vector<double> tt((size_t)ne), cre((size_t)ne);
    for (int i = 0; i < ne; ++i) {
        const Entry &e = ent[(size_t)i];
        double mk = 1.0;
        for (int j = 0; j < e.level; ++j) mk *= (double)g.m;
        tt[(size_t)i] = (double)e.lag * mk * tunit;
        const double den = (double)e.count * (double)nsel;
        const double vr = sums[(size_t)2 * i] / den * norm;
        const double vi = sums[(size_t)2 * i + 1] / den * norm;
        cre[(size_t)i] = vr;
        if (t) t[i] = tt[(size_t)i];
        if (count) count[i] = e.count;
        if (cplx) {
            c[2 * i] = vr;
            c[2 * i + 1] = vi;
        } else {
            c[i] = vr;
        }
    }
    if (want_slice) {
        for (int64_t s = 0; s < n_slice; ++s)
            for (int i = 0; i < ne; ++i) {
                const double den = (double)ent[(size_t)i].count;
                const double vr = slice[((size_t)s * ne + i) * 2] / den * norm;
                const double vi = slice[((size_t)s * ne + i) * 2 + 1] / den * norm;
                if (cplx) {
                    c_per_channel[((size_t)s * ne + i) * 2] = vr;
                    c_per_channel[((size_t)s * ne + i) * 2 + 1] = vi;
                } else {
                    c_per_channel[(size_t)s * ne + i] = vr;
                }
            }
    }
    // Green-Kubo: trapezoid of Re C over the emitted lag grid from t = 0 (the
    // grid is increasing when m divides p; otherwise it is taken in sorted order).
    double pref = 1.0;
    if (o.gk_kind == 1) pref = o.volume / (o.kB * o.temperature);
    if (o.gk_kind == 2) pref = o.volume / (3.0 * o.kB * o.temperature * o.temperature) * 3.0;
    std::vector<int> ord((size_t)ne);
    for (int i = 0; i < ne; ++i) ord[(size_t)i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return tt[(size_t)a] < tt[(size_t)b]; });
    const double tcut = o.t_cut > 0 ? o.t_cut : tt[(size_t)ord.back()];
    double acc = 0.0, at_cut = 0.0;
    bool cut_done = tcut <= tt[(size_t)ord[0]];
    if (gk_running) gk_running[ord[0]] = 0.0;
    for (int j = 1; j < ne; ++j) {
        const int i0 = ord[(size_t)j - 1], i1 = ord[(size_t)j];
        const double t0 = tt[(size_t)i0], t1 = tt[(size_t)i1];
        const double c0 = cre[(size_t)i0], c1 = cre[(size_t)i1];
        if (!cut_done && tcut < t1) {
            const double f = (tcut - t0) / (t1 - t0);
            const double cc = c0 + f * (c1 - c0);
            at_cut = acc + 0.5 * (tcut - t0) * (c0 + cc);
            cut_done = true;
        }
        acc += 0.5 * (t1 - t0) * (c0 + c1);
        if (gk_running) gk_running[i1] = acc * pref;
    }
    if (!cut_done) at_cut = acc;
    if (gk_at_cut) *gk_at_cut = at_cut * pref;
    return CORR_OK;
}

} // namespace

extern "C" {

int corr_finalize(corr_ctx *ctx, int32_t group, const corr_readout_opts *opts, int32_t *n_out,
                  double *t, double *c, int64_t *count, double *gk_running, double *gk_at_cut,
                  double *c_per_channel)
{
    return finalize_impl(ctx, group, opts, n_out, t, c, count, gk_running, gk_at_cut,
                         c_per_channel, false);
}

int corr_finalize_noalloc(corr_ctx *ctx, int32_t group, const corr_readout_opts *opts,
                          int32_t *n_out, double *t, double *c, int64_t *count, double *gk_running,
                          double *gk_at_cut, double *c_per_channel)
{
    return finalize_impl(ctx, group, opts, n_out, t, c, count, gk_running, gk_at_cut,
                         c_per_channel, true);
}

} // extern "C"
