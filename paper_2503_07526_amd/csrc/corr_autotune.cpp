// corr_autotune.cpp -- launch-shape autotuner with a persistent cache.
//
// The launch shape (tile width, channels per thread, lag batch, persistent
// grid size, issue order, the fold kernel's block length and threads per
// block) changes neither results beyond rounding nor state semantics, only
// speed, and the best choice depends on the mix of groups.  corr_autotune
// times trial contexts over whole flush periods for a fixed list of
// candidates and caches the winner per (device architecture, flags, group
// descriptors) in a text file of JSON lines; corr_create consults the cache
// when the caller passes no tuning.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/corr.h"
#include "corr_internal.h"
#include "corr_tune.h"

namespace corr {

std::string tune_cache_path(const char *explicit_path)
{
    if (explicit_path && *explicit_path) return explicit_path;
    if (const char *e = std::getenv("CORR_TUNE_CACHE")) return e;
    if (const char *h = std::getenv("HOME")) {
        std::string dir = std::string(h) + "/.cache";
        ::mkdir(dir.c_str(), 0755); // may already exist
        return dir + "/corr_gfx950_tune.jsonl";
    }
    return std::string();
}

std::string tune_key(const corr_group_desc *g, int n, uint32_t flags, int device)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::ostringstream os;
    os << "arch=" << arch << ";flags=" << (flags & ~(uint32_t)CORR_FLAG_TIMING);
    for (int i = 0; i < n; ++i) {
        os << ";g" << i << "=" << g[i].n_channels << "," << g[i].levels << "," << g[i].points << ","
           << g[i].m << "," << g[i].dtype << "," << g[i].accum << "," << g[i].source;
        if (g[i].source != CORR_SRC_SAMPLES) os << "," << g[i].n_atoms;
    }
    return os.str();
}

static bool parse_int(const std::string &line, const char *field, int *out)
{
    const std::string pat = std::string("\"") + field + "\":";
    const size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    *out = std::atoi(line.c_str() + p + pat.size());
    return true;
}

bool tune_cache_lookup(const std::string &path, const std::string &key, corr_tuning *out)
{
    if (path.empty()) return false;
    std::ifstream f(path);
    if (!f) return false;
    const std::string want = "\"key\":\"" + key + "\"";
    std::string line;
    bool found = false;
    corr_tuning t{};
    while (std::getline(f, line)) {
        if (line.find(want) == std::string::npos) continue;
        corr_tuning c{};
        if (parse_int(line, "tile_channels", &c.tile_channels) &&
            parse_int(line, "chans_per_thread", &c.chans_per_thread) &&
            parse_int(line, "lag_chunk", &c.lag_chunk) &&
            parse_int(line, "grid_blocks", &c.grid_blocks)) {
            if (!parse_int(line, "overlap_producers", &c.overlap_producers)) c.overlap_producers = 0;
            if (!parse_int(line, "fold_block", &c.fold_block)) c.fold_block = 0;
            if (!parse_int(line, "fold_threads", &c.fold_threads)) c.fold_threads = 0;
            t = c; // the last entry for a key wins
            found = true;
        }
    }
    if (found) *out = t;
    return found;
}

static void tune_cache_store(const std::string &path, const std::string &key, const corr_tuning &t,
                             double ms_per_push)
{
    if (path.empty()) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    f << "{\"key\":\"" << key << "\",\"tile_channels\":" << t.tile_channels
      << ",\"chans_per_thread\":" << t.chans_per_thread << ",\"lag_chunk\":" << t.lag_chunk
      << ",\"grid_blocks\":" << t.grid_blocks << ",\"overlap_producers\":" << t.overlap_producers
      << ",\"fold_block\":" << t.fold_block << ",\"fold_threads\":" << t.fold_threads
      << ",\"ms_per_push\":" << ms_per_push << "}\n";
}

} // namespace corr

using namespace corr;

extern "C" int corr_autotune(const corr_group_desc *groups, int32_t n_groups, int32_t device,
                             void *stream, uint32_t flags, const char *cache_path,
                             int64_t max_trial_channels, int32_t force, corr_tuning *out)
{
    if (!groups || n_groups < 1 || !out) return CORR_E_INVALID;
    const std::string path = tune_cache_path(cache_path);
    const std::string key = tune_key(groups, n_groups, flags, device);
    if (!force && tune_cache_lookup(path, key, out)) return CORR_OK;

    if (max_trial_channels <= 0) max_trial_channels = 8 << 20;
    std::vector<corr_group_desc> trial(groups, groups + n_groups);
    for (auto &g : trial) {
        if (g.source != CORR_SRC_SAMPLES)
            g.n_atoms = std::min<int64_t>(g.n_atoms, 1 << 18);
        else
            g.n_channels = std::min<int64_t>(g.n_channels, max_trial_channels);
    }
    static const corr_tuning cands[] = {
        {256, 1, 8, 2048}, {256, 1, 16, 0},  {512, 2, 8, 2048}, {512, 2, 8, 0},
        {512, 2, 4, 2048}, {256, 2, 8, 2048}, {1024, 4, 4, 2048}, {1024, 4, 4, 0},
        {512, 4, 4, 2048},
    };
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return CORR_E_DEVICE;
    }
    const int period = kDeferT; // whole flush periods of the block-deferred form
    // Channels up to which the issue-order trials run a group at full size.
    constexpr int64_t kOrderTrialChannels = int64_t(32) << 20;
    // ms for 2 periods of pushes after one period of warm-up, or < 0
    auto trial_ms_on = [&](const std::vector<corr_group_desc> &descs,
                           const corr_tuning &cand) -> double {
        corr_ctx *ctx = nullptr;
        const uint32_t tflags = flags & ~(uint32_t)CORR_FLAG_TIMING;
        if (corr_create(descs.data(), n_groups, device, stream, tflags, &cand, &ctx) != CORR_OK)
            return -1.0; // e.g. out of memory for this layout
        bool ok = true;
        for (int s = 0; s < period && ok; ++s) ok = corr_push(ctx, nullptr) == CORR_OK;
        ok = ok && hipEventRecord(e0, st) == hipSuccess;
        for (int s = 0; s < 2 * period && ok; ++s) ok = corr_push(ctx, nullptr) == CORR_OK;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.f;
        if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        corr_destroy(ctx);
        return ok ? (double)ms : -1.0;
    };
    auto trial_ms = [&](const corr_tuning &cand) { return trial_ms_on(trial, cand); };
    double best = 1e300;
    corr_tuning best_t{};
    for (const corr_tuning &cand : cands) {
        const double ms = trial_ms(cand);
        if (ms >= 0.0 && ms < best) {
            best = ms;
            best_t = cand;
        }
    }
    // With the best shape, choose the issue order: everything on one stream,
    // the producers (next to sample-fed groups) on a side stream, or the
    // per-step pushes beside the flush of block-deferred groups.  Which wins
    // depends on the balance of the concurrent kernels, so these trials keep
    // it: every sample-fed group and every producer's atom count are scaled
    // by one factor (groups up to kOrderTrialChannels channels run at full
    // size).  The trial timing covers every stream (the events bracket whole
    // pushes).
    bool producer = false, sampled = false, folded = false;
    int64_t n_max = 0;
    for (int i = 0; i < n_groups; ++i) {
        (groups[i].source == CORR_SRC_SAMPLES ? sampled : producer) = true;
        if (groups[i].source == CORR_SRC_SAMPLES) n_max = std::max<int64_t>(n_max, groups[i].n_channels);
        // groups the library folds in blocks (single-precision real samples,
        // p = 16, m = 2, not pairs)
        if (!(flags & CORR_FLAG_DIRECT) && groups[i].source == CORR_SRC_SAMPLES && !groups[i].pair &&
            groups[i].dtype == CORR_F32 && groups[i].points == 16 && groups[i].m == 2)
            folded = true;
    }
    const double scale = n_max > kOrderTrialChannels ? (double)kOrderTrialChannels / (double)n_max : 1.0;
    std::vector<corr_group_desc> order(groups, groups + n_groups);
    for (auto &g : order) {
        if (g.source != CORR_SRC_SAMPLES)
            g.n_atoms = std::max<int64_t>(std::min<int64_t>(g.n_atoms, 1024),
                                          (int64_t)(scale * (double)g.n_atoms));
        else
            g.n_channels = std::max<int64_t>(1, (int64_t)(scale * (double)g.n_channels));
    }
    if (best < 1e300 && n_groups >= 2) {
        double best_o = 1e300;
        corr_tuning best_o_t = best_t;
        for (int mode = 0; mode <= 2; ++mode) {
            if (mode == 1 && !(producer && sampled)) continue;
            corr_tuning ov = best_t;
            ov.overlap_producers = mode;
            const double ms = trial_ms_on(order, ov);
            if (ms >= 0.0 && ms < best_o) {
                best_o = ms;
                best_o_t = ov;
            }
        }
        if (best_o < 1e300) best_t = best_o_t;
    }
    // Then the fold kernel of the block-deferred groups, in the chosen issue
    // order: threads per block, and the shorter block (more bytes per push, a
    // smaller ring).  How the fold shares the chip with what that order runs
    // beside it does not scale down with the channel count (on scaled trials
    // 64-thread folds won and were slower at full size), so these trials run
    // the groups at full size when that fits, else on the balanced trials;
    // another shape replaces the default (256-push blocks, 128 threads) only
    // when it is at least 2% faster.
    if (best < 1e300 && folded) {
        static const int32_t fold_shapes[][2] = {{256, 128}, {256, 64}, {256, 256},
                                                 {128, 128}, {128, 64}, {128, 256}};
        std::vector<corr_group_desc> full(groups, groups + n_groups);
        double best_f = 1e300, base_f = -1.0;
        corr_tuning best_f_t = best_t;
        const std::vector<corr_group_desc> *fdescs = &full;
        for (const auto &fs : fold_shapes) {
            corr_tuning ft = best_t;
            ft.fold_block = fs[0];
            ft.fold_threads = fs[1];
            double ms = trial_ms_on(*fdescs, ft);
            if (ms < 0.0 && fdescs == &full && base_f < 0.0) { // full size does not fit
                fdescs = &order;
                ms = trial_ms_on(*fdescs, ft);
            }
            if (fs[0] == kDeferT && fs[1] == kFoldThreadsDefault) base_f = ms;
            if (ms >= 0.0 && ms < best_f) {
                best_f = ms;
                best_f_t = ft;
            }
        }
        if (best_f < 1e300) {
            if (base_f >= 0.0 && best_f > 0.98 * base_f) {
                best_f_t.fold_block = kDeferT;
                best_f_t.fold_threads = kFoldThreadsDefault;
            }
            // the block length only when the full-size state fits with it
            // (corr_create falls back to the shorter block by itself)
            if (best_f_t.fold_block == kDeferT) best_f_t.fold_block = 0;
            best_t = best_f_t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best == 1e300) return CORR_E_DEVICE;
    *out = best_t;
    tune_cache_store(path, key, best_t, best / (2 * period));
    return CORR_OK;
}
