// Launch-shape autotuning for the persistent trackers.  The shape (threads
// per workgroup, idle lanes before a wave refills, histories per batch
// chunk, the regroup interval, histories a wave claims at once -- the
// particles per wavefront) changes only the speed: every shape gives the
// same outputs.  The
// tuner times the candidate shapes with HIP events on the caller's stream
// and keeps the winner in a process-wide cache, which gt_batch_create reads
// when it is given no tuning.
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "gt_internal.h"

using namespace gt;

namespace {

std::mutex g_tune_mu;
std::map<uint64_t, gt_tuning> g_track_cache, g_batch_cache;

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h * 0xff51afd7ed558ccdull;
}

unsigned log2_ceil(uint64_t n) {
    unsigned k = 0;
    while (k < 63 && (1ull << k) < n) k++;
    return k;
}

uint64_t track_key(const gt_geometry *g, const gt_track_params *p) {
    uint64_t h = mix(0, (uint64_t)(uintptr_t)g);
    h = mix(h, p->precision);
    h = mix(h, p->flags & (GT_FLAG_NO_STAGING | GT_FLAG_TAIL_COMPACTION));
    return mix(h, log2_ceil(p->n_particles));
}

uint64_t batch_key(const gt_batch_item *items, uint32_t n) {
    uint64_t h = mix(0, n);
    for (uint32_t i = 0; i < n; i++) {
        h = mix(h, (uint64_t)(uintptr_t)items[i].geometry);
        h = mix(h, items[i].params.n_particles);
        h = mix(h, items[i].params.precision);
    }
    return h;
}

// Elapsed milliseconds of `reps` calls of launch() after one untimed call.
template <typename F>
int time_launches(F launch, uint32_t reps, hipStream_t st, float *ms) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        return set_error("hipEventCreate failed"), GT_EHIP;
    }
    int rc = launch();
    if (!rc) rc = hipEventRecord(a, st) == hipSuccess ? GT_OK : (set_error("hipEventRecord failed"), GT_EHIP);
    for (uint32_t r = 0; r < reps && !rc; r++) rc = launch();
    if (!rc) rc = hipEventRecord(b, st) == hipSuccess ? GT_OK : (set_error("hipEventRecord failed"), GT_EHIP);
    if (!rc && hipEventSynchronize(b) != hipSuccess) rc = (set_error("hipEventSynchronize failed"), GT_EHIP);
    if (!rc && hipEventElapsedTime(ms, a, b) != hipSuccess) rc = (set_error("hipEventElapsedTime failed"), GT_EHIP);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

const uint32_t kBlocks[] = {256, 512, 640, 1024};
const uint32_t kRefills[] = {1, 4, 8, 16};
const uint64_t kChunks[] = {0, 1024, 4096, 16384};   // 0: workgroups join whole items
const uint32_t kRegroups[] = {16, 64, 256};   // second stage, at the fastest shape of the first
const uint32_t kWaveTakes[] = {128, 256};     // third stage: histories a wave claims at once (64 is the
                                              // default the first two stages ran with)

}  // namespace

extern "C" int gt_autotune_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o,
                                 uint32_t reps, void *stream, gt_tuning *best, float *best_ms) {
    if (!best) return set_error("gt_autotune_track: best is NULL"), GT_EINVAL;
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    if (p->flags & GT_FLAG_LANE_PER_HISTORY)
        return set_error("gt_autotune_track: the one-history-per-lane schedule has no shape to tune"), GT_EINVAL;
    if (reps < 1) reps = 1;
    const hipStream_t st = (hipStream_t)stream;
    gt_tuning win = {0, 0, 0, 0, 0};
    float win_ms = 0;
    bool any = false;
    auto trial = [&](const gt_tuning &t) {
        gt_track_params q = *p;
        q.block_size = t.block_size;
        q.refill_min = t.refill_min;
        q.regroup_every = t.regroup_every;
        q.wave_histories = t.wave_histories;
        float ms = 0;
        const int r = time_launches([&] { return launch_track(g, &q, o, stream); }, reps, st, &ms);
        if (!r && (!any || ms < win_ms)) {
            win = t;
            win_ms = ms;
            any = true;
        }
        return r;
    };
    for (uint32_t b : kBlocks)
        for (uint32_t r : kRefills)
            if ((rc = trial({b, r, 0, 0, 0}))) return rc;
    const gt_tuning shape = win;
    for (uint32_t rg : kRegroups)
        if ((rc = trial({shape.block_size, shape.refill_min, 0, rg, 0}))) return rc;
    const gt_tuning shape2 = win;
    for (uint32_t wt : kWaveTakes)
        if ((rc = trial({shape2.block_size, shape2.refill_min, 0, shape2.regroup_every, wt}))) return rc;
    // leave the outputs of the caller's own parameters with the chosen shape
    gt_track_params q = *p;
    q.block_size = win.block_size;
    q.refill_min = win.refill_min;
    q.regroup_every = win.regroup_every;
    q.wave_histories = win.wave_histories;
    rc = launch_track(g, &q, o, stream);
    if (rc) return rc;
    *best = win;
    if (best_ms) *best_ms = win_ms / (float)reps;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_track_cache[track_key(g, p)] = win;
    return GT_OK;
}

extern "C" int gt_tuning_lookup(const gt_geometry *g, const gt_track_params *p, gt_tuning *out) {
    if (!g || !p || !out) return set_error("gt_tuning_lookup: null argument"), GT_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_track_cache.find(track_key(g, p));
    if (it == g_track_cache.end()) return 0;
    *out = it->second;
    return 1;
}

extern "C" int gt_autotune_batch(const gt_batch_item *items, uint32_t n_items, uint32_t reps, void *stream,
                                 gt_tuning *best, float *best_ms) {
    if (!best) return set_error("gt_autotune_batch: best is NULL"), GT_EINVAL;
    if (reps < 1) reps = 1;
    const hipStream_t st = (hipStream_t)stream;
    gt_tuning win = {0, 0, 0, 0, 0};
    float win_ms = 0;
    bool any = false;
    auto trial = [&](const gt_tuning &t) {
        gt_batch *bt = nullptr;
        int rc = gt_batch_create(items, n_items, &t, &bt);
        if (rc) return rc;
        float ms = 0;
        rc = time_launches([&] { return gt_batch_launch(bt, stream); }, reps, st, &ms);
        gt_batch_destroy(bt);
        if (!rc && (!any || ms < win_ms)) {
            win = t;
            win_ms = ms;
            any = true;
        }
        return rc;
    };
    // (the first stage keeps the items' own regroup setting)
    for (uint32_t b : kBlocks) {
        if (b < 512) continue;   // a workgroup runs one item at a time: keep workgroups large
        for (uint32_t r : kRefills)
            for (uint64_t c : kChunks)
                if (int rc = trial({b, r, c, 0, 0})) return rc;
    }
    const gt_tuning shape = win;
    for (uint32_t rg : kRegroups)
        if (int rc = trial({shape.block_size, shape.refill_min, shape.chunk, rg, 0})) return rc;
    const gt_tuning shape2 = win;
    for (uint32_t wt : kWaveTakes)
        if (int rc = trial({shape2.block_size, shape2.refill_min, shape2.chunk, shape2.regroup_every, wt})) return rc;
    *best = win;
    if (best_ms) *best_ms = win_ms / (float)reps;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_batch_cache[batch_key(items, n_items)] = win;
    return GT_OK;
}

// The cached tuning of this batch's items, if gt_autotune_batch has seen them.
bool gt::cached_batch_tuning(const gt_batch_item *items, uint32_t n_items, gt_tuning *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_cache.find(batch_key(items, n_items));
    if (it == g_batch_cache.end()) return false;
    *out = it->second;
    return true;
}
