// Host-side launch helpers shared by the kernel translation units of libgt
// (gt_track.hip: the single tracker, batches, event schedule;
// gt_track_axcz.hip and gt_track_vert.hip: the single tracker's builds for
// smaller surface sets; gt_kinds.hip: the trackers that switch on universe
// kind).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "gt_internal.h"

namespace gt {

inline int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return GT_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return GT_EHIP;
}

inline unsigned grid_for(uint64_t n, unsigned block) {
    uint64_t b = (n + block - 1) / block;
    return (unsigned)(b < 1 ? 1 : (b > 0x7FFFFFFFull ? 0x7FFFFFFFull : b));
}

inline unsigned fill_grid(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// LDS of a persistent launch: the level columns, the staged tables (if any),
// the tally cache (up to kTallyCacheMax entries per lane), then the tail
// buffer (with tail compaction), as large as the workgroup's share of the
// compute unit's LDS allows without lowering the number of resident
// workgroups.
struct LdsPlan {
    unsigned dyn, tables_at, tail_at, tail_cap, tail_words, regroup, cache_at, cache_k;
    int blocks;
};

constexpr unsigned kLdsPerCU = 160 * 1024;

int persistent_grid(const void *kernel, unsigned block, unsigned dyn, int device, int *blocks);
int allow_dynamic_lds(const void *kernel, unsigned bytes);
int plan_persistent(const void *kern, unsigned block, unsigned tables, bool tail, bool cache, uint32_t regroup,
                    int device, LdsPlan &lp);
void note_launch(const LdsPlan &lp, int blocks, unsigned block, int kind, int surf);

// Events recorded around the tracking kernels of this thread's next launches
// (set by gt_set_kernel_events; both null = off).
extern thread_local hipEvent_t t_ev_start, t_ev_stop;

inline void mark(hipEvent_t e, hipStream_t st) {
    if (e) (void)hipEventRecord(e, st);
}

// The persistent tracker of a per-kind method (GT_FLAG_TRACKER_SP or
// GT_FLAG_TRACKER_RTK) for a geometry whose launch record is at lr.
int launch_kinds(const gt_geometry *g, const LaunchRec *lr, int prec, int trk, uint64_t n, unsigned block,
                 bool tail, bool cache, bool staging, bool ray, hipStream_t st);

}  // namespace gt
