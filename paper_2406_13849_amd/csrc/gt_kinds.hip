// HIP kernels of libgt for gfx950: the persistent schedule with the
// trackers that keep one tracker type per kind of universe -- the paper's
// comparison methods to the single tracker:
//   - static polymorphism (Section "Static polymorphism (SP) method"): a
//     switch on the kind of each level's universe; rectilinear arrays find
//     a cell by index and cross to the neighbour by index (Algs. 5 and 6),
//     every other universe uses the CSG tracker with its hierarchy;
//   - the fixed-depth reactor tracker (Section "RTK tracking", Algs. 9 and
//     10): the kind of every level known at compile time (an optional
//     one-cell root, one or two array levels, then pins of concentric
//     cylinders and axial planes), so its loops over levels unroll and no
//     kind or hierarchy is read.
// Scheduling, sampling, tallies and outputs are the single tracker's
// (track_pool in gt_device.h); only find_cell, cross_surface and
// distance_to_surface differ, and all three trackers give identical
// outputs.  Kept in its own translation unit so it compiles beside
// gt_track.hip.
#pragma clang fp contract(off)

#include "gt_device.h"
#include "gt_launch.h"

namespace gt {
namespace {

// KIND = staging kind of the geometry's plan with the universe-kind tables
// (stage_arr); TRK = TRK_SP or TRK_RTK; SHAPE = the fixed-depth shape (RTK);
// SF = the surface set the code handles.
template <int PREC, int KIND, int TRK, int SHAPE, int SF>
__global__ void __launch_bounds__(kBlockP) __attribute__((amdgpu_waves_per_eu(4)))
k_track_kinds(const GeomDesc *__restrict__ gd, const LaunchRec *__restrict__ lr, uint32_t tables_at,
              uint32_t tail_at, uint32_t tail_cap, uint32_t tail_round, uint32_t tail_words, uint32_t cache_at,
              uint32_t cache_k) {
    __shared__ uint32_t ctl[1 + kBlockP / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_dyn[];
    uint32_t *cells = (uint32_t *)lds_dyn;   // the cell of each level, one column per lane
    unsigned char *lds_tables = lds_dyn + tables_at;
    if (threadIdx.x == 0) ctl[0] = 0;
    if (KIND != SK_NONE) stage_copy(gd->stage_arr[PREC], (const unsigned char *)gd->dev.coef, lds_tables);
    else __syncthreads();
    const auto g = make_view<KIND, SF>(gd->dev, gd->stage_arr[PREC], lds_tables);
    const KParams &p = lr->p;
    const KOut &o = lr->o;
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const GlobalQueue q = {(unsigned long long *)&o.counters[7], p.n};
    const TailCfg tc = {(uint64_t *)(lds_dyn + tail_at), ctl, tail_cap, tail_round, tail_words, 0u};
    const TallyCache tcache = tally_cache(lds_dyn, cache_at, cache_k);
    track_pool<PREC, false, false, TRK, SHAPE>(g, p, o, rep, cells + threadIdx.x, q, cnt, tc, tcache);
    add_counts(cnt, o.counters);
}

template <int PREC, int KIND, int TRK, int SHAPE, int SF>
int launch_kinds_k(const gt_geometry *g, const LaunchRec *lr, uint64_t n, unsigned block, bool tail, bool cache,
                   hipStream_t st) {
    const unsigned tables = KIND == SK_NONE ? 0 : g->stage_arr[PREC].total;
    const void *kern = (const void *)k_track_kinds<PREC, KIND, TRK, SHAPE, SF>;
    LdsPlan lp;
    int rc = plan_persistent(kern, block, tables, tail, cache, 0, g->device, lp);
    if (rc) return rc;
    int blocks = lp.blocks;
    const uint64_t need = (n + block - 1) / block;
    if ((uint64_t)blocks > need) blocks = (int)need;
    note_launch(lp, blocks, block, KIND, SF);
    hipLaunchKernelGGL((k_track_kinds<PREC, KIND, TRK, SHAPE, SF>), dim3(blocks), dim3(block), lp.dyn, st, g->desc, lr,
                       lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound, lp.tail_words, lp.cache_at, lp.cache_k);
    return GT_OK;
}

template <int PREC, int TRK, int SHAPE, int SF>
int launch_kinds_s(const gt_geometry *g, const LaunchRec *lr, int kind, uint64_t n, unsigned block, bool tail,
                   bool cache, hipStream_t st) {
    switch (kind) {
    case SK_ALL: return launch_kinds_k<PREC, SK_ALL, TRK, SHAPE, SF>(g, lr, n, block, tail, cache, st);
    case SK_LDS: return launch_kinds_k<PREC, SK_LDS, TRK, SHAPE, SF>(g, lr, n, block, tail, cache, st);
    case SK_SPLIT: return launch_kinds_k<PREC, SK_SPLIT, TRK, SHAPE, SF>(g, lr, n, block, tail, cache, st);
    default: return launch_kinds_k<PREC, SK_NONE, TRK, SHAPE, SF>(g, lr, n, block, tail, cache, st);
    }
}

// The build for the geometry's surface set.
template <int PREC, int TRK, int SHAPE>
int launch_kinds_t(const gt_geometry *g, const LaunchRec *lr, int kind, uint64_t n, unsigned block, bool tail,
                   bool cache, bool ray, hipStream_t st) {
    switch (ray ? SF_ALL : (int)g->surf_set) {   // the ray source only in the general build
    case SF_AXCZ: return launch_kinds_s<PREC, TRK, SHAPE, SF_AXCZ>(g, lr, kind, n, block, tail, cache, st);
    case SF_VERT: return launch_kinds_s<PREC, TRK, SHAPE, SF_VERT>(g, lr, kind, n, block, tail, cache, st);
    default: return launch_kinds_s<PREC, TRK, SHAPE, SF_ALL>(g, lr, kind, n, block, tail, cache, st);
    }
}

}  // namespace

int launch_kinds(const gt_geometry *g, const LaunchRec *lr, int prec, int trk, uint64_t n, unsigned block, bool tail,
                 bool cache, bool staging, bool ray, hipStream_t st) {
    if (trk == TRK_RTK) prec = GT_PREC_FP64;
    const int kind = staging ? (int)g->stage_arr[prec].kind : SK_NONE;
    if (trk == TRK_SP)
        return prec == GT_PREC_MIXED ? launch_kinds_t<GT_PREC_MIXED, TRK_SP, 0>(g, lr, kind, n, block, tail, cache, ray, st)
                                     : launch_kinds_t<GT_PREC_FP64, TRK_SP, 0>(g, lr, kind, n, block, tail, cache, ray, st);
    // the fixed-depth tracker takes every decision by index or by the one
    // root cell's test in double precision: no precision mode applies
    switch (g->rtk_shape) {
    case 1: return launch_kinds_t<GT_PREC_FP64, TRK_RTK, 1>(g, lr, kind, n, block, tail, cache, ray, st);
    case 3: return launch_kinds_t<GT_PREC_FP64, TRK_RTK, 3>(g, lr, kind, n, block, tail, cache, ray, st);
    case 5: return launch_kinds_t<GT_PREC_FP64, TRK_RTK, 5>(g, lr, kind, n, block, tail, cache, ray, st);
    case 7: return launch_kinds_t<GT_PREC_FP64, TRK_RTK, 7>(g, lr, kind, n, block, tail, cache, ray, st);
    default: return set_error("gt_track: the geometry is not of the fixed-depth reactor shape"), GT_EINVAL;
    }
}

}  // namespace gt
