// The persistent single-geometry tracker (k_track_persistent) and its
// launchers, compiled for one surface set per translation unit: gt_track.hip
// (SF_ALL), gt_track_axcz.hip (SF_AXCZ) and gt_track_vert.hip (SF_VERT) each
// include this header and define that set's launch_persistent_* below, so the
// three builds compile in parallel.  Not part of the public ABI.
#pragma once

#include "gt_device.h"
#include "gt_launch.h"

namespace gt {
namespace {

// KIND = staging kind of the geometry's plan (see make_view); W = waves per
// SIMD the register budget is cut for: 4 (up to 1024 lanes per workgroup,
// 128 registers) or 5 (640 lanes, two workgroups per compute unit, 96
// registers); SF = the surface set the code handles (SF_AXCZ, SF_VERT or
// SF_ALL; see gt_internal.h).
template <int PREC, int KIND, int W, bool RG, bool MESH, int SF>
__global__ void __launch_bounds__(W == 5 ? 640 : kBlockP) __attribute__((amdgpu_waves_per_eu(W)))
k_track_persistent(const GeomDesc *__restrict__ gd, const LaunchRec *__restrict__ lr, uint32_t tables_at,
                   uint32_t tail_at, uint32_t tail_cap, uint32_t tail_round, uint32_t tail_words, uint32_t regroup,
                   uint32_t cache_at, uint32_t cache_k) {
    __shared__ uint32_t ctl[1 + kBlockP / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_dyn[];
    uint32_t *cells = (uint32_t *)lds_dyn;   // the cell of each level, one column per lane
    unsigned char *lds_tables = lds_dyn + tables_at;
    if (threadIdx.x == 0) ctl[0] = 0;
    if (KIND != SK_NONE) stage_copy(gd->stage[PREC], (const unsigned char *)gd->dev.coef, lds_tables);
    else __syncthreads();
    const auto g = make_view<KIND, SF>(gd->dev, gd->stage[PREC], lds_tables);
    const KParams &p = lr->p;
    const KOut &o = lr->o;
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const GlobalQueue q = {(unsigned long long *)&o.counters[7], p.n};
    const TailCfg tc = {(uint64_t *)(lds_dyn + tail_at), ctl, tail_cap, tail_round, tail_words, regroup};
    const TallyCache tcache = tally_cache(lds_dyn, cache_at, cache_k);
    track_pool<PREC, RG, MESH>(g, p, o, rep, cells + threadIdx.x, q, cnt, tc, tcache);
    add_counts(cnt, o.counters);
}

// One persistent tracker launch for a geometry of staging kind KIND: the
// build with the mesh tally when there is a mesh, else the one with the
// regroup step when one is asked for and finds room, else the plain one.
template <int PREC, int KIND, int W, int SF>
int launch_persistent_k(const gt_geometry *g, const LaunchRec *lr, uint64_t n, unsigned block, bool tail, bool cache,
                        uint32_t regroup, bool mesh, hipStream_t st) {
    const unsigned tables = KIND == SK_NONE ? 0 : g->stage[PREC].total;
    const void *plain = (const void *)k_track_persistent<PREC, KIND, W, false, false, SF>;
    const void *kern = mesh ? (const void *)k_track_persistent<PREC, KIND, W, false, true, SF> : plain;
    LdsPlan lp;
    int rc = GT_OK;
    if (regroup && !mesh) {
        const void *kr = (const void *)k_track_persistent<PREC, KIND, W, true, false, SF>;
        rc = plan_persistent(kr, block, tables, tail, cache, regroup, g->device, lp);
        if (!rc && lp.regroup) kern = kr;
    }
    if (!rc && kern != (const void *)k_track_persistent<PREC, KIND, W, true, false, SF>)
        rc = plan_persistent(kern, block, tables, tail, cache, 0, g->device, lp);
    if (rc) return rc;
    int blocks = lp.blocks;
    const uint64_t need = (n + block - 1) / block;
    if ((uint64_t)blocks > need) blocks = (int)need;
    note_launch(lp, blocks, block, KIND, SF);
    if (mesh)
        hipLaunchKernelGGL((k_track_persistent<PREC, KIND, W, false, true, SF>), dim3(blocks), dim3(block), lp.dyn, st,
                           g->desc, lr, lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound, lp.tail_words, 0u,
                           lp.cache_at, lp.cache_k);
    else if (lp.regroup)
        hipLaunchKernelGGL((k_track_persistent<PREC, KIND, W, true, false, SF>), dim3(blocks), dim3(block), lp.dyn, st,
                           g->desc, lr, lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound, lp.tail_words, lp.regroup,
                           lp.cache_at, lp.cache_k);
    else
        hipLaunchKernelGGL((k_track_persistent<PREC, KIND, W, false, false, SF>), dim3(blocks), dim3(block), lp.dyn, st,
                           g->desc, lr, lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound, lp.tail_words, 0u,
                           lp.cache_at, lp.cache_k);
    return GT_OK;
}

template <int PREC, int W, int SF>
int launch_persistent_s(const gt_geometry *g, const LaunchRec *lr, int kind, uint64_t n, unsigned block, bool tail,
                        bool cache, uint32_t regroup, bool mesh, hipStream_t st) {
    switch (kind) {
    case SK_ALL: return launch_persistent_k<PREC, SK_ALL, W, SF>(g, lr, n, block, tail, cache, regroup, mesh, st);
    case SK_LDS: return launch_persistent_k<PREC, SK_LDS, W, SF>(g, lr, n, block, tail, cache, regroup, mesh, st);
    case SK_SPLIT: return launch_persistent_k<PREC, SK_SPLIT, W, SF>(g, lr, n, block, tail, cache, regroup, mesh, st);
    default: return launch_persistent_k<PREC, SK_NONE, W, SF>(g, lr, n, block, tail, cache, regroup, mesh, st);
    }
}

// Every launch of one surface set: precision and waves per SIMD chosen at run time.
template <int SF>
int launch_persistent_set(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                          unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st) {
    if (prec == GT_PREC_MIXED)
        return w == 5 ? launch_persistent_s<GT_PREC_MIXED, 5, SF>(g, lr, kind, n, block, tail, cache, regroup, mesh, st)
                      : launch_persistent_s<GT_PREC_MIXED, 4, SF>(g, lr, kind, n, block, tail, cache, regroup, mesh, st);
    return w == 5 ? launch_persistent_s<GT_PREC_FP64, 5, SF>(g, lr, kind, n, block, tail, cache, regroup, mesh, st)
                  : launch_persistent_s<GT_PREC_FP64, 4, SF>(g, lr, kind, n, block, tail, cache, regroup, mesh, st);
}

}  // namespace

// One surface set's persistent launch for a geometry whose launch record is
// at lr (w = waves per SIMD of the build: 4 or 5).
int launch_persistent_all(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                          unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st);
int launch_persistent_axcz(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                           unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st);
int launch_persistent_vert(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                           unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st);

}  // namespace gt
