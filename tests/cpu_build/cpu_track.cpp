// CPU build of the tracker's per-lane state machine (test infrastructure):
// gt_device.h compiled for the host with one-lane wave stand-ins, driven
// the way the persistent and batched kernels drive it, on geometries made
// by the real host preprocessor.  Tables are read in place (staging kind 0)
// or from a copy in an emulated LDS buffer made from the staging plan.
#include <vector>

#include "gt_internal.h"
#include "shim.h"
#include "gt_device.h"

namespace gt {
namespace {

constexpr size_t kLdsEmuBytes = 160 * 1024;
thread_local unsigned char g_lds[kLdsEmuBytes];
thread_local uint32_t g_cache_k = kTallyCacheMax;   // tally-cache entries of the lane (0 = off)
// The surface set the lane's code is compiled for: the geometry's own (as the
// library picks it), unless a test forces the build for every type.
thread_local int g_surf = SF_ALL;
thread_local int g_force_surf = -1;

template <int PREC, int KIND, bool MESH, typename Queue, int TRK, int SHAPE, int SF>
void run_lane_s(const Dev &dev, const StagePlan &sp, const KParams &p0, const KOut &o, const Queue &q,
                uint64_t *counts) {
    static thread_local uint32_t cells[GT_MAX_LEVELS];
    static thread_local uint32_t ctl[1 + kBlockP / 64];
    static thread_local uint64_t c_lo[kTallyCacheMax], c_hi[kTallyCacheMax];
    static thread_local uint32_t c_tag[kTallyCacheMax];
    blockDim.x = 1;
    threadIdx.x = 0;
    if (KIND != SK_NONE) stage_copy(sp, (const unsigned char *)dev.coef, g_lds);
    const auto v = make_view<KIND, SF>(dev, sp, g_lds);
    KParams p = p0;
    p.refill_min = 1;   // a one-lane wave refills as soon as its lane is idle
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const TailCfg tc = {nullptr, ctl, 0, kTailRound, 0, 0};
    const TallyCache tcache = {c_lo, c_hi, c_tag, g_cache_k, 1};
    track_pool<PREC, false, MESH, TRK, SHAPE>(v, p, o, o.tally_ws, cells, q, cnt, tc, tcache);
    counts[GT_CNT_ESCAPED] += cnt.escaped;
    counts[GT_CNT_CAPPED] += cnt.capped;
    counts[GT_CNT_LOST] += cnt.lost;
    counts[GT_CNT_SEGCAP] += cnt.segcap;
    counts[GT_CNT_REC_OVERFLOW] += cnt.recovf;
    counts[GT_CNT_SEGMENTS] += cnt.segments;
    counts[GT_CNT_REJECTED] += cnt.rejected;
}

template <int PREC, int KIND, bool MESH, typename Queue, int TRK = TRK_ST, int SHAPE = 0>
void run_lane(const Dev &dev, const StagePlan &sp, const KParams &p0, const KOut &o, const Queue &q, uint64_t *counts) {
    if (g_surf == SF_AXCZ) run_lane_s<PREC, KIND, MESH, Queue, TRK, SHAPE, SF_AXCZ>(dev, sp, p0, o, q, counts);
    else if (g_surf == SF_VERT) run_lane_s<PREC, KIND, MESH, Queue, TRK, SHAPE, SF_VERT>(dev, sp, p0, o, q, counts);
    else run_lane_s<PREC, KIND, MESH, Queue, TRK, SHAPE, SF_ALL>(dev, sp, p0, o, q, counts);
}

int surf_of(const gt_geometry *g) { return g_force_surf >= 0 ? g_force_surf : (int)g->surf_set; }

template <int PREC, bool MESH = false, typename Queue>
int run_kind(int kind, const Dev &dev, const StagePlan &sp, const KParams &p, const KOut &o, const Queue &q,
             uint64_t *counts) {
    if (kind != SK_NONE && sp.total > sizeof(g_lds)) return GT_ECAPACITY;
    switch (kind) {
    case SK_ALL: run_lane<PREC, SK_ALL, MESH>(dev, sp, p, o, q, counts); break;
    case SK_LDS: run_lane<PREC, SK_LDS, MESH>(dev, sp, p, o, q, counts); break;
    case SK_SPLIT: run_lane<PREC, SK_SPLIT, MESH>(dev, sp, p, o, q, counts); break;
    default: run_lane<PREC, SK_NONE, MESH>(dev, sp, p, o, q, counts); break;
    }
    return GT_OK;
}

template <int PREC, int TRK, int SHAPE>
int run_kind_trk(int kind, const Dev &dev, const StagePlan &sp, const KParams &p, const KOut &o,
                 const GlobalQueue &q, uint64_t *counts) {
    if (kind != SK_NONE && sp.total > sizeof(g_lds)) return GT_ECAPACITY;
    switch (kind) {
    case SK_ALL: run_lane<PREC, SK_ALL, false, GlobalQueue, TRK, SHAPE>(dev, sp, p, o, q, counts); break;
    case SK_LDS: run_lane<PREC, SK_LDS, false, GlobalQueue, TRK, SHAPE>(dev, sp, p, o, q, counts); break;
    case SK_SPLIT: run_lane<PREC, SK_SPLIT, false, GlobalQueue, TRK, SHAPE>(dev, sp, p, o, q, counts); break;
    default: run_lane<PREC, SK_NONE, false, GlobalQueue, TRK, SHAPE>(dev, sp, p, o, q, counts); break;
    }
    return GT_OK;
}

void fold_all(const uint64_t *ws, uint64_t *tfx, double *tally, uint64_t n, bool acc) {
    for (uint64_t i = 0; i < n; i++) fold_tally(ws, tfx, tally, n, i, acc);
}

}  // namespace
}  // namespace gt

using namespace gt;

// gt_track on the CPU: the histories of `p` through one lane with the
// geometry's tables held the way staging kind `kind` holds them (0..3; the
// geometry's own kind or 0).  Outputs as gt_track's, in host memory.
extern "C" int cpu_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, int kind) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    const StagePlan &sp = g->stage[p->precision];
    if (kind != SK_NONE && kind != (int)sp.kind) return set_error("cpu_track: the geometry has another staging kind"), GT_EINVAL;
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    g_cache_k = (p->flags & GT_FLAG_NO_TALLY_CACHE) ? 0 : kTallyCacheMax;
    g_surf = p->source == 1 ? SF_ALL : surf_of(g);   // the ray source: the general build only
    std::memset(ko.tally_ws, 0, (size_t)tally_replicas(g->n_inst) * 4 * 8 * g->n_inst);
    std::memset(o->counters, 0, 8 * sizeof(uint64_t));
    if (o->rec) for (uint64_t i = 0; i < (uint64_t)kp.rec_k * kp.rec_cap; i++) o->rec[i] = -1;
    unsigned long long ctr = 0;
    const GlobalQueue q = {&ctr, kp.n};
    rc = p->precision == GT_PREC_MIXED ? run_kind<GT_PREC_MIXED>(kind, g->dev, sp, kp, ko, q, o->counters)
                                       : run_kind<GT_PREC_FP64>(kind, g->dev, sp, kp, ko, q, o->counters);
    if (rc) return rc;
    fold_all(ko.tally_ws, o->tally_fx, o->tally, g->n_inst, (p->flags & GT_FLAG_ACCUMULATE) != 0);
    return GT_OK;
}

// gt_track with GT_FLAG_TRACKER_SP or GT_FLAG_TRACKER_RTK on the CPU: the
// per-kind trackers' state machine through one lane, tables held as the
// plan with the universe-kind tables holds them (staging kind `kind`: that
// plan's kind or 0).
extern "C" int cpu_track_kinds(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, int kind) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    const bool rtk = (p->flags & GT_FLAG_TRACKER_RTK) != 0;
    if (!rtk && !(p->flags & GT_FLAG_TRACKER_SP)) return set_error("cpu_track_kinds: no tracker flag"), GT_EINVAL;
    const int prec = rtk ? GT_PREC_FP64 : (int)p->precision;
    const StagePlan &sp = g->stage_arr[prec];
    if (kind != SK_NONE && kind != (int)sp.kind) return set_error("cpu_track_kinds: another staging kind"), GT_EINVAL;
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    g_cache_k = (p->flags & GT_FLAG_NO_TALLY_CACHE) ? 0 : kTallyCacheMax;
    g_surf = p->source == 1 ? SF_ALL : surf_of(g);   // the ray source: the general build only
    std::memset(ko.tally_ws, 0, (size_t)tally_replicas(g->n_inst) * 4 * 8 * g->n_inst);
    std::memset(o->counters, 0, 8 * sizeof(uint64_t));
    if (o->rec) for (uint64_t i = 0; i < (uint64_t)kp.rec_k * kp.rec_cap; i++) o->rec[i] = -1;
    unsigned long long ctr = 0;
    const GlobalQueue q = {&ctr, kp.n};
    if (!rtk)
        rc = prec == GT_PREC_MIXED ? run_kind_trk<GT_PREC_MIXED, TRK_SP, 0>(kind, g->dev, sp, kp, ko, q, o->counters)
                                   : run_kind_trk<GT_PREC_FP64, TRK_SP, 0>(kind, g->dev, sp, kp, ko, q, o->counters);
    else switch (g->rtk_shape) {
        case 1: rc = run_kind_trk<GT_PREC_FP64, TRK_RTK, 1>(kind, g->dev, sp, kp, ko, q, o->counters); break;
        case 3: rc = run_kind_trk<GT_PREC_FP64, TRK_RTK, 3>(kind, g->dev, sp, kp, ko, q, o->counters); break;
        case 5: rc = run_kind_trk<GT_PREC_FP64, TRK_RTK, 5>(kind, g->dev, sp, kp, ko, q, o->counters); break;
        case 7: rc = run_kind_trk<GT_PREC_FP64, TRK_RTK, 7>(kind, g->dev, sp, kp, ko, q, o->counters); break;
        default: return set_error("cpu_track_kinds: not of the fixed-depth shape"), GT_EINVAL;
        }
    if (rc) return rc;
    fold_all(ko.tally_ws, o->tally_fx, o->tally, g->n_inst, (p->flags & GT_FLAG_ACCUMULATE) != 0);
    return GT_OK;
}

// The mesh walk's bin index (reciprocal fast path with the division as the
// fallback) for n coordinates, for a test against floor(d / w).
extern "C" void cpu_mesh_floor(const double *d, uint64_t n, double w, double *out) {
    const double iw = 1.0 / w;
    for (uint64_t i = 0; i < n; i++) out[i] = mesh_floor(d[i], w, iw);
}

// The kernel's mesh walk over n_seg given segments (p0, u and l as in
// tracking, 3 doubles a point or direction), through one lane's register
// accumulator into one replica of the limb counters, folded into mesh_fx
// ([bins, 2] u64); for a test against the oracle's mesh tally.
extern "C" int cpu_mesh_segments(const double *lo, const double *hi, const uint32_t *n, uint64_t n_seg,
                                 const double *p0, const double *u, const double *l, uint64_t *mesh_fx) {
    MeshDesc md;
    for (int a = 0; a < 3; a++) {
        if (n[a] < 1) return GT_EINVAL;
        md.lo[a] = lo[a];
        md.w[a] = (hi[a] - lo[a]) / (double)n[a];
        md.iw[a] = 1.0 / md.w[a];
        md.n[a] = n[a];
    }
    md.nb = (uint64_t)n[0] * n[1] * n[2];
    std::vector<uint64_t> ws((size_t)tally_replicas(md.nb) * 4 * md.nb, 0);
    md.ws = ws.data();
    TallyAcc acc = {kNone, 0, 0};
    for (uint64_t i = 0; i < n_seg; i++) mesh_segment(md, md.ws, acc, p0 + 3 * i, u + 3 * i, l[i]);
    tally_flush(md.ws, acc);
    std::vector<double> sums(md.nb);
    fold_all(md.ws, mesh_fx, sums.data(), md.nb, false);
    return GT_OK;
}

// gt_track_mesh on the CPU: cpu_track with the mesh tally (the kernel's
// mesh walk), host pointers throughout; the workspace holds the replicas.
extern "C" int cpu_track_mesh(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o,
                              const gt_mesh *m, int kind) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    const StagePlan &sp = g->stage[p->precision];
    if (kind != SK_NONE && kind != (int)sp.kind) return set_error("cpu_track_mesh: another staging kind"), GT_EINVAL;
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    MeshDesc &md = ko.mesh;
    for (int a = 0; a < 3; a++) {
        md.lo[a] = m->lo[a];
        md.w[a] = (m->hi[a] - m->lo[a]) / (double)m->n[a];
        md.iw[a] = 1.0 / md.w[a];
        md.n[a] = m->n[a];
    }
    md.nb = (uint64_t)m->n[0] * m->n[1] * m->n[2];
    md.ws = (uint64_t *)m->workspace;
    if (m->workspace_bytes < gt_mesh_workspace_bytes(md.nb)) return set_error("cpu_track_mesh: workspace"), GT_EINVAL;
    std::memset(md.ws, 0, (size_t)tally_replicas(md.nb) * 4 * 8 * md.nb);
    g_cache_k = kTallyCacheMax;
    g_surf = p->source == 1 ? SF_ALL : surf_of(g);   // the ray source: the general build only
    std::memset(ko.tally_ws, 0, (size_t)tally_replicas(g->n_inst) * 4 * 8 * g->n_inst);
    std::memset(o->counters, 0, 8 * sizeof(uint64_t));
    if (o->rec) for (uint64_t i = 0; i < (uint64_t)kp.rec_k * kp.rec_cap; i++) o->rec[i] = -1;
    unsigned long long ctr = 0;
    const GlobalQueue q = {&ctr, kp.n};
    rc = p->precision == GT_PREC_MIXED ? run_kind<GT_PREC_MIXED, true>(kind, g->dev, sp, kp, ko, q, o->counters)
                                       : run_kind<GT_PREC_FP64, true>(kind, g->dev, sp, kp, ko, q, o->counters);
    if (rc) return rc;
    fold_all(ko.tally_ws, o->tally_fx, o->tally, g->n_inst, (p->flags & GT_FLAG_ACCUMULATE) != 0);
    fold_all(md.ws, m->mesh_fx, m->mesh, md.nb, (p->flags & GT_FLAG_ACCUMULATE) != 0);
    return GT_OK;
}

// gt_track_event on the CPU: the event-based schedule's steps (birth, then
// per iteration distance, move and cross over every history of the bank)
// run one history at a time in host memory, tables read in place.
template <int PREC>
static int cpu_event_t(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o) {
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    std::vector<unsigned char> mem(ev_layout(kp.n, nullptr, nullptr) + 256);
    unsigned char *base = (unsigned char *)(((uintptr_t)mem.data() + 255) & ~(uintptr_t)255);
    EvBank b;
    ev_layout(kp.n, base, &b);
    std::memset(ko.tally_ws, 0, (size_t)tally_replicas(g->n_inst) * 4 * 8 * g->n_inst);
    std::memset(o->counters, 0, 8 * sizeof(uint64_t));
    if (o->rec) for (uint64_t i = 0; i < (uint64_t)kp.rec_k * kp.rec_cap; i++) o->rec[i] = -1;
    blockDim.x = 1;
    threadIdx.x = 0;
    const DevGlobal v = global_view(g->dev);
    uint32_t cells[GT_MAX_LEVELS];
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    uint64_t *rep = ko.tally_ws;
    for (uint64_t i = 0; i < kp.n; i++) ev_birth<PREC>(v, kp, ko, b, rep, i, cells, cnt);
    for (uint64_t it = 0, alive = kp.n; alive; it++) {
        if (it > (uint64_t)kp.max_segs + 1) return set_error("cpu_track_event: histories left"), GT_EHIP;
        for (uint64_t i = 0; i < kp.n; i++) ev_distance(v, kp.n, b, i, cells);
        for (uint64_t i = 0; i < kp.n; i++) ev_move(kp, ko, b, rep, i, cnt);
        alive = 0;
        for (uint64_t i = 0; i < kp.n; i++) alive += ev_cross<PREC>(v, kp, ko, b, rep, i, cells, cnt) ? 1 : 0;
    }
    uint64_t *c = o->counters;
    c[GT_CNT_ESCAPED] += cnt.escaped;
    c[GT_CNT_CAPPED] += cnt.capped;
    c[GT_CNT_LOST] += cnt.lost;
    c[GT_CNT_SEGCAP] += cnt.segcap;
    c[GT_CNT_REC_OVERFLOW] += cnt.recovf;
    c[GT_CNT_SEGMENTS] += cnt.segments;
    c[GT_CNT_REJECTED] += cnt.rejected;
    fold_all(ko.tally_ws, o->tally_fx, o->tally, g->n_inst, (p->flags & GT_FLAG_ACCUMULATE) != 0);
    return GT_OK;
}

extern "C" int cpu_track_event(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    return p->precision == GT_PREC_MIXED ? cpu_event_t<GT_PREC_MIXED>(g, p, o) : cpu_event_t<GT_PREC_FP64>(g, p, o);
}

// The surface set of the lane's code for later calls: -1 (the default) the
// geometry's own, as the library picks it; 0, 1 or 2 forces SF_ALL, SF_AXCZ or
// SF_VERT.
extern "C" void cpu_force_surface_set(int sf) { g_force_surf = sf; }

// gt_track_batch on the CPU: gt_batch_create's descriptors (in host memory)
// executed the way gt_batch_launch executes them -- the fill list, then the
// chunk groups by staging kind (3, 2, 1, 0) each chunk through one lane with
// its item's tables, then the finalize list.  *n_chunks gets the number of
// chunks run.  With whole items (chunk = 0) each kind's item group is run
// by `groups` one-lane workgroups: all of them make their first choice
// (pick_item), then each in turn runs visits (draining its item's counter)
// and chooses again until no item has histories left; *n_chunks then gets
// the number of visits.
extern "C" int cpu_track_batch(const gt_batch_item *items, uint32_t n_items, const gt_tuning *tuning,
                               uint32_t *n_chunks, uint32_t groups) {
    gt_batch *b = nullptr;
    int rc = gt_batch_create(items, n_items, tuning, &b);
    if (rc) return rc;
    for (uint32_t f = 0; f < b->n_fill; f++) {
        const FillRange &r = b->d_fill[f];
        for (uint64_t i = 0; i < r.count; i++) {
            if (r.bytes == 8) ((uint64_t *)r.ptr)[i] = r.value;
            else ((uint32_t *)r.ptr)[i] = (uint32_t)r.value;
        }
    }
    g_cache_k = b->cache ? kTallyCacheMax : 0;
    g_surf = SF_ALL;   // batches run the build for every surface type
    uint32_t first = 0, ran = 0;
    if (b->by_item) {
        if (groups == 0) {
            set_error("cpu_track_batch: no workgroups");
            gt_batch_destroy(b);
            return GT_EINVAL;
        }
        uint32_t first_slot = 0;
        std::vector<uint32_t> pick(groups);
        float rs[1];
        uint32_t ri[1];
        for (int kind = 3; kind >= 0 && !rc; kind--) {
            const uint32_t ns = b->n_slot_kind[kind];
            const BatchSlot *sl = b->d_slots + first_slot;
            first_slot += ns;
            if (!ns) continue;
            gridDim.x = groups;
            for (uint32_t w = 0; w < groups; w++) {
                blockIdx.x = w;
                pick_item(sl, ns, b->d_claimed, b->d_workers, true, rs, ri, &pick[w]);
            }
            for (uint32_t w = 0; w < groups && !rc; w++) {
                blockIdx.x = w;
                while (pick[w] != kNoItem && !rc) {
                    const uint32_t item = pick[w];
                    if (item >= b->n_items) {
                        set_error("cpu_track_batch: a choice names item %u", item);
                        rc = GT_EINVAL;
                        break;
                    }
                    const BatchItem &it = b->d_items[item];
                    const ChunkQueue q = {&b->d_claimed[item], 0, it.p.n};
                    rc = b->precision == GT_PREC_MIXED
                             ? run_kind<GT_PREC_MIXED>(kind, it.dev, it.plan, it.p, it.o, q, it.o.counters)
                             : run_kind<GT_PREC_FP64>(kind, it.dev, it.plan, it.p, it.o, q, it.o.counters);
                    b->d_workers[item] -= 1;
                    ran++;
                    pick_item(sl, ns, b->d_claimed, b->d_workers, false, rs, ri, &pick[w]);
                }
            }
            blockIdx.x = 0;
            gridDim.x = 1;
            for (uint32_t s = 0; s < ns && !rc; s++)
                if (b->d_workers[sl[s].item] != 0 || b->d_claimed[sl[s].item] < sl[s].n) {
                    set_error("cpu_track_batch: item %u left with workers or unclaimed histories", sl[s].item);
                    rc = GT_EINVAL;
                }
        }
        if (!rc && first_slot != b->n_slots) {
            set_error("cpu_track_batch: item groups do not cover the items");
            rc = GT_EINVAL;
        }
    }
    for (int kind = 3; kind >= 0 && !rc && !b->by_item; kind--) {
        for (uint32_t c = first; c < first + b->n_kind[kind] && !rc; c++) {
            const BatchChunk &ch = b->d_chunks[c];
            if (ch.item >= b->n_items) {
                set_error("cpu_track_batch: chunk %u names item %u", c, ch.item);
                rc = GT_EINVAL;
                break;
            }
            const BatchItem &it = b->d_items[ch.item];
            unsigned long long pool = 0;
            const ChunkQueue q = {&pool, ch.first, ch.first + ch.count};
            rc = b->precision == GT_PREC_MIXED ? run_kind<GT_PREC_MIXED>(kind, it.dev, it.plan, it.p, it.o, q, it.o.counters)
                                               : run_kind<GT_PREC_FP64>(kind, it.dev, it.plan, it.p, it.o, q, it.o.counters);
            ran++;
        }
        first += b->n_kind[kind];
    }
    if (!rc && !b->by_item && (first != b->n_chunks || ran != b->n_chunks)) {
        set_error("cpu_track_batch: chunk groups do not cover the chunks");
        rc = GT_EINVAL;
    }
    if (!rc)
        for (uint32_t i = 0; i < b->n_items; i++) {
            const FinalizeItem &f = b->d_fin[i];
            fold_all(f.ws, f.tfx, f.tally, f.n_inst, f.accumulate != 0);
        }
    if (n_chunks) *n_chunks = ran;
    gt_batch_destroy(b);
    return rc;
}
