// HIP kernels of libgt for gfx950 (CDNA4): Monte Carlo geometry tracking
// through nested CSG universes with one CSG tracker and per-universe
// bounding-volume hierarchies (Section "Single tracker (ST) method").
//
// Three schedules share every device function:
//   - persistent (default): one workgroup per compute unit; each wave loops
//     until the particle pool is drained, refilling finished lanes from a
//     wave-local pool of particle ids, and every lane runs a small state
//     machine whose steps (draw random numbers, search one level, one
//     segment) each have a single call site -- k_track_persistent for one
//     geometry, k_track_batch for many in one launch;
//   - k_track (GT_FLAG_LANE_PER_HISTORY): one history per lane;
//   - event-based (gt_track_event): one kernel per operation per iteration
//     over a particle bank in device memory.
// A particle's state lives in registers; the cell of each level lives in
// LDS (one column per lane) so level loops index it without spilling.  The
// persistent single-geometry trackers are built twice: for geometries of
// axis planes and z-cylinders only, and for every surface type.
//
// The device functions are in gt_device.h; this file holds the kernels and
// their host-side launchers (the trackers that switch on universe kind are
// in gt_kinds.hip).
#pragma clang fp contract(off)

#include <algorithm>
#include <mutex>
#include <new>

#include "gt_persistent.h"

namespace gt {
namespace {


template <int PREC>
__global__ void __launch_bounds__(kBlock) k_track(Dev g0, KParams p, KOut o) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t local = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (local < p.n) run_history<PREC>(g, p, o, rep, local, cells + threadIdx.x, cnt);
    add_counts(cnt, o.counters);
}

// ------------------------------------------------------------------ event-based schedule kernels
// One thread per history of the bank; the steps are in gt_device.h.
template <int PREC>
__global__ void __launch_bounds__(kBlock) k_ev_birth(Dev g0, KParams p, KOut o, EvBank b) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) ev_birth<PREC>(g, p, o, b, rep, i, cells + threadIdx.x, cnt);
    add_counts(cnt, o.counters);
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_ev_distance(Dev g0, uint64_t n, EvBank b) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ev_distance(g, n, b, i, cells + threadIdx.x);
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_ev_move(Dev g0, KParams p, KOut o, EvBank b) {
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g0.n_inst)) * 4 * g0.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n) ev_move(p, o, b, rep, i, cnt);
    add_counts(cnt, o.counters);
}

// Also counts the histories left after the iteration into *alive.
template <int PREC>
__global__ void __launch_bounds__(kBlock) k_ev_cross(Dev g0, KParams p, KOut o, EvBank b,
                                                      unsigned long long *alive) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < p.n && ev_cross<PREC>(g, p, o, b, rep, i, cells + threadIdx.x, cnt);
    const uint64_t lm = __ballot(live);
    if (__lane_id() == 0 && lm) atomicAdd(alive, (unsigned long long)__popcll(lm));
    add_counts(cnt, o.counters);
}

// Store a launch's parameters for the tracker that follows on the stream.
__global__ void k_put_launch(LaunchRec r, LaunchRec *dst) {
    if (threadIdx.x == 0) *dst = r;
}

// Many geometries in one persistent launch, in one of two ways:
//  * chunks (n_slots == 0): each workgroup takes chunks (item, range of
//    particle indices) from a device queue and runs the lanes' state machine
//    over the chunk with a workgroup-local id counter, its waves meeting at
//    the end of every chunk;
//  * whole items (n_slots > 0): each workgroup joins an item (pick_item) and
//    its waves claim the item's histories from the item's counter in device
//    memory, which the workgroups on the item share, until none is left;
//    the waves meet only when the workgroup moves to another item.
// Either way the item's tables are copied into LDS when the item changes
// (KIND).
template <int PREC, int KIND, int W, bool RG>
__global__ void __launch_bounds__(W == 5 ? 640 : kBlockP) __attribute__((amdgpu_waves_per_eu(W)))
k_track_batch(const BatchItem *__restrict__ items, const BatchChunk *__restrict__ chunks, uint32_t n_chunks,
              unsigned long long *queue, const BatchSlot *__restrict__ slots, uint32_t n_slots,
              unsigned long long *claimed, unsigned long long *workers, uint32_t tables_at, uint32_t tail_at,
              uint32_t tail_cap, uint32_t tail_round, uint32_t tail_words, uint32_t regroup, uint32_t cache_at,
              uint32_t cache_k) {
    __shared__ uint32_t ctl[1 + kBlockP / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_dyn[];
    __shared__ uint32_t s_chunk;
    __shared__ unsigned long long s_pool;
    __shared__ float red_s[kBlockP / 64];
    __shared__ uint32_t red_i[kBlockP / 64];
    uint32_t *cells = (uint32_t *)lds_dyn;   // the cell of each level, one column per lane
    unsigned char *lds_tables = lds_dyn + tables_at;
    const TailCfg tc = {(uint64_t *)(lds_dyn + tail_at), ctl, tail_cap, tail_round, tail_words, regroup};
    const TallyCache tcache = tally_cache(lds_dyn, cache_at, cache_k);
    const bool by_item = n_slots != 0;
    // the descriptors are read-only for the whole launch: their fields are
    // read where needed (scalar loads the compiler may repeat) rather than
    // carried from chunk to chunk in registers
    uint32_t cur = 0xFFFFFFFFu;
    for (bool first_visit = true;; first_visit = false) {
        if (by_item) {
            pick_item(slots, n_slots, claimed, workers, first_visit, red_s, red_i, &s_chunk);
            if (threadIdx.x == 0) ctl[0] = 0;
        } else if (threadIdx.x == 0) {
            s_chunk = (uint32_t)atomicAdd(queue, 1ull);
            s_pool = 0;
            ctl[0] = 0;
        }
        __syncthreads();
        const uint32_t c = __builtin_amdgcn_readfirstlane(s_chunk);
        if (by_item ? c == kNoItem : c >= n_chunks) break;
        const uint32_t item = by_item ? c : chunks[c].item;
        const BatchItem &it = items[item];
        if (KIND != SK_NONE && item != cur) stage_copy(it.plan, (const unsigned char *)it.dev.coef, lds_tables);
        cur = item;
        const auto g = make_view<KIND>(it.dev, it.plan, lds_tables);
        const KParams &p = it.p;
        const KOut &o = it.o;
        uint64_t *rep = o.tally_ws + (size_t)replica_id(tally_replicas(g.n_inst)) * 4 * g.n_inst;
        Counts cnt = {0, 0, 0, 0, 0, 0, 0};
        const ChunkQueue q = by_item ? ChunkQueue{&claimed[item], 0, p.n}
                                     : ChunkQueue{&s_pool, chunks[c].first, chunks[c].first + chunks[c].count};
        track_pool<PREC, RG>(g, p, o, rep, cells + threadIdx.x, q, cnt, tc, tcache);
        add_counts(cnt, o.counters);
        __syncthreads();
        if (by_item && threadIdx.x == 0) atomicAdd(&workers[item], ~0ull);   // leaves the item
    }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_fill_u64(uint64_t *a, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_fill_i32(int32_t *a, uint64_t n, int32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_finalize(const uint64_t *ws, uint64_t *tfx, double *tally, uint64_t n, int accumulate) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        fold_tally(ws, tfx, tally, n, i, accumulate != 0);
}

// One launch zeroing every range of a batch: blockIdx.y selects the range.
__global__ void k_fill_ranges(const FillRange *r) {
    const FillRange f = r[blockIdx.y];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.count; i += (uint64_t)gridDim.x * blockDim.x) {
        if (f.bytes == 8) ((uint64_t *)f.ptr)[i] = f.value;
        else ((uint32_t *)f.ptr)[i] = (uint32_t)f.value;
    }
}

// k_finalize for every item of a batch: blockIdx.y selects the item.
__global__ void k_finalize_batch(const FinalizeItem *fi) {
    const FinalizeItem f = fi[blockIdx.y];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f.n_inst; i += (uint64_t)gridDim.x * blockDim.x)
        fold_tally(f.ws, f.tfx, f.tally, f.n_inst, i, f.accumulate != 0);
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_find_cell(Dev g0, const double *pos, uint64_t n, int64_t *inst,
                                                      int32_t *cells) {
    __shared__ uint32_t lc[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Particle P;
    P.cell = lc + threadIdx.x;
    P.x = pos[3 * i];
    P.y = pos[3 * i + 1];
    P.z = pos[3 * i + 2];
    P.depth = 0;
    bool ok = false;
    int32_t fill;
    const int32_t c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, fill);
    if (c >= 0) {
        lvl(P, 0) = (uint32_t)c;
        ok = descend<PREC>(g, P, 0, P.x, P.y, P.z);
    }
    inst[i] = ok ? (int64_t)leaf_instance(g, P) : -1;
    if (cells)
        for (int L = 0; L < GT_MAX_LEVELS; L++)
            cells[i * GT_MAX_LEVELS + L] = (c >= 0 && L < P.depth) ? (int32_t)lvl(P, L) : -1;
}

__global__ void __launch_bounds__(kBlock) k_distance(Dev g0, const double *pos, const double *dir,
                                                     const int32_t *state, uint64_t n, double *dist,
                                                     int32_t *level, int32_t *surf) {
    __shared__ uint32_t lc[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Particle P;
    P.cell = lc + threadIdx.x;
    P.x = pos[3 * i];
    P.y = pos[3 * i + 1];
    P.z = pos[3 * i + 2];
    P.u = dir[3 * i];
    P.v = dir[3 * i + 1];
    P.w = dir[3 * i + 2];
    P.on_level = -1;
    P.on_surf = kNone;
    P.depth = 0;
    bool ok = false;
    if (state) {
        // the caller's state: a chain of fills from the root universe down to
        // a material cell, -1 below it, then the (level, surface) it is on
        const int32_t *w = state + (size_t)kStateWords * i;
        uint32_t u = g.root;
        ok = true;
        for (int L = 0; L < GT_MAX_LEVELS; L++) {
            const int32_t c = w[L];
            if (c < 0) break;
            const Univ U = ldv<Univ>(g.univ + u);
            if ((uint32_t)c < U.cell0 || (uint32_t)c - U.cell0 >= U.ncell) { ok = false; break; }
            lvl(P, L) = (uint32_t)c;
            P.depth = L + 1;
            const int32_t f = g.cell[c].fill;
            if (f >= 0) break;
            u = (uint32_t)(-f - 1);
        }
        ok = ok && P.depth > 0 && g.cell[lvl(P, P.depth - 1)].fill >= 0;
        for (int L = P.depth; ok && L < GT_MAX_LEVELS; L++) ok = w[L] == -1;
        const int32_t ol = w[GT_MAX_LEVELS];
        ok = ok && ol >= -1 && ol < P.depth;
        P.on_level = ol;
        P.on_surf = ol >= 0 ? (uint32_t)w[GT_MAX_LEVELS + 1] : kNone;
    } else {
        int32_t fill;
        const int32_t c = search<GT_PREC_FP64>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, fill);
        if (c >= 0) {
            lvl(P, 0) = (uint32_t)c;
            ok = descend<GT_PREC_FP64>(g, P, 0, P.x, P.y, P.z);
        }
    }
    if (!ok) {
        dist[i] = __builtin_nan("");
        level[i] = -1;
        surf[i] = -1;
        return;
    }
    int bl;
    uint32_t bs, bk;
    bool bpos;
    const double d = distance_all(g, P, bl, bs, bpos, bk);
    dist[i] = d;
    level[i] = d == dinf() ? -1 : bl;
    surf[i] = d == dinf() ? -1 : (int32_t)bs;
}

__global__ void k_fp64_check(const double *a, const double *b, uint64_t n, double *q, double *r, double *l) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    q[i] = a[i] / b[i];
    r[i] = sqrt(b[i]);
    l[i] = series_log(b[i]);
}

// ------------------------------------------------------------------ launchers
}  // namespace

// Workgroups that fit on the device at once (all compute units, the
// occupancy the kernel's resources allow), cached per device, kernel, block
// size and dynamic LDS size.
std::mutex g_launch_mu;   // guards the launch-shape caches below

int persistent_grid(const void *kernel, unsigned block, unsigned dyn, int device, int *blocks) {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    static int cache_dev[64], cache_block[64], cache_n[64];
    static unsigned cache_dyn[64];
    static const void *cache_k[64];
    static int used = 0;
    for (int i = 0; i < used; i++)
        if (cache_k[i] == kernel && cache_dev[i] == device && cache_block[i] == (int)block && cache_dyn[i] == dyn) {
            *blocks = cache_n[i];
            return GT_OK;
        }
    int cus = 0, per = 0;
    int rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    if (rc) return rc;
    rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)block, dyn),
                   "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (rc) return rc;
    if (per < 1) per = 1;
    *blocks = cus * per;
    if (used < 64) {
        cache_k[used] = kernel;
        cache_dev[used] = device;
        cache_block[used] = (int)block;
        cache_dyn[used] = dyn;
        cache_n[used] = *blocks;
        used++;
    }
    return GT_OK;
}

// Let a kernel use up to `bytes` of dynamic LDS (once per kernel).
int allow_dynamic_lds(const void *kernel, unsigned bytes) {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    constexpr int kDone = 256;   // kernels remembered (beyond that the attribute is set on every launch)
    static const void *done[kDone];
    static int used = 0;
    for (int i = 0; i < used; i++)
        if (done[i] == kernel) return GT_OK;
    int rc = hip_check(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                       "hipFuncSetAttribute");
    if (rc) return rc;
    if (used < kDone) done[used++] = kernel;
    return GT_OK;
}

// Dynamic LDS of a persistent launch: level columns, staged tables, then --
// within the workgroup's share of the compute unit's LDS that keeps the
// resident workgroups -- the regroup buffer (one word per lane), the tally
// cache, and the rest for the tail compaction buffer (which may reuse the
// regroup buffer).  A regroup that finds no room is left out (it never
// changes a result).
int plan_persistent(const void *kern, unsigned block, unsigned tables, bool tail, bool cache, uint32_t regroup,
                    int device, LdsPlan &lp) {
    hipFuncAttributes fa;
    int rc = hip_check(hipFuncGetAttributes(&fa, kern), "hipFuncGetAttributes");
    if (rc) return rc;
    const unsigned stat = (unsigned)fa.sharedSizeBytes;
    if (stat + GT_MAX_LEVELS * 4u * block + tables + 32u > kLdsPerCU)
        return set_error("staged tables exceed the LDS"), GT_ECAPACITY;
    rc = allow_dynamic_lds(kern, kLdsPerCU - stat);
    if (rc) return rc;
    const unsigned tables_at = (GT_MAX_LEVELS * 4u * block + 15u) & ~15u;
    const unsigned base = tables_at + ((tables + 15u) & ~15u);
    int blocks = 0;
    rc = persistent_grid(kern, block, base, device, &blocks);
    if (rc) return rc;
    int cus = 0;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    if (rc) return rc;
    const unsigned per = (unsigned)std::max(1, blocks / std::max(cus, 1));
    long avail = (long)(kLdsPerCU / per) - (long)stat - (long)base - 512;
    long rg_bytes = 0;
    if (regroup && block > 64 && avail >= 8L * block) rg_bytes = 8L * block;
    else regroup = 0;
    avail -= rg_bytes;
    unsigned ck = 0;
    if (cache && avail > 0) ck = std::min<unsigned>(kTallyCacheMax, (unsigned)(avail / (kTallyCacheEntry * block)));
    const unsigned cache_bytes = (ck * kTallyCacheEntry * block + 15u) & ~15u;
    avail -= (long)cache_bytes;
    const long buf_bytes = rg_bytes + std::max(avail, 0L);   // the buffer may use all that is left
    unsigned cap = 0;
    if (tail && block > 64) {
        cap = (unsigned)std::min<long>(buf_bytes / (kTailFields * 8), (long)block);
        if (cap < 64) cap = 0;
    }
    unsigned words = std::max(cap * kTailFields, regroup ? block : 0u);
    const unsigned tail_at = base + cache_bytes;
    unsigned dyn = tail_at + words * 8u;
    if (dyn != base) {
        int b2 = 0;
        rc = persistent_grid(kern, block, dyn, device, &b2);
        if (rc) return rc;
        if (b2 < blocks) {   // cache and buffer would cost a resident workgroup: go without
            ck = cap = words = regroup = 0;
            dyn = base;
        }
    }
    lp.dyn = dyn;
    lp.tables_at = tables_at;
    lp.cache_at = base;
    lp.cache_k = ck;
    lp.tail_at = ck ? tail_at : base;
    lp.tail_cap = cap;
    lp.tail_words = words;
    lp.regroup = regroup;
    lp.blocks = blocks;
    return GT_OK;
}


// Events recorded around the tracking kernels of this thread's next launches
// (set by gt_set_kernel_events; both null = off).
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

// The plan of this thread's last persistent launch (gt_last_launch).
thread_local gt_launch_info t_last_launch;
thread_local bool t_have_launch = false;

void note_launch(const LdsPlan &lp, int blocks, unsigned block, int kind, int surf) {
    t_last_launch = {(uint32_t)blocks, block, lp.dyn, (uint32_t)kind, lp.cache_k, lp.tail_cap, lp.regroup,
                     (uint32_t)surf};
    t_have_launch = true;
}


namespace {

// The build for the geometry's surface set (the general build for the
// parallel-ray source, whose code the smaller builds leave out).
int launch_persistent(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n, unsigned block,
                      bool tail, bool cache, uint32_t regroup, bool mesh, bool ray, hipStream_t st) {
    switch (ray ? SF_ALL : (int)g->surf_set) {
    case SF_AXCZ: return launch_persistent_axcz(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
    case SF_VERT: return launch_persistent_vert(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
    default: return launch_persistent_all(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
    }
}

// The work of one staging kind of a batch, in one launch: n chunks at ch,
// or (ns > 0) the ns items at sl with nh histories in all.
template <int PREC, int KIND, int W>
int launch_batch_k(gt_batch *b, const BatchChunk *ch, uint32_t n, unsigned long long *q, const BatchSlot *sl,
                   uint32_t ns, uint64_t nh, hipStream_t st) {
    const void *kern = (const void *)k_track_batch<PREC, KIND, W, false>;
    LdsPlan lp;
    int rc = GT_OK;
    if (b->regroup) {
        const void *kr = (const void *)k_track_batch<PREC, KIND, W, true>;
        rc = plan_persistent(kr, b->block, b->lds_bytes[KIND], b->tail, b->cache, b->regroup, b->device, lp);
        if (!rc && lp.regroup) kern = kr;
    }
    if (!rc && kern == (const void *)k_track_batch<PREC, KIND, W, false>)
        rc = plan_persistent(kern, b->block, b->lds_bytes[KIND], b->tail, b->cache, 0, b->device, lp);
    if (rc) return rc;
    int blocks = lp.blocks;
    // no more workgroups than chunks, or than whole workgroups of histories
    const uint64_t cap = ns ? (nh + b->block - 1) / b->block : n;
    if ((uint64_t)blocks > cap) blocks = (int)cap;
    note_launch(lp, blocks, b->block, KIND, SF_ALL);
    if (lp.regroup)
        hipLaunchKernelGGL((k_track_batch<PREC, KIND, W, true>), dim3(blocks), dim3(b->block), lp.dyn, st,
                           b->d_items, ch, n, q, sl, ns, b->d_claimed, b->d_workers, lp.tables_at, lp.tail_at,
                           lp.tail_cap, kTailRound, lp.tail_words, lp.regroup, lp.cache_at, lp.cache_k);
    else
        hipLaunchKernelGGL((k_track_batch<PREC, KIND, W, false>), dim3(blocks), dim3(b->block), lp.dyn, st,
                           b->d_items, ch, n, q, sl, ns, b->d_claimed, b->d_workers, lp.tables_at, lp.tail_at,
                           lp.tail_cap, kTailRound, lp.tail_words, 0u, lp.cache_at, lp.cache_k);
    return GT_OK;
}

// Helper streams of a batch: the launches of different staging kinds share
// no data (each item's chunks, queue counter and outputs belong to one kind),
// so they run on streams forked from and joined back into the caller's; the
// workgroups of a later launch then start on compute units that an earlier
// launch's tail has left (default priority throughout).
struct BatchStreams {
    hipStream_t s[3];
    hipEvent_t fork, join[3];
};

int batch_streams(gt_batch *b, BatchStreams *&bs) {
    bs = (BatchStreams *)b->side;
    if (bs) return GT_OK;
    BatchStreams *n = new (std::nothrow) BatchStreams;
    if (!n) return set_error("host allocation failed"), GT_ENOMEM;
    int streams = 0, joins = 0;
    bool fork = false;
    hipError_t e = hipEventCreateWithFlags(&n->fork, hipEventDisableTiming);
    fork = e == hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; i++) {
        e = hipStreamCreateWithFlags(&n->s[i], hipStreamNonBlocking);
        if (e == hipSuccess) streams++;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&n->join[i], hipEventDisableTiming);
        if (e == hipSuccess) joins++;
    }
    if (e != hipSuccess) {
        for (int i = 0; i < streams; i++) (void)hipStreamDestroy(n->s[i]);
        for (int i = 0; i < joins; i++) (void)hipEventDestroy(n->join[i]);
        if (fork) (void)hipEventDestroy(n->fork);
        delete n;
        return set_error("gt_batch_launch: helper streams: %s", hipGetErrorString(e)), GT_EHIP;
    }
    b->side = bs = n;
    return GT_OK;
}

template <int PREC, int W>
int launch_batch_kinds(gt_batch *b, hipStream_t st) {
    int kinds = 0;
    uint64_t listed = 0, slotted = 0;
    for (int kind = 0; kind < 4; kind++) {
        kinds += (b->by_item ? b->n_slot_kind[kind] : b->n_kind[kind]) ? 1 : 0;
        listed += b->n_kind[kind];
        slotted += b->n_slot_kind[kind];
    }
    // (gt_batch_create checked every chunk and slot; the groups must still
    // add up before any launch reads them)
    if (listed != b->n_chunks || slotted != b->n_slots || (b->by_item ? b->n_chunks : b->n_slots) != 0)
        return set_error("gt_batch_launch: inconsistent chunk or item groups"), GT_EINVAL;
    BatchStreams *bs = nullptr;
    if (kinds > 1) {
        int rc = batch_streams(b, bs);
        if (rc) return rc;
        rc = hip_check(hipEventRecord(bs->fork, st), "hipEventRecord");
        if (rc) return rc;
    }
    uint32_t first = 0, first_slot = 0;
    int lane = 0;
    for (int kind = 3; kind >= 0; kind--) {   // groups in the order gt_batch_create wrote them
        const uint32_t n = b->n_kind[kind], ns = b->n_slot_kind[kind];
        const BatchChunk *ch = b->d_chunks + first;
        const BatchSlot *sl = b->d_slots + first_slot;
        const uint64_t nh = b->n_hist_kind[kind];
        unsigned long long *q = b->d_queue + kind;
        first += n;
        first_slot += ns;
        if (b->by_item ? !ns : !n) continue;
        hipStream_t s = st;
        if (lane > 0) {
            s = bs->s[lane - 1];
            int rc = hip_check(hipStreamWaitEvent(s, bs->fork, 0), "hipStreamWaitEvent");
            if (rc) return rc;
        }
        int rc = kind == SK_ALL     ? launch_batch_k<PREC, SK_ALL, W>(b, ch, n, q, sl, ns, nh, s)
                 : kind == SK_LDS   ? launch_batch_k<PREC, SK_LDS, W>(b, ch, n, q, sl, ns, nh, s)
                 : kind == SK_SPLIT ? launch_batch_k<PREC, SK_SPLIT, W>(b, ch, n, q, sl, ns, nh, s)
                                    : launch_batch_k<PREC, SK_NONE, W>(b, ch, n, q, sl, ns, nh, s);
        if (rc) return rc;
        if (lane > 0) {
            rc = hip_check(hipEventRecord(bs->join[lane - 1], s), "hipEventRecord");
            if (rc) return rc;
            rc = hip_check(hipStreamWaitEvent(st, bs->join[lane - 1], 0), "hipStreamWaitEvent");
            if (rc) return rc;
        }
        lane++;
    }
    return GT_OK;
}

template <int PREC>
int launch_track_t(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, const gt_mesh *mesh,
                   hipStream_t st) {
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    const uint64_t nws = (uint64_t)tally_replicas(g->n_inst) * 4 * g->n_inst;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(nws)), dim3(256), 0, st, ko.tally_ws, nws, (uint64_t)0);
    if (mesh) {
        MeshDesc &m = ko.mesh;
        for (int a = 0; a < 3; a++) {
            m.lo[a] = mesh->lo[a];
            m.w[a] = (mesh->hi[a] - mesh->lo[a]) / (double)mesh->n[a];
            m.iw[a] = 1.0 / m.w[a];
            m.n[a] = mesh->n[a];
        }
        m.nb = (uint64_t)mesh->n[0] * mesh->n[1] * mesh->n[2];
        m.ws = (uint64_t *)mesh->workspace;
        const uint64_t mws = (uint64_t)tally_replicas(m.nb) * 4 * m.nb;
        hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(mws)), dim3(256), 0, st, m.ws, mws, (uint64_t)0);
    }
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, o->counters, (uint64_t)8, (uint64_t)0);
    if (kp.rec_k) {
        const uint64_t nrec = (uint64_t)kp.rec_k * kp.rec_cap;
        hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(nrec)), dim3(256), 0, st, o->rec, nrec, (int32_t)-1);
    }
    mark(t_ev_start, st);
    if (kp.n) {
        if (p->flags & GT_FLAG_LANE_PER_HISTORY) {
            const unsigned block = p->block_size ? p->block_size : kBlock;
            hipLaunchKernelGGL((k_track<PREC>), dim3(grid_for(kp.n, block)), dim3(block), 0, st, g->dev, kp, ko);
        } else {
            const unsigned block = p->block_size ? p->block_size : kBlockP;
            const StagePlan &sp = g->stage[PREC];
            const int kind = (p->flags & GT_FLAG_NO_STAGING) ? SK_NONE : (int)sp.kind;
            LaunchRec rec;
            rec.p = kp;
            rec.o = ko;
            LaunchRec *lrec;
            uint64_t *tws;
            workspace_of(g, o, &lrec, &tws);
            hipLaunchKernelGGL(k_put_launch, dim3(1), dim3(64), 0, st, rec, lrec);
            const bool tail = (p->flags & GT_FLAG_TAIL_COMPACTION) != 0;
            const bool cache = !(p->flags & GT_FLAG_NO_TALLY_CACHE);
            const uint32_t rg = p->regroup_every;
            const bool ms = mesh != nullptr;
            int rc;
            if (p->flags & (GT_FLAG_TRACKER_SP | GT_FLAG_TRACKER_RTK)) {
                rc = launch_kinds(g, lrec, PREC, (p->flags & GT_FLAG_TRACKER_SP) ? TRK_SP : TRK_RTK, kp.n, block, tail,
                                  cache, !(p->flags & GT_FLAG_NO_STAGING), p->source == 1, st);
            } else {
                rc = launch_persistent(g, lrec, PREC, block == 640 ? 5 : 4, kind, kp.n, block, tail, cache, rg, ms,
                                       p->source == 1, st);
            }
            if (rc) return rc;
        }
    }
    mark(t_ev_stop, st);
    hipLaunchKernelGGL(k_finalize, dim3(fill_grid(g->n_inst)), dim3(256), 0, st, (const uint64_t *)ko.tally_ws,
                       o->tally_fx, o->tally, g->n_inst, (int)((p->flags & GT_FLAG_ACCUMULATE) != 0));
    if (mesh)
        hipLaunchKernelGGL(k_finalize, dim3(fill_grid(ko.mesh.nb)), dim3(256), 0, st, (const uint64_t *)ko.mesh.ws,
                           mesh->mesh_fx, mesh->mesh, ko.mesh.nb, (int)((p->flags & GT_FLAG_ACCUMULATE) != 0));
    return hip_check(hipGetLastError(), "gt_track launch");
}

// The event-based schedule: births, then iterations of the three operation
// kernels until no history is left.  The host reads the number of live
// histories back every kEvCheck iterations (the call waits for the stream);
// an iteration adds at most one segment to every history, so at most
// max_segments + 1 iterations run.
constexpr int kEvCheck = 8;

template <int PREC>
int launch_event_t(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *bank, hipStream_t st) {
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    EvBank b;
    ev_layout(kp.n, (unsigned char *)bank, &b);
    const uint64_t nws = (uint64_t)tally_replicas(g->n_inst) * 4 * g->n_inst;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(nws)), dim3(256), 0, st, ko.tally_ws, nws, (uint64_t)0);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, o->counters, (uint64_t)8, (uint64_t)0);
    if (kp.rec_k) {
        const uint64_t nrec = (uint64_t)kp.rec_k * kp.rec_cap;
        hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(nrec)), dim3(256), 0, st, o->rec, nrec, (int32_t)-1);
    }
    mark(t_ev_start, st);
    if (kp.n) {
        const unsigned grid = grid_for(kp.n, kBlock);
        hipLaunchKernelGGL((k_ev_birth<PREC>), dim3(grid), dim3(kBlock), 0, st, g->dev, kp, ko, b);
        unsigned long long left = 1;
        for (uint64_t it = 0; left; it++) {
            if (it > (uint64_t)kp.max_segs + 1)
                return set_error("gt_track_event: histories left after max_segments iterations"), GT_EHIP;
            unsigned long long *a = b.alive + (it & 1);
            hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, (uint64_t *)a, (uint64_t)1, (uint64_t)0);
            hipLaunchKernelGGL((k_ev_distance<PREC>), dim3(grid), dim3(kBlock), 0, st, g->dev, kp.n, b);
            hipLaunchKernelGGL((k_ev_move<PREC>), dim3(grid), dim3(kBlock), 0, st, g->dev, kp, ko, b);
            hipLaunchKernelGGL((k_ev_cross<PREC>), dim3(grid), dim3(kBlock), 0, st, g->dev, kp, ko, b, a);
            if (it % kEvCheck == kEvCheck - 1) {
                int rc = hip_check(hipMemcpyAsync(&left, a, sizeof(left), hipMemcpyDeviceToHost, st),
                                   "hipMemcpyAsync");
                if (!rc) rc = hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                if (rc) return rc;
            }
        }
    }
    mark(t_ev_stop, st);
    hipLaunchKernelGGL(k_finalize, dim3(fill_grid(g->n_inst)), dim3(256), 0, st, (const uint64_t *)ko.tally_ws,
                       o->tally_fx, o->tally, g->n_inst, (int)((p->flags & GT_FLAG_ACCUMULATE) != 0));
    return hip_check(hipGetLastError(), "gt_track_event launch");
}

template <int PREC>
int launch_batch_t(gt_batch *b, hipStream_t st) {
    const uint64_t fx = std::min<uint64_t>((b->max_fill + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_ranges, dim3((unsigned)std::max<uint64_t>(fx, 1), b->n_fill), dim3(256), 0, st, b->d_fill);
    mark(t_ev_start, st);
    int rc = b->block == 640 ? launch_batch_kinds<PREC, 5>(b, st) : launch_batch_kinds<PREC, 4>(b, st);
    if (rc) return rc;
    mark(t_ev_stop, st);
    const uint64_t bx = std::min<uint64_t>((b->max_inst + 255) / 256, 1024);
    hipLaunchKernelGGL(k_finalize_batch, dim3((unsigned)std::max<uint64_t>(bx, 1), b->n_items), dim3(256), 0, st, b->d_fin);
    return hip_check(hipGetLastError(), "gt_batch_launch");
}

}  // namespace


void set_kernel_events(void *start, void *stop) {
    t_ev_start = (hipEvent_t)start;
    t_ev_stop = (hipEvent_t)stop;
}

bool last_launch(gt_launch_info *out) {
    if (t_have_launch) *out = t_last_launch;
    return t_have_launch;
}

int prepare_batch_streams(gt_batch *b) {
    int kinds = 0;
    for (int kind = 0; kind < 4; kind++) kinds += (b->by_item ? b->n_slot_kind[kind] : b->n_kind[kind]) ? 1 : 0;
    BatchStreams *bs = nullptr;
    return kinds > 1 ? batch_streams(b, bs) : GT_OK;
}

void release_batch_streams(gt_batch *b) {
    BatchStreams *bs = (BatchStreams *)b->side;
    if (!bs) return;
    for (int i = 0; i < 3; i++) {
        (void)hipStreamDestroy(bs->s[i]);
        (void)hipEventDestroy(bs->join[i]);
    }
    (void)hipEventDestroy(bs->fork);
    delete bs;
    b->side = nullptr;
}

int launch_batch(gt_batch *b, void *stream) {
    if (b->block > (uint32_t)kBlockP) return set_error("gt_batch_launch: block_size too large"), GT_EINVAL;
    return b->precision == GT_PREC_MIXED ? launch_batch_t<GT_PREC_MIXED>(b, (hipStream_t)stream)
                                         : launch_batch_t<GT_PREC_FP64>(b, (hipStream_t)stream);
}

int launch_event(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *bank, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (p->n_particles > (uint64_t)0x7FFFFFFF * 64ull) return set_error("gt_track_event: too many particles"), GT_ECAPACITY;
    return p->precision == GT_PREC_MIXED ? launch_event_t<GT_PREC_MIXED>(g, p, o, bank, st)
                                         : launch_event_t<GT_PREC_FP64>(g, p, o, bank, st);
}

int launch_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream,
                 const gt_mesh *mesh) {
    hipStream_t st = (hipStream_t)stream;
    if ((p->flags & GT_FLAG_LANE_PER_HISTORY) && p->block_size > (uint32_t)kBlock)
        return set_error("gt_track: block_size must be at most %d with GT_FLAG_LANE_PER_HISTORY", kBlock), GT_EINVAL;
    if (p->n_particles > (uint64_t)0x7FFFFFFF * 64ull) return set_error("gt_track: too many particles"), GT_ECAPACITY;
    return p->precision == GT_PREC_MIXED ? launch_track_t<GT_PREC_MIXED>(g, p, o, mesh, st)
                                         : launch_track_t<GT_PREC_FP64>(g, p, o, mesh, st);
}

int launch_find_cell(const gt_geometry *g, const double *pos, uint64_t n, int64_t *inst, int32_t *cells,
                     uint32_t precision, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if (!n) return GT_OK;
    const unsigned grid = grid_for(n, kBlock);
    if (precision == GT_PREC_MIXED)
        hipLaunchKernelGGL((k_find_cell<GT_PREC_MIXED>), dim3(grid), dim3(kBlock), 0, st, g->dev, pos, n, inst, cells);
    else
        hipLaunchKernelGGL((k_find_cell<GT_PREC_FP64>), dim3(grid), dim3(kBlock), 0, st, g->dev, pos, n, inst, cells);
    return hip_check(hipGetLastError(), "gt_find_cell launch");
}

int launch_distance(const gt_geometry *g, const double *pos, const double *dir, const int32_t *state, uint64_t n,
                    double *dist, int32_t *level, int32_t *surf, void *stream) {
    if (!n) return GT_OK;
    hipLaunchKernelGGL(k_distance, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, g->dev, pos, dir,
                       state, n, dist, level, surf);
    return hip_check(hipGetLastError(), "gt_distance_to_surface launch");
}

int launch_fp64_check(const double *a, const double *b, uint64_t n, double *q, double *r, double *l, void *stream) {
    if (!n) return GT_OK;
    hipLaunchKernelGGL(k_fp64_check, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, a, b, n, q, r, l);
    return hip_check(hipGetLastError(), "gt_fp64_check launch");
}

int launch_persistent_all(const gt_geometry *g, const LaunchRec *lr, int prec, int w, int kind, uint64_t n,
                          unsigned block, bool tail, bool cache, uint32_t regroup, bool mesh, hipStream_t st) {
    return launch_persistent_set<SF_ALL>(g, lr, prec, w, kind, n, block, tail, cache, regroup, mesh, st);
}

}  // namespace gt

// ------------------------------------------------------------------ allocation-free entry point
// gt_track_noalloc's workspace (launch record, then the per-XCD limb
// counters of the tallies) lives in this fixed array: every GPU the library
// runs on holds its own copy until the process ends.  In host code the name
// stands for the host-side shadow, not a device address, so the device
// address is looked up once per device (with that device current) and only
// that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[GT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_at[kMaxDevices];   // device address of `scratch` per device, once looked up
}  // namespace

extern "C" int gt_track_noalloc(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o,
                                void *stream) {
    using namespace gt;
    if (o && o->workspace)
        return set_error("gt_track_noalloc: workspace must be NULL (the library's fixed scratch array is used)"),
               GT_EINVAL;
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    const uint64_t need = track_ws_bytes(g->n_inst);
    if (need > GT_NOALLOC_SCRATCH_BYTES)
        return set_error("gt_track_noalloc: %llu leaf instances need %llu bytes of workspace, above the %llu of "
                         "the fixed scratch array",
                         (unsigned long long)g->n_inst, (unsigned long long)need,
                         (unsigned long long)GT_NOALLOC_SCRATCH_BYTES),
               GT_ECAPACITY;
    int dev = -1;
    rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev != g->device)
        return set_error("gt_track_noalloc: the geometry lives on device %d but device %d is current", g->device,
                         dev),
               GT_EINVAL;
    if (dev < 0 || dev >= kMaxDevices) return set_error("gt_track_noalloc: device %d out of range", dev), GT_EINVAL;
    void *at;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_at[dev]) {
            void *a = nullptr;
            rc = hip_check(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
            if (rc) return rc;
            if (!a || ((uintptr_t)a & 255u))
                return set_error("gt_track_noalloc: scratch array at an unusable address %p", a), GT_EHIP;
            g_scratch_at[dev] = a;
        }
        at = g_scratch_at[dev];
    }
    gt_track_out o2 = *o;
    o2.workspace = at;
    o2.workspace_bytes = GT_NOALLOC_SCRATCH_BYTES;
    return launch_track(g, p, &o2, stream);
}
