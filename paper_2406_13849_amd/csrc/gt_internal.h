// Internal layout of the device geometry tables and kernel launch records.
// Shared by the host preprocessor (gt_geometry.cpp) and the HIP kernels
// (gt_track.hip); not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gt.h"

namespace gt {

enum SurfType : uint32_t { ST_PX = 0, ST_PY = 1, ST_PZ = 2, ST_P = 3, ST_CZ = 4, ST_SPH = 5 };

// Surface sets the tracker code is compiled for: every type; only axis
// planes and z-cylinders (square lattices of pins); or those and general
// planes parallel to the z axis (zero z coefficient: hexagonal lattices),
// whose value and denominator then leave out the z term -- a signed zero,
// which can change only the sign of a zero result, on which no decision
// depends.  The host picks the build from the geometry's surfaces; every
// build gives identical results.
constexpr int SF_ALL = 0, SF_AXCZ = 1, SF_VERT = 2;

// packed half-space: surface id << 4 | positive-side bit << 3 | surface type
__host__ __device__ inline uint32_t hs_pack(uint32_t s, bool pos, uint32_t type) {
    return (s << 4) | ((pos ? 1u : 0u) << 3) | type;
}

constexpr int kBlockP = 1024;   // lanes per workgroup of the persistent trackers (launch bound)
// LDS left for staged geometry tables next to the persistent trackers'
// per-lane level columns (160 KiB per compute unit on gfx950)
constexpr unsigned kStageBudget = 160 * 1024 - GT_MAX_LEVELS * kBlockP * 4 - 1024;
// A wave refills its idle lanes once at least this many are idle, so that
// new histories start together and their first searches (which rarely have
// a good candidate) run once for several lanes.
constexpr uint32_t kRefillMin = 8;
// Histories a wave claims from the work queue at once by default (one per
// lane): the pool it refills its lanes from.
constexpr uint32_t kWaveTake = 64;

constexpr uint32_t kLeafNone = 0xFFFFFFFFu;
// int32 words of one tracking state given to gt_distance_to_surface: the
// cell of each level, then the level and surface the particle is on
constexpr int kStateWords = GT_MAX_LEVELS + 2;
constexpr uint32_t kLeafMax = 4;       // cells per BVH leaf
constexpr uint32_t kHintNone = 0, kHintSquare = 1;

// A cell's plane half-spaces start with slab pairs: two planes of one family
// (the same axis, or bitwise-identical normal coefficients) bounding the
// cell from both sides, the negative-side one first.  Along any direction at
// most one plane of a pair can be reached, chosen by the sign of the shared
// denominator, so a pair costs one distance evaluation.
constexpr uint32_t kPlaneCountMask = 0xFFFu, kMaxPairs = 15;

// 16 bytes per cell; its half-spaces are stored planes first, then quadrics
struct alignas(16) Cell {
    uint32_t hs_off;    // first packed half-space
    uint16_t n_pl;      // plane half-spaces (stored first): low 12 bits their number, high 4 bits
                        // the number of slab pairs at their front (see kPlaneCountMask)
    uint16_t n_hs;      // number of half-spaces
    int32_t fill;       // >= 0 material, < 0 daughter universe -(u+1)
    uint32_t inst_off;  // leaf-instance offset of this cell within its universe
};

// 48 bytes per universe
struct alignas(16) Univ {
    uint32_t cell0, ncell;   // cell range
    uint32_t node0, nnode;   // BVH nodes in depth-first order; nnode == 0: no cell reachable
    int32_t hint, nx, ny, pad;
    float x0, y0, inv_px, inv_py;   // lattice guess (single precision, advisory)
};

// Universe kinds for the trackers that keep one tracker type per kind of
// universe (the static-polymorphism method and the fixed-depth reactor
// tracker; Sections "Static polymorphism (SP) method" and "RTK tracking").
// The preprocessor recognises them from the cells themselves; the single
// tracker never reads them.
//  * rect: an nx x ny pseudo-array whose cell (i, j) is local cell j*nx + i,
//    bounded by x planes X_i < X_{i+1} and y planes Y_j < Y_{j+1} (the outer
//    planes of the first and last row and column may be absent: unbounded),
//    plus the same extra half-spaces in every cell;
//  * pin: concentric z-cylinders of one centre and z planes; cell (slab k,
//    ring r) is local cell k*(ncyl+1) + r, between cylinders r-1 and r and
//    z planes k-1 and k (the innermost ring, the outermost ring and the end
//    slabs unbounded on that side).
constexpr int32_t kKindCsg = 0, kKindRect = 1, kKindPin = 2;

// 48 bytes per universe.  Arrays (aval: values, asurf: surface ids):
//  rect: X_0 .. X_nx, then Y_0 .. Y_ny (+-inf / kLeafNone where a plane is
//        absent); extra half-spaces: nxhs packed entries at ahs[xhs];
//  pin:  r^2 of the n0 cylinders (inner first), the centre (x, y), then the
//        n1 z planes (ascending).
struct alignas(16) UArr {
    int32_t kind;
    uint32_t cell0;
    uint32_t arr;        // first entry in aval / asurf
    uint32_t xhs;        // rect: first extra half-space in ahs
    uint32_t n0, n1;     // rect: nx, ny; pin: cylinders, z planes
    uint32_t nxhs, pad;
    float x0, y0, inv_px, inv_py;   // rect: first-guess index (single precision; corrected exactly)
};

// BVH node with single-precision, outward-rounded bounds (32 bytes).  Nodes
// are stored depth-first; an internal node's first child follows it, and
// `escape` is the next node to visit when the point is outside the node
// (or after a leaf has been searched).  leaf == kLeafNone for internal
// nodes, else first << 4 | (count - 1) into the leaf-cell array.
struct alignas(32) Node32 {
    float lo[3];
    uint32_t escape;
    float hi[3];
    uint32_t leaf;
};

// The same hierarchy with double-precision widened bounds (64 bytes).
struct alignas(64) Node64 {
    double lo[3];
    uint32_t escape, leaf;
    double hi[3];
    uint32_t pad[2];
};

// Device view of one geometry (passed by value to kernels).
struct Dev {
    const double *coef;     // 4 per surface (see gt.h, first four slots)
    const uint32_t *hs;     // packed half-spaces
    const Cell *cell;
    const double *trans;    // 4 per cell: x, y, z, 0
    const Univ *univ;
    const Node32 *node32;
    const Node64 *node64;
    const uint32_t *leaf;   // leaf cell ids
    const float *cbox;      // 8 per cell: lo xyz, 0, hi xyz, 0 (single precision, outward)
    const double *sigma;
    const uint32_t *adj_off;    // per half-space entry: first candidate in adj (n_hs + 1 entries)
    const uint32_t *adj;        // crossing candidates: cells using the surface with the other sense
                                // whose widened boxes touch the cell's box, largest overlap first
    const uint32_t *cell_local; // index of each cell within its universe
    const UArr *uarr;           // per universe: its kind and arrays (see UArr)
    const double *aval;         // array values
    const uint32_t *asurf;      // array surface ids
    const uint32_t *ahs;        // extra half-spaces of rect universes (packed)
    const uint32_t *cell_ij;    // rect cells: i | j << 16; pin cells: ring | slab << 16; others 0
    uint32_t root, n_inst, max_depth, n_cells;
    double lo[3], hi[3];
};

// Blob sections (all 256-byte aligned in one device allocation)
enum Section { SEC_COEF, SEC_HS, SEC_CELL, SEC_TRANS, SEC_UNIV, SEC_NODE32, SEC_NODE64, SEC_LEAF, SEC_CBOX,
               SEC_SIGMA, SEC_ADJOFF, SEC_ADJ, SEC_LOCAL, SEC_UARR, SEC_AVAL, SEC_ASURF, SEC_AHS, SEC_IJ,
               SEC_COUNT };

// Copy of a geometry's hot tables into LDS: sections of the device blob
// (byte offsets, 16-byte multiples) and where each lands in LDS.
struct StagePlan {
    uint32_t n;                 // number of sections copied
    uint32_t total;             // LDS bytes
    uint32_t src[SEC_COUNT], dst[SEC_COUNT], bytes[SEC_COUNT];
    uint32_t at[SEC_COUNT];     // LDS byte offset of each section (0xFFFFFFFF when not copied)
    uint32_t kind;              // 0: nothing copied; 1: the per-segment tables (cells, half-spaces,
                                // surfaces, universes, materials, local indices); 2: those and
                                // the crossing tables (translations, candidate lists); 3: every
                                // table the precision mode reads
};

struct KParams {
    uint64_t seed, first, n;
    uint32_t geom_id, max_coll, source, ray_n1, max_segs, rec_k, rec_cap, refill_min;
    uint32_t wave_take, pad;   // histories a wave claims from the queue at once (a multiple of 64)
};

// A superimposed mesh: bins n[0] x n[1] x n[2] over lo + [0, n] w, with its
// replicas of per-bin limb counters (ws == nullptr: no mesh).
struct MeshDesc {
    double lo[3], w[3];
    double iw[3];       // 1 / w: only for the first guess of a plane index, corrected exactly
    uint32_t n[3], pad;
    uint64_t *ws;
    uint64_t nb;
};

struct KOut {
    MeshDesc mesh;
    uint64_t *tally_ws;     // replicas of per-instance limb counters
    uint32_t *seg_count;
    uint64_t *seq_hash;
    uint8_t *end_code;
    int32_t *rec;
    uint64_t *counters;
};

// Device copy of a geometry's descriptor (read-only for every launch).
struct GeomDesc {
    Dev dev;
    StagePlan stage[2];       // per precision mode, for the single tracker
    StagePlan stage_arr[2];   // the same with the universe-kind tables among the per-segment ones, for
                              // the trackers that switch on universe kind
};

// Parameters of one tracking launch, written to device memory by a small
// kernel ahead of it (so the tracker reads them through a pointer).
struct LaunchRec {
    KParams p;
    KOut o;
};

// Replicas of an array of n sets of four 64-bit limb counters (one set per
// leaf instance, or per mesh bin): one per XCD while the eight copies take at
// most kReplicaBudget bytes, else a single one.  Replica r is used by the
// waves of the XCDs whose id is r mod the replica count.  Few, hot entries
// need the XCDs kept apart (fewer replicas slow the small geometries of a
// batch); many entries are touched rarely, and the memory-side atomics run
// faster on the smaller array (the three-level core's 2.86 M instances take
// 92 MB of counters in one replica instead of 732 MB in eight).
constexpr int kReplicas = 8;   // the most: one per XCD
constexpr uint64_t kReplicaBudget = 64ull << 20;
__host__ __device__ inline uint32_t tally_replicas(uint64_t n) {
    return (uint64_t)kReplicas * 32 * n <= kReplicaBudget ? (uint32_t)kReplicas : 1u;
}

// Tally workspace of one tracking call (the geometry's own, or the caller's
// through gt_track_out.workspace): the launch record, then the replicas of
// n_inst x four 64-bit limb counters.
constexpr uint64_t kWsTallyAt = (sizeof(LaunchRec) + 255) & ~(uint64_t)255;
inline uint64_t track_ws_bytes(uint64_t n_inst) {
    const uint64_t n = n_inst ? n_inst : 1;
    return kWsTallyAt + (uint64_t)tally_replicas(n) * 4 * 8 * n;
}

// One item of a batched launch (device copy).
struct BatchItem {
    Dev dev;
    StagePlan plan;
    KParams p;
    KOut o;
};

// A range of particle indices of one batch item.
struct BatchChunk {
    uint32_t item, pad;
    uint64_t first, count;
};

// One item of a batch launch whose workgroups join whole items (chunk = 0):
// its histories, the estimated cost of one of them, and the running sum of
// n * weight over the launch's slots up to and including this one.
struct BatchSlot {
    uint32_t item;
    float weight;
    uint64_t n;
    double cum;
};
constexpr uint32_t kNoItem = 0xFFFFFFFFu;

// Particle bank of the event-based schedule: structure of arrays in device
// memory, n entries each (the caller's buffer, laid out by ev_layout).
struct EvBank {
    double *x, *y, *z, *u, *v, *w, *tau;
    double *t, *sig;                 // distance to the nearest surface and Sigma of the leaf, this segment
    uint64_t *h, *acc_lo, *acc_hi;   // sequence hash; the history's open tally sum (128-bit)
    uint32_t *cell;                  // GT_MAX_LEVELS x n, level-major
    uint32_t *on_surf, *blk, *segs, *ncoll, *acc_inst, *surf, *inst;
    uint32_t *entry;                 // half-space entry of the nearest surface (its candidate list)
    uint32_t *st;                    // packed: depth | on_level + 1 << 4 | end << 8 | nearest level << 12 |
                                     // nearest sense << 16 | crossing pending << 17 | record overflow << 18 |
                                     // finished << 19
    unsigned long long *alive;       // [2]: histories left after an iteration (alternating)
};

struct FillRange {
    void *ptr;
    uint64_t count, value;
    uint32_t bytes, pad;
};

struct FinalizeItem {
    const uint64_t *ws;
    uint64_t *tfx;
    double *tally;
    uint64_t n_inst;
    uint32_t accumulate, pad;
};

}  // namespace gt

// host-side geometry object behind the opaque ABI handle
struct gt_geometry {
    gt::Dev dev;
    gt::StagePlan stage[2];   // per precision mode (GT_PREC_FP64, GT_PREC_MIXED)
    gt::StagePlan stage_arr[2];   // ... for the trackers that switch on universe kind
    uint32_t rtk_shape;       // 0: not of the fixed-depth reactor shape; else see gt_geometry_kinds
    uint32_t n_rect, n_pin;   // universes recognised as rectilinear arrays and as pins
    uint32_t surf_set;        // SF_AXCZ, SF_VERT or SF_ALL (the smallest set that holds every surface)
    const gt::GeomDesc *desc; // device copy of dev and stage (in the blob)
    void *blob;          // one device allocation holding every table
    uint64_t blob_bytes;
    void *ws;            // the geometry's own tally workspace (track_ws_bytes(n_inst) bytes), used by
                         // calls that bring none: its launch record ...
    gt::LaunchRec *launch;
    uint64_t *tally_ws;  // ... and its limb counters
    uint64_t n_inst;
    uint32_t max_depth;
    int device;
};

// host-side batch object behind the opaque ABI handle
struct gt_batch {
    int device;
    uint32_t precision, n_items, block, refill_min;
    void *dmem;                         // one allocation for everything below
    gt::BatchItem *d_items;
    gt::BatchChunk *d_chunks;           // chunks by staging kind: kind 3, then 2, 1, 0
    uint32_t n_chunks;
    uint32_t n_kind[4];
    // workgroups join whole items (chunk = 0): the items with histories, by
    // staging kind (3, 2, 1, 0), and per item its claim counter and the
    // number of workgroups on it
    bool by_item;
    gt::BatchSlot *d_slots;
    uint32_t n_slots;
    uint32_t n_slot_kind[4];
    uint64_t n_hist_kind[4];
    unsigned long long *d_claimed, *d_workers;
    gt::FillRange *d_fill;
    uint32_t n_fill;
    uint64_t max_fill;
    gt::FinalizeItem *d_fin;
    uint64_t max_inst;
    unsigned long long *d_queue;        // one counter per staging kind
    uint32_t lds_bytes[4];              // staged tables' LDS bytes per kind (largest item)
    bool tail;                          // tail compaction on
    uint32_t regroup;                   // loop trips between regroups (0 = off)
    bool cache;                         // per-lane tally cache on
    void *side;                         // helper streams and events for the staging-kind launches
                                        // (made by gt_batch_create when there are several kinds)
};

namespace gt {
void set_error(const char *fmt, ...);
// The workspace a call uses: the caller's (gt_track_out.workspace) or the geometry's.
void workspace_of(const gt_geometry *g, const gt_track_out *o, LaunchRec **launch, uint64_t **tally);
int check_track_args(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o);
void fill_kparams(const gt_track_params *p, const gt_geometry *g, KParams &kp, KOut &ko, const gt_track_out *o);
unsigned stage_budget();
void set_kernel_events(void *start, void *stop);
bool last_launch(gt_launch_info *out);
bool cached_batch_tuning(const gt_batch_item *items, uint32_t n_items, gt_tuning *out);
int launch_batch(gt_batch *b, void *stream);
int prepare_batch_streams(gt_batch *b);
void release_batch_streams(gt_batch *b);
int launch_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream,
                 const gt_mesh *mesh = nullptr);
int launch_find_cell(const gt_geometry *g, const double *pos, uint64_t n, int64_t *inst, int32_t *cells,
                     uint32_t precision, void *stream);
int launch_distance(const gt_geometry *g, const double *pos, const double *dir, const int32_t *state, uint64_t n,
                    double *dist, int32_t *level, int32_t *surf, void *stream);
int launch_fp64_check(const double *a, const double *b, uint64_t n, double *q, double *r, double *l,
                      void *stream);
uint64_t ev_layout(uint64_t n, unsigned char *base, EvBank *b);
int launch_event(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *bank, void *stream);
}  // namespace gt
