/*
 * gt.h -- C ABI of the MI355X nested-CSG geometry tracker (libgt.so).
 *
 * The library tracks toy-transport Monte Carlo particle histories through
 * nested constructive-solid-geometry universes and pseudo-array lattices
 * with one CSG tracker accelerated by per-universe bounding-volume
 * hierarchies: the "single tracker" method of Biondo et al. (Section
 * "Single tracker (ST) method"), using the tracking operations of Table 1
 * (find_cell, distance_to_surface, move_within_cell, cross_surface,
 * change_direction) inside the history loop of Alg. 2.
 *
 * Conventions for every entry point:
 *   - return 0 on success or a negative GT_E* code; gt_last_error() then
 *     returns a thread-local message naming the offending argument, cell or
 *     surface.  No C++ exception crosses this boundary.
 *   - "host" pointers are read during the call and never retained; "device"
 *     pointers are HIP device memory owned by the caller (for example torch
 *     tensors' data pointers) and are accessed asynchronously on `stream`
 *     (a hipStream_t; NULL is the null stream).  Device results are valid
 *     once the stream has been synchronised by the caller.
 *   - Problems found while tracking (a particle leaving through a gap, a
 *     record buffer too short) are reported through per-particle end codes
 *     and the counters array, not through the return value.
 *   - All arithmetic that decides a cell is IEEE double without fused
 *     multiply-add; single precision is only used to skip candidates whose
 *     conservatively widened bounding box cannot contain the point, so
 *     results do not depend on the precision mode.
 */
#ifndef GT_H
#define GT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define GT_OK 0
#define GT_EINVAL (-1)     /* bad argument (null pointer, size, flag)         */
#define GT_EGEOM (-2)      /* geometry failed validation                      */
#define GT_ENOMEM (-3)     /* host or device allocation failed               */
#define GT_EHIP (-4)       /* a HIP runtime call failed (message has details) */
#define GT_ECAPACITY (-5)  /* a size exceeds a documented limit               */

/* ---- limits ------------------------------------------------------------ */
#define GT_MAX_LEVELS 6          /* nesting depth (root = level 0)            */
#define GT_MAX_INSTANCES 0xFFFFFFF0u

/* ---- surface types (Introduction, CSG construction): positive side is
 *      f(p) > 0, a point with f(p) <= 0 is on the negative side.  Coefficient
 *      slots, 8 doubles per surface:
 *        PX/PY/PZ : d            f = x - d (resp. y, z)
 *        P        : a b c d      f = ((a x + b y) + c z) - d
 *        CZ       : x0 y0 r2     f = ((x-x0)^2 + (y-y0)^2) - r2
 *        SPH      : x0 y0 z0 r2  f = (((x-x0)^2 + (y-y0)^2) + (z-z0)^2) - r2  */
#define GT_SURF_PX 0
#define GT_SURF_PY 1
#define GT_SURF_PZ 2
#define GT_SURF_P 3
#define GT_SURF_CZ 4
#define GT_SURF_SPH 5

/* ---- per-particle end codes ------------------------------------------- */
#define GT_END_NONE 0
#define GT_END_ESCAPE 1   /* crossed out of every root cell (vacuum)         */
#define GT_END_CAP 2      /* reached max_collisions                           */
#define GT_END_LOST 3     /* no cell found below the root after a crossing    */
#define GT_END_SEGCAP 4   /* reached max_segments                             */

/* ---- counters (uint64 each, device array of 8; counters[7] is the work-queue
 *      position used by the persistent schedule) ---------------------------- */
#define GT_CNT_ESCAPED 0
#define GT_CNT_CAPPED 1
#define GT_CNT_LOST 2
#define GT_CNT_SEGCAP 3
#define GT_CNT_REC_OVERFLOW 4   /* recorded particles with more segments than record_cap */
#define GT_CNT_SEGMENTS 5       /* total segments (move_within_cell calls)               */
#define GT_CNT_REJECTED 6       /* birth positions rejected (outside every root cell)     */

/* ---- precision modes ---------------------------------------------------- */
#define GT_PREC_FP64 0    /* double-precision bounding boxes, no lattice guess          */
#define GT_PREC_MIXED 1   /* single-precision widened boxes + lattice index guess, every
                             decision still taken in double precision                   */

/* ---- flags --------------------------------------------------------------- */
#define GT_FLAG_ACCUMULATE 1u          /* add to tally_fx instead of zeroing it first         */
#define GT_FLAG_LANE_PER_HISTORY 2u    /* one history per lane, one launch slot per history
                                          (the plain schedule) instead of the persistent,
                                          refilling schedule                                */
#define GT_FLAG_NO_STAGING 4u          /* persistent schedule: read the geometry tables from
                                          global memory even when they fit in LDS           */
#define GT_FLAG_TAIL_COMPACTION 8u     /* persistent schedule: once the queue is empty, pack the
                                          remaining histories of a workgroup into fewer waves
                                          (off by default: idle waves then wait instead of
                                          ending, which costs more than it saves here)       */
#define GT_FLAG_NO_TALLY_CACHE 16u     /* persistent schedule: flush a lane's tally partial sum
                                          at every change of instance instead of keeping up
                                          to three more in an LDS cache (speed only)         */
/* Tracker method of the persistent schedule (default: the single tracker, ST,
 * of Section "Single tracker (ST) method": every universe is CSG, searched
 * through its bounding-volume hierarchy).  The two others keep one tracker
 * type per kind of universe, as the paper's comparison methods do; the
 * kinds are recognised by gt_geometry_create from the cells themselves
 * (gt_geometry_kinds).  All three give identical outputs. */
#define GT_FLAG_TRACKER_SP 32u         /* static polymorphism (Section "Static polymorphism (SP)
                                          method", Listing 1): a switch on each level's
                                          universe kind; rectilinear arrays find a cell by
                                          index and cross to the neighbour by index (Algs. 5
                                          and 6), other universes use the CSG tracker       */
#define GT_FLAG_TRACKER_RTK 64u        /* the fixed-depth reactor tracker (Section "RTK
                                          tracking", Algs. 9 and 10): levels of known kind
                                          (an optional one-cell root, one or two array
                                          levels, pins of concentric cylinders and axial
                                          planes), loops over levels unrolled; GT_EINVAL for
                                          a geometry not of that shape                       */

typedef struct gt_geometry gt_geometry;   /* opaque; owns its device tables */

/* Flattened geometry, all arrays host memory, copied by gt_geometry_create.
 * A cell is the intersection of its half-spaces (Introduction, CSG cells);
 * a universe is a contiguous range of cells; a cell is filled with a
 * material or with a daughter universe placed with a translation t, the
 * daughter's local coordinates being p - t (Section "Multi-universe CPU
 * tracking", Alg. 7/8).  Arrays are modelled as pseudo-array universes
 * (Section "Single tracker (ST) method").
 * Requirements (checked; violations return GT_EGEOM):
 *   - hs entries are +(s+1) (positive side of surface s) or -(s+1); a
 *     surface appears at most once per cell and belongs to one universe;
 *   - univ_cell_off is non-decreasing with non-empty ranges covering all
 *     cells; the fill graph from `root` is acyclic and at most
 *     GT_MAX_LEVELS deep; materials index sigma_t (> 0, finite);
 *   - every root cell lies inside [domain_lo, domain_hi] (the sampling box).
 * Modelling assumption (not checked): two cells of one universe never
 * both contain a point, i.e. they are separated by a shared surface with
 * opposite senses, by parallel planes of one family, or by concentric
 * cylinders/spheres; a daughter universe never repeats a surface of its
 * parent cell.  Then every search order finds the same cell.
 * lattice_hint: optional (NULL), 8 doubles per universe
 *   [kind, nx, ny, x0, y0, px, py, 0]; kind 1 = square pseudo-array whose
 *   local cell j*nx+i spans [x0+i px, x0+(i+1) px] x [y0+j py, ...].  Used
 *   only as a first guess that is verified in double precision. */
typedef struct {
    uint32_t n_surfaces, n_cells, n_universes, n_materials, n_halfspaces, root;
    const uint8_t *surf_type;      /* [n_surfaces]                 */
    const double *surf_coef;       /* [n_surfaces * 8]             */
    const uint32_t *cell_hs_off;   /* [n_cells + 1]                */
    const int32_t *hs;             /* [n_halfspaces]               */
    const int32_t *cell_fill;      /* [n_cells]: >=0 material, <0 -(universe+1) */
    const double *cell_trans;      /* [n_cells * 3]                */
    const uint32_t *univ_cell_off; /* [n_universes + 1]            */
    const double *lattice_hint;    /* [n_universes * 8] or NULL    */
    const double *sigma_t;         /* [n_materials], 1/cm          */
    double domain_lo[3], domain_hi[3];
} gt_flat_geometry;

/* Validate, preprocess (leaf-instance numbering, cell bounding boxes, one
 * SAH-built bounding-volume hierarchy per universe -- the paper's
 * acceleration structure of Section "Single tracker (ST) method" with the
 * three-candidates-per-axis surface-area heuristic -- and lattice guesses),
 * then upload once to the current HIP device.  *out receives the handle. */
int gt_geometry_create(const gt_flat_geometry *f, gt_geometry **out);

/* Number of leaf instances (the length of the tally arrays), nesting depth
 * and bytes of device memory held.  Any output pointer may be NULL. */
int gt_geometry_info(const gt_geometry *g, uint64_t *n_instances, uint32_t *max_depth,
                     uint64_t *device_bytes);

/* How the persistent trackers hold this geometry's tables for a precision
 * mode: *kind 0 = all in global memory, 1 = the per-segment tables (cells,
 * half-spaces, surfaces, universes, materials) copied to LDS, 2 = those and
 * the crossing tables (translations, candidate lists), 3 = every table; and
 * the LDS bytes copied per workgroup.  Either output may be NULL. */
int gt_geometry_staging(const gt_geometry *g, uint32_t precision, uint32_t *kind, uint32_t *lds_bytes);

/* Universe kinds the per-kind trackers see (GT_FLAG_TRACKER_SP / _RTK):
 * the numbers of universes recognised as rectilinear arrays (nx x ny
 * pseudo-arrays of cells bounded by x and y planes, local cell j*nx + i,
 * with the same extra half-spaces in every cell) and as pins (concentric
 * z-cylinders of one centre and z planes, local cell slab*(cylinders+1) +
 * ring), and the fixed-depth shape: 0 when GT_FLAG_TRACKER_RTK cannot track
 * the geometry, else 1 | (one-cell root above the arrays) << 1 | (two array
 * levels) << 2.  Any output pointer may be NULL. */
int gt_geometry_kinds(const gt_geometry *g, uint32_t *n_rect, uint32_t *n_pin, uint32_t *rtk_shape);

void gt_geometry_destroy(gt_geometry *g);

/* Parameters of one batch of histories (host struct). */
typedef struct {
    uint64_t seed;            /* Philox4x32-10 key                                   */
    uint64_t first_particle;  /* global id of the first particle                     */
    uint64_t n_particles;
    uint32_t geometry_id;     /* fourth Philox counter word                          */
    uint32_t max_collisions;  /* a history ends at this many collisions (>= 1)       */
    uint32_t source;          /* 0 uniform volume source, isotropic;
                                 1 parallel rays along +x from the x = lo face on a
                                 ray_n1 x ceil(n/ray_n1) grid, no collisions         */
    uint32_t ray_n1;
    uint32_t max_segments;    /* a history ends after this many segments (>= 1)      */
    uint32_t precision;       /* GT_PREC_*                                           */
    uint32_t record_first_k;  /* particles [0, k) of the batch record their sequence */
    uint32_t record_cap;      /* entries recorded per particle                       */
    uint32_t flags;           /* GT_FLAG_*                                           */
    uint32_t block_size;      /* threads per workgroup, a multiple of 64: up to 1024
                                 (persistent schedule, default 1024; 640 selects a
                                 build for two workgroups of 10 waves per compute
                                 unit) or up to 256 (GT_FLAG_LANE_PER_HISTORY,
                                 default 256); 0 = default                          */
    uint32_t refill_min;      /* persistent schedule: a wave starts new histories once at
                                 least this many of its lanes are idle (1..64; 0 = 8)   */
    uint32_t regroup_every;   /* persistent schedule: every this many loop trips the
                                 waves of a workgroup meet and sort their lanes'
                                 histories by key (the leaf universe of a history
                                 about to take a segment, else its step; idle lanes
                                 last) with a counting sort in LDS, moving each
                                 history's state whole (regroup by universe, to cut
                                 divergence; speed only).  0 = never (the default);
                                 skipped where the LDS left over cannot hold one
                                 64-bit word per lane or for workgroups of one wave;
                                 must be 0 for GT_FLAG_LANE_PER_HISTORY and for
                                 gt_track_event                                      */
    uint32_t wave_histories;  /* persistent schedule: histories a wavefront claims
                                 from the work queue at once and hands to its idle
                                 lanes as they free up -- the particles per
                                 wavefront of a claim: 64, 128, ..., 1024 (one to
                                 sixteen per lane); 0 = 64.  Speed only.  Must be 0
                                 for GT_FLAG_LANE_PER_HISTORY and gt_track_event     */
} gt_track_params;

/* Outputs, all device memory owned by the caller.
 *   tally_fx  [2 * n_instances] uint64: per leaf instance, the (low, high)
 *             words of a 128-bit fixed-point sum of segment lengths in units
 *             of 2^-96 cm (each length truncated to that quantum; the total
 *             is independent of summation order).  Required.
 *   tally     [n_instances] double or NULL: tally_fx converted to cm.
 *   seg_count [n_particles] uint32, seq_hash [n_particles] uint64,
 *   end_code  [n_particles] uint8, each may be NULL.  seq_hash is the 64-bit
 *             FNV-1a style fold h = (h ^ (inst+1)) * 0x100000001b3 over the
 *             leaf instance of every segment from 0xcbf29ce484222325, then
 *             h ^= end_code.
 *   rec       [record_first_k * record_cap] int32 or NULL: leaf instance of
 *             each segment of the recorded particles, -1 padded.
 *   counters  [8] uint64, required; zeroed by the call (GT_CNT_*).
 *   workspace device scratch of at least workspace_bytes >=
 *             gt_track_workspace_bytes(g) bytes, 256-byte aligned, for the
 *             call's partial tally sums and launch record (overwritten; its
 *             contents are meaningless after the call), or NULL: the call
 *             then uses the geometry's own workspace, so calls on one
 *             geometry that bring no workspace must be ordered (one stream,
 *             or synchronised); calls with distinct workspaces may run
 *             concurrently on different streams. */
typedef struct {
    uint64_t *tally_fx;
    double *tally;
    uint32_t *seg_count;
    uint64_t *seq_hash;
    uint8_t *end_code;
    int32_t *rec;
    uint64_t *counters;
    void *workspace;
    uint64_t workspace_bytes;
} gt_track_out;

/* Bytes of the tally workspace a tracking call on g needs (0 for a NULL g). */
uint64_t gt_track_workspace_bytes(const gt_geometry *g);

/* Sample and track a batch of histories (Alg. 2 reduced to a toy
 * transport: uniform birth position rejected until a root cell contains
 * it, isotropic direction (Marsaglia 1972), exponential optical depth from
 * a counter-based Philox4x32-10 stream keyed by (seed, particle id,
 * geometry id); per segment distance_to_surface over every level, a
 * boundary crossing when it is strictly shorter than tau/Sigma of the leaf
 * material, else a collision with isotropic redirection; vacuum boundary).
 * Asynchronous on `stream`; allocates nothing.  GT_EINVAL also for a
 * workspace that is short or not 256-byte aligned. */
int gt_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream);

/* ---- allocation-free tracking --------------------------------------------
 * For callers that cannot allocate device memory during a call or bring a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): gt_track with its tally workspace and launch
 * record taken from a fixed device array inside the library, of
 * GT_NOALLOC_SCRATCH_BYTES bytes, one copy per GPU, held from the first
 * such call on that GPU until the process ends.  The call allocates
 * nothing (no hipMalloc, no library routine that allocates); inputs and
 * outputs are the caller's, exactly as for gt_track, and the outputs are
 * identical to gt_track's.
 *   o->workspace must be NULL (GT_EINVAL otherwise).
 *   The geometry's device must be the current device (GT_EINVAL).
 *   GT_ECAPACITY when gt_track_workspace_bytes(g) exceeds
 *   GT_NOALLOC_SCRATCH_BYTES (every geometry of up to 131,000 leaf
 *   instances fits).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind; each call clears what it needs.  Calls that may overlap on one GPU
 * (different streams, or threads without ordering) race on the array and
 * must be serialised by the caller. */
#define GT_NOALLOC_SCRATCH_BYTES (32ull << 20)
int gt_track_noalloc(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream);

/* ---- event-based schedule (for comparison) ------------------------------
 * The histories and outputs of gt_track, computed the way an event-based GPU
 * tracker is organised (Section "GPU-based implementation in Shift"): the
 * particle state lives in a bank in device memory and every iteration runs
 * one kernel per tracking operation over the whole bank -- distance to
 * surface, then move / tally / collision, then cross surface -- until no
 * history is left.  Each history takes the same steps in the same order as in
 * gt_track, so every output is identical.
 *   bank:  caller-owned device memory of at least gt_event_bank_bytes(n)
 *          bytes, 256-byte aligned, contents overwritten (may be NULL when
 *          n_particles is 0);
 *   flags: GT_FLAG_ACCUMULATE only; block_size and refill_min must be 0.
 * The host reads the number of live histories back every 8 iterations, so the
 * call waits for `stream` and cannot be captured into a graph.  Errors as
 * gt_track, and GT_EINVAL for a missing, short or misaligned bank. */
uint64_t gt_event_bank_bytes(uint64_t n_particles);   /* 0 above the particle limit */
int gt_track_event(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *bank,
                   uint64_t bank_bytes, void *stream);

/* ---- superimposed mesh tally --------------------------------------------
 * The paper's active cycles add a regular mesh flux tally over the core
 * (Section "NuScale SMR").  gt_track_mesh tracks exactly the histories of
 * gt_track, with the same outputs, and also tallies track length on a mesh of
 * n[0] x n[1] x n[2] bins over the box [lo, hi]; bin (ix, iy, iz) is entry
 * (iz * n[1] + iy) * n[0] + ix.  Each segment p0 + t u, 0 <= t <= l, is cut at
 * every mesh plane lo[a] + k w[a] (w[a] = (hi[a] - lo[a]) / n[a], k = 0..n[a])
 * that it crosses at t = (plane - p0[a]) / u[a] with 0 < t < l, and each piece
 * adds its length to the bin holding its midpoint (bin index floor((mid[a] -
 * lo[a]) / w[a]) per axis); pieces outside the mesh add nothing.  Sums are
 * fixed point as the cell tally's (each piece truncated to 2^-96 cm), so they
 * do not depend on the order of the pieces.
 *   mesh_fx:   [2 * bins] uint64 device, required ((low, high) words per bin);
 *              overwritten, or added to with GT_FLAG_ACCUMULATE;
 *   mesh:      [bins] double device or NULL: mesh_fx in cm;
 *   workspace: caller-owned device memory of gt_mesh_workspace_bytes(bins)
 *              bytes, 256-byte aligned, contents overwritten.
 * Persistent schedule only (no GT_FLAG_LANE_PER_HISTORY, regroup_every 0).
 * Errors as gt_track; GT_EINVAL for a bad mesh (n < 1, lo >= hi or not
 * finite, reserved != 0), a missing mesh_fx, or a missing, short or
 * misaligned workspace; GT_ECAPACITY above 2^24 bins on an axis or 2^31 in
 * all.  Asynchronous; allocates nothing. */
typedef struct {
    double lo[3], hi[3];
    uint32_t n[3];
    uint32_t reserved;         /* must be 0 */
    uint64_t *mesh_fx;
    double *mesh;
    void *workspace;
    uint64_t workspace_bytes;
} gt_mesh;
uint64_t gt_mesh_workspace_bytes(uint64_t bins);   /* 0 for 0 or more than 2^31 bins */
int gt_track_mesh(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, const gt_mesh *m,
                  void *stream);

/* ---- many geometries in one launch -------------------------------------- */
typedef struct gt_batch gt_batch;   /* opaque: device descriptors of a batch */

typedef struct {
    const gt_geometry *geometry;    /* each geometry at most once per batch    */
    gt_track_params params;         /* as for gt_track; one precision for all;
                                       GT_FLAG_LANE_PER_HISTORY not allowed    */
    gt_track_out out;               /* as for gt_track                         */
} gt_batch_item;

typedef struct {
    uint32_t block_size;   /* threads per workgroup, multiple of 64 up to 1024; 0 = 1024      */
    uint32_t refill_min;   /* as gt_track_params.refill_min; 0 = 8                             */
    uint64_t chunk;        /* histories per work item taken from the device queue; 0 = whole
                              items: a workgroup joins an item and claims its histories
                              until none is left (see gt_batch_create)                       */
    uint32_t regroup_every;/* as gt_track_params.regroup_every; 0 = that of the first item    */
    uint32_t wave_histories; /* as gt_track_params.wave_histories; 0 = each item's own          */
} gt_tuning;               /* a NULL gt_tuning* means: the shape gt_autotune_batch found for
                              the same items in this process, else the defaults              */

/* Validate a batch and upload its descriptors: per item the geometry
 * tables, parameters and output pointers, and the work list, largest items
 * first (estimated work: histories x nesting depth).  With chunk > 0 the
 * work list holds (item, particle range) chunks that workgroups take one at
 * a time, their waves meeting at the end of each.  With chunk = 0 (whole
 * items) it lists the items: workgroups first spread over the items in
 * proportion to their estimated work, each workgroup's waves then claim
 * their item's histories from its counter (shared by the workgroups on the
 * item) until none is left, and the workgroup then joins the item with the
 * most estimated work left per workgroup on it.  The histories are exactly
 * those each item's gt_track call would track, with identical outputs. */
int gt_batch_create(const gt_batch_item *items, uint32_t n_items, const gt_tuning *tuning, gt_batch **out);
/* Errors: GT_EINVAL for an empty batch, a rejected item (the message names
 * it), mixed precisions, GT_FLAG_LANE_PER_HISTORY, a geometry used twice or
 * on another device than the current one; GT_ECAPACITY above 16384 items;
 * GT_ENOMEM when the descriptors cannot be allocated.  The batch keeps the
 * geometry tables' and output buffers' addresses: they must outlive it.
 * Work-queue position counters[7] stays 0 for batch items. */

/* Track every item of the batch: one fill launch, then one persistent launch
 * per staging kind present (items whose tables fit the LDS in full, in part,
 * or not at all), then one finalize launch.  The kind launches run on helper
 * streams that the batch owns (made by gt_batch_create when it has several
 * kinds, default priority), forked from `stream` and joined back into it with
 * events before the finalize launch, so later kinds start on compute units
 * that earlier ones have finished with.  Only kernel launches and event
 * records/waits are issued, so the call can be captured into a HIP graph and
 * replayed. */
int gt_batch_launch(gt_batch *b, void *stream);

void gt_batch_destroy(gt_batch *b);

/* ---- launch-shape autotuning ---------------------------------------------
 * Shapes change only the speed, never an output.  Both tuners synchronize
 * the stream and overwrite the outputs they are given. */

/* Time gt_track with every shape block_size in {256, 512, 640, 1024} x refill_min
 * in {1, 4, 8, 16} (one untimed and `reps` timed launches each), then the
 * fastest of these with regroup_every in {16, 64, 256}, on the given
 * parameters (regroup_every 0 in the first stage); *best gets the fastest
 * (chunk = 0) and *best_ms its mean launch time (may be NULL).  The outputs end as those of one gt_track call
 * with the winning shape.  The winner is cached in the process under
 * (geometry, precision, staging and tail flags, histories rounded up to a
 * power of two): see gt_tuning_lookup.  Errors as gt_track, and GT_EINVAL
 * for GT_FLAG_LANE_PER_HISTORY (nothing to tune). */
int gt_autotune_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, uint32_t reps,
                      void *stream, gt_tuning *best, float *best_ms);

/* The cached shape for these parameters: 1 and *out filled if
 * gt_autotune_track has tuned such a launch in this process, else 0. */
int gt_tuning_lookup(const gt_geometry *g, const gt_track_params *p, gt_tuning *out);

/* Time gt_batch_launch for block_size in {512, 640, 1024} x refill_min in
 * {1, 4, 8, 16} x chunk in {0 (whole items), 1024, 4096, 16384}, then the fastest of these
 * with regroup_every in {16, 64, 256}; *best gets the fastest.  The
 * winner is cached in the process for this list of (geometry, histories,
 * precision): gt_batch_create and gt_track_batch given a NULL tuning use it. */
int gt_autotune_batch(const gt_batch_item *items, uint32_t n_items, uint32_t reps, void *stream, gt_tuning *best,
                      float *best_ms);

/* Timing hook (for benchmarks and profilers; the paper times the tracking
 * kernels alone).  With two hipEvent_t handles set, every later gt_track and
 * gt_batch_launch on the calling thread records start_event on its stream
 * right before its tracking kernel launch(es) and stop_event right after, so
 * the elapsed time between them excludes the zeroing and finalize kernels.
 * The events stay the caller's; gt_set_kernel_events(NULL, NULL) turns the
 * hook off.  GT_EINVAL if exactly one handle is NULL. */
int gt_set_kernel_events(void *start_event, void *stop_event);

/* The plan of the calling thread's last persistent tracker launch (gt_track
 * without GT_FLAG_LANE_PER_HISTORY, or the last staging-kind launch of
 * gt_batch_launch), as chosen by the library from the launch shape and the
 * LDS left over: workgroups launched, threads per workgroup, dynamic LDS
 * bytes per workgroup, staging kind (0 tables in global memory ... 3 all
 * in LDS), tally-cache entries per lane, tail-compaction capacity
 * (histories; 0 = off) and regroup interval (loop trips; 0 = no regroup
 * step).  For tests and tuning: 1 and *out filled, or 0 if this thread has
 * made no such launch; GT_EINVAL for a NULL out. */
typedef struct {
    uint32_t workgroups, block_size, lds_bytes, staging_kind;
    uint32_t tally_cache_entries, tail_capacity, regroup_every;
    uint32_t surface_set;   /* the build's surface set: 1 axis planes and z-cylinders only, 2 those and
                               planes parallel to the z axis, 0 every surface type (also every
                               launch with the parallel-ray source) */
} gt_launch_info;
int gt_last_launch(gt_launch_info *out);

/* One-shot form: create, launch, wait for the stream, destroy. */
int gt_track_batch(const gt_batch_item *items, uint32_t n_items, const gt_tuning *tuning, void *stream);

/* Table 1 find_cell for a batch of global positions (device pos[3n]):
 * inst[n] receives the leaf instance or -1, cells[n * GT_MAX_LEVELS] (may be
 * NULL) the cell id per level, -1 padded.  precision selects the candidate
 * search (GT_PREC_*); results do not depend on it. */
int gt_find_cell(const gt_geometry *g, const double *pos, uint64_t n, int64_t *inst, int32_t *cells,
                 uint32_t precision, void *stream);

/* Table 1 distance_to_surface for a batch (device pos[3n], dir[3n]): the
 * distance along dir to the nearest surface of the cells the point is in at
 * every level, ties going to the top-most level, then the lowest surface id
 * (Alg. 8's surf_universe).
 *   state: NULL -- each point is first located with find_cell and is on no
 *          surface; or device int32 [n * (GT_MAX_LEVELS + 2)], per point the
 *          cell id of levels 0..GT_MAX_LEVELS-1 (a chain of fills from the
 *          root universe down to a material cell, -1 below it), then the
 *          level and surface id the point is on (-1 -1 for none), as a
 *          crossing leaves them: a plane the point is on is not hit again,
 *          and a cylinder or sphere it is on gives only its far root.
 * dist[n] receives the distance (+inf if none, NaN if the point is in no
 * cell or its state is not such a chain or names a level below its leaf),
 * level[n]/surf[n] the level and surface id hit (-1 if none).  Asynchronous;
 * GT_EINVAL for a null geometry or, with n > 0, a null array other than
 * state. */
int gt_distance_to_surface(const gt_geometry *g, const double *pos, const double *dir, const int32_t *state,
                           uint64_t n, double *dist, int32_t *level, int32_t *surf, void *stream);

/* Floating-point contract check: for device arrays a[n], b[n] (b > 0)
 * writes a/b, sqrt(b) and the library's logarithm of b (the series used for
 * the exponential flight sampling) computed on the device, so a caller can
 * compare them bit for bit with a host implementation. */
int gt_fp64_check(const double *a, const double *b, uint64_t n, double *quot, double *root, double *logb,
                  void *stream);

/* Thread-local description of the last failure in this thread. */
const char *gt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GT_H */
