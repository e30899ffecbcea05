// HIP kernels of libgt for gfx950 (CDNA4): Monte Carlo geometry tracking
// through nested CSG universes with one CSG tracker and per-universe
// bounding-volume hierarchies (Section "Single tracker (ST) method").
//
// Two schedules share every device function:
//   - k_track_persistent (default): one workgroup per compute unit; each
//     wave loops until the particle pool is drained, refilling finished
//     lanes from a wave-local pool of particle ids, and every lane runs a
//     small state machine whose steps (draw random numbers, search one
//     level, one segment) each have a single call site;
//   - k_track (GT_FLAG_LANE_PER_HISTORY): one history per lane.
// A particle's state lives in registers; the cell of each level lives in
// LDS (one column per lane) so level loops index it without spilling.
//
// Floating point: compiled with -ffp-contract=off and no fast-math, so every
// double operation below is one IEEE operation in the order written; the
// results of find_cell / distance_to_surface / cross_surface are the ones a
// plain double-precision implementation of the same definitions computes.
// Single precision only appears in the optional candidate pruning (widened,
// outward-rounded boxes and a lattice-index guess), which can skip a cell
// only when that cell cannot contain the point.
#pragma clang fp contract(off)

#include <algorithm>
#include <mutex>

#include "gt_internal.h"

namespace gt {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxBirthAttempts = 1000;
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;
constexpr int kBlock = 256;     // lanes per workgroup of the one-history-per-lane kernels
constexpr int kBlockP = 1024;   // lanes per workgroup of the persistent tracker (launch bound)
// LDS left for staged geometry tables next to the persistent tracker's
// per-lane level arrays (160 KiB per compute unit on gfx950)
constexpr unsigned kStageBudget = 160 * 1024 - GT_MAX_LEVELS * kBlockP * 4 - 1024;

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// ------------------------------------------------------------------ table views
// The kernels read the geometry tables through pointers whose address space
// is part of their type, so the compiler emits LDS reads (32-bit addresses)
// for tables staged in LDS and global loads for the others, instead of flat
// loads that must serve both.  A view DevT<A, B, C> holds the per-segment
// tables (cells, half-spaces, surfaces, universes, materials, local indices)
// in address space A, the crossing tables (translations, candidate lists) in
// B and the hierarchy (nodes, leaves, cell boxes) in C; 3 = LDS, 1 = global.
template <int AS, typename T> using cptr = const __attribute__((address_space(AS))) T *;

template <int A, int B, int C>
struct DevT {
    cptr<A, double> coef;
    cptr<A, uint32_t> hs;
    cptr<A, Cell> cell;
    cptr<A, Univ> univ;
    cptr<A, double> sigma;
    cptr<A, uint32_t> cell_local;
    cptr<B, double> trans;
    cptr<B, uint32_t> adj_off;
    cptr<B, uint32_t> adj;
    cptr<C, Node32> node32;
    cptr<C, Node64> node64;
    cptr<C, uint32_t> leaf;
    cptr<C, float> cbox;
    uint32_t root, n_inst, max_depth, n_cells;
    double lo[3], hi[3];
};

typedef DevT<1, 1, 1> DevGlobal;   // every table in global memory
typedef DevT<3, 1, 1> DevSplit;    // per-segment tables in LDS
typedef DevT<3, 3, 1> DevLds;      // per-segment and crossing tables in LDS
typedef DevT<3, 3, 3> DevAll;      // every table in LDS

// Store to global memory (the output arrays) through a typed pointer.
template <typename T, typename V>
__device__ __forceinline__ void gstore(T *base, uint64_t i, V v) {
    ((__attribute__((address_space(1))) T *)base)[i] = (T)v;
}

// A whole record through a typed pointer (the copy goes through a generic
// pointer cast from the typed one, which keeps the address space).
template <typename T, typename P>
__device__ __forceinline__ T ldv(P p) {
    return *(const T *)p;
}

template <int A, int B, int C>
__device__ __forceinline__ void view_scalars(DevT<A, B, C> &d, const Dev &g) {
    d.root = g.root;
    d.n_inst = g.n_inst;
    d.max_depth = g.max_depth;
    d.n_cells = g.n_cells;
    for (int k = 0; k < 3; k++) {
        d.lo[k] = g.lo[k];
        d.hi[k] = g.hi[k];
    }
}

__device__ __forceinline__ DevGlobal global_view(const Dev &g) {
    DevGlobal d;
    d.coef = (cptr<1, double>)g.coef;
    d.hs = (cptr<1, uint32_t>)g.hs;
    d.cell = (cptr<1, Cell>)g.cell;
    d.univ = (cptr<1, Univ>)g.univ;
    d.sigma = (cptr<1, double>)g.sigma;
    d.cell_local = (cptr<1, uint32_t>)g.cell_local;
    d.trans = (cptr<1, double>)g.trans;
    d.adj_off = (cptr<1, uint32_t>)g.adj_off;
    d.adj = (cptr<1, uint32_t>)g.adj;
    d.node32 = (cptr<1, Node32>)g.node32;
    d.node64 = (cptr<1, Node64>)g.node64;
    d.leaf = (cptr<1, uint32_t>)g.leaf;
    d.cbox = (cptr<1, float>)g.cbox;
    view_scalars(d, g);
    return d;
}

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, the key bumped by the
// published Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// One sampling event = one Philox block at counter (b, id lo, id hi,
// geometry id): its 128 bits (word 0 least significant) give three 42-bit
// fields (bits [0,42), [42,84), [84,126)), each mapped exactly to the
// uniform (f + 1/2) 2^-42 in (0,1).
__device__ __forceinline__ void draw_block(uint64_t key, uint32_t gid, uint64_t pid, uint32_t b, double &u0,
                                           double &u1, double &u2) {
    uint32_t o0, o1, o2, o3;
    philox4x32_10(b, (uint32_t)pid, (uint32_t)(pid >> 32), gid, (uint32_t)key, (uint32_t)(key >> 32), o0, o1, o2,
                  o3);
    const uint64_t w0 = ((uint64_t)o1 << 32) | o0, w1 = ((uint64_t)o3 << 32) | o2;
    const uint64_t m42 = (1ull << 42) - 1;
    const uint64_t f0 = w0 & m42;
    const uint64_t f1 = (w0 >> 42) | ((w1 & ((1ull << 20) - 1)) << 22);
    const uint64_t f2 = (w1 >> 20) & m42;
    u0 = ((double)f0 + 0.5) * 0x1p-42;
    u1 = ((double)f1 + 0.5) * 0x1p-42;
    u2 = ((double)f2 + 0.5) * 0x1p-42;
}

// Natural logarithm from log m = 2 atanh(s), s = (m-1)/(m+1), m in
// [sqrt(1/2), sqrt(2)), twelve odd-power terms with coefficients 1/(2k+1)
// (each the correctly rounded quotient), and e*ln2 split in a 32-bit head
// (exact products) and a tail.  Used for the exponential optical depth.
__device__ __forceinline__ double series_log(double x) {
    const uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const double sqrt2 = __longlong_as_double(0x3FF6A09E667F3BCDll);
    if (m >= sqrt2) { m = m * 0.5; e = e + 1; }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double poly = 1.0 / 23.0;
    poly = poly * z + 1.0 / 21.0;
    poly = poly * z + 1.0 / 19.0;
    poly = poly * z + 1.0 / 17.0;
    poly = poly * z + 1.0 / 15.0;
    poly = poly * z + 1.0 / 13.0;
    poly = poly * z + 1.0 / 11.0;
    poly = poly * z + 1.0 / 9.0;
    poly = poly * z + 1.0 / 7.0;
    poly = poly * z + 1.0 / 5.0;
    poly = poly * z + 1.0 / 3.0;
    poly = poly * z + 1.0;
    const double logm = (s + s) * poly;
    const double ln2_hi = __longlong_as_double(0x3FE62E42FEE00000ll);
    const double ln2_lo = __longlong_as_double(0x3DEA39EF35793C76ll);
    const double de = (double)e;
    return de * ln2_hi + (de * ln2_lo + logm);
}

// Marsaglia (1972) isotropic direction from one block's first two fields;
// false when the pair is rejected.
__device__ __forceinline__ bool direction_from(double u0, double u1, double &u, double &v, double &w) {
    const double v1 = 2.0 * u0 - 1.0;
    const double v2 = 2.0 * u1 - 1.0;
    const double s = v1 * v1 + v2 * v2;
    if (!(s < 1.0 && s != 0.0)) return false;
    const double r = sqrt(1.0 - s);
    u = (2.0 * v1) * r;
    v = (2.0 * v2) * r;
    w = 1.0 - 2.0 * s;
    return true;
}

// ------------------------------------------------------------------ surfaces
// Half-spaces of a cell are stored planes first (types PX, PY, PZ, P), then
// quadrics (CZ, SPH), so each loop below runs one surface family.
template <typename CP>
__device__ __forceinline__ double plane_value(uint32_t type, CP c, double x, double y, double z) {
    switch (type) {
    case ST_PX: return x - c[0];
    case ST_PY: return y - c[0];
    case ST_PZ: return z - c[0];
    default: return ((c[0] * x + c[1] * y) + c[2] * z) - c[3];
    }
}

template <typename CP>
__device__ __forceinline__ double quad_value(uint32_t type, CP c, double x, double y, double z) {
    const double dx = x - c[0], dy = y - c[1];
    if (type == ST_CZ) return (dx * dx + dy * dy) - c[2];
    const double dz = z - c[2];
    return ((dx * dx + dy * dy) + dz * dz) - c[3];
}

// Cell containment: the point is on the required side of every half-space;
// on surface force_s the logical sense force_pos is used instead.
template <typename G>
__device__ __forceinline__ bool contains(const G &g, uint32_t c, double x, double y, double z, uint32_t force_s,
                                         bool force_pos) {
    const Cell cc = ldv<Cell>(g.cell + c);
    const auto hs = g.hs + cc.hs_off;
    const uint32_t npl = cc.n_pl & kPlaneCountMask;
    for (uint32_t k = 0; k < npl; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (s == force_s) ? force_pos : (plane_value(h & 7u, g.coef + 4 * (size_t)s, x, y, z) > 0.0);
        if (pos != (bool)((h >> 3) & 1u)) return false;
    }
    for (uint32_t k = npl; k < cc.n_hs; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (s == force_s) ? force_pos : (quad_value(h & 7u, g.coef + 4 * (size_t)s, x, y, z) > 0.0);
        if (pos != (bool)((h >> 3) & 1u)) return false;
    }
    return true;
}

// Distance along (u,v,w) from q to the point where a plane's sense leaves
// the cell's required side `pos`; +inf if it does not (Table 1).
template <typename CP>
__device__ __forceinline__ double plane_den(uint32_t type, CP c, double u, double v, double w) {
    switch (type) {
    case ST_PX: return u;
    case ST_PY: return v;
    case ST_PZ: return w;
    default: return (c[0] * u + c[1] * v) + c[2] * w;
    }
}

template <typename CP>
__device__ __forceinline__ double plane_distance(uint32_t type, CP c, bool pos, double qx, double qy,
                                                 double qz, double u, double v, double w) {
    const double den = plane_den(type, c, u, v, w);
    if (den == 0.0) return dinf();
    if (!((!pos && den > 0.0) || (pos && den < 0.0))) return dinf();
    const double t = (-plane_value(type, c, qx, qy, qz)) / den;
    return (t > 0.0) ? t : 0.0;
}

// The same for a cylinder or sphere: textbook cancellation-free roots;
// `on` marks the surface just crossed (only the far root can be hit).
template <typename CP>
__device__ __forceinline__ double quad_distance(uint32_t type, CP c, bool pos, double qx, double qy,
                                                double qz, double u, double v, double w, bool on) {
    double a, b;
    const double dx = qx - c[0], dy = qy - c[1];
    if (type == ST_CZ) {
        a = u * u + v * v;
        b = dx * u + dy * v;
    } else {
        const double dz = qz - c[2];
        a = (u * u + v * v) + w * w;
        b = (dx * u + dy * v) + dz * w;
    }
    if (a == 0.0) return dinf();
    double t;
    if (on) {
        if (!(!pos && b < 0.0)) return dinf();
        t = (-2.0 * b) / a;
    } else {
        const double cc = quad_value(type, c, qx, qy, qz);
        const double disc = b * b - a * cc;
        if (!(disc > 0.0)) return dinf();
        const double q = sqrt(disc);
        if (!pos) {
            t = (b <= 0.0) ? (q - b) / a : (-cc) / (b + q);
        } else {
            if (!(b < 0.0)) return dinf();
            t = cc / (q - b);
        }
    }
    return (t > 0.0) ? t : 0.0;
}

// ------------------------------------------------------------------ search
// The cell of universe u containing (x,y,z) -- Table 1 find_cell when
// force_s == kNone, the cross_surface candidate test otherwise -- or -1.
// Mixed precision first tries the lattice-index guess at (gx, gy), then
// walks the single-precision hierarchy; double precision walks the
// double-precision hierarchy.  Whichever cell is returned passed the double
// containment test, which at most one cell of a universe passes.
template <int PREC, typename G>
__device__ int32_t search(const G &g, uint32_t u, double x, double y, double z, uint32_t force_s, bool force_pos,
                          int32_t exclude, float gx, float gy) {
    const Univ U = ldv<Univ>(g.univ + u);
    if (PREC == GT_PREC_MIXED && U.hint == (int32_t)kHintSquare) {
        int i = (int)floorf((gx - U.x0) * U.inv_px);
        int j = (int)floorf((gy - U.y0) * U.inv_py);
        i = min(max(i, 0), U.nx - 1);
        j = min(max(j, 0), U.ny - 1);
        const int32_t c = (int32_t)U.cell0 + j * U.nx + i;
        if (c != exclude && contains(g, (uint32_t)c, x, y, z, force_s, force_pos)) return c;
    }
    uint32_t n = U.node0;
    const uint32_t end = U.node0 + U.nnode;
    const float fx = (float)x, fy = (float)y, fz = (float)z;
    while (n < end) {
        bool in;
        uint32_t esc, lf;
        if (PREC == GT_PREC_MIXED) {
            const Node32 nd = ldv<Node32>(g.node32 + n);
            in = fx >= nd.lo[0] && fx <= nd.hi[0] && fy >= nd.lo[1] && fy <= nd.hi[1] && fz >= nd.lo[2] &&
                 fz <= nd.hi[2];
            esc = nd.escape;
            lf = nd.leaf;
        } else {
            const Node64 nd = ldv<Node64>(g.node64 + n);
            in = x >= nd.lo[0] && x <= nd.hi[0] && y >= nd.lo[1] && y <= nd.hi[1] && z >= nd.lo[2] && z <= nd.hi[2];
            esc = nd.escape;
            lf = nd.leaf;
        }
        if (!in) { n = esc; continue; }
        if (lf == kLeafNone) { n++; continue; }
        const uint32_t first = lf >> 4, cnt = (lf & 15u) + 1;
        for (uint32_t k = 0; k < cnt; k++) {
            const uint32_t c = g.leaf[first + k];
            if ((int32_t)c == exclude) continue;
            if (PREC == GT_PREC_MIXED) {
                const auto b = g.cbox + 8 * (size_t)c;
                if (!(fx >= b[0] && fx <= b[4] && fy >= b[1] && fy <= b[5] && fz >= b[2] && fz <= b[6])) continue;
            }
            if (contains(g, c, x, y, z, force_s, force_pos)) return (int32_t)c;
        }
        n = esc;
    }
    return -1;
}

// ------------------------------------------------------------------ particle
struct Particle {
    double x, y, z, u, v, w, tau;
    uint32_t *cell;     // LDS column: cell of level L at cell[L * blockDim.x]
    int depth;
    int on_level;
    uint32_t on_surf;
};

__device__ __forceinline__ uint32_t &lvl(const Particle &P, int L) { return P.cell[L * (int)blockDim.x]; }

// Descend from level L0 (cell set, (qx,qy,qz) its local position): while
// the cell is filled, find the daughter's cell at p - t (Alg. 7).
template <int PREC, typename G>
__device__ __forceinline__ bool descend(const G &g, Particle &P, int L0, double qx, double qy, double qz) {
    int L = L0;
    for (;;) {
        const uint32_t c = lvl(P, L);
        const int32_t fill = g.cell[c].fill;
        if (fill >= 0) break;
        const auto t = g.trans + 4 * (size_t)c;
        qx = qx - t[0];
        qy = qy - t[1];
        qz = qz - t[2];
        const int32_t d = search<PREC>(g, (uint32_t)(-fill - 1), qx, qy, qz, kNone, false, -1, (float)qx, (float)qy);
        if (d < 0) { P.depth = L + 1; return false; }
        L++;
        lvl(P, L) = (uint32_t)d;
    }
    P.depth = L + 1;
    return true;
}

template <typename G>
__device__ __forceinline__ uint32_t leaf_instance(const G &g, const Particle &P) {
    uint32_t i = 0;
    for (int L = 0; L < P.depth; L++) i += g.cell[lvl(P, L)].inst_off;
    return i;
}

// distance_to_surface over every level; ties resolve to the smallest
// (distance, level, surface id), i.e. the top-most level on the surface.
template <typename G>
__device__ __forceinline__ double distance_all(const G &g, const Particle &P, int &bl, uint32_t &bs, bool &bpos,
                                               uint32_t &bk) {
    double bt = dinf();
    bl = GT_MAX_LEVELS;
    bs = kNone;
    bpos = false;
    bk = 0;
    double qx = P.x, qy = P.y, qz = P.z;
    for (int L = 0; L < P.depth; L++) {
        const uint32_t c = lvl(P, L);
        if (L > 0) {
            const auto t = g.trans + 4 * (size_t)lvl(P, L - 1);
            qx = qx - t[0];
            qy = qy - t[1];
            qz = qz - t[2];
        }
        const Cell cc = ldv<Cell>(g.cell + c);
        const auto hs = g.hs + cc.hs_off;
        const uint32_t npl = cc.n_pl & kPlaneCountMask;
        for (uint32_t k = 0; k < npl; k++) {
            const uint32_t h = hs[k];
            const uint32_t s = h >> 4;
            const bool pos = (h >> 3) & 1u;
            if (P.on_level == L && P.on_surf == s) continue;   // a plane just crossed is not hit again
            const double d = plane_distance(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w);
            if (d < bt || (d == bt && d != dinf() && L == bl && s < bs)) {
                bt = d;
                bl = L;
                bs = s;
                bpos = pos;
                bk = cc.hs_off + k;
            }
        }
        for (uint32_t k = npl; k < cc.n_hs; k++) {
            const uint32_t h = hs[k];
            const uint32_t s = h >> 4;
            const bool pos = (h >> 3) & 1u;
            const bool on = (P.on_level == L) && (P.on_surf == s);
            const double d = quad_distance(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
            if (d < bt || (d == bt && d != dinf() && L == bl && s < bs)) {
                bt = d;
                bl = L;
                bs = s;
                bpos = pos;
                bk = cc.hs_off + k;
            }
        }
    }
    return bt;
}

// distance_to_surface as above, also returning what the segment step needs
// without reading the levels' cells again: the leaf instance and material,
// and the universe of the level that holds the nearest surface.
struct Nearest {
    double t;
    int level;
    uint32_t surf, entry, univ, inst;
    int32_t leaf_fill;
    bool pos;
};

template <typename G>
__device__ __forceinline__ void nearest_surface(const G &g, const Particle &P, Nearest &r) {
    r.t = dinf();
    r.level = GT_MAX_LEVELS;
    r.surf = kNone;
    r.entry = 0;
    r.pos = false;
    r.univ = g.root;
    r.inst = 0;
    double qx = P.x, qy = P.y, qz = P.z;
    uint32_t univ = g.root;
    int32_t fill = 0;
    for (int L = 0; L < P.depth; L++) {
        const uint32_t c = lvl(P, L);
        if (L > 0) {
            const auto t = g.trans + 4 * (size_t)lvl(P, L - 1);
            qx = qx - t[0];
            qy = qy - t[1];
            qz = qz - t[2];
            univ = (uint32_t)(-fill - 1);
        }
        const Cell cc = ldv<Cell>(g.cell + c);
        fill = cc.fill;
        r.inst += cc.inst_off;
        const auto hs = g.hs + cc.hs_off;
        const uint32_t npl = cc.n_pl & kPlaneCountMask, npair2 = 2u * (cc.n_pl >> 12);
        bool better = false;
        for (uint32_t k = 0; k < npair2; k += 2) {
            // a slab pair: the shared denominator picks the one plane that can be
            // reached (the negative-side one when it is positive); the other
            // would give no hit
            const uint32_t h0 = hs[k];
            const double den = plane_den(h0 & 7u, g.coef + 4 * (size_t)(h0 >> 4), P.u, P.v, P.w);
            if (den == 0.0) continue;
            const uint32_t kk = den > 0.0 ? k : k + 1;
            const uint32_t h = den > 0.0 ? h0 : hs[k + 1];
            const uint32_t s = h >> 4;
            if (P.on_level == L && P.on_surf == s) continue;   // a plane just crossed is not hit again
            const double t = (-plane_value(h & 7u, g.coef + 4 * (size_t)s, qx, qy, qz)) / den;
            const double d = (t > 0.0) ? t : 0.0;
            if (d < r.t || (d == r.t && d != dinf() && L == r.level && s < r.surf)) {
                r.t = d;
                r.level = L;
                r.surf = s;
                r.pos = den < 0.0;
                r.entry = cc.hs_off + kk;
                better = true;
            }
        }
        for (uint32_t k = npair2; k < npl; k++) {
            const uint32_t h = hs[k];
            const uint32_t s = h >> 4;
            const bool pos = (h >> 3) & 1u;
            if (P.on_level == L && P.on_surf == s) continue;   // a plane just crossed is not hit again
            const double d = plane_distance(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w);
            if (d < r.t || (d == r.t && d != dinf() && L == r.level && s < r.surf)) {
                r.t = d;
                r.level = L;
                r.surf = s;
                r.pos = pos;
                r.entry = cc.hs_off + k;
                better = true;
            }
        }
        for (uint32_t k = npl; k < cc.n_hs; k++) {
            const uint32_t h = hs[k];
            const uint32_t s = h >> 4;
            const bool pos = (h >> 3) & 1u;
            const bool on = (P.on_level == L) && (P.on_surf == s);
            const double d = quad_distance(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
            if (d < r.t || (d == r.t && d != dinf() && L == r.level && s < r.surf)) {
                r.t = d;
                r.level = L;
                r.surf = s;
                r.pos = pos;
                r.entry = cc.hs_off + k;
                better = true;
            }
        }
        if (better) r.univ = univ;
    }
    r.leaf_fill = fill;
}

// cross_surface at level L* on surface s* (Alg. 8) for the one-history-
// per-lane schedule: the cell of that level's universe on the other side
// (the old cell's sense on s* flipped), then descent below it.
template <int PREC, typename G>
__device__ __forceinline__ int cross(const G &g, Particle &P, int Ls, uint32_t ss, bool old_pos) {
    double qx = P.x, qy = P.y, qz = P.z;
    uint32_t univ = g.root;
    for (int L = 0; L < Ls; L++) {
        const uint32_t c = lvl(P, L);
        const auto t = g.trans + 4 * (size_t)c;
        qx = qx - t[0];
        qy = qy - t[1];
        qz = qz - t[2];
        univ = (uint32_t)(-g.cell[c].fill - 1);
    }
    const uint32_t old = lvl(P, Ls);
    // guess point nudged along the flight so that a lattice guess lands on the far side
    float gx = (float)qx, gy = (float)qy;
    if (PREC == GT_PREC_MIXED) {
        const Univ U = ldv<Univ>(g.univ + univ);
        if (U.hint == (int32_t)kHintSquare) {
            gx += (float)P.u * 1e-3f / U.inv_px;
            gy += (float)P.v * 1e-3f / U.inv_py;
        }
    }
    const int32_t c = search<PREC>(g, univ, qx, qy, qz, ss, !old_pos, (int32_t)old, gx, gy);
    if (c < 0) return Ls == 0 ? GT_END_ESCAPE : GT_END_LOST;
    lvl(P, Ls) = (uint32_t)c;
    if (!descend<PREC>(g, P, Ls, qx, qy, qz)) return GT_END_LOST;
    P.on_level = Ls;
    P.on_surf = ss;
    return GT_END_NONE;
}

// ------------------------------------------------------------------ tallies
// Segment lengths are summed as 128-bit integers in units of 2^-96 cm.  In
// the kernel a contribution is split into four 32-bit limbs, each added to
// its own 64-bit counter with an atomic whose result is not used, so no
// carry has to travel back to the lane; the counters are exact for up to
// 2^32 contributions per instance and launch.  Each XCD adds into its own
// replica of the counters, so the atomics stay in that XCD's L2; the
// finalize kernel folds replicas and limbs into the 128-bit total.
constexpr int kReplicas = 8;

__device__ __forceinline__ uint32_t xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kReplicas - 1);   // HW_REG_XCC_ID[3:0]
}

struct TallyAcc {
    uint32_t inst;
    uint64_t lo, hi;   // 128-bit register accumulator for consecutive segments in one instance
};

__device__ __forceinline__ void add_limb(uint64_t *p, uint64_t v) {
    if (v) __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)p, (unsigned long long)v,
                                  __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void tally_flush(uint64_t *rep, TallyAcc &a) {
    if (a.inst == kNone) return;
    uint64_t *p = rep + 4 * (size_t)a.inst;
    add_limb(p + 0, a.lo & 0xFFFFFFFFull);
    add_limb(p + 1, a.lo >> 32);
    add_limb(p + 2, a.hi & 0xFFFFFFFFull);
    add_limb(p + 3, a.hi >> 32);
    a.inst = kNone;
}

__device__ __forceinline__ void tally_add(uint64_t *rep, TallyAcc &a, uint32_t inst, double l) {
    const double v = l * 0x1p32;
    const double fl = floor(v);
    const double fr = v - fl;
    const uint64_t hi = (uint64_t)fl;
    const uint64_t lo = (uint64_t)(fr * 0x1p64);
    if (inst != a.inst) {
        tally_flush(rep, a);
        a.inst = inst;
        a.lo = lo;
        a.hi = hi;
    } else {
        const uint64_t nlo = a.lo + lo;
        a.hi += hi + ((nlo < a.lo) ? 1u : 0u);
        a.lo = nlo;
    }
}

struct Counts {
    uint32_t escaped, capped, lost, segcap, recovf, rejected;
    uint64_t segments;
};

__device__ __forceinline__ void count_end(Counts &cnt, int end, uint32_t segs, bool recovf) {
    cnt.segments += segs;
    cnt.escaped += end == GT_END_ESCAPE;
    cnt.capped += end == GT_END_CAP;
    cnt.lost += end == GT_END_LOST;
    cnt.segcap += end == GT_END_SEGCAP;
    cnt.recovf += recovf;
}

__device__ __forceinline__ void add_counts(const Counts &c, uint64_t *counters) {
    __shared__ unsigned long long sh[7];
    if (threadIdx.x < 7) sh[threadIdx.x] = 0;
    __syncthreads();
    if (c.escaped) atomicAdd(&sh[GT_CNT_ESCAPED], (unsigned long long)c.escaped);
    if (c.capped) atomicAdd(&sh[GT_CNT_CAPPED], (unsigned long long)c.capped);
    if (c.lost) atomicAdd(&sh[GT_CNT_LOST], (unsigned long long)c.lost);
    if (c.segcap) atomicAdd(&sh[GT_CNT_SEGCAP], (unsigned long long)c.segcap);
    if (c.recovf) atomicAdd(&sh[GT_CNT_REC_OVERFLOW], (unsigned long long)c.recovf);
    if (c.segments) atomicAdd(&sh[GT_CNT_SEGMENTS], (unsigned long long)c.segments);
    if (c.rejected) atomicAdd(&sh[GT_CNT_REJECTED], (unsigned long long)c.rejected);
    __syncthreads();
    if (threadIdx.x < 7 && sh[threadIdx.x]) atomicAdd((unsigned long long *)&counters[threadIdx.x], sh[threadIdx.x]);
}

// ------------------------------------------------------------------ plain schedule
// One history per lane: Alg. 2 with the toy transport, straight-line.
template <int PREC, typename G>
__device__ void run_history(const G &g, const KParams &p, const KOut &o, uint64_t *rep, uint64_t local,
                            uint32_t *cells, Counts &cnt) {
    Particle P;
    P.cell = cells;
    const uint64_t pid = p.first + local;
    uint32_t blk = 0;
    P.on_level = -1;
    P.on_surf = kNone;
    P.depth = 1;
    int end = GT_END_NONE;
    double u0, u1, u2;
    // ---- birth
    if (p.source == 1) {
        const uint64_t n1 = p.ray_n1;
        const uint64_t n2 = (p.n + n1 - 1) / n1;
        const uint64_t j = pid % n1, k = pid / n1;
        const double hy = (g.hi[1] - g.lo[1]) / (double)n1;
        const double hz = (g.hi[2] - g.lo[2]) / (double)n2;
        P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * 0x1p-30;
        P.y = g.lo[1] + ((double)j + 0.5) * hy;
        P.z = g.lo[2] + ((double)k + 0.5) * hz;
        P.u = 1.0;
        P.v = 0.0;
        P.w = 0.0;
        P.tau = 0.0;
        const int32_t c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, (float)P.x, (float)P.y);
        if (c < 0) {
            end = GT_END_LOST;
        } else {
            lvl(P, 0) = (uint32_t)c;
            if (!descend<PREC>(g, P, 0, P.x, P.y, P.z)) end = GT_END_LOST;
        }
    } else {
        int32_t c = -1;
        for (int a = 0; a < kMaxBirthAttempts && c < 0; a++) {
            draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
            P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * u0;
            P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * u1;
            P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * u2;
            c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, (float)P.x, (float)P.y);
            if (c < 0) cnt.rejected++;
        }
        if (c < 0) {
            end = GT_END_LOST;
        } else {
            lvl(P, 0) = (uint32_t)c;
            if (!descend<PREC>(g, P, 0, P.x, P.y, P.z)) end = GT_END_LOST;
            do draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
            while (!direction_from(u0, u1, P.u, P.v, P.w));
            P.tau = -series_log(u2);
        }
    }
    // ---- segments
    uint64_t h = kFnvOffset;
    uint32_t segs = 0, ncoll = 0;
    bool recovf = false;
    const bool recorded = local < p.rec_k;
    int32_t *rec = recorded ? o.rec + local * (uint64_t)p.rec_cap : nullptr;
    TallyAcc acc;
    acc.inst = kNone;
    acc.lo = acc.hi = 0;
    while (end == GT_END_NONE) {
        int bl;
        uint32_t bs, bk;
        bool bpos;
        const double dist = distance_all(g, P, bl, bs, bpos, bk);
        const uint32_t lc = lvl(P, P.depth - 1);
        const double sig = g.sigma[g.cell[lc].fill];
        const double sc = (p.source == 1) ? dinf() : P.tau / sig;
        const uint32_t inst = leaf_instance(g, P);
        const bool boundary = dist < sc;
        double l;
        if (boundary) {
            l = dist;
            if (p.source != 1) P.tau = P.tau - sig * dist;
        } else {
            if (sc == dinf()) { end = GT_END_LOST; break; }
            l = sc;
        }
        // move_within_cell
        const double m0 = l * P.u, m1 = l * P.v, m2 = l * P.w;
        P.x = P.x + m0;
        P.y = P.y + m1;
        P.z = P.z + m2;
        // tally and sequence
        tally_add(rep, acc, inst, l);
        h = (h ^ ((uint64_t)inst + 1)) * kFnvPrime;
        if (recorded) {
            if (segs < p.rec_cap) rec[segs] = (int32_t)inst;
            else recovf = true;
        }
        segs++;
        if (boundary) {
            end = cross<PREC>(g, P, bl, bs, bpos);
        } else {
            P.on_level = -1;
            P.on_surf = kNone;
            ncoll++;
            if (ncoll >= p.max_coll) {
                end = GT_END_CAP;
            } else {
                do draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
                while (!direction_from(u0, u1, P.u, P.v, P.w));
                P.tau = -series_log(u2);
            }
        }
        if (end == GT_END_NONE && segs >= p.max_segs) end = GT_END_SEGCAP;
    }
    tally_flush(rep, acc);
    h ^= (uint64_t)end;
    if (o.seg_count) gstore(o.seg_count, local, segs);
    if (o.seq_hash) gstore(o.seq_hash, local, h);
    if (o.end_code) gstore(o.end_code, local, end);
    count_end(cnt, end, segs, recovf);
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_track(Dev g0, KParams p, KOut o) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    const DevGlobal g = global_view(g0);
    uint64_t *rep = o.tally_ws + (size_t)xcc_id() * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t local = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (local < p.n) run_history<PREC>(g, p, o, rep, local, cells + threadIdx.x, cnt);
    add_counts(cnt, o.counters);
}

// ------------------------------------------------------------------ persistent schedule
// Each lane runs a state machine; a wave loops until the shared particle
// pool is drained and all of its lanes are idle.  Finished lanes are
// refilled at once from a wave-local pool of particle ids (ballot +
// per-lane rank, one global atomic per 64 ids), so a wave no longer waits
// for its longest history.  Per loop trip every lane takes at most one of
// each step -- draw one random block (a birth position or a direction
// attempt with its optical depth), search one level, one segment -- and
// each step has one call site, so lanes at different points of their
// histories share one instruction stream per step.
enum Mode : int { M_IDLE = 0, M_POS = 1, M_DIR = 2, M_SEARCH = 3, M_TRACK = 4 };

constexpr uint32_t kChunk = 64;
// A wave refills its idle lanes once at least this many are idle, so that
// new histories start together and their first searches (which rarely have
// a good candidate) run once for several lanes.
constexpr uint32_t kRefillMin = 8;

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Copy the plan's sections of the device blob into LDS (all lanes of the
// workgroup take part).
__device__ __forceinline__ void stage_copy(const StagePlan &sp, const unsigned char *blob, unsigned char *lds) {
    for (uint32_t k = 0; k < sp.n; k++) {
        const uint4 *src = (const uint4 *)(blob + sp.src[k]);
        uint4 *dst = (uint4 *)(lds + sp.dst[k]);
        for (uint32_t i = threadIdx.x; i < sp.bytes[k] / 16; i += blockDim.x) dst[i] = src[i];
    }
    __syncthreads();
}

// Staging kinds of a plan: nothing in LDS, the per-segment tables only, the
// per-segment and crossing tables, or every table.
// (signed, so that loops counting down over the kinds end)
enum StageKind : int { SK_NONE = 0, SK_SPLIT = 1, SK_LDS = 2, SK_ALL = 3 };

template <int KIND> struct ViewOf;
template <> struct ViewOf<SK_NONE> { typedef DevGlobal type; };
template <> struct ViewOf<SK_SPLIT> { typedef DevSplit type; };
template <> struct ViewOf<SK_LDS> { typedef DevLds type; };
template <> struct ViewOf<SK_ALL> { typedef DevAll type; };

// The view of a geometry for a kernel of staging kind KIND: staged tables at
// their LDS copies (`lds`, a workgroup-shared address), the others global.
template <int KIND>
__device__ __forceinline__ typename ViewOf<KIND>::type make_view(const Dev &g, const StagePlan &sp,
                                                                 unsigned char *lds) {
    typedef typename ViewOf<KIND>::type V;
    if constexpr (KIND == SK_NONE) {
        return global_view(g);
    } else {
        V d;
        auto lp = [&](int sec) { return lds + sp.at[sec]; };
        d.coef = (cptr<3, double>)lp(SEC_COEF);
        d.hs = (cptr<3, uint32_t>)lp(SEC_HS);
        d.cell = (cptr<3, Cell>)lp(SEC_CELL);
        d.univ = (cptr<3, Univ>)lp(SEC_UNIV);
        d.sigma = (cptr<3, double>)lp(SEC_SIGMA);
        d.cell_local = (cptr<3, uint32_t>)lp(SEC_LOCAL);
        if constexpr (KIND == SK_SPLIT) {
            d.trans = (cptr<1, double>)g.trans;
            d.adj_off = (cptr<1, uint32_t>)g.adj_off;
            d.adj = (cptr<1, uint32_t>)g.adj;
            d.node32 = (cptr<1, Node32>)g.node32;
            d.node64 = (cptr<1, Node64>)g.node64;
            d.leaf = (cptr<1, uint32_t>)g.leaf;
            d.cbox = (cptr<1, float>)g.cbox;
        } else {
            d.trans = (cptr<3, double>)lp(SEC_TRANS);
            d.adj_off = (cptr<3, uint32_t>)lp(SEC_ADJOFF);
            d.adj = (cptr<3, uint32_t>)lp(SEC_ADJ);
            if constexpr (KIND == SK_LDS) {
                d.node32 = (cptr<1, Node32>)g.node32;
                d.node64 = (cptr<1, Node64>)g.node64;
                d.leaf = (cptr<1, uint32_t>)g.leaf;
                d.cbox = (cptr<1, float>)g.cbox;
            } else {
                // only the precision mode's own hierarchy is staged; the other
                // pointer is never read
                d.node32 = (cptr<3, Node32>)lp(SEC_NODE32);
                d.node64 = (cptr<3, Node64>)lp(SEC_NODE64);
                d.leaf = (cptr<3, uint32_t>)lp(SEC_LEAF);
                d.cbox = (cptr<3, float>)lp(SEC_CBOX);
            }
        }
        view_scalars(d, g);
        return d;
    }
}

// Particle-id sources for the state machine below: a global counter over
// [0, end) for one geometry, or a workgroup (LDS) counter over one chunk of
// a batch item.  take() is called by one lane and returns the first of k ids.
struct GlobalQueue {
    unsigned long long *ctr;
    uint64_t end;
    __device__ __forceinline__ uint64_t take(uint64_t k) const { return atomicAdd(ctr, (unsigned long long)k); }
};

struct ChunkQueue {
    unsigned long long *ctr;   // LDS
    uint64_t first, end;
    __device__ __forceinline__ uint64_t take(uint64_t k) const {
        return first + atomicAdd(ctr, (unsigned long long)k);
    }
};

// Tail compaction.  Once the queue is empty for every wave of the
// workgroup, the histories still running are spread thinly over its waves.
// Every `round` loop trips the waves meet at a barrier; when the live
// histories fit in fewer waves (and in the LDS buffer), each is written to
// the buffer at its rank and read back by the lane of that rank, so fewer,
// fuller waves carry the tail while the emptied ones wait at the barrier.  A
// history's state moves as a whole, so its results do not depend on the lane
// that finishes it.
constexpr int kTailFields = 16;   // 64-bit words per moved history
constexpr uint32_t kTailRound = 8;

struct TailCfg {
    uint64_t *buf;   // LDS, kTailFields x cap words (field-major)
    uint32_t *ctl;   // LDS: [0] waves whose queue is empty, [1 + w] live lanes of wave w
    uint32_t cap;    // histories the buffer holds; 0 = no compaction
    uint32_t round;  // loop trips between compactions
};

// The persistent history loop of one lane (see above); returns when its
// wave has drained the queue and every lane of the wave is idle (with tail
// compaction: when no lane of the workgroup has a history left).
template <int PREC, typename G, typename Queue>
__device__ __forceinline__ void track_pool(const G &g, const KParams &p, const KOut &o, uint64_t *rep,
                                           uint32_t *cells, const Queue &queue, Counts &cnt, const TailCfg &tc) {
    Particle P;
    P.cell = cells;
    for (int L = 0; L < GT_MAX_LEVELS; L++) lvl(P, L) = 0;   // hints below read earlier levels
    P.x = P.y = P.z = P.u = P.v = P.w = P.tau = 0.0;
    P.depth = 1;
    P.on_level = -1;
    P.on_surf = kNone;
    int mode = M_IDLE;
    uint64_t local = 0;
    uint32_t blk = 0;
    // history state
    uint64_t h = 0;
    uint32_t segs = 0, ncoll = 0, attempts = 0;
    bool recovf = false, birth = false;
    TallyAcc acc;
    acc.inst = kNone;
    acc.lo = acc.hi = 0;
    // pending search at level sL: after a crossing, surface sforce (sense
    // sfpos forced) through half-space entry sk; kNone in a descent.  The
    // local position and universe there follow from the position and the
    // cells of the levels above, and are recomputed at each search step.
    int sL = 0;
    uint32_t sforce = kNone, sk = 0;
    bool sfpos = false;
    // wave-uniform pool of particle ids
    uint64_t pool_next = 0, pool_end = 0;
    bool drained = false;
    int end = GT_END_NONE;
    // tail compaction state (wave-uniform)
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u), nwaves = blockDim.x / 64u;
    bool counted = false, in_tail = false;
    uint32_t titer = 0;

    for (;;) {
        if (tc.cap) {
            if (drained && !counted) {
                counted = true;
                if (__lane_id() == 0) atomicAdd(&tc.ctl[0], 1u);
            }
            if (drained && !in_tail)
                in_tail = __builtin_amdgcn_readfirstlane(__atomic_load_n(&tc.ctl[0], __ATOMIC_RELAXED)) == nwaves;
            if (in_tail) {
                const uint64_t act = __ballot(mode != M_IDLE);
                if (act == 0 || ++titer >= tc.round) {
                    titer = 0;
                    if (__lane_id() == 0) tc.ctl[1 + wave] = (uint32_t)__popcll(act);
                    __syncthreads();
                    // (the counts are workgroup-uniform: read them as scalars)
                    uint32_t A = 0, busy = 0, before = 0;
                    for (uint32_t w = 0; w < nwaves; w++) {
                        const uint32_t a = __builtin_amdgcn_readfirstlane(tc.ctl[1 + w]);
                        A += a;
                        busy += a ? 1u : 0u;
                        before += w < wave ? a : 0u;
                    }
                    // every wave has read this round's counts before any wave
                    // can write the next round's
                    __syncthreads();
                    if (A == 0) break;
                    // pack the A live histories into lanes 0..A-1 of the workgroup
                    // when that frees a wave and the buffer holds them all
                    if (A <= tc.cap && (A + 63u) / 64u < busy) {
                        const uint32_t C = tc.cap;
                        if (mode != M_IDLE) {
                            tally_flush(rep, acc);
                            uint64_t *b = tc.buf + before + lane_rank(act);
                            b[0 * C] = __double_as_longlong(P.x);
                            b[1 * C] = __double_as_longlong(P.y);
                            b[2 * C] = __double_as_longlong(P.z);
                            b[3 * C] = __double_as_longlong(P.u);
                            b[4 * C] = __double_as_longlong(P.v);
                            b[5 * C] = __double_as_longlong(P.w);
                            b[6 * C] = __double_as_longlong(P.tau);
                            b[7 * C] = local;
                            b[8 * C] = h;
                            b[9 * C] = (uint64_t)blk | (uint64_t)segs << 32;
                            b[10 * C] = (uint64_t)ncoll | (uint64_t)attempts << 32;
                            b[11 * C] = (uint64_t)sforce | (uint64_t)sk << 32;
                            const uint32_t fl = (uint32_t)mode | (uint32_t)recovf << 3 | (uint32_t)birth << 4 |
                                                (uint32_t)sfpos << 5 | (uint32_t)P.depth << 8 |
                                                (uint32_t)(P.on_level + 1) << 12 | (uint32_t)sL << 16;
                            b[12 * C] = (uint64_t)P.on_surf | (uint64_t)fl << 32;
                            for (int L = 0; L < GT_MAX_LEVELS; L += 2)
                                b[(13 + L / 2) * C] = (uint64_t)lvl(P, L) | (uint64_t)lvl(P, L + 1) << 32;
                        }
                        __syncthreads();
                        if (threadIdx.x < A) {
                            const uint64_t *b = tc.buf + threadIdx.x;
                            P.x = __longlong_as_double(b[0 * C]);
                            P.y = __longlong_as_double(b[1 * C]);
                            P.z = __longlong_as_double(b[2 * C]);
                            P.u = __longlong_as_double(b[3 * C]);
                            P.v = __longlong_as_double(b[4 * C]);
                            P.w = __longlong_as_double(b[5 * C]);
                            P.tau = __longlong_as_double(b[6 * C]);
                            local = b[7 * C];
                            h = b[8 * C];
                            blk = (uint32_t)b[9 * C];
                            segs = (uint32_t)(b[9 * C] >> 32);
                            ncoll = (uint32_t)b[10 * C];
                            attempts = (uint32_t)(b[10 * C] >> 32);
                            sforce = (uint32_t)b[11 * C];
                            sk = (uint32_t)(b[11 * C] >> 32);
                            P.on_surf = (uint32_t)b[12 * C];
                            const uint32_t fl = (uint32_t)(b[12 * C] >> 32);
                            mode = (int)(fl & 7u);
                            recovf = (fl >> 3) & 1u;
                            birth = (fl >> 4) & 1u;
                            sfpos = (fl >> 5) & 1u;
                            P.depth = (int)((fl >> 8) & 15u);
                            P.on_level = (int)((fl >> 12) & 15u) - 1;
                            sL = (int)((fl >> 16) & 15u);
                            for (int L = 0; L < GT_MAX_LEVELS; L += 2) {
                                const uint64_t v = b[(13 + L / 2) * C];
                                lvl(P, L) = (uint32_t)v;
                                lvl(P, L + 1) = (uint32_t)(v >> 32);
                            }
                        } else {
                            // no history here any more (all of the old one is in the buffer)
                            mode = M_IDLE;
                            P.x = P.y = P.z = P.u = P.v = P.w = P.tau = 0.0;
                            local = h = 0;
                            blk = segs = ncoll = attempts = sk = 0;
                            sforce = P.on_surf = kNone;
                            recovf = birth = sfpos = false;
                            P.depth = 1;
                            P.on_level = -1;
                            sL = 0;
                        }
                        end = GT_END_NONE;
                    }
                    continue;
                }
            }
        }
        // ---- refill idle lanes
        if (!drained) {
            uint64_t idle = __ballot(mode == M_IDLE);
            if ((uint32_t)__popcll(idle) < p.refill_min) idle = 0;
            while (idle) {
                if (pool_next == pool_end) {
                    const int leader = __ffsll((unsigned long long)idle) - 1;
                    unsigned long long base = 0;
                    if ((int)__lane_id() == leader) base = queue.take(kChunk);
                    base = __shfl(base, leader);
                    if (base >= queue.end) { drained = true; break; }
                    pool_next = base;
                    pool_end = min((uint64_t)base + kChunk, queue.end);
                }
                const uint64_t avail = pool_end - pool_next;
                const uint32_t r = lane_rank(idle);
                if (mode == M_IDLE && r < avail) {
                    local = pool_next + r;
                    blk = 0;
                    h = kFnvOffset;
                    segs = ncoll = attempts = 0;
                    recovf = false;
                    birth = true;
                    P.on_level = -1;
                    P.on_surf = kNone;
                    P.depth = 1;
                    end = GT_END_NONE;
                    mode = M_POS;
                }
                const uint64_t nidle = (uint64_t)__popcll(idle);
                pool_next += nidle < avail ? nidle : avail;
                idle = __ballot(mode == M_IDLE);
            }
        }
        if (__ballot(mode != M_IDLE) == 0) {
            if (!tc.cap) break;
            // the queue is empty for this wave: wait for the workgroup's tail
            // (no lane holds a history: the state is dead)
            P.x = P.y = P.z = P.u = P.v = P.w = P.tau = 0.0;
            local = h = 0;
            blk = segs = ncoll = attempts = sk = 0;
            sforce = P.on_surf = kNone;
            recovf = birth = sfpos = false;
            P.depth = 1;
            P.on_level = -1;
            sL = 0;
            end = GT_END_NONE;
            __builtin_amdgcn_s_sleep(2);
            continue;
        }

        // ---- draw: a birth-position attempt, or a direction attempt and its optical depth
        if (mode == M_POS || mode == M_DIR) {
            if (mode == M_POS && p.source == 1) {
                const uint64_t n1 = p.ray_n1;
                const uint64_t n2 = (p.n + n1 - 1) / n1;
                const uint64_t pid = p.first + local;
                const uint64_t j = pid % n1, k = pid / n1;
                const double hy = (g.hi[1] - g.lo[1]) / (double)n1;
                const double hz = (g.hi[2] - g.lo[2]) / (double)n2;
                P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * 0x1p-30;
                P.y = g.lo[1] + ((double)j + 0.5) * hy;
                P.z = g.lo[2] + ((double)k + 0.5) * hz;
                P.u = 1.0;
                P.v = 0.0;
                P.w = 0.0;
                P.tau = 0.0;
            } else if (mode == M_POS && attempts >= (uint32_t)kMaxBirthAttempts) {
                end = GT_END_LOST;
            } else {
                double u0, u1, u2;
                draw_block(p.seed, p.geom_id, p.first + local, blk++, u0, u1, u2);
                if (mode == M_POS) {
                    P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * u0;
                    P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * u1;
                    P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * u2;
                    attempts++;
                } else if (direction_from(u0, u1, P.u, P.v, P.w)) {
                    P.tau = -series_log(u2);
                    mode = M_TRACK;
                }
            }
            if (mode == M_POS && end == GT_END_NONE) {
                sL = 0;
                sforce = kNone;
                mode = M_SEARCH;
            }
        }

        // ---- one level of find_cell / cross_surface
        if (mode == M_SEARCH) {
            // local position and universe at level sL (translations applied
            // level by level from the global position, as in the descent)
            double qx = P.x, qy = P.y, qz = P.z;
            uint32_t su = g.root;
            for (int L = 0; L < sL; L++) {
                const uint32_t cl = lvl(P, L);
                const auto t = g.trans + 4 * (size_t)cl;
                qx = qx - t[0];
                qy = qy - t[1];
                qz = qz - t[2];
                su = (uint32_t)(-g.cell[cl].fill - 1);
            }
            const Univ U = ldv<Univ>(g.univ + su);
            // guess point for a lattice index; after a crossing it is nudged
            // along the flight so that it lands on the far side
            float gx = (float)qx, gy = (float)qy;
            if (PREC == GT_PREC_MIXED && sforce != kNone && U.hint == (int32_t)kHintSquare) {
                gx += (float)P.u * 1e-3f / U.inv_px;
                gy += (float)P.v * 1e-3f / U.inv_py;
            }
            // quick candidates first: after a crossing, the cells listed for the
            // crossed half-space; in a descent, the cell with the same index in
            // the new universe as the lane had at this level before
            uint32_t k0, k1, hint = 0;
            int32_t excl = -1;
            if (sforce != kNone) {
                k0 = g.adj_off[sk];
                k1 = g.adj_off[sk + 1];
                excl = (int32_t)lvl(P, sL);   // the cell being left
            } else {
                const uint32_t loc = g.cell_local[lvl(P, sL)];
                hint = U.cell0 + loc;
                k0 = 0;
                k1 = loc < U.ncell ? 1u : 0u;
            }
            int32_t c = -1;
            for (uint32_t k = k0; k < k1; k++) {
                const uint32_t d = sforce != kNone ? g.adj[k] : hint;
                if (contains(g, d, qx, qy, qz, sforce, sfpos)) { c = (int32_t)d; break; }
            }
            if (c < 0) c = search<PREC>(g, su, qx, qy, qz, sforce, sfpos, excl, gx, gy);
            if (c < 0) {
                if (birth) {
                    if (sL == 0 && p.source != 1) { cnt.rejected++; mode = M_POS; }
                    else end = GT_END_LOST;
                } else {
                    end = (sforce != kNone && sL == 0) ? GT_END_ESCAPE : GT_END_LOST;
                }
            } else {
                lvl(P, sL) = (uint32_t)c;
                if (g.cell[c].fill < 0) {
                    sL++;
                    sforce = kNone;
                } else {
                    P.depth = sL + 1;
                    if (birth) {
                        birth = false;
                        mode = p.source == 1 ? M_TRACK : M_DIR;
                    } else {
                        if (segs >= p.max_segs) end = GT_END_SEGCAP;
                        mode = M_TRACK;
                    }
                }
            }
        }

        // ---- one segment: distance_to_surface, move, tally, then crossing or collision
        if (mode == M_TRACK && end == GT_END_NONE) {
            Nearest nr;
            nearest_surface(g, P, nr);
            const double sig = g.sigma[nr.leaf_fill];
            const double sc = (p.source == 1) ? dinf() : P.tau / sig;
            const uint32_t inst = nr.inst;
            const bool boundary = nr.t < sc;
            if (!boundary && sc == dinf()) {
                end = GT_END_LOST;
            } else {
                double l;
                if (boundary) {
                    l = nr.t;
                    if (p.source != 1) P.tau = P.tau - sig * nr.t;
                } else {
                    l = sc;
                }
                const double m0 = l * P.u, m1 = l * P.v, m2 = l * P.w;
                P.x = P.x + m0;
                P.y = P.y + m1;
                P.z = P.z + m2;
                tally_add(rep, acc, inst, l);
                h = (h ^ ((uint64_t)inst + 1)) * kFnvPrime;
                if (local < p.rec_k) {
                    if (segs < p.rec_cap) gstore(o.rec, local * (uint64_t)p.rec_cap + segs, inst);
                    else recovf = true;
                }
                segs++;
                if (boundary) {
                    // cross_surface at level nr.level on surface nr.surf (Alg. 8),
                    // at the local position there of the moved global position
                    sL = nr.level;
                    sforce = nr.surf;
                    sfpos = !nr.pos;
                    sk = nr.entry;
                    P.on_level = nr.level;
                    P.on_surf = nr.surf;
                    mode = M_SEARCH;
                } else {
                    P.on_level = -1;
                    P.on_surf = kNone;
                    ncoll++;
                    if (ncoll >= p.max_coll) end = GT_END_CAP;
                    else if (segs >= p.max_segs) end = GT_END_SEGCAP;
                    else mode = M_DIR;
                }
            }
        }

        // ---- history finished: outputs, then the lane is free
        if (mode != M_IDLE && end != GT_END_NONE) {
            tally_flush(rep, acc);
            h ^= (uint64_t)end;
            if (o.seg_count) gstore(o.seg_count, local, segs);
            if (o.seq_hash) gstore(o.seq_hash, local, h);
            if (o.end_code) gstore(o.end_code, local, end);
            count_end(cnt, end, segs, recovf);
            mode = M_IDLE;
        }
    }
}

// Dynamic LDS of the persistent kernels: the level columns, the staged
// tables at byte offset tables_at, then the tail buffer at tail_at.
// KIND = staging kind of the geometry's plan (see make_view); W = waves per
// SIMD the register budget is cut for: 4 (up to 1024 lanes per workgroup,
// 128 registers) or 5 (640 lanes, two workgroups per compute unit, 96
// registers).
template <int PREC, int KIND, int W>
__global__ void __launch_bounds__(W == 5 ? 640 : kBlockP) __attribute__((amdgpu_waves_per_eu(W)))
k_track_persistent(const GeomDesc *__restrict__ gd, const LaunchRec *__restrict__ lr, uint32_t tables_at,
                   uint32_t tail_at, uint32_t tail_cap, uint32_t tail_round) {
    __shared__ uint32_t ctl[1 + kBlockP / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_dyn[];
    uint32_t *cells = (uint32_t *)lds_dyn;   // the cell of each level, one column per lane
    unsigned char *lds_tables = lds_dyn + tables_at;
    if (threadIdx.x == 0) ctl[0] = 0;
    if (KIND != SK_NONE) stage_copy(gd->stage[PREC], (const unsigned char *)gd->dev.coef, lds_tables);
    else __syncthreads();
    const auto g = make_view<KIND>(gd->dev, gd->stage[PREC], lds_tables);
    const KParams &p = lr->p;
    const KOut &o = lr->o;
    uint64_t *rep = o.tally_ws + (size_t)xcc_id() * 4 * g.n_inst;
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const GlobalQueue q = {(unsigned long long *)&o.counters[7], p.n};
    const TailCfg tc = {(uint64_t *)(lds_dyn + tail_at), ctl, tail_cap, tail_round};
    track_pool<PREC>(g, p, o, rep, cells + threadIdx.x, q, cnt, tc);
    add_counts(cnt, o.counters);
}

// Store a launch's parameters for the tracker that follows on the stream.
__global__ void k_put_launch(LaunchRec r, LaunchRec *dst) {
    if (threadIdx.x == 0) *dst = r;
}

// Many geometries in one persistent launch: each workgroup takes chunks
// (item, range of particle indices) from a device queue, copies the item's
// tables into LDS when the item changes (KIND), and runs the lanes' state
// machine over the chunk with a workgroup-local id counter.
template <int PREC, int KIND, int W>
__global__ void __launch_bounds__(W == 5 ? 640 : kBlockP) __attribute__((amdgpu_waves_per_eu(W)))
k_track_batch(const BatchItem *__restrict__ items,
                                                         const BatchChunk *__restrict__ chunks,
                                                         uint32_t n_chunks, unsigned long long *queue,
                                                         uint32_t tables_at, uint32_t tail_at, uint32_t tail_cap,
                                                         uint32_t tail_round) {
    __shared__ uint32_t ctl[1 + kBlockP / 64];
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_dyn[];
    __shared__ uint32_t s_chunk;
    __shared__ unsigned long long s_pool;
    uint32_t *cells = (uint32_t *)lds_dyn;   // the cell of each level, one column per lane
    unsigned char *lds_tables = lds_dyn + tables_at;
    const TailCfg tc = {(uint64_t *)(lds_dyn + tail_at), ctl, tail_cap, tail_round};
    // the descriptors are read-only for the whole launch: their fields are
    // read where needed (scalar loads the compiler may repeat) rather than
    // carried from chunk to chunk in registers
    uint32_t cur = 0xFFFFFFFFu;
    for (;;) {
        if (threadIdx.x == 0) {
            s_chunk = (uint32_t)atomicAdd(queue, 1ull);
            s_pool = 0;
            ctl[0] = 0;
        }
        __syncthreads();
        const uint32_t c = __builtin_amdgcn_readfirstlane(s_chunk);
        if (c >= n_chunks) break;
        const uint32_t item = chunks[c].item;
        const uint64_t first = chunks[c].first, count = chunks[c].count;
        const BatchItem &it = items[item];
        if (KIND != SK_NONE && item != cur) stage_copy(it.plan, (const unsigned char *)it.dev.coef, lds_tables);
        cur = item;
        const auto g = make_view<KIND>(it.dev, it.plan, lds_tables);
        const KParams &p = it.p;
        const KOut &o = it.o;
        uint64_t *rep = o.tally_ws + (size_t)xcc_id() * 4 * g.n_inst;
        Counts cnt = {0, 0, 0, 0, 0, 0, 0};
        const ChunkQueue q = {&s_pool, first, first + count};
        track_pool<PREC>(g, p, o, rep, cells + threadIdx.x, q, cnt, tc);
        add_counts(cnt, o.counters);
        __syncthreads();
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

// Fold the replicas' limb counters of instance i into the 128-bit
// fixed-point total (plus the previous total when accumulating), then convert
// it to cm: high word * 2^-32 + low word * 2^-96.
__device__ __forceinline__ void fold_tally(const uint64_t *ws, uint64_t *tfx, double *tally, uint64_t n, uint64_t i,
                                           bool accumulate) {
    uint64_t lo = accumulate ? tfx[2 * i] : 0, hi = accumulate ? tfx[2 * i + 1] : 0;
    for (int r = 0; r < kReplicas; r++) {
        const uint64_t *L = ws + ((size_t)r * n + i) * 4;
        for (int k = 0; k < 4; k++) {
            // add L[k] * 2^(32 k) to (hi, lo) modulo 2^128
            const uint64_t v = L[k];
            uint64_t add_lo, add_hi;
            switch (k) {
            case 0: add_lo = v; add_hi = 0; break;
            case 1: add_lo = v << 32; add_hi = v >> 32; break;
            case 2: add_lo = 0; add_hi = v; break;
            default: add_lo = 0; add_hi = v << 32; break;
            }
            const uint64_t nlo = lo + add_lo;
            hi += add_hi + (nlo < lo ? 1u : 0u);
            lo = nlo;
        }
    }
    tfx[2 * i] = lo;
    tfx[2 * i + 1] = hi;
    if (tally) tally[i] = (double)hi * 0x1p-32 + (double)lo * 0x1p-96;
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
    const int32_t c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, (float)P.x, (float)P.y);
    if (c >= 0) {
        lvl(P, 0) = (uint32_t)c;
        ok = descend<PREC>(g, P, 0, P.x, P.y, P.z);
    }
    inst[i] = ok ? (int64_t)leaf_instance(g, P) : -1;
    if (cells)
        for (int L = 0; L < GT_MAX_LEVELS; L++)
            cells[i * GT_MAX_LEVELS + L] = (c >= 0 && L < P.depth) ? (int32_t)lvl(P, L) : -1;
}

__global__ void __launch_bounds__(kBlock) k_distance(Dev g0, const double *pos, const double *dir, uint64_t n,
                                                     double *dist, int32_t *level, int32_t *surf) {
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
    const int32_t c = search<GT_PREC_FP64>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.f, 0.f);
    bool ok = false;
    if (c >= 0) {
        lvl(P, 0) = (uint32_t)c;
        ok = descend<GT_PREC_FP64>(g, P, 0, P.x, P.y, P.z);
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
    static const void *done[16];
    static int used = 0;
    for (int i = 0; i < used; i++)
        if (done[i] == kernel) return GT_OK;
    int rc = hip_check(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes),
                       "hipFuncSetAttribute");
    if (rc) return rc;
    if (used < 16) done[used++] = kernel;
    return GT_OK;
}

// LDS of a persistent launch: the staged tables (if any), then the tail
// buffer, as large as the workgroup's share of the compute unit's LDS allows
// without lowering the number of resident workgroups.
struct LdsPlan {
    unsigned dyn, tables_at, tail_at, tail_cap;
    int blocks;
};

constexpr unsigned kLdsPerCU = 160 * 1024;

int plan_persistent(const void *kern, unsigned block, unsigned tables, bool tail, int device, LdsPlan &lp) {
    hipFuncAttributes fa;
    int rc = hip_check(hipFuncGetAttributes(&fa, kern), "hipFuncGetAttributes");
    if (rc) return rc;
    const unsigned stat = (unsigned)fa.sharedSizeBytes;
    if (stat + GT_MAX_LEVELS * 4u * block + tables + 32u > kLdsPerCU)
        return set_error("staged tables exceed the LDS"), GT_ECAPACITY;
    rc = allow_dynamic_lds(kern, kLdsPerCU - stat);
    if (rc) return rc;
    // dynamic LDS: level columns, staged tables, tail buffer
    const unsigned tables_at = (GT_MAX_LEVELS * 4u * block + 15u) & ~15u;
    const unsigned base = tables_at + ((tables + 15u) & ~15u);
    int blocks = 0;
    rc = persistent_grid(kern, block, base, device, &blocks);
    if (rc) return rc;
    int cus = 0;
    rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    if (rc) return rc;
    const unsigned per = (unsigned)std::max(1, blocks / std::max(cus, 1));
    unsigned cap = 0;
    if (tail && block > 64) {
        const long avail = (long)(kLdsPerCU / per) - (long)stat - (long)base - 512;
        if (avail > 0) cap = std::min<unsigned>((unsigned)(avail / (kTailFields * 8)), block);
        if (cap < 64) cap = 0;
    }
    unsigned dyn = base + cap * kTailFields * 8;
    if (cap) {
        int b2 = 0;
        rc = persistent_grid(kern, block, dyn, device, &b2);
        if (rc) return rc;
        if (b2 < blocks) {   // the buffer would cost a resident workgroup: go without
            cap = 0;
            dyn = base;
        }
    }
    lp.dyn = dyn;
    lp.tables_at = tables_at;
    lp.tail_at = base;
    lp.tail_cap = cap;
    lp.blocks = blocks;
    return GT_OK;
}


// Events recorded around the tracking kernels of this thread's next launches
// (set by gt_set_kernel_events; both null = off).
thread_local hipEvent_t t_ev_start = nullptr, t_ev_stop = nullptr;

inline void mark(hipEvent_t e, hipStream_t st) {
    if (e) (void)hipEventRecord(e, st);
}

// One persistent tracker launch for a geometry of staging kind KIND.
template <int PREC, int KIND, int W>
int launch_persistent_k(const gt_geometry *g, uint64_t n, unsigned block, bool tail, hipStream_t st) {
    const void *kern = (const void *)k_track_persistent<PREC, KIND, W>;
    LdsPlan lp;
    int rc = plan_persistent(kern, block, KIND == SK_NONE ? 0 : g->stage[PREC].total, tail, g->device, lp);
    if (rc) return rc;
    int blocks = lp.blocks;
    const uint64_t need = (n + block - 1) / block;
    if ((uint64_t)blocks > need) blocks = (int)need;
    hipLaunchKernelGGL((k_track_persistent<PREC, KIND, W>), dim3(blocks), dim3(block), lp.dyn, st, g->desc,
                       (const LaunchRec *)g->launch, lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound);
    return GT_OK;
}

template <int PREC, int W>
int launch_persistent(const gt_geometry *g, int kind, uint64_t n, unsigned block, bool tail, hipStream_t st) {
    switch (kind) {
    case SK_ALL: return launch_persistent_k<PREC, SK_ALL, W>(g, n, block, tail, st);
    case SK_LDS: return launch_persistent_k<PREC, SK_LDS, W>(g, n, block, tail, st);
    case SK_SPLIT: return launch_persistent_k<PREC, SK_SPLIT, W>(g, n, block, tail, st);
    default: return launch_persistent_k<PREC, SK_NONE, W>(g, n, block, tail, st);
    }
}

// The chunks of one staging kind of a batch, in one launch.
template <int PREC, int KIND, int W>
int launch_batch_k(gt_batch *b, const BatchChunk *ch, uint32_t n, unsigned long long *q, hipStream_t st) {
    const void *kern = (const void *)k_track_batch<PREC, KIND, W>;
    LdsPlan lp;
    int rc = plan_persistent(kern, b->block, b->lds_bytes[KIND], b->tail, b->device, lp);
    if (rc) return rc;
    int blocks = lp.blocks;
    if ((uint32_t)blocks > n) blocks = (int)n;
    hipLaunchKernelGGL((k_track_batch<PREC, KIND, W>), dim3(blocks), dim3(b->block), lp.dyn, st, b->d_items, ch, n, q,
                       lp.tables_at, lp.tail_at, lp.tail_cap, kTailRound);
    return GT_OK;
}

template <int PREC, int W>
int launch_batch_kinds(gt_batch *b, hipStream_t st) {
    uint32_t first = 0;
    for (int kind = 3; kind >= 0; kind--) {   // chunk groups in the order gt_batch_create wrote them
        const uint32_t n = b->n_kind[kind];
        const BatchChunk *ch = b->d_chunks + first;
        unsigned long long *q = b->d_queue + kind;
        first += n;
        if (!n) continue;
        int rc = kind == SK_ALL     ? launch_batch_k<PREC, SK_ALL, W>(b, ch, n, q, st)
                 : kind == SK_LDS   ? launch_batch_k<PREC, SK_LDS, W>(b, ch, n, q, st)
                 : kind == SK_SPLIT ? launch_batch_k<PREC, SK_SPLIT, W>(b, ch, n, q, st)
                                    : launch_batch_k<PREC, SK_NONE, W>(b, ch, n, q, st);
        if (rc) return rc;
    }
    if (first != b->n_chunks) return set_error("gt_batch_launch: inconsistent chunk groups"), GT_EINVAL;
    return GT_OK;
}

template <int PREC>
int launch_track_t(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, hipStream_t st) {
    KParams kp;
    KOut ko;
    fill_kparams(p, g, kp, ko, o);
    const uint64_t nws = (uint64_t)kReplicas * 4 * g->n_inst;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(nws)), dim3(256), 0, st, g->tally_ws, nws, (uint64_t)0);
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
            hipLaunchKernelGGL(k_put_launch, dim3(1), dim3(64), 0, st, rec, g->launch);
            const bool tail = !(p->flags & GT_FLAG_NO_TAIL_COMPACTION);
            int rc = block == 640 ? launch_persistent<PREC, 5>(g, kind, kp.n, block, tail, st)
                                  : launch_persistent<PREC, 4>(g, kind, kp.n, block, tail, st);
            if (rc) return rc;
        }
    }
    mark(t_ev_stop, st);
    hipLaunchKernelGGL(k_finalize, dim3(fill_grid(g->n_inst)), dim3(256), 0, st, (const uint64_t *)g->tally_ws,
                       o->tally_fx, o->tally, g->n_inst, (int)((p->flags & GT_FLAG_ACCUMULATE) != 0));
    return hip_check(hipGetLastError(), "gt_track launch");
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

void fill_kparams(const gt_track_params *p, const gt_geometry *g, KParams &kp, KOut &ko, const gt_track_out *o) {
    kp.seed = p->seed;
    kp.first = p->first_particle;
    kp.n = p->n_particles;
    kp.geom_id = p->geometry_id;
    kp.max_coll = p->max_collisions;
    kp.source = p->source;
    kp.ray_n1 = p->ray_n1;
    kp.max_segs = p->max_segments;
    kp.rec_k = (uint32_t)((uint64_t)p->record_first_k < p->n_particles ? p->record_first_k : p->n_particles);
    kp.rec_cap = p->record_cap;
    kp.refill_min = p->refill_min ? p->refill_min : kRefillMin;
    ko.tally_ws = g->tally_ws;
    ko.seg_count = o->seg_count;
    ko.seq_hash = o->seq_hash;
    ko.end_code = o->end_code;
    ko.rec = o->rec;
    ko.counters = o->counters;
}

unsigned stage_budget() { return kStageBudget; }

void set_kernel_events(void *start, void *stop) {
    t_ev_start = (hipEvent_t)start;
    t_ev_stop = (hipEvent_t)stop;
}

int launch_batch(gt_batch *b, void *stream) {
    if (b->block > (uint32_t)kBlockP) return set_error("gt_batch_launch: block_size too large"), GT_EINVAL;
    return b->precision == GT_PREC_MIXED ? launch_batch_t<GT_PREC_MIXED>(b, (hipStream_t)stream)
                                         : launch_batch_t<GT_PREC_FP64>(b, (hipStream_t)stream);
}

int launch_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    if ((p->flags & GT_FLAG_LANE_PER_HISTORY) && p->block_size > (uint32_t)kBlock)
        return set_error("gt_track: block_size must be at most %d with GT_FLAG_LANE_PER_HISTORY", kBlock), GT_EINVAL;
    if (p->n_particles > (uint64_t)0x7FFFFFFF * 64ull) return set_error("gt_track: too many particles"), GT_ECAPACITY;
    return p->precision == GT_PREC_MIXED ? launch_track_t<GT_PREC_MIXED>(g, p, o, st)
                                         : launch_track_t<GT_PREC_FP64>(g, p, o, st);
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

int launch_distance(const gt_geometry *g, const double *pos, const double *dir, uint64_t n, double *dist,
                    int32_t *level, int32_t *surf, void *stream) {
    if (!n) return GT_OK;
    hipLaunchKernelGGL(k_distance, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, (hipStream_t)stream, g->dev, pos, dir, n,
                       dist, level, surf);
    return hip_check(hipGetLastError(), "gt_distance_to_surface launch");
}

int launch_fp64_check(const double *a, const double *b, uint64_t n, double *q, double *r, double *l, void *stream) {
    if (!n) return GT_OK;
    hipLaunchKernelGGL(k_fp64_check, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, a, b, n, q, r, l);
    return hip_check(hipGetLastError(), "gt_fp64_check launch");
}

}  // namespace gt
