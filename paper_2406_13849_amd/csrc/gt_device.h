// Device functions of the tracker (everything below the kernels): table
// views, random numbers, surfaces, search, distances, tallies and the
// persistent per-lane state machine.  Included by gt_track.hip; the tests
// also compile it for the host, with one-lane stand-ins for the wave
// intrinsics and GT_AS defined empty, to check the per-lane logic against
// the oracle on a CPU.
//
// Floating point: compiled with -ffp-contract=off and no fast-math, so every
// double operation below is one IEEE operation in the order written; the
// results of find_cell / distance_to_surface / cross_surface are the ones a
// plain double-precision implementation of the same definitions computes.
// Single precision only appears in the optional candidate pruning (widened,
// outward-rounded boxes and a lattice-index guess), which can skip a cell
// only when that cell cannot contain the point.
#pragma once
#pragma clang fp contract(off)

#include "gt_internal.h"

// Address-space qualifier of typed table pointers (LDS = 3, global = 1).
#ifndef GT_AS
#define GT_AS(n) __attribute__((address_space(n)))
#endif

namespace gt {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxBirthAttempts = 1000;
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;
constexpr int kBlock = 256;     // lanes per workgroup of the one-history-per-lane kernels

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// ------------------------------------------------------------------ table views
// The kernels read the geometry tables through pointers whose address space
// is part of their type, so the compiler emits LDS reads (32-bit addresses)
// for tables staged in LDS and global loads for the others, instead of flat
// loads that must serve both.  A view DevT<A, B, C> holds the per-segment
// tables (cells, half-spaces, surfaces, universes, materials, local indices)
// in address space A, the crossing tables (translations, candidate lists) in
// B and the hierarchy (nodes, leaves, cell boxes) in C; 3 = LDS, 1 = global.
// S is the set of surface types the code handles (SF_ALL, SF_AXCZ or
// SF_VERT; see gt_internal.h): the surface functions below are compiled for
// that set alone.
template <int AS, typename T> using cptr = const GT_AS(AS) T *;

template <int A, int B, int C, int S = SF_ALL>
struct DevT {
    static constexpr int kSurf = S;
    cptr<A, double> coef;
    cptr<A, uint32_t> hs;
    cptr<A, Cell> cell;
    cptr<A, Univ> univ;
    cptr<A, double> sigma;
    cptr<A, uint32_t> cell_local;
    // universe-kind tables (read only by the trackers that switch on kind;
    // staged with the per-segment tables in their plans)
    cptr<A, UArr> uarr;
    cptr<A, double> aval;
    cptr<A, uint32_t> asurf;
    cptr<A, uint32_t> ahs;
    cptr<A, uint32_t> cell_ij;
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
    ((GT_AS(1) T *)base)[i] = (T)v;
}

// A whole record through a typed pointer (the copy goes through a generic
// pointer cast from the typed one, which keeps the address space).
template <typename T, typename P>
__device__ __forceinline__ T ldv(P p) {
    return *(const T *)p;
}

template <int A, int B, int C, int S>
__device__ __forceinline__ void view_scalars(DevT<A, B, C, S> &d, const Dev &g) {
    d.root = g.root;
    d.n_inst = g.n_inst;
    d.max_depth = g.max_depth;
    d.n_cells = g.n_cells;
    for (int k = 0; k < 3; k++) {
        d.lo[k] = g.lo[k];
        d.hi[k] = g.hi[k];
    }
}

template <int S = SF_ALL>
__device__ __forceinline__ DevT<1, 1, 1, S> global_view(const Dev &g) {
    DevT<1, 1, 1, S> d;
    d.coef = (cptr<1, double>)g.coef;
    d.hs = (cptr<1, uint32_t>)g.hs;
    d.cell = (cptr<1, Cell>)g.cell;
    d.univ = (cptr<1, Univ>)g.univ;
    d.sigma = (cptr<1, double>)g.sigma;
    d.cell_local = (cptr<1, uint32_t>)g.cell_local;
    d.uarr = (cptr<1, UArr>)g.uarr;
    d.aval = (cptr<1, double>)g.aval;
    d.asurf = (cptr<1, uint32_t>)g.asurf;
    d.ahs = (cptr<1, uint32_t>)g.ahs;
    d.cell_ij = (cptr<1, uint32_t>)g.cell_ij;
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
template <int SF, typename CP>
__device__ __forceinline__ double plane_value(uint32_t type, CP c, double x, double y, double z) {
    if constexpr (SF == SF_AXCZ) {
        switch (type) {
        case ST_PX: return x - c[0];
        case ST_PY: return y - c[0];
        default: return z - c[0];
        }
    } else if constexpr (SF == SF_VERT) {
        switch (type) {
        case ST_PX: return x - c[0];
        case ST_PY: return y - c[0];
        case ST_PZ: return z - c[0];
        default: return (c[0] * x + c[1] * y) - c[3];
        }
    } else {
        switch (type) {
        case ST_PX: return x - c[0];
        case ST_PY: return y - c[0];
        case ST_PZ: return z - c[0];
        default: return ((c[0] * x + c[1] * y) + c[2] * z) - c[3];
        }
    }
}

// plane_value split as linear part minus offset (the same operations):
// the coordinate, or ((a x + b y) + c z); then d.
template <int SF, typename CP>
__device__ __forceinline__ double plane_linear(uint32_t type, CP c, double x, double y, double z) {
    if constexpr (SF == SF_AXCZ) {
        switch (type) {
        case ST_PX: return x;
        case ST_PY: return y;
        default: return z;
        }
    } else if constexpr (SF == SF_VERT) {
        switch (type) {
        case ST_PX: return x;
        case ST_PY: return y;
        case ST_PZ: return z;
        default: return c[0] * x + c[1] * y;
        }
    } else {
        switch (type) {
        case ST_PX: return x;
        case ST_PY: return y;
        case ST_PZ: return z;
        default: return (c[0] * x + c[1] * y) + c[2] * z;
        }
    }
}

template <int SF, typename CP>
__device__ __forceinline__ double plane_offset(uint32_t type, CP c) {
    if constexpr (SF == SF_AXCZ) return c[0];
    else return type == ST_P ? c[3] : c[0];
}

template <int SF, typename CP>
__device__ __forceinline__ double quad_value(uint32_t type, CP c, double x, double y, double z) {
    const double dx = x - c[0], dy = y - c[1];
    if (SF != SF_ALL || type == ST_CZ) return (dx * dx + dy * dy) - c[2];
    const double dz = z - c[2];
    return ((dx * dx + dy * dy) + dz * dz) - c[3];
}

// Cell containment: the point is on the required side of every half-space;
// on surface force_s the logical sense force_pos is used instead.
template <typename G>
__device__ __forceinline__ bool contains(const G &g, uint32_t c, double x, double y, double z, uint32_t force_s,
                                         bool force_pos, int32_t &fill) {
    const Cell cc = ldv<Cell>(g.cell + c);
    fill = cc.fill;
    const auto hs = g.hs + cc.hs_off;
    const uint32_t npl = cc.n_pl & kPlaneCountMask, npair2 = 2u * (cc.n_pl >> 12);
    for (uint32_t k = 0; k < npair2; k += 2) {
        // a slab pair: one plane family, so both planes' values take the same
        // coordinate, or the same dot product with their bitwise-identical
        // normal, minus their own offsets (the arithmetic of plane_value)
        const uint32_t h0 = hs[k], h1 = hs[k + 1];
        const uint32_t s0 = h0 >> 4, s1 = h1 >> 4, t = h0 & 7u;
        const auto c0 = g.coef + 4 * (size_t)s0, c1 = g.coef + 4 * (size_t)s1;
        const double lin = plane_linear<G::kSurf>(t, c0, x, y, z);
        const bool p0 = (s0 == force_s) ? force_pos : (lin - plane_offset<G::kSurf>(t, c0) > 0.0);
        const bool p1 = (s1 == force_s) ? force_pos : (lin - plane_offset<G::kSurf>(t, c1) > 0.0);
        if (p0 != (bool)((h0 >> 3) & 1u) || p1 != (bool)((h1 >> 3) & 1u)) return false;
    }
    for (uint32_t k = npair2; k < npl; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (s == force_s) ? force_pos : (plane_value<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, x, y, z) > 0.0);
        if (pos != (bool)((h >> 3) & 1u)) return false;
    }
    for (uint32_t k = npl; k < cc.n_hs; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (s == force_s) ? force_pos : (quad_value<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, x, y, z) > 0.0);
        if (pos != (bool)((h >> 3) & 1u)) return false;
    }
    return true;
}

template <typename G>
__device__ __forceinline__ bool contains(const G &g, uint32_t c, double x, double y, double z, uint32_t force_s,
                                         bool force_pos) {
    int32_t fill;
    return contains(g, c, x, y, z, force_s, force_pos, fill);
}

// Distance along (u,v,w) from q to the point where a plane's sense leaves
// the cell's required side `pos`; +inf if it does not (Table 1).
template <int SF, typename CP>
__device__ __forceinline__ double plane_den(uint32_t type, CP c, double u, double v, double w) {
    if constexpr (SF == SF_AXCZ) {
        switch (type) {
        case ST_PX: return u;
        case ST_PY: return v;
        default: return w;
        }
    } else if constexpr (SF == SF_VERT) {
        switch (type) {
        case ST_PX: return u;
        case ST_PY: return v;
        case ST_PZ: return w;
        default: return c[0] * u + c[1] * v;
        }
    } else {
        switch (type) {
        case ST_PX: return u;
        case ST_PY: return v;
        case ST_PZ: return w;
        default: return (c[0] * u + c[1] * v) + c[2] * w;
        }
    }
}

template <int SF, typename CP>
__device__ __forceinline__ double plane_distance(uint32_t type, CP c, bool pos, double qx, double qy,
                                                 double qz, double u, double v, double w) {
    const double den = plane_den<SF>(type, c, u, v, w);
    if (den == 0.0) return dinf();
    if (!((!pos && den > 0.0) || (pos && den < 0.0))) return dinf();
    const double t = (-plane_value<SF>(type, c, qx, qy, qz)) / den;
    return (t > 0.0) ? t : 0.0;
}

// The same for a cylinder or sphere: textbook cancellation-free roots;
// `on` marks the surface just crossed (only the far root can be hit).
// Written without branches: every case's operands are formed, and the one
// division takes those of the case that applies, so the quotient is the one
// the case-by-case formula gives (lanes of a wave often take different cases).
__device__ __forceinline__ double quad_root(double a, double b, double cc, bool pos, bool on);

template <int SF, typename CP>
__device__ __forceinline__ double quad_distance(uint32_t type, CP c, bool pos, double qx, double qy,
                                                double qz, double u, double v, double w, bool on) {
    const bool cyl = SF != SF_ALL || type == ST_CZ;
    const double c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3];
    const double dx = qx - c0, dy = qy - c1, dz = qz - c2;
    const double a2 = u * u + v * v, b2 = dx * u + dy * v, r2 = dx * dx + dy * dy;
    const double a = cyl ? a2 : a2 + w * w;
    const double b = cyl ? b2 : b2 + dz * w;
    const double cc = cyl ? r2 - c2 : (r2 + dz * dz) - c3;
    return quad_root(a, b, cc, pos, on);
}

// The root step of quad_distance from the quadratic's a, b (half the linear
// coefficient) and c = f(q); shared with the pin tracker, which forms a, b
// and the squared radius once for all cylinders of a pin.
__device__ __forceinline__ double quad_root(double a, double b, double cc, bool pos, bool on) {
    const double disc = b * b - a * cc;
    const double q = sqrt(disc > 0.0 ? disc : 0.0);
    double num, den;
    bool hit;
    if (on) {
        hit = !pos && b < 0.0;
        num = -2.0 * b;
        den = a;
    } else if (!pos) {
        hit = disc > 0.0;
        num = (b <= 0.0) ? q - b : -cc;
        den = (b <= 0.0) ? a : b + q;
    } else {
        hit = disc > 0.0 && b < 0.0;
        num = cc;
        den = q - b;
    }
    const double t = num / den;
    return (hit && a != 0.0) ? ((t > 0.0) ? t : 0.0) : dinf();
}

// ------------------------------------------------------------------ search
// The cell of universe u containing (x,y,z) -- Table 1 find_cell when
// force_s == kNone, the cross_surface candidate test otherwise -- or -1.
// Mixed precision first tries the lattice-index guess, then walks the
// single-precision hierarchy; double precision walks the double-precision
// hierarchy.  The guess is taken at (x + nu * pitch, y + nv * pitch) in
// single precision: after a crossing (nu, nv) is a small step along the
// flight, so that the guess lands on the far side.  Whichever cell is
// returned passed the double containment test, which at most one cell of a
// universe passes.  The cell's fill is returned in *fill.
template <int PREC, typename G>
__device__ int32_t search(const G &g, uint32_t u, double x, double y, double z, uint32_t force_s, bool force_pos,
                          int32_t exclude, float nu, float nv, int32_t &fill) {
    const Univ U = ldv<Univ>(g.univ + u);
    if (PREC == GT_PREC_MIXED && U.hint == (int32_t)kHintSquare) {
        const float gx = (float)x + nu / U.inv_px, gy = (float)y + nv / U.inv_py;
        int i = (int)floorf((gx - U.x0) * U.inv_px);
        int j = (int)floorf((gy - U.y0) * U.inv_py);
        i = min(max(i, 0), U.nx - 1);
        j = min(max(j, 0), U.ny - 1);
        const int32_t c = (int32_t)U.cell0 + j * U.nx + i;
        if (c != exclude && contains(g, (uint32_t)c, x, y, z, force_s, force_pos, fill)) return c;
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
            if (contains(g, c, x, y, z, force_s, force_pos, fill)) return (int32_t)c;
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
        int32_t dfill;
        const int32_t d = search<PREC>(g, (uint32_t)(-fill - 1), qx, qy, qz, kNone, false, -1, 0.0f, 0.0f, dfill);
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
            const double d = plane_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w);
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
            const double d = quad_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
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
            // would give no hit.  No branches: a plane that cannot be hit, or was
            // just crossed, gets +inf.
            const uint32_t h0 = hs[k], h1 = hs[k + 1];
            const auto c0 = g.coef + 4 * (size_t)(h0 >> 4);
            const double den = plane_den<G::kSurf>(h0 & 7u, c0, P.u, P.v, P.w);
            const uint32_t kk = den > 0.0 ? k : k + 1;
            const uint32_t h = den > 0.0 ? h0 : h1;
            const uint32_t s = h >> 4;
            // the pair shares its normal: the linear part from h0's record, the
            // offset from the reached plane's (the operations of plane_value)
            const double t = (-(plane_linear<G::kSurf>(h0 & 7u, c0, qx, qy, qz) - plane_offset<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s))) / den;
            const bool skip = den == 0.0 || (P.on_level == L && P.on_surf == s);
            const double d = skip ? dinf() : ((t > 0.0) ? t : 0.0);
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
            const double d = plane_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w);
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
            const double d = quad_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
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
    int32_t cfill;
    const int32_t c = search<PREC>(g, univ, qx, qy, qz, ss, !old_pos, (int32_t)old, (float)P.u * 1e-3f,
                                   (float)P.v * 1e-3f, cfill);
    if (c < 0) return Ls == 0 ? GT_END_ESCAPE : GT_END_LOST;
    lvl(P, Ls) = (uint32_t)c;
    if (!descend<PREC>(g, P, Ls, qx, qy, qz)) return GT_END_LOST;
    P.on_level = Ls;
    P.on_surf = ss;
    return GT_END_NONE;
}

// ------------------------------------------------------------------ per-kind trackers
// The static-polymorphism method (Section "Static polymorphism (SP) method")
// keeps one tracker type per kind of universe and switches on the kind of
// each level's universe; the fixed-depth reactor tracker (Section "RTK
// tracking") knows every level's kind at compile time: an optional one-cell
// root, one or two levels of rectilinear arrays, then pins.  An array
// tracker finds a cell by index and crosses to the neighbour by index
// (Algs. 5 and 6); a pin tracker does the same over rings and axial slabs.
// Both reach exactly the single tracker's cells: an index along an axis is
// the number of grid boundaries the coordinate is strictly beyond, taken
// with the double-precision difference of the half-space test itself, so it
// names the one cell whose tests all pass.
enum Tracker : int { TRK_ST = 0, TRK_SP = 1, TRK_RTK = 2 };
// RTK shapes (the preprocessor's code): bit 1 a one-cell root above the
// arrays, bit 2 two array levels instead of one
constexpr int kRtkRootCsg = 2, kRtkTwoArrays = 4;
__host__ __device__ constexpr int rtk_depth(int shape) {
    return ((shape & kRtkRootCsg) ? 1 : 0) + ((shape & kRtkTwoArrays) ? 2 : 1) + 1;
}
// The kind of level L of the fixed-depth shape.
__device__ __forceinline__ int rtk_kind(int shape, int L) {
    const int root = (shape & kRtkRootCsg) ? 1 : 0;
    const int arrays = (shape & kRtkTwoArrays) ? 2 : 1;
    return L < root ? kKindCsg : (L < root + arrays ? kKindRect : kKindPin);
}

// Nearest.entry of a hit on a grid boundary: kArrHit | axis << 28 | p
// (boundary p separates slabs p - 1 and p); kArrExtra: an extra half-space
// of a rect universe (its crossing leaves every cell of the array).
constexpr uint32_t kArrHit = 1u << 31, kArrExtra = kArrHit | (7u << 28);

// Slab of coordinate x over boundaries B[0..n] (ascending, -inf / +inf where
// absent), from the first guess i: the i in [0, n) with x - B[i] > 0 and not
// x - B[i+1] > 0; -1 when x is not beyond B[0], n when it is beyond B[n]
// (bounded ends only).
template <typename VP>
__device__ __forceinline__ int slab_of(VP B, int n, double x, int i) {
    i = min(max(i, 0), n - 1);
    while (i > 0 && !(x - B[i] > 0.0)) i--;
    while (i < n - 1 && x - B[i + 1] > 0.0) i++;
    if (!(x - B[i] > 0.0)) return -1;
    if (x - B[i + 1] > 0.0) return n;
    return i;
}

// The slab a crossing of boundary p leads to, the crossed boundary's sense
// forced (fpos: beyond it) and every other boundary taken numerically
// (i_num: the numeric slab of the moved point).  Beyond B_p the only cell
// that uses B_p is slab p, which holds the point unless it is numerically
// beyond B_{p+1}; short of B_p it is slab p - 1, unless the point is not
// beyond B_{p-1}.  -1: no slab.
__device__ __forceinline__ int forced_slab(int i_num, int p, bool fpos, int n) {
    const int i = fpos ? (i_num <= p ? p : i_num) : (i_num >= p - 1 ? p - 1 : i_num);
    return (i >= 0 && i < n) ? i : -1;
}

// The extra half-spaces every cell of a rect universe has (numeric senses,
// or the forced sense on surface force_s).
template <typename G, typename AP>
__device__ __forceinline__ bool rect_extras(const G &g, AP A, double x, double y, double z, uint32_t force_s,
                                            bool force_pos) {
    const uint32_t n = A->nxhs, at = A->xhs;
    for (uint32_t k = 0; k < n; k++) {
        const uint32_t h = g.ahs[at + k];
        const uint32_t s = h >> 4, t = h & 7u;
        const auto c = g.coef + 4 * (size_t)s;
        const double f = t < ST_CZ ? plane_value<G::kSurf>(t, c, x, y, z) : quad_value<G::kSurf>(t, c, x, y, z);
        const bool pos = s == force_s ? force_pos : f > 0.0;
        if (pos != (bool)((h >> 3) & 1u)) return false;
    }
    return true;
}

// find_cell in a rect universe (Alg. 5 with the uniform-pitch first guess):
// the cell (i, j) by index, then the extra half-spaces; -1 if none.
template <typename G, typename AP>
__device__ __forceinline__ int32_t rect_locate(const G &g, AP A, double x, double y, double z) {
    const uint32_t nx = A->n0, ny = A->n1;
    const auto X = g.aval + A->arr;
    const auto Y = X + (nx + 1);
    const int gi = (int)floorf(((float)x - A->x0) * A->inv_px), gj = (int)floorf(((float)y - A->y0) * A->inv_py);
    const int i = slab_of(X, (int)nx, x, gi), j = slab_of(Y, (int)ny, y, gj);
    if (i < 0 || i >= (int)nx || j < 0 || j >= (int)ny) return -1;
    if (A->nxhs && !rect_extras(g, A, x, y, z, kNone, false)) return -1;
    return (int32_t)(A->cell0 + (uint32_t)j * nx + (uint32_t)i);
}

// cross_surface in a rect universe (Alg. 6): from cell `old` across the grid
// boundary named by `entry` (forced sense fpos) to the neighbour by index,
// the other axis re-checked from the old index; -1 when the crossing leaves
// the array.
template <typename G, typename AP>
__device__ __forceinline__ int32_t rect_cross(const G &g, AP A, uint32_t old, uint32_t entry, bool fpos, double x,
                                             double y, double z) {
    if ((entry & kArrExtra) == kArrExtra) return -1;
    const int nx = (int)A->n0, ny = (int)A->n1;
    const auto X = g.aval + A->arr;
    const auto Y = X + (nx + 1);
    const uint32_t ij = g.cell_ij[old];
    int i = (int)(ij & 0xFFFFu), j = (int)(ij >> 16);
    const int p = (int)(entry & 0x0FFFFFFFu);
    if (((entry >> 28) & 7u) == 0) {
        i = forced_slab(slab_of(X, nx, x, i), p, fpos, nx);
        j = slab_of(Y, ny, y, j);
    } else {
        j = forced_slab(slab_of(Y, ny, y, j), p, fpos, ny);
        i = slab_of(X, nx, x, i);
    }
    if (i < 0 || i >= nx || j < 0 || j >= ny) return -1;
    if (A->nxhs && !rect_extras(g, A, x, y, z, kNone, false)) return -1;
    return (int32_t)(A->cell0 + (uint32_t)j * (uint32_t)nx + (uint32_t)i);
}

// Pin universe: ring and slab of a point.  The ring is the number of
// cylinders the point is strictly outside, from the one squared radius
// (x - cx)^2 + (y - cy)^2 every cylinder's test forms; the slab is the
// number of z planes it is strictly above (binary search).
template <typename G, typename AP>
__device__ __forceinline__ int pin_ring(const G &g, AP A, double x, double y) {
    const int nc = (int)A->n0;
    const auto R = g.aval + A->arr;
    const double dx = x - R[nc], dy = y - R[nc + 1];
    const double s2 = dx * dx + dy * dy;
    int r = 0;
    while (r < nc && s2 - R[r] > 0.0) r++;
    return r;
}

template <typename G, typename AP>
__device__ __forceinline__ int pin_slab(const G &g, AP A, double z) {
    const auto Z = g.aval + A->arr + A->n0 + 2;
    int lo = 0, hi = (int)A->n1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (z - Z[mid] > 0.0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename G, typename AP>
__device__ __forceinline__ int32_t pin_locate(const G &g, AP A, double x, double y, double z) {
    return (int32_t)(A->cell0 + (uint32_t)pin_slab(g, A, z) * (A->n0 + 1) + (uint32_t)pin_ring(g, A, x, y));
}

// Crossing inside a pin: a cylinder (axis 0; boundary p = cylinder + 1) or a
// z plane (axis 1; boundary p = plane + 1), the other coordinate numeric.
template <typename G, typename AP>
__device__ __forceinline__ int32_t pin_cross(const G &g, AP A, uint32_t entry, bool fpos, double x, double y,
                                            double z) {
    const int p = (int)(entry & 0x0FFFFFFFu);
    int r = pin_ring(g, A, x, y), k = pin_slab(g, A, z);
    if (((entry >> 28) & 7u) == 0) r = forced_slab(r, p, fpos, (int)A->n0 + 1);
    else k = forced_slab(k, p, fpos, (int)A->n1 + 1);
    if (r < 0 || k < 0) return -1;
    return (int32_t)(A->cell0 + (uint32_t)k * (A->n0 + 1) + (uint32_t)r);
}

// The nearest-surface bookkeeping shared by the per-kind distance steps:
// the lexicographic minimum of (distance, level, surface id).
__device__ __forceinline__ bool nearer(Nearest &r, double d, int L, uint32_t s, bool pos, uint32_t entry) {
    if (d < r.t || (d == r.t && d != dinf() && L == r.level && s < r.surf)) {
        r.t = d;
        r.level = L;
        r.surf = s;
        r.pos = pos;
        r.entry = entry;
        return true;
    }
    return false;
}

// distance_to_surface of one level that is a CSG cell (the single tracker's
// loop over the cell's half-spaces: slab pairs, other planes, quadrics).
template <typename G>
__device__ __forceinline__ bool csg_level_distance(const G &g, const Particle &P, int L, const Cell &cc, double qx,
                                                   double qy, double qz, Nearest &r) {
    const auto hs = g.hs + cc.hs_off;
    const uint32_t npl = cc.n_pl & kPlaneCountMask, npair2 = 2u * (cc.n_pl >> 12);
    bool better = false;
    for (uint32_t k = 0; k < npair2; k += 2) {
        const uint32_t h0 = hs[k], h1 = hs[k + 1];
        const auto c0 = g.coef + 4 * (size_t)(h0 >> 4);
        const double den = plane_den<G::kSurf>(h0 & 7u, c0, P.u, P.v, P.w);
        const uint32_t kk = den > 0.0 ? k : k + 1;
        const uint32_t h = den > 0.0 ? h0 : h1;
        const uint32_t s = h >> 4;
        // the pair shares its normal: the linear part from h0's record, the
        // offset from the reached plane's (the operations of plane_value)
        const double t = (-(plane_linear<G::kSurf>(h0 & 7u, c0, qx, qy, qz) - plane_offset<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s))) / den;
        const bool skip = den == 0.0 || (P.on_level == L && P.on_surf == s);
        const double d = skip ? dinf() : ((t > 0.0) ? t : 0.0);
        better |= nearer(r, d, L, s, den < 0.0, cc.hs_off + kk);
    }
    for (uint32_t k = npair2; k < npl; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (h >> 3) & 1u;
        if (P.on_level == L && P.on_surf == s) continue;
        const double d = plane_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w);
        better |= nearer(r, d, L, s, pos, cc.hs_off + k);
    }
    for (uint32_t k = npl; k < cc.n_hs; k++) {
        const uint32_t h = hs[k];
        const uint32_t s = h >> 4;
        const bool pos = (h >> 3) & 1u;
        const bool on = (P.on_level == L) && (P.on_surf == s);
        const double d = quad_distance<G::kSurf>(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
        better |= nearer(r, d, L, s, pos, cc.hs_off + k);
    }
    return better;
}

// distance_to_surface of one level that is a rect cell (i, j): the grid
// plane ahead along x and along y (the same difference and quotient as the
// plane's half-space), then the extra half-spaces.
template <typename G, typename AP>
__device__ __forceinline__ bool rect_level_distance(const G &g, const Particle &P, int L, AP A, uint32_t c,
                                                    double qx, double qy, double qz, Nearest &r) {
    const uint32_t ij = g.cell_ij[c];
    const int i = (int)(ij & 0xFFFFu), j = (int)(ij >> 16);
    const uint32_t arr = A->arr;
    bool better = false;
    if (P.u != 0.0) {
        const uint32_t p = (uint32_t)(P.u > 0.0 ? i + 1 : i);
        const uint32_t s = g.asurf[arr + p];
        if (s != kLeafNone && !(P.on_level == L && P.on_surf == s)) {
            const double t = (-(qx - g.aval[arr + p])) / P.u;
            better |= nearer(r, t > 0.0 ? t : 0.0, L, s, P.u < 0.0, kArrHit | p);
        }
    }
    if (P.v != 0.0) {
        const uint32_t p = (uint32_t)(P.v > 0.0 ? j + 1 : j);
        const uint32_t at = arr + A->n0 + 1 + p;
        const uint32_t s = g.asurf[at];
        if (s != kLeafNone && !(P.on_level == L && P.on_surf == s)) {
            const double t = (-(qy - g.aval[at])) / P.v;
            better |= nearer(r, t > 0.0 ? t : 0.0, L, s, P.v < 0.0, kArrHit | 1u << 28 | p);
        }
    }
    const uint32_t nx = A->nxhs, xat = A->xhs;
    for (uint32_t k = 0; k < nx; k++) {
        const uint32_t h = g.ahs[xat + k];
        const uint32_t s = h >> 4;
        const bool pos = (h >> 3) & 1u;
        const bool on = (P.on_level == L) && (P.on_surf == s);
        const auto cf = g.coef + 4 * (size_t)s;
        double d;
        if ((h & 7u) < ST_CZ) d = on ? dinf() : plane_distance<G::kSurf>(h & 7u, cf, pos, qx, qy, qz, P.u, P.v, P.w);
        else d = quad_distance<G::kSurf>(h & 7u, cf, pos, qx, qy, qz, P.u, P.v, P.w, on);
        better |= nearer(r, d, L, s, pos, kArrExtra);
    }
    return better;
}

// distance_to_surface of one level that is a pin cell (ring, slab): one
// bounding cylinder (a, b and the squared radius formed once) and the z
// plane ahead.  A flight that reaches the inner cylinder (moving inward,
// positive discriminant) meets it before the outer one -- its near root is
// below -b/a and the outer cylinder's far root, which the point inside it
// can only meet, is above -b/a by at least as much -- so the outer
// cylinder's root is formed only when the inner one is not reached: the
// nearest of the two, as both half-space tests would give it.
template <typename G, typename AP>
__device__ __forceinline__ bool pin_level_distance(const G &g, const Particle &P, int L, AP A, uint32_t c,
                                                   double qx, double qy, double qz, Nearest &r) {
    const uint32_t rk = g.cell_ij[c];
    const int ring = (int)(rk & 0xFFFFu), slab = (int)(rk >> 16);
    const uint32_t arr = A->arr, nc = A->n0;
    const auto R = g.aval + arr;
    const double dx = qx - R[nc], dy = qy - R[nc + 1];
    const double a2 = P.u * P.u + P.v * P.v, b2 = dx * P.u + dy * P.v, r2 = dx * dx + dy * dy;
    bool better = false;
    {
        // the inner cylinder when the flight reaches it (its hit comes before
        // any hit of the outer one), else the outer cylinder: one root
        const uint32_t mi = ring > 0 ? (uint32_t)ring - 1 : 0u;
        const uint32_t si = g.asurf[arr + mi];
        const double cci = r2 - R[mi];
        const bool inner =
            ring > 0 && !(P.on_level == L && P.on_surf == si) && b2 < 0.0 && b2 * b2 - a2 * cci > 0.0;
        if (inner || ring < (int)nc) {
            const uint32_t m = inner ? mi : (uint32_t)ring;
            const uint32_t s = inner ? si : g.asurf[arr + m];
            const bool on = !inner && (P.on_level == L) && (P.on_surf == s);
            better |= nearer(r, quad_root(a2, b2, inner ? cci : r2 - R[m], inner, on), L, s, inner,
                             kArrHit | (m + 1));
        }
    }
    if (P.w != 0.0) {
        const int p = P.w > 0.0 ? slab + 1 : slab;
        if (p >= 1 && p <= (int)A->n1) {
            const uint32_t at = arr + nc + 2 + (uint32_t)p - 1;
            const uint32_t s = g.asurf[at];
            if (!(P.on_level == L && P.on_surf == s)) {
                const double t = (-(qz - g.aval[at])) / P.w;
                better |= nearer(r, t > 0.0 ? t : 0.0, L, s, P.w < 0.0, kArrHit | 1u << 28 | (uint32_t)p);
            }
        }
    }
    return better;
}

// distance_to_surface of the fixed-depth reactor shape: the levels' kinds
// are compile-time constants (the optional one-cell root, the array levels,
// the pin), so the level loop unrolls into straight code.
template <int SHAPE, typename G>
__device__ __forceinline__ void nearest_surface_rtk(const G &g, const Particle &P, Nearest &r) {
    constexpr int kRoot = (SHAPE & kRtkRootCsg) ? 1 : 0;
    constexpr int kDepth = rtk_depth(SHAPE);
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
#pragma unroll
    for (int L = 0; L < kDepth; L++) {
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
        bool better;
        if (L < kRoot) better = csg_level_distance(g, P, L, cc, qx, qy, qz, r);
        else if (L < kDepth - 1) better = rect_level_distance(g, P, L, g.uarr + univ, c, qx, qy, qz, r);
        else better = pin_level_distance(g, P, L, g.uarr + univ, c, qx, qy, qz, r);
        if (better) r.univ = univ;
    }
    r.leaf_fill = fill;
}

// distance_to_surface over every level for the static-polymorphism
// tracker: the kind read per level, arrays by index, every other universe
// by its half-spaces (what the segment step needs, as nearest_surface).
template <typename G>
__device__ __forceinline__ void nearest_surface_sp(const G &g, const Particle &P, Nearest &r) {
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
        const bool better = g.uarr[univ].kind == kKindRect
                                ? rect_level_distance(g, P, L, g.uarr + univ, c, qx, qy, qz, r)
                                : csg_level_distance(g, P, L, cc, qx, qy, qz, r);
        if (better) r.univ = univ;
    }
    r.leaf_fill = fill;
}

// ------------------------------------------------------------------ tallies
// Segment lengths are summed as 128-bit integers in units of 2^-96 cm.  In
// the kernel a contribution is split into four 32-bit limbs, each added to
// its own 64-bit counter with an atomic whose result is not used, so no
// carry has to travel back to the lane; the counters are exact for up to
// 2^32 contributions per instance and launch.  Each XCD adds into the
// replica of the counters its id selects (on device memory of the default
// type the L2 forwards these atomics to the memory side; replicas keep the
// XCDs off each other's addresses where few entries are hot); the finalize
// kernel folds replicas and limbs into the 128-bit total.
// (nrep: the replica count of the array, 1 or 8)
__device__ __forceinline__ uint32_t replica_id(uint32_t nrep) {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (nrep - 1);   // HW_REG_XCC_ID[3:0]
}

struct TallyAcc {
    uint32_t inst;
    uint64_t lo, hi;   // 128-bit register accumulator for consecutive segments in one instance
};

// Agent scope: workgroups on the compute units of one XCD, or of all, add
// into one replica (on gfx950 this is the same global_atomic_add_x2, with no cache
// bits, as at workgroup scope).
__device__ __forceinline__ void add_limb(uint64_t *p, uint64_t v) {
    if (v) __hip_atomic_fetch_add((GT_AS(1) unsigned long long *)p, (unsigned long long)v,
                                  __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
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

// ------------------------------------------------------------------ mesh tally
// Track length of the segment p0 + t u (0 <= t <= l) on a regular mesh:
// the segment is cut at every mesh plane lo[a] + k w[a] (k = 0..n[a]) that it
// crosses at t = (plane - p0[a]) / u[a] with 0 < t < l, and each piece adds
// its length to the bin holding its midpoint p0 + ((t0 + t1) / 2) u (bin
// index floor((mid - lo) / w) per axis; nothing outside the mesh).  On each
// axis t is monotone in k, so the planes crossed form one run of k, walked in
// increasing t; merging the three runs lists the cuts in increasing order
// (equal cuts give pieces of length 0, which add nothing).
__device__ __forceinline__ double mesh_cut(const MeshDesc &m, int a, int k, double p0, double u) {
    const double x = m.lo[a] + (double)k * m.w[a];
    return (x - p0) / u;
}

// floor(d / w), the bin index of a coordinate d past the mesh's low face,
// as the definition forms it: from the product with the reciprocal when that
// is clearly away from an integer (the two quotients are within a few ulps
// of each other, so they then have the same floor), else from the division.
__device__ __forceinline__ double mesh_floor(double d, double w, double iw) {
    const double q = d * iw;
    const double fq = floor(q);
    const double r = q - fq;
    const double tol = 0x1p-50 * fabs(q) + 0x1p-1000;
    return (r > tol && r < 1.0 - tol) ? fq : floor(d / w);
}

// mesh_cut(k) > 0 without the division: a nonzero difference divided by
// |u| <= 1 cannot round to zero, so the quotient is positive exactly when
// the difference has the sign of u.
__device__ __forceinline__ bool mesh_cut_ahead(const MeshDesc &m, int a, int k, double p0, double u) {
    const double d = (m.lo[a] + (double)k * m.w[a]) - p0;
    return u > 0.0 ? d > 0.0 : d < 0.0;
}

// An axis's cut that lies ahead, at plane offset d = (lo + k w) - p0 of u's
// sign, is certainly at t >= l when |d| > reach, reach = (l |u|)(1 + 2^-50):
// the two roundings leave reach above the exact l |u|, so |d / u| > l
// exactly and the rounded quotient is not below l.  Without that certainty
// (reach of no use when l |u| is tiny or zero) the quotient is formed.
__device__ __forceinline__ double mesh_reach(double l, double u) {
    const double lu = l * fabs(u);
    return lu > 0x1p-1000 ? lu * (1.0 + 0x1p-50) : -1.0;
}

__device__ __forceinline__ bool mesh_cut_beyond(const MeshDesc &m, int a, int k, double p0, double reach) {
    return reach >= 0.0 && fabs((m.lo[a] + (double)k * m.w[a]) - p0) > reach;
}

__device__ __forceinline__ void mesh_segment(const MeshDesc &m, uint64_t *rep, TallyAcc &acc, const double p0[3],
                                             const double u[3], double l) {
    int k[3], step[3];
    double tn[3], reach[3];
    uint32_t pend = 0;   // axes whose first cut ahead may lie within the segment
    for (int a = 0; a < 3; a++) {
        tn[a] = dinf();
        step[a] = 0;
        k[a] = 0;
        reach[a] = mesh_reach(l, u[a]);
        if (u[a] == 0.0) continue;
        const int n = (int)m.n[a];
        // first guess of the plane index by the reciprocal, then exact steps
        const double f = floor((p0[a] - m.lo[a]) * m.iw[a]);
        int kk;
        if (u[a] > 0.0) {
            // first k with a cut ahead (t > 0): near floor(...) + 1, then exact
            kk = f < -1.0 ? 0 : (f > (double)n ? n + 1 : (int)f + 1);
            while (kk > 0 && mesh_cut_ahead(m, a, kk - 1, p0[a], u[a])) kk--;
            while (kk <= n && !mesh_cut_ahead(m, a, kk, p0[a], u[a])) kk++;
            step[a] = 1;
        } else {
            // last k with a cut ahead, walking down
            kk = f < -1.0 ? -1 : (f > (double)n ? n : (int)f);
            while (kk < n && mesh_cut_ahead(m, a, kk + 1, p0[a], u[a])) kk++;
            while (kk >= 0 && !mesh_cut_ahead(m, a, kk, p0[a], u[a])) kk--;
            step[a] = -1;
        }
        k[a] = kk;
        if (kk >= 0 && kk <= n && !mesh_cut_beyond(m, a, kk, p0[a], reach[a])) pend |= 1u << a;
    }
    // one division site for the axes that need their cut (most segments
    // cross no plane, and a lane's divergent branches would each be issued)
    while (pend) {
        const int a = __builtin_ctz(pend);
        pend &= pend - 1;
        const double t = mesh_cut(m, a, k[a], p0[a], u[a]);
        tn[a] = t < l ? t : dinf();
    }
    double t0 = 0.0;
    for (;;) {
        double t1 = l;
        int a1 = -1;
        for (int a = 0; a < 3; a++)
            if (tn[a] < t1) {
                t1 = tn[a];
                a1 = a;
            }
        // the piece [t0, t1]
        const double tm = (t0 + t1) * 0.5;
        uint32_t idx[3];
        bool inside = true;
        for (int a = 0; a < 3; a++) {
            const double mid = p0[a] + tm * u[a];
            const double f = mesh_floor(mid - m.lo[a], m.w[a], m.iw[a]);
            inside = inside && f >= 0.0 && f < (double)m.n[a];
            idx[a] = inside ? (uint32_t)f : 0u;
        }
        if (inside) {
            // into the lane's register accumulator while the bin stays the same
            // (a segment's last piece and the next segment's first share one)
            const double v = (t1 - t0) * 0x1p32;
            const double fl = floor(v);
            const double fr = v - fl;
            const uint64_t hi = (uint64_t)fl, lo = (uint64_t)(fr * 0x1p64);
            const uint32_t b = (uint32_t)(((uint64_t)idx[2] * m.n[1] + idx[1]) * m.n[0] + idx[0]);
            if (b == acc.inst) {
                const uint64_t nlo = acc.lo + lo;
                acc.hi += hi + (nlo < lo ? 1u : 0u);
                acc.lo = nlo;
            } else {
                tally_flush(rep, acc);
                acc.inst = b;
                acc.lo = lo;
                acc.hi = hi;
            }
        }
        if (a1 < 0) break;
        t0 = t1;
        const int kk = k[a1] + step[a1];
        k[a1] = kk;
        const bool ok = kk >= 0 && kk <= (int)m.n[a1] && !mesh_cut_beyond(m, a1, kk, p0[a1], reach[a1]);
        const double t = ok ? mesh_cut(m, a1, kk, p0[a1], u[a1]) : dinf();
        tn[a1] = t < l ? t : dinf();
    }
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

// A lane's recent-instance cache in LDS for the persistent schedule.  The
// counters' atomics are carried out beyond the L2, and at two or more per
// contribution their stream limits the tracker; a particle often returns to
// an instance it left a few segments earlier, so each lane keeps up to k
// more 128-bit partial sums (besides the one in registers) and flushes one
// only when it is evicted (round robin) or at the end.  Sums are integers,
// so grouping contributions differently leaves the totals unchanged.
struct TallyCache {
    uint64_t *lo, *hi;   // LDS: entry e of this lane at [e * stride]
    uint32_t *tag;       // instance of each entry, kNone when empty
    uint32_t k, stride;
};

constexpr uint32_t kTallyCacheMax = 3;     // entries per lane at most
constexpr uint32_t kTallyCacheEntry = 20;  // LDS bytes per entry: two 64-bit words and a tag

// The cache of k entries per lane at byte offset `at` of the dynamic LDS:
// all low words, then all high words, then all tags, lane-interleaved.
__device__ __forceinline__ TallyCache tally_cache(unsigned char *lds, uint32_t at, uint32_t k) {
    uint64_t *lo = (uint64_t *)(lds + at);
    const size_t n = (size_t)k * blockDim.x;
    return TallyCache{lo + threadIdx.x, lo + n + threadIdx.x, (uint32_t *)(lo + 2 * n) + threadIdx.x, k, blockDim.x};
}

__device__ __forceinline__ void tally_add_cached(uint64_t *rep, TallyAcc &a, const TallyCache &c, uint32_t &rr,
                                                 uint32_t inst, double l) {
    const double v = l * 0x1p32;
    const double fl = floor(v);
    const double fr = v - fl;
    uint64_t hi = (uint64_t)fl;
    uint64_t lo = (uint64_t)(fr * 0x1p64);
    if (inst != a.inst) {
        uint32_t j = kNone;
        for (uint32_t e = 0; e < c.k; e++)
            if (c.tag[e * c.stride] == inst) j = e;
        const uint32_t slot = j != kNone ? j : rr;
        const size_t at = (size_t)slot * c.stride;
        TallyAcc old;
        old.inst = c.tag[at];
        old.lo = c.lo[at];
        old.hi = c.hi[at];
        c.tag[at] = a.inst;
        c.lo[at] = a.lo;
        c.hi[at] = a.hi;
        if (j != kNone) {
            // a hit: continue that partial sum in registers
            const uint64_t nlo = old.lo + lo;
            hi = old.hi + hi + ((nlo < old.lo) ? 1u : 0u);
            lo = nlo;
        } else {
            rr = rr + 1 == c.k ? 0u : rr + 1;
            tally_flush(rep, old);
        }
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
        int32_t rfill;
        const int32_t c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, rfill);
        if (c < 0) {
            end = GT_END_LOST;
        } else {
            lvl(P, 0) = (uint32_t)c;
            if (!descend<PREC>(g, P, 0, P.x, P.y, P.z)) end = GT_END_LOST;
        }
    } else {
        int32_t c = -1, rfill;
        for (int a = 0; a < kMaxBirthAttempts && c < 0; a++) {
            draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
            P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * u0;
            P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * u1;
            P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * u2;
            c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, rfill);
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

// ------------------------------------------------------------------ persistent schedule
// Each lane runs a state machine; a wave loops until the shared particle
// pool is drained and all of its lanes are idle.  Finished lanes are
// refilled at once from a wave-local pool of particle ids (ballot +
// per-lane rank, one global atomic per 64 ids), so a wave no longer waits
// for its longest history.  Per loop trip every lane takes at most one of
// each step -- draw one random block (a birth position or a direction
// attempt with its optical depth), search up to kSearchLevels levels, one
// segment -- and each step has one call site, so lanes at different points
// of their histories share one instruction stream per step.
enum Mode : int { M_IDLE = 0, M_POS = 1, M_DIR = 2, M_SEARCH = 3, M_TRACK = 4 };

// Search levels a lane may take per loop trip: two lets a crossing of a
// lattice cell and the descent into the pin below it finish in one trip, so
// the lane still tracks a segment in that trip.
constexpr int kSearchLevels = 2;

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

template <int KIND, int S> struct ViewOf;
template <int S> struct ViewOf<SK_NONE, S> { typedef DevT<1, 1, 1, S> type; };
template <int S> struct ViewOf<SK_SPLIT, S> { typedef DevT<3, 1, 1, S> type; };
template <int S> struct ViewOf<SK_LDS, S> { typedef DevT<3, 3, 1, S> type; };
template <int S> struct ViewOf<SK_ALL, S> { typedef DevT<3, 3, 3, S> type; };

// The view of a geometry for a kernel of staging kind KIND: staged tables at
// their LDS copies (`lds`, a workgroup-shared address), the others global.
template <int KIND, int S = SF_ALL>
__device__ __forceinline__ typename ViewOf<KIND, S>::type make_view(const Dev &g, const StagePlan &sp,
                                                                    unsigned char *lds) {
    typedef typename ViewOf<KIND, S>::type V;
    if constexpr (KIND == SK_NONE) {
        return global_view<S>(g);
    } else {
        V d;
        auto lp = [&](int sec) { return lds + sp.at[sec]; };
        d.coef = (cptr<3, double>)lp(SEC_COEF);
        d.hs = (cptr<3, uint32_t>)lp(SEC_HS);
        d.cell = (cptr<3, Cell>)lp(SEC_CELL);
        d.univ = (cptr<3, Univ>)lp(SEC_UNIV);
        d.sigma = (cptr<3, double>)lp(SEC_SIGMA);
        d.cell_local = (cptr<3, uint32_t>)lp(SEC_LOCAL);
        if (sp.at[SEC_UARR] != 0xFFFFFFFFu) {
            d.uarr = (cptr<3, UArr>)lp(SEC_UARR);
            d.aval = (cptr<3, double>)lp(SEC_AVAL);
            d.asurf = (cptr<3, uint32_t>)lp(SEC_ASURF);
            d.ahs = (cptr<3, uint32_t>)lp(SEC_AHS);
            d.cell_ij = (cptr<3, uint32_t>)lp(SEC_IJ);
        } else {
            // a plan without the universe-kind tables (the single tracker's):
            // never read through these
            d.uarr = nullptr;
            d.aval = nullptr;
            d.asurf = d.ahs = d.cell_ij = nullptr;
        }
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
// [0, end) for one geometry, or, in a batch, a counter over one chunk of an
// item (in LDS) or over all of an item's histories (in device memory, shared
// by the workgroups on the item).  take() is called by one lane and returns
// the first of k ids.
struct GlobalQueue {
    unsigned long long *ctr;
    uint64_t end;
    __device__ __forceinline__ uint64_t take(uint64_t k) const { return atomicAdd(ctr, (unsigned long long)k); }
};

struct ChunkQueue {
    unsigned long long *ctr;   // LDS or device memory
    uint64_t first, end;
    __device__ __forceinline__ uint64_t take(uint64_t k) const {
        return first + atomicAdd(ctr, (unsigned long long)k);
    }
};

// Which item of a batch launch a workgroup works on next, when workgroups
// join whole items.  Every lane of the workgroup calls it; lane 0 stores the
// item (kNoItem once every item's histories are claimed) in *pick and counts
// the workgroup in workers[item]; the caller's barrier publishes it.
//  * first call: the workgroups are spread over the slots in proportion to
//    their estimated work (n x weight): workgroup b takes the slot whose
//    running sum first exceeds (b + 1/2) / grid of the total;
//  * later calls: the item with the most estimated work left per workgroup
//    on it, counting the one joining -- (n - claimed) x weight / (workers + 1).
// Only the order in which histories run depends on this choice, never a
// result.  The counters are read with agent-scope atomic loads after the
// barrier that ends a visit, so a workgroup that has seen an item's counter
// reach n never chooses that item again: a visit that claims nothing finds
// its item exhausted, each workgroup makes at most (its claims + the number
// of items) visits, and the loop over visits ends.  red_s, red_i: LDS, one
// entry per wave.
__device__ __forceinline__ void pick_item(const BatchSlot *slots, uint32_t n_slots, unsigned long long *claimed,
                                          unsigned long long *workers, bool first, float *red_s, uint32_t *red_i,
                                          uint32_t *pick) {
    if (first) {
        if (threadIdx.x == 0) {
            const double total = slots[n_slots - 1].cum;
            const double at = ((double)blockIdx.x + 0.5) / (double)gridDim.x * total;
            uint32_t lo = 0, hi = n_slots - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2;
                if (slots[mid].cum > at) hi = mid;
                else lo = mid + 1;
            }
            const uint32_t it = slots[lo].item;
            atomicAdd(&workers[it], 1ull);
            *pick = it;
        }
        return;
    }
    float best = 0.0f;
    uint32_t bi = kNoItem;
    for (uint32_t s = threadIdx.x; s < n_slots; s += blockDim.x) {
        const BatchSlot sl = slots[s];
        const uint64_t c = __hip_atomic_load(&claimed[sl.item], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (c >= sl.n) continue;
        const uint64_t w = __hip_atomic_load(&workers[sl.item], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const float score = (float)(sl.n - c) * sl.weight / (float)(w + 1);
        if (bi == kNoItem || score > best) {
            best = score;
            bi = sl.item;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {   // the wave's best (lowest item among equal scores)
        const float bs = __shfl_xor(best, o);
        const uint32_t bo = __shfl_xor(bi, o);
        if (bo != kNoItem && (bi == kNoItem || bs > best || (bs == best && bo < bi))) {
            best = bs;
            bi = bo;
        }
    }
    if (__lane_id() == 0) {
        red_s[threadIdx.x / 64] = best;
        red_i[threadIdx.x / 64] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float b = 0.0f;
        uint32_t it = kNoItem;
        for (uint32_t w = 0; w < (blockDim.x + 63) / 64; w++)
            if (red_i[w] != kNoItem && (it == kNoItem || red_s[w] > b || (red_s[w] == b && red_i[w] < it))) {
                b = red_s[w];
                it = red_i[w];
            }
        if (it != kNoItem) atomicAdd(&workers[it], 1ull);
        *pick = it;
    }
}

// Meetings of the workgroup's waves.  The persistent loop runs per wave;
// two optional, result-neutral steps make the waves meet at a barrier and
// move histories between lanes through an LDS buffer.  A history's state
// moves as a whole (kTailFields words: position, direction, optical depth,
// id, hash, counters, search state, the cell of each level); the lane's
// tally accumulator and cache stay with the lane, since the tallies are sums
// over all histories.  So no result depends on the lane that finishes a
// history.
//  * Tail compaction: once the queue is empty for every wave, every `round`
//    loop trips, when the live histories fit in fewer waves (and in the
//    buffer), each is written at its rank and read back by the lane of that
//    rank, so fewer, fuller waves carry the tail while the emptied ones wait
//    at the barrier.  Off by default: waves that wait for the tail keep taking
//    issue slots that finished waves would leave to working ones.
//  * Regroup: every `regroup` loop trips (from the start), the lanes are sorted
//    by a key -- the leaf universe of a history about to take a segment, else
//    its step (birth position, direction, search), idle lanes last -- with a
//    counting sort in LDS, so lanes that run the same code sit in the same
//    waves.  The buffer holds one word per lane; the state moves a word per
//    pass.
constexpr int kTailFields = 16;   // 64-bit words per moved history
constexpr uint32_t kTailRound = 8;
constexpr uint32_t kRgBuckets = 64;   // regroup keys (one wave scans them)
static_assert(13 + GT_MAX_LEVELS / 2 == kTailFields, "moved state: 13 words + the levels, two per word");

struct TailCfg {
    uint64_t *buf;     // LDS buffer of `words` 64-bit words
    uint32_t *ctl;     // LDS: [0] waves whose queue is empty (compaction),
                       // [1 + w] live lanes of wave w, bit 31: its queue is empty
    uint32_t cap;      // compaction: histories the buffer holds field-major; 0 = off
    uint32_t round;    // compaction: loop trips between meetings in the tail
    uint32_t words;    // buffer size
    uint32_t regroup;  // loop trips between regroups; 0 = off (needs words >= lanes)
};

// The persistent history loop of one lane (see above); returns when its
// wave has drained the queue and every lane of the wave is idle (with tail
// compaction: when no lane of the workgroup has a history left).
template <int PREC, bool RG = false, bool MESH = false, int TRK = TRK_ST, int SHAPE = 0, typename G,
          typename Queue>
__device__ __forceinline__ void track_pool(const G &g, const KParams &p, const KOut &o, uint64_t *rep,
                                           uint32_t *cells, const Queue &queue, Counts &cnt, const TailCfg &tc,
                                           const TallyCache &tcache) {
    // the parallel-ray source exists in the builds for every surface type only
    // (the host sends ray launches there); the smaller builds drop its code
    const bool ray = G::kSurf == SF_ALL && p.source == 1;
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
    TallyAcc macc;   // the mesh tally's accumulator (MESH builds)
    macc.inst = kNone;
    macc.lo = macc.hi = 0;
    uint32_t rr = 0;   // next tally-cache entry to evict
    for (uint32_t e = 0; e < tcache.k; e++) tcache.tag[e * tcache.stride] = kNone;
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

    // (RG: the build with the regroup step; without it the step's code is left out)
    const uint32_t regroup = RG && tc.words >= blockDim.x ? tc.regroup : 0u;
    const bool meetings = tc.cap != 0 || regroup != 0;   // workgroup-uniform

    // the moved state of a history, word by word (see TailCfg)
    auto get_word = [&](int f) -> uint64_t {
        switch (f) {
        case 0: return (uint64_t)__double_as_longlong(P.x);
        case 1: return (uint64_t)__double_as_longlong(P.y);
        case 2: return (uint64_t)__double_as_longlong(P.z);
        case 3: return (uint64_t)__double_as_longlong(P.u);
        case 4: return (uint64_t)__double_as_longlong(P.v);
        case 5: return (uint64_t)__double_as_longlong(P.w);
        case 6: return (uint64_t)__double_as_longlong(P.tau);
        case 7: return local;
        case 8: return h;
        case 9: return (uint64_t)blk | (uint64_t)segs << 32;
        case 10: return (uint64_t)ncoll | (uint64_t)attempts << 32;
        case 11: return (uint64_t)sforce | (uint64_t)sk << 32;
        case 12: {
            const uint32_t fl = (uint32_t)mode | (uint32_t)recovf << 3 | (uint32_t)birth << 4 | (uint32_t)sfpos << 5 |
                                (uint32_t)P.depth << 8 | (uint32_t)(P.on_level + 1) << 12 | (uint32_t)sL << 16;
            return (uint64_t)P.on_surf | (uint64_t)fl << 32;
        }
        default: {
            const int L = 2 * (f - 13);
            return (uint64_t)lvl(P, L) | (uint64_t)lvl(P, L + 1) << 32;
        }
        }
    };
    auto set_word = [&](int f, uint64_t v) {
        switch (f) {
        case 0: P.x = __longlong_as_double((long long)v); break;
        case 1: P.y = __longlong_as_double((long long)v); break;
        case 2: P.z = __longlong_as_double((long long)v); break;
        case 3: P.u = __longlong_as_double((long long)v); break;
        case 4: P.v = __longlong_as_double((long long)v); break;
        case 5: P.w = __longlong_as_double((long long)v); break;
        case 6: P.tau = __longlong_as_double((long long)v); break;
        case 7: local = v; break;
        case 8: h = v; break;
        case 9: blk = (uint32_t)v; segs = (uint32_t)(v >> 32); break;
        case 10: ncoll = (uint32_t)v; attempts = (uint32_t)(v >> 32); break;
        case 11: sforce = (uint32_t)v; sk = (uint32_t)(v >> 32); break;
        case 12: {
            P.on_surf = (uint32_t)v;
            const uint32_t fl = (uint32_t)(v >> 32);
            mode = (int)(fl & 7u);
            recovf = (fl >> 3) & 1u;
            birth = (fl >> 4) & 1u;
            sfpos = (fl >> 5) & 1u;
            P.depth = (int)((fl >> 8) & 15u);
            P.on_level = (int)((fl >> 12) & 15u) - 1;
            sL = (int)((fl >> 16) & 15u);
            break;
        }
        default: {
            const int L = 2 * (f - 13);
            lvl(P, L) = (uint32_t)v;
            lvl(P, L + 1) = (uint32_t)(v >> 32);
        }
        }
    };
    // a lane without a history
    auto clear_state = [&]() {
        mode = M_IDLE;
        P.x = P.y = P.z = P.u = P.v = P.w = P.tau = 0.0;
        local = h = 0;
        blk = segs = ncoll = attempts = sk = 0;
        sforce = P.on_surf = kNone;
        recovf = birth = sfpos = false;
        P.depth = 1;
        P.on_level = -1;
        sL = 0;
        end = GT_END_NONE;
    };

    for (;;) {
        if (meetings) {
            const uint64_t act = __ballot(mode != M_IDLE);
            bool meet;
            if (RG && regroup) {
                // every `regroup` trips; a wave with nothing left to do waits at once
                meet = ++titer >= regroup || (drained && act == 0);
            } else {
                if (drained && !counted) {
                    counted = true;
                    if (__lane_id() == 0) atomicAdd(&tc.ctl[0], 1u);
                }
                if (drained && !in_tail)
                    in_tail =
                        __builtin_amdgcn_readfirstlane(__atomic_load_n(&tc.ctl[0], __ATOMIC_RELAXED)) == nwaves;
                meet = in_tail && (act == 0 || ++titer >= tc.round);
            }
            if (meet) {
                titer = 0;
                if (__lane_id() == 0) tc.ctl[1 + wave] = (uint32_t)__popcll(act) | (drained ? 1u << 31 : 0u);
                __syncthreads();
                // (the counts are workgroup-uniform: read them as scalars)
                uint32_t A = 0, busy = 0, before = 0, D = 0;
                for (uint32_t w = 0; w < nwaves; w++) {
                    const uint32_t cw = __builtin_amdgcn_readfirstlane(tc.ctl[1 + w]);
                    const uint32_t a = cw & 0x7FFFFFFFu;
                    A += a;
                    busy += a ? 1u : 0u;
                    before += w < wave ? a : 0u;
                    D += cw >> 31;
                }
                // every wave has read this meeting's counts before any wave
                // can write the next meeting's
                __syncthreads();
                if (A == 0 && D == nwaves) break;
                if (tc.cap && D == nwaves && A <= tc.cap && (A + 63u) / 64u < busy) {
                    // pack the A live histories into lanes 0..A-1 of the workgroup
                    const uint32_t C = tc.cap;
                    if (mode != M_IDLE) {
                        uint64_t *b = tc.buf + before + lane_rank(act);
#pragma unroll
                        for (int f = 0; f < kTailFields; f++) b[f * C] = get_word(f);
                    }
                    __syncthreads();
                    if (threadIdx.x < A) {
                        const uint64_t *b = tc.buf + threadIdx.x;
#pragma unroll
                        for (int f = 0; f < kTailFields; f++) set_word(f, b[f * C]);
                    } else {
                        clear_state();   // (all of the old history is in the buffer)
                    }
                    end = GT_END_NONE;
                } else if (RG && regroup) {
                    // counting sort of the lanes by key: histogram, exclusive
                    // scan by one wave, destination = bucket start + rank
                    uint32_t key = kRgBuckets - 1;
                    if (mode == M_TRACK) {
                        const uint32_t u =
                            P.depth > 1 ? (uint32_t)(-g.cell[lvl(P, P.depth - 2)].fill - 1) : g.root;
                        key = u % (kRgBuckets - 4);
                    } else if (mode != M_IDLE) {
                        key = kRgBuckets - 4 + (uint32_t)mode - 1;   // birth position, direction, search
                    }
                    uint32_t *hist = (uint32_t *)tc.buf;
                    if (threadIdx.x < kRgBuckets) hist[threadIdx.x] = 0;
                    __syncthreads();
                    const uint32_t rank = atomicAdd(&hist[key], 1u);
                    __syncthreads();
                    if (wave == 0) {
                        const uint32_t n = hist[__lane_id()];
                        uint32_t incl = n;
                        for (int d = 1; d < 64; d <<= 1) {
                            const uint32_t t = __shfl_up(incl, d);
                            if ((int)__lane_id() >= d) incl += t;
                        }
                        hist[__lane_id()] = incl - n;
                    }
                    __syncthreads();
                    const uint32_t dest = hist[key] + rank;   // a permutation of 0 .. lanes-1
                    __syncthreads();
                    // one word of the state per pass (no register holds more
                    // than the word in flight)
#pragma unroll
                    for (int f = 0; f < kTailFields; f++) {
                        tc.buf[dest] = get_word(f);
                        __syncthreads();
                        set_word(f, tc.buf[threadIdx.x]);
                        __syncthreads();
                    }
                    end = GT_END_NONE;
                }
                // on into a loop trip: a wave with histories advances them
                // before it can meet again (so any interval, down to one
                // trip, makes progress)
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
                    if ((int)__lane_id() == leader) base = queue.take(p.wave_take);
                    base = __shfl(base, leader);
                    if (base >= queue.end) { drained = true; break; }
                    pool_next = base;
                    pool_end = min((uint64_t)base + p.wave_take, queue.end);
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
            if (!meetings) break;
            // the queue is empty for this wave: wait for the workgroup's next
            // meeting (no lane holds a history: the state is dead)
            clear_state();
            __builtin_amdgcn_s_sleep(2);
            continue;
        }

        // ---- draw: a birth-position attempt, or a direction attempt and its optical depth
        if (mode == M_POS || mode == M_DIR) {
            if (mode == M_POS && ray) {
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

        // ---- up to kSearchLevels levels of find_cell / cross_surface (the
        // fixed-depth tracker: every level below the crossing in this trip)
        constexpr int kLevelsPerTrip = TRK == TRK_RTK ? rtk_depth(SHAPE) : kSearchLevels;
#pragma unroll 1
        for (int sn = 0; sn < kLevelsPerTrip && mode == M_SEARCH && end == GT_END_NONE; sn++) {
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
            int32_t c = -1, fill = 0;
            bool by_kind = false;
            if constexpr (TRK != TRK_ST) {
                // the tracker of this level's kind: arrays and pins by index; the
                // fixed-depth tracker's one-cell root by its containment test
                // (a crossing of its boundary leaves the geometry)
                const int kind = TRK == TRK_RTK ? rtk_kind(SHAPE, sL) : g.uarr[su].kind;
                if (kind == kKindRect || (TRK == TRK_RTK && kind == kKindPin)) {
                    by_kind = true;
                    const auto A = g.uarr + su;
                    if (kind == kKindRect)
                        c = sforce != kNone ? rect_cross(g, A, lvl(P, sL), sk, sfpos, qx, qy, qz)
                                            : rect_locate(g, A, qx, qy, qz);
                    else
                        c = sforce != kNone ? pin_cross(g, A, sk, sfpos, qx, qy, qz) : pin_locate(g, A, qx, qy, qz);
                    if (c >= 0) fill = g.cell[c].fill;
                } else if (TRK == TRK_RTK) {
                    by_kind = true;
                    const uint32_t c0 = g.uarr[su].cell0;
                    if (sforce == kNone && contains(g, c0, qx, qy, qz, kNone, false, fill)) c = (int32_t)c0;
                }
            }
            if (!by_kind) {
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
                    const Univ U = ldv<Univ>(g.univ + su);
                    hint = U.cell0 + loc;
                    k0 = 0;
                    k1 = loc < U.ncell ? 1u : 0u;
                }
                for (uint32_t k = k0; k < k1; k++) {
                    const uint32_t d = sforce != kNone ? g.adj[k] : hint;
                    if (contains(g, d, qx, qy, qz, sforce, sfpos, fill)) { c = (int32_t)d; break; }
                }
                // the full search; after a crossing its lattice guess is taken a
                // little along the flight, so that it lands on the far side
                if (c < 0) {
                    const float nu = sforce != kNone ? (float)P.u * 1e-3f : 0.0f;
                    const float nv = sforce != kNone ? (float)P.v * 1e-3f : 0.0f;
                    c = search<PREC>(g, su, qx, qy, qz, sforce, sfpos, excl, nu, nv, fill);
                }
            }
            if (c < 0) {
                if (birth) {
                    if (sL == 0 && !ray) { cnt.rejected++; mode = M_POS; }
                    else end = GT_END_LOST;
                } else {
                    end = (sforce != kNone && sL == 0) ? GT_END_ESCAPE : GT_END_LOST;
                }
            } else {
                lvl(P, sL) = (uint32_t)c;
                if (fill < 0) {
                    sL++;
                    sforce = kNone;
                } else {
                    P.depth = sL + 1;
                    if (birth) {
                        birth = false;
                        mode = ray ? M_TRACK : M_DIR;
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
            if constexpr (TRK == TRK_ST) nearest_surface(g, P, nr);
            else if constexpr (TRK == TRK_RTK) nearest_surface_rtk<SHAPE>(g, P, nr);
            else nearest_surface_sp(g, P, nr);
            const double sig = g.sigma[nr.leaf_fill];
            const double sc = ray ? dinf() : P.tau / sig;
            const uint32_t inst = nr.inst;
            const bool boundary = nr.t < sc;
            if (!boundary && sc == dinf()) {
                end = GT_END_LOST;
            } else {
                double l;
                if (boundary) {
                    l = nr.t;
                    if (!ray) P.tau = P.tau - sig * nr.t;
                } else {
                    l = sc;
                }
                if constexpr (MESH) {
                    const double p0[3] = {P.x, P.y, P.z}, uu[3] = {P.u, P.v, P.w};
                    mesh_segment(o.mesh, o.mesh.ws + (size_t)replica_id(tally_replicas(o.mesh.nb)) * 4 * o.mesh.nb, macc, p0, uu, l);
                }
                const double m0 = l * P.u, m1 = l * P.v, m2 = l * P.w;
                P.x = P.x + m0;
                P.y = P.y + m1;
                P.z = P.z + m2;
                if (tcache.k) tally_add_cached(rep, acc, tcache, rr, inst, l);
                else tally_add(rep, acc, inst, l);
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
            h ^= (uint64_t)end;
            if (o.seg_count) gstore(o.seg_count, local, segs);
            if (o.seq_hash) gstore(o.seq_hash, local, h);
            if (o.end_code) gstore(o.end_code, local, end);
            count_end(cnt, end, segs, recovf);
            mode = M_IDLE;
        }
    }
    // the lane's partial tally sums
    tally_flush(rep, acc);
    if constexpr (MESH) tally_flush(o.mesh.ws + (size_t)replica_id(tally_replicas(o.mesh.nb)) * 4 * o.mesh.nb, macc);
    for (uint32_t e = 0; e < tcache.k; e++) {
        TallyAcc c;
        c.inst = tcache.tag[e * tcache.stride];
        c.lo = tcache.lo[e * tcache.stride];
        c.hi = tcache.hi[e * tcache.stride];
        tally_flush(rep, c);
    }
}

// A workgroup's end counts, summed in LDS, then one atomic per counter.
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

// ------------------------------------------------------------------ event-based schedule
// The same histories as gt_track, with the state in a bank in device memory
// and one kernel per operation over the whole bank per iteration:
// distance_to_surface, then move / tally / collision, then cross_surface
// (the organisation of an event-based tracker; kept for comparison).  Each
// step below loads history i from the bank, takes its one step with the
// device functions of the persistent schedule (slab pairs, candidate lists)
// in the operation order of run_history, and stores it back.
constexpr uint32_t kEvDone = 1u << 19, kEvPending = 1u << 17, kEvRecOvf = 1u << 18;

__device__ __forceinline__ uint32_t ev_pack(int depth, int on_level, int end, int bl, bool bpos, bool pending,
                                            bool recovf, bool done) {
    return (uint32_t)depth | (uint32_t)(on_level + 1) << 4 | (uint32_t)end << 8 | (uint32_t)bl << 12 |
           (uint32_t)bpos << 16 | (uint32_t)pending << 17 | (uint32_t)recovf << 18 | (uint32_t)done << 19;
}

__device__ __forceinline__ void ev_load(const EvBank &b, uint64_t n, uint64_t i, uint32_t st, Particle &P) {
    P.x = b.x[i];
    P.y = b.y[i];
    P.z = b.z[i];
    P.u = b.u[i];
    P.v = b.v[i];
    P.w = b.w[i];
    P.tau = b.tau[i];
    P.depth = (int)(st & 15u);
    P.on_level = (int)((st >> 4) & 15u) - 1;
    P.on_surf = b.on_surf[i];
    // levels below the history's depth read as cell 0 (a descent's hint
    // reads the previous cell of each level it enters)
    for (int L = 0; L < GT_MAX_LEVELS; L++) lvl(P, L) = L < P.depth ? b.cell[(size_t)L * n + i] : 0u;
}

__device__ __forceinline__ void ev_store_geom(const EvBank &b, uint64_t n, uint64_t i, const Particle &P) {
    for (int L = 0; L < P.depth; L++) b.cell[(size_t)L * n + i] = lvl(P, L);
    b.on_surf[i] = P.on_surf;
}

// cross_surface as the persistent schedule takes it: the crossed
// half-space's candidate list first, then the full search, then descent.
template <int PREC, typename G>
__device__ __forceinline__ int cross_listed(const G &g, Particle &P, int Ls, uint32_t ss, bool old_pos,
                                            uint32_t entry) {
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
    int32_t c = -1, fill = 0;
    for (uint32_t k = g.adj_off[entry]; k < g.adj_off[entry + 1]; k++) {
        const uint32_t d = g.adj[k];
        if (contains(g, d, qx, qy, qz, ss, !old_pos, fill)) {
            c = (int32_t)d;
            break;
        }
    }
    if (c < 0)
        c = search<PREC>(g, univ, qx, qy, qz, ss, !old_pos, (int32_t)old, (float)P.u * 1e-3f, (float)P.v * 1e-3f,
                         fill);
    if (c < 0) return Ls == 0 ? GT_END_ESCAPE : GT_END_LOST;
    lvl(P, Ls) = (uint32_t)c;
    // descent: first the cell with the same index in the new universe as the
    // history had at that level before, then the full search
    int L = Ls;
    while (fill < 0) {
        const auto t = g.trans + 4 * (size_t)lvl(P, L);
        qx = qx - t[0];
        qy = qy - t[1];
        qz = qz - t[2];
        const uint32_t u = (uint32_t)(-fill - 1);
        L++;
        const Univ U = ldv<Univ>(g.univ + u);
        const uint32_t loc = g.cell_local[lvl(P, L)];
        int32_t d = -1;
        if (loc < U.ncell && contains(g, U.cell0 + loc, qx, qy, qz, kNone, false, fill)) d = (int32_t)(U.cell0 + loc);
        if (d < 0) d = search<PREC>(g, u, qx, qy, qz, kNone, false, -1, 0.0f, 0.0f, fill);
        if (d < 0) {
            P.depth = L;
            return GT_END_LOST;
        }
        lvl(P, L) = (uint32_t)d;
    }
    P.depth = L + 1;
    P.on_level = Ls;
    P.on_surf = ss;
    return GT_END_NONE;
}

// A history's end: its open tally sum, hash and outputs (as run_history).
__device__ __forceinline__ void ev_finish(const EvBank &b, const KOut &o, uint64_t *rep, uint64_t i, int end,
                                          bool recovf, Counts &cnt) {
    TallyAcc acc;
    acc.inst = b.acc_inst[i];
    acc.lo = b.acc_lo[i];
    acc.hi = b.acc_hi[i];
    tally_flush(rep, acc);
    b.acc_inst[i] = kNone;
    const uint64_t h = b.h[i] ^ (uint64_t)end;
    const uint32_t segs = b.segs[i];
    if (o.seg_count) gstore(o.seg_count, i, segs);
    if (o.seq_hash) gstore(o.seq_hash, i, h);
    if (o.end_code) gstore(o.end_code, i, end);
    count_end(cnt, end, segs, recovf);
}

// Birth of history i (as run_history), written to the bank.
template <int PREC, typename G>
__device__ __forceinline__ void ev_birth(const G &g, const KParams &p, const KOut &o, const EvBank &b, uint64_t *rep,
                                         uint64_t i, uint32_t *cells, Counts &cnt) {
    {
        Particle P;
        P.cell = cells;
        for (int L = 0; L < GT_MAX_LEVELS; L++) lvl(P, L) = 0;
        const uint64_t pid = p.first + i;
        uint32_t blk = 0;
        P.on_level = -1;
        P.on_surf = kNone;
        P.depth = 1;
        P.u = P.v = P.w = P.tau = 0.0;
        int end = GT_END_NONE;
        double u0, u1, u2;
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
            int32_t rfill;
            const int32_t c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, rfill);
            if (c < 0) {
                end = GT_END_LOST;
            } else {
                lvl(P, 0) = (uint32_t)c;
                if (!descend<PREC>(g, P, 0, P.x, P.y, P.z)) end = GT_END_LOST;
            }
        } else {
            int32_t c = -1, rfill;
            for (int a = 0; a < kMaxBirthAttempts && c < 0; a++) {
                draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
                P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * u0;
                P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * u1;
                P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * u2;
                c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, 0.0f, 0.0f, rfill);
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
        b.x[i] = P.x;
        b.y[i] = P.y;
        b.z[i] = P.z;
        b.u[i] = P.u;
        b.v[i] = P.v;
        b.w[i] = P.w;
        b.tau[i] = P.tau;
        if (P.depth < 1) P.depth = 1;
        ev_store_geom(b, p.n, i, P);
        b.blk[i] = blk;
        b.segs[i] = 0;
        b.ncoll[i] = 0;
        b.h[i] = kFnvOffset;
        b.acc_inst[i] = kNone;
        b.acc_lo[i] = 0;
        b.acc_hi[i] = 0;
        b.st[i] = ev_pack(P.depth, P.on_level, end, 0, false, false, false, end != GT_END_NONE);
        if (end != GT_END_NONE) ev_finish(b, o, rep, i, end, false, cnt);
    }
}

// distance_to_surface over every level (as the persistent schedule takes it),
// with the leaf's Sigma and instance.
template <typename G>
__device__ __forceinline__ void ev_distance(const G &g, uint64_t n, const EvBank &b, uint64_t i, uint32_t *cells) {
    const uint32_t st = b.st[i];
    if (st & kEvDone) return;
    Particle P;
    P.cell = cells;
    ev_load(b, n, i, st, P);
    Nearest nr;
    nearest_surface(g, P, nr);
    b.t[i] = nr.t;
    b.sig[i] = g.sigma[nr.leaf_fill];
    b.inst[i] = nr.inst;
    b.surf[i] = nr.surf;
    b.entry[i] = nr.entry;
    b.st[i] = (st & ~(0xFu << 12 | 1u << 16)) | (uint32_t)nr.level << 12 | (uint32_t)nr.pos << 16;
}

// The segment: boundary or collision, move, tally, sequence, new direction.
__device__ __forceinline__ void ev_move(const KParams &p, const KOut &o, const EvBank &b, uint64_t *rep, uint64_t i,
                                        Counts &cnt) {
    const uint32_t st = b.st[i];
    if (!(st & kEvDone)) {
        const uint64_t local = i, pid = p.first + i;
        double tau = b.tau[i];
        const double t = b.t[i], sig = b.sig[i];
        const uint32_t inst = b.inst[i];
        bool recovf = (st & kEvRecOvf) != 0;
        int end = GT_END_NONE;
        const double sc = (p.source == 1) ? dinf() : tau / sig;
        const bool boundary = t < sc;
        if (!boundary && sc == dinf()) {
            end = GT_END_LOST;
            b.st[i] = st | kEvDone | (uint32_t)end << 8;
            ev_finish(b, o, rep, i, end, recovf, cnt);
        } else {
            double l;
            if (boundary) {
                l = t;
                if (p.source != 1) tau = tau - sig * t;
            } else {
                l = sc;
            }
            double u = b.u[i], v = b.v[i], w = b.w[i];
            const double m0 = l * u, m1 = l * v, m2 = l * w;
            b.x[i] = b.x[i] + m0;
            b.y[i] = b.y[i] + m1;
            b.z[i] = b.z[i] + m2;
            TallyAcc acc;
            acc.inst = b.acc_inst[i];
            acc.lo = b.acc_lo[i];
            acc.hi = b.acc_hi[i];
            tally_add(rep, acc, inst, l);
            b.acc_inst[i] = acc.inst;
            b.acc_lo[i] = acc.lo;
            b.acc_hi[i] = acc.hi;
            b.h[i] = (b.h[i] ^ ((uint64_t)inst + 1)) * kFnvPrime;
            uint32_t segs = b.segs[i];
            if (local < p.rec_k) {
                if (segs < p.rec_cap) gstore(o.rec, local * (uint64_t)p.rec_cap + segs, inst);
                else recovf = true;
            }
            segs++;
            b.segs[i] = segs;
            uint32_t nst = st & ~(kEvRecOvf | kEvPending);
            if (recovf) nst |= kEvRecOvf;
            if (boundary) {
                nst |= kEvPending;
            } else {
                // collision: off every surface, then CAP or a new direction and depth
                nst = (nst & ~(0xFu << 4));
                b.on_surf[i] = kNone;
                const uint32_t ncoll = b.ncoll[i] + 1;
                b.ncoll[i] = ncoll;
                if (ncoll >= p.max_coll) {
                    end = GT_END_CAP;
                } else {
                    uint32_t blk = b.blk[i];
                    double u0, u1, u2;
                    do draw_block(p.seed, p.geom_id, pid, blk++, u0, u1, u2);
                    while (!direction_from(u0, u1, u, v, w));
                    tau = -series_log(u2);
                    b.blk[i] = blk;
                    b.u[i] = u;
                    b.v[i] = v;
                    b.w[i] = w;
                }
                if (end == GT_END_NONE && segs >= p.max_segs) end = GT_END_SEGCAP;
            }
            b.tau[i] = tau;
            if (end != GT_END_NONE) nst |= kEvDone | (uint32_t)end << 8;
            b.st[i] = nst;
            if (end != GT_END_NONE) ev_finish(b, o, rep, i, end, recovf, cnt);
        }
    }
}

// cross_surface for history i if its segment ended on a surface; true while
// the history goes on.
template <int PREC, typename G>
__device__ __forceinline__ bool ev_cross(const G &g, const KParams &p, const KOut &o, const EvBank &b, uint64_t *rep,
                                         uint64_t i, uint32_t *cells, Counts &cnt) {
    uint32_t st = b.st[i];
    if (!(st & kEvDone) && (st & kEvPending)) {
        Particle P;
        P.cell = cells;
        ev_load(b, p.n, i, st, P);
        const int bl = (int)((st >> 12) & 15u);
        const bool bpos = (st >> 16) & 1u;
        int end = cross_listed<PREC>(g, P, bl, b.surf[i], bpos, b.entry[i]);
        ev_store_geom(b, p.n, i, P);
        if (end == GT_END_NONE && b.segs[i] >= p.max_segs) end = GT_END_SEGCAP;
        const bool recovf = (st & kEvRecOvf) != 0;
        st = ev_pack(P.depth, P.on_level, end, bl, bpos, false, recovf, end != GT_END_NONE);
        b.st[i] = st;
        if (end != GT_END_NONE) ev_finish(b, o, rep, i, end, recovf, cnt);
    }
    return !(st & kEvDone);
}

// Fold the replicas' limb counters of instance i into the 128-bit
// fixed-point total (plus the previous total when accumulating), then convert
// it to cm: high word * 2^-32 + low word * 2^-96.
__device__ __forceinline__ void fold_tally(const uint64_t *ws, uint64_t *tfx, double *tally, uint64_t n, uint64_t i,
                                           bool accumulate) {
    uint64_t lo = accumulate ? tfx[2 * i] : 0, hi = accumulate ? tfx[2 * i + 1] : 0;
    const uint32_t nrep = tally_replicas(n);
    for (uint32_t r = 0; r < nrep; r++) {
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

}  // namespace
}  // namespace gt
