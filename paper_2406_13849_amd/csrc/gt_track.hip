// HIP kernels of libgt for gfx950 (CDNA4): Monte Carlo geometry tracking
// through nested CSG universes with one CSG tracker and per-universe
// bounding-volume hierarchies (Section "Single tracker (ST) method").
//
// One lane carries one history at a time; its whole state (position,
// direction, optical depth, the cell at every level, random-stream
// position, tally accumulator) lives in registers.  Geometry tables are
// read-only and shared by all lanes.
//
// Floating point: compiled with -ffp-contract=off and no fast-math, so every
// double operation below is one IEEE operation in the order written; the
// results of find_cell / distance_to_surface / cross_surface are therefore
// the ones a plain double-precision implementation of the same definitions
// computes.  Single precision only appears in the optional candidate
// pruning (widened, outward-rounded boxes and a lattice-index guess), which
// can skip a cell only when that cell cannot contain the point.
#pragma clang fp contract(off)

#include "gt_internal.h"

namespace gt {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxBirthAttempts = 1000;
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;

__device__ __forceinline__ double dinf() { return __builtin_huge_val(); }

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, the key bumped by the
// published Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

// Stream of 64-bit words of one particle: word k is half (k & 1) of block
// k >> 1 under counter (block, id lo, id hi, geometry id), low half first.
struct Stream {
    uint64_t key, pid, stash;
    uint32_t gid, k;

    __device__ __forceinline__ uint64_t word() {
        uint64_t w;
        if (k & 1u) {
            w = stash;
        } else {
            uint32_t o0, o1, o2, o3;
            philox4x32_10(k >> 1, (uint32_t)pid, (uint32_t)(pid >> 32), gid, (uint32_t)key, (uint32_t)(key >> 32),
                          o0, o1, o2, o3);
            w = ((uint64_t)o1 << 32) | o0;
            stash = ((uint64_t)o3 << 32) | o2;
        }
        k++;
        return w;
    }
    // uniform on (0,1): top 52 bits plus one half, times 2^-52 (exact)
    __device__ __forceinline__ double u01() { return ((double)(word() >> 12) + 0.5) * 0x1p-52; }
};

// Natural logarithm from log m = 2 atanh(s), s = (m-1)/(m+1), m in
// [sqrt(1/2), sqrt(2)), twelve odd-power terms with coefficients 1/(2k+1)
// (each the correctly rounded quotient), and e*ln2 split in a 32-bit head
// (exact products) and a tail.  Used for the exponential optical depth.
__device__ __forceinline__ double series_log(double x) {
    uint64_t bits = (uint64_t)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ffu) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    const double sqrt2 = __longlong_as_double(0x3FF6A09E667F3BCDll);
    if (m >= sqrt2) { m = m * 0.5; e = e + 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
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
    double logm = (s + s) * poly;
    const double ln2_hi = __longlong_as_double(0x3FE62E42FEE00000ll);
    const double ln2_lo = __longlong_as_double(0x3DEA39EF35793C76ll);
    double de = (double)e;
    return de * ln2_hi + (de * ln2_lo + logm);
}

// ------------------------------------------------------------------ surfaces
// f(p); the positive side is f > 0 (outside of cylinders and spheres)
__device__ __forceinline__ double surf_value(uint32_t type, const double *c, double x, double y, double z) {
    switch (type) {
    case ST_PX: return x - c[0];
    case ST_PY: return y - c[0];
    case ST_PZ: return z - c[0];
    case ST_P: return ((c[0] * x + c[1] * y) + c[2] * z) - c[3];
    case ST_CZ: {
        double dx = x - c[0], dy = y - c[1];
        return (dx * dx + dy * dy) - c[2];
    }
    default: {
        double dx = x - c[0], dy = y - c[1], dz = z - c[2];
        return ((dx * dx + dy * dy) + dz * dz) - c[3];
    }
    }
}

// Cell containment: the point is on the required side of every half-space;
// on surface force_s the logical sense force_pos is used instead.
__device__ __forceinline__ bool contains(const Dev &g, uint32_t c, double x, double y, double z, uint32_t force_s,
                                         bool force_pos) {
    const Cell cc = g.cell[c];
    for (uint32_t k = 0; k < cc.hs_n; k++) {
        uint32_t h = g.hs[cc.hs_off + k];
        uint32_t s = h >> 4;
        bool want = (h >> 3) & 1u;
        bool pos = (s == force_s) ? force_pos : (surf_value(h & 7u, g.coef + 4 * (size_t)s, x, y, z) > 0.0);
        if (pos != want) return false;
    }
    return true;
}

// Distance along (u,v,w) from q to the point where the sense of surface s
// leaves the cell's required side `pos`; +inf if it does not.  `on` marks the
// surface the particle has just crossed (Table 1 distance_to_surface).
__device__ __forceinline__ double hs_distance(uint32_t type, const double *c, bool pos, double qx, double qy,
                                              double qz, double u, double v, double w, bool on) {
    double t;
    if (type <= ST_P) {
        if (on) return dinf();
        double den;
        switch (type) {
        case ST_PX: den = u; break;
        case ST_PY: den = v; break;
        case ST_PZ: den = w; break;
        default: den = (c[0] * u + c[1] * v) + c[2] * w; break;
        }
        if (den == 0.0) return dinf();
        if (!((!pos && den > 0.0) || (pos && den < 0.0))) return dinf();
        t = (-surf_value(type, c, qx, qy, qz)) / den;
    } else {
        double a, b;
        double dx = qx - c[0], dy = qy - c[1];
        if (type == ST_CZ) {
            a = u * u + v * v;
            b = dx * u + dy * v;
        } else {
            double dz = qz - c[2];
            a = (u * u + v * v) + w * w;
            b = (dx * u + dy * v) + dz * w;
        }
        if (a == 0.0) return dinf();
        if (on) {
            if (!pos && b < 0.0) t = (-2.0 * b) / a;
            else return dinf();
        } else {
            double cc = surf_value(type, c, qx, qy, qz);
            double disc = b * b - a * cc;
            if (!(disc > 0.0)) return dinf();
            double q = sqrt(disc);
            if (!pos) {
                t = (b <= 0.0) ? (q - b) / a : (-cc) / (b + q);
            } else {
                if (b < 0.0) t = cc / (q - b);
                else return dinf();
            }
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
template <int PREC>
__device__ int32_t search(const Dev &g, uint32_t u, double x, double y, double z, uint32_t force_s, bool force_pos,
                          int32_t exclude, float gx, float gy) {
    const Univ U = g.univ[u];
    if (PREC == GT_PREC_MIXED && U.hint == (int32_t)kHintSquare) {
        int i = (int)floorf((gx - U.x0) * U.inv_px);
        int j = (int)floorf((gy - U.y0) * U.inv_py);
        i = min(max(i, 0), U.nx - 1);
        j = min(max(j, 0), U.ny - 1);
        int32_t c = (int32_t)U.cell0 + j * U.nx + i;
        if (c != exclude && contains(g, (uint32_t)c, x, y, z, force_s, force_pos)) return c;
    }
    uint32_t n = U.node0;
    const uint32_t end = U.node0 + U.nnode;
    const float fx = (float)x, fy = (float)y, fz = (float)z;
    while (n < end) {
        bool in;
        uint32_t esc, lf;
        if (PREC == GT_PREC_MIXED) {
            const Node32 nd = g.node32[n];
            in = fx >= nd.lo[0] && fx <= nd.hi[0] && fy >= nd.lo[1] && fy <= nd.hi[1] && fz >= nd.lo[2] &&
                 fz <= nd.hi[2];
            esc = nd.escape;
            lf = nd.leaf;
        } else {
            const Node64 nd = g.node64[n];
            in = x >= nd.lo[0] && x <= nd.hi[0] && y >= nd.lo[1] && y <= nd.hi[1] && z >= nd.lo[2] && z <= nd.hi[2];
            esc = nd.escape;
            lf = nd.leaf;
        }
        if (!in) { n = esc; continue; }
        if (lf == kLeafNone) { n++; continue; }
        const uint32_t first = lf >> 4, cnt = (lf & 15u) + 1;
        for (uint32_t k = 0; k < cnt; k++) {
            uint32_t c = g.leaf[first + k];
            if ((int32_t)c == exclude) continue;
            if (PREC == GT_PREC_MIXED) {
                const float *b = g.cbox + 8 * (size_t)c;
                if (!(fx >= b[0] && fx <= b[4] && fy >= b[1] && fy <= b[5] && fz >= b[2] && fz <= b[6])) continue;
            }
            if (contains(g, c, x, y, z, force_s, force_pos)) return (int32_t)c;
        }
        n = esc;
    }
    return -1;
}

// ------------------------------------------------------------------ particle
constexpr int kBlock = 256;       // lanes per workgroup of the one-history-per-lane kernels
constexpr int kBlockP = 1024;     // lanes per workgroup of the persistent tracker (launch bound)

// Per-lane state.  The cell of every level lives in LDS, one column per
// lane (cell[L * blockDim.x]), so that level loops index it dynamically
// without spilling and without unrolling the per-level search code.
struct Particle {
    double x, y, z, u, v, w, tau;
    uint32_t *cell;
    int depth;
    int on_level;
    uint32_t on_surf;
};

__device__ __forceinline__ uint32_t &lvl(const Particle &P, int L) { return P.cell[L * (int)blockDim.x]; }

// Descend from level L0 (cell set, (qx,qy,qz) its local position): while
// the cell is filled, find the daughter's cell at p - t (Alg. 7).
template <int PREC>
__device__ __forceinline__ bool descend(const Dev &g, Particle &P, int L0, double qx, double qy, double qz) {
    int L = L0;
    for (;;) {
        const uint32_t c = lvl(P, L);
        const int32_t fill = g.cell[c].fill;
        if (fill >= 0) break;
        const double *t = g.trans + 4 * (size_t)c;
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

__device__ __forceinline__ uint32_t leaf_instance(const Dev &g, const Particle &P) {
    uint32_t i = 0;
    for (int L = 0; L < P.depth; L++) i += g.cell[lvl(P, L)].inst_off;
    return i;
}

// distance_to_surface over every level; ties resolve to the smallest
// (distance, level, surface id), i.e. the top-most level on the surface.
__device__ __forceinline__ double distance_all(const Dev &g, const Particle &P, int &bl, uint32_t &bs, bool &bpos) {
    double bt = dinf();
    bl = GT_MAX_LEVELS;
    bs = kNone;
    bpos = false;
    double qx = P.x, qy = P.y, qz = P.z;
    for (int L = 0; L < P.depth; L++) {
        const uint32_t c = lvl(P, L);
        if (L > 0) {
            const double *t = g.trans + 4 * (size_t)lvl(P, L - 1);
            qx = qx - t[0];
            qy = qy - t[1];
            qz = qz - t[2];
        }
        const Cell cc = g.cell[c];
        for (uint32_t k = 0; k < cc.hs_n; k++) {
            const uint32_t h = g.hs[cc.hs_off + k];
            const uint32_t s = h >> 4;
            const bool pos = (h >> 3) & 1u;
            const bool on = (P.on_level == L) && (P.on_surf == s);
            const double d = hs_distance(h & 7u, g.coef + 4 * (size_t)s, pos, qx, qy, qz, P.u, P.v, P.w, on);
            if (d < bt || (d == bt && d != dinf() && L == bl && s < bs)) {
                bt = d;
                bl = L;
                bs = s;
                bpos = pos;
            }
        }
    }
    return bt;
}

// cross_surface at level L* on surface s* (Alg. 8): the cell of that level's
// universe on the other side (the old cell's sense on s* flipped), then
// descent below it.  Returns an end code (GT_END_NONE if tracking goes on).
template <int PREC>
__device__ __forceinline__ int cross(const Dev &g, Particle &P, int Ls, uint32_t ss, bool old_pos) {
    double qx = P.x, qy = P.y, qz = P.z;
    uint32_t univ = g.root;
    for (int L = 0; L < Ls; L++) {
        const uint32_t c = lvl(P, L);
        const double *t = g.trans + 4 * (size_t)c;
        qx = qx - t[0];
        qy = qy - t[1];
        qz = qz - t[2];
        univ = (uint32_t)(-g.cell[c].fill - 1);
    }
    const uint32_t old = lvl(P, Ls);
    // guess point nudged along the flight so that a lattice guess lands on the far side
    float gx = (float)qx, gy = (float)qy;
    if (PREC == GT_PREC_MIXED) {
        const Univ U = g.univ[univ];
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

__device__ __forceinline__ void sample_direction(Stream &rng, double &u, double &v, double &w) {
    double v1, v2, s;
    for (;;) {
        v1 = 2.0 * rng.u01() - 1.0;
        v2 = 2.0 * rng.u01() - 1.0;
        s = v1 * v1 + v2 * v2;
        if (s < 1.0 && s != 0.0) break;
    }
    const double r = sqrt(1.0 - s);
    u = (2.0 * v1) * r;
    v = (2.0 * v2) * r;
    w = 1.0 - 2.0 * s;
}

// 128-bit fixed-point accumulator of segment lengths, quantum 2^-96 cm
struct TallyAcc {
    uint32_t inst;
    uint64_t lo, hi;
};

__device__ __forceinline__ void tally_flush(uint64_t *tfx, TallyAcc &a) {
    if (a.inst == kNone) return;
    unsigned long long *p = (unsigned long long *)(tfx + 2 * (size_t)a.inst);
    const unsigned long long old = atomicAdd(p, (unsigned long long)a.lo);
    const uint64_t carry = (old + a.lo < old) ? 1u : 0u;
    const uint64_t h = a.hi + carry;
    if (h) atomicAdd(p + 1, (unsigned long long)h);
    a.inst = kNone;
}

__device__ __forceinline__ void tally_add(uint64_t *tfx, TallyAcc &a, uint32_t inst, double l) {
    const double v = l * 0x1p32;
    const double fl = floor(v);
    const double fr = v - fl;
    const uint64_t hi = (uint64_t)fl;
    const uint64_t lo = (uint64_t)(fr * 0x1p64);
    if (inst != a.inst) {
        tally_flush(tfx, a);
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

// One history: Alg. 2 with the toy transport.
template <int PREC>
__device__ void run_history(const Dev &g, const KParams &p, const KOut &o, uint64_t local, uint32_t *cells,
                            Counts &cnt) {
    Particle P;
    P.cell = cells;
    Stream rng;
    rng.key = p.seed;
    rng.pid = p.first + local;
    rng.gid = p.geom_id;
    rng.k = 0;
    rng.stash = 0;
    P.on_level = -1;
    P.on_surf = kNone;
    P.depth = 1;
    int end = GT_END_NONE;
    // ---- birth
    if (p.source == 1) {
        const uint64_t n1 = p.ray_n1;
        const uint64_t n2 = (p.n + n1 - 1) / n1;
        const uint64_t j = rng.pid % n1, k = rng.pid / n1;
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
            P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * rng.u01();
            P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * rng.u01();
            P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * rng.u01();
            c = search<PREC>(g, g.root, P.x, P.y, P.z, kNone, false, -1, (float)P.x, (float)P.y);
            if (c < 0) cnt.rejected++;
        }
        if (c < 0) {
            end = GT_END_LOST;
        } else {
            lvl(P, 0) = (uint32_t)c;
            if (!descend<PREC>(g, P, 0, P.x, P.y, P.z)) end = GT_END_LOST;
            sample_direction(rng, P.u, P.v, P.w);
            P.tau = -series_log(rng.u01());
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
        uint32_t bs;
        bool bpos;
        const double dist = distance_all(g, P, bl, bs, bpos);
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
        tally_add(o.tally_fx, acc, inst, l);
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
                sample_direction(rng, P.u, P.v, P.w);
                P.tau = -series_log(rng.u01());
            }
        }
        if (end == GT_END_NONE && segs >= p.max_segs) end = GT_END_SEGCAP;
    }
    tally_flush(o.tally_fx, acc);
    h ^= (uint64_t)end;
    if (o.seg_count) o.seg_count[local] = segs;
    if (o.seq_hash) o.seq_hash[local] = h;
    if (o.end_code) o.end_code[local] = (uint8_t)end;
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


// ------------------------------------------------------------------ persistent tracker
// Each lane runs a small state machine; a wave loops until the shared
// particle pool is drained and all of its lanes are idle.  Finished lanes
// are refilled at once from a wave-local pool of particle ids (ballot +
// per-lane rank, one global atomic per 64 ids), so a wave no longer waits
// for its longest history.  The candidate search, the sampling and the
// segment step each have a single call site, so lanes that are at different
// steps of their histories share one instruction stream per step.
enum Mode : int { M_IDLE = 0, M_POS = 1, M_SEARCH = 2, M_SAMPLE = 3, M_TRACK = 4 };

constexpr uint32_t kChunk = 64;

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <int PREC>
__global__ void __launch_bounds__(kBlockP) k_track_persistent(Dev g, KParams p, KOut o) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlockP];
    unsigned long long *queue = (unsigned long long *)&o.counters[7];
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    Particle P;
    P.cell = cells + threadIdx.x;
    Stream rng;
    rng.key = p.seed;
    rng.gid = p.geom_id;
    int mode = M_IDLE;
    uint64_t local = 0;
    // history state
    uint64_t h = 0;
    uint32_t segs = 0, ncoll = 0, attempts = 0;
    bool recovf = false, birth = false;
    TallyAcc acc;
    acc.inst = kNone;
    acc.lo = acc.hi = 0;
    // pending search: universe su at local point (qx,qy,qz) for level sL
    int sL = 0;
    uint32_t su = 0, sforce = kNone;
    bool sfpos = false;
    int32_t sexcl = -1;
    double qx = 0, qy = 0, qz = 0;
    float gx = 0, gy = 0;
    // wave-uniform pool of particle ids
    uint64_t pool_next = 0, pool_end = 0;
    bool drained = false;
    int end = GT_END_NONE;

    for (;;) {
        // ---- refill idle lanes
        if (!drained) {
            uint64_t idle = __ballot(mode == M_IDLE);
            while (idle) {
                if (pool_next == pool_end) {
                    const int leader = __ffsll((unsigned long long)idle) - 1;
                    unsigned long long base = 0;
                    if ((int)__lane_id() == leader) base = atomicAdd(queue, (unsigned long long)kChunk);
                    base = __shfl(base, leader);
                    if (base >= p.n) { drained = true; break; }
                    pool_next = base;
                    pool_end = min((uint64_t)base + kChunk, p.n);
                }
                const uint64_t avail = pool_end - pool_next;
                const uint32_t r = lane_rank(idle);
                if (mode == M_IDLE && r < avail) {
                    local = pool_next + r;
                    rng.pid = p.first + local;
                    rng.k = 0;
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
        if (__ballot(mode != M_IDLE) == 0) break;

        // ---- birth position (uniform in the box, retried until a root cell has it)
        if (mode == M_POS) {
            if (p.source == 1) {
                const uint64_t n1 = p.ray_n1;
                const uint64_t n2 = (p.n + n1 - 1) / n1;
                const uint64_t j = rng.pid % n1, k = rng.pid / n1;
                const double hy = (g.hi[1] - g.lo[1]) / (double)n1;
                const double hz = (g.hi[2] - g.lo[2]) / (double)n2;
                P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * 0x1p-30;
                P.y = g.lo[1] + ((double)j + 0.5) * hy;
                P.z = g.lo[2] + ((double)k + 0.5) * hz;
                P.u = 1.0;
                P.v = 0.0;
                P.w = 0.0;
                P.tau = 0.0;
                mode = M_SEARCH;
            } else if (attempts >= (uint32_t)kMaxBirthAttempts) {
                end = GT_END_LOST;
            } else {
                P.x = g.lo[0] + (g.hi[0] - g.lo[0]) * rng.u01();
                P.y = g.lo[1] + (g.hi[1] - g.lo[1]) * rng.u01();
                P.z = g.lo[2] + (g.hi[2] - g.lo[2]) * rng.u01();
                attempts++;
                mode = M_SEARCH;
            }
            sL = 0;
            su = g.root;
            sforce = kNone;
            sexcl = -1;
            qx = P.x;
            qy = P.y;
            qz = P.z;
            gx = (float)qx;
            gy = (float)qy;
        }

        // ---- one level of find_cell / cross_surface
        if (mode == M_SEARCH) {
            const int32_t c = search<PREC>(g, su, qx, qy, qz, sforce, sfpos, sexcl, gx, gy);
            if (c < 0) {
                if (birth) {
                    if (sL == 0 && p.source != 1) { cnt.rejected++; mode = M_POS; }
                    else end = GT_END_LOST;
                } else {
                    end = (sforce != kNone && sL == 0) ? GT_END_ESCAPE : GT_END_LOST;
                }
            } else {
                lvl(P, sL) = (uint32_t)c;
                const int32_t fill = g.cell[c].fill;
                if (fill < 0) {
                    const double *t = g.trans + 4 * (size_t)c;
                    qx = qx - t[0];
                    qy = qy - t[1];
                    qz = qz - t[2];
                    gx = (float)qx;
                    gy = (float)qy;
                    su = (uint32_t)(-fill - 1);
                    sL++;
                    sforce = kNone;
                    sexcl = -1;
                } else {
                    P.depth = sL + 1;
                    if (birth) {
                        birth = false;
                        mode = p.source == 1 ? M_TRACK : M_SAMPLE;
                    } else {
                        if (segs >= p.max_segs) end = GT_END_SEGCAP;
                        mode = M_TRACK;
                    }
                }
            }
        }

        // ---- change_direction and a new optical depth
        if (mode == M_SAMPLE && end == GT_END_NONE) {
            sample_direction(rng, P.u, P.v, P.w);
            P.tau = -series_log(rng.u01());
            mode = M_TRACK;
        }

        // ---- one segment: distance_to_surface, move, tally, then crossing or collision
        if (mode == M_TRACK && end == GT_END_NONE) {
            int bl;
            uint32_t bs;
            bool bpos;
            const double dist = distance_all(g, P, bl, bs, bpos);
            const uint32_t lc = lvl(P, P.depth - 1);
            const double sig = g.sigma[g.cell[lc].fill];
            const double sc = (p.source == 1) ? dinf() : P.tau / sig;
            const uint32_t inst = leaf_instance(g, P);
            const bool boundary = dist < sc;
            if (!boundary && sc == dinf()) {
                end = GT_END_LOST;
            } else {
                double l;
                if (boundary) {
                    l = dist;
                    if (p.source != 1) P.tau = P.tau - sig * dist;
                } else {
                    l = sc;
                }
                const double m0 = l * P.u, m1 = l * P.v, m2 = l * P.w;
                P.x = P.x + m0;
                P.y = P.y + m1;
                P.z = P.z + m2;
                tally_add(o.tally_fx, acc, inst, l);
                h = (h ^ ((uint64_t)inst + 1)) * kFnvPrime;
                if (local < p.rec_k) {
                    if (segs < p.rec_cap) o.rec[local * (uint64_t)p.rec_cap + segs] = (int32_t)inst;
                    else recovf = true;
                }
                segs++;
                if (boundary) {
                    // set up cross_surface at level bl on surface bs (Alg. 8)
                    qx = P.x;
                    qy = P.y;
                    qz = P.z;
                    su = g.root;
                    for (int L = 0; L < bl; L++) {
                        const uint32_t c = lvl(P, L);
                        const double *t = g.trans + 4 * (size_t)c;
                        qx = qx - t[0];
                        qy = qy - t[1];
                        qz = qz - t[2];
                        su = (uint32_t)(-g.cell[c].fill - 1);
                    }
                    sL = bl;
                    sforce = bs;
                    sfpos = !bpos;
                    sexcl = (int32_t)lvl(P, bl);
                    gx = (float)qx;
                    gy = (float)qy;
                    if (PREC == GT_PREC_MIXED) {
                        const Univ U = g.univ[su];
                        if (U.hint == (int32_t)kHintSquare) {
                            gx += (float)P.u * 1e-3f / U.inv_px;
                            gy += (float)P.v * 1e-3f / U.inv_py;
                        }
                    }
                    P.on_level = bl;
                    P.on_surf = bs;
                    mode = M_SEARCH;
                } else {
                    P.on_level = -1;
                    P.on_surf = kNone;
                    ncoll++;
                    if (ncoll >= p.max_coll) end = GT_END_CAP;
                    else if (segs >= p.max_segs) end = GT_END_SEGCAP;
                    else mode = M_SAMPLE;
                }
            }
        }

        // ---- history finished: outputs, then the lane is free
        if (mode != M_IDLE && end != GT_END_NONE) {
            tally_flush(o.tally_fx, acc);
            h ^= (uint64_t)end;
            if (o.seg_count) o.seg_count[local] = segs;
            if (o.seq_hash) o.seq_hash[local] = h;
            if (o.end_code) o.end_code[local] = (uint8_t)end;
            cnt.segments += segs;
            cnt.escaped += end == GT_END_ESCAPE;
            cnt.capped += end == GT_END_CAP;
            cnt.lost += end == GT_END_LOST;
            cnt.segcap += end == GT_END_SEGCAP;
            cnt.recovf += recovf;
            mode = M_IDLE;
        }
    }
    add_counts(cnt, o.counters);
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_track(Dev g, KParams p, KOut o) {
    __shared__ uint32_t cells[GT_MAX_LEVELS * kBlock];
    Counts cnt = {0, 0, 0, 0, 0, 0, 0};
    const uint64_t local = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (local < p.n) run_history<PREC>(g, p, o, local, cells + threadIdx.x, cnt);
    add_counts(cnt, o.counters);
}

__global__ void k_fill_u64(uint64_t *a, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_fill_i32(int32_t *a, uint64_t n, int32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// fixed point (units of 2^-96 cm) to double: high word * 2^-32 + low * 2^-96
__global__ void k_finalize(const uint64_t *tfx, double *tally, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        tally[i] = (double)tfx[2 * i + 1] * 0x1p-32 + (double)tfx[2 * i] * 0x1p-96;
}

template <int PREC>
__global__ void __launch_bounds__(kBlock) k_find_cell(Dev g, const double *pos, uint64_t n, int64_t *inst,
                                                      int32_t *cells) {
    __shared__ uint32_t lc[GT_MAX_LEVELS * kBlock];
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

__global__ void __launch_bounds__(kBlock) k_distance(Dev g, const double *pos, const double *dir, uint64_t n,
                                                     double *dist, int32_t *level, int32_t *surf) {
    __shared__ uint32_t lc[GT_MAX_LEVELS * kBlock];
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
    uint32_t bs;
    bool bpos;
    const double d = distance_all(g, P, bl, bs, bpos);
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
// occupancy the kernel's resources allow), cached per device and block size.
int persistent_grid(const void *kernel, unsigned block, int device, int *blocks) {
    static int cache_dev[64], cache_block[64], cache_n[64];
    static const void *cache_k[64];
    static int used = 0;
    for (int i = 0; i < used; i++)
        if (cache_k[i] == kernel && cache_dev[i] == device && cache_block[i] == (int)block) {
            *blocks = cache_n[i];
            return GT_OK;
        }
    int cus = 0, per = 0;
    int rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device), "hipDeviceGetAttribute");
    if (rc) return rc;
    rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)block, 0),
                   "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (rc) return rc;
    if (per < 1) per = 1;
    *blocks = cus * per;
    if (used < 64) {
        cache_k[used] = kernel;
        cache_dev[used] = device;
        cache_block[used] = (int)block;
        cache_n[used] = *blocks;
        used++;
    }
    return GT_OK;
}

template <int PREC>
int launch_track_t(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, hipStream_t st) {
    KParams kp;
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
    kp.pad = 0;
    KOut ko;
    ko.tally_fx = o->tally_fx;
    ko.seg_count = o->seg_count;
    ko.seq_hash = o->seq_hash;
    ko.end_code = o->end_code;
    ko.rec = o->rec;
    ko.counters = o->counters;
    if (!(p->flags & GT_FLAG_ACCUMULATE))
        hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(2 * g->n_inst)), dim3(256), 0, st, o->tally_fx, 2 * g->n_inst,
                           (uint64_t)0);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, o->counters, (uint64_t)8, (uint64_t)0);
    if (kp.rec_k) {
        const uint64_t nrec = (uint64_t)kp.rec_k * kp.rec_cap;
        hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(nrec)), dim3(256), 0, st, o->rec, nrec, (int32_t)-1);
    }
    if (kp.n) {
        if (p->flags & GT_FLAG_LANE_PER_HISTORY) {
            const unsigned block = p->block_size ? p->block_size : kBlock;
            hipLaunchKernelGGL((k_track<PREC>), dim3(grid_for(kp.n, block)), dim3(block), 0, st, g->dev, kp, ko);
        } else {
            const unsigned block = p->block_size ? p->block_size : kBlockP;
            int blocks = 0;
            int rc = persistent_grid((const void *)k_track_persistent<PREC>, block, g->device, &blocks);
            if (rc) return rc;
            const uint64_t need = (kp.n + block - 1) / block;
            if ((uint64_t)blocks > need) blocks = (int)need;
            hipLaunchKernelGGL((k_track_persistent<PREC>), dim3(blocks), dim3(block), 0, st, g->dev, kp, ko);
        }
    }
    if (o->tally)
        hipLaunchKernelGGL(k_finalize, dim3(fill_grid(g->n_inst)), dim3(256), 0, st, o->tally_fx, o->tally, g->n_inst);
    return hip_check(hipGetLastError(), "gt_track launch");
}

}  // namespace

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
