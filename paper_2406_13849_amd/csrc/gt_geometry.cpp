// Host side of libgt: validation of a flattened geometry, preprocessing into
// device tables, one upload, and the extern "C" entry points.
//
// Preprocessing steps:
//   1. validation (ranges, surface ownership, acyclic fills, depth);
//   2. leaf-instance numbering: a material cell counts one instance, a
//      filled cell the instances of its daughter (per-instance cell tallies,
//      Section "Empire microreactor" tallies every pin sub-cell instance);
//   3. reachable extent of every universe, propagated from the root's
//      sampling box through each filled cell's box minus its translation;
//   4. an axis-aligned box per cell: the universe extent clipped by the
//      cell's axis planes, the boxes of its inside-of-cylinder/sphere
//      half-spaces, and the polygon cut out by its vertical general planes
//      (exact convex clipping, where the paper truncates the universe box by
//      each surface's bounding planes), then widened outward by a margin far
//      larger than any rounding in the point evaluation;
//   5. per universe a bounding-volume hierarchy over those boxes, split with
//      the surface-area heuristic over three equally spaced candidate planes
//      per axis (Section "Single tracker (ST) method"); children may
//      overlap and every cell appears once;
//   6. single-precision copies of all boxes rounded outward (lower bounds
//      down, upper bounds up), so a point rounded to nearest can never be
//      rejected by a box that contains it in double precision.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "gt_internal.h"

namespace gt {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

namespace {

struct Box {
    double lo[3], hi[3];
    static Box empty() {
        Box b;
        for (int k = 0; k < 3; k++) { b.lo[k] = INFINITY; b.hi[k] = -INFINITY; }
        return b;
    }
    bool is_empty() const { return lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]; }
    void grow(const Box &o) {
        for (int k = 0; k < 3; k++) { lo[k] = std::min(lo[k], o.lo[k]); hi[k] = std::max(hi[k], o.hi[k]); }
    }
    void widen(double d) {
        for (int k = 0; k < 3; k++) { lo[k] -= d; hi[k] += d; }
    }
    double area() const {
        double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct HalfPlane { double a, b, d; bool pos; };

// Sutherland-Hodgman clip of a convex polygon by a closed half-plane.
static void clip_polygon(std::vector<double> &px, std::vector<double> &py, const HalfPlane &h) {
    std::vector<double> ox, oy;
    size_t n = px.size();
    auto val = [&](size_t i) {
        double f = (h.a * px[i] + h.b * py[i]) - h.d;
        return h.pos ? f : -f;   // keep val >= 0
    };
    for (size_t i = 0; i < n; i++) {
        size_t j = (i + 1) % n;
        double vi = val(i), vj = val(j);
        if (vi >= 0) { ox.push_back(px[i]); oy.push_back(py[i]); }
        if ((vi >= 0) != (vj >= 0)) {
            double t = vi / (vi - vj);
            ox.push_back(px[i] + t * (px[j] - px[i]));
            oy.push_back(py[i] + t * (py[j] - py[i]));
        }
    }
    px.swap(ox);
    py.swap(oy);
}

static float round_down(double v) {
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -INFINITY);
    return f;
}

static float round_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}

struct Builder {
    const gt_flat_geometry *f;
    std::vector<uint32_t> cell_univ;
    std::vector<uint64_t> ninst, inst_off;
    std::vector<uint32_t> depth;
    std::vector<Box> ext, cbox;
    std::vector<uint8_t> reached;
    std::vector<uint32_t> topo;
    double delta = 0;
    // outputs
    std::vector<Node32> n32;
    std::vector<Node64> n64;
    std::vector<uint32_t> leaf;
    std::vector<Univ> univ;

    // universe kinds for the trackers that switch on them (see UArr)
    std::vector<UArr> uarr;
    std::vector<double> aval;
    std::vector<uint32_t> asurf, ahs, cell_ij;
    uint32_t rtk_shape = 0;

    uint32_t surf_of(int32_t h) const { return (uint32_t)(h < 0 ? -(int64_t)h : h) - 1; }

    int validate() {
        const gt_flat_geometry &F = *f;
        if (F.n_universes == 0 || F.n_cells == 0) { set_error("geometry has no universes or cells"); return GT_EGEOM; }
        if (!F.surf_type && F.n_surfaces) return set_error("surf_type is NULL"), GT_EINVAL;
        if (!F.surf_coef && F.n_surfaces) return set_error("surf_coef is NULL"), GT_EINVAL;
        if (!F.cell_hs_off || !F.cell_fill || !F.cell_trans || !F.univ_cell_off || !F.sigma_t ||
            (!F.hs && F.n_halfspaces))
            return set_error("a required geometry array is NULL"), GT_EINVAL;
        if (F.root >= F.n_universes) return set_error("root universe %u out of range", F.root), GT_EGEOM;
        if (F.n_surfaces >= (1u << 28)) return set_error("too many surfaces (%u)", F.n_surfaces), GT_ECAPACITY;
        for (uint32_t s = 0; s < F.n_surfaces; s++) {
            if (F.surf_type[s] > ST_SPH) return set_error("surface %u: unknown type %u", s, F.surf_type[s]), GT_EGEOM;
            for (int k = 0; k < 8; k++)
                if (!std::isfinite(F.surf_coef[8 * (size_t)s + k]))
                    return set_error("surface %u: non-finite coefficient", s), GT_EGEOM;
            if (F.surf_type[s] == ST_CZ && !(F.surf_coef[8 * (size_t)s + 2] > 0))
                return set_error("surface %u: cylinder r^2 must be > 0", s), GT_EGEOM;
            if (F.surf_type[s] == ST_SPH && !(F.surf_coef[8 * (size_t)s + 3] > 0))
                return set_error("surface %u: sphere r^2 must be > 0", s), GT_EGEOM;
        }
        for (uint32_t m = 0; m < F.n_materials; m++)
            if (!(F.sigma_t[m] > 0) || !std::isfinite(F.sigma_t[m]))
                return set_error("material %u: sigma_t must be finite and > 0", m), GT_EGEOM;
        for (int k = 0; k < 3; k++)
            if (!(F.domain_lo[k] < F.domain_hi[k]) || !std::isfinite(F.domain_lo[k]) || !std::isfinite(F.domain_hi[k]))
                return set_error("domain box empty or infinite on axis %d", k), GT_EGEOM;
        if (F.univ_cell_off[0] != 0 || F.univ_cell_off[F.n_universes] != F.n_cells)
            return set_error("univ_cell_off must start at 0 and end at n_cells"), GT_EGEOM;
        if (F.cell_hs_off[0] != 0 || F.cell_hs_off[F.n_cells] != F.n_halfspaces)
            return set_error("cell_hs_off must start at 0 and end at n_halfspaces"), GT_EGEOM;
        cell_univ.assign(F.n_cells, 0);
        for (uint32_t u = 0; u < F.n_universes; u++) {
            if (F.univ_cell_off[u + 1] <= F.univ_cell_off[u]) return set_error("universe %u has no cells", u), GT_EGEOM;
            for (uint32_t c = F.univ_cell_off[u]; c < F.univ_cell_off[u + 1]; c++) cell_univ[c] = u;
        }
        std::vector<int64_t> owner(F.n_surfaces, -1);
        for (uint32_t c = 0; c < F.n_cells; c++) {
            if (F.cell_hs_off[c + 1] < F.cell_hs_off[c]) return set_error("cell %u: decreasing cell_hs_off", c), GT_EGEOM;
            if (F.cell_hs_off[c + 1] - F.cell_hs_off[c] > 0xFFFFu) return set_error("cell %u: too many half-spaces", c), GT_ECAPACITY;
            for (uint32_t k = F.cell_hs_off[c]; k < F.cell_hs_off[c + 1]; k++) {
                int32_t h = F.hs[k];
                if (h == 0 || (uint32_t)(h < 0 ? -(int64_t)h : h) > F.n_surfaces)
                    return set_error("cell %u: half-space %d names no surface", c, h), GT_EGEOM;
                uint32_t s = surf_of(h);
                for (uint32_t k2 = F.cell_hs_off[c]; k2 < k; k2++)
                    if (surf_of(F.hs[k2]) == s) return set_error("cell %u: surface %u appears twice", c, s), GT_EGEOM;
                if (owner[s] >= 0 && owner[s] != (int64_t)cell_univ[c])
                    return set_error("surface %u is used by universes %lld and %u", s, (long long)owner[s], cell_univ[c]), GT_EGEOM;
                owner[s] = cell_univ[c];
            }
            int32_t fl = F.cell_fill[c];
            if (fl >= 0 && (uint32_t)fl >= F.n_materials) return set_error("cell %u: material %d out of range", c, fl), GT_EGEOM;
            if (fl < 0 && (uint64_t)(-(int64_t)fl - 1) >= F.n_universes)
                return set_error("cell %u: daughter universe %lld out of range", c, (long long)(-(int64_t)fl - 1)), GT_EGEOM;
            for (int k = 0; k < 3; k++)
                if (!std::isfinite(F.cell_trans[3 * (size_t)c + k])) return set_error("cell %u: non-finite translation", c), GT_EGEOM;
        }
        // instances, depth and a parents-first order of the universes reachable from the root
        ninst.assign(F.n_universes, 0);
        inst_off.assign(F.n_cells, 0);
        depth.assign(F.n_universes, 0);
        std::vector<uint8_t> state(F.n_universes, 0);
        std::vector<uint32_t> post;
        int rc = visit(F.root, state, post);
        if (rc) return rc;
        topo.assign(post.rbegin(), post.rend());
        if (depth[F.root] > GT_MAX_LEVELS)
            return set_error("nesting depth %u exceeds %d", depth[F.root], GT_MAX_LEVELS), GT_ECAPACITY;
        if (ninst[F.root] > GT_MAX_INSTANCES)
            return set_error("%llu leaf instances exceed the limit", (unsigned long long)ninst[F.root]), GT_ECAPACITY;
        if (F.lattice_hint) {
            for (uint32_t u = 0; u < F.n_universes; u++) {
                const double *h = F.lattice_hint + 8 * (size_t)u;
                if (h[0] == 0) continue;
                if (h[0] != 1) return set_error("universe %u: unknown lattice hint kind %g", u, h[0]), GT_EGEOM;
                uint32_t nc = F.univ_cell_off[u + 1] - F.univ_cell_off[u];
                if (!(h[1] >= 1 && h[2] >= 1 && h[1] * h[2] == (double)nc && h[5] > 0 && h[6] > 0 &&
                      std::isfinite(h[3]) && std::isfinite(h[4]) && std::isfinite(h[5]) && std::isfinite(h[6])))
                    return set_error("universe %u: lattice hint does not match its %u cells", u, nc), GT_EGEOM;
            }
        }
        return GT_OK;
    }

    int visit(uint32_t u, std::vector<uint8_t> &state, std::vector<uint32_t> &post) {
        if (state[u] == 2) return GT_OK;
        if (state[u] == 1) return set_error("fill graph has a cycle through universe %u", u), GT_EGEOM;
        state[u] = 1;
        uint64_t n = 0;
        uint32_t d = 1;
        for (uint32_t c = f->univ_cell_off[u]; c < f->univ_cell_off[u + 1]; c++) {
            inst_off[c] = n;
            int32_t fl = f->cell_fill[c];
            if (fl >= 0) { n += 1; continue; }
            uint32_t du = (uint32_t)(-(int64_t)fl - 1);
            int rc = visit(du, state, post);
            if (rc) return rc;
            n += ninst[du];
            d = std::max(d, depth[du] + 1);
            if (n > (uint64_t)GT_MAX_INSTANCES) return set_error("too many leaf instances"), GT_ECAPACITY;
        }
        ninst[u] = n;
        depth[u] = d;
        state[u] = 2;
        post.push_back(u);
        return GT_OK;
    }

    Box clip_cell(uint32_t c, const Box &start) const {
        Box b = start;
        std::vector<HalfPlane> planes;
        for (uint32_t k = f->cell_hs_off[c]; k < f->cell_hs_off[c + 1]; k++) {
            int32_t h = f->hs[k];
            uint32_t s = surf_of(h);
            bool pos = h > 0;
            const double *q = f->surf_coef + 8 * (size_t)s;
            switch (f->surf_type[s]) {
            case ST_PX: case ST_PY: case ST_PZ: {
                int ax = f->surf_type[s];
                if (pos) b.lo[ax] = std::max(b.lo[ax], q[0]);
                else b.hi[ax] = std::min(b.hi[ax], q[0]);
                break;
            }
            case ST_CZ:
                if (!pos) {
                    double r = std::sqrt(q[2]);
                    b.lo[0] = std::max(b.lo[0], q[0] - r); b.hi[0] = std::min(b.hi[0], q[0] + r);
                    b.lo[1] = std::max(b.lo[1], q[1] - r); b.hi[1] = std::min(b.hi[1], q[1] + r);
                }
                break;
            case ST_SPH:
                if (!pos) {
                    double r = std::sqrt(q[3]);
                    for (int k2 = 0; k2 < 3; k2++) {
                        b.lo[k2] = std::max(b.lo[k2], q[k2] - r);
                        b.hi[k2] = std::min(b.hi[k2], q[k2] + r);
                    }
                }
                break;
            case ST_P:
                if (q[2] == 0.0 && (q[0] != 0.0 || q[1] != 0.0)) planes.push_back({q[0], q[1], q[3], pos});
                break;   // planes that are not vertical only make the box conservative
            }
        }
        if (b.is_empty()) return Box::empty();
        if (!planes.empty()) {
            std::vector<double> px = {b.lo[0], b.hi[0], b.hi[0], b.lo[0]};
            std::vector<double> py = {b.lo[1], b.lo[1], b.hi[1], b.hi[1]};
            for (const HalfPlane &h : planes) {
                clip_polygon(px, py, h);
                if (px.empty()) return Box::empty();
            }
            double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
            for (size_t i = 0; i < px.size(); i++) {
                x0 = std::min(x0, px[i]); x1 = std::max(x1, px[i]);
                y0 = std::min(y0, py[i]); y1 = std::max(y1, py[i]);
            }
            b.lo[0] = std::max(b.lo[0], x0); b.hi[0] = std::min(b.hi[0], x1);
            b.lo[1] = std::max(b.lo[1], y0); b.hi[1] = std::min(b.hi[1], y1);
            if (b.is_empty()) return Box::empty();
        }
        b.widen(delta);
        return b;
    }

    int boxes() {
        const gt_flat_geometry &F = *f;
        double scale = 1.0;
        for (int k = 0; k < 3; k++) scale = std::max({scale, std::fabs(F.domain_lo[k]), std::fabs(F.domain_hi[k])});
        delta = std::ldexp(scale, -26);
        ext.assign(F.n_universes, Box::empty());
        cbox.assign(F.n_cells, Box::empty());
        reached.assign(F.n_universes, 0);
        // root: every root cell must lie inside the sampling box
        Box dom;
        for (int k = 0; k < 3; k++) { dom.lo[k] = F.domain_lo[k]; dom.hi[k] = F.domain_hi[k]; }
        Box big = dom;
        for (int k = 0; k < 3; k++) { double w = dom.hi[k] - dom.lo[k]; big.lo[k] -= w; big.hi[k] += w; }
        for (uint32_t c = F.univ_cell_off[F.root]; c < F.univ_cell_off[F.root + 1]; c++) {
            Box b = clip_cell(c, big);
            if (b.is_empty()) continue;
            for (int k = 0; k < 3; k++)
                if (b.lo[k] < dom.lo[k] - 2 * delta || b.hi[k] > dom.hi[k] + 2 * delta)
                    return set_error("root cell %u is not bounded inside the domain box (axis %d)", c, k), GT_EGEOM;
        }
        Box root_ext = dom;
        root_ext.widen(delta);
        ext[F.root] = root_ext;
        reached[F.root] = 1;
        for (uint32_t u : topo) {
            if (!reached[u]) continue;
            for (uint32_t c = F.univ_cell_off[u]; c < F.univ_cell_off[u + 1]; c++) {
                Box b = clip_cell(c, ext[u]);
                cbox[c] = b;
                if (b.is_empty() || F.cell_fill[c] >= 0) continue;
                uint32_t du = (uint32_t)(-(int64_t)F.cell_fill[c] - 1);
                Box local = b;
                for (int k = 0; k < 3; k++) {
                    local.lo[k] -= F.cell_trans[3 * (size_t)c + k];
                    local.hi[k] += -F.cell_trans[3 * (size_t)c + k];
                }
                local.widen(delta);
                ext[du].grow(local);
                reached[du] = 1;
            }
        }
        return GT_OK;
    }

    struct Item { uint32_t cell; Box b; double c[3]; };

    uint32_t build_node(std::vector<Item> &it, size_t b0, size_t b1) {
        uint32_t idx = (uint32_t)n64.size();
        n64.emplace_back();
        Box bb = Box::empty();
        for (size_t i = b0; i < b1; i++) bb.grow(it[i].b);
        size_t n = b1 - b0;
        uint32_t leafv = kLeafNone;
        if (n <= kLeafMax) {
            leafv = ((uint32_t)leaf.size() << 4) | (uint32_t)(n - 1);
            for (size_t i = b0; i < b1; i++) leaf.push_back(it[i].cell);
        } else {
            // surface-area heuristic, three equally spaced candidates per axis
            double best = INFINITY;
            int bax = -1;
            double bplane = 0;
            for (int ax = 0; ax < 3; ax++) {
                double cmin = INFINITY, cmax = -INFINITY;
                for (size_t i = b0; i < b1; i++) { cmin = std::min(cmin, it[i].c[ax]); cmax = std::max(cmax, it[i].c[ax]); }
                if (!(cmax > cmin)) continue;
                for (int k = 1; k <= 3; k++) {
                    double plane = cmin + (cmax - cmin) * (double)k / 4.0;
                    Box L = Box::empty(), R = Box::empty();
                    size_t nl = 0;
                    for (size_t i = b0; i < b1; i++) {
                        if (it[i].c[ax] < plane) { L.grow(it[i].b); nl++; }
                        else R.grow(it[i].b);
                    }
                    if (nl == 0 || nl == n) continue;
                    double cost = (double)nl * L.area() + (double)(n - nl) * R.area();
                    if (cost < best) { best = cost; bax = ax; bplane = plane; }
                }
            }
            size_t mid;
            if (bax >= 0) {
                auto m = std::stable_partition(it.begin() + b0, it.begin() + b1,
                                               [&](const Item &x) { return x.c[bax] < bplane; });
                mid = (size_t)(m - it.begin());
            } else {   // all centres coincide: split the list in two
                mid = b0 + n / 2;
            }
            build_node(it, b0, mid);
            build_node(it, mid, b1);
        }
        Node64 &nd = n64[idx];
        for (int k = 0; k < 3; k++) { nd.lo[k] = bb.lo[k]; nd.hi[k] = bb.hi[k]; }
        nd.leaf = leafv;
        nd.escape = (uint32_t)n64.size();
        nd.pad[0] = nd.pad[1] = 0;
        return idx;
    }

    // A square-hinted universe whose cells are exactly an nx x ny pseudo-array
    // (see UArr): fills the rect entry and returns true.
    bool detect_rect(uint32_t u) {
        const gt_flat_geometry &F = *f;
        if (!F.lattice_hint || F.lattice_hint[8 * (size_t)u] != 1) return false;
        const uint32_t nx = (uint32_t)F.lattice_hint[8 * (size_t)u + 1], ny = (uint32_t)F.lattice_hint[8 * (size_t)u + 2];
        const uint32_t c0 = F.univ_cell_off[u];
        if (nx < 1 || ny < 1 || nx > 4096 || ny > 4096 || (uint64_t)nx * ny != F.univ_cell_off[u + 1] - c0) return false;
        const int64_t kAbsent = -1;
        std::vector<int64_t> lox(nx, -2), upx(nx, -2), loy(ny, -2), upy(ny, -2);
        std::vector<int32_t> extra_ref;
        for (uint32_t j = 0; j < ny; j++)
            for (uint32_t i = 0; i < nx; i++) {
                const uint32_t c = c0 + j * nx + i;
                int64_t lx = kAbsent, ux = kAbsent, ly = kAbsent, uy = kAbsent;
                std::vector<int32_t> extra;
                for (uint32_t k = F.cell_hs_off[c]; k < F.cell_hs_off[c + 1]; k++) {
                    const int32_t h = F.hs[k];
                    const uint32_t sf = surf_of(h);
                    const uint32_t t = F.surf_type[sf];
                    int64_t *slot = nullptr;
                    if (t == ST_PX) slot = h > 0 ? &lx : &ux;
                    else if (t == ST_PY) slot = h > 0 ? &ly : &uy;
                    if (!slot) { extra.push_back(h); continue; }
                    if (*slot != kAbsent) return false;   // two planes bound one side
                    *slot = sf;
                }
                std::sort(extra.begin(), extra.end());
                if (c == c0) extra_ref = extra;
                else if (extra != extra_ref) return false;
                if ((j > 0 && (lox[i] != lx || upx[i] != ux)) || (i > 0 && (loy[j] != ly || upy[j] != uy))) return false;
                lox[i] = lx; upx[i] = ux; loy[j] = ly; upy[j] = uy;
            }
        auto grid = [&](const std::vector<int64_t> &lo, const std::vector<int64_t> &up, uint32_t n,
                        std::vector<double> &v, std::vector<uint32_t> &sid) {
            for (uint32_t i = 0; i + 1 < n; i++)
                if (up[i] == kAbsent || up[i] != lo[i + 1]) return false;
            v.assign(n + 1, 0.0);
            sid.assign(n + 1, kLeafNone);
            for (uint32_t k = 0; k <= n; k++) {
                const int64_t sf = k < n ? lo[k] : up[n - 1];
                if (sf == kAbsent) {
                    if (k != 0 && k != n) return false;
                    v[k] = k == 0 ? -INFINITY : INFINITY;
                } else {
                    v[k] = F.surf_coef[8 * (size_t)sf];
                    sid[k] = (uint32_t)sf;
                }
            }
            for (uint32_t k = 0; k < n; k++)
                if (!(v[k] < v[k + 1])) return false;
            return true;
        };
        std::vector<double> vx, vy;
        std::vector<uint32_t> sx, sy;
        if (!grid(lox, upx, nx, vx, sx) || !grid(loy, upy, ny, vy, sy)) return false;
        UArr &A = uarr[u];
        A.kind = kKindRect;
        A.x0 = (float)F.lattice_hint[8 * (size_t)u + 3];
        A.y0 = (float)F.lattice_hint[8 * (size_t)u + 4];
        A.inv_px = (float)(1.0 / F.lattice_hint[8 * (size_t)u + 5]);
        A.inv_py = (float)(1.0 / F.lattice_hint[8 * (size_t)u + 6]);
        A.arr = (uint32_t)aval.size();
        A.n0 = nx;
        A.n1 = ny;
        aval.insert(aval.end(), vx.begin(), vx.end());
        aval.insert(aval.end(), vy.begin(), vy.end());
        asurf.insert(asurf.end(), sx.begin(), sx.end());
        asurf.insert(asurf.end(), sy.begin(), sy.end());
        A.xhs = (uint32_t)ahs.size();
        A.nxhs = (uint32_t)extra_ref.size();
        for (int32_t h : extra_ref) {
            const uint32_t sf = surf_of(h);
            ahs.push_back(hs_pack(sf, h > 0, F.surf_type[sf]));
        }
        for (uint32_t j = 0; j < ny; j++)
            for (uint32_t i = 0; i < nx; i++) cell_ij[c0 + j * nx + i] = i | j << 16;
        return true;
    }

    // A universe of concentric z-cylinders (one centre) and z planes whose
    // cells are exactly the (slab, ring) regions in the order of UArr.
    bool detect_pin(uint32_t u) {
        const gt_flat_geometry &F = *f;
        const uint32_t c0 = F.univ_cell_off[u], nc = F.univ_cell_off[u + 1] - c0;
        std::vector<uint32_t> cyl, zp;
        for (uint32_t c = c0; c < c0 + nc; c++)
            for (uint32_t k = F.cell_hs_off[c]; k < F.cell_hs_off[c + 1]; k++) {
                const uint32_t sf = surf_of(F.hs[k]);
                const uint32_t t = F.surf_type[sf];
                if (t == ST_CZ) cyl.push_back(sf);
                else if (t == ST_PZ) zp.push_back(sf);
                else return false;
            }
        std::sort(cyl.begin(), cyl.end());
        cyl.erase(std::unique(cyl.begin(), cyl.end()), cyl.end());
        std::sort(zp.begin(), zp.end());
        zp.erase(std::unique(zp.begin(), zp.end()), zp.end());
        if (cyl.empty() || cyl.size() > 64 || zp.size() > 4096) return false;
        const double *q0 = F.surf_coef + 8 * (size_t)cyl[0];
        for (uint32_t sf : cyl)
            if (std::memcmp(F.surf_coef + 8 * (size_t)sf, q0, 2 * sizeof(double)) != 0) return false;
        auto coef = [&](uint32_t sf, int k) { return F.surf_coef[8 * (size_t)sf + k]; };
        std::sort(cyl.begin(), cyl.end(), [&](uint32_t a, uint32_t b) { return coef(a, 2) < coef(b, 2); });
        std::sort(zp.begin(), zp.end(), [&](uint32_t a, uint32_t b) { return coef(a, 0) < coef(b, 0); });
        for (size_t k = 0; k + 1 < cyl.size(); k++)
            if (!(coef(cyl[k], 2) < coef(cyl[k + 1], 2))) return false;
        for (size_t k = 0; k + 1 < zp.size(); k++)
            if (!(coef(zp[k], 0) < coef(zp[k + 1], 0))) return false;
        const uint32_t nr = (uint32_t)cyl.size() + 1, ns = (uint32_t)zp.size() + 1;
        if ((uint64_t)nr * ns != nc) return false;
        for (uint32_t k = 0; k < ns; k++)
            for (uint32_t r = 0; r < nr; r++) {
                const uint32_t c = c0 + k * nr + r;
                std::vector<int32_t> want, have(F.hs + F.cell_hs_off[c], F.hs + F.cell_hs_off[c + 1]);
                if (r > 0) want.push_back((int32_t)cyl[r - 1] + 1);
                if (r + 1 < nr) want.push_back(-((int32_t)cyl[r] + 1));
                if (k > 0) want.push_back((int32_t)zp[k - 1] + 1);
                if (k + 1 < ns) want.push_back(-((int32_t)zp[k] + 1));
                std::sort(want.begin(), want.end());
                std::sort(have.begin(), have.end());
                if (want != have) return false;
            }
        UArr &A = uarr[u];
        A.kind = kKindPin;
        A.arr = (uint32_t)aval.size();
        A.n0 = (uint32_t)cyl.size();
        A.n1 = (uint32_t)zp.size();
        for (uint32_t sf : cyl) { aval.push_back(coef(sf, 2)); asurf.push_back(sf); }
        aval.push_back(q0[0]);
        aval.push_back(q0[1]);
        asurf.push_back(kLeafNone);
        asurf.push_back(kLeafNone);
        for (uint32_t sf : zp) { aval.push_back(coef(sf, 0)); asurf.push_back(sf); }
        for (uint32_t k = 0; k < ns; k++)
            for (uint32_t r = 0; r < nr; r++) cell_ij[c0 + k * nr + r] = r | k << 16;
        return true;
    }

    // The fixed-depth reactor shape (Section "RTK tracking"): an optional root
    // of one cell filled with a rect universe, then one or two levels of rect
    // universes every cell of which is filled, then pin universes of
    // material cells.  Returns 1 | root_csg << 1 | (rect levels - 1) << 2,
    // or 0 when the geometry is not of that shape.
    uint32_t detect_rtk_shape() const {
        const gt_flat_geometry &F = *f;
        std::vector<uint32_t> level = {F.root};
        uint32_t root_csg = 0, nrect = 0;
        auto daughters = [&](const std::vector<uint32_t> &us, std::vector<uint32_t> &out) {
            out.clear();
            for (uint32_t u : us)
                for (uint32_t c = F.univ_cell_off[u]; c < F.univ_cell_off[u + 1]; c++) {
                    if (F.cell_fill[c] >= 0) return false;
                    out.push_back((uint32_t)(-(int64_t)F.cell_fill[c] - 1));
                }
            std::sort(out.begin(), out.end());
            out.erase(std::unique(out.begin(), out.end()), out.end());
            return true;
        };
        std::vector<uint32_t> next;
        if (uarr[F.root].kind == kKindCsg) {
            if (F.univ_cell_off[F.root + 1] - F.univ_cell_off[F.root] != 1) return 0;
            if (!daughters(level, next)) return 0;
            level = next;
            root_csg = 1;
        }
        for (;;) {
            for (uint32_t u : level)
                if (uarr[u].kind != kKindRect) goto leaf;
            if (++nrect > 2) return 0;
            if (!daughters(level, next)) return 0;
            level = next;
        }
    leaf:
        if (nrect == 0) return 0;
        for (uint32_t u : level) {
            if (uarr[u].kind != kKindPin) return 0;
            for (uint32_t c = F.univ_cell_off[u]; c < F.univ_cell_off[u + 1]; c++)
                if (F.cell_fill[c] < 0) return 0;
        }
        return 1u | root_csg << 1 | (nrect - 1) << 2;
    }

    void kinds() {
        const gt_flat_geometry &F = *f;
        uarr.assign(F.n_universes, UArr{});
        cell_ij.assign(F.n_cells, 0);
        for (uint32_t u = 0; u < F.n_universes; u++) {
            uarr[u].kind = kKindCsg;
            uarr[u].cell0 = F.univ_cell_off[u];
            if (!detect_rect(u)) detect_pin(u);
        }
        rtk_shape = detect_rtk_shape();
    }

    int hierarchies() {
        const gt_flat_geometry &F = *f;
        univ.assign(F.n_universes, Univ{});
        for (uint32_t u = 0; u < F.n_universes; u++) {
            Univ &U = univ[u];
            U.cell0 = F.univ_cell_off[u];
            U.ncell = F.univ_cell_off[u + 1] - F.univ_cell_off[u];
            U.node0 = (uint32_t)n64.size();
            U.nnode = 0;
            U.hint = kHintNone;
            if (F.lattice_hint && F.lattice_hint[8 * (size_t)u] == 1) {
                const double *h = F.lattice_hint + 8 * (size_t)u;
                U.hint = kHintSquare;
                U.nx = (int32_t)h[1];
                U.ny = (int32_t)h[2];
                U.x0 = (float)h[3];
                U.y0 = (float)h[4];
                U.inv_px = (float)(1.0 / h[5]);
                U.inv_py = (float)(1.0 / h[6]);
            }
            if (!reached[u]) continue;
            std::vector<Item> items;
            for (uint32_t c = U.cell0; c < U.cell0 + U.ncell; c++) {
                if (cbox[c].is_empty()) continue;
                Item x;
                x.cell = c;
                x.b = cbox[c];
                for (int k = 0; k < 3; k++) x.c[k] = 0.5 * (x.b.lo[k] + x.b.hi[k]);
                items.push_back(x);
            }
            if (items.empty()) continue;
            build_node(items, 0, items.size());
            U.nnode = (uint32_t)n64.size() - U.node0;
        }
        if (leaf.size() >= (1u << 28)) return set_error("too many leaf entries"), GT_ECAPACITY;
        n32.resize(n64.size());
        for (size_t i = 0; i < n64.size(); i++) {
            for (int k = 0; k < 3; k++) { n32[i].lo[k] = round_down(n64[i].lo[k]); n32[i].hi[k] = round_up(n64[i].hi[k]); }
            n32[i].escape = n64[i].escape;
            n32[i].leaf = n64[i].leaf;
        }
        return GT_OK;
    }
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace gt

using namespace gt;

extern "C" const char *gt_last_error(void) { return g_err; }

extern "C" int gt_geometry_create(const gt_flat_geometry *f, gt_geometry **out) {
    if (!f || !out) return set_error("gt_geometry_create: null argument"), GT_EINVAL;
    *out = nullptr;
    try {
        Builder B;
        B.f = f;
        int rc = B.validate();
        if (rc) return rc;
        rc = B.boxes();
        if (rc) return rc;
        rc = B.hierarchies();
        if (rc) return rc;
        B.kinds();
        const gt_flat_geometry &F = *f;
        // host images of every table
        std::vector<double> coef(4 * (size_t)F.n_surfaces, 0.0);
        for (uint32_t s = 0; s < F.n_surfaces; s++) {
            const double *q = F.surf_coef + 8 * (size_t)s;
            double *o = &coef[4 * (size_t)s];
            switch (F.surf_type[s]) {
            case ST_PX: case ST_PY: case ST_PZ: o[0] = q[0]; break;
            case ST_P: o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[3]; break;
            case ST_CZ: o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; break;
            default: o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[3]; break;
            }
        }
        // each cell's half-spaces: slab pairs, the other planes, then quadrics
        // (the order never changes a result: containment is a conjunction and
        // distance ties break on surface id)
        std::vector<uint32_t> hs(F.n_halfspaces);
        std::vector<Cell> cell(F.n_cells);
        auto same_family = [&](uint32_t a, uint32_t b) {
            if (F.surf_type[a] != F.surf_type[b]) return false;
            if (F.surf_type[a] != ST_P) return true;   // one axis
            return std::memcmp(F.surf_coef + 8 * (size_t)a, F.surf_coef + 8 * (size_t)b, 3 * sizeof(double)) == 0;
        };
        for (uint32_t c = 0; c < F.n_cells; c++) {
            const uint32_t k0 = F.cell_hs_off[c], k1 = F.cell_hs_off[c + 1];
            std::vector<uint32_t> planes, quads;
            for (uint32_t k = k0; k < k1; k++)
                (F.surf_type[B.surf_of(F.hs[k])] >= ST_CZ ? quads : planes).push_back(k);
            if (planes.size() > kPlaneCountMask) return set_error("cell %u: too many plane half-spaces", c), GT_ECAPACITY;
            // a family with exactly one negative and one positive half-space forms a pair
            std::vector<uint32_t> order, rest;
            std::vector<bool> used(planes.size(), false);
            uint32_t npair = 0;
            for (size_t i = 0; i < planes.size(); i++) {
                if (used[i]) continue;
                std::vector<size_t> fam = {i};
                for (size_t j = i + 1; j < planes.size(); j++)
                    if (!used[j] && same_family(B.surf_of(F.hs[planes[i]]), B.surf_of(F.hs[planes[j]]))) fam.push_back(j);
                for (size_t j : fam) used[j] = true;
                if (fam.size() == 2 && (F.hs[planes[fam[0]]] > 0) != (F.hs[planes[fam[1]]] > 0) && npair < kMaxPairs) {
                    const bool first_neg = F.hs[planes[fam[0]]] < 0;
                    order.push_back(planes[first_neg ? fam[0] : fam[1]]);
                    order.push_back(planes[first_neg ? fam[1] : fam[0]]);
                    npair++;
                } else {
                    for (size_t j : fam) rest.push_back(planes[j]);
                }
            }
            order.insert(order.end(), rest.begin(), rest.end());
            order.insert(order.end(), quads.begin(), quads.end());
            uint32_t o = k0;
            for (uint32_t k : order) {
                const uint32_t s = B.surf_of(F.hs[k]);
                hs[o++] = hs_pack(s, F.hs[k] > 0, F.surf_type[s]);
            }
            cell[c].n_pl = (uint16_t)(planes.size() | (size_t)npair << 12);
        }
        std::vector<double> trans(4 * (size_t)F.n_cells, 0.0);
        std::vector<float> cb(8 * (size_t)F.n_cells, 0.0f);
        for (uint32_t c = 0; c < F.n_cells; c++) {
            cell[c].hs_off = F.cell_hs_off[c];
            cell[c].n_hs = (uint16_t)(F.cell_hs_off[c + 1] - F.cell_hs_off[c]);
            cell[c].fill = F.cell_fill[c];
            cell[c].inst_off = (uint32_t)B.inst_off[c];
            for (int k = 0; k < 3; k++) trans[4 * (size_t)c + k] = F.cell_trans[3 * (size_t)c + k];
            const Box &b = B.cbox[c];
            for (int k = 0; k < 3; k++) {
                cb[8 * (size_t)c + k] = b.is_empty() ? INFINITY : round_down(b.lo[k]);
                cb[8 * (size_t)c + 4 + k] = b.is_empty() ? -INFINITY : round_up(b.hi[k]);
            }
        }
        // crossing candidates per half-space entry (device order): cells of the
        // same universe that use the surface with the other sense and whose
        // widened boxes overlap this cell's box; first those that share the
        // most of this cell's other half-spaces (the cell straight across a
        // face usually keeps the bounds along the face: the y planes across an
        // x plane, the cylinders across an axial plane), then the largest
        // box overlap
        std::vector<std::vector<std::pair<uint32_t, bool>>> users(F.n_surfaces);
        for (uint32_t c = 0; c < F.n_cells; c++)
            for (uint32_t k = F.cell_hs_off[c]; k < F.cell_hs_off[c + 1]; k++)
                users[B.surf_of(F.hs[k])].push_back({c, F.hs[k] > 0});
        std::vector<uint32_t> adj_off(F.n_halfspaces + 1, 0), adj;
        for (uint32_t c = 0; c < F.n_cells; c++) {
            const Box &bc = B.cbox[c];
            for (uint32_t k = F.cell_hs_off[c]; k < F.cell_hs_off[c + 1]; k++) {
                adj_off[k] = (uint32_t)adj.size();
                if (bc.is_empty()) continue;
                const uint32_t s = hs[k] >> 4;
                const bool pos = (hs[k] >> 3) & 1u;
                struct Cand {
                    int shared;
                    double v;
                    uint32_t cell;
                };
                std::vector<Cand> cand;
                for (const auto &us : users[s]) {
                    if (us.first == c || us.second == pos) continue;
                    const Box &bd = B.cbox[us.first];
                    if (bd.is_empty()) continue;
                    double v = 1.0;
                    for (int ax = 0; ax < 3; ax++) {
                        const double w = std::min(bc.hi[ax], bd.hi[ax]) - std::max(bc.lo[ax], bd.lo[ax]);
                        v = w < 0 ? -1.0 : v * w;
                        if (v < 0) break;
                    }
                    if (v < 0) continue;
                    int shared = 0;
                    for (uint32_t a = F.cell_hs_off[us.first]; a < F.cell_hs_off[us.first + 1]; a++)
                        for (uint32_t q = F.cell_hs_off[c]; q < F.cell_hs_off[c + 1]; q++)
                            if (q != k && F.hs[q] == F.hs[a]) shared++;
                    cand.push_back({shared, v, us.first});
                }
                std::stable_sort(cand.begin(), cand.end(), [](const Cand &x, const Cand &y) {
                    return x.shared != y.shared ? x.shared > y.shared : x.v > y.v;
                });
                for (size_t i = 0; i < cand.size() && i < 16; i++) adj.push_back(cand[i].cell);
            }
        }
        adj_off[F.n_halfspaces] = (uint32_t)adj.size();
        std::vector<uint32_t> cell_local(F.n_cells);
        for (uint32_t c = 0; c < F.n_cells; c++) cell_local[c] = c - F.univ_cell_off[B.cell_univ[c]];
        // one blob
        size_t off[SEC_COUNT], sz[SEC_COUNT];
        sz[SEC_COEF] = coef.size() * 8;
        sz[SEC_HS] = hs.size() * 4;
        sz[SEC_CELL] = cell.size() * sizeof(Cell);
        sz[SEC_TRANS] = trans.size() * 8;
        sz[SEC_UNIV] = B.univ.size() * sizeof(Univ);
        sz[SEC_NODE32] = B.n32.size() * sizeof(Node32);
        sz[SEC_NODE64] = B.n64.size() * sizeof(Node64);
        sz[SEC_LEAF] = B.leaf.size() * 4;
        sz[SEC_CBOX] = cb.size() * 4;
        sz[SEC_SIGMA] = (size_t)F.n_materials * 8;
        sz[SEC_ADJOFF] = adj_off.size() * 4;
        sz[SEC_ADJ] = adj.size() * 4;
        sz[SEC_LOCAL] = cell_local.size() * 4;
        sz[SEC_UARR] = B.uarr.size() * sizeof(UArr);
        sz[SEC_AVAL] = B.aval.size() * 8;
        sz[SEC_ASURF] = B.asurf.size() * 4;
        sz[SEC_AHS] = B.ahs.size() * 4;
        sz[SEC_IJ] = B.cell_ij.size() * 4;
        size_t total = 0;
        for (int i = 0; i < SEC_COUNT; i++) { off[i] = total; total = align_up(total + std::max(sz[i], (size_t)16)); }
        std::vector<unsigned char> img(total, 0);
        const void *src[SEC_COUNT] = {coef.data(), hs.data(), cell.data(), trans.data(), B.univ.data(),
                                      B.n32.data(), B.n64.data(), B.leaf.data(), cb.data(), F.sigma_t,
                                      adj_off.data(), adj.data(), cell_local.data(), B.uarr.data(),
                                      B.aval.data(), B.asurf.data(), B.ahs.data(), B.cell_ij.data()};
        for (int i = 0; i < SEC_COUNT; i++)
            if (sz[i]) std::memcpy(img.data() + off[i], src[i], sz[i]);
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return set_error("hipGetDevice failed"), GT_EHIP;
        const size_t desc_at = total;
        total = align_up(total + sizeof(GeomDesc));
        void *blob = nullptr;
        hipError_t e = hipMalloc(&blob, total);
        if (e != hipSuccess) return set_error("hipMalloc(%zu): %s", total, hipGetErrorString(e)), GT_ENOMEM;
        e = hipMemcpy(blob, img.data(), desc_at, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(blob);
            return set_error("hipMemcpy: %s", hipGetErrorString(e)), GT_EHIP;
        }
        void *ws = nullptr;
        const size_t ws_bytes = (size_t)track_ws_bytes(B.ninst[F.root]);
        e = hipMalloc(&ws, ws_bytes);
        if (e != hipSuccess) {
            (void)hipFree(blob);
            return set_error("hipMalloc(%zu) for the tally workspace: %s", ws_bytes, hipGetErrorString(e)), GT_ENOMEM;
        }
        gt_geometry *g = new gt_geometry;
        unsigned char *base = (unsigned char *)blob;
        g->dev.coef = (const double *)(base + off[SEC_COEF]);
        g->dev.hs = (const uint32_t *)(base + off[SEC_HS]);
        g->dev.cell = (const Cell *)(base + off[SEC_CELL]);
        g->dev.trans = (const double *)(base + off[SEC_TRANS]);
        g->dev.univ = (const Univ *)(base + off[SEC_UNIV]);
        g->dev.node32 = (const Node32 *)(base + off[SEC_NODE32]);
        g->dev.node64 = (const Node64 *)(base + off[SEC_NODE64]);
        g->dev.leaf = (const uint32_t *)(base + off[SEC_LEAF]);
        g->dev.cbox = (const float *)(base + off[SEC_CBOX]);
        g->dev.sigma = (const double *)(base + off[SEC_SIGMA]);
        g->dev.adj_off = (const uint32_t *)(base + off[SEC_ADJOFF]);
        g->dev.adj = (const uint32_t *)(base + off[SEC_ADJ]);
        g->dev.cell_local = (const uint32_t *)(base + off[SEC_LOCAL]);
        g->dev.uarr = (const UArr *)(base + off[SEC_UARR]);
        g->dev.aval = (const double *)(base + off[SEC_AVAL]);
        g->dev.asurf = (const uint32_t *)(base + off[SEC_ASURF]);
        g->dev.ahs = (const uint32_t *)(base + off[SEC_AHS]);
        g->dev.cell_ij = (const uint32_t *)(base + off[SEC_IJ]);
        g->dev.root = F.root;
        g->dev.n_inst = (uint32_t)B.ninst[F.root];
        g->dev.max_depth = B.depth[F.root];
        g->dev.n_cells = F.n_cells;
        // the smallest surface set of the tracker builds that holds every surface
        bool general = false, vertical = false;
        for (uint32_t s = 0; s < F.n_surfaces; s++) {
            if (F.surf_type[s] == ST_SPH) general = true;
            if (F.surf_type[s] == ST_P) (F.surf_coef[8 * (size_t)s + 2] == 0.0 ? vertical : general) = true;
        }
        g->surf_set = general ? SF_ALL : vertical ? SF_VERT : SF_AXCZ;
        for (int k = 0; k < 3; k++) { g->dev.lo[k] = F.domain_lo[k]; g->dev.hi[k] = F.domain_hi[k]; }
        // LDS staging plans per precision mode: the per-segment tables (cells,
        // half-spaces, surfaces, universes, materials, local indices) if they
        // fit, then the crossing tables (translations, candidate lists) if
        // those fit too, then as many hierarchy tables as fit; whatever is not
        // copied is read from global memory
        // (the plans for the trackers that switch on universe kind count the
        // universe-kind tables among the per-segment ones)
        static const int kTierA[] = {SEC_CELL, SEC_HS, SEC_COEF, SEC_UNIV, SEC_SIGMA, SEC_LOCAL,
                                     SEC_UARR, SEC_AVAL, SEC_ASURF, SEC_AHS, SEC_IJ};
        static const int kTierB[] = {SEC_TRANS, SEC_ADJOFF, SEC_ADJ};
        const uint64_t budget = stage_budget();
        for (int plan = 0; plan < 4; plan++) {
            const int prec = plan & 1;
            const bool arr = plan >= 2;
            StagePlan &P = arr ? g->stage_arr[prec] : g->stage[prec];
            std::memset(&P, 0, sizeof P);
            for (int i = 0; i < SEC_COUNT; i++) P.at[i] = 0xFFFFFFFFu;
            uint64_t at = 0;
            auto bytes = [&](int i) { return (std::max<size_t>(sz[i], 16) + 15) & ~(uint64_t)15; };
            auto add = [&](int i) {
                P.src[P.n] = (uint32_t)off[i];
                P.dst[P.n] = (uint32_t)at;
                P.bytes[P.n] = (uint32_t)bytes(i);
                P.at[i] = (uint32_t)at;
                P.n++;
                at += bytes(i);
            };
            const int n_tier_a = arr ? 11 : 6;
            uint64_t need_a = 0, need_b = 0;
            for (int k = 0; k < n_tier_a; k++) need_a += bytes(kTierA[k]);
            for (int i : kTierB) need_b += bytes(i);
            if (need_a <= budget) {
                for (int k = 0; k < n_tier_a; k++) add(kTierA[k]);
                P.kind = 1;
                if (need_a + need_b <= budget) {
                    for (int i : kTierB) add(i);
                    P.kind = 2;
                    const int cold[] = {prec == GT_PREC_MIXED ? SEC_NODE32 : SEC_NODE64, SEC_LEAF,
                                        prec == GT_PREC_MIXED ? SEC_CBOX : -1};
                    uint64_t need_c = 0;
                    for (int i : cold)
                        if (i >= 0) need_c += bytes(i);
                    if (need_a + need_b + need_c <= budget) {
                        for (int i : cold)
                            if (i >= 0) add(i);
                        P.kind = 3;
                    }
                }
            }
            P.total = (uint32_t)at;
        }
        GeomDesc desc;
        desc.dev = g->dev;
        desc.stage[0] = g->stage[0];
        desc.stage[1] = g->stage[1];
        desc.stage_arr[0] = g->stage_arr[0];
        desc.stage_arr[1] = g->stage_arr[1];
        e = hipMemcpy(base + desc_at, &desc, sizeof desc, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(blob);
            (void)hipFree(ws);
            delete g;
            return set_error("hipMemcpy: %s", hipGetErrorString(e)), GT_EHIP;
        }
        g->desc = (const GeomDesc *)(base + desc_at);
        g->blob = blob;
        g->blob_bytes = total + ws_bytes;
        g->ws = ws;
        g->launch = (LaunchRec *)ws;
        g->tally_ws = (uint64_t *)((unsigned char *)ws + kWsTallyAt);
        g->n_inst = B.ninst[F.root];
        g->max_depth = B.depth[F.root];
        g->device = dev;
        g->rtk_shape = B.rtk_shape;
        g->n_rect = g->n_pin = 0;
        for (const UArr &A : B.uarr) {
            g->n_rect += A.kind == kKindRect;
            g->n_pin += A.kind == kKindPin;
        }
        *out = g;
        return GT_OK;
    } catch (const std::bad_alloc &) {
        return set_error("host allocation failed"), GT_ENOMEM;
    } catch (...) {
        return set_error("unexpected exception in gt_geometry_create"), GT_EINVAL;
    }
}

extern "C" int gt_geometry_info(const gt_geometry *g, uint64_t *n_instances, uint32_t *max_depth,
                                uint64_t *device_bytes) {
    if (!g) return set_error("gt_geometry_info: null geometry"), GT_EINVAL;
    if (n_instances) *n_instances = g->n_inst;
    if (max_depth) *max_depth = g->max_depth;
    if (device_bytes) *device_bytes = g->blob_bytes;
    return GT_OK;
}

extern "C" int gt_geometry_staging(const gt_geometry *g, uint32_t precision, uint32_t *kind, uint32_t *lds_bytes) {
    if (!g) return set_error("gt_geometry_staging: null geometry"), GT_EINVAL;
    if (precision > GT_PREC_MIXED) return set_error("gt_geometry_staging: unknown precision %u", precision), GT_EINVAL;
    if (kind) *kind = g->stage[precision].kind;
    if (lds_bytes) *lds_bytes = g->stage[precision].total;
    return GT_OK;
}

extern "C" int gt_geometry_kinds(const gt_geometry *g, uint32_t *n_rect, uint32_t *n_pin, uint32_t *rtk_shape) {
    if (!g) return set_error("gt_geometry_kinds: null geometry"), GT_EINVAL;
    if (n_rect) *n_rect = g->n_rect;
    if (n_pin) *n_pin = g->n_pin;
    if (rtk_shape) *rtk_shape = g->rtk_shape;
    return GT_OK;
}

extern "C" void gt_geometry_destroy(gt_geometry *g) {
    if (!g) return;
    int cur = 0;
    bool switched = hipGetDevice(&cur) == hipSuccess && cur != g->device && hipSetDevice(g->device) == hipSuccess;
    (void)hipFree(g->blob);
    (void)hipFree(g->ws);
    if (switched) (void)hipSetDevice(cur);
    delete g;
}

void gt::fill_kparams(const gt_track_params *p, const gt_geometry *g, KParams &kp, KOut &ko, const gt_track_out *o) {
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
    kp.wave_take = p->wave_histories ? p->wave_histories : kWaveTake;
    kp.pad = 0;
    ko.mesh = MeshDesc{};
    LaunchRec *lr;
    workspace_of(g, o, &lr, &ko.tally_ws);
    ko.seg_count = o->seg_count;
    ko.seq_hash = o->seq_hash;
    ko.end_code = o->end_code;
    ko.rec = o->rec;
    ko.counters = o->counters;
}

void gt::workspace_of(const gt_geometry *g, const gt_track_out *o, LaunchRec **launch, uint64_t **tally) {
    if (o && o->workspace) {
        *launch = (LaunchRec *)o->workspace;
        *tally = (uint64_t *)((unsigned char *)o->workspace + kWsTallyAt);
    } else {
        *launch = g->launch;
        *tally = g->tally_ws;
    }
}

unsigned gt::stage_budget() { return kStageBudget; }

extern "C" uint64_t gt_track_workspace_bytes(const gt_geometry *g) {
    return g ? track_ws_bytes(g->n_inst) : 0;
}

int gt::check_track_args(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o) {
    if (!g || !p || !o) return set_error("gt_track: null argument"), GT_EINVAL;
    if (!o->tally_fx || !o->counters) return set_error("gt_track: tally_fx and counters are required"), GT_EINVAL;
    if (o->workspace && (o->workspace_bytes < track_ws_bytes(g->n_inst) || ((uintptr_t)o->workspace & 255u)))
        return set_error("gt_track: the workspace needs %llu bytes, 256-byte aligned",
                         (unsigned long long)track_ws_bytes(g->n_inst)), GT_EINVAL;
    if (p->max_collisions < 1) return set_error("gt_track: max_collisions must be >= 1"), GT_EINVAL;
    if (p->max_segments < 1) return set_error("gt_track: max_segments must be >= 1"), GT_EINVAL;
    if (p->precision > GT_PREC_MIXED) return set_error("gt_track: unknown precision %u", p->precision), GT_EINVAL;
    if (p->source > 1) return set_error("gt_track: unknown source %u", p->source), GT_EINVAL;
    if (p->source == 1 && p->ray_n1 < 1) return set_error("gt_track: ray source needs ray_n1 >= 1"), GT_EINVAL;
    if (p->record_first_k && (!o->rec || p->record_cap < 1))
        return set_error("gt_track: recording needs rec and record_cap >= 1"), GT_EINVAL;
    if (p->flags & ~(GT_FLAG_ACCUMULATE | GT_FLAG_LANE_PER_HISTORY | GT_FLAG_NO_STAGING | GT_FLAG_TAIL_COMPACTION |
                     GT_FLAG_NO_TALLY_CACHE | GT_FLAG_TRACKER_SP | GT_FLAG_TRACKER_RTK))
        return set_error("gt_track: unknown flags 0x%x", p->flags), GT_EINVAL;
    if (p->flags & (GT_FLAG_TRACKER_SP | GT_FLAG_TRACKER_RTK)) {
        if ((p->flags & GT_FLAG_TRACKER_SP) && (p->flags & GT_FLAG_TRACKER_RTK))
            return set_error("gt_track: GT_FLAG_TRACKER_SP and GT_FLAG_TRACKER_RTK exclude each other"), GT_EINVAL;
        if (p->flags & GT_FLAG_LANE_PER_HISTORY)
            return set_error("gt_track: the SP and RTK trackers run on the persistent schedule only"), GT_EINVAL;
        if (p->regroup_every)
            return set_error("gt_track: regroup_every is not available with the SP and RTK trackers"), GT_EINVAL;
        if ((p->flags & GT_FLAG_TRACKER_RTK) && !g->rtk_shape)
            return set_error("gt_track: the geometry is not of the fixed-depth reactor shape (GT_FLAG_TRACKER_RTK)"),
                   GT_EINVAL;
    }
    if (p->block_size && (p->block_size % 64 || p->block_size > 1024))
        return set_error("gt_track: block_size must be a multiple of 64 up to 1024"), GT_EINVAL;
    if (p->refill_min > 64) return set_error("gt_track: refill_min must be at most 64"), GT_EINVAL;
    if (p->wave_histories % 64 || p->wave_histories > 1024)
        return set_error("gt_track: wave_histories must be a multiple of 64 up to 1024"), GT_EINVAL;
    if (p->wave_histories && (p->flags & GT_FLAG_LANE_PER_HISTORY))
        return set_error("gt_track: wave_histories needs the persistent schedule"), GT_EINVAL;
    if (p->regroup_every && (p->flags & GT_FLAG_LANE_PER_HISTORY))
        return set_error("gt_track: regroup_every needs the persistent schedule"), GT_EINVAL;
    if (p->first_particle + p->n_particles < p->first_particle)
        return set_error("gt_track: particle id range overflows"), GT_EINVAL;
    if ((uint64_t)p->record_first_k * p->record_cap > (1ull << 40))
        return set_error("gt_track: record buffer too large"), GT_ECAPACITY;
    return GT_OK;
}

extern "C" int gt_track(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *stream) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    return launch_track(g, p, o, stream);
}

namespace gt {
// The event bank's arrays, each 256-byte aligned from `base` (which may be
// null to size it); returns the bytes used.
uint64_t ev_layout(uint64_t n, unsigned char *base, EvBank *b) {
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        unsigned char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(uint64_t)255;
        return p;
    };
    EvBank e;
    double **d[] = {&e.x, &e.y, &e.z, &e.u, &e.v, &e.w, &e.tau, &e.t, &e.sig};
    for (double **q : d) *q = (double *)take(8 * n);
    uint64_t **w[] = {&e.h, &e.acc_lo, &e.acc_hi};
    for (uint64_t **q : w) *q = (uint64_t *)take(8 * n);
    e.cell = (uint32_t *)take(4 * n * GT_MAX_LEVELS);
    uint32_t **u[] = {&e.on_surf, &e.blk, &e.segs, &e.ncoll, &e.acc_inst, &e.surf, &e.inst, &e.entry, &e.st};
    for (uint32_t **q : u) *q = (uint32_t *)take(4 * n);
    e.alive = (unsigned long long *)take(16);
    if (b) *b = e;
    return off;
}
}  // namespace gt

extern "C" uint64_t gt_event_bank_bytes(uint64_t n_particles) {
    if (n_particles > (uint64_t)0x7FFFFFFF * 64ull) return 0;
    return ev_layout(n_particles, nullptr, nullptr);
}

extern "C" uint64_t gt_mesh_workspace_bytes(uint64_t bins) {
    if (bins == 0 || bins > (1ull << 31)) return 0;
    return (uint64_t)tally_replicas(bins) * 4 * 8 * bins;   // replicas x limbs x bytes, as the cell tally's workspace
}

extern "C" int gt_track_mesh(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o,
                             const gt_mesh *m, void *stream) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    if (!m) return set_error("gt_track_mesh: mesh is NULL"), GT_EINVAL;
    if (p->flags & GT_FLAG_LANE_PER_HISTORY)
        return set_error("gt_track_mesh: the mesh tally needs the persistent schedule"), GT_EINVAL;
    if (p->regroup_every) return set_error("gt_track_mesh: regroup_every must be 0"), GT_EINVAL;
    if (p->flags & (GT_FLAG_TRACKER_SP | GT_FLAG_TRACKER_RTK))
        return set_error("gt_track_mesh: the mesh tally runs with the single tracker only"), GT_EINVAL;
    if (m->reserved) return set_error("gt_track_mesh: reserved must be 0"), GT_EINVAL;
    uint64_t bins = 1;
    for (int a = 0; a < 3; a++) {
        if (m->n[a] < 1) return set_error("gt_track_mesh: n[%d] must be >= 1", a), GT_EINVAL;
        if (m->n[a] > (1u << 24)) return set_error("gt_track_mesh: n[%d] above 2^24", a), GT_ECAPACITY;
        if (!std::isfinite(m->lo[a]) || !std::isfinite(m->hi[a]) || !(m->hi[a] > m->lo[a]))
            return set_error("gt_track_mesh: axis %d needs finite lo < hi", a), GT_EINVAL;
        if (!(((m->hi[a] - m->lo[a]) / (double)m->n[a]) > 0.0))
            return set_error("gt_track_mesh: axis %d bins have no width", a), GT_EINVAL;
        bins *= m->n[a];
        if (bins > (1ull << 31)) return set_error("gt_track_mesh: more than 2^31 bins"), GT_ECAPACITY;
    }
    if (!m->mesh_fx) return set_error("gt_track_mesh: mesh_fx is required"), GT_EINVAL;
    const uint64_t need = gt_mesh_workspace_bytes(bins);
    if (!m->workspace || m->workspace_bytes < need)
        return set_error("gt_track_mesh: the workspace needs %llu bytes", (unsigned long long)need), GT_EINVAL;
    if (((uintptr_t)m->workspace) & 255u)
        return set_error("gt_track_mesh: the workspace must be 256-byte aligned"), GT_EINVAL;
    return launch_track(g, p, o, stream, m);
}

extern "C" int gt_track_event(const gt_geometry *g, const gt_track_params *p, const gt_track_out *o, void *bank,
                              uint64_t bank_bytes, void *stream) {
    int rc = check_track_args(g, p, o);
    if (rc) return rc;
    if (p->flags & ~GT_FLAG_ACCUMULATE)
        return set_error("gt_track_event: only GT_FLAG_ACCUMULATE applies"), GT_EINVAL;
    if (p->block_size || p->refill_min || p->regroup_every || p->wave_histories)
        return set_error("gt_track_event: no launch shape to set"), GT_EINVAL;
    const uint64_t need = ev_layout(p->n_particles, nullptr, nullptr);
    if (p->n_particles && (!bank || bank_bytes < need))
        return set_error("gt_track_event: the bank needs %llu bytes", (unsigned long long)need), GT_EINVAL;
    if (((uintptr_t)bank) & 255u) return set_error("gt_track_event: the bank must be 256-byte aligned"), GT_EINVAL;
    return launch_event(g, p, o, bank, stream);
}

extern "C" int gt_batch_create(const gt_batch_item *items, uint32_t n_items, const gt_tuning *tuning, gt_batch **out) {
    if (!out || (n_items && !items)) return set_error("gt_batch_create: null argument"), GT_EINVAL;
    *out = nullptr;
    if (n_items == 0) return set_error("gt_batch_create: empty batch"), GT_EINVAL;
    if (n_items > 16384) return set_error("gt_batch_create: at most 16384 items"), GT_ECAPACITY;
    gt_tuning cached;
    if (!tuning && cached_batch_tuning(items, n_items, &cached)) tuning = &cached;
    const uint32_t block = tuning && tuning->block_size ? tuning->block_size : 1024;
    const uint32_t refill = tuning && tuning->refill_min ? tuning->refill_min : 0;
    // 0: workgroups join whole items (the default); else histories per chunk
    const uint64_t chunk = tuning ? tuning->chunk : 0;
    const bool by_item = chunk == 0;
    if (block % 64 || block > 1024) return set_error("gt_batch_create: block_size must be a multiple of 64 up to 1024"), GT_EINVAL;
    if (refill > 64) return set_error("gt_batch_create: refill_min must be at most 64"), GT_EINVAL;
    const uint32_t wave = tuning ? tuning->wave_histories : 0;
    if (wave % 64 || wave > 1024)
        return set_error("gt_batch_create: wave_histories must be a multiple of 64 up to 1024"), GT_EINVAL;
    const uint32_t regroup =
        tuning && tuning->regroup_every ? tuning->regroup_every : items[0].params.regroup_every;
    try {
        const uint32_t prec = items[0].params.precision;
        const int dev = items[0].geometry ? items[0].geometry->device : 0;
        std::vector<BatchItem> bi(n_items);
        std::vector<FillRange> fills;
        std::vector<FinalizeItem> fin(n_items);
        std::vector<std::pair<double, uint32_t>> order;
        std::vector<uint8_t> kind(n_items);
        uint32_t lds[4] = {0, 0, 0, 0};
        uint64_t max_inst = 1, max_fill = 2;
        for (uint32_t i = 0; i < n_items; i++) {
            const gt_batch_item &it = items[i];
            int rc = check_track_args(it.geometry, &it.params, &it.out);
            if (rc) return set_error("gt_batch_create: item %u: %s", i, gt_last_error()), rc;
            if (it.params.precision != prec) return set_error("gt_batch_create: item %u: precision differs", i), GT_EINVAL;
            if (it.params.flags & GT_FLAG_LANE_PER_HISTORY)
                return set_error("gt_batch_create: item %u: GT_FLAG_LANE_PER_HISTORY is not available in batches", i), GT_EINVAL;
            if (it.params.flags & (GT_FLAG_TRACKER_SP | GT_FLAG_TRACKER_RTK))
                return set_error("gt_batch_create: item %u: batches run the single tracker only", i), GT_EINVAL;
            if (it.geometry->device != dev) return set_error("gt_batch_create: item %u: geometry on another device", i), GT_EINVAL;
            const gt_geometry *g = it.geometry;
            const void *wsi = it.out.workspace ? it.out.workspace : g->ws;
            for (uint32_t j = 0; j < i; j++)
                if ((items[j].out.workspace ? items[j].out.workspace : items[j].geometry->ws) == wsi)
                    return set_error("gt_batch_create: items %u and %u share a tally workspace (the same geometry "
                                     "without workspaces of their own)", j, i), GT_EINVAL;
            BatchItem &b = bi[i];
            b.dev = g->dev;
            b.plan = g->stage[prec];
            gt_track_params p = it.params;
            p.refill_min = refill ? refill : p.refill_min;
            p.wave_histories = wave ? wave : p.wave_histories;
            fill_kparams(&p, g, b.p, b.o, &it.out);
            kind[i] = (it.params.flags & GT_FLAG_NO_STAGING) ? 0 : (uint8_t)b.plan.kind;
            lds[kind[i]] = std::max(lds[kind[i]], kind[i] ? b.plan.total : 0u);
            fills.push_back({b.o.tally_ws, (uint64_t)tally_replicas(g->n_inst) * 4 * g->n_inst, 0, 8, 0});
            fills.push_back({it.out.counters, 8, 0, 8, 0});
            if (b.p.rec_k) fills.push_back({it.out.rec, (uint64_t)b.p.rec_k * b.p.rec_cap, (uint64_t)(uint32_t)-1, 4, 0});
            fin[i] = {b.o.tally_ws, it.out.tally_fx, it.out.tally, g->n_inst,
                      (uint32_t)((it.params.flags & GT_FLAG_ACCUMULATE) != 0), 0};
            max_inst = std::max(max_inst, g->n_inst);
            order.push_back({(double)it.params.n_particles * (double)g->max_depth, i});
        }
        // chunks grouped by staging kind (3, 2, 1, 0), each group largest cost first
        std::stable_sort(order.begin(), order.end(),
                         [](const std::pair<double, uint32_t> &a, const std::pair<double, uint32_t> &b) {
                             return a.first > b.first;
                         });
        std::vector<BatchChunk> chunks;
        std::vector<BatchSlot> slots;
        uint32_t n_kind[4] = {0, 0, 0, 0}, n_slot_kind[4] = {0, 0, 0, 0};
        uint64_t n_hist_kind[4] = {0, 0, 0, 0};
        for (int k = 3; k >= 0; k--) {
            const size_t before = chunks.size(), before_s = slots.size();
            double cum = 0.0;
            for (const auto &o : order) {
                const uint32_t i = o.second;
                if (kind[i] != k) continue;
                const uint64_t n = items[i].params.n_particles;
                if (n == 0) continue;
                n_hist_kind[k] += n;
                if (by_item) {
                    const float w = (float)items[i].geometry->max_depth;
                    cum += (double)n * w;
                    slots.push_back({i, w, n, cum});
                } else {
                    for (uint64_t f = 0; f < n; f += chunk) chunks.push_back({i, 0, f, std::min(chunk, n - f)});
                }
            }
            n_kind[k] = (uint32_t)(chunks.size() - before);
            n_slot_kind[k] = (uint32_t)(slots.size() - before_s);
        }
        if (chunks.size() > 0xFFFFFFF0u) return set_error("gt_batch_create: too many chunks"), GT_ECAPACITY;
        // Before anything reaches the device: the chunk groups are ordered by
        // kind (3 .. 0) and sized by n_kind, each chunk names an item of its
        // group's kind and is non-empty and at most `chunk` long, and each
        // item's chunks cover its histories [0, n) once, in order; or, with
        // whole items, every item with histories has one slot, in its kind's
        // group, with its n, a positive weight and a rising running sum.
        {
            std::vector<uint64_t> covered(n_items, 0);
            size_t at = 0;
            for (int k = 3; k >= 0; k--)
                for (uint32_t c = 0; c < n_kind[k]; c++, at++) {
                    const BatchChunk &ch = chunks[at];
                    if (ch.item >= n_items || kind[ch.item] != k || ch.count == 0 || ch.count > chunk ||
                        ch.first != covered[ch.item])
                        return set_error("gt_batch_create: chunk %zu is inconsistent", at), GT_EINVAL;
                    covered[ch.item] += ch.count;
                }
            if (at != chunks.size()) return set_error("gt_batch_create: chunk groups do not add up"), GT_EINVAL;
            at = 0;
            for (int k = 3; k >= 0; k--) {
                double prev = 0.0;
                for (uint32_t c = 0; c < n_slot_kind[k]; c++, at++) {
                    const BatchSlot &sl = slots[at];
                    if (sl.item >= n_items || kind[sl.item] != k || sl.n == 0 || covered[sl.item] != 0 ||
                        sl.n != items[sl.item].params.n_particles || !(sl.weight > 0.0f) || !(sl.cum > prev))
                        return set_error("gt_batch_create: item slot %zu is inconsistent", at), GT_EINVAL;
                    covered[sl.item] = sl.n;
                    prev = sl.cum;
                }
            }
            if (at != slots.size()) return set_error("gt_batch_create: item groups do not add up"), GT_EINVAL;
            for (uint32_t i = 0; i < n_items; i++)
                if (covered[i] != items[i].params.n_particles)
                    return set_error("gt_batch_create: item %u's histories are not covered by its %s", i,
                                     by_item ? "slot" : "chunks"),
                           GT_EINVAL;
        }
        // one device allocation: items, chunks, item slots, fills, finalize
        // items, then the counters: four queue counters (one per staging
        // kind), each item's claim counter and each item's workgroup count
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t n_ctr = 4 + 2 * (size_t)n_items;
        const size_t o_items = 0;
        const size_t o_chunks = al(o_items + bi.size() * sizeof(BatchItem));
        const size_t o_slots = al(o_chunks + std::max<size_t>(chunks.size(), 1) * sizeof(BatchChunk));
        const size_t o_queue = al(o_slots + std::max<size_t>(slots.size(), 1) * sizeof(BatchSlot));
        const size_t o_fill = al(o_queue + n_ctr * sizeof(unsigned long long));
        const size_t o_fin = al(o_fill + (fills.size() + 1) * sizeof(FillRange));
        const size_t total = al(o_fin + fin.size() * sizeof(FinalizeItem));
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return set_error("hipGetDevice failed"), GT_EHIP;
        if (cur != dev) return set_error("gt_batch_create: current device is not the geometries' device"), GT_EINVAL;
        void *dm = nullptr;
        hipError_t e = hipMalloc(&dm, total);
        if (e != hipSuccess) return set_error("hipMalloc(%zu): %s", total, hipGetErrorString(e)), GT_ENOMEM;
        unsigned char *base = (unsigned char *)dm;
        fills.push_back({base + o_queue, n_ctr, 0, 8, 0});
        for (const FillRange &f : fills) max_fill = std::max(max_fill, f.count);
        std::vector<unsigned char> img(total, 0);
        std::memcpy(img.data() + o_items, bi.data(), bi.size() * sizeof(BatchItem));
        if (!chunks.empty()) std::memcpy(img.data() + o_chunks, chunks.data(), chunks.size() * sizeof(BatchChunk));
        if (!slots.empty()) std::memcpy(img.data() + o_slots, slots.data(), slots.size() * sizeof(BatchSlot));
        std::memcpy(img.data() + o_fill, fills.data(), fills.size() * sizeof(FillRange));
        std::memcpy(img.data() + o_fin, fin.data(), fin.size() * sizeof(FinalizeItem));
        e = hipMemcpy(dm, img.data(), total, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dm);
            return set_error("hipMemcpy: %s", hipGetErrorString(e)), GT_EHIP;
        }
        gt_batch *b = new gt_batch;
        b->device = dev;
        b->precision = prec;
        b->n_items = n_items;
        b->block = block;
        b->refill_min = refill;
        b->dmem = dm;
        b->d_items = (BatchItem *)(base + o_items);
        b->d_chunks = (BatchChunk *)(base + o_chunks);
        b->n_chunks = (uint32_t)chunks.size();
        for (int k = 0; k < 4; k++) b->n_kind[k] = n_kind[k];
        b->d_fill = (FillRange *)(base + o_fill);
        b->n_fill = (uint32_t)fills.size();
        b->max_fill = max_fill;
        b->d_fin = (FinalizeItem *)(base + o_fin);
        b->max_inst = max_inst;
        b->d_queue = (unsigned long long *)(base + o_queue);
        b->by_item = by_item;
        b->d_slots = (BatchSlot *)(base + o_slots);
        b->n_slots = (uint32_t)slots.size();
        for (int k = 0; k < 4; k++) {
            b->n_slot_kind[k] = n_slot_kind[k];
            b->n_hist_kind[k] = n_hist_kind[k];
        }
        b->d_claimed = b->d_queue + 4;
        b->d_workers = b->d_queue + 4 + n_items;
        for (int k = 0; k < 4; k++) b->lds_bytes[k] = lds[k];
        b->tail = (items[0].params.flags & GT_FLAG_TAIL_COMPACTION) != 0;
        b->regroup = regroup;
        b->cache = !(items[0].params.flags & GT_FLAG_NO_TALLY_CACHE);
        b->side = nullptr;
        const int rcs = prepare_batch_streams(b);
        if (rcs) {
            gt_batch_destroy(b);
            return rcs;
        }
        *out = b;
        return GT_OK;
    } catch (const std::bad_alloc &) {
        return set_error("host allocation failed"), GT_ENOMEM;
    } catch (...) {
        return set_error("unexpected exception in gt_batch_create"), GT_EINVAL;
    }
}

extern "C" int gt_last_launch(gt_launch_info *out) {
    if (!out) return set_error("gt_last_launch: out is NULL"), GT_EINVAL;
    return last_launch(out) ? 1 : 0;
}

extern "C" int gt_set_kernel_events(void *start_event, void *stop_event) {
    if ((start_event == nullptr) != (stop_event == nullptr))
        return set_error("gt_set_kernel_events: give both events or neither"), GT_EINVAL;
    set_kernel_events(start_event, stop_event);
    return GT_OK;
}

extern "C" int gt_batch_launch(gt_batch *b, void *stream) {
    if (!b) return set_error("gt_batch_launch: null batch"), GT_EINVAL;
    return launch_batch(b, stream);
}

extern "C" void gt_batch_destroy(gt_batch *b) {
    if (!b) return;
    int cur = 0;
    bool switched = hipGetDevice(&cur) == hipSuccess && cur != b->device && hipSetDevice(b->device) == hipSuccess;
    release_batch_streams(b);
    (void)hipFree(b->dmem);
    if (switched) (void)hipSetDevice(cur);
    delete b;
}

extern "C" int gt_track_batch(const gt_batch_item *items, uint32_t n_items, const gt_tuning *tuning, void *stream) {
    gt_batch *b = nullptr;
    int rc = gt_batch_create(items, n_items, tuning, &b);
    if (rc) return rc;
    rc = gt_batch_launch(b, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    gt_batch_destroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return set_error("hipStreamSynchronize: %s", hipGetErrorString(e)), GT_EHIP;
    return GT_OK;
}

extern "C" int gt_find_cell(const gt_geometry *g, const double *pos, uint64_t n, int64_t *inst, int32_t *cells,
                            uint32_t precision, void *stream) {
    if (!g || (n && (!pos || !inst))) return set_error("gt_find_cell: null argument"), GT_EINVAL;
    if (precision > GT_PREC_MIXED) return set_error("gt_find_cell: unknown precision %u", precision), GT_EINVAL;
    return launch_find_cell(g, pos, n, inst, cells, precision, stream);
}

extern "C" int gt_distance_to_surface(const gt_geometry *g, const double *pos, const double *dir,
                                      const int32_t *state, uint64_t n, double *dist, int32_t *level, int32_t *surf,
                                      void *stream) {
    if (!g || (n && (!pos || !dir || !dist || !level || !surf)))
        return set_error("gt_distance_to_surface: null argument"), GT_EINVAL;
    return launch_distance(g, pos, dir, state, n, dist, level, surf, stream);
}

extern "C" int gt_fp64_check(const double *a, const double *b, uint64_t n, double *quot, double *root, double *logb,
                             void *stream) {
    if (n && (!a || !b || !quot || !root || !logb)) return set_error("gt_fp64_check: null argument"), GT_EINVAL;
    return launch_fp64_check(a, b, n, quot, root, logb, stream);
}
