/*
 * oracle.c -- plain CPU oracle for Monte Carlo geometry tracking through
 * nested CSG universes (Biondo et al., "Comparison of nested geometry
 * treatments within GPU-based Monte Carlo neutron transport simulations of
 * fission reactors").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant generator with the HIP path.
 *
 * What it computes is the plain definition of the method:
 *   - find_cell:      linear scan over a universe's cells (Section "Single
 *                     universe tracking", Alg. 3), descending through fills
 *                     (Section "Multi-universe CPU tracking", Alg. 7);
 *   - cross_surface:  scan of the crossed surface's neighbour list, skipping
 *                     the cell of origin (Alg. 4), at the top-most level the
 *                     particle is on a surface, then descent (Alg. 8);
 *   - distance_to_surface / move_within_cell / change_direction: Table 1;
 *   - the history loop of Alg. 2, reduced to a toy transport: exponential
 *     flights with a per-material attenuation coefficient, isotropic
 *     redirection at each collision, a collision cap and a vacuum boundary.
 * No tree, no lattice arithmetic, no reduced precision: every decision is an
 * IEEE double comparison evaluated in the operation order fixed below.
 *
 * Readings where the paper is silent (documented with the design notes):
 *   sense of a point exactly on a surface is negative (f <= 0);
 *   cells are intersections of half-spaces; a fill places its daughter with a
 *   translation, local = parent - t;  distance ties break on (distance,
 *   level, surface id) so the top-most level wins (the "surf_universe" of
 *   Alg. 8);  a distance equal to the collision distance is a collision (the
 *   strict "d < tau/Sigma" of Alg. 2);  tallies are per leaf instance.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -msse2 -shared -fPIC
 *        (no FMA contraction, SSE2 doubles, denormals on).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 8
#define OR_MAX_THREADS 256
#define OR_MAX_BIRTH_ATTEMPTS 1000

enum { S_PX = 0, S_PY = 1, S_PZ = 2, S_P = 3, S_CZ = 4, S_SPH = 5 };
enum { END_NONE = 0, END_ESCAPE = 1, END_CAP = 2, END_LOST = 3, END_SEGCAP = 4 };
enum { C_ESCAPED = 0, C_CAPPED, C_LOST, C_SEGCAP, C_RECOVF, C_SEGMENTS, C_REJECTED, C_NC };

/* Work meter (off unless or_count_work runs): counts the double-precision
 * arithmetic operations (+ - * / sqrt; comparisons and sign flips excluded)
 * that the method itself requires -- every distance evaluation of every
 * level, the moves, the sampling, and one containment test of each cell
 * that is located -- but not the extra candidates a linear scan tries. */
static __thread uint64_t *meter;
#define METER(n) do { if (meter) *meter += (uint64_t)(n); } while (0)

/* ------------------------------------------------------------------ */
/* input contract                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t n_surfaces, n_cells, n_universes, n_materials, n_hs, root;
    const uint8_t *surf_type;
    const double *surf_coef;      /* 8 per surface */
    const uint32_t *cell_hs_off;  /* n_cells + 1 */
    const int32_t *hs;            /* +-(surface+1) */
    const int32_t *cell_fill;     /* >=0 material, <0 -(universe+1) */
    const double *cell_trans;     /* 3 per cell */
    const uint32_t *univ_cell_off;/* n_universes + 1 */
    const double *sigma_t;
    double domain_lo[3], domain_hi[3];
} or_flat;

typedef struct {
    uint64_t seed, first_particle, n_particles;
    uint32_t geometry_id, max_collisions;
    uint32_t source;       /* 0 volume-uniform isotropic; 1 parallel rays along +x */
    uint32_t ray_n1;       /* ray grid: particle i -> (i % n1, i / n1) on the x = lo face */
    uint32_t max_segments; /* per particle; reaching it ends the history (SEGCAP) */
    uint32_t record_first_k, record_cap, pad;
} or_params;

typedef struct {
    uint64_t *tally_fx;   /* [2 * n_inst]: (lo, hi) of a 128-bit fixed-point sum, quantum 2^-96 */
    double *tally;        /* [n_inst] Neumaier sum of segment lengths */
    double *tally_fxd;    /* [n_inst] the fixed-point sum rounded to double */
    uint32_t *seg_count;  /* [n_particles] */
    uint64_t *seq_hash;   /* [n_particles] */
    uint8_t *end_code;    /* [n_particles] */
    int32_t *rec;         /* [record_first_k * record_cap], -1 padded */
    uint64_t *counters;   /* [8] */
    const struct or_mesh *mesh;   /* superimposed mesh tally, or NULL */
} or_out;

/* Superimposed mesh tally (the paper's active cycles add a regular mesh
 * flux tally over the core): n[0] x n[1] x n[2] bins over the box [lo, hi],
 * bin (ix, iy, iz) at index (iz * n[1] + iy) * n[0] + ix.  Outputs as the
 * cell tally: 128-bit fixed point (quantum 2^-96), Neumaier sum, and the
 * fixed point rounded to double; each may be NULL. */
typedef struct or_mesh {
    double lo[3], hi[3];
    uint32_t n[3], pad;
    uint64_t *mesh_fx;    /* [2 * bins] */
    double *mesh;         /* [bins] */
    double *mesh_fxd;     /* [bins] */
} or_mesh;

typedef struct {          /* per-segment record of one particle */
    uint32_t cap, n, n_flights, pad;
    double *seg_len, *seg_sigma, *seg_pos;   /* pos: end of segment, 3 per */
    int64_t *seg_inst;
    uint8_t *seg_kind;                       /* 0 boundary, 1 collision */
    double *flight_tau;                      /* tau sampled at each flight start */
    double birth_pos[3], birth_dir[3];
    uint8_t end_code, pad2[7];
    /* optional (NULL): the tracking state at the start of each segment --
     * position and direction (3 each), and OR_STATE_W int32 words: the cell
     * of levels 0..OR_STATE_LEVELS-1 (-1 below the leaf), then the level and
     * surface the particle is on (-1, -1 when on none) */
    double *st_pos, *st_dir;
    int32_t *st_state;
} or_trace;

#define OR_STATE_LEVELS 6
#define OR_STATE_W (OR_STATE_LEVELS + 2)

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t ns, nc, nu, nm, nh, root;
    uint8_t *stype;
    double *coef;
    uint32_t *hs_off;
    int32_t *hs;
    int32_t *fill;
    double *trans;
    uint32_t *uoff;
    double *sigma;
    double lo[3], hi[3];
    /* derived */
    uint32_t *cell_univ;
    uint64_t *univ_ninst;
    uint64_t *inst_off;
    uint32_t *nb_off, *nb;    /* neighbour list per surface: cells using it, ascending */
    uint32_t max_depth;
    uint64_t n_inst;
} or_geom;

static void *dup(const void *src, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (p && bytes) memcpy(p, src, bytes);
    return p;
}

void or_geometry_destroy(or_geom *g) {
    if (!g) return;
    free(g->stype); free(g->coef); free(g->hs_off); free(g->hs); free(g->fill);
    free(g->trans); free(g->uoff); free(g->sigma); free(g->cell_univ);
    free(g->univ_ninst); free(g->inst_off); free(g->nb_off); free(g->nb);
    free(g);
}

/* number of leaf instances below universe u: materials count 1, fills count
 * their daughter's instances (the per-instance cell tallies of the Empire
 * study are this quantity for the pin sub-cells). */
static int count_inst(or_geom *g, uint32_t u, uint8_t *state, uint32_t *depth) {
    if (state[u] == 2) return 0;
    if (state[u] == 1) return -1; /* cycle */
    state[u] = 1;
    uint64_t n = 0;
    uint32_t d = 1;
    for (uint32_t c = g->uoff[u]; c < g->uoff[u + 1]; c++) {
        g->inst_off[c] = n;
        if (g->fill[c] >= 0) {
            n += 1;
        } else {
            uint32_t du = (uint32_t)(-g->fill[c] - 1);
            if (count_inst(g, du, state, depth)) return -1;
            n += g->univ_ninst[du];
            if (depth[du] + 1 > d) d = depth[du] + 1;
        }
    }
    g->univ_ninst[u] = n;
    depth[u] = d;
    state[u] = 2;
    return 0;
}

int or_geometry_create(const or_flat *f, or_geom **out, char *err, int errlen) {
#define FAIL(...) do { if (err) snprintf(err, errlen, __VA_ARGS__); or_geometry_destroy(g); return -2; } while (0)
    *out = NULL;
    or_geom *g = calloc(1, sizeof *g);
    if (!g) return -3;
    g->ns = f->n_surfaces; g->nc = f->n_cells; g->nu = f->n_universes;
    g->nm = f->n_materials; g->nh = f->n_hs; g->root = f->root;
    g->stype = dup(f->surf_type, g->ns);
    g->coef = dup(f->surf_coef, sizeof(double) * 8 * g->ns);
    g->hs_off = dup(f->cell_hs_off, sizeof(uint32_t) * (g->nc + 1));
    g->hs = dup(f->hs, sizeof(int32_t) * g->nh);
    g->fill = dup(f->cell_fill, sizeof(int32_t) * g->nc);
    g->trans = dup(f->cell_trans, sizeof(double) * 3 * g->nc);
    g->uoff = dup(f->univ_cell_off, sizeof(uint32_t) * (g->nu + 1));
    g->sigma = dup(f->sigma_t, sizeof(double) * g->nm);
    memcpy(g->lo, f->domain_lo, sizeof g->lo);
    memcpy(g->hi, f->domain_hi, sizeof g->hi);
    if (g->nu == 0 || g->nc == 0) FAIL("empty geometry");
    if (g->root >= g->nu) FAIL("root universe %u out of range", g->root);
    for (uint32_t s = 0; s < g->ns; s++)
        if (g->stype[s] > S_SPH) FAIL("surface %u: bad type %u", s, g->stype[s]);
    for (uint32_t m = 0; m < g->nm; m++)
        if (!(g->sigma[m] > 0) || isinf(g->sigma[m])) FAIL("material %u: bad sigma", m);
    if (g->uoff[0] != 0 || g->uoff[g->nu] != g->nc) FAIL("universe offsets do not cover the cells");
    if (g->hs_off[0] != 0 || g->hs_off[g->nc] != g->nh) FAIL("half-space offsets inconsistent");
    for (int k = 0; k < 3; k++) if (!(g->lo[k] < g->hi[k])) FAIL("domain box empty on axis %d", k);
    g->cell_univ = malloc(sizeof(uint32_t) * g->nc);
    for (uint32_t u = 0; u < g->nu; u++) {
        if (g->uoff[u + 1] <= g->uoff[u]) FAIL("universe %u has no cells", u);
        for (uint32_t c = g->uoff[u]; c < g->uoff[u + 1]; c++) g->cell_univ[c] = u;
    }
    /* surface ownership and neighbour lists */
    int64_t *owner = malloc(sizeof(int64_t) * (g->ns ? g->ns : 1));
    for (uint32_t s = 0; s < g->ns; s++) owner[s] = -1;
    g->nb_off = calloc(g->ns + 1, sizeof(uint32_t));
    for (uint32_t c = 0; c < g->nc; c++) {
        if (g->hs_off[c + 1] < g->hs_off[c]) { free(owner); FAIL("cell %u: bad half-space range", c); }
        for (uint32_t k = g->hs_off[c]; k < g->hs_off[c + 1]; k++) {
            int32_t h = g->hs[k];
            if (h == 0 || (uint32_t)abs(h) > g->ns) { free(owner); FAIL("cell %u: bad half-space %d", c, h); }
            uint32_t s = (uint32_t)abs(h) - 1;
            for (uint32_t k2 = g->hs_off[c]; k2 < k; k2++)
                if ((uint32_t)abs(g->hs[k2]) - 1 == s) { free(owner); FAIL("cell %u: surface %u repeated", c, s); }
            if (owner[s] >= 0 && owner[s] != (int64_t)g->cell_univ[c]) {
                long long prev = (long long)owner[s];
                free(owner); FAIL("surface %u used by universes %lld and %u", s, prev, g->cell_univ[c]);
            }
            owner[s] = g->cell_univ[c];
            g->nb_off[s + 1]++;
        }
        if (g->fill[c] >= 0) {
            if ((uint32_t)g->fill[c] >= g->nm) { free(owner); FAIL("cell %u: material out of range", c); }
        } else if ((uint32_t)(-(int64_t)g->fill[c] - 1) >= g->nu) {
            free(owner); FAIL("cell %u: daughter universe out of range", c);
        }
    }
    free(owner);
    for (uint32_t s = 0; s < g->ns; s++) g->nb_off[s + 1] += g->nb_off[s];
    g->nb = malloc(sizeof(uint32_t) * (g->nb_off[g->ns] ? g->nb_off[g->ns] : 1));
    uint32_t *fillpos = calloc(g->ns + 1, sizeof(uint32_t));
    for (uint32_t c = 0; c < g->nc; c++)          /* ascending cell id */
        for (uint32_t k = g->hs_off[c]; k < g->hs_off[c + 1]; k++) {
            uint32_t s = (uint32_t)abs(g->hs[k]) - 1;
            g->nb[g->nb_off[s] + fillpos[s]++] = c;
        }
    free(fillpos);
    /* instances and depth */
    g->univ_ninst = calloc(g->nu, sizeof(uint64_t));
    g->inst_off = calloc(g->nc, sizeof(uint64_t));
    uint8_t *state = calloc(g->nu, 1);
    uint32_t *depth = calloc(g->nu, sizeof(uint32_t));
    int rc = count_inst(g, g->root, state, depth);
    for (uint32_t u = 0; u < g->nu && rc == 0; u++) rc = count_inst(g, u, state, depth);
    g->max_depth = depth[g->root];
    free(state); free(depth);
    if (rc) FAIL("fill graph has a cycle");
    if (g->max_depth > OR_MAXL) FAIL("nesting depth %u exceeds %d", g->max_depth, OR_MAXL);
    g->n_inst = g->univ_ninst[g->root];
    *out = g;
    return 0;
#undef FAIL
}

uint64_t or_geometry_n_instances(const or_geom *g) { return g->n_inst; }
uint32_t or_geometry_max_depth(const or_geom *g) { return g->max_depth; }

/* ------------------------------------------------------------------ */
/* surfaces: value f(p) and sense (positive iff f > 0)                 */
/* ------------------------------------------------------------------ */
static double surf_f(const or_geom *g, uint32_t s, const double p[3]) {
    const double *c = g->coef + 8 * (size_t)s;
    double dx, dy, dz;
    switch (g->stype[s]) {
    case S_PX: return p[0] - c[0];
    case S_PY: return p[1] - c[0];
    case S_PZ: return p[2] - c[0];
    case S_P:  return ((c[0] * p[0] + c[1] * p[1]) + c[2] * p[2]) - c[3];
    case S_CZ:
        dx = p[0] - c[0]; dy = p[1] - c[1];
        return (dx * dx + dy * dy) - c[2];
    default:
        dx = p[0] - c[0]; dy = p[1] - c[1]; dz = p[2] - c[2];
        return ((dx * dx + dy * dy) + dz * dz) - c[3];
    }
}

/* A cell contains p when p is on the required side of every half-space.
 * When force_s >= 0 the sense on that surface is taken as force_pos instead
 * of being evaluated (the logical sense of the surface being crossed). */
static int cell_contains(const or_geom *g, uint32_t c, const double p[3], int64_t force_s, int force_pos) {
    for (uint32_t k = g->hs_off[c]; k < g->hs_off[c + 1]; k++) {
        int32_t h = g->hs[k];
        uint32_t s = (uint32_t)abs(h) - 1;
        int want_pos = h > 0;
        int is_pos = ((int64_t)s == force_s) ? force_pos : (surf_f(g, s, p) > 0.0);
        if (is_pos != want_pos) return 0;
    }
    return 1;
}

static uint64_t surf_value_ops(int type) {
    switch (type) {
    case S_PX: case S_PY: case S_PZ: return 1;
    case S_P: case S_CZ: return 6;
    default: return 9;
    }
}

/* operations of one containment test of cell c (forced surface free) */
static void meter_verify(const or_geom *g, int64_t c, int64_t force_s) {
    if (!meter || c < 0) return;
    for (uint32_t k = g->hs_off[c]; k < g->hs_off[c + 1]; k++) {
        int64_t s = abs(g->hs[k]) - 1;
        if (s != force_s) *meter += surf_value_ops(g->stype[s]);
    }
}

/* Alg. 3: first cell of universe u containing p, or -1. */
static int64_t find_cell_in(const or_geom *g, uint32_t u, const double p[3]) {
    for (uint32_t c = g->uoff[u]; c < g->uoff[u + 1]; c++)
        if (cell_contains(g, c, p, -1, 0)) { meter_verify(g, c, -1); return c; }
    return -1;
}

/* ------------------------------------------------------------------ */
/* particle state                                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    double p[3], u[3], tau;
    int64_t cell[OR_MAXL];
    int depth;
    int on_level;          /* -1: not on a surface */
    int64_t on_surf;
    uint64_t pid;
    uint32_t draw;         /* index of the next random-number block */
} ptl;

static void local_pos(const or_geom *g, const ptl *t, int level, double q[3]) {
    q[0] = t->p[0]; q[1] = t->p[1]; q[2] = t->p[2];
    for (int L = 0; L < level; L++) {
        const double *tr = g->trans + 3 * (size_t)t->cell[L];
        q[0] = q[0] - tr[0]; q[1] = q[1] - tr[1]; q[2] = q[2] - tr[2];
    }
}

/* Alg. 7 descent below `level`: while the cell is filled, find the cell of
 * the daughter universe containing the local position.  0 ok, -1 none. */
static int descend(const or_geom *g, ptl *t, int level, double q[3]) {
    int L = level;
    while (g->fill[t->cell[L]] < 0) {
        uint32_t du = (uint32_t)(-g->fill[t->cell[L]] - 1);
        const double *tr = g->trans + 3 * (size_t)t->cell[L];
        q[0] = q[0] - tr[0]; q[1] = q[1] - tr[1]; q[2] = q[2] - tr[2];
        METER(3);
        int64_t c = find_cell_in(g, du, q);
        if (c < 0) { t->depth = L + 1; return -1; }
        t->cell[++L] = c;
    }
    t->depth = L + 1;
    return 0;
}

static uint64_t leaf_inst(const or_geom *g, const ptl *t) {
    uint64_t i = 0;
    for (int L = 0; L < t->depth; L++) i += g->inst_off[t->cell[L]];
    return i;
}

static uint32_t leaf_material(const or_geom *g, const ptl *t) {
    return (uint32_t)g->fill[t->cell[t->depth - 1]];
}

/* ------------------------------------------------------------------ */
/* Table 1: distance_to_surface                                        */
/* ------------------------------------------------------------------ */
/* distance along u from q to the point where the sense of surface s flips
 * away from the cell's required sense (pos = required side is positive);
 * INFINITY when it does not.  `on` marks the surface just crossed. */
static double hs_distance(const or_geom *g, uint32_t s, int pos, const double q[3], const double u[3], int on) {
    const double *c = g->coef + 8 * (size_t)s;
    int type = g->stype[s];
    double t;
    if (type <= S_P) {
        if (on) return INFINITY;
        double den;
        switch (type) {
        case S_PX: den = u[0]; break;
        case S_PY: den = u[1]; break;
        case S_PZ: den = u[2]; break;
        default:   den = (c[0] * u[0] + c[1] * u[1]) + c[2] * u[2]; METER(5); break;
        }
        if (den == 0.0) return INFINITY;
        if (!((!pos && den > 0.0) || (pos && den < 0.0))) return INFINITY;
        t = (-surf_f(g, s, q)) / den;
        METER(surf_value_ops(type) + 1);
    } else {
        double a, b, dx = q[0] - c[0], dy = q[1] - c[1];
        if (type == S_CZ) {
            a = u[0] * u[0] + u[1] * u[1];
            b = dx * u[0] + dy * u[1];
        } else {
            double dz = q[2] - c[2];
            a = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
            b = (dx * u[0] + dy * u[1]) + dz * u[2];
        }
        METER(type == S_CZ ? 8 : 13);
        if (a == 0.0) return INFINITY;
        if (on) {
            if (!pos && b < 0.0) { t = (-2.0 * b) / a; METER(2); }
            else return INFINITY;
        } else {
            double cc = surf_f(g, s, q);
            double disc = b * b - a * cc;
            METER(type == S_CZ ? 7 : 9);
            if (!(disc > 0.0)) return INFINITY;
            double qq = sqrt(disc);
            METER(3);
            if (!pos) {
                t = (b <= 0.0) ? (qq - b) / a : (-cc) / (b + qq);
            } else {
                if (b < 0.0) t = cc / (qq - b);
                else return INFINITY;
            }
        }
    }
    if (!(t > 0.0)) t = 0.0;   /* clamp negatives and -0 to +0 */
    return t;
}

/* minimum over all levels and all half-spaces of each level's cell; ties go
 * to the top-most level, then the lowest surface id. */
static double distance_to_surface(const or_geom *g, const ptl *t, int *out_level, int64_t *out_surf) {
    double best = INFINITY;
    int bl = OR_MAXL;
    int64_t bs = INT64_MAX;
    double q[3];
    for (int L = 0; L < t->depth; L++) {
        local_pos(g, t, L, q);
        if (L > 0) METER(3);
        int64_t c = t->cell[L];
        for (uint32_t k = g->hs_off[c]; k < g->hs_off[c + 1]; k++) {
            int32_t h = g->hs[k];
            int64_t s = abs(h) - 1;
            int on = (t->on_level == L && t->on_surf == s);
            double d = hs_distance(g, (uint32_t)s, h > 0, q, t->u, on);
            if (d < best || (d == best && (L < bl || (L == bl && s < bs)))) {
                if (d == INFINITY) continue;
                best = d; bl = L; bs = s;
            }
        }
    }
    *out_level = bl;
    *out_surf = bs;
    return best;
}

/* ------------------------------------------------------------------ */
/* Alg. 4 / Alg. 8: cross_surface at the top-most level on the surface  */
/* ------------------------------------------------------------------ */
static int cross_surface(const or_geom *g, ptl *t, int level, int64_t surf) {
    double q[3];
    local_pos(g, t, level, q);
    METER(3 * level);
    int64_t old = t->cell[level];
    int old_pos = -1;
    for (uint32_t k = g->hs_off[old]; k < g->hs_off[old + 1]; k++)
        if (abs(g->hs[k]) - 1 == surf) old_pos = g->hs[k] > 0;
    int force_pos = !old_pos;
    int64_t found = -1;
    for (uint32_t k = g->nb_off[surf]; k < g->nb_off[surf + 1] && found < 0; k++) {
        uint32_t c = g->nb[k];
        if ((int64_t)c == old) continue;
        if (cell_contains(g, c, q, surf, force_pos)) found = c;
    }
    if (found < 0) {  /* fall back to every cell of the universe */
        uint32_t u = g->cell_univ[old];
        for (uint32_t c = g->uoff[u]; c < g->uoff[u + 1] && found < 0; c++) {
            if ((int64_t)c == old) continue;
            if (cell_contains(g, c, q, surf, force_pos)) found = c;
        }
    }
    if (found < 0) return level == 0 ? END_ESCAPE : END_LOST;
    meter_verify(g, found, surf);
    t->cell[level] = found;
    if (descend(g, t, level, q)) return END_LOST;
    t->on_level = level;
    t->on_surf = surf;
    return END_NONE;
}

/* ------------------------------------------------------------------ */
/* random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)    */
/* ------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Random numbers.  Every sampling event of a particle takes one whole
 * Philox4x32-10 block: counter (b, pid lo, pid hi, geometry id) under the
 * key = seed, b being the particle's block index (0, 1, 2, ... in order of
 * use).  The block's 128 bits (word 0 least significant) are cut into three
 * 42-bit fields f0 = bits [0,42), f1 = [42,84), f2 = [84,126), each mapped
 * to the uniform (f + 1/2) 2^-42 in (0,1).  A birth-position attempt uses
 * f0, f1, f2 for x, y, z; a direction attempt uses f0, f1 for Marsaglia's
 * pair and, once accepted, f2 for the optical depth of the next flight. */
static void rng_fields(uint64_t seed, uint32_t geom_id, uint64_t pid, uint32_t b, uint64_t f[3]) {
    uint32_t ctr[4] = { b, (uint32_t)pid, (uint32_t)(pid >> 32), geom_id };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t o[4];
    or_philox4x32_10(ctr, key, o);
    uint64_t w0 = (uint64_t)o[1] << 32 | o[0], w1 = (uint64_t)o[3] << 32 | o[2];
    const uint64_t m42 = (1ull << 42) - 1;
    f[0] = w0 & m42;
    f[1] = (w0 >> 42) | ((w1 & ((1ull << 20) - 1)) << 22);
    f[2] = (w1 >> 20) & m42;
}

/* uniform double in (0,1) from a 42-bit field: (f + 1/2) 2^-42, exact */
double or_u01(uint64_t f) {
    METER(2);
    return ((double)f + 0.5) * 0x1p-42;
}

/* natural log of a positive normal double, from the series
 * log m = 2 atanh(s), s = (m-1)/(m+1), with m in [sqrt(1/2), sqrt(2)).
 * Coefficients 1/(2k+1) are single IEEE divisions. */
static double LOGC[12];
static pthread_once_t logc_once = PTHREAD_ONCE_INIT;
static void logc_init(void) { for (int k = 0; k < 12; k++) LOGC[k] = 1.0 / (double)(2 * k + 1); }

double or_mc_log(double x) {
    pthread_once(&logc_once, logc_init);
    uint64_t bits;
    memcpy(&bits, &x, 8);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    uint64_t mb = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mb, 8);
    const uint64_t sqrt2_bits = 0x3FF6A09E667F3BCDull;
    double sqrt2;
    memcpy(&sqrt2, &sqrt2_bits, 8);
    if (m >= sqrt2) { m = m * 0.5; e = e + 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    METER(4 + 22 + 2 + 4);
    double poly = LOGC[11];
    for (int k = 10; k >= 0; k--) poly = poly * z + LOGC[k];
    double logm = (s + s) * poly;
    const uint64_t hi_bits = 0x3FE62E42FEE00000ull, lo_bits = 0x3DEA39EF35793C76ull;
    double ln2_hi, ln2_lo;
    memcpy(&ln2_hi, &hi_bits, 8);
    memcpy(&ln2_lo, &lo_bits, 8);
    double de = (double)e;
    return de * ln2_hi + (de * ln2_lo + logm);
}

void or_mc_log_batch(const double *x, uint64_t n, double *out) {
    for (uint64_t i = 0; i < n; i++) out[i] = or_mc_log(x[i]);
}

static void next_block(const or_params *pr, ptl *t, uint64_t f[3]) {
    rng_fields(pr->seed, pr->geometry_id, t->pid, t->draw++, f);
}

/* change_direction (Table 1) to an isotropic direction, Marsaglia (1972),
 * and a new exponential(1) optical depth tau = -log U for the next flight */
static void sample_flight(const or_params *pr, ptl *t) {
    double v1, v2, s;
    uint64_t f[3];
    for (;;) {
        next_block(pr, t, f);
        v1 = 2.0 * or_u01(f[0]) - 1.0;
        v2 = 2.0 * or_u01(f[1]) - 1.0;
        s = v1 * v1 + v2 * v2;
        METER(7);
        if (s < 1.0 && s != 0.0) break;
    }
    METER(8);
    double r = sqrt(1.0 - s);
    t->u[0] = (2.0 * v1) * r;
    t->u[1] = (2.0 * v2) * r;
    t->u[2] = 1.0 - 2.0 * s;
    t->tau = -or_mc_log(or_u01(f[2]));
}

/* Birth (Alg. 2 sampling lines): uniform position in the domain box,
 * rejected until the root universe has a cell there; then descent,
 * direction, optical depth.  Returns END_NONE or END_LOST. */
static int birth(const or_geom *g, const or_params *pr, ptl *t, uint64_t local, uint64_t *rejected) {
    memset(t, 0, sizeof *t);
    t->pid = pr->first_particle + local;
    t->on_level = -1;
    t->on_surf = -1;
    double q[3];
    if (pr->source == 1) {
        uint64_t n1 = pr->ray_n1 ? pr->ray_n1 : 1;
        uint64_t n2 = (pr->n_particles + n1 - 1) / n1;
        uint64_t j = t->pid % n1, k = t->pid / n1;
        double hy = (g->hi[1] - g->lo[1]) / (double)n1;
        double hz = (g->hi[2] - g->lo[2]) / (double)n2;
        t->p[0] = g->lo[0] + (g->hi[0] - g->lo[0]) * 0x1p-30;
        t->p[1] = g->lo[1] + ((double)j + 0.5) * hy;
        t->p[2] = g->lo[2] + ((double)k + 0.5) * hz;
        t->u[0] = 1.0; t->u[1] = 0.0; t->u[2] = 0.0;
        t->tau = 0.0;
        int64_t c = find_cell_in(g, g->root, t->p);
        if (c < 0) return END_LOST;
        t->cell[0] = c;
        q[0] = t->p[0]; q[1] = t->p[1]; q[2] = t->p[2];
        return descend(g, t, 0, q) ? END_LOST : END_NONE;
    }
    int64_t c = -1;
    for (int a = 0; a < OR_MAX_BIRTH_ATTEMPTS && c < 0; a++) {
        uint64_t f[3];
        next_block(pr, t, f);
        for (int k = 0; k < 3; k++) t->p[k] = g->lo[k] + (g->hi[k] - g->lo[k]) * or_u01(f[k]);
        METER(9);
        c = find_cell_in(g, g->root, t->p);
        if (c < 0) (*rejected)++;
    }
    if (c < 0) return END_LOST;
    t->cell[0] = c;
    q[0] = t->p[0]; q[1] = t->p[1]; q[2] = t->p[2];
    int rc = descend(g, t, 0, q) ? END_LOST : END_NONE;
    sample_flight(pr, t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* tallies                                                              */
/* ------------------------------------------------------------------ */
typedef unsigned __int128 u128;

/* fixed-point quantisation of a segment length: a 128-bit integer in units
 * of 2^-96 cm (32 integer bits, 96 fraction bits), truncated.  Lengths of
 * 2^-43 cm or more are represented exactly. */
static u128 fx_of(double l) {
    double v = ldexp(l, 32);
    double fl = floor(v);
    double fr = v - fl;
    uint64_t hi = (uint64_t)fl;
    uint64_t lo = (uint64_t)ldexp(fr, 64);
    return ((u128)hi << 64) | lo;
}

static double fx_to_double(u128 v) {
    uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return (double)hi * 0x1p-32 + (double)lo * 0x1p-96;
}

typedef struct {
    double *sum, *comp;
    u128 *fx;
    /* mesh tally (when mesh is not NULL): per bin, and a buffer of cuts */
    const or_mesh *mesh;
    double *msum, *mcomp, *cuts;
    u128 *mfx;
} tally_acc;

static void neumaier_add(double *s, double *c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* ------------------------------------------------------------------ */
/* mesh tally of one segment                                            */
/* ------------------------------------------------------------------ */
static uint64_t mesh_bins(const or_mesh *m) { return (uint64_t)m->n[0] * m->n[1] * m->n[2]; }

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Track-length estimate of the segment p0 + t u, 0 <= t <= l, on the mesh.
 * Plane k of axis a (k = 0 .. n[a]) sits at lo[a] + k w[a], w[a] = (hi[a] -
 * lo[a]) / n[a]; the segment is cut at every t = (plane - p0[a]) / u[a] with
 * 0 < t < l.  Each piece [t0, t1] between consecutive cuts (and the ends)
 * adds t1 - t0 to the bin holding its midpoint p0 + ((t0 + t1) / 2) u, the
 * bin index on axis a being floor((mid[a] - lo[a]) / w[a]); pieces whose
 * midpoint is outside the mesh add nothing. */
static void mesh_segment(tally_acc *acc, const double p0[3], const double u[3], double l) {
    const or_mesh *m = acc->mesh;
    double w[3];
    for (int a = 0; a < 3; a++) w[a] = (m->hi[a] - m->lo[a]) / (double)m->n[a];
    int nc = 0;
    acc->cuts[nc++] = 0.0;
    for (int a = 0; a < 3; a++) {
        if (u[a] == 0.0) continue;
        for (uint32_t k = 0; k <= m->n[a]; k++) {
            double x = m->lo[a] + (double)k * w[a];
            double t = (x - p0[a]) / u[a];
            if (t > 0.0 && t < l) acc->cuts[nc++] = t;
        }
    }
    acc->cuts[nc++] = l;
    qsort(acc->cuts, (size_t)nc, sizeof(double), cmp_double);
    for (int i = 0; i + 1 < nc; i++) {
        double t0 = acc->cuts[i], t1 = acc->cuts[i + 1];
        double tm = (t0 + t1) * 0.5;
        uint64_t idx[3];
        int inside = 1;
        for (int a = 0; a < 3; a++) {
            double mid = p0[a] + tm * u[a];
            double f = floor((mid - m->lo[a]) / w[a]);
            if (!(f >= 0.0 && f < (double)m->n[a])) { inside = 0; break; }
            idx[a] = (uint64_t)f;
        }
        if (!inside) continue;
        uint64_t b = (idx[2] * m->n[1] + idx[1]) * m->n[0] + idx[0];
        double piece = t1 - t0;
        neumaier_add(&acc->msum[b], &acc->mcomp[b], piece);
        acc->mfx[b] += fx_of(piece);
    }
}

/* ------------------------------------------------------------------ */
/* Alg. 2 (toy transport): one history                                  */
/* ------------------------------------------------------------------ */
#define FNV_OFFSET 0xcbf29ce484222325ull
#define FNV_PRIME 0x100000001b3ull

typedef struct {
    uint32_t segs;
    uint64_t hash;
    uint8_t end;
    int rec_overflow;
} hist_result;

static void run_history(const or_geom *g, const or_params *pr, uint64_t local, tally_acc *acc,
                        int32_t *rec, or_trace *tr, hist_result *res, uint64_t *rejected) {
    ptl t;
    uint64_t h = FNV_OFFSET;
    uint32_t segs = 0;
    uint32_t ncoll = 0;
    int recovf = 0;
    int end = birth(g, pr, &t, local, rejected);
    if (tr) {
        memcpy(tr->birth_pos, t.p, sizeof t.p);
        memcpy(tr->birth_dir, t.u, sizeof t.u);
        tr->n = 0;
        tr->n_flights = 0;
        if (tr->cap) tr->flight_tau[tr->n_flights++] = t.tau;
    }
    while (end == END_NONE) {
        int bl;
        int64_t bs;
        if (tr && tr->st_state && tr->n < tr->cap) {
            uint32_t n = tr->n;
            memcpy(tr->st_pos + 3 * n, t.p, sizeof t.p);
            memcpy(tr->st_dir + 3 * n, t.u, sizeof t.u);
            int32_t *w = tr->st_state + (size_t)OR_STATE_W * n;
            for (int L = 0; L < OR_STATE_LEVELS; L++) w[L] = L < t.depth ? (int32_t)t.cell[L] : -1;
            w[OR_STATE_LEVELS] = t.on_level;
            w[OR_STATE_LEVELS + 1] = t.on_level < 0 ? -1 : (int32_t)t.on_surf;
        }
        double dist = distance_to_surface(g, &t, &bl, &bs);
        double sig = g->sigma[leaf_material(g, &t)];
        double sc = (pr->source == 1) ? INFINITY : t.tau / sig;
        METER(pr->source == 1 ? 0 : 1);
        uint64_t inst = leaf_inst(g, &t);
        int boundary = dist < sc;
        double l;
        if (boundary) {
            l = dist;
            if (pr->source != 1) { t.tau = t.tau - sig * dist; METER(2); }
        } else {
            if (sc == INFINITY) { end = END_LOST; break; }
            l = sc;
        }
        /* move_within_cell */
        const double p0[3] = { t.p[0], t.p[1], t.p[2] };
        double m0 = l * t.u[0], m1 = l * t.u[1], m2 = l * t.u[2];
        t.p[0] = t.p[0] + m0; t.p[1] = t.p[1] + m1; t.p[2] = t.p[2] + m2;
        METER(6);
        /* tally and sequence */
        if (acc) {
            neumaier_add(&acc->sum[inst], &acc->comp[inst], l);
            acc->fx[inst] += fx_of(l);
            if (acc->mesh) mesh_segment(acc, p0, t.u, l);
        }
        h = (h ^ (inst + 1)) * FNV_PRIME;
        if (rec) {
            if (segs < pr->record_cap) rec[segs] = (int32_t)inst;
            else recovf = 1;
        }
        if (tr && tr->n < tr->cap) {
            uint32_t n = tr->n++;
            tr->seg_len[n] = l; tr->seg_sigma[n] = sig; tr->seg_inst[n] = (int64_t)inst;
            tr->seg_kind[n] = (uint8_t)!boundary;
            tr->seg_pos[3 * n] = t.p[0]; tr->seg_pos[3 * n + 1] = t.p[1]; tr->seg_pos[3 * n + 2] = t.p[2];
        }
        segs++;
        if (boundary) {
            end = cross_surface(g, &t, bl, bs);
        } else {
            t.on_level = -1;
            t.on_surf = -1;
            ncoll++;
            if (ncoll >= pr->max_collisions) {
                end = END_CAP;
            } else {
                sample_flight(pr, &t);
                if (tr && tr->n_flights < tr->cap) tr->flight_tau[tr->n_flights++] = t.tau;
            }
        }
        if (end == END_NONE && segs >= pr->max_segments) end = END_SEGCAP;
    }
    h ^= (uint64_t)end;
    res->segs = segs;
    res->hash = h;
    res->end = (uint8_t)end;
    res->rec_overflow = recovf;
    if (tr) tr->end_code = (uint8_t)end;
}

/* ------------------------------------------------------------------ */
/* threaded driver: static particle ranges, merged in thread order      */
/* ------------------------------------------------------------------ */
typedef struct {
    const or_geom *g;
    const or_params *pr;
    const or_out *out;
    uint64_t i0, i1;
    tally_acc acc;
    uint64_t counters[C_NC];
    int err;
} job;

static void *worker(void *arg) {
    job *j = arg;
    const or_params *pr = j->pr;
    for (uint64_t i = j->i0; i < j->i1; i++) {
        int32_t *rec = NULL;
        if (j->out->rec && i < pr->record_first_k) rec = j->out->rec + i * (uint64_t)pr->record_cap;
        hist_result r;
        run_history(j->g, pr, i, j->acc.sum ? &j->acc : NULL, rec, NULL, &r, &j->counters[C_REJECTED]);
        if (j->out->seg_count) j->out->seg_count[i] = r.segs;
        if (j->out->seq_hash) j->out->seq_hash[i] = r.hash;
        if (j->out->end_code) j->out->end_code[i] = r.end;
        j->counters[C_SEGMENTS] += r.segs;
        if (r.end == END_ESCAPE) j->counters[C_ESCAPED]++;
        if (r.end == END_CAP) j->counters[C_CAPPED]++;
        if (r.end == END_LOST) j->counters[C_LOST]++;
        if (r.end == END_SEGCAP) j->counters[C_SEGCAP]++;
        if (r.rec_overflow) j->counters[C_RECOVF]++;
    }
    return NULL;
}

int or_track(const or_geom *g, const or_params *pr, const or_out *out, int n_threads) {
    if (!g || !pr || !out) return -1;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > OR_MAX_THREADS) n_threads = OR_MAX_THREADS;
    if ((uint64_t)n_threads > pr->n_particles && pr->n_particles > 0) n_threads = (int)pr->n_particles;
    if (pr->record_first_k && out->rec) {
        uint64_t nrec = (uint64_t)pr->record_first_k * pr->record_cap;
        for (uint64_t k = 0; k < nrec; k++) out->rec[k] = -1;
    }
    int want_tally = out->tally || out->tally_fx || out->tally_fxd;
    job *jobs = calloc((size_t)n_threads, sizeof(job));
    pthread_t *th = calloc((size_t)n_threads, sizeof(pthread_t));
    uint64_t n = pr->n_particles;
    for (int k = 0; k < n_threads; k++) {
        jobs[k].g = g; jobs[k].pr = pr; jobs[k].out = out;
        jobs[k].i0 = n * (uint64_t)k / (uint64_t)n_threads;
        jobs[k].i1 = n * (uint64_t)(k + 1) / (uint64_t)n_threads;
        if (want_tally || out->mesh) {
            jobs[k].acc.sum = calloc(g->n_inst, sizeof(double));
            jobs[k].acc.comp = calloc(g->n_inst, sizeof(double));
            jobs[k].acc.fx = calloc(g->n_inst, sizeof(u128));
            if (!jobs[k].acc.sum || !jobs[k].acc.comp || !jobs[k].acc.fx) jobs[k].err = 1;
        }
        if (out->mesh) {
            const or_mesh *m = out->mesh;
            uint64_t nb = mesh_bins(m);
            jobs[k].acc.mesh = m;
            jobs[k].acc.msum = calloc(nb, sizeof(double));
            jobs[k].acc.mcomp = calloc(nb, sizeof(double));
            jobs[k].acc.mfx = calloc(nb, sizeof(u128));
            jobs[k].acc.cuts = malloc(sizeof(double) * ((size_t)m->n[0] + m->n[1] + m->n[2] + 5));
            if (!jobs[k].acc.msum || !jobs[k].acc.mcomp || !jobs[k].acc.mfx || !jobs[k].acc.cuts) jobs[k].err = 1;
        }
    }
    if (out->mesh) {
        const or_mesh *m = out->mesh;
        for (int a = 0; a < 3; a++)
            if (m->n[a] < 1 || !(m->hi[a] > m->lo[a]) || !isfinite(m->lo[a]) || !isfinite(m->hi[a])) {
                for (int k = 0; k < n_threads; k++) jobs[k].err = 1;
                break;
            }
    }
    int err = 0;
    for (int k = 0; k < n_threads; k++) err |= jobs[k].err;
    if (!err) {
        for (int k = 1; k < n_threads; k++) pthread_create(&th[k], NULL, worker, &jobs[k]);
        worker(&jobs[0]);
        for (int k = 1; k < n_threads; k++) pthread_join(th[k], NULL);
        uint64_t cnt[C_NC] = {0};
        for (int k = 0; k < n_threads; k++)
            for (int c = 0; c < C_NC; c++) cnt[c] += jobs[k].counters[c];
        if (out->counters) { memset(out->counters, 0, 8 * sizeof(uint64_t)); memcpy(out->counters, cnt, sizeof cnt); }
        if (want_tally) {
            for (uint64_t i = 0; i < g->n_inst; i++) {
                double s = 0.0, c = 0.0;
                u128 fx = 0;
                for (int k = 0; k < n_threads; k++) {
                    neumaier_add(&s, &c, jobs[k].acc.sum[i]);
                    neumaier_add(&s, &c, jobs[k].acc.comp[i]);
                    fx += jobs[k].acc.fx[i];
                }
                if (out->tally) out->tally[i] = s + c;
                if (out->tally_fx) { out->tally_fx[2 * i] = (uint64_t)fx; out->tally_fx[2 * i + 1] = (uint64_t)(fx >> 64); }
                if (out->tally_fxd) out->tally_fxd[i] = fx_to_double(fx);
            }
        }
        if (out->mesh) {
            const or_mesh *m = out->mesh;
            for (uint64_t b = 0; b < mesh_bins(m); b++) {
                double s = 0.0, c = 0.0;
                u128 fx = 0;
                for (int k = 0; k < n_threads; k++) {
                    neumaier_add(&s, &c, jobs[k].acc.msum[b]);
                    neumaier_add(&s, &c, jobs[k].acc.mcomp[b]);
                    fx += jobs[k].acc.mfx[b];
                }
                if (m->mesh) m->mesh[b] = s + c;
                if (m->mesh_fx) { m->mesh_fx[2 * b] = (uint64_t)fx; m->mesh_fx[2 * b + 1] = (uint64_t)(fx >> 64); }
                if (m->mesh_fxd) m->mesh_fxd[b] = fx_to_double(fx);
            }
        }
    }
    for (int k = 0; k < n_threads; k++) {
        free(jobs[k].acc.sum); free(jobs[k].acc.comp); free(jobs[k].acc.fx);
        free(jobs[k].acc.msum); free(jobs[k].acc.mcomp); free(jobs[k].acc.mfx); free(jobs[k].acc.cuts);
    }
    free(jobs);
    free(th);
    return err ? -3 : 0;
}

/* Work meter over particles [first, first+n) of pr: out[0] = double
 * operations the method requires (see `meter`), out[1] = segments. */
int or_count_work(const or_geom *g, const or_params *pr, uint64_t *out) {
    uint64_t ops = 0, segs = 0, rej = 0;
    meter = &ops;
    for (uint64_t i = 0; i < pr->n_particles; i++) {
        hist_result r;
        run_history(g, pr, i, NULL, NULL, NULL, &r, &rej);
        segs += r.segs;
    }
    meter = NULL;
    out[0] = ops;
    out[1] = segs;
    return 0;
}

/* one history with every segment recorded (for invariant checks) */
int or_trace_particle(const or_geom *g, const or_params *pr, uint64_t local, or_trace *tr) {
    hist_result r;
    uint64_t rej = 0;
    run_history(g, pr, local, NULL, NULL, tr, &r, &rej);
    return (int)r.segs;
}

/* births of particles [first, first+n): position, direction, tau, leaf
 * instance (-1 when lost) */
int or_sample_births(const or_geom *g, const or_params *pr, double *pos, double *dir, double *tau, int64_t *inst) {
    uint64_t rej = 0;
    for (uint64_t i = 0; i < pr->n_particles; i++) {
        ptl t;
        int rc = birth(g, pr, &t, i, &rej);
        memcpy(pos + 3 * i, t.p, sizeof t.p);
        memcpy(dir + 3 * i, t.u, sizeof t.u);
        tau[i] = t.tau;
        inst[i] = rc == END_NONE ? (int64_t)leaf_inst(g, &t) : -1;
    }
    return 0;
}

/* Table 1 find_cell over a batch of global points: leaf instance (-1 when
 * outside the root or in a gap) and the cell at every level (-1 padded). */
int or_find_cell(const or_geom *g, const double *pos, uint64_t n, int64_t *inst, int32_t *cells) {
    for (uint64_t i = 0; i < n; i++) {
        ptl t;
        memset(&t, 0, sizeof t);
        memcpy(t.p, pos + 3 * i, sizeof t.p);
        int64_t c = find_cell_in(g, g->root, t.p);
        int ok = 0;
        t.depth = 0;
        if (c >= 0) {
            double q[3] = { t.p[0], t.p[1], t.p[2] };
            t.cell[0] = c;
            ok = descend(g, &t, 0, q) == 0;
        }
        inst[i] = ok ? (int64_t)leaf_inst(g, &t) : -1;
        if (cells)
            for (int L = 0; L < OR_MAXL; L++)
                cells[i * OR_MAXL + L] = (c >= 0 && L < t.depth) ? (int32_t)t.cell[L] : -1;
    }
    return 0;
}

/* Table 1 distance_to_surface for a batch of (position, direction): the
 * particle is located with find_cell and is not on any surface. */
int or_distance_to_surface(const or_geom *g, const double *pos, const double *dir, uint64_t n,
                           double *dist, int32_t *level, int32_t *surf) {
    for (uint64_t i = 0; i < n; i++) {
        ptl t;
        memset(&t, 0, sizeof t);
        memcpy(t.p, pos + 3 * i, sizeof t.p);
        memcpy(t.u, dir + 3 * i, sizeof t.u);
        t.on_level = -1;
        t.on_surf = -1;
        int64_t c = find_cell_in(g, g->root, t.p);
        int ok = 0;
        if (c >= 0) {
            double q[3] = { t.p[0], t.p[1], t.p[2] };
            t.cell[0] = c;
            ok = descend(g, &t, 0, q) == 0;
        }
        if (!ok) { dist[i] = NAN; level[i] = -1; surf[i] = -1; continue; }
        int bl;
        int64_t bs;
        dist[i] = distance_to_surface(g, &t, &bl, &bs);
        level[i] = dist[i] == INFINITY ? -1 : bl;
        surf[i] = dist[i] == INFINITY ? -1 : (int32_t)bs;
    }
    return 0;
}

/* neighbour list of a surface (cells referencing it, ascending) */
/* Table 1 distance_to_surface from explicit tracking states (the layout of
 * or_trace.st_state): the cell of each level and the surface the particle
 * is on, as cross_surface leaves them.  A state whose cells do not form a
 * chain of fills from the root down to a material cell, or whose on-level
 * is not one of its levels, gives NaN and -1. */
int or_distance_to_surface_state(const or_geom *g, const double *pos, const double *dir, const int32_t *state,
                                 uint64_t n, double *dist, int32_t *level, int32_t *surf) {
    for (uint64_t i = 0; i < n; i++) {
        const int32_t *w = state + (size_t)OR_STATE_W * i;
        ptl t;
        memset(&t, 0, sizeof t);
        memcpy(t.p, pos + 3 * i, sizeof t.p);
        memcpy(t.u, dir + 3 * i, sizeof t.u);
        int ok = 1;
        uint32_t u = g->root;
        t.depth = 0;
        for (int L = 0; L < OR_STATE_LEVELS && ok; L++) {
            int32_t c = w[L];
            if (c < 0) break;
            if ((uint32_t)c >= g->nc || g->cell_univ[c] != u) { ok = 0; break; }
            t.cell[L] = c;
            t.depth = L + 1;
            if (g->fill[c] >= 0) break;
            u = (uint32_t)(-g->fill[c] - 1);
        }
        if (t.depth == 0 || g->fill[t.cell[t.depth - 1]] < 0) ok = 0;
        for (int L = t.depth; ok && L < OR_STATE_LEVELS; L++)
            if (w[L] != -1) ok = 0;
        t.on_level = w[OR_STATE_LEVELS];
        t.on_surf = w[OR_STATE_LEVELS + 1];
        if (t.on_level < -1 || t.on_level >= t.depth) ok = 0;
        if (t.on_level < 0) t.on_surf = -1;
        if (!ok) { dist[i] = NAN; level[i] = -1; surf[i] = -1; continue; }
        int bl;
        int64_t bs;
        dist[i] = distance_to_surface(g, &t, &bl, &bs);
        level[i] = dist[i] == INFINITY ? -1 : bl;
        surf[i] = dist[i] == INFINITY ? -1 : (int32_t)bs;
    }
    return 0;
}

int or_neighbours(const or_geom *g, uint32_t s, uint32_t *out, uint32_t cap) {
    uint32_t n = g->nb_off[s + 1] - g->nb_off[s];
    for (uint32_t k = 0; k < n && k < cap; k++) out[k] = g->nb[g->nb_off[s] + k];
    return (int)n;
}

void or_fx_quantise(const double *l, uint64_t n, uint64_t *lohi) {
    for (uint64_t i = 0; i < n; i++) {
        u128 v = fx_of(l[i]);
        lohi[2 * i] = (uint64_t)v;
        lohi[2 * i + 1] = (uint64_t)(v >> 64);
    }
}

/* Test entry: the superimposed mesh tally of n_seg given segments, segment
 * i running from p0[3i..3i+2] along the unit direction u[3i..3i+2] for the
 * length l[i], each added as a tracking segment is (mesh_segment above).
 * Outputs as or_track's mesh outputs; -1 for an invalid mesh. */
int or_mesh_segments(const or_mesh *m, uint64_t n_seg, const double *p0, const double *u, const double *l) {
    for (int a = 0; a < 3; a++)
        if (m->n[a] < 1 || !(m->hi[a] > m->lo[a]) || !isfinite(m->lo[a]) || !isfinite(m->hi[a])) return -1;
    uint64_t nb = mesh_bins(m);
    tally_acc acc;
    memset(&acc, 0, sizeof acc);
    acc.mesh = m;
    acc.msum = calloc(nb, sizeof(double));
    acc.mcomp = calloc(nb, sizeof(double));
    acc.mfx = calloc(nb, sizeof(u128));
    acc.cuts = malloc(sizeof(double) * ((size_t)m->n[0] + m->n[1] + m->n[2] + 5));
    int rc = 0;
    if (!acc.msum || !acc.mcomp || !acc.mfx || !acc.cuts) rc = -2;
    for (uint64_t i = 0; !rc && i < n_seg; i++) mesh_segment(&acc, p0 + 3 * i, u + 3 * i, l[i]);
    for (uint64_t b = 0; !rc && b < nb; b++) {
        if (m->mesh) m->mesh[b] = acc.msum[b] + acc.mcomp[b];
        if (m->mesh_fx) { m->mesh_fx[2 * b] = (uint64_t)acc.mfx[b]; m->mesh_fx[2 * b + 1] = (uint64_t)(acc.mfx[b] >> 64); }
        if (m->mesh_fxd) m->mesh_fxd[b] = fx_to_double(acc.mfx[b]);
    }
    free(acc.msum); free(acc.mcomp); free(acc.mfx); free(acc.cuts);
    return rc;
}
