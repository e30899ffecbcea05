"""Pin for the oracle's whole history loop: a second tracker, written here in
plain Python straight from the definitions (surface functions and senses of
the Introduction's CSG construction, distance_to_surface / cross_surface /
find_cell of Table 1, the multi-level rules of Alg. 7/8, the toy transport
of Alg. 2), with none of the oracle's search structure: every find_cell and
every crossing scans all cells of the universe, every distance is taken
over every half-space of every level.  Only the random stream and the
logarithm -- pinned on their own (published Philox vectors; 2 ulp of libm)
-- are taken from the oracle, because their bits define the histories.

Per history it must give the oracle's segment count, sequence hash, end
code and recorded sequence; per instance the exact fixed-point tally."""

import math
from fractions import Fraction

import pytest

import oracle
from paper_2406_13849_amd import synth

PX, PY, PZ, P, CZ, SPH = 0, 1, 2, 3, 4, 5
ESCAPE, CAP, LOST, SEGCAP = 1, 2, 3, 4
FNV_OFFSET, FNV_PRIME, M64 = 0xcbf29ce484222325, 0x100000001b3, (1 << 64) - 1
INF = math.inf


class Geo:
    def __init__(self, fg):
        self.fg = fg
        self.type = [int(t) for t in fg.surf_type]
        self.coef = [[float(v) for v in row] for row in fg.surf_coef]
        off = [int(v) for v in fg.cell_hs_off]
        self.cell_hs = [[int(h) for h in fg.hs[off[c]:off[c + 1]]] for c in range(fg.n_cells)]
        self.fill = [int(v) for v in fg.cell_fill]
        self.trans = [tuple(float(v) for v in row) for row in fg.cell_trans]
        uo = [int(v) for v in fg.univ_cell_off]
        self.univ_cells = [list(range(uo[u], uo[u + 1])) for u in range(len(uo) - 1)]
        self.root = int(fg.root)
        self.lo = [float(v) for v in fg.domain_lo]
        self.hi = [float(v) for v in fg.domain_hi]
        self.sigma = [float(v) for v in fg.sigma_t]
        # leaf instances: n_inst(U) = sum over U's cells of 1 (material) or n_inst(daughter)
        memo = {}

        def n_inst(u):
            if u not in memo:
                memo[u] = sum(1 if self.fill[c] >= 0 else n_inst(-self.fill[c] - 1) for c in self.univ_cells[u])
            return memo[u]
        self.inst_off = {}
        for u, cells in enumerate(self.univ_cells):
            acc = 0
            for c in cells:
                self.inst_off[c] = acc
                acc += 1 if self.fill[c] >= 0 else n_inst(-self.fill[c] - 1)

    def f(self, s, x, y, z):
        t, c = self.type[s], self.coef[s]
        if t == PX:
            return x - c[0]
        if t == PY:
            return y - c[0]
        if t == PZ:
            return z - c[0]
        if t == P:
            return ((c[0] * x + c[1] * y) + c[2] * z) - c[3]
        dx, dy = x - c[0], y - c[1]
        if t == CZ:
            return (dx * dx + dy * dy) - c[2]
        dz = z - c[2]
        return ((dx * dx + dy * dy) + dz * dz) - c[3]

    def contains(self, cell, q, force=None):
        """Every half-space on its required side; on the surface `force`
        = (s, sense) the given sense instead of the numeric one."""
        for h in self.cell_hs[cell]:
            s, want = abs(h) - 1, h > 0
            sense = force[1] if (force is not None and s == force[0]) else self.f(s, *q) > 0.0
            if sense != want:
                return False
        return True

    def find(self, u, q, force=None, exclude=None):
        hits = [c for c in self.univ_cells[u] if c != exclude and self.contains(c, q, force)]
        assert len(hits) <= 1, "cells overlap"
        return hits[0] if hits else None

    def descend(self, cells, q):
        """Append the cells below cells[-1] (numeric senses); False if a
        daughter universe has no cell there."""
        while self.fill[cells[-1]] < 0:
            t = self.trans[cells[-1]]
            q = (q[0] - t[0], q[1] - t[1], q[2] - t[2])
            c = self.find(-self.fill[cells[-1]] - 1, q)
            if c is None:
                return False
            cells.append(c)
        return True

    def local(self, cells, p, L):
        q = p
        for M in range(L):
            t = self.trans[cells[M]]
            q = (q[0] - t[0], q[1] - t[1], q[2] - t[2])
        return q

    def dist(self, s, want_pos, q, d, on):
        t, c = self.type[s], self.coef[s]
        u, v, w = d
        if t <= P:
            if on:
                return INF
            den = {PX: u, PY: v, PZ: w}.get(t)
            if den is None:
                den = (c[0] * u + c[1] * v) + c[2] * w
            if den == 0.0 or not ((not want_pos and den > 0.0) or (want_pos and den < 0.0)):
                return INF
            r = (-self.f(s, *q)) / den
            return r if r > 0.0 else 0.0
        dx, dy = q[0] - c[0], q[1] - c[1]
        if t == CZ:
            a = u * u + v * v
            b = dx * u + dy * v
        else:
            dz = q[2] - c[2]
            a = (u * u + v * v) + w * w
            b = (dx * u + dy * v) + dz * w
        if a == 0.0:
            return INF
        if on:
            if not want_pos and b < 0.0:
                r = (-2.0 * b) / a
                return r if r > 0.0 else 0.0
            return INF
        cc = self.f(s, *q)
        disc = b * b - a * cc
        if not disc > 0.0:
            return INF
        qq = math.sqrt(disc)
        if not want_pos:
            r = (qq - b) / a if b <= 0.0 else (-cc) / (b + qq)
        else:
            if not b < 0.0:
                return INF
            r = cc / (qq - b)
        return r if r > 0.0 else 0.0

    def nearest(self, cells, p, d, on_level, on_surf):
        best = (INF, None, None, None)
        for L, cell in enumerate(cells):
            q = self.local(cells, p, L)
            for h in self.cell_hs[cell]:
                s = abs(h) - 1
                r = self.dist(s, h > 0, q, d, on_level == L and on_surf == s)
                if r < INF and (r, L, s) < best[:3]:
                    best = (r, L, s, h > 0)
        return best


def fields(seed, gid, pid, blk):
    o = [int(v) for v in oracle.philox4x32_10([blk, pid & 0xFFFFFFFF, pid >> 32, gid],
                                              [seed & 0xFFFFFFFF, seed >> 32])]
    w0, w1 = o[0] | (o[1] << 32), o[2] | (o[3] << 32)
    m42 = (1 << 42) - 1
    f = (w0 & m42, (w0 >> 42) | ((w1 & ((1 << 20) - 1)) << 22), (w1 >> 20) & m42)
    return [(float(x) + 0.5) * 2.0 ** -42 for x in f]


def history(g, seed, gid, pid, max_coll=20, max_segs=100_000):
    """One history; returns (segments, hash, end, sequence, [(inst, length)])."""
    blk = 0
    cells = None
    for _ in range(1000):
        u0, u1, u2 = fields(seed, gid, pid, blk)
        blk += 1
        p = tuple(g.lo[k] + (g.hi[k] - g.lo[k]) * (u0, u1, u2)[k] for k in range(3))
        c = g.find(g.root, p)
        if c is not None:
            cells = [c]
            break
    seq, contrib = [], []
    if cells is None or not g.descend(cells, g.local([], p, 0)):
        return 0, FNV_OFFSET ^ LOST, LOST, seq, contrib

    def new_direction(blk):
        while True:
            a, b, c = fields(seed, gid, pid, blk)
            blk += 1
            v1, v2 = 2.0 * a - 1.0, 2.0 * b - 1.0
            s = v1 * v1 + v2 * v2
            if s < 1.0 and s != 0.0:
                r = math.sqrt(1.0 - s)
                return ((2.0 * v1) * r, (2.0 * v2) * r, 1.0 - 2.0 * s), -float(oracle.mc_log([c])[0]), blk
    d, tau, blk = new_direction(blk)
    h, segs, ncoll, end = FNV_OFFSET, 0, 0, 0
    on_level, on_surf = -1, None
    while end == 0:
        t, L, s, spos = g.nearest(cells, p, d, on_level, on_surf)
        sig = g.sigma[g.fill[cells[-1]]]
        sc = tau / sig
        boundary = t < sc
        if not boundary and sc == INF:
            end = LOST
            break
        if boundary:
            ln = t
            tau = tau - sig * t
        else:
            ln = sc
        p = (p[0] + ln * d[0], p[1] + ln * d[1], p[2] + ln * d[2])
        inst = sum(g.inst_off[c] for c in cells)
        contrib.append((inst, ln))
        seq.append(inst)
        h = ((h ^ (inst + 1)) * FNV_PRIME) & M64
        segs += 1
        if boundary:
            q = g.local(cells, p, L)
            c = g.find(g.univ_of(L, cells), q, force=(s, not spos), exclude=cells[L])
            if c is None:
                end = ESCAPE if L == 0 else LOST
            else:
                cells = cells[:L] + [c]
                if not g.descend(cells, q):
                    end = LOST
                on_level, on_surf = L, s
        else:
            on_level, on_surf = -1, None
            ncoll += 1
            if ncoll >= max_coll:
                end = CAP
            else:
                d, tau, blk = new_direction(blk)
        if end == 0 and segs >= max_segs:
            end = SEGCAP
    return segs, h ^ end, end, seq, contrib


def _univ_of(self, L, cells):
    return self.root if L == 0 else -self.fill[cells[L - 1]] - 1


Geo.univ_of = _univ_of


def _geometry(name):
    if name.startswith("cfg"):
        i = int(name[3:])
        return synth.make_config(i), synth.particle_seed(i), i
    return getattr(synth, name)(), 4321, 17


def fx(l):
    return math.floor(Fraction(l) * (1 << 96))


@pytest.mark.parametrize("name,n,kw", [
    ("cfg1", 400, {}),
    ("sphere", 300, dict(max_collisions=3)),
    ("box", 200, {}),
    ("cfg2", 60, {}),
    ("cfg3", 12, {}),
    ("cfg4", 12, {}),
    ("hex_pin_box", 40, {}),
    ("nested_box", 200, {}),
])
def test_bruteforce_tracker_matches_oracle(name, n, kw):
    fg, seed, gid = _geometry(name)
    g = Geo(fg)
    og = oracle.OracleGeometry(fg)
    max_coll = kw.get("max_collisions", 20)
    o = oracle.track(og, oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid, record_first_k=n,
                                            record_cap=4096, max_collisions=max_coll), n_threads=1)
    tal = {}
    for i in range(n):
        segs, h, end, seq, contrib = history(g, seed, gid, i, max_coll=max_coll)
        assert (segs, h, end) == (int(o.seg_count[i]), int(o.seq_hash[i]), int(o.end_code[i])), (name, i)
        rec = o.rec[i][o.rec[i] >= 0]
        assert seq == [int(v) for v in rec], (name, i)
        for inst, ln in contrib:
            tal[inst] = tal.get(inst, 0) + fx(ln)
    want = {int(k): (int(o.tally_fx[k][1]) << 64) | int(o.tally_fx[k][0]) for k in range(o.tally_fx.shape[0])
            if o.tally_fx[k].any()}
    assert {k: v for k, v in tal.items() if v} == want


def _states(og, seed, gid, n):
    """Tracking states at the start of every segment of n histories (many of
    them just after a crossing, so on a surface)."""
    pos, dirs, st, lens, kinds = [], [], [], [], []
    for i in range(n):
        t = oracle.trace_particle(og, oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid), i,
                                  cap=5000, states=True)
        pos.append(t.st_pos)
        dirs.append(t.st_dir)
        st.append(t.st_state)
        lens.append(t.seg_len)
        kinds.append(t.seg_kind)
    import numpy as np
    return (np.concatenate(pos), np.concatenate(dirs), np.concatenate(st), np.concatenate(lens),
            np.concatenate(kinds))


@pytest.mark.parametrize("name,n", [("cfg1", 60), ("cfg2", 12), ("cfg3", 4), ("cfg4", 4), ("sphere", 60),
                                    ("hex_pin_box", 10), ("nested_box", 60)])
def test_distance_from_tracking_states_matches_bruteforce(name, n):
    """distance_to_surface from explicit states (the cell of each level and
    the surface the particle is on, as a crossing leaves them): the oracle's
    distance, level and surface equal the brute-force minimum over every
    half-space of every level, and for a boundary segment the distance is
    the traced segment length."""
    import numpy as np
    fg, seed, gid = _geometry(name)
    g = Geo(fg)
    og = oracle.OracleGeometry(fg)
    pos, dirs, st, lens, kinds = _states(og, seed, gid, n)
    d, lev, srf = og.distance_to_surface_state(pos, dirs, st)
    W = oracle.STATE_LEVELS
    on = 0
    for i in range(pos.shape[0]):
        cells = [int(c) for c in st[i, :W] if c >= 0]
        ol, os_ = int(st[i, W]), int(st[i, W + 1])
        on += ol >= 0
        r, L, s, _ = g.nearest(cells, tuple(pos[i]), tuple(dirs[i]), ol, os_)
        assert (d[i], lev[i], srf[i]) == (r, -1 if L is None else L, -1 if s is None else s), (name, i)
    assert np.array_equal(d[kinds == 0], lens[kinds == 0])
    assert np.all(d[kinds == 1] >= lens[kinds == 1])
    if name not in ("sphere", "nested_box"):   # (their crossings leave the geometry)
        assert on > pos.shape[0] // 2


def test_distance_from_invalid_states():
    """States that are not a chain of fills from the root to a material
    cell, or whose on-level is not one of their levels, give NaN and -1."""
    import numpy as np
    fg, seed, gid = _geometry("cfg2")
    og = oracle.OracleGeometry(fg)
    pos, dirs, st, _, _ = _states(og, seed, gid, 1)
    good = st[0].copy()
    W = oracle.STATE_LEVELS
    bad = []
    s = good.copy(); s[1] = -1; bad.append(s)                  # stops at a filled cell
    s = good.copy(); s[0] = fg.n_cells; bad.append(s)          # no such cell
    s = good.copy(); s[1] = good[0]; bad.append(s)             # level 1 not in the daughter universe
    s = good.copy(); s[2] = good[1]; bad.append(s)             # a cell below the leaf
    s = good.copy(); s[W] = 2; bad.append(s)                   # on a level below the leaf
    s = good.copy(); s[W] = -2; bad.append(s)
    states = np.stack([good] + bad)
    d, lev, srf = og.distance_to_surface_state(np.repeat(pos[:1], len(states), 0),
                                               np.repeat(dirs[:1], len(states), 0), states)
    assert not np.isnan(d[0])
    assert np.all(np.isnan(d[1:])) and np.all(lev[1:] == -1) and np.all(srf[1:] == -1)


class _NoForcedSense(Geo):
    def find(self, u, q, force=None, exclude=None):
        return super().find(u, q, None, exclude)


class _TranslationAdded(Geo):
    def local(self, cells, p, L):
        q = p
        for M in range(L):
            t = self.trans[cells[M]]
            q = (q[0] + t[0], q[1] + t[1], q[2] + t[2])
        return q


class _OnSurfaceIgnored(Geo):
    def dist(self, s, want_pos, q, d, on):
        return super().dist(s, want_pos, q, d, False)


class _SphereDzDropped(Geo):
    def dist(self, s, want_pos, q, d, on):
        if self.type[s] == SPH:
            d = (d[0], d[1], 0.0 * d[2])
        return super().dist(s, want_pos, q, d, on)


class _BottomLevelFirst(Geo):
    def nearest(self, cells, p, d, on_level, on_surf):
        best = (INF, None, None, None)
        for L, cell in enumerate(cells):
            q = self.local(cells, p, L)
            for h in self.cell_hs[cell]:
                s = abs(h) - 1
                r = self.dist(s, h > 0, q, d, on_level == L and on_surf == s)
                if r < INF and (best[1] is None or r < best[0] or (r == best[0] and L > best[1])):
                    best = (r, L, s, h > 0)
        return best


def _mismatches(geo_cls, name, n):
    fg, seed, gid = _geometry(name)
    o = oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid),
                     n_threads=1)
    g = geo_cls(fg)
    bad, tal = 0, {}
    for k in range(n):
        try:
            segs, h, end, _, contrib = history(g, seed, gid, k)
        except AssertionError:   # a planted mistake may make cells overlap
            bad += 1
            continue
        bad += (segs, h, end) != (int(o.seg_count[k]), int(o.seq_hash[k]), int(o.end_code[k]))
        for inst, ln in contrib:
            tal[inst] = tal.get(inst, 0) + fx(ln)
    want = {int(k): (int(o.tally_fx[k][1]) << 64) | int(o.tally_fx[k][0]) for k in range(o.tally_fx.shape[0])
            if o.tally_fx[k].any()}
    return bad + ({k: v for k, v in tal.items() if v} != want)


@pytest.mark.parametrize("geo_cls,name,n", [
    (_NoForcedSense, "cfg2", 30),
    (_TranslationAdded, "cfg2", 30),
    (_OnSurfaceIgnored, "cfg1", 200),
    (_SphereDzDropped, "sphere", 100),
    (_BottomLevelFirst, "nested_box", 50),
])
def test_comparison_detects_planted_mistakes(geo_cls, name, n):
    """The comparison above has teeth: each plausible slip (a crossing decided
    by the numeric sense, a translation's sign, the on-surface rule of a
    quadric, a dropped term, the tie order between levels) put into the
    brute-force tracker makes some history disagree with the oracle."""
    assert _mismatches(geo_cls, name, n) > 0


def test_shared_surface_rejected_with_both_universes_named():
    fg = synth.nested_box()
    fg.hs = fg.hs.copy()
    fg.hs[-2:] = [1, -2]      # the daughter cell reuses the box's own x-planes
    with pytest.raises(ValueError, match="surface 0 used by universes 0 and 1"):
        oracle.OracleGeometry(fg)
