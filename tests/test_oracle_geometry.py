"""Pins for the oracle's geometry operations (Table 1 find_cell and
distance_to_surface; the neighbour lists of Alg. 4).  Expected values come
from closed forms and from the lattices' analytic structure (index
arithmetic, radii), never from re-evaluating the CSG half-spaces."""

import math

import numpy as np
import pytest

import oracle
from paper_2406_13849_amd import synth

EPS = np.finfo(float).eps


# ---------------------------------------------------------------- distances
def test_sphere_from_centre_and_chords():
    og = oracle.OracleGeometry(synth.sphere(2.0))
    rng = np.random.default_rng(1)
    d = rng.normal(size=(1000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    t, lev, s = og.distance_to_surface(np.zeros((1000, 3)), d)
    assert np.all(lev == 0) and np.all(s == 0)
    assert np.max(np.abs(t - 2.0)) <= 8 * EPS
    # chord from an interior point: t solves |p + t u| = R
    p = rng.uniform(-1, 1, size=(1000, 3)) * 0.5
    t, _, _ = og.distance_to_surface(p, d)
    bb = (p * d).sum(1)
    exact = -bb + np.sqrt(bb * bb - ((p * p).sum(1) - 4.0))
    assert np.max(np.abs(t - exact)) <= 1e-14 * 2.0


def test_box_planes_closed_form():
    og = oracle.OracleGeometry(synth.box((1.0, 2.0, 3.0)))
    th = np.linspace(-1.2, 1.2, 25)
    d = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], 1)
    t, lev, s = og.distance_to_surface(np.zeros((th.size, 3)), d)
    want = np.minimum(1.0 / np.abs(np.cos(th)), 2.0 / np.abs(np.sin(th) + 1e-300))
    assert np.allclose(t, want, rtol=4 * EPS, atol=0)
    # surface ids: PX+ is surface 1, PY+ is 3, PY- is 2
    hit_x = 1.0 / np.abs(np.cos(th)) < 2.0 / np.abs(np.sin(th) + 1e-300)
    assert np.all(s[hit_x] == 1)
    assert np.all(s[~hit_x & (th > 0)] == 3) and np.all(s[~hit_x & (th < 0)] == 2)
    # axis-parallel flight along -z from the centre
    t, _, s = og.distance_to_surface(np.zeros((1, 3)), np.array([[0.0, 0.0, -1.0]]))
    assert t[0] == 3.0 and s[0] == 4


def test_pin_cylinders_from_pin_centre():
    """cfg1's central pin: along +x from its centre the fuel cylinder is hit
    at exactly r = 0.4; from inside the clad ring the next surface is r=0.5."""
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    t, lev, s = og.distance_to_surface(np.array([[0.0, 0.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    assert lev[0] == 1 and abs(t[0] - 0.4) <= 2 * np.spacing(0.4)
    # from x=0.47 (clad) along +x -> r=0.5 at distance 0.03
    t, lev, s = og.distance_to_surface(np.array([[0.47, 0.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    assert lev[0] == 1 and abs(t[0] - 0.03) <= 1e-15
    # from the moderator towards the pin: outside root of r=0.5, from x=0.6 along -x
    t, lev, s = og.distance_to_surface(np.array([[0.6, 0.0, 0.0]]), np.array([[-1.0, 0.0, 0.0]]))
    assert abs(t[0] - 0.1) <= 1e-15
    # moving away from the pin in the moderator: next hit is the lattice plane x=0.625
    t, lev, s = og.distance_to_surface(np.array([[0.55, 0.0, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    assert lev[0] == 0 and abs(t[0] - 0.075) <= 1e-15


def test_tangent_ray_does_not_hit():
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    # line y = 0.5 grazes the r=0.5 cylinder of the central pin: no sense flip
    t, lev, s = og.distance_to_surface(np.array([[-0.6, 0.5, 0.0]]), np.array([[1.0, 0.0, 0.0]]))
    assert lev[0] == 0  # the next surface is a lattice plane, not the tangent cylinder
    assert abs(t[0] - 1.225) <= 1e-15


def test_roots_land_on_surface_and_flip_sense():
    """Random rays in cfg1: the point at the returned distance lies on the
    returned surface (|f| tiny) and the cell found just past it differs."""
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    rng = np.random.default_rng(3)
    p = rng.uniform(-1.8, 1.8, size=(4000, 3))
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    t, lev, s = og.distance_to_surface(p, d)
    inst0, _ = og.find_cell(p)
    q = p + t[:, None] * d
    for i in range(4000):
        st, c = g.surf_type[s[i]], g.surf_coef[s[i]]
        x = q[i].copy()
        if lev[i] == 1:  # pin level: local coordinates relative to the pin centre
            _, cells = og.find_cell(p[i:i + 1])
            x -= g.cell_trans[cells[0, 0]]
        if st == synth.CZ:
            f = (x[0] - c[0]) ** 2 + (x[1] - c[1]) ** 2 - c[2]
            assert abs(f) < 1e-12
        else:
            assert abs(x[st] - c[0]) < 1e-12
    past = p + (t + 1e-9)[:, None] * d
    before = p + (t - 1e-9)[:, None] * d
    ia, _ = og.find_cell(past)
    ib, _ = og.find_cell(before)
    ok = t > 2e-9
    assert np.all(ib[ok] == inst0[ok])
    assert np.all(ia[ok] != inst0[ok])


# ---------------------------------------------------------------- find_cell
def _cfg2_expected(g, pts):
    """Leaf instance of cfg2 points from lattice arithmetic: pin (i,j),
    radial zone from the radius, axial slab from z."""
    pitch, h = 1.25, 10.625
    zpl = np.array([-100 + k * 200 / 11 for k in range(1, 11)])
    radii = np.array([0.40, 0.45, 0.50])
    out = np.full(len(pts), -1, np.int64)
    ambiguous = np.zeros(len(pts), bool)
    for n, (x, y, z) in enumerate(pts):
        if not (-h < x < h and -h < y < h and -100 < z < 100):
            continue
        i = int(math.floor((x + h) / pitch))
        j = int(math.floor((y + h) / pitch))
        cx, cy = -h + (i + 0.5) * pitch, -h + (j + 0.5) * pitch
        r = math.hypot(x - cx, y - cy)
        zone = int(np.searchsorted(radii, r))
        slab = int(np.searchsorted(zpl, z))
        edge_d = min(abs((x + h) / pitch - round((x + h) / pitch)), abs((y + h) / pitch - round((y + h) / pitch)))
        if edge_d < 1e-9 or np.min(np.abs(radii - r)) < 1e-9 or np.min(np.abs(zpl - z)) < 1e-9:
            ambiguous[n] = True
        out[n] = (j * 17 + i) * 44 + slab * 4 + zone
    return out, ambiguous


def test_find_cell_cfg2_matches_lattice_arithmetic():
    g = synth.make_config(2)
    og = oracle.OracleGeometry(g)
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform([-11, -11, -101], [11, 11, 101], size=(20000, 3)),
                          rng.uniform([-10.6, -10.6, -99], [10.6, 10.6, 99], size=(20000, 3))])
    inst, cells = og.find_cell(pts)
    want, amb = _cfg2_expected(g, pts)
    assert np.all(inst[~amb] == want[~amb])
    assert (want == -1).sum() > 100  # some points outside the domain
    # the root cell found is the one whose fill is recorded for that lattice slot
    inside = want >= 0
    assert np.all(cells[inside, 0] == (want[inside] // 44))


def test_find_cell_cfg3_three_levels():
    g = synth.make_config(3)
    og = oracle.OracleGeometry(g)
    rng = np.random.default_rng(5)
    pts = rng.uniform([-145, -145, -99], [145, 145, 99], size=(20000, 3))
    inst, cells = og.find_cell(pts)
    zpl = np.array([-100 + k * 200 / 11 for k in range(1, 11)])
    radii = np.array([0.40, 0.45, 0.50])
    n_pin, n_asm_inst = 44, 289 * 44
    checked = 0
    for n, (x, y, z) in enumerate(pts):
        rr = math.hypot(x, y)
        if abs(rr - 140) < 1e-9:
            continue
        if rr > 140:
            assert inst[n] == -1
            continue
        I = int(math.floor((x + 159.375) / 21.25))
        J = int(math.floor((y + 159.375) / 21.25))
        ax, ay = x - (-159.375 + (I + 0.5) * 21.25), y - (-159.375 + (J + 0.5) * 21.25)
        i = min(max(int(math.floor((ax + 10.625) / 1.25)), 0), 16)
        j = min(max(int(math.floor((ay + 10.625) / 1.25)), 0), 16)
        px, py = ax - (-10.625 + (i + 0.5) * 1.25), ay - (-10.625 + (j + 0.5) * 1.25)
        r = math.hypot(px, py)
        if np.min(np.abs(radii - r)) < 1e-9 or np.min(np.abs(zpl - z)) < 1e-9:
            continue
        zone = int(np.searchsorted(radii, r))
        slab = int(np.searchsorted(zpl, z))
        want = (J * 15 + I) * n_asm_inst + (j * 17 + i) * n_pin + slab * 4 + zone
        assert inst[n] == want, (n, x, y, z)
        assert cells[n, 0] == 0 and cells[n, 1] == 1 + J * 15 + I
        checked += 1
    assert checked > 10000
    assert og.n_instances == 225 * 289 * 44 and og.max_depth == 4


def test_every_point_in_at_most_one_cell_per_universe():
    """Brute force over every cell of every universe at random local points:
    the cells of a universe never overlap (the uniqueness that makes any
    search order give the same find_cell result).  Uses per-universe
    single-point geometries built from the same arrays."""
    g = synth.make_config(2)
    rng = np.random.default_rng(6)
    pts = rng.uniform([-11, -11, -101], [11, 11, 101], size=(3000, 3))
    for u in range(g.n_universes):
        cells = list(g.universe_cells(u))
        counts = np.zeros(len(pts), int)
        for c in cells:
            ok = np.ones(len(pts), bool)
            for h in g.cell_halfspaces(c):
                s = abs(int(h)) - 1
                st, cf = g.surf_type[s], g.surf_coef[s]
                if st <= 2:
                    f = pts[:, st] - cf[0]
                else:
                    f = (pts[:, 0] - cf[0]) ** 2 + (pts[:, 1] - cf[1]) ** 2 - cf[2]
                ok &= (f > 0) == (h > 0)
            counts += ok
        assert counts.max() <= 1


# ---------------------------------------------------------------- neighbours
@pytest.mark.parametrize("cfg,n", [(1, 3), (2, 17)])
def test_pseudo_array_plane_neighbour_counts(cfg, n):
    """An unbounded plane of an n x n pseudo-array bounds a whole row of
    cells on each side: an interior plane lists 2n cells, an outer one n
    (the blow-up illustrated in the paper's neighbour-list figure)."""
    g = synth.make_config(cfg)
    og = oracle.OracleGeometry(g)
    counts = {}
    for s in range(g.n_surfaces):
        if g.surf_type[s] in (synth.PX, synth.PY):
            counts[s] = len(og.neighbours(s))
    vals = sorted(counts.values())
    assert vals.count(n) == 4 and vals.count(2 * n) == 2 * (n - 1)
    # pin cylinders: each bounds the two radial zones of every axial slab
    for s in range(g.n_surfaces):
        if g.surf_type[s] == synth.CZ:
            nb = og.neighbours(s)
            assert len(nb) == 2 * (11 if cfg == 2 else 1)
            assert np.all(np.diff(nb) > 0)


# ---------------------------------------------------------------- hexagonal pseudo-arrays
def _hex_round(fi, fj):
    """Nearest hexagonal lattice point of fractional axial coordinates
    (cube-coordinate rounding)."""
    x, z = fi, fj
    y = -x - z
    rx, ry, rz = round(x), round(y), round(z)
    dx, dy, dz = abs(rx - x), abs(ry - y), abs(rz - z)
    if dx > dy and dx > dz:
        rx = -ry - rz
    elif dy > dz:
        ry = -rx - rz
    else:
        rz = -rx - ry
    return int(rx), int(rz)


def test_hex_ring_counts():
    """n rings hold 3 n (n - 1) + 1 cells: 9 rings = 217 pins, 7 rings = 127
    assemblies (the Empire assemblies' 217 pins)."""
    assert len(synth.hex_ring_cells(9)) == 217
    assert len(synth.hex_ring_cells(7)) == 127
    g = synth.make_config(4)
    assert g.univ_cell_off[1] - g.univ_cell_off[0] == 127
    assert g.univ_cell_off[2] - g.univ_cell_off[1] == len(synth.hex_ring_cells(11))


def test_find_cell_hex_matches_axial_rounding():
    """cfg4: the assembly and the pin found for a point are the nearest
    lattice points in the core's and the assembly's axial coordinates; the
    radial zone follows from the distance to the pin centre."""
    g = synth.make_config(4)
    og = oracle.OracleGeometry(g)
    rng = np.random.default_rng(9)
    pts = rng.uniform(g.domain_lo, g.domain_hi, size=(20000, 3))
    inst, cells = og.find_cell(pts)
    p = synth.HEX_PIN_PITCH
    F = 2.0 * (8 * p * math.sqrt(3) / 2.0 + p / math.sqrt(3)) + 2 * synth.HEX_GAP
    core = synth.hex_ring_cells(7)
    pins = synth.hex_ring_cells(9)
    rim = synth.hex_ring_cells(11)
    checked = 0
    for n, (x, y, z) in enumerate(pts):
        # core: a1 = F (1, 0), a2 = F (1/2, sqrt3/2)
        fj = y / (F * math.sqrt(3) / 2)
        fi = x / F - fj / 2
        I, J = _hex_round(fi, fj)
        if (I, J) not in core:
            continue
        cx, cy = F * (I + J / 2), F * J * math.sqrt(3) / 2
        lx, ly = x - cx, y - cy
        # distance to the assembly hexagon's edges (pointy-top: normals at 0, 60, 120 deg)
        edge = min(F / 2 - abs(lx * math.cos(a) + ly * math.sin(a)) for a in (0, math.pi / 3, 2 * math.pi / 3))
        # pins: a1 = p (cos30, sin30), a2 = p (0, 1)
        fi2 = lx / (p * math.sqrt(3) / 2)
        fj2 = ly / p - fi2 / 2
        i, j = _hex_round(fi2, fj2)
        px, py = p * i * math.sqrt(3) / 2, p * (i / 2 + j)
        r = math.hypot(lx - px, ly - py)
        pedge = min(p / 2 - abs((lx - px) * math.cos(a) + (ly - py) * math.sin(a))
                    for a in (math.pi / 6, math.pi / 2, 5 * math.pi / 6))
        if edge < 1e-7 or pedge < 1e-7 or min(abs(r - 0.4), abs(r - 0.5)) < 1e-7:
            continue
        assert cells[n, 0] == core.index((I, J)), n
        k = rim.index((i, j))
        assert cells[n, 1] == g.univ_cell_off[1 + (g.cell_fill[cells[n, 0]] * -1 - 2)] + k, n
        if (i, j) in pins:
            assert cells[n, 2] - g.univ_cell_off[g.cell_fill[cells[n, 1]] * -1 - 1] == (0 if r < 0.4 else (1 if r < 0.5 else 2))
        checked += 1
    assert checked > 10000


def test_hex_cells_never_overlap():
    g = synth.make_config(4)
    rng = np.random.default_rng(10)
    pts = rng.uniform(-14, 14, size=(4000, 3))
    for u in (1, 2, 3):
        counts = np.zeros(len(pts), int)
        for c in g.universe_cells(u):
            ok = np.ones(len(pts), bool)
            for h in g.cell_halfspaces(c):
                s = abs(int(h)) - 1
                a, b, _, d = g.surf_coef[s][:4]
                ok &= ((a * pts[:, 0] + b * pts[:, 1]) - d > 0) == (h > 0)
            counts += ok
        assert counts.max() <= 1
