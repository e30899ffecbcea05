"""Seeded synthetic inputs: flattened nested-CSG geometries.

This module only *describes* geometries (surface coefficients, cell half-space
lists, fills, translations, per-material attenuation coefficients).  It holds
none of the tracking arithmetic: no containment test, distance, sampling or
tally code lives here.  Both the CPU oracle (tests) and the HIP library take
the same :class:`FlatGeometry` arrays as input.

Geometry model (paper, Introduction and Fig. 2/3 discussion; Section
"Tracking algorithms"):

* a *surface* is a plane, a z-cylinder or a sphere; its positive side is
  ``f(p) > 0`` (outside of a cylinder/sphere is positive);
* a *cell* is an intersection of signed half-spaces, filled either with a
  material or with a daughter *universe* placed with a translation;
* a *universe* is a contiguous range of cells; arrays are modelled as
  pseudo-array CSG universes (one explicit cell per lattice element, Section
  "Single tracker (ST) method").

Encodings (identical to ``include/gt.h``):

* ``surf_type``: 0 PX, 1 PY, 2 PZ (coef[0] = d), 3 P (a, b, c, d),
  4 CZ (x0, y0, r^2), 5 SPH (x0, y0, z0, r^2); 8 coefficient slots/surface.
* ``hs``: +(s+1) for the positive side of surface s, -(s+1) for the negative.
* ``cell_fill``: >= 0 material id, < 0 daughter universe -(u+1).
* ``lattice_hint``: 8 doubles per universe
  ``[kind, nx, ny, x0, y0, px, py, 0]``; kind 1 = square pseudo-lattice whose
  local cell ``j*nx + i`` spans ``[x0 + i*px, x0 + (i+1)*px]`` (edge cells may
  be unbounded outward).  Optional, advisory: it never changes a result.

Workload recipes follow the paper's shapes: 17x17 rectilinear assemblies of
pins split axially (Section "NuScale SMR"), 9-ring hexagonal assemblies of
217 pins (Section "Empire microreactor").
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PX, PY, PZ, P, CZ, SPH = 0, 1, 2, 3, 4, 5
N_COEF = 8
HINT_NONE, HINT_SQUARE = 0, 1


@dataclasses.dataclass
class FlatGeometry:
    surf_type: np.ndarray        # u8  [n_surfaces]
    surf_coef: np.ndarray        # f64 [n_surfaces, 8]
    cell_hs_off: np.ndarray      # u32 [n_cells + 1]
    hs: np.ndarray               # i32 [n_halfspaces]
    cell_fill: np.ndarray        # i32 [n_cells]
    cell_trans: np.ndarray       # f64 [n_cells, 3]
    univ_cell_off: np.ndarray    # u32 [n_universes + 1]
    root: int
    lattice_hint: np.ndarray     # f64 [n_universes, 8]
    sigma_t: np.ndarray          # f64 [n_materials]
    domain_lo: np.ndarray        # f64 [3]
    domain_hi: np.ndarray        # f64 [3]
    name: str = ""

    @property
    def n_surfaces(self) -> int:
        return int(self.surf_type.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cell_fill.shape[0])

    @property
    def n_universes(self) -> int:
        return int(self.univ_cell_off.shape[0] - 1)

    @property
    def n_materials(self) -> int:
        return int(self.sigma_t.shape[0])

    def universe_cells(self, u: int) -> range:
        return range(int(self.univ_cell_off[u]), int(self.univ_cell_off[u + 1]))

    def cell_halfspaces(self, c: int) -> np.ndarray:
        return self.hs[self.cell_hs_off[c]:self.cell_hs_off[c + 1]]


class GeomBuilder:
    """Accumulates surfaces and universes; universes are appended whole so
    that each universe's cells stay contiguous."""

    def __init__(self) -> None:
        self.stype: List[int] = []
        self.scoef: List[List[float]] = []
        self.cells: List[Tuple[List[int], int, Tuple[float, float, float]]] = []
        self.uoff: List[int] = [0]
        self.hints: List[List[float]] = []

    def surface(self, stype: int, *coef: float) -> int:
        c = [float(v) for v in coef] + [0.0] * (N_COEF - len(coef))
        self.stype.append(stype)
        self.scoef.append(c)
        return len(self.stype) - 1

    def universe(self, cells: Sequence[Tuple[List[int], int, Tuple[float, float, float]]],
                 hint: Optional[List[float]] = None) -> int:
        """cells: list of (halfspaces, fill, translation).  Returns the id."""
        for c in cells:
            self.cells.append((list(c[0]), int(c[1]), tuple(float(v) for v in c[2])))
        self.uoff.append(len(self.cells))
        self.hints.append(list(hint) if hint is not None else [0.0] * 8)
        return len(self.uoff) - 2

    def build(self, root: int, sigma_t: Sequence[float], lo, hi, name="") -> FlatGeometry:
        hs_off = [0]
        hs: List[int] = []
        for h, _, _ in self.cells:
            hs.extend(h)
            hs_off.append(len(hs))
        return FlatGeometry(
            surf_type=np.asarray(self.stype, dtype=np.uint8),
            surf_coef=np.asarray(self.scoef, dtype=np.float64).reshape(-1, N_COEF),
            cell_hs_off=np.asarray(hs_off, dtype=np.uint32),
            hs=np.asarray(hs, dtype=np.int32),
            cell_fill=np.asarray([c[1] for c in self.cells], dtype=np.int32),
            cell_trans=np.asarray([c[2] for c in self.cells], dtype=np.float64).reshape(-1, 3),
            univ_cell_off=np.asarray(self.uoff, dtype=np.uint32),
            root=int(root),
            lattice_hint=np.asarray(self.hints, dtype=np.float64).reshape(-1, 8),
            sigma_t=np.asarray(sigma_t, dtype=np.float64),
            domain_lo=np.asarray(lo, dtype=np.float64),
            domain_hi=np.asarray(hi, dtype=np.float64),
            name=name,
        )


def pos(s: int) -> int:
    return s + 1


def neg(s: int) -> int:
    return -(s + 1)


def fill_universe(u: int) -> int:
    return -(u + 1)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def _pin_universe(b: GeomBuilder, radii: Sequence[float], mat0: int,
                  zplanes: Sequence[float] = ()) -> int:
    """Concentric z-cylinders centred on the local origin; the outermost
    region (moderator) and the outer axial slabs are unbounded, so the pin
    universe tiles space and never repeats a parent's boundary surface."""
    cyl = [b.surface(CZ, 0.0, 0.0, r * r) for r in radii]
    zs = [b.surface(PZ, z) for z in zplanes]
    nr = len(radii) + 1
    cells = []
    for k in range(len(zs) + 1):
        slab = []
        if k > 0:
            slab.append(pos(zs[k - 1]))
        if k < len(zs):
            slab.append(neg(zs[k]))
        for r in range(nr):
            h = []
            if r > 0:
                h.append(pos(cyl[r - 1]))
            if r < nr - 1:
                h.append(neg(cyl[r]))
            cells.append((h + slab, mat0 + r, (0.0, 0.0, 0.0)))
    return b.universe(cells)


def _square_lattice(b: GeomBuilder, n: int, pitch: float, fills: np.ndarray,
                    bounded_outer: bool, zbounds: Optional[Tuple[float, float]] = None) -> int:
    """n x n pseudo-array universe centred at the origin.  Cell (i, j) is
    local cell j*n + i and is filled with universe fills[j, i] translated to
    its centre.  With bounded_outer=False the edge cells are unbounded
    outward (an infinite daughter); otherwise all n+1 planes per axis exist."""
    x0 = -0.5 * n * pitch
    edges = [x0 + k * pitch for k in range(n + 1)]
    lo_k = 0 if bounded_outer else 1
    hi_k = n if bounded_outer else n - 1
    sx = {k: b.surface(PX, edges[k]) for k in range(lo_k, hi_k + 1)}
    sy = {k: b.surface(PY, edges[k]) for k in range(lo_k, hi_k + 1)}
    zs = None
    if zbounds is not None:
        zs = (b.surface(PZ, zbounds[0]), b.surface(PZ, zbounds[1]))
    cells = []
    for j in range(n):
        for i in range(n):
            h = []
            if i in sx:
                h.append(pos(sx[i]))
            if i + 1 in sx:
                h.append(neg(sx[i + 1]))
            if j in sy:
                h.append(pos(sy[j]))
            if j + 1 in sy:
                h.append(neg(sy[j + 1]))
            if zs is not None:
                h += [pos(zs[0]), neg(zs[1])]
            cx = x0 + (i + 0.5) * pitch
            cy = x0 + (j + 0.5) * pitch
            cells.append((h, fill_universe(int(fills[j, i])), (cx, cy, 0.0)))
    hint = [HINT_SQUARE, n, n, x0, x0, pitch, pitch, 0.0]
    return b.universe(cells, hint)


def _sigmas(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(0.3, 1.0, size=n)


PIN_RADII = (0.40, 0.45, 0.50)
SQ_PITCH = 1.25


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

def config1(seed: int = 1001) -> FlatGeometry:
    """3x3 square lattice, pitch 1.25, one pin universe of 3 concentric
    z-cylinders r = 0.40/0.45/0.50 (4 materials); root cells bounded by 6
    planes; domain [-1.875, 1.875]^3, vacuum outside."""
    rng = np.random.default_rng(seed)
    b = GeomBuilder()
    h = 1.875
    # root first so that it is universe 0; its fills are patched below
    root_slot = len(b.uoff) - 1
    pin_placeholder = 1
    root = _square_lattice(b, 3, SQ_PITCH, np.full((3, 3), pin_placeholder), True, (-h, h))
    pin = _pin_universe(b, PIN_RADII, 0)
    assert root == root_slot and pin == pin_placeholder
    return b.build(root, _sigmas(rng, 4), (-h, -h, -h), (h, h, h), "cfg1_3x3")


def _axial_planes(n_interior: int, zlo: float, zhi: float) -> List[float]:
    return [zlo + k * (zhi - zlo) / (n_interior + 1) for k in range(1, n_interior + 1)]


def config2(seed: int = 1002) -> FlatGeometry:
    """17x17 square lattice of pins at the root, pitch 1.25, |z| <= 100;
    3 pin types in a seeded layout; each pin has 10 interior z-planes
    (11 slabs x 4 radial regions = 44 cells); 12 materials."""
    rng = np.random.default_rng(seed)
    n = 17
    layout = rng.integers(0, 3, size=(n, n))
    sig = _sigmas(rng, 12)
    b = GeomBuilder()
    root = _square_lattice(b, n, SQ_PITCH, layout + 1, True, (-100.0, 100.0))
    zpl = _axial_planes(10, -100.0, 100.0)
    pins = [_pin_universe(b, PIN_RADII, 4 * t, zpl) for t in range(3)]
    assert root == 0 and pins == [1, 2, 3]
    h = 0.5 * n * SQ_PITCH
    return b.build(root, sig, (-h, -h, -100.0), (h, h, 100.0), "cfg2_17x17")


def config3(seed: int = 1003) -> FlatGeometry:
    """Root cell (inside CZ r=140, |z| <= 100) filled with a 15x15 core
    lattice (pitch 21.25) of 5 seeded assembly types, each a 17x17 lattice
    of 3 pin types (pins as config 2).  Core and assembly lattices are
    infinite daughters (edge cells unbounded outward)."""
    rng = np.random.default_rng(seed)
    n_core, n_asm = 15, 17
    core_layout = rng.integers(0, 5, size=(n_core, n_core))
    asm_layouts = [rng.integers(0, 3, size=(n_asm, n_asm)) for _ in range(5)]
    sig = _sigmas(rng, 12)
    b = GeomBuilder()
    # universe ids: 0 root, 1 core, 2..6 assemblies, 7..9 pins
    rcyl = b.surface(CZ, 0.0, 0.0, 140.0 * 140.0)
    zlo = b.surface(PZ, -100.0)
    zhi = b.surface(PZ, 100.0)
    root = b.universe([([neg(rcyl), pos(zlo), neg(zhi)], fill_universe(1), (0.0, 0.0, 0.0))])
    core = _square_lattice(b, n_core, n_asm * SQ_PITCH, core_layout + 2, False)
    asms = [_square_lattice(b, n_asm, SQ_PITCH, asm_layouts[a] + 7, False) for a in range(5)]
    zpl = _axial_planes(10, -100.0, 100.0)
    pins = [_pin_universe(b, PIN_RADII, 4 * t, zpl) for t in range(3)]
    assert (root, core, asms, pins) == (0, 1, [2, 3, 4, 5, 6], [7, 8, 9])
    return b.build(root, sig, (-140.0, -140.0, -100.0), (140.0, 140.0, 100.0), "cfg3_core15x15")


# --------------------------------------------------------------------------
# hexagonal pseudo-arrays from planes only (Section "Empire microreactor":
# hexagonal assemblies tracked without hexagon-specific routines)
# --------------------------------------------------------------------------

def hex_ring_cells(rings: int) -> List[Tuple[int, int]]:
    """Axial coordinates (i, j) of a hexagonal arrangement of `rings` rings
    (1 + 3 r (r-1) cells), ordered ring by ring.  Hex distance
    max(|i|, |j|, |i + j|)."""
    out = []
    for r in range(rings):
        ring = [(i, j) for i in range(-r, r + 1) for j in range(-r, r + 1)
                if max(abs(i), abs(j), abs(i + j)) == r]
        ring.sort(key=lambda ij: (math.atan2(*_axial_dir(ij)), ij))
        out.extend(ring)
    return out


def _axial_dir(ij):
    i, j = ij
    # direction of i*a1 + j*a2 with a1 at 30 deg, a2 at 90 deg (for ordering only)
    return (i * 0.5 + j, i * math.sqrt(3) / 2)


class HexFamilies:
    """Three families of parallel planes (normals n_k at angles phi_k, all
    planes of a family share bitwise-identical normal coefficients) spaced
    by half a pitch.  A hexagonal cell of flat-to-flat width `pitch` centred
    on the lattice point i*a1 + j*a2 (a1 = pitch * n_0, a2 = pitch * n_1) is
    the slab between planes m_k - 1 and m_k + 1 (in units of pitch/2) of each
    family, with m_0 = 2i + j, m_1 = i + 2j, m_2 = -i + j."""

    def __init__(self, b: "GeomBuilder", pitch: float, phi0_deg: float):
        self.b = b
        self.pitch = pitch
        angs = [math.radians(phi0_deg + 60.0 * k) for k in range(3)]
        self.n = [(math.cos(a), math.sin(a)) for a in angs]
        self.planes: dict = {}

    def plane(self, k: int, m: int) -> int:
        key = (k, m)
        if key not in self.planes:
            a, bb = self.n[k]
            self.planes[key] = self.b.surface(P, a, bb, 0.0, m * (self.pitch / 2.0))
        return self.planes[key]

    def cell(self, i: int, j: int) -> List[int]:
        ms = (2 * i + j, i + 2 * j, -i + j)
        h = []
        for k, m in enumerate(ms):
            h += [pos(self.plane(k, m - 1)), neg(self.plane(k, m + 1))]
        return h

    def centre(self, i: int, j: int) -> Tuple[float, float]:
        (a0, b0), (a1, b1) = self.n[0], self.n[1]
        return (self.pitch * (i * a0 + j * a1), self.pitch * (i * b0 + j * b1))

    def vertices(self, i: int, j: int) -> List[Tuple[float, float]]:
        cx, cy = self.centre(i, j)
        rc = self.pitch / math.sqrt(3.0)
        # vertices lie halfway between the face normals
        phi = math.atan2(self.n[0][1], self.n[0][0])
        return [(cx + rc * math.cos(phi + math.radians(30 + 60 * k)), cy + rc * math.sin(phi + math.radians(30 + 60 * k)))
                for k in range(6)]


HEX_PIN_PITCH = 1.3
HEX_PIN_RADII = (0.4, 0.5)
HEX_GAP = 0.05


def config4(seed: int = 1004, core_rings: int = 7, asm_rings: int = 9, rim_rings: int = 2) -> FlatGeometry:
    """7-ring core of hexagonal assemblies, each a 9-ring (217-pin) hexagonal
    lattice of pins (two z-cylinders r = 0.4/0.5, pitch 1.3), built from
    planes only and tracked through the generic hierarchy (no lattice hint).

    Pins are flat-top hexagons (plane families at 30/90/150 degrees);
    assemblies are pointy-top hexagons (families at 0/60/120 degrees) of
    flat-to-flat 26 p / sqrt(3) + 2 g, so no pin plane is ever parallel to an
    assembly boundary.  Each assembly universe adds `rim_rings` rings of
    moderator hexagons around its pins; they cover the whole assembly
    hexagon (the only region its parent can reach).  Three pin types
    (fuel-, moderator-, heat-pipe-like: 3 materials each) and three seeded
    assembly layouts; the root is the core pseudo-array of hexagonal prisms
    with |z| <= 100 and vacuum outside its jagged union."""
    rng = np.random.default_rng(seed)
    p = HEX_PIN_PITCH
    # circumscribing pointy-top hexagon of the pin union, plus the gap on each side
    F = 2.0 * ((asm_rings - 1) * p * math.sqrt(3) / 2.0 + p / math.sqrt(3)) + 2 * HEX_GAP
    n_pin_types, n_asm_types = 3, 3
    sig = _sigmas(rng, 3 * n_pin_types + 1)
    mod_mat = 3 * n_pin_types
    pins_in = hex_ring_cells(asm_rings)
    rim = hex_ring_cells(asm_rings + rim_rings)[len(pins_in):]
    layouts = [rng.choice(n_pin_types, size=len(pins_in), p=[0.5, 0.3, 0.2]) for _ in range(n_asm_types)]
    core = hex_ring_cells(core_rings)
    core_types = rng.integers(0, n_asm_types, size=len(core))
    b = GeomBuilder()
    # universe ids: 0 root (core), 1..3 assemblies, 4..6 pins
    fam_core = HexFamilies(b, F, 0.0)
    zlo = b.surface(PZ, -100.0)
    zhi = b.surface(PZ, 100.0)
    cells = []
    for (i, j), t in zip(core, core_types):
        cx, cy = fam_core.centre(i, j)
        cells.append((fam_core.cell(i, j) + [pos(zlo), neg(zhi)], fill_universe(1 + int(t)), (cx, cy, 0.0)))
    root = b.universe(cells)
    asms = []
    for a in range(n_asm_types):
        fam = HexFamilies(b, p, 30.0)
        cells = []
        for (i, j), t in zip(pins_in, layouts[a]):
            cx, cy = fam.centre(i, j)
            cells.append((fam.cell(i, j), fill_universe(4 + int(t)), (cx, cy, 0.0)))
        for (i, j) in rim:
            cells.append((fam.cell(i, j), mod_mat, (0.0, 0.0, 0.0)))
        asms.append(b.universe(cells))
    pins = [_pin_universe(b, HEX_PIN_RADII, 3 * t) for t in range(n_pin_types)]
    assert root == 0 and asms == [1, 2, 3] and pins == [4, 5, 6]
    xs, ys = [], []
    for (i, j) in core:
        for vx, vy in fam_core.vertices(i, j):
            xs.append(vx)
            ys.append(vy)
    m = 1e-9 * max(max(map(abs, xs)), max(map(abs, ys)))
    lo = (min(xs) - m, min(ys) - m, -100.0)
    hi = (max(xs) + m, max(ys) + m, 100.0)
    return b.build(root, sig, lo, hi, "cfg4_hex7x9")


# --------------------------------------------------------------------------
# batched workload: many geometries of uneven size
# --------------------------------------------------------------------------

BATCH_HALF_HEIGHT = 10.0


def _square_flat(b: GeomBuilder, n: int, pitch: float, types: np.ndarray, radii, zb) -> int:
    """One universe holding an n x n lattice with every pin's cylinders
    flattened into it: per slot a fuel cell (inside the inner cylinder), a
    ring cell and a moderator cell bounded by the slot's planes.  The
    lattice's outer planes and z planes bound every cell."""
    x0 = -0.5 * n * pitch
    sx = [b.surface(PX, x0 + k * pitch) for k in range(n + 1)]
    sy = [b.surface(PY, x0 + k * pitch) for k in range(n + 1)]
    z0, z1 = b.surface(PZ, -zb), b.surface(PZ, zb)
    cells = []
    for j in range(n):
        for i in range(n):
            cx, cy = x0 + (i + 0.5) * pitch, x0 + (j + 0.5) * pitch
            cyl = [b.surface(CZ, cx, cy, r * r) for r in radii]
            box = [pos(sx[i]), neg(sx[i + 1]), pos(sy[j]), neg(sy[j + 1]), pos(z0), neg(z1)]
            m0 = 3 * int(types[j, i])
            cells.append(([neg(cyl[0]), pos(z0), neg(z1)], m0, (0.0, 0.0, 0.0)))
            cells.append(([pos(cyl[0]), neg(cyl[1]), pos(z0), neg(z1)], m0 + 1, (0.0, 0.0, 0.0)))
            cells.append(([pos(cyl[1])] + box, m0 + 2, (0.0, 0.0, 0.0)))
    return b.universe(cells)


def _hex_flat(b: GeomBuilder, rings: int, pitch: float, types, radii, zb) -> Tuple[int, HexFamilies, list]:
    fam = HexFamilies(b, pitch, 30.0)
    z0, z1 = b.surface(PZ, -zb), b.surface(PZ, zb)
    cells = []
    slots = hex_ring_cells(rings)
    for (i, j), t in zip(slots, types):
        cx, cy = fam.centre(i, j)
        cyl = [b.surface(CZ, cx, cy, r * r) for r in radii]
        m0 = 3 * int(t)
        cells.append(([neg(cyl[0]), pos(z0), neg(z1)], m0, (0.0, 0.0, 0.0)))
        cells.append(([pos(cyl[0]), neg(cyl[1]), pos(z0), neg(z1)], m0 + 1, (0.0, 0.0, 0.0)))
        cells.append(([pos(cyl[1])] + fam.cell(i, j) + [pos(z0), neg(z1)], m0 + 2, (0.0, 0.0, 0.0)))
    return b.universe(cells), fam, slots


def batch_item(j: int) -> Tuple[FlatGeometry, int]:
    """Geometry j of the batched workload and its history count (seeds 5000+j
    for the geometry, 6000+j for the particles).  Square (pitch 1.25) or
    hexagonal (pitch 1.3) with equal probability; lattice dimension (square
    side, or hexagonal rings) uniform in 3..33; nesting levels uniform in
    1..3: 1 = one universe with every pin's cylinders flattened into it,
    2 = a lattice of pin universes at the root, 3 = a small lattice (3x3 or
    2 rings) of such lattices; pins have cylinders r = 0.4/0.5 and three
    types; |z| <= 10; histories log-uniform in [1e4, 1e6]."""
    rng = np.random.default_rng(5000 + j)
    hexa = bool(rng.integers(0, 2))
    dim = int(rng.integers(3, 34))
    levels = int(rng.integers(1, 4))
    n_hist = int(round(math.exp(rng.uniform(math.log(1e4), math.log(1e6)))))
    radii = (0.4, 0.5)
    zb = BATCH_HALF_HEIGHT
    sig = _sigmas(rng, 9)
    b = GeomBuilder()
    if not hexa:
        pitch = SQ_PITCH
        if levels == 1:
            types = rng.integers(0, 3, size=(dim, dim))
            root = _square_flat(b, dim, pitch, types, radii, zb)
            h = 0.5 * dim * pitch
        elif levels == 2:
            types = rng.integers(0, 3, size=(dim, dim))
            root = _square_lattice(b, dim, pitch, types + 1, True, (-zb, zb))
            pins = [_pin_universe(b, radii, 3 * t) for t in range(3)]
            assert root == 0 and pins == [1, 2, 3]
            h = 0.5 * dim * pitch
        else:
            n_core, n_asm_types = 3, 2
            core_types = rng.integers(0, n_asm_types, size=(n_core, n_core))
            apitch = dim * pitch
            root = _square_lattice(b, n_core, apitch, core_types + 1, True, (-zb, zb))
            asms = [_square_lattice(b, dim, pitch, rng.integers(0, 3, size=(dim, dim)) + 1 + n_asm_types, False)
                    for _ in range(n_asm_types)]
            pins = [_pin_universe(b, radii, 3 * t) for t in range(3)]
            assert root == 0 and asms == [1, 2] and pins == [3, 4, 5]
            h = 0.5 * n_core * apitch
        g = b.build(root, sig, (-h, -h, -zb), (h, h, zb), "batch%02d_sq%d_L%d" % (j, dim, levels))
        return g, n_hist
    pitch = HEX_PIN_PITCH
    if levels == 1:
        types = rng.integers(0, 3, size=len(hex_ring_cells(dim)))
        root, fam, slots = _hex_flat(b, dim, pitch, types, radii, zb)
        verts = [v for (i, jj) in slots for v in fam.vertices(i, jj)]
    elif levels == 2:
        fam = HexFamilies(b, pitch, 30.0)
        z0, z1 = b.surface(PZ, -zb), b.surface(PZ, zb)
        slots = hex_ring_cells(dim)
        types = rng.integers(0, 3, size=len(slots))
        cells = []
        for (i, jj), t in zip(slots, types):
            cx, cy = fam.centre(i, jj)
            cells.append((fam.cell(i, jj) + [pos(z0), neg(z1)], fill_universe(1 + int(t)), (cx, cy, 0.0)))
        root = b.universe(cells)
        pins = [_pin_universe(b, radii, 3 * t) for t in range(3)]
        assert root == 0 and pins == [1, 2, 3]
        verts = [v for (i, jj) in slots for v in fam.vertices(i, jj)]
    else:
        n_asm_types = 2
        F = 2.0 * ((dim - 1) * pitch * math.sqrt(3) / 2.0 + pitch / math.sqrt(3)) + 2 * HEX_GAP
        fam_core = HexFamilies(b, F, 0.0)
        z0, z1 = b.surface(PZ, -zb), b.surface(PZ, zb)
        core = hex_ring_cells(2)
        core_types = rng.integers(0, n_asm_types, size=len(core))
        cells = []
        for (i, jj), t in zip(core, core_types):
            cx, cy = fam_core.centre(i, jj)
            cells.append((fam_core.cell(i, jj) + [pos(z0), neg(z1)], fill_universe(1 + int(t)), (cx, cy, 0.0)))
        root = b.universe(cells)
        pins_in = hex_ring_cells(dim)
        rim = hex_ring_cells(dim + 2)[len(pins_in):]
        asms = []
        for a in range(n_asm_types):
            fam = HexFamilies(b, pitch, 30.0)
            types = rng.integers(0, 3, size=len(pins_in))
            cells = []
            for (i, jj), t in zip(pins_in, types):
                cx, cy = fam.centre(i, jj)
                cells.append((fam.cell(i, jj), fill_universe(1 + n_asm_types + int(t)), (cx, cy, 0.0)))
            for (i, jj) in rim:
                cells.append((fam.cell(i, jj), 2, (0.0, 0.0, 0.0)))
            asms.append(b.universe(cells))
        pins = [_pin_universe(b, radii, 3 * t) for t in range(3)]
        assert root == 0 and asms == [1, 2] and pins == [3, 4, 5]
        verts = [v for (i, jj) in core for v in fam_core.vertices(i, jj)]
    xs, ys = [v[0] for v in verts], [v[1] for v in verts]
    m = 1e-9 * max(max(map(abs, xs)), max(map(abs, ys)))
    g = b.build(0, sig, (min(xs) - m, min(ys) - m, -zb), (max(xs) + m, max(ys) + m, zb),
                "batch%02d_hex%d_L%d" % (j, dim, levels))
    return g, n_hist


BATCH_SIZE = 64


def config5() -> List[Tuple[FlatGeometry, int]]:
    """The batched workload: 64 geometries and their history counts."""
    return [batch_item(j) for j in range(BATCH_SIZE)]


def hex_pin_box(half: float = 6.0, rings: int = 8, seed: int = 1104) -> FlatGeometry:
    """A box |x|,|y| <= half, |z| <= 100 filled with a flat-top hexagonal
    lattice of identical pins (pitch 1.3, cylinders 0.4/0.5) large enough to
    cover the box; used to check hexagonal pin volumes with stratified rays."""
    rng = np.random.default_rng(seed)
    b = GeomBuilder()
    s = [b.surface(PX, -half), b.surface(PX, half), b.surface(PY, -half), b.surface(PY, half),
         b.surface(PZ, -100.0), b.surface(PZ, 100.0)]
    root = b.universe([([pos(s[0]), neg(s[1]), pos(s[2]), neg(s[3]), pos(s[4]), neg(s[5])],
                        fill_universe(1), (0.0, 0.0, 0.0))])
    fam = HexFamilies(b, HEX_PIN_PITCH, 30.0)
    cells = []
    for (i, j) in hex_ring_cells(rings):
        cx, cy = fam.centre(i, j)
        cells.append((fam.cell(i, j), fill_universe(2), (cx, cy, 0.0)))
    lat = b.universe(cells)
    pin = _pin_universe(b, HEX_PIN_RADII, 0)
    assert (root, lat, pin) == (0, 1, 2)
    return b.build(root, _sigmas(rng, 3), (-half, -half, -100.0), (half, half, 100.0), "hex_pin_box")


def sphere(radius: float = 1.0, sigma: float = 1.0) -> FlatGeometry:
    """A single sphere of one material (for first-flight escape checks)."""
    b = GeomBuilder()
    s = b.surface(SPH, 0.0, 0.0, 0.0, radius * radius)
    root = b.universe([([neg(s)], 0, (0.0, 0.0, 0.0))])
    r = radius
    return b.build(root, [sigma], (-r, -r, -r), (r, r, r), "sphere")


def box(half: Tuple[float, float, float] = (1.0, 1.0, 1.0), sigma: float = 1.0) -> FlatGeometry:
    """A single rectangular cell of one material."""
    b = GeomBuilder()
    hx, hy, hz = half
    s = [b.surface(PX, -hx), b.surface(PX, hx), b.surface(PY, -hy), b.surface(PY, hy),
         b.surface(PZ, -hz), b.surface(PZ, hz)]
    root = b.universe([([pos(s[0]), neg(s[1]), pos(s[2]), neg(s[3]), pos(s[4]), neg(s[5])],
                        0, (0.0, 0.0, 0.0))])
    return b.build(root, [sigma], (-hx, -hy, -hz), (hx, hy, hz), "box")


def nested_box(half: float = 1.0, sigma: float = 0.7) -> FlatGeometry:
    """A box whose one cell holds a universe whose one cell is bounded by two
    x-planes equal to the box's own (distinct surfaces, same coefficients):
    every exit through x = +-half ties between the two levels at one
    distance, which the top level must take (from the daughter there is no
    neighbour)."""
    b = GeomBuilder()
    h = half
    s = [b.surface(PX, -h), b.surface(PX, h), b.surface(PY, -h), b.surface(PY, h),
         b.surface(PZ, -h), b.surface(PZ, h), b.surface(PX, -h), b.surface(PX, h)]
    root = b.universe([([pos(s[0]), neg(s[1]), pos(s[2]), neg(s[3]), pos(s[4]), neg(s[5])],
                        fill_universe(1), (0.0, 0.0, 0.0))])
    inner = b.universe([([pos(s[6]), neg(s[7])], 0, (0.0, 0.0, 0.0))])
    assert (root, inner) == (0, 1)
    return b.build(root, [sigma], (-h, -h, -h), (h, h, h), "nested_box")


def deep_slabs(levels: int = 6, sigma: float = 0.5) -> FlatGeometry:
    """The deepest nesting the library takes: a root box |x|, |y|, |z| < 2
    filled with universe 1, and each universe k = 1 .. levels-2 split along
    x into a left slab, a middle slab filled with universe k+1 (translated a
    little in x and y) and a right slab, the slabs narrowing with k; the
    last universe is a z-cylinder of radius 0.3 and what lies outside it.
    Materials differ by level, so tallies tell the levels apart."""
    if not 2 <= levels <= 6:
        raise ValueError("levels must be 2..6")
    b = GeomBuilder()
    box = [b.surface(PX, -2.0), b.surface(PX, 2.0), b.surface(PY, -2.0), b.surface(PY, 2.0),
           b.surface(PZ, -2.0), b.surface(PZ, 2.0)]
    root = b.universe([([pos(box[0]), neg(box[1]), pos(box[2]), neg(box[3]), pos(box[4]), neg(box[5])],
                        fill_universe(1), (0.1, -0.05, 0.0))])
    for k in range(1, levels - 1):
        a = 1.8 - 0.3 * k
        sl, sr = b.surface(PX, -a), b.surface(PX, a)
        u = b.universe([([neg(sl)], k % 3, (0.0, 0.0, 0.0)),
                        ([pos(sl), neg(sr)], fill_universe(k + 1), (0.03 * k, 0.02, 0.0)),
                        ([pos(sr)], (k + 1) % 3, (0.0, 0.0, 0.0))])
        assert u == k
    cyl = b.surface(CZ, 0.0, 0.0, 0.09)
    last = b.universe([([neg(cyl)], 1, (0.0, 0.0, 0.0)), ([pos(cyl)], 2, (0.0, 0.0, 0.0))])
    assert last == levels - 1 and root == 0
    return b.build(root, [sigma, 0.8 * sigma, 1.3 * sigma], (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0), "deep_slabs")


WORKLOADS = {1: config1, 2: config2, 3: config3, 4: config4}

# particle counts of the workload table, and the seeds: geometry 1000+i,
# particles 2000+i.
CONFIG_PARTICLES = {1: 10_000, 2: 1_000_000, 3: 10_000_000, 4: 10_000_000}


def make_config(i: int) -> FlatGeometry:
    return WORKLOADS[i](1000 + i)


def particle_seed(i: int) -> int:
    return 2000 + i


def batch_particle_seed(j: int) -> int:
    """Particle seed of item j of the batched workload."""
    return 6000 + j


def batch_geometry_id(j: int) -> int:
    """Geometry id (the fourth Philox counter word) of batch item j."""
    return 100 + j
