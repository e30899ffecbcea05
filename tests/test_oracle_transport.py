"""Pins for the oracle's history loop (Alg. 2 reduced to the toy transport)
and its outputs: analytic cell volumes from uniform parallel rays, the
optical-depth and path-length invariants of each flight, the first-flight
escape probability of a sphere (a textbook closed form), symmetry, and
determinism/additivity of the outputs."""

import math

import numpy as np
import pytest

import oracle
from paper_2406_13849_amd import synth


def _ray_volumes(g, og, n1, n2):
    p = oracle.TrackParams(seed=0, n_particles=n1 * n2, source=1, ray_n1=n1, max_collisions=1)
    r = oracle.track(og, p, n_threads=8)
    assert r.counters["escaped"] == n1 * n2 and r.counters["lost"] == 0
    hy = (g.domain_hi[1] - g.domain_lo[1]) / n1
    hz = (g.domain_hi[2] - g.domain_lo[2]) / n2
    return r.tally * hy * hz, r


def test_ray_volumes_cfg1_pin_regions():
    """Uniform parallel rays: V_c = (face area / N) * sum of chord lengths.
    cfg1 has no axial structure, so one ray row in z integrates exactly."""
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    vol, _ = _ray_volumes(g, og, 21000, 1)   # 7000 rays per pin row: grid aligned with the lattice
    H = 3.75
    ring = [math.pi * 0.16, math.pi * (0.2025 - 0.16), math.pi * (0.25 - 0.2025), 1.25 ** 2 - math.pi * 0.25]
    want = np.tile(np.array(ring) * H, 9)
    assert np.allclose(vol, want, rtol=1e-4, atol=0)
    assert abs(vol.sum() - 3.75 ** 3) < 1e-6 * 3.75 ** 3


def test_ray_volumes_cfg2_axial_slabs():
    g = synth.make_config(2)
    og = oracle.OracleGeometry(g)
    vol, _ = _ray_volumes(g, og, 6800, 22)   # 22 = 2 rays per axial slab, grid aligned with slabs
    slab = 200.0 / 11
    ring = np.array([math.pi * 0.16, math.pi * (0.2025 - 0.16), math.pi * (0.25 - 0.2025),
                     1.25 ** 2 - math.pi * 0.25])
    want = np.tile(np.tile(ring, 11) * slab, 289)
    assert np.allclose(vol, want, rtol=2e-4, atol=0)


def test_flight_optical_depth_and_path_length():
    """Every flight that ends in a collision spends exactly its sampled tau:
    sum of Sigma*l over its segments equals tau; and the segments of one
    flight are collinear, so their lengths add up to the chord from the
    flight's start to its end."""
    g = synth.make_config(2)
    og = oracle.OracleGeometry(g)
    p = oracle.TrackParams(seed=2002, n_particles=400, geometry_id=2)
    n_fl = 0
    for i in range(400):
        t = oracle.trace_particle(og, p, i)
        start = t.birth_pos
        k0 = 0
        f = 0
        for k in range(len(t.seg_len)):
            if t.seg_kind[k] == 1 or k == len(t.seg_len) - 1:
                segs = slice(k0, k + 1)
                end = t.seg_pos[k]
                chord = float(np.linalg.norm(end - start))
                plen = math.fsum(t.seg_len[segs])
                assert abs(plen - chord) <= 1e-12 * max(1.0, abs(start).max()), (i, k)
                if t.seg_kind[k] == 1:
                    od = math.fsum(t.seg_len[segs] * t.seg_sigma[segs])
                    assert abs(od - t.flight_tau[f]) <= 1e-12 * max(1.0, t.flight_tau[f]), (i, k)
                    n_fl += 1
                f += 1
                start = end
                k0 = k + 1
    assert n_fl > 1000


def test_tally_is_sum_of_segment_lengths():
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    p = oracle.TrackParams(seed=77, n_particles=300, geometry_id=1)
    r = oracle.track(og, p, n_threads=2)
    per_inst = np.zeros(og.n_instances)
    nseg = 0
    for i in range(300):
        t = oracle.trace_particle(og, p, i)
        assert len(t.seg_len) == r.seg_count[i]
        assert t.end_code == r.end_code[i]
        np.add.at(per_inst, t.seg_inst, t.seg_len)
        nseg += len(t.seg_len)
    assert nseg == r.counters["segments"]
    assert np.allclose(r.tally, per_inst, rtol=1e-13, atol=0)
    # fixed-point tally agrees with the exact fixed-point sum of the quantised lengths
    assert np.allclose(r.tally_fxd, r.tally, rtol=1e-13, atol=0)


def _sphere_escape(a):
    """First-flight escape probability from a sphere of optical radius a
    with a uniform isotropic source (Case, de Hoffmann and Placzek)."""
    return 3.0 / (8.0 * a ** 3) * (2 * a * a - 1 + (1 + 2 * a) * math.exp(-2 * a))


@pytest.mark.parametrize("R,sigma", [(1.0, 1.0), (2.0, 0.35), (0.5, 0.8)])
def test_sphere_first_flight_escape(R, sigma):
    g = synth.sphere(R, sigma)
    og = oracle.OracleGeometry(g)
    n = 200_000
    p = oracle.TrackParams(seed=31, n_particles=n, geometry_id=9, max_collisions=1)
    r = oracle.track(og, p, n_threads=8, tallies=False)
    assert r.counters["escaped"] + r.counters["capped"] == n
    pe = _sphere_escape(R * sigma)
    frac = r.counters["escaped"] / n
    assert abs(frac - pe) < 4.5 * math.sqrt(pe * (1 - pe) / n), (frac, pe)


def test_symmetry_of_identical_pins():
    """cfg1's nine pins are identical and the source is uniform: the four
    corner pins' fuel tallies share one expectation (batch-means bound)."""
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    nb, per = 10, 20_000
    corners = [0, 2, 6, 8]
    vals = []
    for b in range(nb):
        p = oracle.TrackParams(seed=1234, n_particles=per, first_particle=b * per, geometry_id=1)
        r = oracle.track(og, p, n_threads=8)
        vals.append([r.tally[c * 4] for c in corners])
    v = np.array(vals)
    mean = v.mean(0)
    se = v.std(0, ddof=1) / math.sqrt(nb)
    grand = mean.mean()
    assert np.all(np.abs(mean - grand) < 4 * se.max() + 1e-12)


def test_thread_count_and_range_split_do_not_change_results():
    g = synth.make_config(2)
    og = oracle.OracleGeometry(g)
    p = oracle.TrackParams(seed=2002, n_particles=4000, geometry_id=2, record_first_k=50, record_cap=200)
    a = oracle.track(og, p, n_threads=1)
    b = oracle.track(og, p, n_threads=7)
    for f in ("seg_count", "seq_hash", "end_code", "rec", "tally_fx"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert np.allclose(a.tally, b.tally, rtol=1e-14, atol=0)
    # two halves by first_particle reproduce the per-particle outputs, and
    # the fixed-point tallies add exactly (mod 2^128)
    h1 = oracle.track(og, oracle.TrackParams(seed=2002, n_particles=1500, geometry_id=2), n_threads=3)
    h2 = oracle.track(og, oracle.TrackParams(seed=2002, n_particles=2500, first_particle=1500, geometry_id=2),
                      n_threads=3)
    assert np.array_equal(np.concatenate([h1.seq_hash, h2.seq_hash]), a.seq_hash)
    assert np.array_equal(np.concatenate([h1.seg_count, h2.seg_count]), a.seg_count)
    lo = h1.tally_fx[:, 0].astype(object) + h2.tally_fx[:, 0].astype(object)
    hi = h1.tally_fx[:, 1].astype(object) + h2.tally_fx[:, 1].astype(object) + lo // (1 << 64)
    assert np.array_equal((lo % (1 << 64)).astype(np.uint64), a.tally_fx[:, 0])
    assert np.array_equal((hi % (1 << 64)).astype(np.uint64), a.tally_fx[:, 1])


def test_fixed_point_quantisation_exact():
    """Lengths >= 2^-43 are represented exactly: integer part * 2^96 plus
    fraction * 2^96."""
    from fractions import Fraction
    rng = np.random.default_rng(2)
    ls = np.concatenate([rng.uniform(0, 3, 1000), rng.uniform(0, 1e-6, 100), [0.0, 1.0, 2.5, 2.0 ** -43, 1e-20]])
    q = oracle.fx_quantise(ls)
    for l, (lo, hi) in zip(ls, q):
        v = (int(hi) << 64) | int(lo)
        exact = Fraction(float(l)) * (1 << 96)
        assert v == math.floor(exact)


def test_record_and_hash_consistency():
    g = synth.make_config(1)
    og = oracle.OracleGeometry(g)
    p = oracle.TrackParams(seed=5, n_particles=200, geometry_id=1, record_first_k=200, record_cap=8)
    r = oracle.track(og, p, n_threads=4)
    FNV_OFF, FNV_P = 0xcbf29ce484222325, 0x100000001b3
    ovf = 0
    for i in range(200):
        t = oracle.trace_particle(og, p, i)
        h = FNV_OFF
        for inst in t.seg_inst:
            h = ((h ^ (int(inst) + 1)) * FNV_P) % (1 << 64)
        h ^= t.end_code
        assert h == int(r.seq_hash[i])
        k = min(8, len(t.seg_inst))
        assert np.array_equal(r.rec[i, :k], t.seg_inst[:k])
        assert np.all(r.rec[i, k:] == -1)
        ovf += len(t.seg_inst) > 8
    assert r.counters["rec_overflow"] == ovf


def test_segment_cap_and_collision_cap():
    g = synth.make_config(2)
    og = oracle.OracleGeometry(g)
    p = oracle.TrackParams(seed=3, n_particles=500, geometry_id=2, max_segments=10)
    r = oracle.track(og, p, n_threads=2)
    assert r.seg_count.max() == 10
    segcap = r.end_code == oracle.END_SEGCAP
    assert segcap.sum() > 0 and np.all(r.seg_count[segcap] == 10)
    assert r.counters["segcap"] == segcap.sum()
    p = oracle.TrackParams(seed=3, n_particles=500, geometry_id=2, max_collisions=3)
    r = oracle.track(og, p, n_threads=2)
    assert set(np.unique(r.end_code)) <= {oracle.END_ESCAPE, oracle.END_CAP}


def test_work_meter_hand_count():
    """Rays along +x through a single box: locating the birth cell tests 6
    axis half-spaces (6 ops), the one segment evaluates the +x plane (2 ops:
    subtract, divide; the -x plane is receding and y/z planes are parallel)
    and moves (6 ops): 14 operations per history, one segment each."""
    og = oracle.OracleGeometry(synth.box((1.0, 2.0, 3.0)))
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=0, n_particles=100, source=1, ray_n1=10))
    assert segs == 100 and ops == 1400


def _box_planes(b, h):
    return [b.surface(synth.PX, -h), b.surface(synth.PX, h), b.surface(synth.PY, -h),
            b.surface(synth.PY, h), b.surface(synth.PZ, -h), b.surface(synth.PZ, h)]


def _inside_box(s):
    return [synth.pos(s[0]), synth.neg(s[1]), synth.pos(s[2]), synth.neg(s[3]), synth.pos(s[4]), synth.neg(s[5])]


def _ray_grid(n1, n2, h):
    """(y, z) of the stratified ray grid of ray mode over the face [-h, h]^2."""
    return [(-h + (j + 0.5) * 2 * h / n1, -h + (k + 0.5) * 2 * h / n2) for k in range(n2) for j in range(n1)]


def test_work_meter_hand_count_cylinder():
    """Rays along +x through a z-cylinder (r = 1) inside a box [-2, 2]^3:
    cell 0 is the inside of the cylinder (slab |z| <= 2), cell 1 the rest of
    the box.  By hand, a ray that meets the cylinder costs:
      birth, containment of cell 1: cylinder value 6 + six axis planes 6 = 12;
      segment 1 (cell 1): cylinder root with a, b 8, c and discriminant 7,
        sqrt, subtraction, division 3; the +x plane 2; move 6; crossing into
        cell 0, its two z-planes checked 2 -> 28;
      segment 2 (cell 0, on the cylinder): a, b 8, far root -2b/a 2; move 6;
        crossing into cell 1, six axis planes 6 -> 22;
      segment 3 (cell 1, on the cylinder, receding): a, b 8; +x plane 2;
        move 6 -> 16 (then the ray escapes);
    78 operations, 3 segments.  A ray that misses it: 12 + (8 + 7 + 2 + 6)
    = 35 operations, 1 segment."""
    b = synth.GeomBuilder()
    cz = b.surface(synth.CZ, 0.0, 0.0, 1.0)
    s = _box_planes(b, 2.0)
    u = b.universe([([synth.neg(cz), synth.pos(s[4]), synth.neg(s[5])], 0, (0.0, 0.0, 0.0)),
                    ([synth.pos(cz)] + _inside_box(s), 1, (0.0, 0.0, 0.0))])
    og = oracle.OracleGeometry(b.build(u, [1.0, 1.0], (-2.0,) * 3, (2.0,) * 3))
    n1, n2 = 8, 2
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=0, n_particles=n1 * n2, source=1, ray_n1=n1))
    hits = sum(abs(y) < 1.0 for y, z in _ray_grid(n1, n2, 2.0))
    miss = n1 * n2 - hits
    assert hits == 8
    assert segs == 3 * hits + miss and ops == 78 * hits + 35 * miss


def test_work_meter_hand_count_sphere():
    """The same with a sphere (r = 1): cell 1's containment 9 + 6 = 15;
    segment 1: a, b 13, c and discriminant 9, root 3, the +x plane 2, move 6
    (cell 0 has no other surface to check) -> 33; segment 2 on the sphere:
    13 + 2, move 6, six axis planes 6 -> 27; segment 3: 13 + 2 + 6 -> 21:
    96 operations and 3 segments for a ray that meets it, 15 + (13 + 9 + 2
    + 6) = 45 and 1 segment for one that does not."""
    b = synth.GeomBuilder()
    sp = b.surface(synth.SPH, 0.0, 0.0, 0.0, 1.0)
    s = _box_planes(b, 2.0)
    u = b.universe([([synth.neg(sp)], 0, (0.0, 0.0, 0.0)),
                    ([synth.pos(sp)] + _inside_box(s), 1, (0.0, 0.0, 0.0))])
    og = oracle.OracleGeometry(b.build(u, [1.0, 1.0], (-2.0,) * 3, (2.0,) * 3))
    n1 = n2 = 8
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=0, n_particles=n1 * n2, source=1, ray_n1=n1))
    hits = sum(y * y + z * z < 1.0 for y, z in _ray_grid(n1, n2, 2.0))
    miss = n1 * n2 - hits
    assert hits == 12
    assert segs == 3 * hits + miss and ops == 96 * hits + 45 * miss


def test_work_meter_hand_count_general_plane():
    """A general plane x + y = 0 splitting the box [-2, 2]^3: birth in
    cell 0, containment 6 (plane value) + 6 = 12; segment 1: the plane's
    denominator 5 and root 6 + 1, the +x plane 2, move 6, crossing into
    cell 1 with its six axis planes 6 -> 26; segment 2 (on the plane): the
    +x plane 2, move 6 -> 8; 46 operations and 2 segments per ray."""
    b = synth.GeomBuilder()
    pl = b.surface(synth.P, 1.0, 1.0, 0.0, 0.0)
    s = _box_planes(b, 2.0)
    u = b.universe([([synth.neg(pl)] + _inside_box(s), 0, (0.0, 0.0, 0.0)),
                    ([synth.pos(pl)] + _inside_box(s), 1, (0.0, 0.0, 0.0))])
    og = oracle.OracleGeometry(b.build(u, [1.0, 1.0], (-2.0,) * 3, (2.0,) * 3))
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=0, n_particles=24, source=1, ray_n1=6))
    assert segs == 2 * 24 and ops == 46 * 24


def _philox_fields(seed, gid, pid, blk):
    o = oracle.philox4x32_10([blk, pid & 0xFFFFFFFF, pid >> 32, gid], [seed & 0xFFFFFFFF, seed >> 32])
    w0 = int(o[1]) << 32 | int(o[0])
    w1 = int(o[3]) << 32 | int(o[2])
    m42 = (1 << 42) - 1
    return [w0 & m42, (w0 >> 42) | ((w1 & ((1 << 20) - 1)) << 22), (w1 >> 20) & m42]


def test_work_meter_hand_count_birth():
    """One birth and one collision in a box whose attenuation is so large
    that the first flight always ends in a collision, with a cap of one
    collision.  By hand: a position attempt is three uniforms (2 each) and
    three scalings (3 each) = 15, never rejected (the box is the domain);
    the box cell's containment 6; each direction attempt two uniforms (4),
    2u - 1 twice (4) and s = v1^2 + v2^2 (3) = 11; the accepted direction
    8 (square root of 1 - s, three scalings); the optical depth, one
    uniform 2 and the series logarithm 32; then the segment: three axis
    planes 6, tau / Sigma 1, move 6.  76 + 11 m operations for m direction
    attempts, which follow from the Philox blocks 1, 2, ... (Marsaglia's
    rejection of s >= 1)."""
    seed, gid, n = 77, 9, 40
    og = oracle.OracleGeometry(synth.box((1.0, 1.0, 1.0), sigma=1e12))
    p = oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid, max_collisions=1)
    ops, segs = oracle.count_work(og, p)
    want = 0
    for pid in range(n):
        m, blk = 0, 1
        while True:
            f = _philox_fields(seed, gid, pid, blk)
            v1 = 2.0 * ((f[0] + 0.5) * 2.0 ** -42) - 1.0
            v2 = 2.0 * ((f[1] + 0.5) * 2.0 ** -42) - 1.0
            m += 1
            blk += 1
            s = v1 * v1 + v2 * v2
            if s < 1.0 and s != 0.0:
                break
        want += 76 + 11 * m
    assert segs == n
    assert ops == want
    assert want != 87 * n   # some history needed a second direction attempt


def test_ray_volumes_hex_pins():
    """Hexagonal pins (three plane families, flat-to-flat 1.3) filling a box:
    for every pin whose hexagon lies inside the box, stratified rays give
    fuel and clad volumes pi r^2 * 200 and moderator ((sqrt3/2) p^2 -
    pi 0.5^2) * 200."""
    g = synth.hex_pin_box(6.0)
    og = oracle.OracleGeometry(g)
    vol, _ = _ray_volumes(g, og, 24000, 1)
    p, H = synth.HEX_PIN_PITCH, 200.0
    want = np.array([math.pi * 0.16, math.pi * (0.25 - 0.16), math.sqrt(3) / 2 * p * p - math.pi * 0.25]) * H
    ring = synth.hex_ring_cells(8)
    inside = 0
    for k, (i, j) in enumerate(ring):
        cx, cy = p * i * math.sqrt(3) / 2, p * (i / 2 + j)
        rc = p / math.sqrt(3)
        if abs(cx) + rc < 6.0 and abs(cy) + p / 2 < 6.0:
            assert np.allclose(vol[3 * k:3 * k + 3], want, rtol=2e-4), (k, vol[3 * k:3 * k + 3], want)
            inside += 1
    assert inside >= 40
    assert abs(vol.sum() - 12.0 * 12.0 * H) < 1e-6 * 12.0 * 12.0 * H
