"""The tracker's device functions compiled for the host (one-lane waves;
tests/cpu_build) against the oracle, bit for bit, on a CPU.  This covers the
per-lane logic of the HIP path -- birth sampling, searches with candidate
lists, hints and hierarchies, slab pairs, distances, crossings, tallies,
recording -- for every table staging kind, and the batched launch's
descriptors (fills, chunk groups, finalize), without a GPU.  The wave-level
scheduling (refill, tail compaction) is covered by the GPU tests.  A second
run under AddressSanitizer checks that no table or output is read or written
out of bounds."""

import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2406_13849_amd import gt, synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "cpu_build"))
import build as cpu_build  # noqa: E402


class HostLib:
    """The CPU build loaded with the binding's structures (a second ctypes
    handle; the GPU library is not touched)."""

    def __init__(self, path):
        L = C.CDLL(path)
        vp = C.c_void_p
        L.gt_geometry_create.argtypes = [C.POINTER(gt._Flat), C.POINTER(vp)]
        L.gt_geometry_info.argtypes = [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]
        L.gt_geometry_staging.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.gt_geometry_destroy.argtypes = [vp]
        L.gt_geometry_destroy.restype = None
        L.gt_last_error.restype = C.c_char_p
        L.cpu_track.argtypes = [vp, C.POINTER(gt._Params), C.POINTER(gt._Out), C.c_int]
        L.cpu_force_surface_set.argtypes = [C.c_int]
        L.cpu_force_surface_set.restype = None
        L.cpu_track_batch.argtypes = [C.POINTER(gt._BatchItem), C.c_uint32, C.POINTER(gt._Tuning),
                                      C.POINTER(C.c_uint32), C.c_uint32]
        L.cpu_track_mesh.argtypes = [vp, C.POINTER(gt._Params), C.POINTER(gt._Out), C.POINTER(gt._Mesh), C.c_int]
        L.gt_mesh_workspace_bytes.argtypes = [C.c_uint64]
        L.gt_mesh_workspace_bytes.restype = C.c_uint64
        self.L = L

    def check(self, rc):
        if rc != 0:
            raise gt.GtError(rc, (self.L.gt_last_error() or b"").decode())

    def geometry(self, fg):
        keep = []
        f = gt.flat_struct(fg, keep)
        h = C.c_void_p()
        self.check(self.L.gt_geometry_create(C.byref(f), C.byref(h)))
        ni, md, nb = C.c_uint64(), C.c_uint32(), C.c_uint64()
        self.check(self.L.gt_geometry_info(h, C.byref(ni), C.byref(md), C.byref(nb)))
        return h.value, int(ni.value)

    def staging(self, h, prec):
        k, b = C.c_uint32(), C.c_uint32()
        self.check(self.L.gt_geometry_staging(h, prec, C.byref(k), C.byref(b)))
        return int(k.value)


class Outs:
    def __init__(self, n_inst, n, k, cap):
        self.a = dict(tally_fx=np.zeros((n_inst, 2), np.uint64), tally=np.zeros(n_inst),
                      seg_count=np.zeros(n, np.uint32), seq_hash=np.zeros(n, np.uint64),
                      end_code=np.zeros(n, np.uint8), rec=np.full((max(k, 1), max(cap, 1)), -1, np.int32),
                      counters=np.zeros(8, np.uint64))

    def struct(self):
        a = self.a
        return gt._Out(tally_fx=a["tally_fx"].ctypes.data, tally=a["tally"].ctypes.data,
                       seg_count=a["seg_count"].ctypes.data, seq_hash=a["seq_hash"].ctypes.data,
                       end_code=a["end_code"].ctypes.data, rec=a["rec"].ctypes.data,
                       counters=a["counters"].ctypes.data)


def same(a, o, k):
    assert np.array_equal(a["seq_hash"], o.seq_hash)
    assert np.array_equal(a["seg_count"], o.seg_count)
    assert np.array_equal(a["end_code"], o.end_code)
    assert np.array_equal(a["tally_fx"], o.tally_fx)
    assert np.array_equal(a["tally"], o.tally_fxd)
    if k:
        assert np.array_equal(a["rec"], o.rec)
    names = ("escaped", "capped", "lost", "segcap", "rec_overflow", "segments", "rejected")
    assert {n: int(v) for n, v in zip(names, a["counters"])} == {n: o.counters[n] for n in names}


@pytest.fixture(scope="module")
def host():
    try:
        return HostLib(cpu_build.build())
    except RuntimeError as e:
        if str(e).startswith("no clang++"):
            pytest.skip(str(e))
        raise   # a build that fails is a failure, not a skip


GEOMS = [("cfg", 1), ("cfg", 2), ("cfg", 4), ("fn", "sphere"), ("fn", "nested_box"), ("fn", "deep_slabs"), ("batch", 3),
         ("batch", 5), ("batch", 41), ("batch", 57), ("batch", 2), ("batch", 63)]


def make(what, k):
    if what == "cfg":
        return synth.make_config(k), dict(seed=synth.particle_seed(k), geometry_id=k)
    if what == "fn":
        return getattr(synth, k)(), dict(seed=77, geometry_id=9)
    fg, _ = synth.batch_item(k)
    return fg, dict(seed=synth.batch_particle_seed(k), geometry_id=synth.batch_geometry_id(k))


@pytest.mark.parametrize("what,k", GEOMS, ids=["%s%s" % g for g in GEOMS])
def test_cpu_build_matches_oracle(host, what, k):
    """Every staging kind the geometry can be held in (its own and all
    global), both precisions, with and without the lane's tally cache, 400
    histories with recorded sequences; the code built for the geometry's own
    surface set and the code built for every surface type."""
    fg, kw = make(what, k)
    h, ni = host.geometry(fg)
    n, rk, cap = 400, 30, 48
    o = oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(n_particles=n, record_first_k=rk,
                                                                    record_cap=cap, **kw), n_threads=4)
    try:
        for sf in (-1, 0):
            host.L.cpu_force_surface_set(sf)
            for prec in (gt.PREC_FP64, gt.PREC_MIXED):
                for kind in sorted({0, host.staging(h, prec)}):
                    for cache in ((True, False) if kind else (True,)):
                        out = Outs(ni, n, rk, cap)
                        prm = gt._params(kw["seed"], n, geometry_id=kw["geometry_id"], precision=prec,
                                         record_first_k=rk, record_cap=cap, tally_cache=cache)
                        host.check(host.L.cpu_track(h, C.byref(prm), C.byref(out.struct()), kind))
                        same(out.a, o, rk)
    finally:
        host.L.cpu_force_surface_set(-1)
    host.L.gt_geometry_destroy(h)


@pytest.mark.parametrize("what,k", [("cfg", 1), ("cfg", 2), ("cfg", 4)])
def test_cpu_ray_source_matches_oracle(host, what, k):
    """The parallel-ray source (no collisions) through the lane's state
    machine, which runs it in the build for every surface type: the oracle's
    histories and tallies, both precisions."""
    fg, kw = make(what, k)
    h, ni = host.geometry(fg)
    n1 = 600
    n, rk, cap = 3 * n1, 20, 48
    kw = dict(seed=0, geometry_id=kw["geometry_id"], source=1, ray_n1=n1, max_collisions=1)
    o = oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(n_particles=n, record_first_k=rk, record_cap=cap,
                                                                    **kw), n_threads=4)
    for prec in (gt.PREC_FP64, gt.PREC_MIXED):
        out = Outs(ni, n, rk, cap)
        prm = gt._params(0, n, geometry_id=kw["geometry_id"], precision=prec, record_first_k=rk, record_cap=cap,
                         source=1, ray_n1=n1, max_collisions=1)
        host.check(host.L.cpu_track(h, C.byref(prm), C.byref(out.struct()), host.staging(h, prec)))
        same(out.a, o, rk)
    host.L.gt_geometry_destroy(h)


@pytest.mark.parametrize("what,k", [("cfg", 1), ("cfg", 2), ("cfg", 4), ("fn", "sphere"), ("fn", "nested_box"),
                                     ("batch", 41)],
                         ids=["cfg1", "cfg2", "cfg4", "sphere", "nested_box", "batch41"])
def test_cpu_event_schedule_matches_oracle(host, what, k):
    """The event-based schedule's steps, run one history at a time over a
    bank in host memory, give the oracle's histories and tallies (both
    precisions)."""
    fg, kw = make(what, k)
    h, ni = host.geometry(fg)
    n, rk, cap = 300, 25, 48
    o = oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(n_particles=n, record_first_k=rk,
                                                                    record_cap=cap, **kw), n_threads=4)
    host.L.cpu_track_event.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    for prec in (gt.PREC_FP64, gt.PREC_MIXED):
        out = Outs(ni, n, rk, cap)
        prm = gt._params(kw["seed"], n, geometry_id=kw["geometry_id"], precision=prec, record_first_k=rk,
                         record_cap=cap)
        host.check(host.L.cpu_track_event(h, C.byref(prm), C.byref(out.struct())))
        same(out.a, o, rk)
    host.L.gt_geometry_destroy(h)


def test_cpu_build_covers_every_staging_kind(host):
    kinds = set()
    for what, k in GEOMS:
        fg, _ = make(what, k)
        h, _ = host.geometry(fg)
        kinds.add(host.staging(h, gt.PREC_MIXED))
        host.L.gt_geometry_destroy(h)
    assert kinds == {0, 1, 2, 3}


def batch_run(host, items_spec, prec, chunk, groups=1):
    arr = (gt._BatchItem * len(items_spec))()
    outs, want, hs = [], [], []
    for i, (j, n, staging) in enumerate(items_spec):
        fg, kw = make("batch", j)
        h, ni = host.geometry(fg)
        hs.append(h)
        out = Outs(ni, n, 20, 32)
        outs.append(out)
        arr[i].geometry = h
        arr[i].params = gt._params(kw["seed"], n, geometry_id=kw["geometry_id"], precision=prec, record_first_k=20,
                                   record_cap=32, staging=staging)
        arr[i].out = out.struct()
        want.append(oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(n_particles=n, record_first_k=20,
                                                                                 record_cap=32, **kw), n_threads=4))
    ran = C.c_uint32()
    host.check(host.L.cpu_track_batch(arr, len(items_spec), C.byref(gt._Tuning(0, 0, chunk)), C.byref(ran), groups))
    for out, o in zip(outs, want):
        same(out.a, o, 20)
    for h in hs:
        host.L.gt_geometry_destroy(h)
    return ran.value


@pytest.mark.parametrize("prec", [gt.PREC_FP64, gt.PREC_MIXED])
def test_cpu_batch_descriptors(host, prec):
    """A batch of items of every staging kind (and some forced global), with
    small ragged chunks: the chunk groups by staging kind cover every chunk
    exactly once, and every item's outputs equal the oracle's."""
    spec = [(57, 700, True), (3, 500, True), (5, 450, True), (2, 380, True), (41, 333, False), (63, 300, True)]
    ran = batch_run(host, spec, prec, 97)
    assert ran == sum((n + 96) // 97 for _, n, _ in spec)


@pytest.mark.parametrize("prec", [gt.PREC_FP64, gt.PREC_MIXED])
@pytest.mark.parametrize("groups", [1, 3, 40])
def test_cpu_batch_whole_items(host, prec, groups):
    """Whole items (chunk = 0): the item groups by staging kind, the first
    choice of every workgroup, the later choices and the shared claim
    counters cover every item's histories exactly once, every workgroup
    leaves its items (the driver checks the counters), and every item's
    outputs equal the oracle's; one item with no histories and more
    workgroups than items included."""
    spec = [(57, 700, True), (3, 500, True), (5, 450, True), (2, 0, True), (41, 333, False), (63, 300, True)]
    ran = batch_run(host, spec, prec, 0, groups)
    busy = sum(1 for _, n, _ in spec if n)
    # each item drained in one visit; at most one empty visit per workgroup and kind
    # (several workgroups: some first choices land on items drained before them)
    assert busy <= ran <= busy + 4 * groups and (groups == 1 or ran > busy)


def test_cpu_build_under_address_sanitizer():
    """The same per-lane logic, event-based steps and batch planner with
    AddressSanitizer, in a child process (the sanitizer runtime must be
    loaded first)."""
    try:
        lib = cpu_build.build(asan=True)
    except RuntimeError as e:
        if str(e).startswith("no clang++"):
            pytest.skip(str(e))
        raise
    rt = cpu_build.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime")
    code = r"""
import sys, ctypes as C
sys.path.insert(0, %r); sys.path.insert(0, %r)
import test_cpu_build as t
host = t.HostLib(%r)
for what, k in [("cfg", 2), ("batch", 3), ("batch", 5), ("batch", 2)]:
    fg, kw = t.make(what, k)
    h, ni = host.geometry(fg)
    for prec in (0, 1):
        for kind in sorted({0, host.staging(h, prec)}):
            out = t.Outs(ni, 200, 10, 16)
            prm = t.gt._params(kw["seed"], 200, geometry_id=kw["geometry_id"], precision=prec, record_first_k=10,
                               record_cap=16)
            host.check(host.L.cpu_track(h, C.byref(prm), C.byref(out.struct()), kind))
        out = t.Outs(ni, 150, 10, 16)
        prm = t.gt._params(kw["seed"], 150, geometry_id=kw["geometry_id"], precision=prec, record_first_k=10,
                           record_cap=16)
        host.L.cpu_track_event.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        host.check(host.L.cpu_track_event(h, C.byref(prm), C.byref(out.struct())))
        if what == "cfg":   # the mesh walk, over a corner of the domain and over more than it
            lo, hi = fg.domain_lo, fg.domain_hi
            t.mesh_run(host, h, ni, kw, prec, lo + 0.3 * (hi - lo), lo + 0.8 * (hi - lo), (9, 4, 6), 150, 10, 16)
            t.mesh_run(host, h, ni, kw, prec, lo - 1.0, hi + 2.0, (5, 7, 3), 150, 10, 16)
    host.L.gt_geometry_destroy(h)
t.batch_run(host, [(57, 300, True), (5, 200, True), (41, 150, False)], 1, 64)
t.batch_run(host, [(57, 300, True), (5, 200, True), (41, 150, False)], 1, 0, 3)
print("asan clean")
""" % (os.path.dirname(HERE), HERE, lib)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "asan clean" in r.stdout, (r.stdout[-2000:] + r.stderr[-4000:])


def test_event_bank_layout(host):
    """gt_event_bank_bytes: 256-byte multiples growing with the particle
    count, 0 above the particle limit (host-only arithmetic)."""
    f = host.L.gt_event_bank_bytes
    f.argtypes = [C.c_uint64]
    f.restype = C.c_uint64
    prev = 0
    for n in (0, 1, 255, 256, 1000, 10**6):
        b = f(n)
        assert b % 256 == 0 and b >= prev and b >= 152 * n
        prev = b
    assert f(0x7FFFFFFF * 64 + 1) == 0


def mesh_run(host, h, ni, kw, prec, lo, hi, bins, n, rk, cap):
    """cpu_track_mesh in host memory: (outputs, mesh_fx, mesh)."""
    nb = int(np.prod(bins))
    out = Outs(ni, n, rk, cap)
    mfx, msum = np.zeros((nb, 2), np.uint64), np.zeros(nb)
    ws = np.zeros(int(host.L.gt_mesh_workspace_bytes(nb)) // 8, np.uint64)
    m = gt._Mesh(mesh_fx=mfx.ctypes.data, mesh=msum.ctypes.data, workspace=ws.ctypes.data,
                 workspace_bytes=ws.nbytes)
    m.lo[:] = [float(v) for v in lo]
    m.hi[:] = [float(v) for v in hi]
    m.n[:] = list(bins)
    prm = gt._params(kw["seed"], n, geometry_id=kw["geometry_id"], precision=prec, record_first_k=rk,
                     record_cap=cap)
    host.check(host.L.cpu_track_mesh(h, C.byref(prm), C.byref(out.struct()), C.byref(m), host.staging(h, prec)))
    return out, mfx, msum


MESH_CASES = [
    (("cfg", 1), "domain", (7, 5, 3)),
    (("cfg", 2), "domain", (17, 17, 10)),
    (("cfg", 2), "corner", (9, 4, 6)),
    (("fn", "sphere"), "domain", (3, 4, 5)),
    (("fn", "nested_box"), "domain", (4, 4, 1)),
]


@pytest.mark.parametrize("geom,cover,bins", MESH_CASES,
                         ids=["%s%s-%s-%dx%dx%d" % (g[0], g[1], c, *b) for g, c, b in MESH_CASES])
def test_cpu_mesh_tally_matches_oracle(host, geom, cover, bins):
    """The kernel's mesh walk (per-axis runs of planes merged in order of t,
    midpoint binning) gives the oracle's mesh tally bit for bit, with the
    histories and cell tallies unchanged; a mesh over the whole domain or over
    a corner of it, both precisions, the geometry's own staging kind."""
    fg, kw = make(*geom)
    h, ni = host.geometry(fg)
    lo, hi = fg.domain_lo.copy(), fg.domain_hi.copy()
    if cover == "corner":
        lo, hi = lo + 0.3 * (hi - lo), lo + 0.8 * (hi - lo)
    n, rk, cap = 300, 10, 48
    o = oracle.track(oracle.OracleGeometry(fg), oracle.TrackParams(n_particles=n, record_first_k=rk,
                                                                    record_cap=cap, **kw),
                     n_threads=4, mesh=(lo, hi, bins))
    for prec in (gt.PREC_FP64, gt.PREC_MIXED):
        out, mfx, msum = mesh_run(host, h, ni, kw, prec, lo, hi, bins, n, rk, cap)
        same(out.a, o, rk)
        assert np.array_equal(mfx, o.mesh_fx), (geom, cover, prec)
        assert np.array_equal(msum, o.mesh_fxd)
        assert (mfx[:, 1] > 0).sum() > 0
    host.L.gt_geometry_destroy(h)


def _mesh_segment_cases(rng, lo, hi, n, count):
    """Segments whose ends fall exactly on a mesh plane's cut, one ulp to
    either side of it, or anywhere; directions with zero, tiny and subnormal
    components as well as random ones."""
    lo, hi, n = np.asarray(lo, float), np.asarray(hi, float), np.asarray(n)
    w = (hi - lo) / n
    p0 = rng.uniform(lo - 0.2 * w, hi + 0.2 * w, size=(count, 3))
    u = rng.normal(size=(count, 3))
    kinds = rng.integers(0, 6, size=count)
    u[kinds == 1, rng.integers(0, 3)] = 0.0                      # one axis not moving
    u[kinds == 2, 2] = 1e-300                                   # a component far below the rest
    u[kinds == 3, 1] = 4e-320                                   # a subnormal component
    u /= np.linalg.norm(u, axis=1)[:, None]
    l = rng.uniform(0.0, 3.0, size=count) * w.max()
    # end the segment on the cut of a plane it crosses (as the walk computes
    # it), or one ulp short of or past that cut
    a = rng.integers(0, 3, size=count)
    ua = u[np.arange(count), a]
    pa = p0[np.arange(count), a]
    k = np.floor((pa - lo[a]) / w[a]) + np.where(ua > 0, 1 + rng.integers(0, 3, size=count),
                                                    -rng.integers(0, 3, size=count))
    with np.errstate(over="ignore"):
        t = ((lo[a] + k * w[a]) - pa) / np.where(ua == 0.0, 1.0, ua)
    on = (kinds >= 4) & (ua != 0.0) & (t > 0)
    nudge = rng.integers(-1, 2, size=count)
    tt = np.where(nudge < 0, np.nextafter(t, -np.inf), np.where(nudge > 0, np.nextafter(t, np.inf), t))
    l = np.where(on, tt, l)
    l[rng.integers(0, count, size=count // 50)] = 0.0            # empty segments
    return p0, u, l


def test_mesh_walk_matches_oracle_on_plane_edges(host):
    """The kernel's mesh walk (the first cut ahead per axis found without
    dividing, divisions skipped for cuts certainly past the segment's end)
    gives the oracle's mesh tally bit for bit on segments that end exactly on
    a plane's cut or one ulp from it, that run along an axis, or whose
    direction has a tiny or subnormal component, on meshes of the
    benchmark's and of odd widths."""
    rng = np.random.default_rng(23)
    fn = host.L.cpu_mesh_segments
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p,
                   C.c_void_p]
    fn.restype = C.c_int
    for lo, hi, n in (((-140.0, -140.0, -183.0), (140.0, 140.0, 183.0), (119, 119, 30)),
                      ((-10.625, -10.625, -1.0), (10.625, 10.625, 1.0), (17, 17, 3)),
                      ((-3.3, 0.0, -2.5), (7.1, 1.0, 9.25), (13, 3, 7))):
        p0, u, l = _mesh_segment_cases(rng, lo, hi, n, 40000)
        want = oracle.mesh_segments((lo, hi, n), p0, u, l)
        got = np.zeros_like(want)
        lo_a, hi_a = np.array(lo, float), np.array(hi, float)
        n_a = np.array(n, np.uint32)
        assert fn(lo_a.ctypes.data, hi_a.ctypes.data, n_a.ctypes.data, l.size, p0.ctypes.data, u.ctypes.data,
                  l.ctypes.data, got.ctypes.data) == 0
        assert np.array_equal(got, want), (lo, hi, n)
        assert (want[:, 1] > 0).sum() > 100


def test_mesh_floor_matches_division(host):
    """The mesh walk's bin index from the reciprocal (with the division as
    the fallback near integers) equals floor(d / w) for coordinates on, next
    to and between the planes of meshes of the benchmark's and odd widths."""
    rng = np.random.default_rng(11)
    host.L.cpu_mesh_floor.argtypes = [C.c_void_p, C.c_uint64, C.c_double, C.c_void_p]
    host.L.cpu_mesh_floor.restype = None
    for lo, hi, n in ((-140.0, 140.0, 119), (-100.0, 100.0, 30), (-10.625, 10.625, 17), (0.0, 1.0, 3),
                      (-1.875, 1.875, 7), (-3.3, 7.1, 113)):
        w = (hi - lo) / n
        k = rng.integers(-2, n + 3, size=20000).astype(np.float64)
        planes = lo + k * w
        near = np.concatenate([planes, np.nextafter(planes, np.inf), np.nextafter(planes, -np.inf),
                               np.nextafter(np.nextafter(planes, np.inf), np.inf),
                               planes + rng.uniform(-1e-12, 1e-12, planes.size),
                               rng.uniform(lo - w, hi + w, 40000)])
        d = near - lo
        out = np.empty_like(d)
        host.L.cpu_mesh_floor(d.ctypes.data, d.size, w, out.ctypes.data)
        assert np.array_equal(out, np.floor(d / w)), (lo, hi, n)
