"""Python binding of libgt.so (the C ABI declared in include/gt.h).

Argument marshalling only: every step of the tracking runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.
There is no fallback: if the library is not built, or there is no GPU, the
calls raise.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgt.so")

GT_OK, GT_EINVAL, GT_EGEOM, GT_ENOMEM, GT_EHIP, GT_ECAPACITY = 0, -1, -2, -3, -4, -5
MAX_LEVELS = 6
PREC_FP64, PREC_MIXED = 0, 1
FLAG_ACCUMULATE = 1
FLAG_LANE_PER_HISTORY = 2
FLAG_NO_STAGING = 4
FLAG_TAIL_COMPACTION = 8
FLAG_NO_TALLY_CACHE = 16
FLAG_TRACKER_SP = 32
FLAG_TRACKER_RTK = 64
TRACKER_FLAGS = {"st": 0, "sp": FLAG_TRACKER_SP, "rtk": FLAG_TRACKER_RTK}
END_NONE, END_ESCAPE, END_CAP, END_LOST, END_SEGCAP = 0, 1, 2, 3, 4
COUNTERS = ("escaped", "capped", "lost", "segcap", "rec_overflow", "segments", "rejected", "spare")


class GtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libgt error %d: %s" % (code, msg))
        self.code = code


class _Flat(C.Structure):
    _fields_ = [
        ("n_surfaces", C.c_uint32), ("n_cells", C.c_uint32), ("n_universes", C.c_uint32),
        ("n_materials", C.c_uint32), ("n_halfspaces", C.c_uint32), ("root", C.c_uint32),
        ("surf_type", C.c_void_p), ("surf_coef", C.c_void_p), ("cell_hs_off", C.c_void_p),
        ("hs", C.c_void_p), ("cell_fill", C.c_void_p), ("cell_trans", C.c_void_p),
        ("univ_cell_off", C.c_void_p), ("lattice_hint", C.c_void_p), ("sigma_t", C.c_void_p),
        ("domain_lo", C.c_double * 3), ("domain_hi", C.c_double * 3),
    ]


class _Params(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64), ("first_particle", C.c_uint64), ("n_particles", C.c_uint64),
        ("geometry_id", C.c_uint32), ("max_collisions", C.c_uint32), ("source", C.c_uint32),
        ("ray_n1", C.c_uint32), ("max_segments", C.c_uint32), ("precision", C.c_uint32),
        ("record_first_k", C.c_uint32), ("record_cap", C.c_uint32), ("flags", C.c_uint32),
        ("block_size", C.c_uint32), ("refill_min", C.c_uint32), ("regroup_every", C.c_uint32),
        ("wave_histories", C.c_uint32),
    ]


class _Out(C.Structure):
    _fields_ = [
        ("tally_fx", C.c_void_p), ("tally", C.c_void_p), ("seg_count", C.c_void_p),
        ("seq_hash", C.c_void_p), ("end_code", C.c_void_p), ("rec", C.c_void_p), ("counters", C.c_void_p),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_uint64),
    ]


class _BatchItem(C.Structure):
    _fields_ = [("geometry", C.c_void_p), ("params", _Params), ("out", _Out)]


class _Tuning(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("refill_min", C.c_uint32), ("chunk", C.c_uint64),
                ("regroup_every", C.c_uint32), ("wave_histories", C.c_uint32)]


class _Mesh(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3), ("n", C.c_uint32 * 3), ("reserved", C.c_uint32),
                ("mesh_fx", C.c_void_p), ("mesh", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_uint64)]


class _LaunchInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("workgroups", "block_size", "lds_bytes", "staging_kind",
                                          "tally_cache_entries", "tail_capacity", "regroup_every", "surface_set")]


_lib = None


def lib():
    """Load libgt.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgt.so is not built (run paper_2406_13849_amd/build.py or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32, i32 = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int
        L.gt_geometry_create.argtypes = [C.POINTER(_Flat), C.POINTER(vp)]
        L.gt_geometry_create.restype = i32
        L.gt_geometry_info.argtypes = [vp, C.POINTER(u64), C.POINTER(u32), C.POINTER(u64)]
        L.gt_geometry_info.restype = i32
        L.gt_geometry_staging.argtypes = [vp, u32, C.POINTER(u32), C.POINTER(u32)]
        L.gt_geometry_staging.restype = i32
        L.gt_geometry_kinds.argtypes = [vp, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.gt_geometry_kinds.restype = i32
        L.gt_geometry_destroy.argtypes = [vp]
        L.gt_geometry_destroy.restype = None
        L.gt_track.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Out), vp]
        L.gt_track.restype = i32
        L.gt_track_noalloc.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Out), vp]
        L.gt_track_noalloc.restype = i32
        L.gt_track_workspace_bytes.argtypes = [vp]
        L.gt_track_workspace_bytes.restype = u64
        L.gt_event_bank_bytes.argtypes = [u64]
        L.gt_event_bank_bytes.restype = u64
        L.gt_track_event.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Out), vp, u64, vp]
        L.gt_track_event.restype = i32
        L.gt_batch_create.argtypes = [C.POINTER(_BatchItem), u32, C.POINTER(_Tuning), C.POINTER(vp)]
        L.gt_batch_create.restype = i32
        L.gt_batch_launch.argtypes = [vp, vp]
        L.gt_batch_launch.restype = i32
        L.gt_batch_destroy.argtypes = [vp]
        L.gt_batch_destroy.restype = None
        L.gt_last_launch.argtypes = [C.POINTER(_LaunchInfo)]
        L.gt_last_launch.restype = i32
        L.gt_mesh_workspace_bytes.argtypes = [u64]
        L.gt_mesh_workspace_bytes.restype = u64
        L.gt_track_mesh.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Out), C.POINTER(_Mesh), vp]
        L.gt_track_mesh.restype = i32
        L.gt_track_batch.argtypes = [C.POINTER(_BatchItem), u32, C.POINTER(_Tuning), vp]
        L.gt_track_batch.restype = i32
        L.gt_autotune_track.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Out), u32, vp, C.POINTER(_Tuning),
                                        C.POINTER(C.c_float)]
        L.gt_autotune_track.restype = i32
        L.gt_tuning_lookup.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Tuning)]
        L.gt_tuning_lookup.restype = i32
        L.gt_autotune_batch.argtypes = [C.POINTER(_BatchItem), u32, u32, vp, C.POINTER(_Tuning),
                                        C.POINTER(C.c_float)]
        L.gt_autotune_batch.restype = i32
        L.gt_set_kernel_events.argtypes = [vp, vp]
        L.gt_set_kernel_events.restype = i32
        L.gt_find_cell.argtypes = [vp, vp, u64, vp, vp, u32, vp]
        L.gt_find_cell.restype = i32
        L.gt_distance_to_surface.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp]
        L.gt_distance_to_surface.restype = i32
        L.gt_fp64_check.argtypes = [vp, vp, u64, vp, vp, vp, vp]
        L.gt_fp64_check.restype = i32
        L.gt_last_error.argtypes = []
        L.gt_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != GT_OK:
        raise GtError(rc, (lib().gt_last_error() or b"").decode())


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def flat_struct(g, keep: list) -> _Flat:
    """Marshal a FlatGeometry (numpy arrays) into the ABI struct; `keep`
    holds the contiguous arrays alive for the duration of the call."""
    arrs = [np.ascontiguousarray(g.surf_type, np.uint8), np.ascontiguousarray(g.surf_coef, np.float64),
            np.ascontiguousarray(g.cell_hs_off, np.uint32), np.ascontiguousarray(g.hs, np.int32),
            np.ascontiguousarray(g.cell_fill, np.int32), np.ascontiguousarray(g.cell_trans, np.float64),
            np.ascontiguousarray(g.univ_cell_off, np.uint32),
            None if g.lattice_hint is None else np.ascontiguousarray(g.lattice_hint, np.float64),
            np.ascontiguousarray(g.sigma_t, np.float64)]
    keep.extend(arrs)
    st, sc, ho, hs, cf, ct, uo, lh, sg = arrs

    def p(a):
        return None if a is None or a.size == 0 else a.ctypes.data

    f = _Flat(n_surfaces=st.shape[0], n_cells=cf.shape[0], n_universes=uo.shape[0] - 1, n_materials=sg.shape[0],
              n_halfspaces=hs.shape[0], root=int(g.root), surf_type=p(st), surf_coef=p(sc), cell_hs_off=p(ho),
              hs=p(hs), cell_fill=p(cf), cell_trans=p(ct), univ_cell_off=p(uo), lattice_hint=p(lh), sigma_t=p(sg))
    f.domain_lo[:] = [float(v) for v in g.domain_lo]
    f.domain_hi[:] = [float(v) for v in g.domain_hi]
    return f


class Geometry:
    """A flattened geometry uploaded to the current HIP device."""

    def __init__(self, g):
        keep: list = []
        f = flat_struct(g, keep)
        h = C.c_void_p()
        _check(lib().gt_geometry_create(C.byref(f), C.byref(h)))
        self.h = h
        ni, md, nb = C.c_uint64(), C.c_uint32(), C.c_uint64()
        _check(lib().gt_geometry_info(h, C.byref(ni), C.byref(md), C.byref(nb)))
        self.n_instances = int(ni.value)
        self.max_depth = int(md.value)
        self.device_bytes = int(nb.value)

    def staging(self, precision: int = PREC_MIXED):
        """gt_geometry_staging: (kind, LDS bytes) of the persistent trackers'
        copy of the tables (kind 0 none, 1 per-segment, 2 + crossing, 3 all)."""
        k, b = C.c_uint32(), C.c_uint32()
        _check(lib().gt_geometry_staging(self.h, precision, C.byref(k), C.byref(b)))
        return int(k.value), int(b.value)

    def kinds(self):
        """gt_geometry_kinds: (rectilinear arrays, pins, fixed-depth shape;
        0 = not trackable with tracker="rtk")."""
        r, p, s = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().gt_geometry_kinds(self.h, C.byref(r), C.byref(p), C.byref(s)))
        return int(r.value), int(p.value), int(s.value)

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.gt_geometry_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


@dataclass
class TrackOutputs:
    """Device tensors written by gt_track (int64 tensors hold uint64 bits)."""
    tally_fx: "object"    # int64 [n_inst, 2]
    tally: "object"       # float64 [n_inst]
    seg_count: "object"   # int32 [n]
    seq_hash: "object"    # int64 [n]
    end_code: "object"    # uint8 [n]
    rec: "object"         # int32 [k, cap] or None
    counters: "object"    # int64 [8]
    workspace: "object" = None   # uint8 [gt_track_workspace_bytes] or None (the geometry's own)

    def counters_dict(self) -> dict:
        c = self.counters.cpu().numpy().view(np.uint64)
        return {k: int(v) for k, v in zip(COUNTERS, c)}


def track_workspace_bytes(geom: Geometry) -> int:
    """gt_track_workspace_bytes: device bytes of a tracking call's tally workspace."""
    return int(lib().gt_track_workspace_bytes(geom.h))


def alloc_outputs(geom: Geometry, n: int, record_first_k: int = 0, record_cap: int = 0, device="cuda",
                  per_particle: bool = True, workspace: bool = False) -> TrackOutputs:
    """Output tensors for n histories; workspace=True also gives the call a
    tally workspace of its own (so calls on one geometry may overlap)."""
    import torch
    ni = geom.n_instances
    return TrackOutputs(
        tally_fx=torch.zeros((ni, 2), dtype=torch.int64, device=device),
        tally=torch.zeros(ni, dtype=torch.float64, device=device),
        seg_count=torch.zeros(n, dtype=torch.int32, device=device) if per_particle else None,
        seq_hash=torch.zeros(n, dtype=torch.int64, device=device) if per_particle else None,
        end_code=torch.zeros(n, dtype=torch.uint8, device=device) if per_particle else None,
        rec=torch.full((record_first_k, record_cap), -1, dtype=torch.int32, device=device)
        if record_first_k else None,
        counters=torch.zeros(8, dtype=torch.int64, device=device),
        workspace=torch.empty(track_workspace_bytes(geom), dtype=torch.uint8, device=device) if workspace else None,
    )


def track(geom: Geometry, seed: int, n_particles: int, *, first_particle: int = 0, geometry_id: int = 0,
          max_collisions: int = 20, source: int = 0, ray_n1: int = 0, max_segments: int = 100_000,
          precision: int = PREC_MIXED, record_first_k: int = 0, record_cap: int = 0, accumulate: bool = False,
          lane_per_history: bool = False, staging: bool = True, block_size: int = 0, refill_min: int = 0,
          tail_compaction: bool = False, tally_cache: bool = True, regroup_every: int = 0, tracker: str = "st",
          wave_histories: int = 0, out: Optional[TrackOutputs] = None, stream=None) -> TrackOutputs:
    """gt_track: sample and track n_particles histories (asynchronous).
    lane_per_history selects the plain one-history-per-lane schedule instead
    of the persistent refilling one; staging=False keeps the geometry tables
    in global memory even when they fit in LDS; tail_compaction=True packs
    the histories left after the queue has drained into fewer waves; tally_cache=False
    flushes a lane's tally sum at every change of instance; regroup_every=R
    sorts a workgroup's histories by leaf universe every R loop trips;
    tracker selects the tracker method: "st" the single tracker (default),
    "sp" one tracker per universe kind switched per level, "rtk" the
    fixed-depth reactor tracker (GT_FLAG_TRACKER_*); wave_histories is the
    number of histories a wavefront claims from the queue at once (a
    multiple of 64; 0 = 64)."""
    if out is None:
        out = alloc_outputs(geom, n_particles, record_first_k, record_cap)
    prm = _params(seed, n_particles, first_particle, geometry_id, max_collisions, source, ray_n1, max_segments,
                  precision, record_first_k, record_cap, accumulate, lane_per_history, staging, block_size,
                  refill_min, tail_compaction, tally_cache, regroup_every, tracker, wave_histories)
    o = _out_struct(out)
    _check(lib().gt_track(geom.h, C.byref(prm), C.byref(o), _stream(stream)))
    return out



NOALLOC_SCRATCH_BYTES = 32 << 20   # GT_NOALLOC_SCRATCH_BYTES


def track_noalloc(geom: Geometry, seed: int, n_particles: int, *, out: TrackOutputs, stream=None,
                  **kwargs) -> TrackOutputs:
    """gt_track_noalloc: gt_track with the tally workspace in the library's
    fixed per-GPU scratch array (no device allocation in the call).  The
    caller brings every output (`out`, without a workspace); the keyword
    arguments are those of track()."""
    if getattr(out, "workspace", None) is not None:
        raise ValueError("track_noalloc: the outputs must not carry a workspace")
    prm = _params(seed, n_particles, **kwargs)
    o = _out_struct(out)
    _check(lib().gt_track_noalloc(geom.h, C.byref(prm), C.byref(o), _stream(stream)))
    return out

@dataclass
class MeshOutputs:
    """Device outputs of a mesh tally: mesh_fx [bins, 2] int64 (the (low,
    high) words of 128-bit fixed point, quantum 2^-96 cm), mesh [bins]
    float64 (cm), and the caller-owned workspace."""
    mesh_fx: object
    mesh: object
    workspace: object


def mesh_workspace_bytes(bins: int) -> int:
    """gt_mesh_workspace_bytes: device bytes of a mesh tally's workspace."""
    return int(lib().gt_mesh_workspace_bytes(bins))


def alloc_mesh(bins: int, device="cuda") -> MeshOutputs:
    import torch
    ws = mesh_workspace_bytes(bins)
    if ws == 0:
        raise GtError(GT_ECAPACITY, "mesh of %d bins" % bins)
    return MeshOutputs(mesh_fx=torch.zeros((bins, 2), dtype=torch.int64, device=device),
                       mesh=torch.zeros(bins, dtype=torch.float64, device=device),
                       workspace=torch.empty(ws, dtype=torch.uint8, device=device))


def track_mesh(geom: Geometry, seed: int, n_particles: int, mesh_lo, mesh_hi, mesh_n, *,
               out: Optional[TrackOutputs] = None, mesh_out: Optional[MeshOutputs] = None, stream=None,
               **kwargs):
    """gt_track_mesh: the histories and outputs of track() plus a track-length
    tally on a regular mesh of mesh_n = (nx, ny, nz) bins over [mesh_lo,
    mesh_hi] (bin (ix, iy, iz) at (iz * ny + iy) * nx + ix).  kwargs as
    track() (persistent schedule).  Returns (out, mesh_out)."""
    if out is None:
        out = alloc_outputs(geom, n_particles, kwargs.get("record_first_k", 0), kwargs.get("record_cap", 0))
    bins = int(mesh_n[0]) * int(mesh_n[1]) * int(mesh_n[2])
    if mesh_out is None:
        mesh_out = alloc_mesh(bins)
    m = _Mesh(mesh_fx=_ptr(mesh_out.mesh_fx), mesh=_ptr(mesh_out.mesh), workspace=_ptr(mesh_out.workspace),
              workspace_bytes=mesh_out.workspace.numel())
    m.lo[:] = [float(v) for v in mesh_lo]
    m.hi[:] = [float(v) for v in mesh_hi]
    m.n[:] = [int(v) for v in mesh_n]
    prm = _params(seed, n_particles, **kwargs)
    _check(lib().gt_track_mesh(geom.h, C.byref(prm), C.byref(_out_struct(out)), C.byref(m), _stream(stream)))
    return out, mesh_out


def event_bank_bytes(n_particles: int) -> int:
    """gt_event_bank_bytes: device bytes of the event-based schedule's bank."""
    return int(lib().gt_event_bank_bytes(n_particles))


def track_event(geom: Geometry, seed: int, n_particles: int, *, bank=None, out: Optional[TrackOutputs] = None,
                stream=None, **kwargs) -> TrackOutputs:
    """gt_track_event: the same histories and outputs as track(), by the
    event-based schedule (one kernel per operation per iteration over a
    particle bank in device memory; waits for the stream).  kwargs as
    track() (first_particle, geometry_id, max_collisions, source, ray_n1,
    max_segments, precision, record_first_k, record_cap, accumulate)."""
    import torch
    if out is None:
        out = alloc_outputs(geom, n_particles, kwargs.get("record_first_k", 0), kwargs.get("record_cap", 0))
    need = event_bank_bytes(n_particles)
    if bank is None:
        bank = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    prm = _params(seed, n_particles, **kwargs)
    o = _out_struct(out)
    _check(lib().gt_track_event(geom.h, C.byref(prm), C.byref(o), _ptr(bank), bank.numel(), _stream(stream)))
    return out


def _params(seed, n_particles, first_particle=0, geometry_id=0, max_collisions=20, source=0, ray_n1=0,
            max_segments=100_000, precision=PREC_MIXED, record_first_k=0, record_cap=0, accumulate=False,
            lane_per_history=False, staging=True, block_size=0, refill_min=0, tail_compaction=False,
            tally_cache=True, regroup_every=0, tracker="st", wave_histories=0) -> _Params:
    if tracker not in TRACKER_FLAGS:
        raise ValueError("tracker must be one of %s" % sorted(TRACKER_FLAGS))
    return _Params(seed=seed, first_particle=first_particle, n_particles=n_particles, geometry_id=geometry_id,
                   max_collisions=max_collisions, source=source, ray_n1=ray_n1, max_segments=max_segments,
                   precision=precision, record_first_k=record_first_k, record_cap=record_cap,
                   flags=(FLAG_ACCUMULATE if accumulate else 0) | (FLAG_LANE_PER_HISTORY if lane_per_history else 0)
                   | (0 if staging else FLAG_NO_STAGING) | (FLAG_TAIL_COMPACTION if tail_compaction else 0)
                   | (0 if tally_cache else FLAG_NO_TALLY_CACHE) | TRACKER_FLAGS[tracker],
                   block_size=block_size, refill_min=refill_min, regroup_every=regroup_every,
                   wave_histories=wave_histories)


def _out_struct(out: TrackOutputs) -> _Out:
    ws = getattr(out, "workspace", None)
    return _Out(tally_fx=_ptr(out.tally_fx), tally=_ptr(out.tally), seg_count=_ptr(out.seg_count),
                seq_hash=_ptr(out.seq_hash), end_code=_ptr(out.end_code), rec=_ptr(out.rec),
                counters=_ptr(out.counters), workspace=_ptr(ws), workspace_bytes=0 if ws is None else ws.numel())


@dataclass
class BatchItem:
    """One (geometry, histories) pair of a batch: the keyword arguments of
    track() except the schedule options, plus the output tensors."""
    geom: Geometry
    seed: int
    n_particles: int
    out: TrackOutputs
    kwargs: dict


class Batch:
    """gt_batch_create / gt_batch_launch / gt_batch_destroy: many geometries
    tracked by one persistent launch.  The descriptors hold the geometries'
    tables and the outputs' addresses, so both are kept alive here."""

    def __init__(self, items, block_size: int = 0, refill_min: int = 0, chunk: int = 0, regroup_every: int = 0,
                 wave_histories: int = 0, tuned: bool = False):
        """tuned=True passes no tuning: the shape gt_autotune_batch found for
        these items (else the defaults)."""
        self.items = list(items)
        arr = _batch_array(self.items)
        tun = None if tuned else C.byref(_Tuning(block_size=block_size, refill_min=refill_min, chunk=chunk,
                                                 regroup_every=regroup_every, wave_histories=wave_histories))
        h = C.c_void_p()
        _check(lib().gt_batch_create(arr, len(self.items), tun, C.byref(h)))
        self.h = h.value

    def launch(self, stream=None):
        if not self.h:
            raise GtError(GT_EINVAL, "batch is closed")
        _check(lib().gt_batch_launch(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().gt_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def batch_item(geom: Geometry, seed: int, n_particles: int, out: Optional[TrackOutputs] = None,
               **kwargs) -> BatchItem:
    """A batch item with freshly allocated outputs unless given."""
    if out is None:
        out = alloc_outputs(geom, n_particles, kwargs.get("record_first_k", 0), kwargs.get("record_cap", 0))
    return BatchItem(geom, seed, n_particles, out, kwargs)


def track_batch(items, block_size: int = 0, refill_min: int = 0, chunk: int = 0, regroup_every: int = 0,
                wave_histories: int = 0, tuned: bool = False, stream=None):
    """gt_track_batch: one-shot batch (waits for the stream)."""
    arr = _batch_array(items)
    tun = None if tuned else C.byref(_Tuning(block_size=block_size, refill_min=refill_min, chunk=chunk,
                                             regroup_every=regroup_every, wave_histories=wave_histories))
    _check(lib().gt_track_batch(arr, len(items), tun, _stream(stream)))
    return [it.out for it in items]


def autotune_track(geom: Geometry, seed: int, n_particles: int, out: Optional[TrackOutputs] = None, reps: int = 3,
                   stream=None, **kwargs) -> dict:
    """gt_autotune_track: the fastest (block_size, refill_min, regroup_every, wave_histories) for these
    parameters (the outputs are overwritten and end as those of one launch
    with that shape); also cached in the library for gt_tuning_lookup."""
    if out is None:
        out = alloc_outputs(geom, n_particles, kwargs.get("record_first_k", 0), kwargs.get("record_cap", 0))
    prm = _params(seed, n_particles, **kwargs)
    best = _Tuning()
    ms = C.c_float()
    _check(lib().gt_autotune_track(geom.h, C.byref(prm), C.byref(_out_struct(out)), reps, _stream(stream),
                                   C.byref(best), C.byref(ms)))
    return dict(block_size=best.block_size, refill_min=best.refill_min, regroup_every=best.regroup_every,
                wave_histories=best.wave_histories, ms=ms.value)


def tuning_lookup(geom: Geometry, seed: int, n_particles: int, **kwargs) -> Optional[dict]:
    """gt_tuning_lookup: the cached shape for such a launch, or None."""
    best = _Tuning()
    prm = _params(seed, n_particles, **kwargs)
    rc = lib().gt_tuning_lookup(geom.h, C.byref(prm), C.byref(best))
    if rc < 0:
        _check(rc)
    return (dict(block_size=best.block_size, refill_min=best.refill_min, regroup_every=best.regroup_every,
                 wave_histories=best.wave_histories) if rc == 1 else None)


def _batch_array(items):
    arr = (_BatchItem * max(len(items), 1))()
    for i, it in enumerate(items):
        arr[i].geometry = it.geom.h
        arr[i].params = _params(it.seed, it.n_particles, **it.kwargs)
        arr[i].out = _out_struct(it.out)
    return arr


def autotune_batch(items, reps: int = 1, stream=None) -> dict:
    """gt_autotune_batch: the fastest (block_size, refill_min, chunk, regroup_every, wave_histories) for this
    list of items; Batch(items) and track_batch(items) then use it."""
    best = _Tuning()
    ms = C.c_float()
    _check(lib().gt_autotune_batch(_batch_array(items), len(items), reps, _stream(stream), C.byref(best),
                                   C.byref(ms)))
    return dict(block_size=best.block_size, refill_min=best.refill_min, chunk=best.chunk,
                regroup_every=best.regroup_every, wave_histories=best.wave_histories, ms=ms.value)


def last_launch() -> Optional[dict]:
    """gt_last_launch: the plan of this thread's last persistent tracker
    launch (workgroups, block size, LDS bytes, staging kind, tally-cache
    entries, tail capacity, regroup interval), or None."""
    info = _LaunchInfo()
    rc = lib().gt_last_launch(C.byref(info))
    if rc < 0:
        _check(rc)
    return {n: getattr(info, n) for n, _ in _LaunchInfo._fields_} if rc == 1 else None


def set_kernel_events(start: Optional[int], stop: Optional[int]):
    """gt_set_kernel_events: raw hipEvent_t handles (ints) or None, None."""
    _check(lib().gt_set_kernel_events(start, stop))


def find_cell(geom: Geometry, pos, precision: int = PREC_MIXED, stream=None):
    """gt_find_cell on a device tensor pos [n, 3] float64."""
    import torch
    n = pos.shape[0]
    inst = torch.empty(n, dtype=torch.int64, device=pos.device)
    cells = torch.empty((n, MAX_LEVELS), dtype=torch.int32, device=pos.device)
    _check(lib().gt_find_cell(geom.h, _ptr(pos), n, _ptr(inst), _ptr(cells), precision, _stream(stream)))
    return inst, cells


def distance_to_surface(geom: Geometry, pos, dirs, state=None, stream=None):
    """gt_distance_to_surface on device tensors pos, dirs [n, 3] float64;
    state (optional) int32 [n, MAX_LEVELS + 2]: the cell of each level (-1
    below the leaf) and the (level, surface) the point is on (-1, -1)."""
    import torch
    n = pos.shape[0]
    if state is not None and tuple(state.shape) != (n, MAX_LEVELS + 2):
        raise GtError(GT_EINVAL, "state must be [n, %d] int32" % (MAX_LEVELS + 2))
    dist = torch.empty(n, dtype=torch.float64, device=pos.device)
    lev = torch.empty(n, dtype=torch.int32, device=pos.device)
    srf = torch.empty(n, dtype=torch.int32, device=pos.device)
    _check(lib().gt_distance_to_surface(geom.h, _ptr(pos), _ptr(dirs), _ptr(state), n, _ptr(dist), _ptr(lev),
                                        _ptr(srf), _stream(stream)))
    return dist, lev, srf


def fp64_check(a, b, stream=None):
    """gt_fp64_check: device a/b, sqrt(b) and the library logarithm of b."""
    import torch
    n = a.shape[0]
    q = torch.empty_like(a)
    r = torch.empty_like(a)
    lg = torch.empty_like(a)
    _check(lib().gt_fp64_check(_ptr(a), _ptr(b), n, _ptr(q), _ptr(r), _ptr(lg), _stream(stream)))
    return q, r, lg
