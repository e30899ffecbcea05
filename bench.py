#!/usr/bin/env python3
"""Benchmark: track segments per second on one MI355X, mixed precision vs
all-FP64, with every leg's outputs checked against the CPU oracle.

Headline workload (the one the metric is quoted on): the three-level square
core -- a root cell inside a z-cylinder of radius 140 cm, |z| <= 100, filled
with a 15 x 15 core lattice of five seeded assembly types, each a 17 x 17
lattice of three axially split pin types (2,861,100 leaf-instance tallies) --
with 1e7 toy-transport histories (uniform volume source, isotropic, at most 20
collisions) and the sequences of the first 1e5 histories recorded.  A step is
one gt_track call: zero the tallies and counters, pad the record buffer, sample
and track every history, write the per-particle outputs and recorded
sequences, finalize the tallies.  Inputs (geometry tables) are resident in HBM
before the timed region.  `value` is the mixed-precision persistent tracker
(single-precision pruning, double-precision decisions); `fp64` the
all-double tracker on the same schedule, the denominator of `mixed_over_fp64`.

Further legs on the same workload (each with its own output buffers, each
checked against the oracle; none of them is `value`): the paper's two
comparison trackers -- static polymorphism (`sp_tracker_mixed`: a switch on
each level's universe kind, arrays by index) and the fixed-depth reactor
tracker (`rtk_tracker`), with the ratios `st_over_rtk`, `sp_over_rtk` and
`st_over_sp` beside the paper's own (context only) -- the plain all-FP64
tracker with one history per lane, the event-based schedule, the single
tracker with the lattice hints removed (hierarchy searches only), the regroup
step, and the paper's 119 x 119 x 30 superimposed mesh tally.  Beside it: the
hexagonal core (7-ring core of 9-ring hexagonal assemblies, planes only, 1e7
histories) mixed vs all-FP64, and the 64-geometry batch in one persistent
launch at the shape gt_autotune_batch picks (eager and as a replayed HIP
graph) against 64 sequential gt_track launches.

Parity gate: the oracle tracks every history of every workload on the host
cores; each leg's per-particle hashes, segment counts and end codes, recorded
sequences, counters and fixed-point tallies must be identical, and its
finalized tallies within 1e-12 relative.  The JSON line carries a flag per
leg; the script exits with status 1 when any leg differs.  The oracle run of
the headline workload is also the `cpu_baseline` timing (all the host cores
this process may use); one core on a 1e4-history slice gives the per-core rate.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks: FP64 vector 78.6 TFLOP/s (a fused multiply-add counts
# two), i.e. 256 CUs x 64 FP64 lanes x 2.4 GHz = 39.3e12 instructions/s issue
# of non-fused adds, multiplies, divides or square roots.
PEAK_FP64_FLOPS = 78.6e12
PEAK_FP64_NONFMA_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12                     # bytes/s, HBM3E
L2_BYTES_PER_XCD = 4 * 1024 * 1024

# The paper's relative rates on Frontier (one MI250X GCD), quoted as context
# only (full continuous-energy transport, not this toy; Table 3 and the
# tracking-kernel times of Section "Performance results").
PAPER_CONTEXT = {
    "source": "arXiv 2406.13849, Table 3 and the tracking-kernel time ratios (MI250X GCD)",
    "st_rate_over_rtk_inactive": 0.834, "st_rate_over_rtk_active": 0.910,
    "sp_rate_over_rtk_inactive": 0.912, "dp_rate_over_rtk_inactive": 0.778,
    "st_tracking_kernel_time_over_rtk": 2.02, "sp_tracking_kernel_time_over_rtk": 1.5,
    "note": "full Shift k-eigenvalue transport on the NuScale SMR model; not comparable to these toy-transport "
            "segment rates",
}

WORKLOAD_NAMES = {1: "3x3 square lattice of one pin type (two levels)",
                  2: "17x17 square lattice of 3 axially split pin types (two levels)",
                  3: "three-level square core: r=140 cylinder, 15x15 core of 5 assembly types, 17x17 pins of "
                     "3 types (four levels)",
                  4: "7-ring hexagonal core of 9-ring hexagonal assemblies, planes only (three levels)"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2406_13849_amd", "csrc", f)
                  for f in ("gt_device.h", "gt_track.hip", "gt_internal.h", "gt_geometry.cpp", "gt_launch.h",
                            "gt_persistent.h", "gt_track_axcz.hip", "gt_track_vert.hip")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--aux-steps", type=int, default=2,
                    help="timed steps of the comparison legs that take most of a second per step "
                         "(plain one-history-per-lane, event-based, mesh, regroup, no hints)")
    ap.add_argument("--config", type=int, choices=[1, 2, 3, 4], default=3,
                    help="headline workload: 1 one 3x3 pin lattice, 2 the 17x17 lattice, 3 the three-level "
                         "core (default; the metric's workload), 4 the hexagonal core")
    ap.add_argument("--particles", type=int, default=0, help="histories (0 = the workload's own count)")
    ap.add_argument("--record-k", type=int, default=100_000, help="histories whose sequences are recorded")
    ap.add_argument("--record-cap", type=int, default=384, help="entries recorded per history")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0, help="refill_min of the persistent schedule (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (and so the parity gate): for profiling runs only")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of tracking, run a plain device copy of this many bytes --steps times "
                         "(reference kernel for scaling HBM counters)")
    ap.add_argument("--only", choices=["mixed", "fp64", "plain_fp64", "event", "batch", "sp", "rtk", "mesh"],
                    default=None,
                    help="time one leg of the headline workload only (profiling; prints that leg's summary)")
    ap.add_argument("--no-trackers", action="store_true",
                    help="skip the SP and RTK tracker legs of the headline workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-geometry batched workload")
    ap.add_argument("--no-hex", action="store_true", help="skip the hexagonal core")
    ap.add_argument("--no-aux", action="store_true", help="skip the comparison legs of the headline workload")
    ap.add_argument("--tail", action="store_true", help="switch on tail compaction (comparison)")
    ap.add_argument("--regroup-leg", type=int, default=64,
                    help="interval of the leg timing the headline with the regroup step (0 = no such leg)")
    ap.add_argument("--mesh", type=int, nargs=3, default=[119, 119, 30], metavar=("NX", "NY", "NZ"),
                    help="bins of the superimposed mesh tally leg over the domain (the paper's 119 x 119 x 30)")
    ap.add_argument("--autotune", action="store_true",
                    help="time the headline at the launch shape gt_autotune_track picks")
    ap.add_argument("--no-tune-batch", action="store_true", help="batched launch at the library defaults")
    return ap.parse_args()


class HipEvents:
    """hipEvent_t pairs from the HIP runtime, handed to the library's timing
    hook so that only the tracking kernel launch is bracketed (the zeroing and
    finalize kernels of a step are outside)."""

    def __init__(self):
        import ctypes as C
        self.C = C
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]

    def pair(self):
        a, b = self.C.c_void_p(), self.C.c_void_p()
        if self.hip.hipEventCreate(self.C.byref(a)) or self.hip.hipEventCreate(self.C.byref(b)):
            raise RuntimeError("hipEventCreate failed")
        return a.value, b.value

    def elapsed_ms(self, a, b):
        ms = self.C.c_float()
        if self.hip.hipEventElapsedTime(self.C.byref(ms), a, b):
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self, a, b):
        self.hip.hipEventDestroy(a)
        self.hip.hipEventDestroy(b)


def run_timed(gt, step, steps, warmup, hev):
    """Warm up, then time `steps` calls of step(): torch events around each
    whole step on the launch stream, HIP events (through the library's hook)
    around its tracking kernels."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    kev = [hev.pair() for _ in range(steps)]
    t0 = time.perf_counter()
    for (a, b), (ka, kb) in zip(ev, kev):
        gt.set_kernel_events(ka, kb)
        a.record()
        step()
        b.record()
    gt.set_kernel_events(None, None)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    kms = [hev.elapsed_ms(ka, kb) for ka, kb in kev]
    for ka, kb in kev:
        hev.destroy(ka, kb)
    return dict(ms=ms, kernel_ms=kms, wall=wall, steps=steps)


def mean(v):
    return sum(v) / len(v)


def log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- parity
def host_outputs(out):
    """A leg's device outputs copied to host arrays."""
    import numpy as np
    return dict(tally_fx=out.tally_fx.cpu().numpy().view(np.uint64), tally=out.tally.cpu().numpy(),
                seg_count=out.seg_count.cpu().numpy().view(np.uint32),
                seq_hash=out.seq_hash.cpu().numpy().view(np.uint64), end_code=out.end_code.cpu().numpy(),
                rec=None if out.rec is None else out.rec.cpu().numpy(), counters=out.counters_dict())


def compare(g, o):
    """Parity of one leg's host outputs g with the oracle's result o: the
    per-particle hashes, segment counts and end codes, the recorded
    sequences, the counters and the fixed-point tallies identical; finalized
    tallies within 1e-12 relative (exactly 0 where the oracle's are 0)."""
    import numpy as np
    bad = []
    for k in ("seq_hash", "seg_count", "end_code"):
        if not np.array_equal(g[k], getattr(o, k)):
            bad.append(k)
    if (o.rec is None) != (g["rec"] is None) or (o.rec is not None and not np.array_equal(g["rec"], o.rec)):
        bad.append("rec")
    for k in ("escaped", "capped", "lost", "segcap", "rec_overflow", "segments", "rejected"):
        if g["counters"][k] != o.counters[k]:
            bad.append("counter " + k)
    if not np.array_equal(g["tally_fx"], o.tally_fx):
        bad.append("tally_fx")
    nz = o.tally != 0
    rel = float(np.max(np.abs(g["tally"][nz] - o.tally[nz]) / o.tally[nz])) if nz.any() else 0.0
    if rel > 1e-12 or np.any(g["tally"][~nz] != 0):
        bad.append("tally")
    return dict(identical=not bad, differs=bad, max_tally_rel_err=rel)


def host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------- roofline inputs
def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_fields(path):
    """`- key: value` lines of a committed rocprofv3 summary."""
    kv = {}
    if not os.path.exists(path):
        return kv
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    return kv


def counters_for(workload_tag):
    """HBM bytes per tracking launch and the FP64 issue figures from the
    committed counter summary of this workload's headline kernel, or None for
    each when the kernel sources have changed since the counters were taken.
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by what the
    same counter reads for a device copy of known size."""
    kv = profile_fields(os.path.join(ROOT, "profiles", "hbm_traffic_k_track_persistent_%s.md" % workload_tag))
    if not kv or kv.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        r = {"traffic": (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
                         + float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])) * 1024.0}
        for k in ("fp64_valu_insts_per_dispatch", "valu_insts_per_dispatch", "valu_lane_utilisation",
                  "lds_bank_conflict_over_lds_insts", "valu_busy_frac", "counter_kernel_us"):
            if k in kv:
                r[k] = float(kv[k])
        return r
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------- legs
def track_leg(gt, G, n, seed, gid, args, prec, steps, warmup, hev, rec=True, **kw):
    """One gt_track leg with its own outputs: timing, launch plan, outputs."""
    rk, rc = (args.record_k, args.record_cap) if rec else (0, 0)
    rk = min(rk, n)
    out = gt.alloc_outputs(G, n, rk, rc)
    call = dict(seed=seed, n_particles=n, geometry_id=gid, precision=prec, record_first_k=rk, record_cap=rc,
                out=out, tail_compaction=args.tail)
    call.update(kw)
    if not call.get("lane_per_history"):
        call.setdefault("block_size", args.block)
        call.setdefault("refill_min", args.refill)
    r = run_timed(gt, lambda: gt.track(G, **call), steps, warmup, hev)
    r["segments"] = out.counters_dict()["segments"]
    r["out"] = out
    if not call.get("lane_per_history"):
        r["plan"] = gt.last_launch()
    r["shape"] = {k: call.get(k, 0) for k in ("block_size", "refill_min", "regroup_every", "wave_histories")}
    return r


def summary(r, extra=None):
    ms = mean(r["ms"])
    d = {"value": r["segments"] / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": mean(r["kernel_ms"]),
         "steps": r["steps"]}
    if extra:
        d.update(extra)
    return d


def workload_legs(gt, synth, cfg, n, args, hev, aux):
    """The mixed and all-FP64 legs of one workload, and (aux) its comparison legs."""
    import torch
    seed = synth.particle_seed(cfg)
    fg = synth.make_config(cfg)
    G = gt.Geometry(fg)
    legs = {}
    shape_note = None
    kw_mixed = {}
    if args.autotune and cfg == args.config:
        out = gt.alloc_outputs(G, n, min(args.record_k, n), args.record_cap)
        shape_note = gt.autotune_track(G, seed=seed, n_particles=n, geometry_id=cfg, precision=gt.PREC_MIXED,
                                       record_first_k=min(args.record_k, n), record_cap=args.record_cap, out=out,
                                       reps=2)
        kw_mixed = {k: shape_note[k] for k in ("block_size", "refill_min", "regroup_every", "wave_histories")}
        del out
    for name, prec in (("mixed", gt.PREC_MIXED), ("fp64", gt.PREC_FP64)):
        if args.only is None or args.only == name:
            legs[name] = track_leg(gt, G, n, seed, cfg, args, prec, args.steps, args.warmup, hev,
                                   **(kw_mixed if name == "mixed" else {}))
            log("cfg%d %s: %.3f ms/step, %d segments" % (cfg, name, mean(legs[name]["ms"]), legs[name]["segments"]))
    # the paper's comparison trackers on the same workload: static
    # polymorphism (arrays by index, mixed precision elsewhere) and the
    # fixed-depth reactor tracker where the geometry has its shape
    if args.only in (None, "sp") and not args.no_trackers:
        legs["sp"] = track_leg(gt, G, n, seed, cfg, args, gt.PREC_MIXED, args.steps, args.warmup, hev, tracker="sp")
        log("cfg%d SP tracker (mixed): %.3f ms/step" % (cfg, mean(legs["sp"]["ms"])))
    if args.only in (None, "rtk") and not args.no_trackers and G.kinds()[2]:
        legs["rtk"] = track_leg(gt, G, n, seed, cfg, args, gt.PREC_FP64, args.steps, args.warmup, hev, tracker="rtk")
        log("cfg%d RTK tracker: %.3f ms/step" % (cfg, mean(legs["rtk"]["ms"])))
    a_steps, a_warm = min(args.aux_steps, args.steps), min(args.warmup, 1)
    if aux and args.only in (None, "plain_fp64"):
        legs["plain_fp64"] = track_leg(gt, G, n, seed, cfg, args, gt.PREC_FP64, a_steps, a_warm, hev,
                                       lane_per_history=True)
        log("cfg%d plain fp64 (one history per lane): %.3f ms/step" % (cfg, mean(legs["plain_fp64"]["ms"])))
    if aux and args.only in (None, "event"):
        rk = min(args.record_k, n)
        out = gt.alloc_outputs(G, n, rk, args.record_cap)
        bank = torch.empty(gt.event_bank_bytes(n), dtype=torch.uint8, device="cuda")
        r = run_timed(gt, lambda: gt.track_event(G, seed=seed, n_particles=n, geometry_id=cfg,
                                                 precision=gt.PREC_MIXED, record_first_k=rk,
                                                 record_cap=args.record_cap, out=out, bank=bank),
                      a_steps, a_warm, hev)
        r["segments"] = out.counters_dict()["segments"]
        r["out"] = out
        legs["event"] = r
        del bank
        log("cfg%d event-based: %.3f ms/step" % (cfg, mean(r["ms"])))
    if aux and args.only is None:
        if fg.lattice_hint.any():
            # the single tracker with the lattice hints removed: no index
            # guess, every full search through the hierarchy
            fg2 = synth.make_config(cfg)
            fg2.lattice_hint[:] = 0
            G2 = gt.Geometry(fg2)
            legs["nohint"] = track_leg(gt, G2, n, seed, cfg, args, gt.PREC_MIXED, a_steps, a_warm, hev)
            legs["nohint"]["geometry"] = G2
            log("cfg%d mixed without lattice hints: %.3f ms/step" % (cfg, mean(legs["nohint"]["ms"])))
        if args.regroup_leg:
            legs["regroup"] = track_leg(gt, G, n, seed, cfg, args, gt.PREC_MIXED, a_steps, a_warm, hev,
                                        regroup_every=args.regroup_leg)
            log("cfg%d mixed, regroup every %d: %.3f ms/step" % (cfg, args.regroup_leg,
                                                                 mean(legs["regroup"]["ms"])))
    if aux and args.only in (None, "mesh"):
        mb = tuple(args.mesh)
        out = gt.alloc_outputs(G, n, min(args.record_k, n), args.record_cap)
        mesh_out = gt.alloc_mesh(mb[0] * mb[1] * mb[2])
        r = run_timed(gt, lambda: gt.track_mesh(G, seed, n, fg.domain_lo, fg.domain_hi, mb, geometry_id=cfg,
                                                precision=gt.PREC_MIXED, record_first_k=min(args.record_k, n),
                                                record_cap=args.record_cap, out=out, mesh_out=mesh_out),
                      a_steps, a_warm, hev)
        r["segments"] = out.counters_dict()["segments"]
        r["out"] = out
        torch.cuda.synchronize()
        r["mesh"] = {"bins": list(mb), "track_length_cm": float(mesh_out.mesh.sum().item()),
                     "cell_tally_track_length_cm": float(out.tally.sum().item())}
        legs["mesh"] = r
        del mesh_out
        log("cfg%d mixed with the %dx%dx%d mesh tally: %.3f ms/step" % ((cfg,) + mb + (mean(r["ms"]),)))
    return fg, G, legs, shape_note


def oracle_run(fg, n, seed, gid, args, threads, record=True):
    import oracle
    og = oracle.OracleGeometry(fg)
    rk = min(args.record_k, n) if record else 0
    p = oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid, record_first_k=rk,
                           record_cap=args.record_cap if rk else 0)
    t0 = time.perf_counter()
    o = oracle.track(og, p, n_threads=threads)
    return og, o, time.perf_counter() - t0


def check_legs(legs, o, rec_legs):
    """Parity of every leg against the oracle result o (legs without recorded
    sequences are compared without them)."""
    res = {}
    for name, r in legs.items():
        g = host_outputs(r["out"])
        if name not in rec_legs:
            g["rec"] = o.rec
        res[name] = compare(g, o)
        if name == "mesh":
            m = r["mesh"]
            ok = abs(m["track_length_cm"] - m["cell_tally_track_length_cm"]) <= 1e-9 * m["cell_tally_track_length_cm"]
            res[name]["mesh_total_equals_cell_total"] = ok
            if not ok:
                res[name]["identical"] = False
                res[name]["differs"].append("mesh total")
        r["out"] = None
    return res


def batched(gt, synth, args, hev, threads):
    """The 64-geometry workload: one batched mixed-precision launch (at the
    autotuned shape) against 64 sequential gt_track launches (all-double, and
    mixed); every item of every leg checked against the oracle."""
    import torch
    import oracle
    items, geoms = [], []
    for j in range(synth.BATCH_SIZE):
        fg, n = synth.batch_item(j)
        G = gt.Geometry(fg)
        geoms.append((fg, G, n, j))
        items.append(gt.batch_item(G, synth.batch_particle_seed(j), n, geometry_id=synth.batch_geometry_id(j),
                                   precision=gt.PREC_MIXED, tail_compaction=args.tail))
    tuned = None
    if not args.no_tune_batch:
        tuned = gt.autotune_batch(items, reps=1)
        log("batch autotuned shape: %s" % tuned)
    b = gt.Batch(items, tuned=not args.no_tune_batch)
    res = {"batched_mixed": run_timed(gt, b.launch, args.steps, args.warmup, hev)}
    segs = sum(it.out.counters_dict()["segments"] for it in items)
    outs = {"batched_mixed": [host_outputs(it.out) for it in items]}
    # the same launch captured once into a HIP graph and replayed
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        b.launch(s)
    for it in items:
        it.out.seq_hash.zero_()
        it.out.tally_fx.zero_()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, e in gev:
        a.record()
        graph.replay()
        e.record()
    torch.cuda.synchronize()
    res["batched_mixed_graph_replay"] = {"ms": [a.elapsed_time(e) for a, e in gev], "steps": args.steps}
    outs["batched_mixed_graph_replay"] = [host_outputs(it.out) for it in items]
    del graph
    b.close()
    for name, prec in (("sequential_fp64", gt.PREC_FP64), ("sequential_mixed", gt.PREC_MIXED)):
        seq_out = [gt.alloc_outputs(G, n) for (_, G, n, _) in geoms]

        def step(prec=prec, seq_out=seq_out):
            for (fg, G, n, j), out in zip(geoms, seq_out):
                gt.track(G, seed=synth.batch_particle_seed(j), n_particles=n, geometry_id=synth.batch_geometry_id(j),
                         precision=prec, block_size=args.block, refill_min=args.refill, out=out,
                         tail_compaction=args.tail)
        res[name] = run_timed(gt, step, args.steps, args.warmup, hev)
        outs[name] = [host_outputs(o) for o in seq_out]
        del seq_out
    log("batch legs timed; oracle over every item")
    parity = {k: True for k in outs}
    bad = []
    t0 = time.perf_counter()
    for (fg, G, n, j) in geoms:
        o = oracle.track(oracle.OracleGeometry(fg),
                         oracle.TrackParams(seed=synth.batch_particle_seed(j), n_particles=n,
                                            geometry_id=synth.batch_geometry_id(j)), n_threads=threads)
        for k in outs:
            g = outs[k][j]
            g["rec"] = o.rec
            c = compare(g, o)
            if not c["identical"]:
                parity[k] = False
                bad.append((k, j, c["differs"]))
    oracle_s = time.perf_counter() - t0
    out = {"workload": "64 seeded square/hexagonal geometries, 1-3 levels, %d histories" %
           sum(n for _, _, n, _ in geoms), "segments_per_step": segs, "batch_shape": tuned}
    for k, r in res.items():
        ms = mean(r["ms"])
        out[k] = {"value": segs / (ms * 1e-3), "ms_per_step": ms, "steps": r["steps"],
                  "every_item_identical_to_oracle": parity[k]}
    out["batched_over_sequential_fp64"] = out["batched_mixed"]["value"] / out["sequential_fp64"]["value"]
    out["batched_over_sequential_mixed"] = out["batched_mixed"]["value"] / out["sequential_mixed"]["value"]
    out["oracle_s"] = oracle_s
    if bad:
        out["mismatches"] = [str(x) for x in bad[:10]]
    for (_, G, _, _) in geoms:
        G.close()
    return out, all(parity.values())


def alg_bytes_per_segment(n_inst, histories, segments, recorded_segments):
    """Algorithmic HBM bytes per segment: 4 B per recorded sequence entry, a
    16-byte tally read-modify-write for the share of uniformly spread tally
    updates that miss a 4 MiB L2 (none when the tally array fits), and the
    13 bytes of per-particle outputs per history."""
    tally_bytes = 16.0 * n_inst
    miss = max(0.0, 1.0 - L2_BYTES_PER_XCD / tally_bytes)
    return (4.0 * recorded_segments + 16.0 * miss * segments + 13.0 * histories) / segments, miss


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the tracker has no multi-GPU path "
              "(histories would shard across GPUs by particle-id range; only the one-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    if args.copy_bytes:
        a = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "steps": args.steps}))
        return
    from paper_2406_13849_amd import gt, synth
    hev = HipEvents()
    threads = host_cores()
    cfg = args.config
    n = args.particles or synth.CONFIG_PARTICLES[cfg]
    seed = synth.particle_seed(cfg)

    if args.only == "batch":
        bat, ok = batched(gt, synth, args, hev, threads) if not args.no_cpu_baseline else (None, True)
        print(json.dumps({"batched": bat}, default=str), flush=True)
        sys.exit(0 if ok else 1)

    fg, G, legs, tuned_shape = workload_legs(gt, synth, cfg, n, args, hev,
                                             aux=not args.no_aux and args.only not in ("mixed", "fp64"))
    if args.only is not None:
        res = {k: summary(v) for k, v in legs.items()}
        ok = True
        if not args.no_cpu_baseline:
            _, o, _ = oracle_run(fg, n, seed, cfg, args, host_cores())
            par = check_legs(legs, o, rec_legs=set(legs))
            for k in res:
                res[k]["identical_to_oracle"] = par[k]["identical"]
                ok = ok and par[k]["identical"]
        print(json.dumps(res), flush=True)
        sys.exit(0 if ok else 1)
    hex_res = None
    hex_legs = None
    if cfg != 4 and not args.no_hex:
        n4 = synth.CONFIG_PARTICLES[4]
        fg4, G4, hex_legs, _ = workload_legs(gt, synth, 4, n4, args, hev, aux=False)

    ok = True
    parity = {}
    cb = None
    if not args.no_cpu_baseline:
        log("oracle over the whole workload on %d host threads" % threads)
        og, o, dt = oracle_run(fg, n, seed, cfg, args, threads)
        parity = check_legs(legs, o, rec_legs=set(legs))
        import oracle
        # one core on a 10^4-history slice; the work meter over a sample
        t0 = time.perf_counter()
        o1 = oracle.track(og, oracle.TrackParams(seed=seed, n_particles=min(n, 10_000), geometry_id=cfg),
                          n_threads=1)
        per_core = o1.counters["segments"] / (time.perf_counter() - t0)
        ops, msegs = oracle.count_work(og, oracle.TrackParams(seed=seed, n_particles=min(n, 20_000),
                                                              geometry_id=cfg))
        recorded = int((o.rec >= 0).sum()) if o.rec is not None else 0
        cb = dict(value=o.counters["segments"] / dt, unit="segments/s", cores=threads, kind="oracle",
                  sample="the whole workload (%d histories, %d segments, first %d sequences recorded), %.1f s"
                         % (n, o.counters["segments"], min(args.record_k, n), dt),
                  cpu_model=cpu_model(), per_core_value=per_core,
                  per_core_sample="one thread, histories 0..%d" % (min(n, 10_000) - 1),
                  ops_per_segment=ops / msegs, recorded_segments=recorded, n_inst=int(o.tally.shape[0]))
        del o
        if hex_legs is not None:
            log("oracle over the hexagonal core")
            _, o4, dt4 = oracle_run(fg4, synth.CONFIG_PARTICLES[4], synth.particle_seed(4), 4, args, threads)
            hp = check_legs(hex_legs, o4, rec_legs=set(hex_legs))
            hex_res = {"workload": "%s, %d histories" % (WORKLOAD_NAMES[4], synth.CONFIG_PARTICLES[4]),
                       "segments_per_step": hex_legs["mixed"]["segments"],
                       "oracle_segments_per_s": o4.counters["segments"] / dt4}
            for k, r in hex_legs.items():
                hex_res[k] = summary(r, {"identical_to_oracle": hp[k]["identical"]})
                ok = ok and hp[k]["identical"]
            hex_res["mixed_over_fp64"] = hex_res["mixed"]["value"] / hex_res["fp64"]["value"]
            del o4
    elif hex_legs is not None:
        hex_res = {k: summary(r) for k, r in hex_legs.items()}

    bat = None
    if args.only is None and not args.no_batch and not args.no_cpu_baseline:
        bat, bok = batched(gt, synth, args, hev, threads)
        ok = ok and bok
        log("batch: %s" % json.dumps(bat))

    head = legs["mixed"] if "mixed" in legs else legs["fp64"]
    ms_step = mean(head["ms"])
    seg_s = head["segments"] / (ms_step * 1e-3)
    kernel_ms = mean(head["kernel_ms"])
    line = {
        "metric": "track segments/sec on 1 MI355X (mixed vs FP64), exact cell sequences",
        "value": seg_s,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s, %d histories" % (WORKLOAD_NAMES[cfg], n),
                   "histories": n, "segments_per_step": head["segments"],
                   "recorded_sequences": [min(args.record_k, n), args.record_cap],
                   "precision": "mixed" if "mixed" in legs else "fp64", "parallelism": "none (1 GPU)",
                   "launch_shape": dict(head["shape"], plan=head.get("plan"), autotuned=tuned_shape is not None)},
    }
    labels = (("fp64", "fp64"), ("sp", "sp_tracker_mixed"), ("rtk", "rtk_tracker"),
              ("plain_fp64", "plain_fp64_lane_per_history"), ("event", "event_based_mixed"),
              ("nohint", "mixed_without_lattice_hints"), ("regroup", "mixed_with_regroup"),
              ("mesh", "mixed_with_mesh_tally"))
    for name, label in labels:
        if name in legs:
            extra = {}
            if name in parity:
                extra["identical_to_oracle"] = parity[name]["identical"]
            if name == "regroup":
                extra["regroup_every"] = args.regroup_leg
            if name == "mesh":
                extra.update(legs["mesh"]["mesh"])
                extra["time_over_headline"] = mean(legs["mesh"]["ms"]) / ms_step
            line[label] = summary(legs[name], extra)
    if "mixed" in legs and "fp64" in legs:
        line["mixed_over_fp64"] = line["value"] / line["fp64"]["value"]
    if "mixed" in legs and "rtk" in legs:
        # the paper's Table 3 ratio (a tracking rate over the RTK rate) on this workload
        line["st_over_rtk"] = line["value"] / line["rtk_tracker"]["value"]
        if "sp" in legs:
            line["sp_over_rtk"] = line["sp_tracker_mixed"]["value"] / line["rtk_tracker"]["value"]
    if "mixed" in legs and "sp" in legs:
        line["st_over_sp"] = line["value"] / line["sp_tracker_mixed"]["value"]
    if "mixed" in legs and "plain_fp64" in legs:
        line["mixed_over_plain_fp64"] = line["value"] / line["plain_fp64_lane_per_history"]["value"]
    if "mixed" in legs and "event" in legs:
        line["persistent_over_event_based"] = line["value"] / line["event_based_mixed"]["value"]
    if hex_res is not None:
        line["hexagonal"] = hex_res
    if bat is not None:
        line["batched"] = bat
    line["paper_context"] = PAPER_CONTEXT
    if cb is not None:
        line["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "cpu_model",
                                                   "per_core_value", "per_core_sample")}
        line["cpu_baseline"]["gpu_in_core_equivalents"] = seg_s / cb["per_core_value"]
        line["parity"] = {name: parity[name] for name in parity}
        line["parity"]["all_legs_identical_to_oracle"] = all(p["identical"] for p in parity.values()) and ok
        ok = ok and line["parity"]["all_legs_identical_to_oracle"]
        achieved = cb["ops_per_segment"] * head["segments"] / (kernel_ms * 1e-3)
        tag = {3: "core15x15_1e7", 2: "17x17_1e6", 4: "hex_core_1e7", 1: "3x3_1e4"}[cfg]
        cnt = counters_for(tag) if n == synth.CONFIG_PARTICLES[cfg] else None
        kind = G.staging(gt.PREC_MIXED)[0]
        line["roofline"] = {
            "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_FLOPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_FLOPS, "traffic": cnt["traffic"] if cnt else None,
            "ops_per_segment": cb["ops_per_segment"], "kernel_ms": kernel_ms,
            "kernel": "k_track_persistent<mixed, staging kind %d>" % kind,
            "peak_nonfma_fp64_ops": PEAK_FP64_NONFMA_OPS / 1e12,
            "frac_of_nonfma_issue": achieved / PEAK_FP64_NONFMA_OPS,
        }
        if cnt and "fp64_valu_insts_per_dispatch" in cnt:
            # FP64 VALU wave instructions x 64 lanes over the FP64 lane-issue capacity of the kernel's time
            line["roofline"]["fp64_valu_issue_frac"] = (cnt["fp64_valu_insts_per_dispatch"] * 64.0
                                                        / (PEAK_FP64_NONFMA_OPS * kernel_ms * 1e-3))
            for k in ("valu_lane_utilisation", "valu_busy_frac", "lds_bank_conflict_over_lds_insts"):
                if k in cnt:
                    line["roofline"][k] = cnt[k]
        alg, miss = alg_bytes_per_segment(cb["n_inst"], n, head["segments"], cb["recorded_segments"])
        tr = line["roofline"]["traffic"]
        line["hbm"] = {"algorithmic_bytes_per_segment": alg, "tally_l2_miss_share": miss,
                       "algorithmic_bytes_per_launch": alg * head["segments"],
                       "algorithmic_GBps": alg * head["segments"] / (kernel_ms * 1e-3) / 1e9,
                       "measured_bytes_per_launch": tr,
                       "measured_over_algorithmic": (tr / (alg * head["segments"])) if tr else None,
                       "measured_GBps": (tr / (kernel_ms * 1e-3) / 1e9) if tr else None,
                       "peak_GBps": PEAK_HBM / 1e9,
                       "algorithmic_frac": alg * head["segments"] / (kernel_ms * 1e-3) / PEAK_HBM,
                       "measured_frac": (tr / (kernel_ms * 1e-3) / PEAK_HBM) if tr else None}
    print(json.dumps(line, default=str), flush=True)
    if not ok:
        log("PARITY FAILURE: a leg's outputs differ from the oracle's")
        sys.exit(1)


if __name__ == "__main__":
    main()
