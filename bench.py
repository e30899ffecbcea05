#!/usr/bin/env python3
"""Benchmark: track segments per second on one MI355X.

Workload: the two-level 17x17 square lattice of axially split pins (three
pin types, 12 materials, 12,716 leaf-instance tallies) with 1e6 toy-transport
histories (uniform volume source, isotropic, at most 20 collisions), i.e.
the second workload configuration.  Both precision modes are timed; `value`
is the mixed-precision tracker (single-precision pruning, double-precision
decisions), `fp64` the all-double tracker on the same persistent schedule,
`plain_fp64_lane_per_history` the plain all-double tracker with one history
per lane (the baseline the mixed tracker must beat).  Inputs (the geometry tables) are
resident in HBM before the timed region; a step is one gt_track call: zero
the tallies, sample and track every history, write per-particle outputs,
finalize the tallies.

Further legs (each reported beside the headline, none of them is `value`):
the same histories without lattice hints, with the regroup step
(`mixed_with_regroup`, outputs compared with the headline's), with the
119 x 119 x 30 superimposed mesh tally (`mixed_with_mesh_tally`, its total
compared with the cell tallies' track length), by the event-based schedule,
and the 64-geometry batched launch.  `--config N` runs another workload at
its own size.

The GPU results of the timed steps are checked against the CPU oracle
(identical per-particle hashes, segment counts, end codes; bit-identical
fixed-point tallies) in the cpu_baseline leg, which also times the oracle on
the host cores.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak FP64 rate for non-fused operations: 256 CUs x 64 FP64 lanes x 2.4 GHz
# (the published 78.6 TFLOP/s counts a fused multiply-add as two operations;
# the tracker is compiled without contraction, so every add/mul/div/sqrt is
# one operation).
PEAK_FP64_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12                     # bytes/s, MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, choices=[1, 2, 3, 4], default=2,
                    help="workload: 1 one 3x3 pin lattice, 2 the 17x17 lattice (default, the headline), "
                         "3 the three-level core, 4 the hexagonal core")
    ap.add_argument("--particles", type=int, default=0, help="histories (0 = the workload's own count)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--refill", type=int, default=0, help="refill_min of the persistent schedule (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of tracking, run a plain device copy of this many bytes --steps times "
                         "(reference kernel for scaling HBM counters)")
    ap.add_argument("--only", choices=["mixed", "fp64", "plain_fp64", "event", "batch"], default=None,
                    help="time one mode only (profiling)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-geometry batched workload")
    ap.add_argument("--no-event", action="store_true", help="skip the event-based schedule leg")
    ap.add_argument("--tail", action="store_true", help="switch on tail compaction (comparison)")
    ap.add_argument("--regroup", type=int, default=0,
                    help="regroup the lanes by leaf universe every this many loop trips (comparison; 0 = off)")
    ap.add_argument("--regroup-leg", type=int, default=64,
                    help="interval of the extra leg timing the headline with regroup on (0 = no such leg)")
    ap.add_argument("--mesh", type=int, nargs=3, default=[119, 119, 30], metavar=("NX", "NY", "NZ"),
                    help="bins of the superimposed mesh tally leg over the domain (the paper's 119 x 119 x 30)")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh tally leg")
    ap.add_argument("--autotune", action="store_true",
                    help="time the launch shape gt_autotune_track picks instead of the library default")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)   # the default
    ap.add_argument("--tune-batch", action="store_true", help="autotune the batched launch shape first")
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


def run_timed(gt, step, args, hev):
    """Warm up, then time args.steps calls of step(): torch events around
    each whole step on the launch stream, HIP events (through the library's
    hook) around its tracking kernels."""
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    kev = [hev.pair() for _ in range(args.steps)]
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
    return dict(ms=ms, kernel_ms=kms, wall=wall)


def timed(gt, G, out, args, prec, hev, lane=False, regroup=None):
    kw = dict(seed=args.seed, n_particles=args.particles, geometry_id=args.config, precision=prec,
              block_size=args.block, out=out,
              lane_per_history=lane, refill_min=0 if lane else args.refill, tail_compaction=args.tail,
              regroup_every=0 if lane else (args.regroup if regroup is None else regroup))
    shape = None
    if not lane and args.autotune and not args.block and not args.refill and regroup is None:
        shape = gt.autotune_track(G, reps=2, **{k: v for k, v in kw.items()
                                                if k not in ("block_size", "refill_min", "regroup_every")})
        kw["block_size"], kw["refill_min"] = shape["block_size"], shape["refill_min"]
        kw["regroup_every"] = shape["regroup_every"]
    r = run_timed(gt, lambda: gt.track(G, **kw), args, hev)
    r["segments"] = out.counters_dict()["segments"]
    r["shape"] = {"block_size": kw["block_size"], "refill_min": kw["refill_min"],
                  "regroup_every": kw["regroup_every"], "autotuned": shape is not None}
    if not lane:
        r["shape"]["plan"] = gt.last_launch()
    return r


def timed_event(gt, G, args, hev):
    """The event-based schedule on the same workload (mixed precision): one
    kernel per tracking operation per iteration over a particle bank in
    device memory (its own outputs and bank)."""
    import torch
    n = args.particles
    out = gt.alloc_outputs(G, n)
    bank = torch.empty(gt.event_bank_bytes(n), dtype=torch.uint8, device="cuda")
    r = run_timed(gt, lambda: gt.track_event(G, seed=args.seed, n_particles=n, geometry_id=args.config,
                                             precision=gt.PREC_MIXED,
                                             out=out, bank=bank), args, hev)
    r["segments"] = out.counters_dict()["segments"]
    return r


def batched(gt, synth, args, hev):
    """The 64-geometry workload: one batched mixed-precision launch against
    64 sequential gt_track launches (all-double, and mixed)."""
    items, geoms = [], []
    for j in range(synth.BATCH_SIZE):
        fg, n = synth.batch_item(j)
        G = gt.Geometry(fg)
        geoms.append((G, n, j))
        items.append(gt.batch_item(G, synth.batch_particle_seed(j), n, geometry_id=synth.batch_geometry_id(j),
                                   precision=gt.PREC_MIXED, tail_compaction=args.tail))
    tuned = None
    if args.tune_batch:
        tuned = gt.autotune_batch(items, reps=1)
    b = gt.Batch(items, block_size=args.block, refill_min=args.refill, tuned=args.tune_batch)
    res = {"batched_mixed": run_timed(gt, b.launch, args, hev)}
    segs = sum(it.out.counters_dict()["segments"] for it in items)
    # the same launch captured once into a HIP graph and replayed
    import torch
    s = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        b.launch(s)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, e in gev:
        a.record()
        graph.replay()
        e.record()
    torch.cuda.synchronize()
    res["batched_mixed_graph_replay"] = {"ms": [a.elapsed_time(e) for a, e in gev]}
    if sum(it.out.counters_dict()["segments"] for it in items) != segs:
        raise RuntimeError("graph replay and eager segment counts differ")
    del graph
    for name, prec in (("sequential_fp64", gt.PREC_FP64), ("sequential_mixed", gt.PREC_MIXED)):
        def step(prec=prec):
            for (G, n, j), it in zip(geoms, items):
                gt.track(G, seed=synth.batch_particle_seed(j), n_particles=n, geometry_id=synth.batch_geometry_id(j),
                         precision=prec, block_size=args.block, refill_min=args.refill, out=it.out,
                         tail_compaction=args.tail)
        res[name] = run_timed(gt, step, args, hev)
        if sum(it.out.counters_dict()["segments"] for it in items) != segs:
            raise RuntimeError("batched and sequential segment counts differ")
    b.close()
    out = {"workload": "64 seeded square/hexagonal geometries, 1-3 levels, %d histories" %
           sum(n for _, n, _ in geoms), "segments_per_step": segs, "batch_shape": tuned}
    for k, r in res.items():
        ms = sum(r["ms"]) / len(r["ms"])
        out[k] = {"value": segs / (ms * 1e-3), "ms_per_step": ms}
    out["batched_over_sequential_fp64"] = out["batched_mixed"]["value"] / out["sequential_fp64"]["value"]
    out["batched_over_sequential_mixed"] = out["batched_mixed"]["value"] / out["sequential_mixed"]["value"]
    return out


def cpu_baseline(fg, gpu_out, n, seed, gid):
    """Oracle on the host cores over the whole workload, and the parity
    gate of the GPU outputs against it."""
    import numpy as np

    import oracle
    cores = min(16, os.cpu_count() or 1)
    og = oracle.OracleGeometry(fg)
    p = oracle.TrackParams(seed=seed, n_particles=n, geometry_id=gid)
    t0 = time.perf_counter()
    o = oracle.track(og, p, n_threads=cores)
    dt = time.perf_counter() - t0
    g_hash = gpu_out.seq_hash.cpu().numpy().view(np.uint64)
    g_seg = gpu_out.seg_count.cpu().numpy().view(np.uint32)
    g_end = gpu_out.end_code.cpu().numpy()
    g_fx = gpu_out.tally_fx.cpu().numpy().view(np.uint64)
    parity = bool(np.array_equal(g_hash, o.seq_hash) and np.array_equal(g_seg, o.seg_count)
                  and np.array_equal(g_end, o.end_code) and np.array_equal(g_fx, o.tally_fx))
    nz = o.tally != 0
    g_t = gpu_out.tally.cpu().numpy()
    rel = float(np.max(np.abs(g_t[nz] - o.tally[nz]) / o.tally[nz])) if nz.any() else 0.0
    # one core on a 10^4-history slice
    t0 = time.perf_counter()
    o1 = oracle.track(og, oracle.TrackParams(seed=seed, n_particles=min(n, 10_000), geometry_id=gid), n_threads=1)
    per_core = o1.counters["segments"] / (time.perf_counter() - t0)
    # algorithmic double-precision operations per segment (work meter over a sample)
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=seed, n_particles=min(n, 20_000), geometry_id=gid))
    return dict(value=o.counters["segments"] / dt, unit="segments/s", cores=cores, kind="oracle",
                sample="the whole workload (%d histories, %d segments), %.1f s" % (n, o.counters["segments"], dt),
                parity=parity, max_tally_rel_err=rel, ops_per_segment=ops / segs, per_core=per_core)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_k_track_persistent_17x17_1e6.md")
WORKLOAD_NAMES = {1: "3x3 square lattice of one pin type (two levels)",
                  2: "17x17 square lattice of 3 axially split pin types (two levels)",
                  3: "15x15 core of 17x17 assemblies of 3 pin types in a cylinder (four levels)",
                  4: "7-ring hexagonal core of 9-ring hexagonal assemblies, planes only (three levels)"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2406_13849_amd", "csrc", f)
                  for f in ("gt_device.h", "gt_track.hip", "gt_internal.h", "gt_geometry.cpp")]


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch():
    """HBM bytes per tracking launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by the
    factor a plain device copy of known size gives), or None when the kernel
    sources have changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    try:
        if kv["kernel_source_sha256"] != kernel_source_digest():
            return None
        return (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
                + float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])) * 1024.0
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the tracker has no multi-GPU path "
              "(histories would shard across GPUs by particle-id range; only the one-GPU path is built)", file=sys.stderr)
        sys.exit(2)
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
    args.seed = synth.particle_seed(args.config)
    if not args.particles:
        args.particles = synth.CONFIG_PARTICLES[args.config]
    fg = synth.make_config(args.config)
    G = gt.Geometry(fg)
    n = args.particles
    out = gt.alloc_outputs(G, n)
    res = {}
    modes = [("plain_fp64", gt.PREC_FP64, True), ("fp64", gt.PREC_FP64, False), ("mixed", gt.PREC_MIXED, False)]
    if args.only:
        modes = [m for m in modes if m[0] == args.only]
    hev = HipEvents()
    for name, prec, lane in modes:
        res[name] = timed(gt, G, out, args, prec, hev, lane)
        print("# %s: %.3f ms/step, %d segments/step" % (name, sum(res[name]["ms"]) / args.steps,
                                                        res[name]["segments"]), file=sys.stderr, flush=True)
    if args.only is None and synth.make_config(args.config).lattice_hint.any():
        # the same workload with the lattice hints removed: no FP32 index
        # guess, every full search through the hierarchy (the plain single
        # tracker against its lattice-aware form)
        fg2 = synth.make_config(args.config)
        fg2.lattice_hint[:] = 0
        G2 = gt.Geometry(fg2)
        res["nohint"] = timed(gt, G2, gt.alloc_outputs(G2, n), args, gt.PREC_MIXED, hev, False)
        print("# mixed without lattice hints: %.3f ms/step" % (sum(res["nohint"]["ms"]) / args.steps),
              file=sys.stderr, flush=True)
        G2.close()
    if args.only is None and args.regroup_leg:
        # the headline with the regroup step on (lanes sorted by leaf universe)
        out_rg = gt.alloc_outputs(G, n)
        res["regroup"] = timed(gt, G, out_rg, args, gt.PREC_MIXED, hev, False, regroup=args.regroup_leg)
        if "mixed" in res:   # result-neutral: the same sequences and tallies as the headline's
            torch.cuda.synchronize()
            res["regroup"]["identical"] = bool(torch.equal(out_rg.tally_fx, out.tally_fx) and
                                               torch.equal(out_rg.seq_hash, out.seq_hash) and
                                               torch.equal(out_rg.seg_count, out.seg_count))
        print("# mixed with regroup every %d trips: %.3f ms/step" % (args.regroup_leg,
                                                                     sum(res["regroup"]["ms"]) / args.steps),
              file=sys.stderr, flush=True)
    if args.only is None and not args.no_mesh:
        # the headline with the superimposed mesh tally (the paper's active cycles)
        mb = tuple(args.mesh)
        out_m, mesh_out = gt.alloc_outputs(G, n), gt.alloc_mesh(mb[0] * mb[1] * mb[2])
        rm = run_timed(gt, lambda: gt.track_mesh(G, args.seed, n, fg.domain_lo, fg.domain_hi, mb,
                                                 geometry_id=args.config, precision=gt.PREC_MIXED, out=out_m,
                                                 mesh_out=mesh_out), args, hev)
        rm["segments"] = out_m.counters_dict()["segments"]
        torch.cuda.synchronize()
        total = float(out_m.tally.sum().item())
        rm["mesh"] = {"bins": list(mb), "track_length_cm": float(mesh_out.mesh.sum().item()),
                      "cell_tally_track_length_cm": total,
                      "identical_histories": bool(torch.equal(out_m.seq_hash, out.seq_hash) and
                                                  torch.equal(out_m.tally_fx, out.tally_fx))
                      if "mixed" in res else None}
        res["mesh"] = rm
        print("# mixed with the %dx%dx%d mesh tally: %.3f ms/step" % (mb + (sum(rm["ms"]) / args.steps,)),
              file=sys.stderr, flush=True)
    if args.only in (None, "event") and not args.no_event:
        res["event"] = timed_event(gt, G, args, hev)
        print("# event: %.3f ms/step, %d segments/step" % (sum(res["event"]["ms"]) / args.steps,
                                                           res["event"]["segments"]), file=sys.stderr, flush=True)
    bat = None
    if (args.only in (None, "batch")) and not args.no_batch:
        bat = batched(gt, synth, args, hev)
        print("# batch: %s" % json.dumps(bat), file=sys.stderr, flush=True)
    if not any(k in res for k in ("mixed", "fp64")):
        print(json.dumps({"batched": bat, "event": res.get("event")}, default=str), flush=True)
        return
    head = res["mixed"] if "mixed" in res else res["fp64"]
    ms_step = sum(head["ms"]) / len(head["ms"])
    seg_s = head["segments"] / (ms_step * 1e-3)
    kernel_ms = sum(head["kernel_ms"]) / len(head["kernel_ms"])
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
        "config": {"workload": "%s, %d histories" % (WORKLOAD_NAMES[args.config], n),
                   "histories": n, "segments_per_step": head["segments"],
                   "precision": "mixed" if "mixed" in res else "fp64", "parallelism": "none (1 GPU)",
                   "launch_shape": head["shape"]},
    }
    for name, label in (("fp64", "fp64"), ("plain_fp64", "plain_fp64_lane_per_history"),
                        ("event", "event_based_mixed"), ("nohint", "mixed_without_lattice_hints"),
                        ("regroup", "mixed_with_regroup"), ("mesh", "mixed_with_mesh_tally")):
        if name in res:
            f = res[name]
            fms = sum(f["ms"]) / len(f["ms"])
            line[label] = {"value": f["segments"] / (fms * 1e-3), "ms_per_step": fms}
            if name == "regroup":
                line[label]["regroup_every"] = f["shape"]["regroup_every"]
                line[label]["identical_to_headline"] = f.get("identical")
    if "mesh" in res:
        line["mixed_with_mesh_tally"].update(res["mesh"]["mesh"])
        line["mixed_with_mesh_tally"]["time_over_headline"] = \
            line["mixed_with_mesh_tally"]["ms_per_step"] / ms_step
    if "mixed" in res and "fp64" in res:
        line["mixed_over_fp64"] = line["value"] / line["fp64"]["value"]
    if "mixed" in res and "plain_fp64" in res:
        line["mixed_over_plain_fp64"] = line["value"] / line["plain_fp64_lane_per_history"]["value"]
    if "mixed" in res and "event" in res:
        line["persistent_over_event_based"] = line["value"] / line["event_based_mixed"]["value"]
    if bat is not None:
        line["batched"] = bat
    if not args.no_cpu_baseline:
        cb = cpu_baseline(fg, out, n, args.seed, args.config)
        line["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        line["parity"] = {"sequences_and_fixed_point_tallies_identical": cb["parity"],
                          "max_tally_rel_err": cb["max_tally_rel_err"]}
        line["cpu_baseline"]["per_core_value"] = cb["per_core"]
        line["cpu_baseline"]["gpu_in_core_equivalents"] = seg_s / cb["per_core"]
        achieved = cb["ops_per_segment"] * head["segments"] / (kernel_ms * 1e-3)
        line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_OPS,
                            "traffic": traffic_per_launch() if (args.config == 2 and n == 1_000_000) else None,
                            "ops_per_segment": cb["ops_per_segment"], "kernel_ms": kernel_ms,
                            "kernel": "k_track_persistent<mixed, staging kind %d>" % G.staging(gt.PREC_MIXED)[0]}
        # the HBM side of the same kernel: algorithmic bytes (per-particle
        # outputs; no sequences are recorded here, the tallies fit in the L2)
        # and the measured bytes per launch from the committed counters
        alg = 13.0 * n / head["segments"]
        tr = line["roofline"]["traffic"]
        line["hbm"] = {"algorithmic_bytes_per_segment": alg,
                       "algorithmic_GBps": alg * seg_s / 1e9,
                       "measured_bytes_per_launch": tr,
                       "measured_GBps": (tr / (kernel_ms * 1e-3) / 1e9) if tr else None,
                       "peak_GBps": PEAK_HBM / 1e9,
                       "algorithmic_frac": alg * seg_s / PEAK_HBM,
                       "measured_frac": (tr / (kernel_ms * 1e-3) / PEAK_HBM) if tr else None}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
