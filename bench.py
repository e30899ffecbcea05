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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--particles", type=int, default=1_000_000)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of tracking, run a plain device copy of this many bytes --steps times "
                         "(reference kernel for scaling HBM counters)")
    ap.add_argument("--only", choices=["mixed", "fp64", "plain_fp64"], default=None,
                    help="time one mode only (profiling)")
    return ap.parse_args()


def timed(gt, G, out, args, prec, lane=False):
    import torch
    kw = dict(seed=2002, n_particles=args.particles, geometry_id=2, precision=prec, block_size=args.block, out=out,
              lane_per_history=lane)
    for _ in range(args.warmup):
        gt.track(G, **kw)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        gt.track(G, **kw)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    segs = out.counters_dict()["segments"]
    return dict(ms=ms, wall=wall, segments=segs)


def cpu_baseline(fg, gpu_out, n):
    """Oracle on the host cores over the whole workload, and the parity
    gate of the GPU outputs against it."""
    import numpy as np

    import oracle
    cores = min(16, os.cpu_count() or 1)
    og = oracle.OracleGeometry(fg)
    p = oracle.TrackParams(seed=2002, n_particles=n, geometry_id=2)
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
    # algorithmic double-precision operations per segment (work meter over a sample)
    ops, segs = oracle.count_work(og, oracle.TrackParams(seed=2002, n_particles=min(n, 20_000), geometry_id=2))
    return dict(value=o.counters["segments"] / dt, unit="segments/s", cores=cores, kind="oracle",
                sample="the whole workload (%d histories, %d segments), %.1f s" % (n, o.counters["segments"], dt),
                parity=parity, max_tally_rel_err=rel, ops_per_segment=ops / segs)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the tracker has no multi-GPU path "
              "(histories shard by particle-id range; see the design notes)", file=sys.stderr)
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
    fg = synth.make_config(2)
    G = gt.Geometry(fg)
    n = args.particles
    out = gt.alloc_outputs(G, n)
    res = {}
    modes = [("plain_fp64", gt.PREC_FP64, True), ("fp64", gt.PREC_FP64, False), ("mixed", gt.PREC_MIXED, False)]
    if args.only:
        modes = [m for m in modes if m[0] == args.only]
    for name, prec, lane in modes:
        res[name] = timed(gt, G, out, args, prec, lane)
        print("# %s: %.3f ms/step, %d segments/step" % (name, sum(res[name]["ms"]) / args.steps,
                                                        res[name]["segments"]), file=sys.stderr, flush=True)
    head = res["mixed"] if "mixed" in res else res["fp64"]
    ms_step = sum(head["ms"]) / len(head["ms"])
    seg_s = head["segments"] / (ms_step * 1e-3)
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
        "config": {"workload": "17x17 square lattice of 3 axially split pin types (two levels), %d histories" % n,
                   "histories": n, "segments_per_step": head["segments"],
                   "precision": "mixed" if "mixed" in res else "fp64", "parallelism": "none (1 GPU)"},
    }
    for name, label in (("fp64", "fp64"), ("plain_fp64", "plain_fp64_lane_per_history")):
        if name in res:
            f = res[name]
            fms = sum(f["ms"]) / len(f["ms"])
            line[label] = {"value": f["segments"] / (fms * 1e-3), "ms_per_step": fms}
    if "mixed" in res and "fp64" in res:
        line["mixed_over_fp64"] = line["value"] / line["fp64"]["value"]
    if "mixed" in res and "plain_fp64" in res:
        line["mixed_over_plain_fp64"] = line["value"] / line["plain_fp64_lane_per_history"]["value"]
    if not args.no_cpu_baseline:
        cb = cpu_baseline(fg, out, n)
        line["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        line["parity"] = {"sequences_and_fixed_point_tallies_identical": cb["parity"],
                          "max_tally_rel_err": cb["max_tally_rel_err"]}
        achieved = cb["ops_per_segment"] * seg_s
        line["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_OPS, "traffic": None,
                            "ops_per_segment": cb["ops_per_segment"],
                            "kernel": "k_track_persistent (mixed precision)"}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
