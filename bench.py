"""Benchmark: energy-dispersive CT projection, rays/s on one MI355X.

Workload: cone-beam point source (Kramers continuum + two lines, 20-150
keV), 256^3 uint8 phantom of 1 mm voxels (8 materials, seed 1), 256 x 64
pixel x 128 energy-bin detector at 1.2 m, 1e9 rays per step, FP64
throughout.  One step = one mxr_run of all 1e9 rays into freshly zeroed
histograms; inputs are resident in HBM before the timed region.

Prints one JSON line: throughput, the roofline of the tracing kernel (HIP
events on the launch stream), and the CPU oracle timed on a bounded sample
of the same run on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/s (ED-CT projection) + time to 1% per-bin error, learned vs plain"
N_RAYS = 10**9
# Algorithmic bytes per emitted ray of the projection: one voxel byte per
# visit (269.6 visits per emitted ray on this phantom and geometry, ~270) and
# 24 B of histogram update for the 30.2 % of rays that reach the detector.
BYTES_PER_RAY = 270 * 1 + 0.302 * 24
HBM_PEAK_GBS = 8000.0
# cone cells per side of the stratified source: 4096^2 cells of ~60 rays, so
# the 64 rays of a wave leave the source in almost the same direction
STRATA = 4096


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--rays", type=int, default=N_RAYS)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=4_000_000)
    p.add_argument("--calibrate-copy", action="store_true",
                   help="copy 1 GiB device to device before the timed region: a kernel of known traffic "
                        "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def cpu_baseline(instr, n_sample: int, n_total: int):
    """The oracle on the host cores, on 64 equal ray ranges spread evenly over
    the run (the stratified source orders rays by direction, so a contiguous
    prefix would only sample the edge of the cone)."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    chunks = 64
    per = max(1, n_sample // chunks)
    t0 = time.perf_counter()
    for c in range(chunks):
        first = (n_total // chunks) * c
        oracle.run(instr, per, seed=1, first=first, n_total=n_total, threads=threads)
    dt = time.perf_counter() - t0
    done = per * chunks
    return {"value": done / dt, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{chunks} ranges of {per} rays spread over the {n_total:.0e}-ray projection "
                      f"({done} rays, {threads} host threads, {dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the tracer is data-parallel over rays and the multi-GPU "
              "split (disjoint ray ranges + one histogram reduce) is not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    vol = workloads.make_phantom(256, seed=1)
    mu = workloads.make_mu_tables(1)
    instr = workloads.edct_projection(vol, mu, angle=0.0, strata=STRATA)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    I = mxr.Instrument(instr, dev)
    tallies = I.new_tallies()
    stream = torch.cuda.current_stream()
    n = args.rays

    def step(seed):
        for t in tallies:
            for v in t.values():
                v.zero_()
        I.run(n, seed=seed, n_total=n, tallies=tallies, stream=stream)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        step(100 + w)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        for t in tallies:
            for v in t.values():
                v.zero_()
        events[k][0].record(stream)
        I.run(n, seed=1 + k, n_total=n, tallies=tallies, stream=stream)
        events[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    wall = t1 - t0
    value = n * args.steps / wall
    achieved = BYTES_PER_RAY * n / (kern_ms * 1e-3) / 1e9
    detected = int(tallies[0]["count"].sum())

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "edct_projection", "n_rays": n, "phantom": "256^3 uint8, 1 mm voxels, seed 1",
                   "detector": "256x64 px x 128 E-bins", "strata": STRATA, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "kernel_ms": kern_ms,
        "detected_fraction": detected / n,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(instr, args.cpu_sample, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
