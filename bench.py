"""Benchmark: energy-dispersive CT projection, rays/s on one MI355X.

Workload: cone-beam point source (Kramers continuum + two lines, 20-150
keV), 256^3 uint8 phantom of 1 mm voxels (8 materials, seed 1), 256 x 64
pixel x 128 energy-bin detector at 1.2 m, 1e9 rays per step, FP64
throughout.  One step = one mxr_run of all 1e9 rays into freshly zeroed
histograms; inputs are resident in HBM before the timed region.

Prints one JSON line: throughput, the roofline of the tracing kernel (HIP
events on the launch stream), the time to 1 % per-bin error of the plain and
the learned-proposal source (time_to_1pct), and the CPU oracle timed on a
bounded sample of the same run on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
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
# wave64 VALU instructions per second: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# FP64 operations per emitted ray of the projection's walk: ~6 per voxel visit
# (the plane alpha, two comparisons, the segment length, the optical-depth
# fused multiply-add) over 270 visits, plus ~400 for source, clip and tally
FP64_FLOP_PER_RAY = 6 * 270 + 400
# rays of the oracle's timed sample (several seconds of host work each; the per-ray
# tracer returns ~80 B per ray, so the cheap instruments stop at 2e8)
PROJECTION_CPU_SAMPLE = 16_000_000
CHEAP_CPU_SAMPLE = 200_000_000
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
    p.add_argument("--no-learned", action="store_true", help="skip the time-to-1%% measurement (plain vs learned)")
    p.add_argument("--cpu-sample", type=int, default=None,
                   help="rays of the oracle's timed sample (default: 1.6e7 for the projection, 2e8 for the "
                        "basic, beamline and focusing instruments, whose rays cost the oracle ~30x less)")
    p.add_argument("--train-hits", type=int, default=25 * 10**6, help="learned: detector hits collected for training")
    p.add_argument("--epochs", type=int, default=5, help="learned: training epochs")
    p.add_argument("--alpha", type=float, default=0.1, help="learned: share of the plain source in the proposal")
    p.add_argument("--no-confirm", action="store_true",
                   help="learned: skip the direct runs at the extrapolated 1 %% ray counts")
    p.add_argument("--eval-rays", type=int, default=16 * 10**8, help="learned: rays per error evaluation (16 replicas)")
    p.add_argument("--workload", choices=("projection", "batch", "learned", "train", "stepping", "crl", "scatter",
                                          "peaks", "basic", "beamline"),
                   default="projection",
                   help="projection: one 1e9-ray projection of the 256^3 phantom per step; batch: every angle "
                        "of phantoms of uneven size in one captured launch per step, beside one launch per job; "
                        "learned: time to 1%% per-bin error of the plain and the learned-proposal source; "
                        "train: proposal-network training steps; stepping: the same projection with the "
                        "fixed-step phantom model beside the exact path (speed and optical-depth error); "
                        "crl: the focusing instrument with a 16-lens compound refractive lens; scatter: the "
                        "projection's once- and twice-scattered images beside the uncollided one; peaks: the "
                        "measured FP64 FMA, multiply-high, exp, HBM read and FP64 atomic rates; basic / beamline: the "
                        "basic absorber and the beamline optics instruments with their ALU rooflines")
    p.add_argument("--step", type=float, default=1.0 / 3.0, help="stepping: step length (mm)")
    p.add_argument("--batch-rays", type=int, default=10**8, help="rays per job of the batch")
    p.add_argument("--batch-angles", type=int, default=360)
    p.add_argument("--batch-forms", action="store_true", help="batch: also time every launch form once")
    p.add_argument("--batch-sizes", default="64,128,256,512", help="phantom edges (voxels) of the batch")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="copy 1 GiB device to device before the timed region: a kernel of known traffic "
                        "for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


KERNEL_SOURCES = ["paper_2410_08747_amd/csrc/mxr.hip", "paper_2410_08747_amd/csrc/mxr_device.h", "include/mxr.h",
                  "paper_2410_08747_amd/build.py"]
PROFILE = "profiles/k_trace_edct_projection_256.md"
PROFILE_STEP = "profiles/k_trace_edct_step_256.md"
PROFILE_CRL = "profiles/k_trace_crl_focusing.md"
PROFILE_SCATTER = "profiles/k_trace_edct_scatter_256.md"
# FP64 VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one add, multiply, divide or square root counted as one operation)
FP64_OPS_PEAK = 256 * 4 * 16 * 2.4e9
# FP64 operations per lens of the compound refractive lens: two surfaces of
# 66 (intersection quadratic 19 + root 4 + hit point 6 + aperture 4 + normal
# 10 + Snell 14 + direction update 9) plus the lens centre and path sum (4)
CRL_OPS_PER_LENS = 2 * 66 + 4


def measured_traffic(profile=PROFILE):
    """HBM bytes per launch of a tracing kernel from the committed
    FETCH_SIZE / WRITE_SIZE counters, scaled by the copy calibration; None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(ROOT, profile)) as fh:
            line = [l for l in fh if l.startswith("counters:")][-1]
    except (OSError, IndexError):
        return None
    kv = dict(x.split("=") for x in line.split()[1:])
    if kv.get("source") != h.hexdigest()[:16]:
        return None
    return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) + float(kv["write_kib"]) * float(kv["write_scale"])) * 1024.0


def profile_line(prefix, profile=PROFILE):
    """key=value fields of the committed profile's last line starting with
    prefix; None when the kernel sources changed since it was taken."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(ROOT, profile)) as fh:
            line = [l for l in fh if l.startswith(prefix)][-1]
    except (OSError, IndexError):
        return None
    kv = dict(x.split("=") for x in line.split()[1:])
    if kv.get("source") != h.hexdigest()[:16]:
        return None
    return kv


def measured_valu(profile=PROFILE):
    """VALU wave-instructions per launch of the projection kernel from the
    committed SQ_INSTS_VALU count; None when the kernel sources changed since
    it was taken."""
    kv = profile_line("issue:", profile)
    return None if kv is None else float(kv["valu_insts"])


def measured_fp64_flop(profile=PROFILE):
    """FP64 operations per launch of the projection kernel from the committed
    SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 counts: 64 lanes per wave
    instruction, an FMA as two operations (every lane of an instruction is
    counted, masked or not, so this bounds the executed work from above)."""
    kv = profile_line("fp64:", profile)
    if kv is None:
        return None
    return 64.0 * (float(kv["add"]) + float(kv["mul"]) + 2.0 * float(kv["fma"]) + float(kv["trans"]))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(instr, n_sample: int, n_total: int, repeats: int = 5):
    """The oracle on the host cores, on rays spread evenly over the run (the
    stratified source orders rays by direction, so a contiguous prefix would
    only sample one edge of the cone): each repeat traces rays
    r, r + s, r + 2s, ... of the n_total-ray run with the oracle's per-ray
    tracer (every ray's full path through every component, detector bin
    included; only the three histogram additions of a run are left out, and
    with them a run's fixed cost of allocating and summing 2M-bin histograms,
    which a 1e9-ray run amortises).  Reported: the median of ``repeats``
    timings on all the cores of one GPU's host share (at most 16 threads, each
    tracing every 16th ray of the sample in a single-thread oracle call, all
    at once), and the median of ``repeats`` single-thread timings on a sample
    16x smaller (the paper's baseline is one CPU thread, wall clock, repeated
    runs)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    nproc = os.cpu_count() or 1
    threads = min(nproc, 16)

    def ids(m, r):
        return (np.uint64(r) + np.arange(m, dtype=np.uint64) * np.uint64(n_total // m))

    def timed(m, r, pool):
        sample = ids(m, r)
        t0 = time.perf_counter()
        if pool is None:
            oracle.trace_rays(instr, sample, 1, n_total)
        else:
            list(pool.map(lambda t: oracle.trace_rays(instr, sample[t::threads], 1, n_total), range(threads)))
        return m, time.perf_counter() - t0

    m_all = max(threads, n_sample // repeats)
    m_one = max(1, n_sample // (16 * repeats))
    with ThreadPoolExecutor(max_workers=threads) as pool:
        all_core = [timed(m_all, r, pool) for r in range(repeats)]
    one = [timed(m_one, r, None) for r in range(repeats)]
    rate = lambda runs: float(np.median([d / t for d, t in runs]))
    return {"value": rate(all_core), "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{repeats} repeats of {m_all} rays evenly spaced over the {n_total:.0e}-ray run "
                      f"(oracle per-ray tracer, every {threads}th ray per host thread, {threads} threads at once; "
                      f"median of the repeats)",
            "single_thread": {"value": rate(one), "unit": "rays/s", "cores": 1,
                              "sample": f"{repeats} repeats of {m_one} rays evenly spaced over the run, median"},
            "nproc": nproc, "cpu_model": cpu_model(), "repeats": repeats}


# The paper's own speed-ups, quoted as context (not a target; different code,
# instruments and hardware): GPU runs of the basic, focusing and EDXCT
# instruments against one thread of the paper's CPU.
PAPER_CONTEXT = {
    "speedup": "~250-600x (up to >600x for the focusing instrument on the H100)",
    "gpus": "NVIDIA GTX 1080 and H100 (FP64)",
    "baseline": "one thread of an Intel Xeon E5-2687W v4, wall clock",
    "source": "paper abstract and section 4 (results)",
}


def visits_per_ray(instr, samples: int = 200000, seed: int = 7, step: float = None) -> float:
    """Mean number of voxels a source ray visits: directions uniform over
    the cone's solid angle, chord through the phantom's box, one visit per
    voxel the chord enters (1 + the voxel planes it crosses); with ``step``,
    the fixed-step model's steps per ray instead (ceil(chord / step))."""
    src, ph = instr["components"][0], instr["components"][1]
    rng = np.random.default_rng(seed)
    ct = 1.0 - rng.random(samples) * (1.0 - np.cos(src["half_angle"]))
    st = np.sqrt(1.0 - ct * ct)
    phi = 2.0 * np.pi * rng.random(samples)
    d = np.stack([st * np.cos(phi), st * np.sin(phi), ct], axis=1)
    R = np.asarray(ph["rot"], dtype=np.float64).reshape(3, 3)
    pos = np.asarray(ph["pos"], dtype=np.float64)
    o = R.T @ (-pos)            # source in the phantom frame (lab = R local + pos)
    dl = d @ R                  # directions in the phantom frame
    nz, ny, nx = ph["volume"].shape
    v = ph["voxel"]
    half = 0.5 * v * np.array([nx, ny, nz], dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (-half - o) / dl
        t2 = (half - o) / dl
    tmin = np.nanmax(np.minimum(t1, t2), axis=1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=1)
    hit = tmax > np.maximum(tmin, 0.0)
    if step is not None:
        return float(np.sum(np.ceil((tmax[hit] - np.maximum(tmin[hit], 0.0)) / step)) / samples)
    a = o + np.maximum(tmin[hit], 0.0)[:, None] * dl[hit]
    b = o + tmax[hit][:, None] * dl[hit]
    n = np.array([nx, ny, nz])
    ia = np.clip(np.floor((a + half) / v), 0, n - 1)
    ib = np.clip(np.floor((b + half) / v), 0, n - 1)
    return float(np.sum(1.0 + np.abs(ib - ia).sum(axis=1)) / samples)


def batch_bench(args):
    """Every angle of every phantom as one job; one captured launch per step
    (autotuned shape), then the same jobs as one mxr_run each."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    mu = workloads.make_mu_tables(1)
    sizes = [int(x) for x in args.batch_sizes.split(",")]
    n_ang = args.batch_angles
    shared = {}
    jobs, bytes_total = [], 0.0
    for n in sizes:
        vol = workloads.make_phantom(n, seed=1)
        print(f"[bench] phantom {n}^3 built", file=sys.stderr, flush=True)
        for k in range(n_ang):
            ins = workloads.edct_projection(vol, mu, angle=2.0 * np.pi * k / n_ang, strata=STRATA)
            vis = visits_per_ray(ins, samples=20000, seed=k)
            I = mxr.Instrument(ins, dev, shared=shared)
            jobs.append((I, args.batch_rays, 1 + len(jobs), len(jobs), I.new_tallies()))
            bytes_total += args.batch_rays * (vis + 0.302 * 24)
    n_rays = args.batch_rays * len(jobs)
    stream = torch.cuda.current_stream()

    def zero():
        for j in jobs:
            for v in j[4][0].values():
                v.zero_()

    B = mxr.Batch(jobs)
    t_tune = time.perf_counter()
    sched = B.autotune(0.01)
    t_tune = time.perf_counter() - t_tune
    print(f"[bench] autotuned {sched} in {t_tune:.1f} s", file=sys.stderr, flush=True)
    times = {}
    for mode in ("batch", "separate"):
        for w in range(args.warmup + args.steps):
            zero()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            if mode == "batch":
                B.run(stream)
            else:
                for I, nr, seed, job, t in jobs:
                    I.run(nr, seed=seed, job=job, tallies=t, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if w >= args.warmup:
                times.setdefault(mode, []).append((wall, e0.elapsed_time(e1)))
            print(f"[bench] {mode} pass {w}: {wall:.2f} s", file=sys.stderr, flush=True)
    wall_b = float(np.mean([t[0] for t in times["batch"]]))
    kern_b = float(np.mean([t[1] for t in times["batch"]]))
    wall_s = float(np.mean([t[0] for t in times["separate"]]))
    achieved = bytes_total / (kern_b * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": n_rays / wall_b,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_b * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched_edct", "jobs": len(jobs), "angles": n_ang, "phantoms": sizes,
                   "rays_per_job": args.batch_rays, "strata": STRATA, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "schedule": {"form": ["grid", "persistent", "launches"][sched[0]], "groups_per_cu": sched[1],
                     "tile_rays": sched[2], "branches": sched[3], "autotune_s": t_tune},
        "separate_launches": {"value": n_rays / wall_s, "unit": "rays/s", "ms_per_step": wall_s * 1e3},
        "batch_over_separate": wall_s / wall_b,
    }
    if args.batch_forms:
        # every launch form once (after a capturing warm-up pass), beside
        # the separate launches timed above
        forms = {}
        for sch in ((0, 0, 0, 0), (1, 4, 65536, 0), (1, 8, 16384, 0), (2, 0, 0, 4)):
            B.schedule = sch
            zero()
            B.run(stream)
            zero()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.run(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            name = ["grid", "persistent", "launches"][sch[0]] + str(list(sch[1:]))
            forms[name] = {"s_per_pass": wall, "rays_per_s": n_rays / wall}
            print(f"[bench] form {name}: {wall:.2f} s", file=sys.stderr, flush=True)
        out["forms"] = forms
    print(json.dumps(out), flush=True)


def time_to_1pct(args):
    """Time to 1 % per-bin relative error (q95 over signal bins, batch means
    over 16 replicas) of the plain stratified source and of the learned
    proposal on the 256^3 projection.  The network is trained once on rows
    collected at 8 projection angles (context = angle) and evaluated at a
    training angle (0) and at an angle it has not seen (0.3 rad); the learned
    time includes collecting the training rays, the weights, training and
    inference, and is also given amortised over the 360 projections of an
    acquisition."""
    import math
    import torch
    import paper_2410_08747_amd as mxr
    import workloads
    from paper_2410_08747_amd import metrics

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    vol = workloads.make_phantom(256, seed=1)
    mu = workloads.make_mu_tables(1)
    shared = {}
    nb = 256 * 64 * 128
    R = 16
    stream = torch.cuda.current_stream()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)

    def instrument(angle):
        ins = workloads.edct_projection(vol, mu, angle=angle, strata=STRATA)
        return ins, mxr.Instrument(ins, dev, shared=shared)

    def instrument_early_out(angle):
        ins = workloads.edct_projection(vol, mu, angle=angle, strata=STRATA, early_out=True)
        return ins, mxr.Instrument(ins, dev, shared=shared)

    def new_tally(sum_w=None):
        return {"count": torch.zeros(nb, dtype=torch.int64, device=dev),
                "sum_w": torch.zeros(nb, dtype=torch.float64, device=dev) if sum_w is None else sum_w,
                "sum_w2": torch.zeros(nb, dtype=torch.float64, device=dev)}

    last = {}

    def replicas(I, n_rays):
        per = n_rays // R
        sums = torch.zeros(R, nb, dtype=torch.float64, device=dev)
        tallies = [[new_tally(sums[r])] for r in range(R)]
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(R):
            I.run(per, seed=1, purpose=3 + r, tallies=tallies[r], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        secs = e0.elapsed_time(e1) * 1e-3
        mean, rel = mxr.batch_means(sums, per)
        # share of the emitted rays that reached the detector
        last["detected"] = float(sum(int(t[0]["count"].sum().item()) for t in tallies)) / (per * R)
        return mean.cpu().numpy(), rel.cpu().numpy(), secs, per * R

    # training rows (purpose 1) from 8 angles, each run covering its whole cone
    # and every hit of a run kept; weights per angle from that angle's image
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    train_angles = [2.0 * math.pi * k / 8 for k in range(8)]
    cap = int(args.train_hits)
    hits = None
    starts, emitted = [], 0
    images = []
    for a_i, ang in enumerate(train_angles):
        ins, I = instrument(ang)
        if hits is None:
            hits = I.new_hits(cap)
        ctx = workloads.projection_context(ang, 256)
        coll = [new_tally()]
        start = int(hits["count"].item())
        budget = (cap * (a_i + 1)) // len(train_angles) - start
        pilot = max(10**6, budget // 100)
        I.collect(pilot, seed=1, context=ctx, hits=hits, purpose=1, job=2 * a_i, tallies=coll, stream=stream)
        got = int(hits["count"].item()) - start
        main = int((budget - got) / (got / pilot) * 0.97)
        I.collect(main, seed=1, context=ctx, hits=hits, purpose=1, job=2 * a_i + 1, tallies=coll, stream=stream)
        end = int(hits["count"].item())
        assert end <= cap, "training rows overflowed the buffer"
        emitted += pilot + main
        images.append(coll[0]["sum_w"])
        starts.append(start)
        del I, coll
    n_rows = int(hits["count"].item())
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    # training weights per angle from that angle's image, then Adam: one library call
    net = mxr.ProposalNet(workloads.init_mlp_params(1), batch=65536, device=dev)
    steps = args.epochs * ((n_rows + 65535) // 65536)
    loss_log = torch.zeros(steps, dtype=torch.float64, device=dev)
    _, I0 = instrument(0.0)
    net.train_from_runs(I0, hits, starts + [n_rows], images, epochs=args.epochs, lr=1e-3, seed=1,
                        loss_log=loss_log, stream=stream)
    torch.cuda.synchronize()
    del I0
    t_train = time.perf_counter() - t0 - t_collect
    t_learn = time.perf_counter() - t0  # inference (one forward per projection) is timed below
    ll = loss_log.cpu().numpy()
    log(f"collected {n_rows:.2e} hits at {len(train_angles)} angles from {emitted:.2e} rays in {t_collect:.2f} s; "
        f"trained {steps} steps in {t_train:.2f} s; loss {ll[:10].mean():.4f} -> {ll[-10:].mean():.4f}")
    del hits, images

    def spread(rel, mask, n):
        # relative variance per emitted ray of each signal bin, n rel_b^2
        # (independent of n): the rays a bin needs for a 100 % error
        v = n * rel[mask] ** 2
        return {"median": float(np.median(v)), "q95": float(np.percentile(v, 95.0))}

    def confirm(I, n_p, q, mask):
        # one direct run at the extrapolated ray count, rounded up to whole
        # replicas: its q95 should come out at 1 %
        N = int(math.ceil(n_p * (q / 0.01) ** 2 / R)) * R
        _, rc, tc, nc = replicas(I, N)
        return {"rays": nc, "seconds": tc, "q95": metrics.q95(rc, mask)}

    results = {}
    for name, ang in (("angle_0", 0.0), ("angle_0.3_unseen", 0.3)):
        ins, I = instrument(ang)
        n_ref = 4 * 10**9
        ref = [new_tally()]
        I.run(n_ref, seed=7, purpose=2, tallies=ref)
        torch.cuda.synchronize()
        I_ref = ref[0]["sum_w"].cpu().numpy() / n_ref
        var_ref = ref[0]["sum_w2"].cpu().numpy() / n_ref ** 2
        del ref
        mask = metrics.signal_bins(I_ref, metrics.flat_field(ins))
        mp, rp, tp, n_p = replicas(I, args.eval_rays)
        det_p = last["detected"]
        q_p = metrics.q95(rp, mask)
        T_p = metrics.time_to_1pct(tp / n_p, n_p, q_p)
        direct = name == "angle_0" and not args.no_confirm
        conf_p = confirm(I, n_p, q_p, mask) if direct else None
        # context: the plain source behind an aperture that ends the rays
        # bound elsewhere before the phantom (the same image)
        _, Ie = instrument_early_out(ang)
        me, re_, te, n_e = replicas(Ie, args.eval_rays)
        det_e = last["detected"]
        del Ie
        q_e = metrics.q95(re_, mask)
        T_e = metrics.time_to_1pct(te / n_e, n_e, q_e)
        torch.cuda.synchronize()
        ti = time.perf_counter()
        I.apply_proposal(net, workloads.projection_context(ang, 256), alpha=args.alpha, stream=stream)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - ti
        ml, rl, tl, n_l = replicas(I, args.eval_rays)
        det_l = last["detected"]
        q_l = metrics.q95(rl, mask)
        T_l = metrics.time_to_1pct(tl / n_l, n_l, q_l)
        conf_l = confirm(I, n_l, q_l, mask) if direct else None
        z = (ml - I_ref)[mask] / np.sqrt((rl * ml)[mask] ** 2 + var_ref[mask])
        log(f"{name}: plain q95 {q_p:.4f} T_1% {T_p:.2f} s; early-out T_1% {T_e:.2f} s; learned q95 {q_l:.4f} "
            f"T_1% {T_l:.2f} s (+{t_learn + t_inf:.2f} s to learn); mean z^2 {np.mean(z * z):.3f}"
            + (f"; direct runs at 1 %: plain q95 {conf_p['q95']:.4f} in {conf_p['seconds']:.2f} s, "
               f"learned q95 {conf_l['q95']:.4f} in {conf_l['seconds']:.2f} s" if direct else ""))
        results[name] = {
            "signal_bins": int(mask.sum()),
            "plain": {"rays_per_s": n_p / tp, "q95": q_p, "time_to_1pct_s": T_p, "detected_fraction": det_p,
                      "rel_var_per_ray": spread(rp, mask, n_p), "confirmed": conf_p},
            "plain_early_out": {"rays_per_s": n_e / te, "q95": q_e, "time_to_1pct_s": T_e, "detected_fraction": det_e,
                                "rel_var_per_ray": spread(re_, mask, n_e),
                                "max_rel_diff_vs_plain_mean": float(np.max(np.abs(me - mp)[mask] / mp[mask]))},
            "learned": {"rays_per_s": n_l / tl, "q95": q_l, "time_to_1pct_s": T_l, "inference_s": t_inf,
                        "detected_fraction": det_l,
                        "rel_var_per_ray": spread(rl, mask, n_l), "confirmed": conf_l,
                        "time_to_1pct_with_learning_s": T_l + t_learn + t_inf,
                        "time_to_1pct_amortised_360_s": T_l + t_learn / 360 + t_inf,
                        "bias_mean_z2": float(np.mean(z * z)),
                        "bias_frac_abs_z_gt_4": float(np.mean(np.abs(z) > 4))},
            "gain_excl_learning": T_p / T_l,
            "gain_excl_learning_vs_early_out": T_e / T_l,
            "gain_incl_learning": T_p / (T_l + t_learn + t_inf),
            "gain_amortised_360": T_p / (T_l + t_learn / 360 + t_inf),
        }
        del I
    return {
        "replicas": R, "eval_rays": args.eval_rays, "train_hits": n_rows, "train_rays": emitted,
        "train_angles": len(train_angles), "epochs": args.epochs, "alpha": args.alpha,
        "learn_s": t_learn, "collect_s": t_collect, "train_s": t_train,
        "loss_first": float(ll[:10].mean()), "loss_last": float(ll[-10:].mean()),
        "confirmed_q95": (None if results["angle_0"]["plain"]["confirmed"] is None else
                          {"plain": results["angle_0"]["plain"]["confirmed"]["q95"],
                           "learned": results["angle_0"]["learned"]["confirmed"]["q95"]}),
        **results,
    }


def learned_bench(args):
    r = time_to_1pct(args)
    out = {
        "metric": METRIC,
        "value": r["angle_0"]["learned"]["time_to_1pct_with_learning_s"],
        "unit": "s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": r["angle_0"]["learned"]["time_to_1pct_with_learning_s"] * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "edct_projection_time_to_1pct", "phantom": "256^3 uint8, 1 mm voxels, seed 1",
                   "detector": "256x64 px x 128 E-bins", "parallelism": "none (1 GPU)"},
        "time_to_1pct": r,
    }
    print(json.dumps(out), flush=True)


def train_bench(args):
    """Proposal-network training throughput: 2^20 seeded synthetic rows
    (random contexts, targets uniform in the box, weights in [0.1, 2]),
    one warm-up epoch, then args.steps epochs of 65,536-row Adam steps;
    rows/s, ms per step and the step's MFMA / HBM rooflines."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    rng = np.random.default_rng(1)
    n, batch = 1 << 20, 65536
    lo, hi = (-0.176, -0.176, 20.0), (0.176, 0.176, 150.0)
    ctx = torch.tensor(rng.normal(size=(n, 6)).astype(np.float32), device=dev)
    y = torch.tensor(np.stack([rng.uniform(lo[d], hi[d], n) for d in range(3)], 1), device=dev)
    w = torch.tensor(rng.uniform(0.1, 2.0, n), device=dev)
    net = mxr.ProposalNet(workloads.init_mlp_params(1), batch=batch, device=dev)
    net.train(ctx, y, w, lo, hi, epochs=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.train(ctx, y, w, lo, hi, epochs=args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = args.steps * (n // batch)
    flop = 2 * (6 * 128 + 128 * 128 + 128 * 56) * 3 * batch  # forward + two backward products per row
    out = {
        "metric": "proposal-network training rows/s", "value": steps * batch / dt, "unit": "rows/s", "n_gpus": 1,
        "steps": steps, "warmup": n // batch, "ms_per_step": dt / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "proposal_training", "rows": n, "batch": batch, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "mfma", "achieved": flop / (dt / steps) / 1e12, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": flop / (dt / steps) / 1e12 / 2500.0, "traffic": None},
    }
    print(json.dumps(out), flush=True)


def stepping_bench(args):
    """The projection with the paper's fixed-step phantom model (step h)
    beside the exact path: kernel time of each on the same 1e9 rays, the
    per-ray optical-depth error on a sample of those rays (same seeds, so
    the same source rays), and the image bias in units of the per-bin
    statistical error."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads
    from paper_2410_08747_amd import metrics

    vol = workloads.make_phantom(256, seed=1)
    mu = workloads.make_mu_tables(1)
    exact = workloads.edct_projection(vol, mu, angle=0.0, strata=STRATA)
    stepped = workloads.edct_projection(vol, mu, angle=0.0, strata=STRATA, step=args.step)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n = args.rays
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    shared = {}
    res = {}
    for name, ins in (("exact", exact), ("step", stepped)):
        I = mxr.Instrument(ins, dev, shared=shared)
        tallies = I.new_tallies()

        def zero():
            for v in tallies[0].values():
                v.zero_()

        for w in range(args.warmup):
            zero()
            I.run(n, seed=100 + w, n_total=n, tallies=tallies, stream=stream)
        torch.cuda.synchronize()
        ms = []
        for k in range(args.steps):
            zero()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            I.run(n, seed=1, n_total=n, tallies=tallies, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
            print(f"[stepping] {name} step {k}: {ms[-1]:.1f} ms", file=sys.stderr, flush=True)
        ids = (np.arange(1 << 20, dtype=np.uint64) * np.uint64(n // (1 << 20))).astype(np.uint64)
        rays = I.trace_rays(ids, seed=1, n_total=n)
        res[name] = {"ms": float(np.mean(ms)), "sum_w": tallies[0]["sum_w"].cpu().numpy(),
                     "sum_w2": tallies[0]["sum_w2"].cpu().numpy(), "w": rays["w"].cpu().numpy()}
        del I, tallies
    # source weights of the same rays: the instrument without its phantom
    bare = {"components": [exact["components"][0], exact["components"][2]]}
    w0 = mxr.Instrument(bare, dev).trace_rays(ids, seed=1, n_total=n)["w"].cpu().numpy()
    e, s = res["exact"], res["step"]
    tau_e = np.log(w0 / e["w"])
    live = (w0 > 0) & (e["w"] > 0) & (s["w"] > 0) & (tau_e > 0)  # rays that cross material
    tau_e = tau_e[live]
    dtau = np.log(e["w"][live] / s["w"][live])  # tau_step - tau_exact
    I_ref = e["sum_w"] / n
    sig = metrics.signal_bins(I_ref, metrics.flat_field(exact))
    rel = (s["sum_w"][sig] - e["sum_w"][sig]) / e["sum_w"][sig]
    stat = np.sqrt(e["sum_w2"][sig]) / e["sum_w"][sig]
    steps = visits_per_ray(stepped, step=args.step)
    bytes_per_ray = steps + 0.302 * 24
    achieved = bytes_per_ray * n / (s["ms"] * 1e-3) / 1e9
    out = {
        "metric": f"rays/s (ED-CT projection, fixed-step phantom model, step {args.step:.4g} mm)",
        "value": n / (s["ms"] * 1e-3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": s["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "edct_projection_fixed_step", "n_rays": n, "step_mm": args.step,
                   "phantom": "256^3 uint8, 1 mm voxels, seed 1", "detector": "256x64 px x 128 E-bins",
                   "strata": STRATA, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(PROFILE_STEP)},
        "steps_per_ray": steps,
        "exact": {"kernel_ms": e["ms"], "rays_per_s": n / (e["ms"] * 1e-3), "visits_per_ray": visits_per_ray(exact)},
        "time_vs_exact": s["ms"] / e["ms"],
        "tau_error": {"rays": int(live.sum()), "mean_tau_exact": float(np.mean(tau_e)),
                      "mean": float(np.mean(dtau)), "rms": float(np.sqrt(np.mean(dtau ** 2))),
                      "max_abs": float(np.max(np.abs(dtau))),
                      "median_abs_rel": float(np.median(np.abs(dtau) / tau_e)),
                      "frac_abs_gt_1e-3": float(np.mean(np.abs(dtau) > 1e-3)),
                      "frac_abs_gt_1e-2": float(np.mean(np.abs(dtau) > 1e-2))},
        "image_bias": {"signal_bins": int(sig.sum()), "median_abs_rel": float(np.median(np.abs(rel))),
                       "mean_rel": float(np.mean(rel)), "median_stat_rel_err": float(np.median(stat)),
                       "frac_bias_gt_stat": float(np.mean(np.abs(rel) > stat)),
                       "frac_bias_gt_3stat": float(np.mean(np.abs(rel) > 3 * stat))},
    }
    print(json.dumps(out), flush=True)


# Arithmetic of the ALU-bound instruments, counted from the per-ray code as
# lane operations (FP64 add, multiply, fused multiply-add, compare, floor and
# 32-bit integer add, xor, shift each one; a division, square root or
# transcendental function one; a 32 x 32 -> 64-bit product two, its high and
# low halves): per Philox4x32-10 block (ten rounds of two products, four
# xors and two key additions), per uniform drawn (64-bit word to a double),
# and per ray entering each component (its frame transforms included).
OPS_PHILOX_BLOCK = 10 * (2 * 2 + 4 + 2)
OPS_UNIFORM = 4
OPS_COMPONENT = {"source_rect_cone": 56, "slit": 80, "box": 63, "detector": 95, "source_gaussian": 71,
                 "mirror_elliptic": 165, "dcm": 159, "powder": 125}
# Philox blocks and uniforms of each component's draws (the powder's two
# uniforms come after the source's five: the rest of block 2 and block 3)
DRAWS_COMPONENT = {"source_rect_cone": (3, 5), "source_gaussian": (3, 5), "powder": (1, 2)}


def alu_bench(args):
    """The basic absorber (rectangular emitter, slit, homogeneous box,
    128 x 128 monitor) or the beamline (Gaussian source, elliptic mirror,
    two-crystal monochromator, powder, 1024 x 1024 monitor) at args.rays rays
    per step: rays/s and the ALU roofline from the counted lane operations
    per emitted ray (OPS_COMPONENT, weighted by the fraction of emitted rays
    that reach each component, measured on 2^20 traced rays)."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    instr = workloads.basic_absorber() if args.workload == "basic" else workloads.beamline()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    I = mxr.Instrument(instr, dev)
    tallies = I.new_tallies()
    stream = torch.cuda.current_stream()
    n = args.rays

    def zero():
        for t in tallies:
            for v in t.values():
                v.zero_()

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        zero()
        I.run(n, seed=100 + w, n_total=n, tallies=tallies, stream=stream)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        zero()
        events[k][0].record(stream)
        I.run(n, seed=1 + k, n_total=n, tallies=tallies, stream=stream)
        events[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    detected = int(tallies[-1]["count"].sum())
    # fraction of emitted rays entering each component, from traced rays
    m = 1 << 20
    tr = I.trace_rays(np.arange(m, dtype=np.uint64), seed=1, n_total=n)
    dead = tr["dead_at"].cpu().numpy()
    comps = instr["components"]
    reach, ops = [], 0.0
    for k, c in enumerate(comps):
        f = 1.0 if k == 0 else float(np.mean((dead < 0) | (dead >= k)))
        reach.append(f)
        blocks, uniforms = DRAWS_COMPONENT.get(c["type"], (0, 0))
        ops += f * (OPS_COMPONENT[c["type"]] + blocks * OPS_PHILOX_BLOCK + uniforms * OPS_UNIFORM)
    achieved = ops * n / (kern_ms * 1e-3)
    name = "basic absorber" if args.workload == "basic" else "beamline optics"
    out = {
        "metric": f"rays/s ({name})", "value": n * args.steps / wall, "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "basic_absorber" if args.workload == "basic" else "beamline", "n_rays": n,
                   "components": [c["type"] for c in comps], "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_OPS_PEAK / 1e12,
                     "unit": "T lane ops/s", "frac": achieved / FP64_OPS_PEAK, "traffic": None},
        "kernel_ms": kern_ms,
        "ops_per_ray": ops,
        "fraction_reaching": dict(zip([c["type"] for c in comps], reach)),
        "detected_fraction": detected / n,
        "launch_shape": list(I.launch_shape),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(instr, args.cpu_sample or CHEAP_CPU_SAMPLE, n)
        out["speedup_vs_oracle"] = {"one_thread": out["value"] / out["cpu_baseline"]["single_thread"]["value"],
                                    "all_cores": out["value"] / out["cpu_baseline"]["value"],
                                    "cores": out["cpu_baseline"]["cores"], "paper_context": PAPER_CONTEXT}
    print(json.dumps(out), flush=True)


def crl_bench(args):
    """The focusing instrument (Gaussian source, 1 x 1 mm crop, 16-lens
    compound refractive lens, 0.1 mm slit 14 m downstream, position and
    energy monitors) at args.rays rays per step: rays/s and the FP64
    arithmetic roofline of the lens."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    instr = workloads.crl_focusing()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    I = mxr.Instrument(instr, dev)
    tallies = I.new_tallies()
    stream = torch.cuda.current_stream()
    n = args.rays

    def zero():
        for t in tallies:
            for v in t.values():
                v.zero_()

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for w in range(args.warmup):
        zero()
        I.run(n, seed=100 + w, n_total=n, tallies=tallies, stream=stream)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        zero()
        events[k][0].record(stream)
        I.run(n, seed=1 + k, n_total=n, tallies=tallies, stream=stream)
        events[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    # rays entering the lens: the source emits weight 1, so the ledger's
    # weight entering the lens counts them
    m = min(n, 1 << 26)
    led = I.new_ledger()
    zero()
    I.run(m, seed=1, n_total=m, tallies=tallies, ledger=led, stream=stream)
    lv = led.cpu().numpy()
    f_lens = float(lv[4 * 2] / m)
    f_det = float(lv[4 * 4 + 3] / lv[0])
    ops = f_lens * 16 * CRL_OPS_PER_LENS
    achieved = ops * n / (kern_ms * 1e-3)
    out = {
        "metric": "rays/s (focusing instrument, 16-lens compound refractive lens)", "value": n * args.steps / wall,
        "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "crl_focusing", "n_rays": n, "lenses": 16, "source": "Gaussian 48.2 x 9.5 um, "
                   "100 x 4.3 urad, 23.32 keV +-1 keV", "monitors": "120x120 px PSD, 130-bin energy",
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_OPS_PEAK / 1e12,
                     "unit": "T FP64 ops/s", "frac": achieved / FP64_OPS_PEAK, "traffic": measured_traffic(PROFILE_CRL)},
        "kernel_ms": kern_ms,
        "fraction_through_crop": f_lens,
        "fraction_weight_detected": f_det,
        "fp64_ops_per_ray": ops,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(instr, args.cpu_sample or CHEAP_CPU_SAMPLE, n)
        out["speedup_vs_oracle"] = {"one_thread": out["value"] / out["cpu_baseline"]["single_thread"]["value"],
                                    "all_cores": out["value"] / out["cpu_baseline"]["value"],
                                    "cores": out["cpu_baseline"]["cores"], "paper_context": PAPER_CONTEXT}
    print(json.dumps(out), flush=True)


def scatter_bench(args):
    """The 256^3 projection split by scatter order: the uncollided image
    (order 0, the plain kernel) and the photons scattered once and twice
    (forced interactions, the last one aimed at the detector), each over
    args.rays rays: kernel times, rays/s of the order-1 kernel, and the
    share of each order in the detected intensity."""
    import torch
    import paper_2410_08747_amd as mxr
    import workloads

    vol = workloads.make_phantom(256, seed=1)
    mu = workloads.make_mu_tables(1)
    tab = workloads.make_scatter_tables(mu, 1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n = args.rays
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    shared = {}
    res = {}
    for order in (0, 1, 2):
        ins = workloads.edct_projection(vol, tab if order else mu, angle=0.0, strata=STRATA,
                                        scatter_order=order if order else None)
        I = mxr.Instrument(ins, dev, shared=shared)
        tallies = I.new_tallies()

        def zero():
            for v in tallies[0].values():
                v.zero_()

        for w in range(args.warmup):
            zero()
            I.run(n, seed=100 + w, n_total=n, tallies=tallies, stream=stream)
        torch.cuda.synchronize()
        ms = []
        for k in range(args.steps):
            zero()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            I.run(n, seed=1, n_total=n, tallies=tallies, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
            print(f"[scatter] order {order} step {k}: {ms[-1]:.1f} ms", file=sys.stderr, flush=True)
        sw = tallies[0]["sum_w"].sum().item()
        sw2 = tallies[0]["sum_w2"].sum().item()
        res[order] = {"kernel_ms": float(np.mean(ms)), "rays_per_s": n / (np.mean(ms) * 1e-3),
                      "intensity_per_ray": sw / n, "rel_err_total": math.sqrt(max(sw2 - sw * sw / n, 0.0)) / sw,
                      "detected": int(tallies[0]["count"].sum().item())}
        del I, tallies
    total = sum(r["intensity_per_ray"] for r in res.values())
    for r in res.values():
        r["share"] = r["intensity_per_ray"] / total
    visits = visits_per_ray(workloads.edct_projection(vol, mu, angle=0.0, strata=STRATA))
    # proxy bytes of an order-1 ray: two walks of the primary chord (optical
    # depth, then the interaction point), one exit walk (counted as a full
    # chord), one voxel byte per visit, plus the tally
    bytes_per_ray = 3 * visits + 0.302 * 24
    achieved = bytes_per_ray * n / (res[1]["kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": "rays/s (ED-CT projection, once-scattered photons, forced interaction aimed at the detector)",
        "value": res[1]["rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res[1]["kernel_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "edct_projection_scatter", "n_rays": n, "phantom": "256^3 uint8, 1 mm voxels, seed 1",
                   "tables": "total/Rayleigh/Compton, seed 1", "detector": "256x64 px x 128 E-bins",
                   "strata": STRATA, "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(PROFILE_SCATTER)},
        "orders": {str(k): v for k, v in res.items()},
        "scatter_to_primary": (res[1]["intensity_per_ray"] + res[2]["intensity_per_ray"]) / res[0]["intensity_per_ray"],
    }
    print(json.dumps(out), flush=True)


def peaks_bench(args):
    """Measured achievable rates beside the vendor figures: FP64 FMA issue,
    32-bit multiply-high, FP64 exp, an HBM read stream (4 GiB), and FP64
    atomic adds against the number of distinct target addresses."""
    import torch
    import paper_2410_08747_amd as mxr

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    groups = 256 * 32  # 32 work-groups of 256 lanes per CU

    def timed(kind, buf, spread=1, iters=1, g=groups, reps=3):
        best = None
        for r in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            work = mxr.mxr_peak_launch(kind, buf.data_ptr(), buf.numel() * buf.element_size(), spread, iters, g,
                                       stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            if r > 0:  # the first launch warms up
                t = a.elapsed_time(b) * 1e-3
                best = t if best is None else min(best, t)
        return work / best

    sink = torch.zeros(groups * 256, dtype=torch.float64, device=dev)
    out = {"fp64_fma_tflops": timed("fp64_fma", sink, iters=4096) / 1e12,
           "u32_mulhi_tops": timed("u32_mulhi", sink, iters=4096) / 1e12,
           "fp64_exp_gops": timed("fp64_exp", sink, iters=256) / 1e9}
    big = torch.ones(1 << 29, dtype=torch.float64, device=dev)  # 4 GiB
    out["hbm_read_gbs"] = timed("read", big, g=256 * 64) / 1e9
    del big
    atom = torch.zeros(1 << 21, dtype=torch.float64, device=dev)
    out["fp64_atomic_gops_by_spread"] = {str(sp): timed("atomic_f64", atom, spread=sp, iters=64, g=256 * 16) / 1e9
                                         for sp in (1, 130, 14400, 1 << 21)}
    vendor = {"fp64_fma_tflops": 78.6, "hbm_read_gbs": 8000.0}
    line = {"metric": "measured MI355X rates (FP64 FMA, u32 mul-hi, FP64 exp, HBM read, FP64 atomics)",
            "value": out["fp64_fma_tflops"], "unit": "TFLOP/s (FP64 FMA)", "n_gpus": 1, "steps": 3, "warmup": 1,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "micro-benchmarks", "groups": groups, "parallelism": "none (1 GPU)"},
            "measured": out, "vendor": vendor,
            "fraction_of_vendor": {"fp64_fma": out["fp64_fma_tflops"] / vendor["fp64_fma_tflops"],
                                   "hbm_read": out["hbm_read_gbs"] / vendor["hbm_read_gbs"]}}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the tracer is data-parallel over rays and the multi-GPU "
              "split (disjoint ray ranges + one histogram reduce) is not implemented here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "learned":
        learned_bench(args)
        return
    if args.workload == "train":
        train_bench(args)
        return
    if args.workload == "stepping":
        stepping_bench(args)
        return
    if args.workload == "crl":
        crl_bench(args)
        return
    if args.workload == "scatter":
        scatter_bench(args)
        return
    if args.workload == "peaks":
        peaks_bench(args)
        return
    if args.workload in ("basic", "beamline"):
        alu_bench(args)
        return
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
    kern_ms_median = float(np.median([a.elapsed_time(b) for a, b in events]))
    wall = t1 - t0
    value = n * args.steps / wall
    achieved = BYTES_PER_RAY * n / (kern_ms * 1e-3) / 1e9
    detected = int(tallies[0]["count"].sum())
    traffic = measured_traffic()
    valu = measured_valu()
    fp64 = measured_fp64_flop()

    # end to end, outside the timed region: an instrument created from the
    # host arrays (the volume's and tables' uploads, the phantom scan), the
    # run, and the image copied back to the host; warm, median of 5
    def end_to_end():
        torch.cuda.synchronize()
        t = time.perf_counter()
        J = mxr.Instrument(instr, dev)
        tl = J.new_tallies()
        J.run(n, seed=1, n_total=n, tallies=tl, stream=stream)
        host = {k: v.cpu().numpy() for k, v in tl[0].items()}
        torch.cuda.synchronize()
        del J, tl, host
        return time.perf_counter() - t

    end_to_end()
    e2e = float(np.median([end_to_end() for _ in range(5)]))

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
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "kernel_ms": kern_ms,
        "kernel_ms_median": kern_ms_median,
        "end_to_end": {"median_ms": e2e * 1e3, "repeats": 5, "rays_per_s": n / e2e,
                       "includes": "instrument create from host arrays (16 MiB volume and tables uploaded, "
                                   "phantom scan) + the run + the 3 x 16 MiB image copied to the host"},
        "detected_fraction": detected / n,
        # the same time against the other limits: the HBM bytes the counters
        # measured (the volume stays in the caches) and the FP64 arithmetic
        # of the walk (about 6 operations per voxel visit + 400 per ray of
        # source, clip and tally: a model count of 2.0 kflop per ray)
        "roofline_detail": {
            "gather_model": "1 B per voxel visit (270 per ray) + 24 B per detected ray; L2/MALL-resident, "
                            "the HBM proxy this workload is quoted on",
            "measured_hbm": (None if traffic is None else
                             {"bytes_per_launch": traffic, "achieved_GBs": traffic / (kern_ms * 1e-3) / 1e9,
                              "frac": traffic / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}),
            "fp64": {"flop_per_ray": FP64_FLOP_PER_RAY, "achieved_TFLOPs": FP64_FLOP_PER_RAY * n / (kern_ms * 1e-3) / 1e12,
                     "peak_TFLOPs": 78.6, "frac": FP64_FLOP_PER_RAY * n / (kern_ms * 1e-3) / 78.6e12,
                     # the same from the committed FP64 op-class counters
                     "measured_flop_per_ray": (None if fp64 is None else fp64 / n),
                     "measured_frac": (None if fp64 is None else fp64 / (kern_ms * 1e-3) / 78.6e12)},
            # the binding limit: VALU instruction issue (the launch's committed
            # SQ_INSTS_VALU count over this run's kernel time, against one
            # wave64 VALU instruction per SIMD per 4 cycles)
            "valu_issue": (None if valu is None else
                           {"insts_per_launch": valu, "achieved_per_s": valu / (kern_ms * 1e-3),
                            "peak_per_s": VALU_ISSUE_PEAK, "frac": valu / (kern_ms * 1e-3) / VALU_ISSUE_PEAK}),
            "binding": "valu_issue",
        },
    }
    if not args.no_learned:
        del tallies, I
        torch.cuda.empty_cache()
        out["time_to_1pct"] = time_to_1pct(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(instr, args.cpu_sample or PROJECTION_CPU_SAMPLE, n)
        cb = out["cpu_baseline"]
        out["speedup_vs_oracle"] = {"one_thread": value / cb["single_thread"]["value"],
                                    "all_cores": value / cb["value"], "cores": cb["cores"],
                                    "paper_context": PAPER_CONTEXT}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
