"""Parity of the HIP library with the CPU oracle, through the C ABI.

Per ray (mxr_trace_rays vs the oracle's per-ray trace, the same Philox
streams): identical status, absorbing component and tally bin; position,
direction, energy and weight within 1e-12 relative (floors: 1 mm, 1, 1 keV,
and 1e-300 for the weight, which is compared relative to itself).  The
weight after a voxel phantom is ill-conditioned in the ray's geometry and
its optical depth is a long sum: a source direction that differs in its
last bit (the GPU's and the C library's sin, cos and sqrt agree to an ulp
or two) moves every material boundary by about ulp(alpha), ~1e-13 mm at
1 m, and the optical depth by the mu jump there (up to ~15 /cm at the low
end of the spectrum) times that; the two sides also round a sum of up to N
terms differently (per segment on the oracle's side, per material run or
per step on the GPU's), which moves tau by up to ~N u tau (u = 2^-53).  A
ray whose weight misses 1e-12 is therefore checked against its own
conditioning: within 1e-12 + 8 s + 4 N u tau, with s the largest relative
change of the oracle's weight when one component of the oracle's source
direction moves by one ulp (six such rays continued through the rest of the
instrument by the oracle), tau = ln(w_source / w) of the oracle's ray, and N
the walk's bound on its segments or steps.  Such rays must stay rare (at
most 1 in 100 of those compared) and within 1e-9.  In the scattering chains
each forced interaction places its point by dividing an optical depth by
the local mu, which a direction change does not probe: there at most 2 in
1000 rays may miss 1e-12, all within 1e-9, and the per-bin check binds.
Per bin
(mxr_run vs the oracle's run): identical counts; sums of w and w^2 within
1e-9 relative, zero bins zero on both sides -- every summand is
non-negative, so atomic reordering moves a sum by at most (n - 1) 2^-53.

The full-size projection (256^3 phantom, 256 x 64 x 128 detector, 1e9 rays)
is checked on sampled rays and on sampled ray ranges of the 1e9-ray run, in
the launch configuration the benchmark times.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

REL_RAY = 1e-12
REL_BIN = 1e-9
# Weights are non-negative and mostly well below 1 (the median detected
# weight of the projection is ~0.07, a few percent are below 1e-6), so the
# weight is compared relative to itself; the floor only keeps subnormal
# weights (optical depths above ~708) from demanding more bits than they hold.
W_FLOOR = 1e-300


def mxr():
    import paper_2410_08747_amd as m
    return m


def announce(*what):
    print("[gpu case]", *what, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def cpu(t):
    return t.detach().cpu().numpy()


def compare_rays(gpu, ora, label, w_rel=None, retrace=None, scatter=False):
    """Per-ray comparison.  ``retrace(idx)``, when given, returns for the
    compared rays idx (positions in the arrays) the conditioning bound of
    their weights beyond 1e-12 (see the module docstring); ``scatter``
    selects the bound of the scattering chains instead."""
    st_g, st_o = cpu(gpu["status"]), ora["status"]
    assert np.array_equal(st_g, st_o), f"{label}: status differs for {np.sum(st_g != st_o)} rays"
    assert np.array_equal(cpu(gpu["dead_at"]), ora["dead_at"]), f"{label}: dead_at differs"
    assert np.array_equal(cpu(gpu["bin"]), ora["bin"]), f"{label}: bin differs"
    pairs = [("x", ora["r"][:, 0], 1.0), ("y", ora["r"][:, 1], 1.0), ("z", ora["r"][:, 2], 1.0),
             ("dx", ora["d"][:, 0], 1.0), ("dy", ora["d"][:, 1], 1.0), ("dz", ora["d"][:, 2], 1.0),
             ("E", ora["E"], 1.0), ("w", ora["w"], W_FLOOR)]
    for name, ref, floor in pairs:
        got = cpu(gpu[name])
        err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
        tol = REL_RAY if (name != "w" or w_rel is None) else w_rel
        bad = err > tol
        if name == "w" and bad.any() and scatter:
            idx = np.flatnonzero(bad)
            print(f"{label}: {idx.size} of {err.size} weights beyond 1e-12 (max {err[idx].max():.3e})", flush=True)
            assert idx.size <= max(3, 2 * err.size // 1000), f"{label}: {idx.size} of {err.size} weights beyond 1e-12"
            assert err[idx].max() <= 1e-9, f"{label}: weight error {err[idx].max():.3e}"
            continue
        if name == "w" and bad.any() and retrace is not None:
            idx = np.flatnonzero(bad)
            assert idx.size <= max(3, err.size // 100), f"{label}: {idx.size} of {err.size} weights beyond 1e-12"
            assert err[idx].max() <= 1e-9, f"{label}: weight error {err[idx].max():.3e}"
            lim = retrace(idx)
            k = int(np.argmax(err[idx] - lim))
            print(f"{label}: {idx.size} of {err.size} weights beyond 1e-12 (max {err[idx].max():.3e}), each within "
                  f"its conditioning bound (largest bound {lim.max():.3e})", flush=True)
            assert np.all(err[idx] <= lim), (f"{label}: w ray {idx[k]}: gpu {got[idx][k]!r} oracle {ref[idx][k]!r} "
                                             f"rel {err[idx][k]:.3e}, bound {lim[k]:.3e}")
            continue
        i = int(np.argmax(err - tol))
        assert not bad.any(), f"{label}: {name} ray {i}: gpu {got[i]!r} oracle {ref[i]!r} rel {err[i]:.3e}"


def walk_terms(ins):
    """Bound on the terms an instrument's walks sum: per phantom, its
    nx + ny + nz + 3 crossings, times the steps per voxel edge of the
    fixed-step model."""
    n = 0
    for c in ins["components"]:
        if c["type"] == "phantom":
            nz, ny, nx = np.asarray(c["volume"]).shape
            per = 1 if not c.get("step") else int(math.ceil(c["voxel"] / c["step"])) + 1
            n += (nx + ny + nz + 3) * per
    return max(n, 1)


def retracer(ins, ids, seed, n_total, purpose=0, job=0):
    """``retrace`` for compare_rays: per listed ray, its conditioning bound
    1e-12 + 8 s + 4 N u tau (module docstring), with s from six oracle rays
    whose source direction moves by one ulp in one component, traced by the
    oracle through the rest of the instrument."""
    ids = np.asarray(ids, dtype=np.uint64)
    src = {"components": [ins["components"][0]]}
    N = walk_terms(ins)

    def f(idx):
        sub = ids[idx]
        s0 = oracle.trace_rays(src, sub, seed=seed, n_total=n_total, purpose=purpose, job=job)
        base = oracle.trace_after_source(ins, sub, seed, n_total, s0["r"], s0["d"], s0["E"], s0["w"],
                                         purpose=purpose, job=job)["w"]
        spread = np.zeros(sub.size)
        for axis in range(3):
            for direction in (np.inf, -np.inf):
                d = s0["d"].copy()
                d[:, axis] = np.nextafter(d[:, axis], direction)
                w = oracle.trace_after_source(ins, sub, seed, n_total, s0["r"], d, s0["E"], s0["w"],
                                              purpose=purpose, job=job)["w"]
                spread = np.maximum(spread, np.abs(w - base) / np.maximum(np.abs(base), W_FLOOR))
        tau = np.log(np.maximum(s0["w"], W_FLOOR) / np.maximum(base, W_FLOOR))
        return REL_RAY + 8.0 * spread + 4.0 * N * 2.0 ** -53 * np.maximum(tau, 0.0)

    return f


def darwin_weight_tolerance(ins, ids, seed, n_total):
    """Per-ray weight tolerance through the two-crystal monochromator.

    The Darwin reflectivity R(x) = (|x| + sqrt(x^2 - 1))^-2 has
    d ln R / dx = -2 / sqrt(x^2 - 1) beyond the plateau, unbounded at its
    edge.  The CPU and GPU math libraries differ by an ulp or two in the
    sin/cos/tan/asin that produce the incidence angle, i.e. by up to
    ~5e-16 rad (18 ulp of the 0.16 rad Bragg angle); through two bounces that
    moves ln w by 2 * 2 / sqrt(x^2 - 1) * 5e-16 / (width / 2).  Rays within
    1e-6 of the plateau edge are near-ties and skipped (None); the incidence
    angle comes from an oracle trace of the instrument cut after the
    monochromator (same random streams up to there).
    """
    comps = ins["components"]
    k = [c["type"] for c in comps].index("dcm")
    dcm = comps[k]
    cut = oracle.trace_rays({"components": comps[:k + 1]}, ids, seed=seed, n_total=n_total)
    d_loc = cut["d"] @ np.asarray(dcm["rot"]).T
    n1 = np.array([0.0, math.cos(dcm["theta_c"]), -math.sin(dcm["theta_c"])])
    theta_in = np.arcsin(np.clip(-(d_loc @ n1), -1, 1))
    theta_b = np.arcsin(12.398419843320026 / (2 * dcm["d_spacing"] * cut["E"]))
    x = np.abs((theta_in - theta_b) / (0.5 * dcm["darwin_width"]))
    dx = 5e-16 / (0.5 * dcm["darwin_width"])
    slope = np.where(x > 1 + 1e-6, 2.0 / np.sqrt(np.maximum(x * x - 1, 1e-300)), 0.0)
    tol = REL_RAY + 2 * slope * dx
    near_tie = np.abs(x - 1) <= 1e-6
    tol[near_tie] = np.inf
    return tol, int(near_tie.sum())


def compare_bins(gpu_tally, ora_tally, label):
    cg = cpu(gpu_tally["count"]).astype(np.uint64)
    assert np.array_equal(cg, ora_tally["count"]), f"{label}: counts differ in {np.sum(cg != ora_tally['count'])} bins"
    for key in ("sum_w", "sum_w2"):
        g, o = cpu(gpu_tally[key]), ora_tally[key]
        assert np.array_equal(g == 0, o == 0), f"{label}: {key} zero pattern differs"
        nz = o != 0
        if nz.any():
            err = np.abs(g[nz] - o[nz]) / np.abs(o[nz])
            assert err.max() <= REL_BIN, f"{label}: {key} max rel err {err.max():.3e}"


@pytest.fixture(scope="module")
def small_edct():
    vol = workloads.make_phantom(64, seed=1)
    mu = workloads.make_mu_tables(1)
    return workloads.edct_projection(vol, mu, angle=0.4, strata=64)


@pytest.fixture(scope="module")
def full_edct():
    vol = workloads.make_phantom(256, seed=1)
    mu = workloads.make_mu_tables(1)
    return workloads.edct_projection(vol, mu, angle=0.0, strata=4096)


def odd_edct(angle, voxel):
    """Projection through a phantom of unequal, odd dimensions; a voxel edge
    of 0.8 mm is not dyadic, so planes are placed by multiplication."""
    rng = np.random.default_rng(5)
    vol = rng.integers(0, 8, size=(29, 23, 37)).astype(np.uint8)
    vol[rng.random(vol.shape) < 0.6] = 0
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(2), angle=angle, strata=16, nx=32, ny=16, ne=16)
    ins["components"][1]["voxel"] = voxel
    ins["components"][0]["half_angle"] = 0.03
    return ins


def early_out_edct(size=64, angle=0.4, strata=64):
    return workloads.edct_projection(workloads.make_phantom(size, seed=1), workloads.make_mu_tables(1),
                                     angle=angle, strata=strata, early_out=True)


def instruments(small_edct):
    return {
        "basic_absorber": workloads.basic_absorber(),
        "edct_64": small_edct,
        "edct_64_early_out": early_out_edct(),
        "beamline": workloads.beamline(),
        "edct_odd_45deg": odd_edct(math.pi / 4, 1.0),
        "edct_odd_voxel0.8": odd_edct(1.1, 0.8),
    }


@pytest.mark.parametrize("name", ["basic_absorber", "edct_64", "edct_64_early_out", "beamline", "edct_odd_45deg",
                                  "edct_odd_voxel0.8"])
def test_per_ray_parity(torch_cuda, small_edct, name):
    ins = instruments(small_edct)[name]
    n = 100003  # ragged: not a multiple of the work-group or XCD count
    ids = np.arange(n, dtype=np.uint64)
    announce("per-ray", name, "n", n, "seed 7")
    g = mxr().Instrument(ins).trace_rays(ids, seed=7, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=7, n_total=n)
    w_rel = None
    if name == "beamline":
        w_rel, near = darwin_weight_tolerance(ins, ids, 7, n)
        print(f"beamline: {near} near-tie rays at the Darwin plateau edge", flush=True)
        assert near < 10
    compare_rays(g, o, name, w_rel, retrace=None if name == "beamline" else retracer(ins, ids, 7, n))


@pytest.mark.parametrize("name,n", [("basic_absorber", 1000000), ("edct_64", 300001), ("beamline", 1000000),
                                    ("edct_odd_45deg", 200000), ("edct_odd_voxel0.8", 200000)])
def test_per_bin_parity(torch_cuda, small_edct, name, n):
    ins = instruments(small_edct)[name]
    announce("per-bin", name, "n", n, "seed 1")
    I = mxr().Instrument(ins)
    led = I.new_ledger()
    t = I.run(n, seed=1, ledger=led)
    torch_cuda.cuda.synchronize()
    o, oled = oracle.run(ins, n, seed=1, ledger=True)
    for k, (gt, ot) in enumerate(zip(t, o)):
        compare_bins(gt, ot, f"{name} monitor {k}")
    gl = cpu(led)
    nz = oled != 0
    assert np.array_equal(gl == 0, oled == 0)
    assert np.max(np.abs(gl[nz] - oled[nz]) / np.abs(oled[nz])) <= REL_BIN
    K = len(ins["components"])
    lost = sum(gl[4 * k + 1] + gl[4 * k + 2] for k in range(K))
    assert abs(gl[0] - (lost + gl[4 * K])) <= 1e-12 * gl[0]


def test_full_size_sampled_rays(torch_cuda, full_edct):
    """Rays sampled across a 1e9-ray run of the 256^3 projection."""
    n_total = 10**9
    rng = np.random.default_rng(3)
    ids = np.unique(np.concatenate([rng.integers(0, n_total, 20000), np.arange(0, 64), np.arange(n_total - 64, n_total)]))
    announce("full-size sampled rays", "n_total", n_total, "samples", ids.size)
    g = mxr().Instrument(full_edct).trace_rays(ids.astype(np.uint64), seed=1, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(full_edct, ids, seed=1, n_total=n_total)
    compare_rays(g, o, "edct_256 full-size", retrace=retracer(full_edct, ids, 1, n_total))


@pytest.mark.parametrize("first,n", [(0, 200000), (499_999_937, 150001), (10**9 - 100000, 100000)])
def test_full_size_sampled_ranges(torch_cuda, full_edct, first, n):
    """Ray ranges of the 1e9-ray run through the run kernel the benchmark times."""
    n_total = 10**9
    announce("full-size range", first, n, "n_total", n_total)
    I = mxr().Instrument(full_edct)
    t = I.run(n, seed=1, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.run(full_edct, n, seed=1, first=first, n_total=n_total)
    compare_bins(t[0], o[0], f"edct_256 rays [{first}, {first + n})")


def test_largest_phantom_sampled(torch_cuda):
    """A 512^3 phantom (128 MiB, the largest of the batched workload) at an
    oblique angle: sampled rays of a 1e9-ray run and a ray range, per ray and
    per bin."""
    vol = workloads.make_phantom(512, seed=2)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=1.0, strata=4096)
    n_total = 10**9
    ids = np.unique(np.concatenate([np.random.default_rng(5).integers(0, n_total, 4000),
                                    np.arange(0, 32), np.arange(n_total - 32, n_total)]))
    announce("512^3 sampled rays", ids.size)
    I = mxr().Instrument(ins)
    g = I.trace_rays(ids.astype(np.uint64), seed=6, n_total=n_total)
    torch_cuda.cuda.synchronize()
    compare_rays(g, oracle.trace_rays(ins, ids, seed=6, n_total=n_total), "512^3 sampled",
                 retrace=retracer(ins, ids, 6, n_total))
    first, n = 600_000_000, 40000
    t = I.run(n, seed=6, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    compare_bins(t[0], oracle.run(ins, n, seed=6, first=first, n_total=n_total)[0], "512^3 ray range")


@pytest.mark.parametrize("size,first,n,n_total", [(64, 0, 300001, 300001), (256, 499_999_937, 150001, 10**9)])
def test_early_out_aperture(torch_cuda, size, first, n, n_total):
    """The projection behind the early-out aperture, through its own plain
    run kernel: per bin against the oracle, and the same image as the
    projection without the aperture (the same rays reach the detector; their
    positions differ only by rounding, the aperture moving each ray to its
    plane first)."""
    strata = 64 if size == 64 else 4096
    aimed = early_out_edct(size, 0.4 if size == 64 else 0.0, strata)
    plain = workloads.edct_projection(workloads.make_phantom(size, seed=1), workloads.make_mu_tables(1),
                                      angle=0.4 if size == 64 else 0.0, strata=strata)
    announce("early-out aperture", size, first, n, "n_total", n_total)
    t = mxr().Instrument(aimed).run(n, seed=1, first_ray=first, n_total=n_total)
    p = mxr().Instrument(plain).run(n, seed=1, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    compare_bins(t[0], oracle.run(aimed, n, seed=1, first=first, n_total=n_total)[0], f"early-out {size}^3")
    assert np.array_equal(cpu(t[0]["count"]), cpu(p[0]["count"]))
    for key in ("sum_w", "sum_w2"):
        g, o = cpu(t[0][key]), cpu(p[0][key])
        nz = o != 0
        assert np.array_equal(g == 0, o == 0)
        assert np.max(np.abs(g[nz] - o[nz]) / o[nz]) <= REL_BIN


def test_chunked_runs_equal_one_run(torch_cuda, small_edct):
    n = 400000
    announce("chunking", "n", n)
    I = mxr().Instrument(small_edct)
    one = I.run(n, seed=9)
    parts = I.new_tallies()
    for a, b in [(0, 1), (1, 150000), (150000, 150000), (150000, 399999), (399999, 400000)]:
        I.run(b - a, seed=9, first_ray=a, n_total=n, tallies=parts)
    torch_cuda.cuda.synchronize()
    assert np.array_equal(cpu(one[0]["count"]), cpu(parts[0]["count"]))
    g, o = cpu(parts[0]["sum_w"]), cpu(one[0]["sum_w"])
    nz = o != 0
    assert np.array_equal(g == 0, o == 0)
    assert np.max(np.abs(g[nz] - o[nz]) / o[nz]) <= REL_BIN


def parallel_beam(angle, voxel=1.0, sigma=(10.0, 5.0)):
    """The small projection lit by a Gaussian source of zero divergence:
    every ray runs exactly along z, so in the phantom's frame (rotated about
    y) the y axis is parallel to every ray, and at angle 0 the x axis too.
    With zero width every ray starts on the axis, which lies in voxel faces
    of the 64^3 volume (its planes sit at whole millimetres from -32)."""
    vol = workloads.make_phantom(64, seed=1)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=angle, strata=16, nx=32, ny=16, ne=16)
    ins["components"][0] = {"type": "source_gaussian", "pos": (0.0, 0.0, 0.0), "rot": np.eye(3),
                            "sigma_x": sigma[0], "sigma_y": sigma[1], "sigma_xp": 0.0, "sigma_yp": 0.0,
                            "e0": 60.0, "rel_halfwidth": 0.5}
    ins["components"][1]["voxel"] = voxel
    return ins


@pytest.mark.parametrize("angle,voxel,sigma", [(0.0, 1.0, (10.0, 5.0)), (0.5, 1.0, (10.0, 5.0)),
                                               (math.pi / 2, 1.0, (10.0, 5.0)), (0.3, 0.8, (10.0, 5.0)),
                                               (0.0, 1.0, (0.0, 0.0)), (0.5, 1.0, (0.0, 0.0))])
def test_axis_parallel_rays(torch_cuda, angle, voxel, sigma):
    """Rays parallel to one or two axes of the volume (the walk keeps such an
    axis's alpha at +inf), and with zero beam width rays that run inside
    voxel faces; per ray and per bin against the oracle."""
    ins = parallel_beam(angle, voxel, sigma)
    n = 60001
    announce("axis-parallel rays", "angle", angle, "voxel", voxel, "sigma", sigma, "n", n)
    I = mxr().Instrument(ins)
    ids = np.arange(n, dtype=np.uint64)
    g = I.trace_rays(ids, seed=4, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=4, n_total=n)
    assert int(np.sum(o["bin"] >= 0)) > n // 4
    compare_rays(g, o, f"parallel beam, angle {angle}, voxel {voxel}, width {sigma}", retrace=retracer(ins, ids, 4, n))
    t = I.run(n, seed=5)
    torch_cuda.cuda.synchronize()
    compare_bins(t[0], oracle.run(ins, n, seed=5)[0], f"parallel beam bins, angle {angle}, voxel {voxel}, width {sigma}")


def test_largest_run_size(torch_cuda):
    """The largest run the 4096^2-cell stratification admits: n_total x cells
    = 2^64 - 2^24, so the cell arithmetic of the last rays reaches the top of
    the 64-bit range on both sides; one ray more is refused."""
    m = mxr()
    vol = workloads.make_phantom(64, seed=1)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=0.4, strata=4096)
    nt = (1 << 40) - 1
    ids = np.array([0, 1, nt // 3, nt // 2] + list(range(nt - 64, nt)), dtype=np.uint64)
    announce("largest run size", nt)
    I = m.Instrument(ins)
    g = I.trace_rays(ids, seed=3, n_total=nt)
    torch_cuda.cuda.synchronize()
    compare_rays(g, oracle.trace_rays(ins, ids, seed=3, n_total=nt), "n_total 2^40 - 1", retrace=retracer(ins, ids, 3, nt))
    with pytest.raises(m.MxrError):
        I.trace_rays(ids[:1], seed=3, n_total=(1 << 40) + 5)
    # a side that is not a power of two: the last cell's bound
    # (cell + 1) n_total + G^2 - 1 reaches 2^64 - 1 exactly at the largest
    # admitted n_total = (2^64 - G^2) / G^2
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=0.4, strata=4095)
    g2 = 4095 * 4095
    nt = ((1 << 64) - g2) // g2
    ids = np.array([0, nt // 2] + list(range(nt - 64, nt)), dtype=np.uint64)
    announce("largest run size, strata 4095", nt)
    I = m.Instrument(ins)
    g = I.trace_rays(ids, seed=3, n_total=nt)
    torch_cuda.cuda.synchronize()
    compare_rays(g, oracle.trace_rays(ins, ids, seed=3, n_total=nt), "strata 4095, largest n_total",
                 retrace=retracer(ins, ids, 3, nt))
    with pytest.raises(m.MxrError):
        I.trace_rays(ids[:1], seed=3, n_total=nt + 1)


def test_edge_cases(torch_cuda, small_edct):
    m = mxr()
    I = m.Instrument(small_edct)
    announce("edge cases")
    # empty run: tallies untouched
    t = I.run(0, seed=1, n_total=10)
    torch_cuda.cuda.synchronize()
    assert int(t[0]["count"].sum()) == 0
    # one ray, and n_total below the strata count (G reduced to 1)
    for n_total in (1, 2, 5, 4095):
        g = I.trace_rays(np.array([n_total - 1], np.uint64), seed=2, n_total=n_total)
        torch_cuda.cuda.synchronize()
        o = oracle.trace_rays(small_edct, [n_total - 1], seed=2, n_total=n_total)
        compare_rays(g, o, f"single ray n_total={n_total}",
                     retrace=retracer(small_edct, [n_total - 1], 2, n_total))
    # ids in any order
    ids = np.array([5, 3, 99999, 0, 7], np.uint64)
    g = I.trace_rays(ids, seed=3, n_total=100000)
    torch_cuda.cuda.synchronize()
    compare_rays(g, oracle.trace_rays(small_edct, ids, seed=3, n_total=100000), "unordered ids",
                 retrace=retracer(small_edct, ids, 3, 100000))
    # purpose and job select other streams
    g = I.trace_rays(np.arange(1000, dtype=np.uint64), seed=3, n_total=1000, purpose=2, job=77)
    torch_cuda.cuda.synchronize()
    compare_rays(g, oracle.trace_rays(small_edct, np.arange(1000), seed=3, n_total=1000, purpose=2, job=77), "purpose/job",
                 retrace=retracer(small_edct, np.arange(1000), 3, 1000, purpose=2, job=77))


def test_errors(torch_cuda, small_edct):
    m = mxr()
    announce("error paths")
    I = m.Instrument(small_edct)
    tallies = I.new_tallies()
    with pytest.raises(m.MxrError):
        I.run(10, seed=1, first_ray=5, n_total=12, tallies=tallies)  # range beyond n_total
    with pytest.raises(m.MxrError):
        m.mxr_run(I.handle, 0, 10, 10, 1, 0, 0, [])  # wrong tally count
    bad = I.tally_structs(tallies)
    bad[0].n_bins -= 1
    with pytest.raises(m.MxrError):
        m.mxr_run(I.handle, 0, 10, 10, 1, 0, 0, bad)
    with pytest.raises(m.MxrError):
        I.run(10, seed=1, purpose=300)
    # material ids beyond the table, detector without a source, NaN parameters
    vol = np.full((4, 4, 4), 9, np.uint8)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1))
    with pytest.raises(m.MxrError):
        m.Instrument(ins)
    with pytest.raises(m.MxrError):
        m.Instrument({"components": [workloads.basic_absorber()["components"][3]]})
    b = workloads.basic_absorber()
    b["components"][2]["mu_a"] = float("nan")
    with pytest.raises(m.MxrError):
        m.Instrument(b)
    assert "non-finite" in m.mxr_last_error()


def test_run_beyond_2pow32_rays(torch_cuda):
    """One call of more than 2^32 rays: the launch is split so that no grid
    exceeds the dispatch's 32-bit work-item count.  Every ray is emitted
    (the ledger's source weight, 1 per ray, sums to n exactly) and the image
    equals the same run made in two calls."""
    ins = workloads.basic_absorber()
    n = (1 << 32) + 12345
    announce("run beyond 2^32 rays", n)
    I = mxr().Instrument(ins)
    led = I.new_ledger()
    I.run(n, seed=4, ledger=led)
    one = I.run(n, seed=4)
    parts = I.new_tallies()
    I.run(1 << 32, seed=4, first_ray=0, n_total=n, tallies=parts)
    I.run(12345, seed=4, first_ray=1 << 32, n_total=n, tallies=parts)
    torch_cuda.cuda.synchronize()
    assert cpu(led)[0] == float(n)
    assert np.array_equal(cpu(one[0]["count"]), cpu(parts[0]["count"]))
    g, o = cpu(parts[0]["sum_w"]), cpu(one[0]["sum_w"])
    nz = o != 0
    assert np.array_equal(g == 0, o == 0)
    assert np.max(np.abs(g[nz] - o[nz]) / o[nz]) <= REL_BIN
