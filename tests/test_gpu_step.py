"""Parity of the fixed-step phantom model (the paper's default crossing of the
voxel sample, section 3.3) between the HIP library and the CPU oracle,
through the C ABI.

Same bar as the exact path: per ray identical status, absorbing component
and bin, states within 1e-12 relative; per bin identical counts, sums within
1e-9.  Both sides compute each step's voxel from the step index with the
same FP64 operations (the kernel truncates and clamps where the oracle
floors and clamps: the same integer for every value in range), so voxel
choices agree exactly and only the summation order of the optical depth
differs.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from test_gpu_batch import same_tally
from test_gpu_parity import announce, compare_bins, compare_rays, retracer, cpu, mxr, odd_edct, parallel_beam

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def with_step(ins, step):
    ins["components"][1]["step"] = step
    return ins


def stepped(name):
    mu = workloads.make_mu_tables(1)
    if name == "edct_64_third":
        return workloads.edct_projection(workloads.make_phantom(64, seed=1), mu, angle=0.4, strata=64, step=1.0 / 3.0)
    if name == "edct_64_coarse":
        # steps longer than a voxel (1.7 mm)
        return workloads.edct_projection(workloads.make_phantom(64, seed=1), mu, angle=2.0, strata=64, step=1.7)
    if name == "odd_45deg_third":
        return with_step(odd_edct(math.pi / 4, 1.0), 1.0 / 3.0)
    if name == "odd_voxel0.8_third":
        return with_step(odd_edct(1.1, 0.8), 0.8 / 3.0)
    if name == "slit_generic":
        # a slit before the phantom: the generic chain dispatches the model
        ins = workloads.edct_projection(workloads.make_phantom(64, seed=3), mu, angle=0.9, strata=64,
                                        step=1.0 / 3.0)
        slit = {"type": "slit", "pos": (0.0, 0.0, 500.0), "rot": np.eye(3), "w": 60.0, "h": 30.0}
        ins["components"].insert(1, slit)
        return ins
    if name == "parallel_third":
        # every ray parallel to the y axis of the volume and, at angle 0, to x
        return with_step(parallel_beam(0.0), 1.0 / 3.0)
    if name == "parallel_0.5_third":
        return with_step(parallel_beam(0.5), 1.0 / 3.0)
    raise KeyError(name)


NAMES = ["edct_64_third", "edct_64_coarse", "odd_45deg_third", "odd_voxel0.8_third", "slit_generic",
         "parallel_third", "parallel_0.5_third"]


@pytest.mark.parametrize("name", NAMES)
def test_per_ray_parity(torch_cuda, name):
    ins = stepped(name)
    n = 100003
    ids = np.arange(n, dtype=np.uint64)
    announce("step per-ray", name, "n", n, "seed 7")
    g = mxr().Instrument(ins).trace_rays(ids, seed=7, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=7, n_total=n)
    compare_rays(g, o, name, retrace=retracer(ins, ids, 7, n))


@pytest.mark.parametrize("name", NAMES)
def test_per_bin_parity(torch_cuda, name):
    ins = stepped(name)
    n = 200001
    announce("step per-bin", name, "n", n, "seed 1")
    I = mxr().Instrument(ins)
    led = I.new_ledger()
    t = I.run(n, seed=1, ledger=led)
    torch_cuda.cuda.synchronize()
    o, oled = oracle.run(ins, n, seed=1, ledger=True)
    compare_bins(t[0], o[0], name)
    gl = cpu(led)
    nz = oled != 0
    assert np.array_equal(gl == 0, oled == 0)
    assert np.max(np.abs(gl[nz] - oled[nz]) / np.abs(oled[nz])) <= 1e-9


@pytest.fixture(scope="module")
def full_step():
    vol = workloads.make_phantom(256, seed=1)
    return workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=0.0, strata=4096, step=1.0 / 3.0)


def test_full_size_sampled_rays(torch_cuda, full_step):
    """Rays sampled across a 1e9-ray run of the 256^3 projection."""
    n_total = 10**9
    rng = np.random.default_rng(8)
    ids = np.unique(np.concatenate([rng.integers(0, n_total, 10000), np.arange(0, 64),
                                    np.arange(n_total - 64, n_total)]))
    announce("step full-size sampled rays", ids.size)
    g = mxr().Instrument(full_step).trace_rays(ids.astype(np.uint64), seed=1, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(full_step, ids, seed=1, n_total=n_total)
    compare_rays(g, o, "step edct_256 full-size", retrace=retracer(full_step, ids, 1, n_total))


@pytest.mark.parametrize("first,n", [(0, 100000), (10**9 - 65536, 65536)])
def test_full_size_sampled_ranges(torch_cuda, full_step, first, n):
    """Ray ranges of the 1e9-ray run through the run kernel the benchmark times."""
    n_total = 10**9
    announce("step full-size range", first, n)
    t = mxr().Instrument(full_step).run(n, seed=1, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.run(full_step, n, seed=1, first=first, n_total=n_total)
    compare_bins(t[0], o[0], f"step edct_256 rays [{first}, {first + n})")


def test_batch_of_stepped_jobs(torch_cuda):
    """A batch of fixed-step projections equals the jobs' separate runs in
    every launch form; a batch mixing the two models is rejected."""
    m = mxr()
    mu = workloads.make_mu_tables(1)
    vol = workloads.make_phantom(48, seed=2)
    spec = [(workloads.edct_projection(vol, mu, angle=a, strata=16, nx=32, ny=16, ne=32, step=1.0 / 3.0), nr, 5 + k)
            for k, (a, nr) in enumerate([(0.0, 70001), (1.0, 257), (2.5, 120000)])]
    announce("step batch", len(spec))
    shared = {}
    jobs = []
    for ins, nr, seed in spec:
        I = m.Instrument(ins, shared=shared)
        jobs.append((I, nr, seed, 3, I.new_tallies()))
    ref = [I.run(nr, seed=seed, job=job) for I, nr, seed, job, _ in jobs]
    for schedule in [(0, 0, 256, 0), (1, 2, 4096, 0), (2, 0, 256, 2)]:
        for j in jobs:
            for v in j[4][0].values():
                v.zero_()
        B = m.Batch(jobs, schedule=schedule)
        B.run()
        torch_cuda.cuda.synchronize()
        for k, (j, r) in enumerate(zip(jobs, ref)):
            same_tally(j[4][0], r[0], f"step batch job {k} schedule {schedule}")
        B.close()
    exact = m.Instrument(workloads.edct_projection(vol, mu, angle=0.3, strata=16, nx=32, ny=16, ne=32), shared=shared)
    with pytest.raises(m.MxrError):
        m.Batch(jobs + [(exact, 100, 1, 0, exact.new_tallies())])


def test_errors(torch_cuda):
    m = mxr()
    vol = workloads.make_phantom(64, seed=1)
    mu = workloads.make_mu_tables(1)
    for bad, status in [(0.0, -1), (-0.5, -1), (1e-9, -2)]:  # MXR_E_INVALID, MXR_E_UNSUPPORTED
        announce("step errors", bad)
        with pytest.raises(m.MxrError) as e:
            m.Instrument(workloads.edct_projection(vol, mu, strata=16, step=bad))
        assert e.value.status == status and "step" in str(e.value)
