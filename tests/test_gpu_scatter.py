"""Parity of the scattering phantom (photons scattered exactly K times,
forced interactions; section 3.3) between the HIP library and the CPU
oracle, through the C ABI: per ray identical status, absorbing component
and bin, states within 1e-12 relative; per bin identical counts, sums
within 1e-9; the 256^3 benchmark run on sampled rays and ray ranges.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from test_gpu_batch import same_tally
from test_gpu_parity import announce, compare_bins, compare_rays, cpu, mxr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def tables(seed=1):
    return workloads.make_scatter_tables(workloads.make_mu_tables(seed), seed)


def variant(name):
    vol = workloads.make_phantom(64, seed=1)
    small = dict(strata=64, nx=64, ny=32, ne=32)
    if name == "order1_aimed":
        return workloads.edct_projection(vol, tables(), angle=0.4, scatter_order=1, **small)
    if name == "order2_aimed":
        return workloads.edct_projection(vol, tables(), angle=1.3, scatter_order=2, **small)
    if name == "order1_isotropic":
        return workloads.edct_projection(vol, tables(), angle=2.2, scatter_order=1, aim=False, **small)
    if name == "order3_aimed_voxel0.8":
        ins = workloads.edct_projection(vol, tables(2), angle=0.7, scatter_order=3, **small)
        ins["components"][1]["voxel"] = 0.8  # planes placed by multiplication
        return ins
    if name == "order1_generic":
        ins = workloads.edct_projection(vol, tables(), angle=0.2, scatter_order=1, **small)
        slit = {"type": "slit", "pos": (0.0, 0.0, 500.0), "rot": np.eye(3), "w": 60.0, "h": 30.0}
        ins["components"].insert(1, slit)
        return ins
    if name == "order1_parallel":
        # a zero-divergence source: every primary ray parallel to the volume's y axis
        ins = workloads.edct_projection(vol, tables(), angle=0.5, scatter_order=1, **small)
        ins["components"][0] = {"type": "source_gaussian", "pos": (0.0, 0.0, 0.0), "rot": np.eye(3),
                                "sigma_x": 10.0, "sigma_y": 5.0, "sigma_xp": 0.0, "sigma_yp": 0.0,
                                "e0": 60.0, "rel_halfwidth": 0.5}
        return ins
    raise KeyError(name)


NAMES = ["order1_aimed", "order2_aimed", "order1_isotropic", "order3_aimed_voxel0.8", "order1_generic",
         "order1_parallel"]


@pytest.mark.parametrize("name", NAMES)
def test_per_ray_parity(torch_cuda, name):
    ins = variant(name)
    n = 100003
    ids = np.arange(n, dtype=np.uint64)
    announce("scatter per-ray", name, "n", n, "seed 7")
    g = mxr().Instrument(ins).trace_rays(ids, seed=7, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=7, n_total=n)
    print(f"{name}: {int(np.sum(o['bin'] >= 0))} rays tallied", flush=True)
    compare_rays(g, o, name, scatter=True)


@pytest.mark.parametrize("name", NAMES)
def test_per_bin_parity(torch_cuda, name):
    ins = variant(name)
    n = 200001
    announce("scatter per-bin", name, "n", n, "seed 1")
    I = mxr().Instrument(ins)
    led = I.new_ledger()
    t = I.run(n, seed=1, ledger=led)
    torch_cuda.cuda.synchronize()
    o, oled = oracle.run(ins, n, seed=1, ledger=True)
    assert o[0]["count"].sum() > 0
    compare_bins(t[0], o[0], name)
    gl = cpu(led)
    nz = oled != 0
    assert np.array_equal(gl == 0, oled == 0)
    assert np.max(np.abs(gl[nz] - oled[nz]) / np.abs(oled[nz])) <= 1e-9


@pytest.fixture(scope="module")
def full_scatter():
    vol = workloads.make_phantom(256, seed=1)
    return workloads.edct_projection(vol, tables(), angle=0.0, strata=4096, scatter_order=1)


def test_full_size_sampled_rays(torch_cuda, full_scatter):
    n_total = 10**9
    rng = np.random.default_rng(10)
    ids = np.unique(np.concatenate([rng.integers(0, n_total, 5000), np.arange(0, 64),
                                    np.arange(n_total - 64, n_total)]))
    announce("scatter full-size sampled rays", ids.size)
    g = mxr().Instrument(full_scatter).trace_rays(ids.astype(np.uint64), seed=1, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(full_scatter, ids, seed=1, n_total=n_total)
    compare_rays(g, o, "scatter 256 full-size", scatter=True)


@pytest.mark.parametrize("first,n", [(0, 50000), (10**9 - 40000, 40000)])
def test_full_size_sampled_ranges(torch_cuda, full_scatter, first, n):
    n_total = 10**9
    announce("scatter full-size range", first, n)
    t = mxr().Instrument(full_scatter).run(n, seed=1, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.run(full_scatter, n, seed=1, first=first, n_total=n_total)
    compare_bins(t[0], o[0], f"scatter 256 rays [{first}, {first + n})")


def test_batch_of_scatter_jobs(torch_cuda):
    m = mxr()
    vol = workloads.make_phantom(48, seed=2)
    tab = tables()
    shared, jobs = {}, []
    for k, (a, nr) in enumerate([(0.0, 30001), (1.0, 257), (2.5, 50000)]):
        ins = workloads.edct_projection(vol, tab, angle=a, strata=16, nx=32, ny=16, ne=32, scatter_order=1)
        I = m.Instrument(ins, shared=shared)
        jobs.append((I, nr, 5 + k, 3, I.new_tallies()))
    announce("scatter batch", len(jobs))
    ref = [I.run(nr, seed=seed, job=job) for I, nr, seed, job, _ in jobs]
    for schedule in [(0, 0, 256, 0), (1, 2, 4096, 0), (2, 0, 256, 2)]:
        for j in jobs:
            for v in j[4][0].values():
                v.zero_()
        B = m.Batch(jobs, schedule=schedule)
        B.run()
        torch_cuda.cuda.synchronize()
        for k, (j, r) in enumerate(zip(jobs, ref)):
            same_tally(j[4][0], r[0], f"scatter batch job {k} schedule {schedule}")
        B.close()


def test_errors(torch_cuda):
    m = mxr()
    vol = workloads.make_phantom(48, seed=1)
    tab = tables()
    base = lambda **kw: workloads.edct_projection(vol, tab, strata=16, **kw)
    cases = []
    for K in (0, 4, 1.5):
        ins = base(scatter_order=1)
        ins["components"][1]["scatter_order"] = K
        cases.append((ins, -1, "scatter order"))
    ins = base(scatter_order=1)
    ins["components"][1]["step"] = 0.3  # both models
    cases.append((ins, -1, "flags"))
    ins = base(scatter_order=1)
    ins["components"][1]["scatter_target"] = ((0, 0, 1200.0), (1.0, 0, 0), (2.0, 0, 0))  # parallel axes
    cases.append((ins, -1, "target"))
    ins = base(scatter_order=1)
    ins["components"][1]["mu_table"] = workloads.make_mu_tables(1)  # one channel only
    cases.append((ins, None, ""))
    for ins, status, word in cases:
        announce("scatter errors", word)
        with pytest.raises(m.MxrError) as e:
            m.Instrument(ins)
        if status is not None:
            assert e.value.status == status and word in str(e.value)
