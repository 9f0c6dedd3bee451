"""Parity of the compound refractive lens and the focusing instrument
(paper, section 3.2) between the HIP library and the CPU oracle, through the
C ABI: per ray identical status, absorbing component and bin, states within
1e-12 relative; per bin identical counts, sums within 1e-9; the 1e9-ray
benchmark run on sampled rays and ray ranges.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import announce, compare_bins, compare_rays, retracer, cpu, mxr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def variant(name):
    ins = workloads.crl_focusing()
    comps = ins["components"]
    if name == "crl_16":
        return ins
    if name == "crl_strong_tilted":
        # exaggerated refraction (delta 2e-5: focus ~0.3 m) and a lens frame
        # turned by a few mrad, monitors at the new focus
        lens = dict(comps[2])
        lens["delta_ref"] = 2e-5
        a = 3e-3
        lens["rot"] = np.array([[np.cos(a), 0, -np.sin(a)], [0, 1, 0], [np.sin(a), 0, np.cos(a)]])
        z = workloads.CRL_LENS_DIST + 320.0
        return {"components": [comps[0], comps[1], lens,
                               {**comps[4], "pos": (0.0, 0.0, z), "xmin": -1.0, "xmax": 1.0, "ymin": -1.0, "ymax": 1.0},
                               {**comps[5], "pos": (0.0, 0.0, z + 1.0), "xmin": -1.0, "xmax": 1.0, "ymin": -1.0,
                                "ymax": 1.0}]}
    if name == "crl_generic":
        # no crop: the lens aperture does the cropping; a box after the lens
        # makes the chain generic
        box = {"type": "box", "pos": (0.0, 0.0, workloads.CRL_LENS_DIST + 200.0), "rot": np.eye(3),
               "hx": 5.0, "hy": 5.0, "hz": 2.0, "mu_a": 950.0, "mu_b": 0.3}
        return {"components": [comps[0], comps[2], box, comps[3], comps[4], comps[5]]}
    raise KeyError(name)


NAMES = ["crl_16", "crl_strong_tilted", "crl_generic"]


@pytest.mark.parametrize("name", NAMES)
def test_per_ray_parity(torch_cuda, name):
    ins = variant(name)
    n = 400003
    ids = np.arange(n, dtype=np.uint64)
    announce("lens per-ray", name, "n", n, "seed 7")
    g = mxr().Instrument(ins).trace_rays(ids, seed=7, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=7, n_total=n)
    lens_k = [c["type"] for c in ins["components"]].index("lens_crl")
    through = np.sum((o["dead_at"] < 0) | (o["dead_at"] > lens_k))
    print(f"{name}: {through} rays through the lens", flush=True)
    assert through > 1000
    compare_rays(g, o, name, retrace=retracer(ins, ids, 7, n))


@pytest.mark.parametrize("name", NAMES)
def test_per_bin_parity(torch_cuda, name):
    ins = variant(name)
    n = 2000001
    announce("lens per-bin", name, "n", n, "seed 1")
    I = mxr().Instrument(ins)
    led = I.new_ledger()
    t = I.run(n, seed=1, ledger=led)
    torch_cuda.cuda.synchronize()
    o, oled = oracle.run(ins, n, seed=1, ledger=True)
    for k, (gt, ot) in enumerate(zip(t, o)):
        assert ot["count"].sum() > 0
        compare_bins(gt, ot, f"{name} monitor {k}")
    gl = cpu(led)
    nz = oled != 0
    assert np.array_equal(gl == 0, oled == 0)
    assert np.max(np.abs(gl[nz] - oled[nz]) / np.abs(oled[nz])) <= 1e-9


def test_full_size_sampled_rays(torch_cuda):
    """Rays sampled across the 1e9-ray benchmark run."""
    ins = workloads.crl_focusing()
    n_total = 10**9
    rng = np.random.default_rng(9)
    ids = np.unique(np.concatenate([rng.integers(0, n_total, 200000), np.arange(0, 64),
                                    np.arange(n_total - 64, n_total)]))
    announce("lens full-size sampled rays", ids.size)
    g = mxr().Instrument(ins).trace_rays(ids.astype(np.uint64), seed=1, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=1, n_total=n_total)
    compare_rays(g, o, "crl full-size", retrace=retracer(ins, ids, 1, n_total))


@pytest.mark.parametrize("first,n", [(0, 1000000), (10**9 - 524288, 524288)])
def test_full_size_sampled_ranges(torch_cuda, first, n):
    ins = workloads.crl_focusing()
    n_total = 10**9
    announce("lens full-size range", first, n)
    t = mxr().Instrument(ins).run(n, seed=1, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.run(ins, n, seed=1, first=first, n_total=n_total)
    for k, (gt, ot) in enumerate(zip(t, o)):
        compare_bins(gt, ot, f"crl rays [{first}, {first + n}) monitor {k}")


def test_errors(torch_cuda):
    m = mxr()
    base = workloads.crl_focusing()
    for key, val in [("pitch", 0.5), ("n_lenses", 0), ("n_lenses", 2.5), ("delta_ref", 0.6), ("R", 0.0),
                     ("aperture", -1.0)]:
        ins = {"components": [dict(c) for c in base["components"]]}
        ins["components"][2][key] = val
        announce("lens errors", key, val)
        with pytest.raises(m.MxrError) as e:
            m.Instrument(ins)
        assert e.value.status == -1 and "lens" in str(e.value)


@pytest.mark.parametrize("name", ["crl_16", "basic_absorber"])
@pytest.mark.parametrize("first,n", [(0, 1), (5, 63), (0, 4097), (123, 1000003)])
def test_compacted_runs(torch_cuda, name, first, n):
    """Plain runs of chains with a crop right after the source go through
    the survivor-compacting kernel: ragged sizes (one ray, part of a wave,
    one past a work-group's 4096 ids, many work-groups) against the oracle."""
    ins = workloads.crl_focusing() if name == "crl_16" else workloads.basic_absorber()
    n_total = first + n + 17
    announce("compacted run", name, first, n)
    t = mxr().Instrument(ins).run(n, seed=3, first_ray=first, n_total=n_total)
    torch_cuda.cuda.synchronize()
    o = oracle.run(ins, n, seed=3, first=first, n_total=n_total)
    for k, (gt, ot) in enumerate(zip(t, o)):
        compare_bins(gt, ot, f"{name} compacted [{first}, {first + n}) monitor {k}")
