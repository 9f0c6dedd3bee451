"""Launch shapes of single-instrument runs and their autotuner.

A shape (occupancy the run kernel is compiled for, XCD ray order, survivor
compaction and its rounds) changes how rays map onto the device, never which
rays are traced: every shape's run must equal the default run per bin (counts
identical, sums within the atomic-reordering bound) and the oracle per bin.
The autotuner must pick one of them, set it, and find it again in its cache
file without timing anything.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

from test_gpu_parity import announce, compare_bins

pytestmark = pytest.mark.gpu


def mxr():
    import paper_2410_08747_amd as m
    return m


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def small_edct():
    vol = workloads.make_phantom(64, seed=1)
    return workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=0.5, strata=256, nx=32, ny=16, ne=32)


# XCD order 2 deals runs of 64 tiles; 400,003 rays make 1,563 tiles, 196 per
# XCD, so its last runs are ragged (4 tiles)
SHAPES_EDCT = [(occ, 1, 0, xo) for occ in (0, 4, 6, 8) for xo in (0, 1, 2)]
SHAPES_BASIC = [(occ, c, r, xo) for occ in (0, 6) for c, r in ((1, 0), (1, 16), (1, 1), (0, 0)) for xo in (0, 1, 2)]


@pytest.mark.parametrize("name", ["edct", "basic"])
def test_every_shape_gives_the_same_image(torch_cuda, name):
    m = mxr()
    ins = small_edct() if name == "edct" else workloads.basic_absorber()
    shapes = SHAPES_EDCT if name == "edct" else SHAPES_BASIC
    n = 400_003
    announce("launch shapes", name, "n", n)
    o = oracle.run(ins, n, seed=3)
    I = m.Instrument(ins)
    # launch order by default with a phantom, contiguous eighths without one
    assert I.launch_shape == ((0, 1, 0, 1) if name == "edct" else (0, 1, 0, 0))
    for shape in shapes:
        I.launch_shape = shape
        t = I.run(n, seed=3)
        torch_cuda.cuda.synchronize()
        for k, (gt, ot) in enumerate(zip(t, o)):
            compare_bins(gt, ot, f"{name} shape {shape} monitor {k}")


def test_autotune_picks_caches_and_keeps_results(torch_cuda, tmp_path):
    m = mxr()
    ins = small_edct()
    I = m.Instrument(ins)
    cache = str(tmp_path / "tune.txt")
    announce("instrument autotune")
    shape = I.autotune(2_000_000, 0.25, cache_path=cache)
    assert shape in SHAPES_EDCT + [(occ, 0, 0, xo) for occ in (0, 4, 6, 8) for xo in (0, 1, 2)]
    assert I.launch_shape == shape
    assert os.path.exists(cache) and open(cache).read().count("\n") == 1
    # a second instrument of the same kind finds the shape in the cache
    J = m.Instrument(ins)
    assert J.autotune(2_000_000, 0.25, cache_path=cache) == shape
    assert open(cache).read().count("\n") == 1
    # the tuned run equals the oracle per bin
    n = 300_001
    t = I.run(n, seed=4)
    torch_cuda.cuda.synchronize()
    compare_bins(t[0], oracle.run(ins, n, seed=4)[0], f"tuned shape {shape}")
    with pytest.raises(m.MxrError):
        I.launch_shape = (5, 1, 0, 0)
    with pytest.raises(m.MxrError):
        I.launch_shape = (0, 2, 0, 0)
    with pytest.raises(m.MxrError):
        I.launch_shape = (0, 1, 65, 0)
    with pytest.raises(m.MxrError):
        I.launch_shape = (0, 1, 0, 3)
    with pytest.raises(m.MxrError):
        I.autotune(1000, 0.0)
