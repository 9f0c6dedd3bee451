"""The proposal-driven source and hit collection of the HIP library against
the oracle, through the C ABI, on the same Philox streams and the same
FP64 mixture table: per ray within 1e-12 relative (status, absorbing
component and bin identical), per bin within 1e-9 (counts identical), and
the collected rows equal the oracle's detected rays.
"""
import numpy as np
import pytest

import oracle
import workloads
from oracle import proposal as P

from test_gpu_parity import compare_bins, compare_rays, cpu, announce

pytestmark = pytest.mark.gpu


def mxr():
    import paper_2410_08747_amd as m
    return m


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def small_instr(angle=0.4):
    vol = workloads.make_phantom(64, seed=1)
    return workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=angle, strata=64, nx=32, ny=16, ne=32)


def mixtures(src):
    lo, hi = P.box_of(src)
    rng = np.random.default_rng(8)
    out = {}
    # broad random mixture
    pi = rng.dirichlet(np.ones(8))
    mu = lo + (hi - lo) * rng.uniform(0.1, 0.9, size=(8, 3))
    sg = 0.5 * (hi - lo) * rng.uniform(0.15, 0.8, size=(8, 3))
    out["broad"] = np.concatenate([pi[:, None], mu, sg], 1).reshape(56)
    # aimed at the detector, some narrow components, one empty component
    g = np.zeros((8, 7))
    for k in range(8):
        g[k] = [1 / 8, -0.015 + 0.03 * (k + 0.5) / 8, 0.002 * (k - 4), 20 + 130 * (k + 0.5) / 8,
                0.004 + 0.001 * k, 0.006, 5.0 + 3 * k]
    g[3, 0] = 0.0
    out["aimed"] = g.reshape(56)
    # components far outside the box in one coordinate (deep tails)
    g2 = np.array(out["broad"]).reshape(8, 7).copy()
    g2[1, 1] = hi[0] + 6 * g2[1, 4]
    g2[2, 3] = lo[2] - 9 * g2[2, 6]
    g2[:, 0] = 0.0
    g2[1, 0] = g2[2, 0] = 1.0  # all the mass in the two tail components
    out["tails"] = g2.reshape(56)
    return out


def sample_points(d, E):
    """y = (dx/dz, dy/dz, E) of final rays (source at the origin, identity
    frame; the projection chain keeps direction and energy)."""
    return np.stack([d[:, 0] / d[:, 2], d[:, 1] / d[:, 2], E], 1)


def compare_proposal_rays(ins, gmm, alpha, n_total, ids, g, o, seed, job, label, purpose=0):
    """Per-ray parity of a proposal run.  Status, component, bin, position,
    direction and energy against the oracle's own trace (1e-12).  The final
    weight against the oracle continuing the GPU's own sample point: both
    sides invert a truncated normal (the ROCm device erfcinv, Wichura's
    AS 241), which agree to a few ulp, and the voxel path amplifies a
    direction change of 1e-15 into optical-depth changes of up to ~1e-13
    (mu jumps at material boundaries), so the weight is compared where both
    sides start from the same point: the oracle's weight function at the
    GPU's (u, v, E) times the oracle's own stratum factor, then the oracle's
    transport from there."""
    w_any = np.full(ids.size, np.inf)
    compare_rays(g, o, label, w_rel=w_any)
    src = ins["components"][0]
    s0 = oracle.trace_rays({"components": [src]}, ids, seed=seed, n_total=n_total, purpose=purpose, job=job,
                           gmm=gmm, alpha=alpha)
    gd = np.stack([cpu(g["dx"]), cpu(g["dy"]), cpu(g["dz"])], 1)
    gE, gw = cpu(g["E"]), cpu(g["w"])
    live = s0["w"] > 0
    assert np.all(gw[~live] == 0.0), f"{label}: rays outside the cone must carry weight 0"
    yg = sample_points(gd[live], gE[live])
    yo = sample_points(s0["d"][live], s0["E"][live])
    W_g = oracle.proposal_weight(src, gmm, alpha, n_total, yg)
    W_o = oracle.proposal_weight(src, gmm, alpha, n_total, yo)
    w0 = W_g * (s0["w"][live] / W_o)
    c = oracle.trace_after_source(ins, ids[live], seed, n_total, s0["r"][live], gd[live], gE[live], w0,
                                  purpose=purpose, job=job)
    err = np.abs(gw[live] - c["w"]) / np.maximum(np.abs(c["w"]), 1e-300)
    k = int(np.argmax(err))
    assert err.max() <= 1e-12, f"{label}: w ray {np.flatnonzero(live)[k]}: gpu {gw[live][k]!r} oracle {c['w'][k]!r}"
    assert np.array_equal(c["bin"], cpu(g["bin"])[live])


@pytest.mark.parametrize("name", ["broad", "aimed", "tails"])
@pytest.mark.parametrize("alpha", [0.1, 1.0, 0.0])
def test_proposal_per_ray(torch_cuda, name, alpha):
    ins = small_instr()
    gmm = mixtures(ins["components"][0])[name]
    announce("proposal per ray", name, "alpha", alpha)
    I = mxr().Instrument(ins)
    I.set_proposal(torch_cuda.tensor(gmm, device="cuda"), alpha)
    n = 50003
    ids = np.arange(n, dtype=np.uint64)
    g = I.trace_rays(ids, seed=5, n_total=n, purpose=0, job=3)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=5, n_total=n, job=3, gmm=gmm, alpha=alpha)
    compare_proposal_rays(ins, gmm, alpha, n, ids, g, o, 5, 3, f"proposal {name} alpha {alpha}")


def test_proposal_per_bin_and_ledger(torch_cuda):
    ins = small_instr(1.2)
    gmm = mixtures(ins["components"][0])["aimed"]
    announce("proposal per bin")
    I = mxr().Instrument(ins)
    I.set_proposal(torch_cuda.tensor(gmm, device="cuda"), 0.1)
    n = 300001
    led = I.new_ledger()
    t = I.run(n, seed=2, ledger=led)
    torch_cuda.cuda.synchronize()
    o, oled = oracle.run(ins, n, seed=2, ledger=True, gmm=gmm, alpha=0.1)
    compare_bins(t[0], o[0], "proposal per bin")
    gl = cpu(led)
    nz = oled != 0
    assert np.array_equal(gl == 0, oled == 0)
    assert np.max(np.abs(gl[nz] - oled[nz]) / np.abs(oled[nz])) <= 1e-9
    # switching the proposal off restores the plain (stratified) source
    I.set_proposal(None)
    t2 = I.run(n, seed=2)
    torch_cuda.cuda.synchronize()
    compare_bins(t2[0], oracle.run(ins, n, seed=2)[0], "proposal cleared")


def test_proposal_generic_chain(torch_cuda):
    """A chain without a compiled recipe (slit before the phantom) takes the
    proposal through the dynamic dispatch."""
    ins = small_instr(0.9)
    slit = workloads._c("slit", pos=(0.0, 0.0, 500.0), w=20.0, h=8.0)
    ins = {"components": [ins["components"][0], slit, *ins["components"][1:]]}
    gmm = mixtures(ins["components"][0])["broad"]
    announce("proposal generic chain")
    I = mxr().Instrument(ins)
    I.set_proposal(torch_cuda.tensor(gmm, device="cuda"), 0.3)
    n = 40000
    ids = np.arange(n, dtype=np.uint64)
    g = I.trace_rays(ids, seed=7, n_total=n)
    torch_cuda.cuda.synchronize()
    o = oracle.trace_rays(ins, ids, seed=7, n_total=n, gmm=gmm, alpha=0.3)
    compare_proposal_rays(ins, gmm, 0.3, n, ids, g, o, 7, 0, "generic proposal")


def detected_rows(o, src_rot=None):
    det = o["bin"] >= 0
    d = o["d"][det]
    y = np.stack([d[:, 0] / d[:, 2], d[:, 1] / d[:, 2], o["E"][det]], 1)
    return o["bin"][det], o["w"][det], y


@pytest.mark.parametrize("with_proposal", [False, True])
def test_collect_rows_equal_detected_rays(torch_cuda, with_proposal):
    ins = small_instr(0.4)
    announce("collect", "proposal", with_proposal)
    I = mxr().Instrument(ins)
    gmm = mixtures(ins["components"][0])["aimed"]
    if with_proposal:
        I.set_proposal(torch_cuda.tensor(gmm, device="cuda"), 0.1)
    n = 100000
    hits = I.new_hits(n)
    ctx = [0.0, 0.0, 0.0, 0.92, 0.39, 0.67]
    t = I.collect(n, seed=3, context=ctx, hits=hits)
    torch_cuda.cuda.synchronize()
    cnt = int(hits["count"].item())
    o = oracle.trace_rays(ins, np.arange(n), seed=3, n_total=n, gmm=gmm if with_proposal else None, alpha=0.1)
    ob, ow, oy = detected_rows(o)
    assert cnt == ob.size
    gb, gw, gy = cpu(hits["bin"])[:cnt], cpu(hits["w"])[:cnt], cpu(hits["y"])[:cnt]
    assert np.allclose(cpu(hits["ctx"])[:cnt], np.float32(ctx)[None, :], rtol=0, atol=0)
    ko = np.lexsort((ow, ob))
    kg = np.lexsort((gw, gb))
    assert np.array_equal(gb[kg], ob[ko])
    assert np.max(np.abs(gw[kg] - ow[ko]) / np.maximum(np.abs(ow[ko]), 1e-300)) <= 1e-12
    assert np.max(np.abs(gy[kg] - oy[ko]) / np.maximum(np.abs(oy[ko]), 1.0)) <= 1e-12
    # the run's histograms are the plain run's
    compare_bins(t[0], oracle.run(ins, n, seed=3, gmm=gmm if with_proposal else None, alpha=0.1)[0], "collect tallies")
    # capacity below the hit count: count reports the total, rows are truncated
    small = I.new_hits(100)
    I.collect(n, seed=3, context=ctx, hits=small)
    torch_cuda.cuda.synchronize()
    assert int(small["count"].item()) == cnt


def test_proposal_errors(torch_cuda):
    m = mxr()
    announce("proposal errors")
    ins = small_instr()
    gmm = mixtures(ins["components"][0])["broad"].reshape(8, 7).copy()
    I = m.Instrument(ins)
    bad = gmm.copy()
    bad[2, 5] = 0.0
    with pytest.raises(m.MxrError):
        I.set_proposal(torch_cuda.tensor(bad.reshape(56), device="cuda"), 0.1)
    bad = gmm.copy()
    bad[0, 0] = -1.0
    with pytest.raises(m.MxrError):
        I.set_proposal(torch_cuda.tensor(bad.reshape(56), device="cuda"), 0.1)
    with pytest.raises(m.MxrError):
        I.set_proposal(torch_cuda.tensor(gmm.reshape(56), device="cuda"), 1.5)
    B = m.Instrument(workloads.basic_absorber())
    with pytest.raises(m.MxrError):
        B.set_proposal(torch_cuda.tensor(gmm.reshape(56), device="cuda"), 0.1)
    hits = B.new_hits(10)
    with pytest.raises(m.MxrError):
        B.collect(10, seed=1, context=[0] * 6, hits=hits)  # rectangular source: no collection
