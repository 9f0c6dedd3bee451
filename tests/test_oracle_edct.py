"""Pins of the oracle on the energy-dispersive CT projection chain.

* flat field (empty phantom): per-bin mean weight = Omega_pixel / Omega_cone
  times the spectrum integrated over the energy bin (chi-square over bins);
* every ray's weight equals w0(E) exp(-tau) with tau from a brute-force
  per-voxel intersection of the ray with the turned phantom, the frame
  transform done independently in numpy;
* stratification changes no expectation: stratified and plain runs agree
  within their errors; chunked runs equal one run;
* weight ledger conservation.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import ndtr

import oracle
import workloads
from test_oracle_siddon import brute_force, ebin


def spectrum(src, E):
    K = src["e0"] * math.log(src["emax"] / src["emin"]) - (src["emax"] - src["emin"])
    g = lambda m: np.exp(-0.5 * ((E - m) / src["line_sigma"]) ** 2) / (src["line_sigma"] * math.sqrt(2 * math.pi))
    return src["f_cont"] * (src["e0"] - E) / E / K + src["f_line1"] * g(src["e_line1"]) + src["f_line2"] * g(src["e_line2"])


def spectrum_bin_integral(src, e1, e2):
    K = src["e0"] * math.log(src["emax"] / src["emin"]) - (src["emax"] - src["emin"])
    cont = src["f_cont"] * (src["e0"] * np.log(e2 / e1) - (e2 - e1)) / K
    s = src["line_sigma"]
    l1 = src["f_line1"] * (ndtr((e2 - src["e_line1"]) / s) - ndtr((e1 - src["e_line1"]) / s))
    l2 = src["f_line2"] * (ndtr((e2 - src["e_line2"]) / s) - ndtr((e1 - src["e_line2"]) / s))
    return cont + l1 + l2


def pixel_solid_angles(det, dist):
    xe = np.linspace(det["xmin"], det["xmax"], det["nx"] + 1)
    ye = np.linspace(det["ymin"], det["ymax"], det["ny"] + 1)
    X, Y = np.meshgrid(xe, ye)  # (ny+1, nx+1)
    F = np.arctan(X * Y / (dist * np.sqrt(dist * dist + X * X + Y * Y)))
    return F[1:, 1:] - F[:-1, 1:] - F[1:, :-1] + F[:-1, :-1]  # (ny, nx)


@pytest.mark.parametrize("strata", [1, 32])
def test_flat_field(strata):
    vol = np.zeros((8, 8, 8), np.uint8)
    mu = np.zeros((8, 256))
    ins = workloads.edct_projection(vol, mu, strata=strata, nx=16, ny=4, ne=13)
    src, det = ins["components"][0], ins["components"][2]
    n = 400000
    out = oracle.run(ins, n, seed=1)[0]
    om = pixel_solid_angles(det, 1200.0)
    cone = 4 * math.pi * math.sin(src["half_angle"] / 2) ** 2
    edges = np.linspace(20.0, 150.0, 14)
    spec = spectrum_bin_integral(src, edges[:-1], edges[1:])
    want = (om[:, :, None] / cone * spec[None, None, :]).reshape(-1)
    mean = out["sum_w"] / n
    var = (out["sum_w2"] / n - mean ** 2) / n
    chi2 = np.sum((mean - want) ** 2 / var)
    assert stats.chi2.sf(chi2, want.size) > 1e-4


def test_per_ray_attenuation_brute_force():
    rng = np.random.default_rng(9)
    n = 16
    vol = rng.integers(0, 8, size=(n, n, n)).astype(np.uint8)
    mu = rng.uniform(0.05, 2.0, size=(8, 256))
    for angle in (0.0, 0.3, math.pi / 4, 2.0):
        ins = workloads.edct_projection(vol, mu, angle=angle, strata=1)
        # a 16 mm phantom only meets the central rays: shrink the cone
        ins["components"][0]["half_angle"] = 0.012
        src, ph = ins["components"][0], ins["components"][1]
        o = oracle.trace_rays(ins, np.arange(3000), seed=2, n_total=3000)
        R, pos = ph["rot"], np.array(ph["pos"])
        hit_any = 0
        for i in range(3000):
            d = o["d"][i]
            q = R @ (np.zeros(3) - pos)
            dl = R @ d
            tau, _, ln = brute_force(vol, mu[:, ebin(o["E"][i])], 1.0, q, dl)
            hit_any += ln.sum() > 0
            w0 = 130.0 * spectrum(src, o["E"][i])
            want = w0 * math.exp(-tau)
            assert abs(o["w"][i] - want) <= 1e-12 * max(want, 1e-300) + 1e-300
        assert hit_any > 1000


def test_stratified_matches_plain():
    rng = np.random.default_rng(1)
    vol = workloads.make_phantom(64, seed=1)
    mu = workloads.make_mu_tables(1)
    a = workloads.edct_projection(vol, mu, strata=1, nx=16, ny=4, ne=4)
    b = workloads.edct_projection(vol, mu, strata=64, nx=16, ny=4, ne=4)
    n = 200000
    ra = oracle.run(a, n, seed=11)[0]
    rb = oracle.run(b, n, seed=12)[0]
    m = ra["count"] > 100
    va = ra["sum_w2"] / n - (ra["sum_w"] / n) ** 2
    vb = rb["sum_w2"] / n - (rb["sum_w"] / n) ** 2
    z = (ra["sum_w"] - rb["sum_w"])[m] / n / np.sqrt((va + vb)[m] / n)
    assert stats.chi2.sf(np.sum(z ** 2), m.sum()) > 1e-4


def test_chunked_run_and_ledger():
    vol = workloads.make_phantom(64, seed=2)
    mu = workloads.make_mu_tables(1)
    ins = workloads.edct_projection(vol, mu, angle=0.5, strata=16, nx=32, ny=8, ne=16)
    n = 60000
    one, led = oracle.run(ins, n, seed=3, threads=2, ledger=True)
    one = one[0]
    parts = [oracle.run(ins, n // 4, seed=3, first=i * (n // 4), n_total=n, threads=1)[0] for i in range(4)]
    assert np.array_equal(one["count"], sum(p["count"] for p in parts))
    tot = sum(p["sum_w"] for p in parts)
    nz = one["sum_w"] > 0
    assert np.max(np.abs(tot[nz] - one["sum_w"][nz]) / one["sum_w"][nz]) < 1e-12
    K = 3
    emitted = led[0]
    lost = sum(led[4 * k + 1] + led[4 * k + 2] for k in range(K))
    assert abs(emitted - (lost + led[4 * K])) <= 1e-12 * emitted


def test_metrics_flat_field_matches_closed_form():
    """The metric module's flat field equals this file's closed form (and
    so the oracle's flat-field image, pinned above)."""
    from paper_2410_08747_amd import metrics
    vol = np.zeros((8, 8, 8), np.uint8)
    ins = workloads.edct_projection(vol, np.zeros((8, 256)), nx=16, ny=4, ne=13)
    src, det = ins["components"][0], ins["components"][2]
    om = pixel_solid_angles(det, 1200.0)
    cone = 4 * math.pi * math.sin(src["half_angle"] / 2) ** 2
    edges = np.linspace(20.0, 150.0, 14)
    want = (om[:, :, None] / cone * spectrum_bin_integral(src, edges[:-1], edges[1:])[None, None, :]).reshape(-1)
    got = metrics.flat_field(ins)
    assert np.allclose(got, want, rtol=1e-12, atol=0)
    # a full detector sums to the fraction of the cone it covers times the band's mass
    assert abs(got.sum() - om.sum() / cone * spectrum_bin_integral(src, 20.0, 150.0)) < 1e-12


def test_early_out_aperture_keeps_the_image():
    """An aperture in front of the phantom that passes the detector
    rectangle (scaled to its distance) removes only rays that miss the
    detector, since the phantom only absorbs: the image keeps its counts,
    and its sums change only by the rounding of the extra propagation."""
    vol = workloads.make_phantom(64, seed=1)
    mu = workloads.make_mu_tables(1)
    n = 200000
    plain = oracle.run(workloads.edct_projection(vol, mu, angle=0.4, strata=64), n, seed=3)[0]
    aimed_ins = workloads.edct_projection(vol, mu, angle=0.4, strata=64, early_out=True)
    assert [c["type"] for c in aimed_ins["components"]][1] == "slit"
    aimed = oracle.run(aimed_ins, n, seed=3)[0]
    assert plain["count"].sum() > 0.2 * n
    assert np.array_equal(plain["count"], aimed["count"])
    for key in ("sum_w", "sum_w2"):
        nz = plain[key] != 0
        assert np.array_equal(nz, aimed[key] != 0)
        assert np.max(np.abs(aimed[key][nz] - plain[key][nz]) / plain[key][nz]) <= 1e-9
    # a narrower aperture does cut detected rays
    narrow = workloads.edct_projection(vol, mu, angle=0.4, strata=64, early_out=True)
    narrow["components"][1]["w"] *= 0.5
    assert oracle.run(narrow, n, seed=3)[0]["count"].sum() < 0.75 * plain["count"].sum()
