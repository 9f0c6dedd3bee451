"""Pins of the oracle's sources against closed forms.

* square emitter + cone: position moments; 1 - cos(theta) uniform on
  [0, 1 - cos(alpha)] (uniform in solid angle); azimuth uniform; flat energy.
* cone-beam source: the same solid-angle law at a wide cone, with and
  without stratification; E[w0] = 1; the energy marginal of the weights equals
  the integral of the spectrum over each bin (Kramers continuum in closed
  form, lines through erf); the fraction of rays inside a rectangle's solid
  angle equals Omega_rect / Omega_cone.
* Gaussian source: moments of position, angle and energy.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.special import ndtr

import oracle
import workloads


def only(*comps):
    return {"components": list(comps)}


def trace(instr, n, seed=1, n_total=None):
    return oracle.trace_rays(instr, np.arange(n), seed=seed, n_total=n_total or n)


def one_minus_cos(d):
    # 1 - cos(theta) = sin^2(theta) / (1 + cos(theta)), no cancellation
    return (d[:, 0] ** 2 + d[:, 1] ** 2) / (1.0 + d[:, 2])


def test_rect_cone_source():
    src = workloads.basic_absorber()["components"][0]
    n = 40000
    o = trace(only(src), n)
    assert np.all(o["status"] == oracle.STATUS_EXITED)
    x, y = o["r"][:, 0], o["r"][:, 1]
    assert np.all(np.abs(x) <= 0.5) and np.all(np.abs(y) <= 0.5)
    assert np.all(o["r"][:, 2] == 0.0)
    for v in (x, y):
        assert abs(v.mean()) < 4 * math.sqrt(1 / 12 / n)
        assert abs(v.var() - 1 / 12) < 4 * math.sqrt(1 / 180 / n)
    d = o["d"]
    assert np.max(np.abs(np.linalg.norm(d, axis=1) - 1)) < 4e-16
    alpha = src["half_angle"]
    u = one_minus_cos(d) / (2 * math.sin(alpha / 2) ** 2)
    assert u.max() <= 1.0 + 1e-12
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    phi = np.arctan2(d[:, 1], d[:, 0])
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-4
    assert stats.kstest((o["E"] - 20) / 60, "uniform").pvalue > 1e-4
    assert np.all(o["w"] == 1.0)


def edct_source(strata):
    vol = np.zeros((2, 2, 2), np.uint8)
    mu = np.zeros((8, 256))
    return workloads.edct_projection(vol, mu, strata=strata)["components"][0]


@pytest.mark.parametrize("strata", [1, 16])
def test_cone_beam_solid_angle_and_weight(strata):
    src = edct_source(strata)
    n = 40000
    o = trace(only(src), n)
    alpha = src["half_angle"]
    u = one_minus_cos(o["d"]) / (2 * math.sin(alpha / 2) ** 2)
    assert u.max() <= 1.0 + 1e-12
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    phi = np.arctan2(o["d"][:, 1], o["d"][:, 0])
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-4
    w = o["w"]
    assert abs(w.mean() - 1.0) < 4 * w.std() / math.sqrt(n)


def spectrum_bin_integral(src, e1, e2):
    E0, emin, emax = src["e0"], src["emin"], src["emax"]
    K = E0 * math.log(emax / emin) - (emax - emin)
    cont = src["f_cont"] * (E0 * np.log(e2 / e1) - (e2 - e1)) / K
    s = src["line_sigma"]
    l1 = src["f_line1"] * (ndtr((e2 - src["e_line1"]) / s) - ndtr((e1 - src["e_line1"]) / s))
    l2 = src["f_line2"] * (ndtr((e2 - src["e_line2"]) / s) - ndtr((e1 - src["e_line2"]) / s))
    return cont + l1 + l2


def test_cone_beam_energy_marginal():
    src = edct_source(1)
    edges = np.linspace(20.0, 150.0, 27)
    want = spectrum_bin_integral(src, edges[:-1], edges[1:])
    assert abs(want.sum() - 1.0) < 1e-12
    n = 200000
    o = trace(only(src), n)
    idx = np.clip(np.searchsorted(edges, o["E"], side="right") - 1, 0, 25)
    sw = np.bincount(idx, weights=o["w"], minlength=26) / n
    sw2 = np.bincount(idx, weights=o["w"] ** 2, minlength=26) / n
    var = (sw2 - sw ** 2) / n
    chi2 = np.sum((sw - want) ** 2 / var)
    assert stats.chi2.sf(chi2, 26) > 1e-4
    # the spectrum itself, pointwise, at a few energies
    for E in (20.0, 59.3, 67.0, 100.0, 149.9):
        K = 150 * math.log(7.5) - 130
        g = lambda m: math.exp(-0.5 * ((E - m) / 0.3) ** 2) / (0.3 * math.sqrt(2 * math.pi))
        ref = 0.8 * (150 - E) / E / K + 0.1 * g(59.3) + 0.1 * g(67.2)
        assert abs(oracle.spectrum(src, E) - ref) <= 1e-14 * ref


def rect_solid_angle(x0, x1, y0, y1, dist):
    F = lambda x, y: np.arctan(x * y / (dist * np.sqrt(dist * dist + x * x + y * y)))
    return F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)


def test_cone_beam_detector_fraction():
    """Only rays inside the detector's solid angle land on it."""
    vol = np.zeros((2, 2, 2), np.uint8)
    ins = workloads.edct_projection(vol, np.zeros((8, 256)), strata=64)
    ins = {"components": [ins["components"][0], ins["components"][2]]}
    n = 100000
    o = trace(ins, n)
    det = ins["components"][1]
    om = rect_solid_angle(det["xmin"], det["xmax"], det["ymin"], det["ymax"], 1200.0)
    cone = 4 * math.pi * math.sin(ins["components"][0]["half_angle"] / 2) ** 2
    p = om / cone
    assert abs(p - 0.30188) < 1e-4
    frac = np.mean(o["bin"] >= 0)
    assert abs(frac - p) < 4 * math.sqrt(p * (1 - p) / n)


def test_gaussian_source():
    src = workloads.beamline()["components"][0]
    n = 40000
    o = trace(only(src), n)
    x, y = o["r"][:, 0], o["r"][:, 1]
    for v in (x, y):
        assert stats.kstest(v / 0.05, "norm").pvalue > 1e-4
    xp = np.arctan(o["d"][:, 0] / o["d"][:, 2])
    yp = np.arctan(o["d"][:, 1] / o["d"][:, 2])
    for v in (xp, yp):
        assert stats.kstest(v / 20e-6, "norm").pvalue > 1e-4
    assert np.corrcoef(x, xp)[0, 1] ** 2 < 16 / n
    assert np.max(np.abs(np.linalg.norm(o["d"], axis=1) - 1)) < 4e-16
    assert stats.kstest((o["E"] / 12.4 - 0.99) / 0.02, "uniform").pvalue > 1e-4
