"""Pins of the oracle's beamline optics.

* elliptic-cylinder mirror: in the meridional plane, hit points lie on the
  ellipse |X - F1| + |X - F2| = p + q and reflected rays from F1 pass
  through F2 (focal property); the reflection law holds about the bisector
  normal of the focal radii, and the weight is the linearly interpolated
  reflectivity at the glancing angle;
* two-bounce monochromator: the exit direction equals the entrance
  direction, the exit ray is the entrance ray shifted by 2 g n1, each ray's
  weight is the square of the Darwin curve (evaluated from its definition in
  extended precision), and the band-averaged weight matches the closed-form
  integral of R^2 (32/15 in reduced units);
* powder: the scattering angle is 2 asin(lambda / 2d) for one of the listed
  d-spacings, the reflection index and the azimuth are uniform;
* the full beamline conserves weight in its ledger.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

HC = 12.398419843320026


def gauss_src(sxp=20e-6, hw=0.01, e0=12.4):
    return {"type": "source_gaussian", "pos": (0, 0, 0), "rot": np.eye(3), "sigma_x": 0.0, "sigma_y": 0.0,
            "sigma_xp": sxp, "sigma_yp": sxp, "e0": e0, "rel_halfwidth": hw}


def test_mirror_focusing_and_reflection():
    bl = workloads.beamline()
    mirror = bl["components"][1]
    ins = {"components": [gauss_src(sxp=40e-6), mirror]}
    n = 20000
    o = oracle.trace_rays(ins, np.arange(n), seed=1, n_total=n)
    hit = o["status"] == oracle.STATUS_EXITED
    # the 1 m mirror accepts about +-1.5 mm of a 1.2 mm (rms) beam
    assert 0.7 < hit.mean() < 0.9
    p, q, t0 = mirror["p"], mirror["q"], mirror["theta0"]
    F1 = np.zeros(3)
    F2 = np.array(mirror["pos"]) + q * np.array([0.0, math.sin(2 * t0), math.cos(2 * t0)])
    X, dout = o["r"][hit], o["d"][hit]
    # an elliptic cylinder focuses in the meridional (y, z) plane: the focal
    # properties hold for the projections on that plane
    yz = lambda a: a[..., 1:]
    s = np.linalg.norm(yz(X - F1), axis=1) + np.linalg.norm(yz(X - F2), axis=1)
    assert np.max(np.abs(s - (p + q))) < 1e-12 * (p + q)
    to_f2 = yz(F2 - X)
    dproj = yz(dout)
    miss = np.abs(to_f2[:, 0] * dproj[:, 1] - to_f2[:, 1] * dproj[:, 0]) / np.linalg.norm(dproj, axis=1)
    assert np.max(miss / np.linalg.norm(to_f2, axis=1)) < 1e-12
    u1 = yz(X - F1) / np.linalg.norm(yz(X - F1), axis=1)[:, None]
    u2 = yz(X - F2) / np.linalg.norm(yz(X - F2), axis=1)[:, None]
    nrm = np.zeros_like(X)
    nrm[:, 1:] = u1 + u2
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    din = (X - F1) / np.linalg.norm(X - F1, axis=1)[:, None]
    dn = np.sum(din * nrm, axis=1)
    want = din - 2 * dn[:, None] * nrm
    assert np.max(np.abs(want - dout)) < 1e-12
    theta = np.arcsin(np.abs(dn))
    tab = mirror["reflectivity"]
    grid = np.linspace(0.0, mirror["theta_max"], tab.size)
    # the bisector normal loses ~1e-14 rad to cancellation; the table slope is
    # a few hundred per rad, so agreement is checked at 1e-10
    assert np.max(np.abs(o["w"][hit] - np.interp(theta, grid, tab))) < 1e-10


def darwin_ld(x):
    x = np.abs(np.asarray(x, dtype=np.longdouble))
    r = np.ones_like(x)
    m = x > 1
    r[m] = (x[m] - np.sqrt(x[m] * x[m] - 1)) ** 2
    return r


def test_monochromator():
    bl = workloads.beamline()
    dcm = dict(bl["components"][2])
    dcm["pos"], dcm["rot"] = (0.0, 0.0, 1000.0), np.eye(3)
    ins = {"components": [gauss_src(sxp=0.0), dcm]}
    n = 400000
    o = oracle.trace_rays(ins, np.arange(n), seed=4, n_total=n)
    assert np.all(o["status"] == oracle.STATUS_EXITED)
    assert np.max(np.abs(o["d"] - np.array([0.0, 0.0, 1.0]))) < 1e-15
    tc, g = dcm["theta_c"], dcm["gap"]
    assert np.max(np.abs(o["r"][:, 1] - 2 * g * math.cos(tc))) < 1e-12 * 2 * g
    assert np.all(o["r"][:, 0] == 0.0)
    E = o["E"]
    theta_b = np.arcsin(HC / (2 * dcm["d_spacing"] * E))
    x = (tc - theta_b) / (0.5 * dcm["darwin_width"])
    want = darwin_ld(x) ** 2
    assert np.max(np.abs(o["w"] - want.astype(float)) / np.maximum(want.astype(float), 1e-300)) < 1e-9
    # band average against the closed form integral of R^2 (= 32/15 in x)
    hw = 0.01
    mean_closed = (32.0 / 15.0) * (0.5 * dcm["darwin_width"]) / (2 * hw * math.tan(tc))
    w = o["w"]
    assert abs(w.mean() - mean_closed) < 4 * w.std() / math.sqrt(n) + 2e-3 * mean_closed
    # on the plateau centre the weight is exactly one
    assert np.all(o["w"][np.abs(x) <= 0.999] == 1.0)


def test_powder_rings():
    dsp = workloads.make_d_spacings(1)
    powder = {"type": "powder", "pos": (0, 0, 100.0), "rot": np.eye(3), "w": 1.0, "h": 1.0, "d_spacings": dsp}
    ins = {"components": [gauss_src(sxp=2e-3), powder]}
    n = 100000
    o = oracle.trace_rays(ins, np.arange(n), seed=5, n_total=n)
    hit = o["status"] == oracle.STATUS_EXITED
    assert 0.5 < hit.mean() < 1.0
    X, dout, E = o["r"][hit], o["d"][hit], o["E"][hit]
    assert np.all(X[:, 2] == 100.0)
    din = X / np.linalg.norm(X, axis=1)[:, None]
    ang = np.arctan2(np.linalg.norm(np.cross(din, dout), axis=1), np.sum(din * dout, axis=1))
    two_theta = 2 * np.arcsin(HC / E[:, None] / (2 * dsp[None, :]))
    err = np.abs(two_theta - ang[:, None])
    j = err.argmin(1)
    assert np.max(err[np.arange(len(j)), j]) < 1e-12
    assert stats.chisquare(np.bincount(j, minlength=dsp.size)).pvalue > 1e-4
    e1 = np.cross(din, np.array([0.0, 1.0, 0.0]))
    e1 /= np.linalg.norm(e1, axis=1)[:, None]
    e2 = np.cross(din, e1)
    eta = np.arctan2(np.sum(dout * e2, 1), np.sum(dout * e1, 1))
    assert stats.kstest((eta + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-4


def test_beamline_ledger_and_survival():
    ins = workloads.beamline()
    n = 300000
    outs, led = oracle.run(ins, n, seed=1, ledger=True)
    K = len(ins["components"])
    emitted = led[0]
    lost = sum(led[4 * k + 1] + led[4 * k + 2] for k in range(K))
    assert abs(emitted - (lost + led[4 * K])) <= 1e-12 * emitted
    # weight after the monochromator ~ mirror reflectivity x Darwin band-pass
    after_dcm = led[4 * 3 + 0] / n
    assert 0.003 < after_dcm < 0.02
    assert outs[0]["count"].sum() > 0
