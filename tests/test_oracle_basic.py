"""Pins of the oracle on the basic absorber instrument (square emitter, 1 mm
slit at 1 m, homogeneous 10 mm box at 1.5 m, monitor at 2 m).

* slit transmission = emitter-averaged solid angle of the slit / cone solid
  angle, by 2-D quadrature of the exact rectangle solid angle;
* per-ray Beer-Lambert: every detected ray carries exp(-mu(E) * 10 / dz / 10)
  since it crosses the box face to face;
* ensemble transmitted weight from the 1-D integral over the flat spectrum;
* weight ledger: emitted = absorbed + attenuated + leaving;
* mirror symmetry of the image;
* chunked runs and thread count do not change the histograms.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import workloads


def rect_solid_angle(x0, x1, y0, y1, dist):
    F = lambda x, y: math.atan(x * y / (dist * math.sqrt(dist * dist + x * x + y * y)))
    return F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)


@pytest.fixture(scope="module")
def p_slit():
    def om(y, x):
        return rect_solid_angle(-0.5 - x, 0.5 - x, -0.5 - y, 0.5 - y, 1000.0)
    mean_om, _ = integrate.dblquad(om, -0.5, 0.5, -0.5, 0.5, epsabs=0, epsrel=1e-12)
    cone = 4 * math.pi * math.sin(5e-3 / 2) ** 2
    return mean_om / cone


def mu_box(E):
    return 2e4 / E ** 3 + 0.2


def test_slit_transmission_closed_form(p_slit):
    assert abs(p_slit - 1.273241560700e-2) < 1e-9
    n = 10**6
    out = oracle.run(workloads.basic_absorber(), n, seed=1)[0]
    k = int(out["count"].sum())
    assert abs(k - n * p_slit) < 4 * math.sqrt(n * p_slit * (1 - p_slit))


def test_transmitted_weight_closed_form(p_slit):
    T1, _ = integrate.quad(lambda E: math.exp(-mu_box(E)) / 60.0, 20, 80, epsrel=1e-12)
    T2, _ = integrate.quad(lambda E: math.exp(-2 * mu_box(E)) / 60.0, 20, 80, epsrel=1e-12)
    assert abs(T1 - 0.609146911161) < 1e-9
    n = 10**6
    out = oracle.run(workloads.basic_absorber(), n, seed=1)[0]
    mean = p_slit * T1
    var = p_slit * T2 - mean ** 2
    assert abs(out["sum_w"].sum() - n * mean) < 4 * math.sqrt(n * var)
    assert abs(out["sum_w2"].sum() - n * p_slit * T2) < 4 * math.sqrt(n * p_slit * T2)


def test_per_ray_beer_lambert():
    ins = workloads.basic_absorber()
    n = 200000
    o = oracle.trace_rays(ins, np.arange(n), seed=1, n_total=n)
    hit = o["bin"] >= 0
    assert hit.sum() > 2000
    E, dz = o["E"][hit], o["d"][hit, 2]
    want = np.exp(-mu_box(E) * (10.0 / dz) / 10.0)
    assert np.max(np.abs(o["w"][hit] - want) / want) < 1e-13
    # rays stopped by the slit are absorbed there, all others reach the end
    absorbed = o["status"] == oracle.STATUS_ABSORBED
    assert np.all(o["dead_at"][absorbed] == 1)
    assert np.all(o["status"][~absorbed] == oracle.STATUS_EXITED)
    # detected rays sit on the monitor plane, inside it
    assert np.all(o["r"][hit, 2] == 2000.0)
    ix = np.floor((o["r"][hit, 0] + 50.0) * (128 / 100.0)).astype(int)
    iy = np.floor((o["r"][hit, 1] + 50.0) * (128 / 100.0)).astype(int)
    assert np.array_equal(o["bin"][hit], iy * 128 + ix)


def test_ledger_conservation():
    ins = workloads.basic_absorber()
    _, led = oracle.run(ins, 200000, seed=3, ledger=True)
    K = len(ins["components"])
    emitted = led[0]
    absorbed = sum(led[4 * k + 1] for k in range(K))
    attenuated = sum(led[4 * k + 2] for k in range(K))
    leaving = led[4 * K]
    assert emitted == 200000.0
    assert abs(emitted - (absorbed + attenuated + leaving)) <= 1e-12 * emitted
    assert led[4 * 3 + 3] == pytest.approx(leaving, rel=1e-12)  # all leaving rays are tallied


def test_image_mirror_symmetry():
    out = oracle.run(workloads.basic_absorber(), 10**6, seed=2)[0]
    img = out["count"].reshape(128, 128).astype(float)
    a, b = img, img[:, ::-1]
    m = (a + b) > 0
    chi2 = np.sum((a[m] - b[m]) ** 2 / (a[m] + b[m])) / 2
    dof = m.sum() / 2
    assert stats.chi2.sf(chi2, dof) > 1e-4


def test_chunked_and_threaded_runs_equal_one_run():
    ins = workloads.basic_absorber()
    n = 300000
    one = oracle.run(ins, n, seed=5, threads=1)[0]
    parts = [oracle.run(ins, n // 3, seed=5, first=i * (n // 3), n_total=n, threads=3)[0] for i in range(3)]
    assert np.array_equal(one["count"], sum(p["count"] for p in parts))
    tot = sum(p["sum_w"] for p in parts)
    nz = one["sum_w"] > 0
    assert np.max(np.abs(tot[nz] - one["sum_w"][nz]) / one["sum_w"][nz]) < 1e-12
    assert np.all(tot[~nz] == 0)
