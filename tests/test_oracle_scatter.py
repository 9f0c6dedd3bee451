"""Pins of the oracle's scattering phantom (forced interactions by scatter
order; section 3.3: the voxel sample models absorption and scattering).

* Klein-Nishina: f(k) (total cross section over 2 pi r_e^2) against a
  quadrature of the differential cross section, and its Thomson limit 4/3;
* the forced interaction depth in a homogeneous cube follows the truncated
  exponential on the chord (KS), the chord from an independent ray/box
  intersection; across three layers of different attenuation and albedo,
  the point follows the layered depth's distribution function (KS) and every
  ray's weight equals the product of slab-geometry factors;
* the weight of a single scatter, divided by the factors the geometry fixes
  (1 - e^-mu L, the albedo, e^-mu L_exit with L_exit from the independent
  intersection), is the angular factor; weighted by it, the scattering
  angles of isotropic draws follow Klein-Nishina (Compton-only medium) and
  Thomson (Rayleigh-only medium) -- binned, z-tests against quadratures;
* Compton energies equal E / (1 + k (1 - cos theta)) ray by ray, Rayleigh
  keeps E;
* the aimed and the isotropic estimators of the single- and double-scatter
  images agree (two different estimators of one quantity);
* a medium without scattering channels gives no weight.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import workloads

ME = 510.99895


def kn_pdf_unnorm(mu, k):
    rho = 1.0 / (1.0 + k * (1.0 - mu))
    return 0.5 * rho * rho * (rho + 1.0 / rho - (1.0 - mu * mu))


@pytest.mark.parametrize("k", [1e-3, 0.04, 0.29, 1.0, 5.0])
def test_klein_nishina_total(k):
    val, _ = integrate.quad(lambda m: kn_pdf_unnorm(m, k), -1.0, 1.0, epsabs=0, epsrel=1e-13)
    assert oracle.kn_f(k) == pytest.approx(val, rel=1e-9 if k < 0.01 else 1e-12)


def test_thomson_limit():
    assert oracle.kn_f(1e-4) == pytest.approx(4.0 / 3.0, rel=1e-3)


N = 12  # homogeneous cube of N^3 voxels of 1 mm


def cube_instrument(mu_t, mu_r, mu_c, order=1, aim=False, half_angle=0.004, detector=False):
    vol = np.ones((N, N, N), np.uint8)
    tab = np.zeros((3, 2, 4))
    tab[0, 1], tab[1, 1], tab[2, 1] = mu_t, mu_r, mu_c
    tab[0, 0] = 1.0  # material 0 unused
    src = {"type": "source_cone_beam", "pos": (0.0, 0.0, 0.0), "rot": np.eye(3), "half_angle": half_angle,
           "emin": 20.0, "emax": 150.0, "e0": 150.0, "f_cont": 0.8, "e_line1": 59.3, "f_line1": 0.1,
           "e_line2": 67.2, "f_line2": 0.1, "line_sigma": 0.3, "strata": 1}
    ph = {"type": "phantom", "pos": (0.0, 0.0, 100.0), "rot": np.eye(3), "voxel": 1.0, "volume": vol,
          "mu_table": tab, "table_emin": 20.0, "table_emax": 150.0, "scatter_order": order}
    comps = [src, ph]
    if aim or detector:
        h = 40.0
        if aim:
            ph["scatter_target"] = ((0.0, 0.0, 200.0), (h, 0.0, 0.0), (0.0, h, 0.0))
        comps.append({"type": "detector", "pos": (0.0, 0.0, 200.0), "rot": np.eye(3), "xmin": -h, "xmax": h,
                      "ymin": -h, "ymax": h, "emin": 0.0, "emax": 200.0, "nx": 8, "ny": 8, "ne": 1})
    return {"components": comps}


def box_interval(q, d, h):
    """[a_in, a_out] of the ray q + a d in the cube |x_i| < h (lengths in mm)."""
    lo, hi = 0.0, np.inf
    for i in range(3):
        if d[i] == 0:
            continue
        a0, a1 = (-h - q[i]) / d[i], (h - q[i]) / d[i]
        lo, hi = max(lo, min(a0, a1)), min(hi, max(a0, a1))
    return lo, hi


def single_scatter_rays(mu_t, mu_r, mu_c, n=20000, seed=3):
    ins = cube_instrument(mu_t, mu_r, mu_c)
    ids = np.arange(n)
    src = oracle.trace_rays({"components": ins["components"][:1]}, ids, seed=seed, n_total=n)
    out = oracle.trace_rays(ins, ids, seed=seed, n_total=n)
    return src, out


def geometry(src, out, mu_t):
    """Per ray: the chord and its truncated-exponential CDF at the
    interaction point, the exit length, and the angle cosine."""
    h = 0.5 * N
    rows = []
    for i in range(len(out["w"])):
        if out["status"][i] != oracle.STATUS_EXITED:
            continue
        q0 = src["r"][i] - np.array([0.0, 0.0, 100.0])
        d0 = src["d"][i]
        a_in, a_out = box_interval(q0, d0, h)
        L = a_out - a_in
        p = out["r"][i] - np.array([0.0, 0.0, 100.0])
        s = np.dot(p - (q0 + a_in * d0), d0)
        d1 = out["d"][i]
        _, l_exit = box_interval(p, d1, h)
        rows.append((i, L, s, l_exit, float(np.dot(d0, d1))))
    return rows


def test_interaction_depth_truncated_exponential():
    mu_t = 1.5  # 1/cm
    src, out = single_scatter_rays(mu_t, 0.3, 1.0)
    rows = geometry(src, out, mu_t)
    assert len(rows) > 15000
    m = mu_t / 10.0
    u = [(1 - math.exp(-m * s)) / (1 - math.exp(-m * L)) for _, L, s, _, _ in rows]
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# layers along z of the cube: voxel planes k in [0, 4), [4, 8), [8, 12)
LAYERS = ((1, 0.6, 0.30), (2, 3.0, 0.60), (3, 1.2, 0.96))  # material, mu_total, mu_Rayleigh (1/cm)


def layered_instrument():
    ins = cube_instrument(1.0, 0.0, 0.0)
    ph = ins["components"][1]
    vol = np.zeros((N, N, N), np.uint8)
    tab = np.zeros((3, 4, 4))
    tab[0, 0] = 1.0  # material 0 unused
    for k, (m, mt, mr) in enumerate(LAYERS):
        vol[4 * k:4 * k + 4] = m
        tab[0, m], tab[1, m] = mt, mr  # Rayleigh only: Thomson angles, energy kept
    ph["volume"], ph["mu_table"] = vol, tab
    return ins


def layered_tau(p, d, length):
    """Optical depth of the segment p + t d, t in [0, length], through the
    z layers (z of the cube from 94 to 106 mm), by interval overlap."""
    tau = 0.0
    for k, (_, mt, _) in enumerate(LAYERS):
        z0, z1 = 94.0 + 4 * k, 98.0 + 4 * k
        if d[2] == 0.0:
            ln = length if z0 <= p[2] < z1 else 0.0
        else:
            t0, t1 = sorted(((z0 - p[2]) / d[2], (z1 - p[2]) / d[2]))
            ln = max(0.0, min(t1, length) - max(t0, 0.0))
        tau += mt * ln / 10.0
    return tau


def test_forced_interaction_across_material_layers():
    """Rays crossing three z layers of different attenuation and albedo
    (Rayleigh only).  The forced interaction point s on the chord has the
    distribution function (1 - e^-tau(s)) / (1 - e^-tau(L)), with tau(s) the
    piecewise-linear depth through the layers (KS on that transform); and
    each ray's weight over its source weight equals (1 - e^-tau(L)) times
    the albedo of the layer holding the point, the Thomson factor
    3/4 (1 + cos^2) of isotropic draws and e^-tau_exit along the new
    direction -- every factor from slab geometry written here, not from the
    voxel walk, so a walk that switches material in the wrong place, keeps
    the first material, or takes the albedo from elsewhere fails."""
    ins = layered_instrument()
    n = 20000
    ids = np.arange(n)
    src = oracle.trace_rays({"components": ins["components"][:1]}, ids, seed=7, n_total=n)
    out = oracle.trace_rays(ins, ids, seed=7, n_total=n)
    h = N / 2.0
    u, seen = [], set()
    for i in range(n):
        assert out["status"][i] == oracle.STATUS_EXITED
        q0 = src["r"][i] - np.array([0.0, 0.0, 100.0])
        d0 = src["d"][i]
        a_in, a_out = box_interval(q0, d0, h)
        L = a_out - a_in
        entry = src["r"][i] + a_in * d0
        tau_L = layered_tau(entry, d0, L)
        p = out["r"][i]
        s = float(np.dot(p - entry, d0))
        u.append((1 - math.exp(-layered_tau(entry, d0, s))) / (1 - math.exp(-tau_L)))
        d1 = out["d"][i]
        _, l_exit = box_interval(p - np.array([0.0, 0.0, 100.0]), d1, h)
        k = min(int((p[2] - 94.0) // 4), 2)
        seen.add(k)
        albedo = LAYERS[k][2] / LAYERS[k][1]
        ct = float(np.dot(d0, d1))
        want = (1 - math.exp(-tau_L)) * albedo * 0.75 * (1 + ct * ct) * math.exp(-layered_tau(p, d1, l_exit))
        got = out["w"][i] / src["w"][i]
        assert abs(got - want) <= 1e-9 * want, (i, got, want, k)
    assert seen == {0, 1, 2}
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def angular_factors(src, out, rows, mu_t, albedo):
    m = mu_t / 10.0
    f = []
    for i, L, s, l_exit, ct in rows:
        geom = (1 - math.exp(-m * L)) * albedo * math.exp(-m * l_exit)
        f.append((ct, out["w"][i] / (src["w"][i] * geom), src["E"][i], out["E"][i]))
    return np.array(f)


@pytest.mark.parametrize("kind", ["compton", "rayleigh"])
def test_weighted_angles(kind):
    mu_t = 0.8
    mu_r, mu_c = (0.0, 0.6) if kind == "compton" else (0.6, 0.0)
    src, out = single_scatter_rays(mu_t, mu_r, mu_c, n=40000, seed=4)
    rows = geometry(src, out, mu_t)
    F = angular_factors(src, out, rows, mu_t, 0.6 / mu_t)
    ct, fac, e_in, e_out = F[:, 0], F[:, 1], F[:, 2], F[:, 3]
    if kind == "compton":
        k = e_in / ME
        np.testing.assert_allclose(e_out, e_in / (1 + k * (1 - ct)), rtol=1e-12)
    else:
        np.testing.assert_array_equal(e_out, e_in)
    # isotropic draws: cos theta uniform, so the weighted histogram estimates
    # the probability of each cos-theta bin under the true law
    edges = np.linspace(-1, 1, 9)
    for b in range(8):
        sel = (ct >= edges[b]) & (ct < edges[b + 1])
        est = np.sum(fac[sel]) / len(ct)
        sd = np.sqrt(np.sum(fac[sel] ** 2) / len(ct) - est ** 2) / np.sqrt(len(ct))
        if kind == "rayleigh":
            want, _ = integrate.quad(lambda m: 0.375 * (1 + m * m), edges[b], edges[b + 1])
        else:
            # average over the source energies of the drawn rays
            ks = e_in[:2000] / ME
            want = np.mean([integrate.quad(lambda m: kn_pdf_unnorm(m, kk), edges[b], edges[b + 1])[0]
                            / oracle.kn_f(kk) for kk in ks])
        assert abs(est - want) <= 5 * sd + 2e-3 * want, (b, est, want, sd)


@pytest.mark.parametrize("order", [1, 2])
def test_aimed_equals_isotropic(order):
    mu_t, mu_r, mu_c = 2.0, 0.2, 1.2
    iso = cube_instrument(mu_t, mu_r, mu_c, order=order, detector=True, half_angle=0.03)
    aim = cube_instrument(mu_t, mu_r, mu_c, order=order, aim=True, half_angle=0.03)
    n_iso, n_aim = 4_000_000, 400_000
    ti = oracle.run(iso, n_iso, seed=11)[0]
    ta = oracle.run(aim, n_aim, seed=12)[0]

    def mean_sd(t, n):
        m = t["sum_w"].sum() / n
        return m, math.sqrt((t["sum_w2"].sum() / n - m * m) / n)

    mi, si = mean_sd(ti, n_iso)
    ma, sa = mean_sd(ta, n_aim)
    assert abs(mi - ma) <= 4 * math.hypot(si, sa), (mi, si, ma, sa)
    assert sa < si  # the aimed estimator is the efficient one


def test_no_scattering_channels():
    ins = cube_instrument(1.0, 0.0, 0.0, detector=True)
    t, led = oracle.run(ins, 20000, seed=1, ledger=True)
    assert t[0]["count"].sum() == 0
    assert led[4 * 1 + 1] == pytest.approx(led[4], rel=1e-12)  # all weight absorbed at the phantom
