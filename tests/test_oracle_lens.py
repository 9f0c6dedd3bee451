"""Pins of the oracle's compound refractive lens (a stack of bi-concave
parabolic lenses, the focusing instrument of the paper's section 3.2).

* against an independent ray trace written here in extended precision
  (numpy longdouble): surface hits by bisection on the surface equation,
  refraction by the scalar form of Snell's law (tangential part scaled by
  n1 / n2, normal part from cos theta_2), the path inside the material summed
  lens by lens -- with a realistic and an exaggerated refractive decrement;
* the refraction-free limit delta = 0: the ray goes straight and a ray
  parallel to the axis at radius rho keeps exp(-mu N (w + rho^2 / R) / 10);
* the paraxial back focal distance against the ray-transfer (ABCD) product of
  N thin lenses of power 2 delta / R spaced by the pitch, at several energies
  (delta ~ E^-2);
* rays meeting a surface outside the aperture are absorbed.
"""
import math

import numpy as np
import pytest

import oracle
import workloads

LD = np.longdouble


def lens_dict(n=3, delta=6.26e-7, e_ref=23.32, aperture=0.75, R=0.2, web=0.05, mu_a=950.0, mu_b=0.3):
    pitch = web + aperture * aperture / R
    return {"type": "lens_crl", "pos": (0, 0, 0), "rot": np.eye(3), "R": R, "n_lenses": n, "web": web,
            "pitch": pitch, "aperture": aperture, "delta_ref": delta, "e_ref": e_ref, "mu_a": mu_a, "mu_b": mu_b}


def surface_hit(q, d, z0, s, R):
    """t >= 0 of the first crossing of z = z0 + s rho^2 / 2R, by bisection."""
    def f(t):
        x, y, z = q + t * d
        return z - z0 - s * (x * x + y * y) / (2 * R)
    lo = LD(0)
    hi = LD(1)
    while f(hi) * f(lo) > 0:  # the surface lies ahead within a few mm
        hi *= 2
        assert hi < 1e6
    for _ in range(200):
        mid = (lo + hi) / 2
        if f(lo) * f(mid) <= 0:
            hi = mid
        else:
            lo = mid
    return (lo + hi) / 2


def refract(d, m, n1, n2):
    """Scalar Snell: the tangential part scales by n1 / n2, the normal part
    follows from the unit length."""
    cos1 = np.dot(d, m)
    tang = d - cos1 * m
    tang2 = tang * (n1 / n2)
    sin2sq = np.dot(tang2, tang2)
    return tang2 + np.sqrt(LD(1) - sin2sq) * m


def reference(L, q, d, E):
    R, N, w, p, ra = (LD(L[k]) for k in ("R", "n_lenses", "web", "pitch", "aperture"))
    delta = LD(L["delta_ref"]) * (LD(L["e_ref"]) / LD(E)) ** 2
    mu = LD(L["mu_a"]) / LD(E) ** 3 + LD(L["mu_b"])
    q = np.array(q, dtype=LD)
    d = np.array(d, dtype=LD)
    n_mat = 1 - delta
    path = LD(0)
    for k in range(int(N)):
        c = (k - (N - 1) / 2) * p
        for z0, s, n1, n2 in ((c - w / 2, -1, LD(1), n_mat), (c + w / 2, 1, n_mat, LD(1))):
            t = surface_hit(q, d, z0, s, R)
            q = q + t * d
            if q[0] ** 2 + q[1] ** 2 > ra * ra:
                return False, q, d, LD(0)
            g = np.array([-s * q[0] / R, -s * q[1] / R, LD(1)])
            m = g / np.sqrt(np.dot(g, g))
            d = refract(d, m, n1, n2)
            if s == 1:
                path += t
    return True, q, d, np.exp(-mu * path / 10)


@pytest.mark.parametrize("n,delta", [(1, 6.26e-7), (3, 6.26e-7), (2, 1e-3), (16, 6.26e-7)])
def test_matches_independent_trace(n, delta):
    rng = np.random.default_rng(20 + n)
    L = lens_dict(n=n, delta=delta)
    half = 0.5 * n * L["pitch"]
    for _ in range(40):
        rho = 0.6 * math.sqrt(rng.random())
        phi = 2 * math.pi * rng.random()
        start = np.array([rho * math.cos(phi), rho * math.sin(phi), -half - 5.0])
        slope = rng.normal(0, 2e-3, 2)
        d = np.array([slope[0], slope[1], 1.0])
        d /= np.linalg.norm(d)
        E = rng.uniform(20, 27)
        ok, qo, do, w = oracle.lens(L, start, d, E)
        okr, qr, dr, wr = reference(L, start, d, E)
        assert ok == okr
        if not ok:
            continue
        assert np.max(np.abs(do - dr.astype(float))) <= 1e-14
        assert np.max(np.abs(qo - qr.astype(float))) <= 1e-12 * max(1.0, float(np.max(np.abs(qr))))
        assert abs(w - float(wr)) <= 1e-13


def test_refraction_free_limit():
    L = lens_dict(n=16, delta=0.0)
    half = 0.5 * 16 * L["pitch"]
    for rho in (0.0, 0.1, 0.37, 0.7):
        E = 23.32
        ok, qo, do, w = oracle.lens(L, [rho, 0.0, -half - 1.0], [0.0, 0.0, 1.0], E)
        assert ok
        assert np.array_equal(do, [0.0, 0.0, 1.0])
        assert qo[0] == rho and qo[1] == 0.0
        mu = L["mu_a"] / E ** 3 + L["mu_b"]
        want = math.exp(-mu * 16 * (L["web"] + rho * rho / L["R"]) / 10)
        assert w == pytest.approx(want, rel=1e-13)
    # a tilted ray also goes straight
    d = np.array([3e-3, -2e-3, 1.0])
    d /= np.linalg.norm(d)
    ok, qo, do, _ = oracle.lens(L, [0.2, 0.1, -half - 1.0], d, 21.0)
    assert ok and np.array_equal(do, d)
    t = (qo[2] - (-half - 1.0)) / d[2]
    assert np.allclose(qo, np.array([0.2, 0.1, -half - 1.0]) + t * d, rtol=0, atol=1e-12)


@pytest.mark.parametrize("E", [20.0, 23.32, 26.0])
def test_paraxial_focal_length(E):
    delta_ref = workloads.be_delta(23.32)
    L = lens_dict(n=16, delta=delta_ref)
    delta = delta_ref * (23.32 / E) ** 2
    p, N = L["pitch"], 16
    half = 0.5 * N * p
    # ray-transfer product of N thin lenses (power 2 delta / R) at the lens
    # centres, from the first centre to the last
    M = np.eye(2)
    P = np.array([[1.0, 0.0], [-2 * delta / L["R"], 1.0]])
    T = np.array([[1.0, p], [0.0, 1.0]])
    for k in range(N):
        M = P @ M
        if k < N - 1:
            M = T @ M
    # a parallel ray at height h leaves the last centre at (A h, C h): it
    # crosses the axis -A / C beyond the last lens centre
    bfd_abcd = -M[0, 0] / M[1, 0] + (half - 0.5 * p)
    h = 0.002
    ok, qo, do, _ = oracle.lens(L, [h, 0.0, -half - 1.0], [0.0, 0.0, 1.0], E)
    assert ok
    bfd = qo[2] - qo[0] * do[2] / do[0]
    assert bfd == pytest.approx(bfd_abcd, rel=1e-4)
    # thin-lens limit R / (2 N delta), about 10 m at 23.32 keV
    assert bfd == pytest.approx(L["R"] / (2 * N * delta), rel=0.01)


def test_aperture():
    L = lens_dict(n=4, aperture=0.3)
    half = 0.5 * 4 * L["pitch"]
    ok, *_ = oracle.lens(L, [0.29, 0.0, -half - 1.0], [0.0, 0.0, 1.0], 23.32)
    assert ok
    ok, *_ = oracle.lens(L, [0.31, 0.0, -half - 1.0], [0.0, 0.0, 1.0], 23.32)
    assert not ok
    # leaving the aperture inside the stack: a steep ray from the axis
    d = np.array([0.2, 0.0, 1.0])
    d /= np.linalg.norm(d)
    ok, *_ = oracle.lens(L, [-0.15, 0.0, -half - 1.0], d, 23.32)
    assert not ok
    # a ray moving away from the stack cannot reach it
    ok, *_ = oracle.lens(L, [0.0, 0.0, -half - 1.0], [0.0, 0.0, -1.0], 23.32)
    assert not ok
