"""Pins of the oracle's voxel traversal (Siddon's merge form).

* homogeneous volume: tau = mu * chord / 10, chord from an independent
  ray/box intersection;
* layered volume crossed face to face: tau = sum_k mu_k * v / |dz| / 10;
* brute force on small volumes: every voxel slab-tested on its own, the
  segment set and tau must agree with the traversal;
* segment lengths sum to the chord, consecutive voxels are face neighbours,
  the segment count is one more than the number of distinct crossings;
* special rays: axis-parallel, through voxel corners and edges, starting
  inside, missing.
"""
import math

import numpy as np
import pytest

import oracle


def phantom(vol, mu, voxel=1.0, emin=20.0, emax=150.0):
    return {"type": "phantom", "pos": (0, 0, 0), "rot": np.eye(3), "voxel": voxel, "volume": vol,
            "mu_table": mu, "table_emin": emin, "table_emax": emax}


def ebin(E, n=256, emin=20.0, emax=150.0):
    return min(max(int(math.floor((E - emin) * (n / (emax - emin)))), 0), n - 1)


def chord(nxyz, voxel, q, d):
    """Length of the ray q + a d (a >= 0) inside the centred box."""
    h = 0.5 * np.asarray(nxyz, float) * voxel
    lo_a, hi_a = 0.0, np.inf
    for i in range(3):
        if d[i] == 0:
            if not (-h[i] < q[i] < h[i]):
                return 0.0
            continue
        a0, a1 = (-h[i] - q[i]) / d[i], (h[i] - q[i]) / d[i]
        lo_a, hi_a = max(lo_a, min(a0, a1)), min(hi_a, max(a0, a1))
    return max(0.0, hi_a - lo_a)


def brute_force(vol, mu_e, voxel, q, d):
    """Per-voxel slab intersection lengths and tau (vol shape (z, y, x))."""
    nz, ny, nx = vol.shape
    n = (nx, ny, nz)
    corner = [-0.5 * n[i] * voxel for i in range(3)]
    idx = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    lo = np.array(corner) + idx * voxel
    hi = lo + voxel
    amin = np.zeros(len(idx))
    amax = np.full(len(idx), np.inf)
    for i in range(3):
        if d[i] == 0:
            inside = (lo[:, i] < q[i]) & (q[i] < hi[:, i])
            amax = np.where(inside, amax, -np.inf)
        else:
            a0 = (lo[:, i] - q[i]) / d[i]
            a1 = (hi[:, i] - q[i]) / d[i]
            amin = np.maximum(amin, np.minimum(a0, a1))
            amax = np.minimum(amax, np.maximum(a0, a1))
    ln = np.maximum(0.0, amax - amin)
    flat = idx[:, 0] + nx * (idx[:, 1] + ny * idx[:, 2])
    mats = vol.reshape(-1)[flat]
    tau = np.sum(mu_e[mats] * ln) / 10.0
    return tau, flat, ln


def random_rays(rng, n, size, inside_frac=0.2):
    rays = []
    for _ in range(n):
        if rng.random() < inside_frac:
            q = rng.uniform(-0.45, 0.45, 3) * size
        else:
            u = rng.normal(size=3)
            q = 3.0 * size * u / np.linalg.norm(u)
        target = rng.uniform(-0.5, 0.5, 3) * size
        d = target - q if np.linalg.norm(target - q) > 0 else rng.normal(size=3)
        d = d / np.linalg.norm(d)
        rays.append((q, d))
    return rays


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(4)
    vol = rng.integers(0, 8, size=(11, 9, 7)).astype(np.uint8)
    mu = rng.uniform(0.01, 3.0, size=(8, 256))
    return vol, mu


def test_homogeneous_closed_form():
    rng = np.random.default_rng(1)
    for voxel in (1.0, 0.8):
        vol = np.full((13, 10, 7), 3, np.uint8)
        mu = np.zeros((8, 256))
        mu[3, :] = 1.7
        ph = phantom(vol, mu, voxel)
        for q, d in random_rays(rng, 200, np.array([7, 10, 13]) * voxel):
            tau, vox, ln = oracle.siddon_segments(ph, q, d, 60.0)
            L = chord((7, 10, 13), voxel, q, d)
            assert abs(tau - 1.7 * L / 10.0) <= 1e-12 * max(tau, 1e-300) + 1e-15
            assert abs(ln.sum() - L) <= 1e-12 * max(L, 1.0)


def test_layered_face_to_face():
    rng = np.random.default_rng(2)
    nz = 12
    mu = rng.uniform(0.1, 2.0, size=(8, 256))
    vol = np.zeros((nz, 6, 6), np.uint8)
    layer_mat = rng.integers(0, 8, nz)
    for k in range(nz):
        vol[k] = layer_mat[k]
    ph = phantom(vol, mu)
    for _ in range(100):
        E = rng.uniform(20, 150)
        e = ebin(E)
        start = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), -20.0])
        end = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), 20.0])
        d = (end - start) / np.linalg.norm(end - start)
        tau, _, _ = oracle.siddon_segments(ph, start, d, E)
        want = sum(mu[layer_mat[k], e] * 1.0 / abs(d[2]) for k in range(nz)) / 10.0
        assert abs(tau - want) <= 1e-13 * want


def test_brute_force_small_volumes(small):
    vol, mu = small
    rng = np.random.default_rng(3)
    for voxel in (1.0, 0.8):
        ph = phantom(vol, mu, voxel)
        size = np.array([7, 9, 11]) * voxel
        for q, d in random_rays(rng, 300, size):
            E = rng.uniform(20, 150)
            tau, vox, ln = oracle.siddon_segments(ph, q, d, E)
            tau_bf, flat, ln_bf = brute_force(vol, mu[:, ebin(E)], voxel, q, d)
            assert abs(tau - tau_bf) <= 1e-12 * max(tau_bf, 1.0)
            # same voxels carry the same lengths
            want = {int(f): l for f, l in zip(flat, ln_bf) if l > 1e-9}
            got = {}
            for v, l in zip(vox, ln):
                got[int(v)] = got.get(int(v), 0.0) + l
            got = {k: v for k, v in got.items() if v > 1e-9}
            assert set(got) == set(want)
            for k in want:
                assert abs(got[k] - want[k]) <= 1e-12 * max(1.0, want[k])


def test_segment_structure(small):
    vol, mu = small
    rng = np.random.default_rng(5)
    ph = phantom(vol, mu)
    nx, ny, nz = 7, 9, 11
    for q, d in random_rays(rng, 200, np.array([7, 9, 11.0]), inside_frac=0.0):
        tau, vox, ln = oracle.siddon_segments(ph, q, d, 50.0)
        if len(vox) == 0:
            assert chord((nx, ny, nz), 1.0, q, d) == 0.0
            continue
        ijk = np.stack([vox % nx, (vox // nx) % ny, vox // (nx * ny)], 1)
        steps = np.abs(np.diff(ijk, axis=0)).sum(1)
        assert np.all(steps == 1)  # generic rays never cross an edge exactly
        # distinct crossings strictly inside the chord, counted independently
        h = 0.5 * np.array([nx, ny, nz], float)
        a_lo = max(0.0, max(min((-h[i] - q[i]) / d[i], (h[i] - q[i]) / d[i]) for i in range(3)))
        a_hi = min(max((-h[i] - q[i]) / d[i], (h[i] - q[i]) / d[i]) for i in range(3))
        crossings = set()
        for i, n in enumerate((nx, ny, nz)):
            for p in range(n + 1):
                a = (-h[i] + p - q[i]) / d[i]
                if a_lo + 1e-9 < a < a_hi - 1e-9:
                    crossings.add(round(a, 9))
        assert len(vox) == len(crossings) + 1


def test_special_rays(small):
    vol, mu = small
    ph = phantom(vol, mu)
    e = ebin(80.0)
    cases = [
        (np.array([0.3, 0.2, -30.0]), np.array([0.0, 0.0, 1.0])),        # along z
        (np.array([-30.0, 0.5, 0.5]), np.array([1.0, 0.0, 0.0])),        # along x, on planes? no: 0.5 is a plane
        (np.array([-30.0, 0.25, 0.75]), np.array([1.0, 0.0, 0.0])),      # along x
        (np.array([0.1, -30.0, 0.2]), np.array([0.0, 1.0, 0.0])),        # along y
        (np.array([-3.5, -4.5, -5.5]) - 3.0, np.array([1.0, 1.0, 1.0]) / math.sqrt(3)),  # through corners
        (np.array([-10.0, 0.0, 0.0]), np.array([1.0, 1.0, 0.0]) / math.sqrt(2)),          # along voxel edges
        (np.array([0.1, 0.2, 0.3]), np.array([0.6, 0.0, 0.8])),          # starts inside
        (np.array([30.0, 30.0, 30.0]), np.array([1.0, 0.0, 0.0])),       # misses
        (np.array([0.0, 0.0, -30.0]), np.array([0.0, 0.0, -1.0])),       # points away
    ]
    for q, d in cases:
        tau, vox, ln = oracle.siddon_segments(ph, q, d, 80.0)
        tau_bf, _, _ = brute_force(vol, mu[:, e], 1.0, q, d)
        on_plane = any(d[i] == 0 and float(q[i] + 0.5 * vol.shape[2 - i]) == round(float(q[i] + 0.5 * vol.shape[2 - i])) for i in range(3))
        if on_plane:
            # a ray running inside a voxel face is outside every open voxel for
            # the brute force; the traversal assigns it to one side -- only
            # check it stays finite and non-negative
            assert tau >= 0 and np.isfinite(tau)
            continue
        assert abs(tau - tau_bf) <= 1e-12 * max(tau_bf, 1.0), (q, d, tau, tau_bf)
        assert np.all(ln > 0)
