"""Seeded synthetic inputs and instrument descriptions.

This module is the one thing the HIP library's tests and the CPU oracle
share: plain parameter values, geometry placement and seeded input arrays
(voxel phantoms, attenuation tables, reflectivity tables, d-spacings).  It
holds none of the tracing arithmetic.  Instruments are neutral dicts::

    {"components": [{"type": ..., "pos": (x, y, z), "rot": 3x3, ...}, ...]}

with ``rot`` the lab-to-local rotation (local = rot @ (lab - pos)), lengths
in mm, energies in keV, angles in rad, attenuation in 1/cm.

The paper's own workloads (section 3: a basic source + monitor instrument, a
focusing instrument with a compound refractive lens, an energy-dispersive CT
scanner with a voxel phantom)
need data that is not available here (tungsten spectrum, water, iron and
lead attenuation, the test piece geometry); the generators below stand in
for them with the shapes the paper gives (1 mm voxels, 128 energy bins,
1e6-1e9 rays).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

HC_KEV_ANGSTROM = 12.398419843320026
SI_LATTICE_ANGSTROM = 5.431020511


def rot_y(phi: float) -> np.ndarray:
    """Lab-to-local rotation for an object turned by phi about +y."""
    c, s = math.cos(phi), math.sin(phi)
    # the object's axes in the lab are R_y(phi) e_i; local = R_y(phi)^T lab
    return np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]], dtype=np.float64)


def frame_along(axis: Sequence[float]) -> np.ndarray:
    """Lab-to-local rotation whose local z is ``axis`` (in the y-z plane) and
    local x is lab x."""
    z = np.asarray(axis, dtype=np.float64)
    z = z / np.linalg.norm(z)
    x = np.array([1.0, 0.0, 0.0])
    y = np.cross(z, x)
    return np.stack([x, y, z])


# ---------------------------------------------------------------- inputs --

def make_mu_tables(seed: int = 1, n_mat: int = 8, n_ebin: int = 256, emin: float = 20.0,
                   emax: float = 150.0) -> np.ndarray:
    """Per-material attenuation tables mu[m, e] in 1/cm at the energy-bin
    centres: a power law with one absorption edge,
    mu_m(E) = A (E/60)^-p * (J if E >= E_edge) + B.

    Material 0 is air (mu(60) = 2e-4), 1 the bag shell (mu(60) = 0.3), and
    2.. objects with mu(60) log-uniform in [0.05, 5]; p ~ U(2.6, 3.2),
    E_edge ~ U(20, 90), J ~ U(2, 8), B = f mu(60) with f ~ U(0.05, 0.2).
    """
    rng = np.random.default_rng(seed)
    centres = emin + (np.arange(n_ebin) + 0.5) * ((emax - emin) / n_ebin)
    tab = np.zeros((n_mat, n_ebin))
    for m in range(n_mat):
        p = rng.uniform(2.6, 3.2)
        e_edge = rng.uniform(20.0, 90.0)
        jump = rng.uniform(2.0, 8.0)
        frac_b = rng.uniform(0.05, 0.2)
        if m == 0:
            mu60, jump = 2e-4, 1.0
        elif m == 1:
            mu60, jump = 0.3, 1.0
        else:
            mu60 = math.exp(rng.uniform(math.log(0.05), math.log(5.0)))
        B = frac_b * mu60
        j60 = jump if 60.0 >= e_edge else 1.0
        A = (mu60 - B) / j60
        jf = np.where(centres >= e_edge, jump, 1.0)
        tab[m] = A * (centres / 60.0) ** (-p) * jf + B
    return tab


def make_scatter_tables(mu_total: np.ndarray, seed: int = 1, emin: float = 20.0, emax: float = 150.0) -> np.ndarray:
    """Three-channel table (total, Rayleigh, Compton) for a scattering
    phantom, shape (3, n_mat, n_ebin), 1/cm at the bin centres.  Channel 0
    is ``mu_total`` unchanged; the synthetic scattering channels are
    Compton c_m (60/E)^0.3 and Rayleigh r_m (60/E)^2 with c_m = U(0.3, 0.6)
    and r_m = U(0.02, 0.08) times mu_total(60 keV), scaled down per bin where
    needed so that Rayleigh + Compton never exceed 0.9 of the total."""
    rng = np.random.default_rng(seed)
    n_mat, n_ebin = mu_total.shape
    centres = emin + (np.arange(n_ebin) + 0.5) * ((emax - emin) / n_ebin)
    i60 = int(np.argmin(np.abs(centres - 60.0)))
    out = np.zeros((3, n_mat, n_ebin))
    out[0] = mu_total
    for m in range(n_mat):
        c = rng.uniform(0.3, 0.6) * mu_total[m, i60]
        r = rng.uniform(0.02, 0.08) * mu_total[m, i60]
        comp = c * (60.0 / centres) ** 0.3
        ray = r * (60.0 / centres) ** 2
        scale = np.minimum(1.0, 0.9 * mu_total[m] / (comp + ray))
        out[1, m] = ray * scale
        out[2, m] = comp * scale
    return out


def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def make_phantom(n: int, seed: int = 1, n_objects: int = 32, n_mat: int = 8) -> np.ndarray:
    """Seeded luggage-like phantom: an n^3 uint8 material-id volume (array
    shape (z, y, x)).  A bag shell (material 1, 3 voxels thick) spans voxels
    [16, n - 16) on every axis; inside and outside is air (material 0).
    Then n_objects objects are painted in order: each an ellipsoid (randomly
    rotated, uniform quaternion) or an axis-aligned box with probability
    1/2, centre uniform inside the bag, semi-axes U(8, 40) voxels scaled by
    n/256, material uniform in {2, ..., n_mat - 1}; a voxel belongs to an
    object when its centre does."""
    rng = np.random.default_rng(seed)
    vol = np.zeros((n, n, n), dtype=np.uint8)
    lo, hi, wall = 16, n - 16, 3
    if hi - lo > 2 * wall:
        vol[lo:hi, lo:hi, lo:hi] = 1
        vol[lo + wall:hi - wall, lo + wall:hi - wall, lo + wall:hi - wall] = 0
    scale = n / 256.0
    for _ in range(n_objects):
        is_ellipsoid = rng.random() < 0.5
        centre = rng.uniform(lo + wall, hi - wall, size=3)
        semi = rng.uniform(8.0, 40.0, size=3) * scale
        mat = int(rng.integers(2, n_mat))
        rot = _random_rotation(rng) if is_ellipsoid else np.eye(3)
        reach = float(semi.max()) if is_ellipsoid else None
        if is_ellipsoid:
            b0 = np.floor(centre - reach).astype(int)
            b1 = np.ceil(centre + reach).astype(int) + 1
        else:
            b0 = np.floor(centre - semi).astype(int)
            b1 = np.ceil(centre + semi).astype(int) + 1
        b0 = np.clip(b0, 0, n)
        b1 = np.clip(b1, 0, n)
        if np.any(b1 <= b0):
            continue
        # voxel centres, order (x, y, z) -> array axes (z, y, x)
        xs = np.arange(b0[0], b1[0]) + 0.5 - centre[0]
        ys = np.arange(b0[1], b1[1]) + 0.5 - centre[1]
        zs = np.arange(b0[2], b1[2]) + 0.5 - centre[2]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        if is_ellipsoid:
            # coordinates in the ellipsoid's own axes: rot^T (p - c)
            u = rot[0, 0] * X + rot[1, 0] * Y + rot[2, 0] * Z
            v = rot[0, 1] * X + rot[1, 1] * Y + rot[2, 1] * Z
            w = rot[0, 2] * X + rot[1, 2] * Y + rot[2, 2] * Z
            inside = (u / semi[0]) ** 2 + (v / semi[1]) ** 2 + (w / semi[2]) ** 2 <= 1.0
        else:
            inside = (np.abs(X) <= semi[0]) & (np.abs(Y) <= semi[1]) & (np.abs(Z) <= semi[2])
        sub = vol[b0[2]:b1[2], b0[1]:b1[1], b0[0]:b1[0]]
        sub[inside] = mat
    return vol


def make_d_spacings(seed: int = 1, n: int = 200, lo: float = 0.8, hi: float = 4.0) -> np.ndarray:
    """n powder d-spacings uniform in [lo, hi] Angstrom."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def make_mirror_reflectivity(n: int = 512, theta_max: float = 6e-3, delta: float = 1.6e-5,
                             beta: float = 1.5e-6) -> np.ndarray:
    """Grazing-incidence Fresnel reflectivity of a mirror coating with
    refractive index 1 - delta + i beta on n angles over [0, theta_max]:
    R = |(t - t_t) / (t + t_t)|^2, t_t = sqrt(t^2 - 2 delta + 2 i beta)."""
    th = np.linspace(0.0, theta_max, n)
    tt = np.sqrt(th.astype(np.complex128) ** 2 - 2 * delta + 2j * beta)
    r = np.abs((th - tt) / (th + tt)) ** 2
    return r.astype(np.float64)


# ----------------------------------------------------------- instruments --

def _c(type_: str, pos=(0.0, 0.0, 0.0), rot=None, **kw) -> Dict:
    d = {"type": type_, "pos": tuple(float(x) for x in pos),
         "rot": np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64)}
    d.update(kw)
    return d


def basic_absorber() -> Dict:
    """Plain tracer, first workload: 1x1 mm emitter, 20-80 keV flat, 5 mrad
    half-angle cone; 1x1 mm slit at 1 m; 10 mm cube at 1.5 m with
    mu(E) = 2e4 E^-3 + 0.2 1/cm; 128x128 monitor, 100x100 mm, at 2 m."""
    return {"name": "basic_absorber", "components": [
        _c("source_rect_cone", wx=1.0, wy=1.0, half_angle=5e-3, emin=20.0, emax=80.0),
        _c("slit", pos=(0, 0, 1000.0), w=1.0, h=1.0),
        _c("box", pos=(0, 0, 1500.0), hx=5.0, hy=5.0, hz=5.0, mu_a=2e4, mu_b=0.2),
        _c("detector", pos=(0, 0, 2000.0), xmin=-50.0, xmax=50.0, ymin=-50.0, ymax=50.0,
           emin=0.0, emax=1000.0, nx=128, ny=128, ne=1),
    ]}


EDCT_SOD = 800.0      # source to phantom centre (mm)
EDCT_SDD = 1200.0     # source to detector (mm)
EDCT_NX, EDCT_NY, EDCT_NE = 256, 64, 128
EDCT_PITCH = 1.6      # mm


def edct_half_angle() -> float:
    hx = 0.5 * EDCT_NX * EDCT_PITCH
    hy = 0.5 * EDCT_NY * EDCT_PITCH
    return math.atan(math.sqrt(hx * hx + hy * hy) / EDCT_SDD)


def edct_projection(volume: np.ndarray, mu_table: np.ndarray, angle: float = 0.0,
                    strata: int = 1024, nx: int = EDCT_NX, ny: int = EDCT_NY, ne: int = EDCT_NE,
                    step: float = None, scatter_order: int = None, aim: bool = True,
                    early_out: bool = False) -> Dict:
    """Energy-dispersive CT projection: cone-beam point source (Kramers
    continuum (150 - E)/E on 20-150 keV plus lines at 59.3 and 67.2 keV,
    sigma 0.3 keV, 10 % of the photons each), voxel phantom of 1 mm voxels
    centred 0.8 m from the source and turned by ``angle`` about +y, ideal
    energy-resolving detector of nx x ny pixels of 1.6 mm and ne energy bins
    over [20, 150) keV at 1.2 m.  The cone circumscribes the detector.
    ``step`` (mm): cross the phantom with the fixed-step model instead of the
    exact path (the paper's default step is a third of the voxel).
    ``scatter_order`` K >= 1: trace the photons scattered exactly K times in
    the phantom instead of the uncollided ones; ``mu_table`` must then be
    the three-channel table of ``make_scatter_tables``; with ``aim`` the last
    scatter is aimed at the detector rectangle.  ``early_out``: an aperture
    100 mm from the source, the detector rectangle scaled to that distance
    (widened by a relative 1e-9), ends the rays bound elsewhere before the
    phantom; the phantom only absorbs, so every ray that would reach the
    detector passes it and the image is that of the plain instrument."""
    hx = 0.5 * nx * EDCT_PITCH
    hy = 0.5 * ny * EDCT_PITCH
    target = None
    if scatter_order is not None and aim:
        target = ((0.0, 0.0, EDCT_SDD), (hx, 0.0, 0.0), (0.0, hy, 0.0))
    aperture = []
    if early_out:
        zs, grow = 100.0, 1.0 + 1e-9
        aperture = [_c("slit", pos=(0, 0, zs), w=2.0 * hx * zs / EDCT_SDD * grow,
                       h=2.0 * hy * zs / EDCT_SDD * grow)]
    return {"name": "edct_projection", "components": [
        _c("source_cone_beam", half_angle=math.atan(math.sqrt(hx * hx + hy * hy) / EDCT_SDD),
           emin=20.0, emax=150.0, e0=150.0, f_cont=0.8, e_line1=59.3, f_line1=0.1,
           e_line2=67.2, f_line2=0.1, line_sigma=0.3, strata=strata),
        *aperture,
        _c("phantom", pos=(0, 0, EDCT_SOD), rot=rot_y(angle), voxel=1.0, volume=volume,
           mu_table=mu_table, table_emin=20.0, table_emax=150.0, step=step, scatter_order=scatter_order,
           scatter_target=target),
        _c("detector", pos=(0, 0, EDCT_SDD), xmin=-hx, xmax=hx, ymin=-hy, ymax=hy,
           emin=20.0, emax=150.0, nx=nx, ny=ny, ne=ne),
    ]}


def beamline(d_spacings: np.ndarray = None, reflectivity: np.ndarray = None) -> Dict:
    """Beamline optics: Gaussian undulator-like source (sigma 50 um,
    divergence 20 urad, 12.4 keV +-1 %); elliptic mirror at 30 m focusing at
    40 m (glancing 3 mrad, 1 m long, 512-angle reflectivity table); two-bounce
    Si(111) monochromator at 35 m (Darwin plateau 30 urad, 10 mm gap); powder
    plate of 200 d-spacings at the focus; 1024x1024 detector of 100 um pixels
    100 mm behind it, normal to the exit beam."""
    if d_spacings is None:
        d_spacings = make_d_spacings(1)
    if reflectivity is None:
        reflectivity = make_mirror_reflectivity()
    p, q, t0 = 30000.0, 10000.0, 3e-3
    beam = np.array([0.0, math.sin(2 * t0), math.cos(2 * t0)])
    pole = np.array([0.0, 0.0, p])
    d_si = SI_LATTICE_ANGSTROM / math.sqrt(3.0)
    theta_c = math.asin(HC_KEV_ANGSTROM / (2.0 * d_si * 12.4))
    gap = 10.0
    R = frame_along(beam)
    dcm_pos = pole + 5000.0 * beam
    n1_lab = R.T @ np.array([0.0, math.cos(theta_c), -math.sin(theta_c)])
    focus = pole + q * beam + 2.0 * gap * n1_lab
    det_pos = focus + 100.0 * beam
    return {"name": "beamline", "components": [
        _c("source_gaussian", sigma_x=0.05, sigma_y=0.05, sigma_xp=20e-6, sigma_yp=20e-6,
           e0=12.4, rel_halfwidth=0.01),
        _c("mirror_elliptic", pos=pole, p=p, q=q, theta0=t0, length=1000.0, width=50.0,
           theta_max=6e-3, reflectivity=reflectivity),
        _c("dcm", pos=dcm_pos, rot=R, d_spacing=d_si, theta_c=theta_c, darwin_width=30e-6, gap=gap),
        _c("powder", pos=focus, rot=R, w=1.0, h=1.0, d_spacings=d_spacings),
        _c("detector", pos=det_pos, rot=R, xmin=-51.2, xmax=51.2, ymin=-51.2, ymax=51.2,
           emin=0.0, emax=1000.0, nx=1024, ny=1024, ne=1),
    ]}


# focusing instrument with a compound refractive lens (beryllium stand-in)
BE_DENSITY = 1.848           # g/cm^3
BE_Z, BE_A = 4.0, 9.0121831  # electrons per atom, g/mol
CLASSICAL_ELECTRON_RADIUS_M = 2.8179403262e-15
AVOGADRO = 6.02214076e23
# attenuation of the stand-in, mu(E) = a / E^3 + b (1/cm): a photoabsorption
# term and a constant scattering term, Be-like in size (~0.42 1/cm at 20 keV,
# ~0.33 1/cm at 30 keV)
BE_MU_A, BE_MU_B = 950.0, 0.30


def be_delta(E: float) -> float:
    """Refractive decrement of beryllium at E keV from its electron density:
    delta = r_e lambda^2 n_e / (2 pi) (far from absorption edges)."""
    n_e = BE_DENSITY * AVOGADRO * BE_Z / BE_A * 1e6  # electrons per m^3
    lam = HC_KEV_ANGSTROM / E * 1e-10                 # m
    return CLASSICAL_ELECTRON_RADIUS_M * lam * lam * n_e / (2.0 * math.pi)


CRL_E0 = 23.32           # keV
CRL_LENS_DIST = 31500.0  # source to the lens stack centre (mm)
CRL_SLIT_DIST = 14000.0  # lens centre to the focusing slit (mm)


def crl_focusing(n_lenses: int = 16, aperture: float = 0.75) -> Dict:
    """Focusing instrument of the paper's section 3.2: a Gaussian
    undulator-like source (sigma 48.2 x 9.5 um, divergence 100 x 4.3 urad,
    23.32 keV +-1 keV flat), cropped to a 1 x 1 mm window just before a stack
    of n_lenses bi-concave parabolic beryllium lenses (apex radius 200 um,
    on-axis thickness 50 um -- the paper's lens-to-lens distance --, aperture
    radius ``aperture`` mm, lenses touching at the aperture rim) centred 31.5 m
    from the source; a circular slit of 0.1 mm diameter 14 m after the lens
    centre; a position-sensitive monitor (120 x 120 px of 1 um) and an energy
    monitor (130 bins of 20 eV) just behind it."""
    R, web = 0.2, 0.05
    pitch = web + aperture * aperture / R
    half = 0.5 * n_lenses * pitch
    zl, zs = CRL_LENS_DIST, CRL_LENS_DIST + CRL_SLIT_DIST
    return {"name": "crl_focusing", "components": [
        _c("source_gaussian", sigma_x=0.0482, sigma_y=0.0095, sigma_xp=100e-6, sigma_yp=4.3e-6,
           e0=CRL_E0, rel_halfwidth=1.0 / CRL_E0),
        _c("slit", pos=(0, 0, zl - half - 1.0), w=1.0, h=1.0),
        _c("lens_crl", pos=(0, 0, zl), R=R, n_lenses=n_lenses, web=web, pitch=pitch, aperture=aperture,
           delta_ref=be_delta(CRL_E0), e_ref=CRL_E0, mu_a=BE_MU_A, mu_b=BE_MU_B),
        _c("slit", pos=(0, 0, zs), circular=True, radius=0.05),
        _c("detector", pos=(0, 0, zs + 1.0), xmin=-0.06, xmax=0.06, ymin=-0.06, ymax=0.06,
           emin=20.0, emax=27.0, nx=120, ny=120, ne=1),
        _c("detector", pos=(0, 0, zs + 2.0), xmin=-0.06, xmax=0.06, ymin=-0.06, ymax=0.06,
           emin=22.0, emax=24.6, nx=1, ny=1, ne=130),
    ]}


# batched CT: projection angles x phantoms of uneven size
BATCH_SIZES = (64, 128, 256, 512)
BATCH_ANGLES = 360


# proposal network: 6 -> 128 -> 128 -> 56, packed W1, b1, W2, b2, W3, b3
MLP_SHAPES = [(6, 128), (128,), (128, 128), (128,), (128, 56), (56,)]


def init_mlp_params(seed: int) -> np.ndarray:
    """Seeded initial parameters of the proposal network (float32 values):
    weights uniform in +-1/sqrt(fan_in), biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            b = 1.0 / math.sqrt(shape[0])
            parts.append(rng.uniform(-b, b, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)


def projection_context(angle: float, n: int) -> np.ndarray:
    """Context of a projection for the proposal network: focal-spot offset
    (0, 0, 0) for a point source, (cos, sin) of the projection angle, and
    log2(n) / 9 for an n^3 phantom."""
    return np.array([0.0, 0.0, 0.0, math.cos(angle), math.sin(angle), math.log2(n) / 9.0], dtype=np.float32)
