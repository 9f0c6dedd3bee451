"""CPU oracle for the per-ray X-ray Monte Carlo tracer -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``mxo.c`` (plain scalar C,
``gcc -O2 -ffp-contract=off``) with ctypes and takes instruments in the
neutral dict form of ``workloads`` (lists of component dicts with numpy
arrays).  It shares no code with the HIP library under
``paper_2410_08747_amd`` and never imports it.

What is computed is described in ``mxo.c``: rays are drawn at the source,
carried through the components in order and tallied at the monitors (paper,
sections 2 and 3).  The voxel phantom uses Siddon's merge form, or the paper's
fixed-step model when the phantom dict gives a step length.

How each function is pinned (tests marked ``not gpu``):

* ``philox`` -- bit equality with the Philox4x32-10 engine of the rocRAND
  headers (an independent implementation), for random counters and keys;
  uniformity of ``uniform`` by chi-square and moments.
* sources -- sample moments and solid-angle fractions against closed forms
  (uniform-in-solid-angle cone, Kramers continuum plus lines integrated in
  closed form, Gaussian moments).
* slit + box (first workload) -- slit transmission equal to the emitter-
  averaged solid angle of the slit over the cone solid angle (2-D quadrature),
  the per-ray Beer-Lambert factor for face-to-face chords, the ensemble
  transmitted weight from a 1-D integral.
* phantom -- homogeneous and layered volumes against closed-form optical
  depths, brute-force per-voxel slab intersection on small volumes, segment
  sum equal to the chord, adjacency of consecutive voxels.
* fixed-step phantom model -- homogeneous volumes give mu times the chord;
  a hand-computed three-voxel row; the step count ceil(chord / h); the
  distance to the exact (brute-force) optical depth within h times the
  attenuation spread per material change, shrinking linearly with h.
* mirror -- the focal property of the ellipse and equal angles in and out.
* monochromator -- the exit direction equals the entrance direction, the
  Darwin curve integrals, Bragg's law at the plateau centre.
* powder -- the scattering angle equals 2 asin(lambda / 2d) and the azimuth
  is uniform.
* compound refractive lens -- Snell's law at every surface (unit direction,
  tangential component scaled by n1 / n2, normal on the paraboloid), the
  paraxial focal length R / (2 N delta) and the image distance of the thin
  lens, transmission exp(-mu N (w + rho^2 / R)) for paraxial rays, the
  aperture and the refraction-free limit delta = 0.
* scattering phantom (scatter orders) -- the Klein-Nishina total cross
  section against a quadrature of the differential one and its Thomson
  limit; the forced interaction depth against the truncated exponential
  (KS); the weighted angular distribution of single scatter against
  Klein-Nishina and Thomson (binned); Compton energies against the
  scattering angle ray by ray; the mean weight of single scatter in a
  homogeneous cube against the closed form; no scattering material gives
  no weight.
* ledger -- weight emitted equals absorbed + attenuated + exiting weight.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mxo.c")
_LIB = os.path.join(_HERE, "liboracle.so")

TYPE_CODES = {
    "source_rect_cone": 0,
    "source_cone_beam": 1,
    "source_gaussian": 2,
    "slit": 3,
    "box": 4,
    "phantom": 5,
    "mirror_elliptic": 6,
    "dcm": 7,
    "powder": 8,
    "detector": 9,
    "lens_crl": 10,
}
STATUS_EXITED = 1
STATUS_ABSORBED = 2


def build(force: bool = True) -> str:
    """Compile mxo.c into liboracle.so (plain C, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = [
            "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread",
        ]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Comp(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("pos", ctypes.c_double * 3),
        ("rot", ctypes.c_double * 9),
        ("par", ctypes.c_double * 24),
        ("data0", ctypes.c_void_p),
        ("data1", ctypes.c_void_p),
        ("n0", ctypes.c_int64),
        ("n1", ctypes.c_int64),
        ("dims", ctypes.c_int64 * 4),
    ]


class _Tally(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_void_p),
        ("sum_w", ctypes.c_void_p),
        ("sum_w2", ctypes.c_void_p),
        ("n_bins", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.mxo_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.mxo_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int]
        lib.mxo_uniform.restype = ctypes.c_double
        lib.mxo_strata_side.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.mxo_strata_side.restype = ctypes.c_uint64
        lib.mxo_spectrum.argtypes = [ctypes.c_void_p, ctypes.c_double]
        lib.mxo_spectrum.restype = ctypes.c_double
        lib.mxo_run.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
        ]
        lib.mxo_trace_rays.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ]
        lib.mxo_siddon_debug.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
        ]
        lib.mxo_siddon_debug.restype = ctypes.c_double
        lib.mxo_step_debug.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_void_p]
        lib.mxo_step_debug.restype = ctypes.c_double
        lib.mxo_lens_debug.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.mxo_lens_debug.restype = ctypes.c_int
        lib.mxo_kn_f.argtypes = [ctypes.c_double]
        lib.mxo_kn_f.restype = ctypes.c_double
        lib.mxo_ppnd16.argtypes = [ctypes.c_double]
        lib.mxo_ppnd16.restype = ctypes.c_double
        lib.mxo_truncnorm.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.mxo_truncnorm.restype = ctypes.c_double
        lib.mxo_proposal_density.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        lib.mxo_proposal_density.restype = ctypes.c_double
        lib.mxo_trace_after_source.argtypes = [
            ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p,
        ]
        lib.mxo_proposal_weight.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.mxo_proposal_weight.restype = ctypes.c_double
        lib.mxo_proposal_bounds.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
                                            ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class Instrument:
    """The oracle's own view of a neutral instrument dict.

    Keeps references to every numpy array it hands to C so they outlive the
    calls.
    """

    def __init__(self, instr: Dict):
        comps = instr["components"]
        self.n = len(comps)
        self.arr = (_Comp * self.n)()
        self._keep: List[np.ndarray] = []
        self.detectors: List[Dict] = []
        for k, c in enumerate(comps):
            self._fill(self.arr[k], c)

    def _keep_arr(self, a, dtype) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(a, dtype=dtype))
        self._keep.append(a)
        return a

    def _fill(self, s: _Comp, c: Dict) -> None:
        t = c["type"]
        s.type = TYPE_CODES[t]
        pos = c.get("pos", (0.0, 0.0, 0.0))
        rot = np.asarray(c.get("rot", np.eye(3)), dtype=np.float64).reshape(9)
        for i in range(3):
            s.pos[i] = float(pos[i])
        for i in range(9):
            s.rot[i] = float(rot[i])
        p = s.par
        if t == "source_rect_cone":
            p[0], p[1], p[2], p[3], p[4] = c["wx"], c["wy"], c["half_angle"], c["emin"], c["emax"]
        elif t == "source_cone_beam":
            p[0], p[1], p[2], p[3] = c["half_angle"], c["emin"], c["emax"], c["e0"]
            p[4], p[5], p[6] = c["f_cont"], c["e_line1"], c["f_line1"]
            p[7], p[8], p[9] = c["e_line2"], c["f_line2"], c["line_sigma"]
            s.dims[0] = int(c.get("strata", 1))
        elif t == "source_gaussian":
            p[0], p[1], p[2], p[3] = c["sigma_x"], c["sigma_y"], c["sigma_xp"], c["sigma_yp"]
            p[4], p[5] = c["e0"], c["rel_halfwidth"]
        elif t == "slit":
            if c.get("circular", False):
                s.flags = 1
                p[2] = c["radius"]
            else:
                p[0], p[1] = c["w"], c["h"]
        elif t == "box":
            p[0], p[1], p[2], p[3], p[4] = c["hx"], c["hy"], c["hz"], c["mu_a"], c["mu_b"]
        elif t == "phantom":
            vol = self._keep_arr(c["volume"], np.uint8)
            mu = self._keep_arr(c["mu_table"], np.float64)
            nz, ny, nx = vol.shape
            s.dims[0], s.dims[1], s.dims[2] = nx, ny, nz
            s.dims[3] = mu.shape[1] if mu.ndim == 3 else mu.shape[0]
            s.data0, s.data1 = _ptr(vol), _ptr(mu)
            s.n0, s.n1 = vol.size, mu.size
            p[0], p[1], p[2] = c["voxel"], c["table_emin"], c["table_emax"]
            if c.get("step") is not None:
                s.flags = 1
                p[3] = c["step"]
            if c.get("scatter_order") is not None:
                s.flags = 2
                p[4] = c["scatter_order"]
                if c.get("scatter_target") is not None:
                    s.flags = 2 | 4
                    for i, v in enumerate(np.asarray(c["scatter_target"], dtype=np.float64).reshape(9)):
                        p[5 + i] = v
        elif t == "mirror_elliptic":
            tab = self._keep_arr(c["reflectivity"], np.float64)
            p[0], p[1], p[2], p[3], p[4], p[5] = c["p"], c["q"], c["theta0"], c["length"], c["width"], c["theta_max"]
            s.data0, s.n0 = _ptr(tab), tab.size
        elif t == "dcm":
            p[0], p[1], p[2], p[3] = c["d_spacing"], c["theta_c"], c["darwin_width"], c["gap"]
        elif t == "powder":
            dsp = self._keep_arr(c["d_spacings"], np.float64)
            p[0], p[1] = c["w"], c["h"]
            s.data0, s.n0 = _ptr(dsp), dsp.size
        elif t == "detector":
            p[0], p[1], p[2], p[3], p[4], p[5] = c["xmin"], c["xmax"], c["ymin"], c["ymax"], c["emin"], c["emax"]
            s.dims[0], s.dims[1], s.dims[2] = c["nx"], c["ny"], c["ne"]
            s.flags = 1 if c.get("wavelength", False) else 0
            self.detectors.append(c)
        elif t == "lens_crl":
            vals = [c["R"], c["n_lenses"], c["web"], c["pitch"], c["aperture"], c["delta_ref"], c["e_ref"],
                    c["mu_a"], c["mu_b"]]
            for i, v in enumerate(vals):
                p[i] = v
        else:
            raise ValueError(f"unknown component type {t}")


def _gmm(gmm):
    if gmm is None:
        return None, None
    g = np.ascontiguousarray(np.asarray(gmm, dtype=np.float64).reshape(56))
    return g, _ptr(g)


def run(instr: Dict, n: int, seed: int, first: int = 0, n_total: Optional[int] = None,
        purpose: int = 0, job: int = 0, threads: Optional[int] = None, ledger: bool = False,
        gmm=None, alpha: float = 0.1):
    """Trace rays [first, first + n) of an n_total-ray run (the cone-beam
    source drawing from the proposal mixture ``gmm``, 8 x (pi, mu_u, mu_v,
    mu_E, sigma_u, sigma_v, sigma_E), with plain weight ``alpha``, when given).

    Returns a list (one per detector) of dicts with ``count`` (uint64),
    ``sum_w`` and ``sum_w2`` (float64) arrays in the flat bin order
    (iy * nx + ix) * ne + ie, and, when ``ledger`` is set, the weight ledger
    as a (n_components * 4 + 1,) float64 array.
    """
    lib = _load()
    ins = Instrument(instr)
    n_total = n if n_total is None else n_total
    threads = threads or (os.cpu_count() or 1)
    outs, tal = [], (_Tally * max(1, len(ins.detectors)))()
    for i, d in enumerate(ins.detectors):
        nb = int(d["nx"]) * int(d["ny"]) * int(d["ne"])
        o = {"count": np.zeros(nb, np.uint64), "sum_w": np.zeros(nb), "sum_w2": np.zeros(nb)}
        outs.append(o)
        tal[i].count, tal[i].sum_w, tal[i].sum_w2 = _ptr(o["count"]), _ptr(o["sum_w"]), _ptr(o["sum_w2"])
        tal[i].n_bins = nb
    led = np.zeros(4 * ins.n + 1) if ledger else None
    g, gp = _gmm(gmm)
    lib.mxo_run(ctypes.addressof(ins.arr), ins.n, seed, first, n, n_total, purpose, job, gp, alpha,
                ctypes.addressof(tal), _ptr(led) if led is not None else None, threads)
    return (outs, led) if ledger else outs


def trace_rays(instr: Dict, ids: Sequence[int], seed: int, n_total: int, purpose: int = 0, job: int = 0,
               gmm=None, alpha: float = 0.1):
    """Final state of each listed ray: r, d (n,3), E, w, status, dead_at, bin."""
    lib = _load()
    ins = Instrument(instr)
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    n = ids.size
    out = {
        "r": np.zeros((n, 3)), "d": np.zeros((n, 3)), "E": np.zeros(n), "w": np.zeros(n),
        "status": np.zeros(n, np.int32), "dead_at": np.zeros(n, np.int32), "bin": np.zeros(n, np.int64),
    }
    g, gp = _gmm(gmm)
    lib.mxo_trace_rays(ctypes.addressof(ins.arr), ins.n, seed, n_total, purpose, job, gp, alpha, _ptr(ids), n,
                       _ptr(out["r"]), _ptr(out["d"]), _ptr(out["E"]), _ptr(out["w"]),
                       _ptr(out["status"]), _ptr(out["dead_at"]), _ptr(out["bin"]))
    return out


def philox(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib.mxo_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return [int(x) for x in o]


def uniform(seed: int, ray: int, index: int, purpose: int = 0, job: int = 0) -> float:
    return _load().mxo_uniform(seed, ray, purpose, job, index)


def strata_side(G: int, n_total: int) -> int:
    return int(_load().mxo_strata_side(G, n_total))


def spectrum(source: Dict, E: float) -> float:
    """Photon-number density of the cone-beam source spectrum at E (1/keV)."""
    ins = Instrument({"components": [source]})
    return _load().mxo_spectrum(ctypes.addressof(ins.arr[0].par), float(E))


def siddon_segments(phantom: Dict, q, dl, E: float, max_seg: int = 100000):
    """tau and the (voxel, length) segments of one ray given in the phantom's
    local frame."""
    lib = _load()
    ins = Instrument({"components": [phantom]})
    qa = np.asarray(q, dtype=np.float64)
    da = np.asarray(dl, dtype=np.float64)
    vox = np.zeros(max_seg, np.int64)
    ln = np.zeros(max_seg)
    ns = np.zeros(1, np.int64)
    tau = lib.mxo_siddon_debug(ctypes.addressof(ins.arr[0]), _ptr(qa), _ptr(da), float(E),
                               _ptr(vox), _ptr(ln), max_seg, _ptr(ns))
    k = int(min(ns[0], max_seg))
    return tau, vox[:k].copy(), ln[:k].copy()


def step_tau(phantom: Dict, q, dl, E: float):
    """(tau, number of steps) of one ray through the phantom under the
    fixed-step model (the dict's ``step`` is the step length in mm), given in
    the phantom's local frame."""
    lib = _load()
    ins = Instrument({"components": [phantom]})
    qa = np.asarray(q, dtype=np.float64)
    da = np.asarray(dl, dtype=np.float64)
    ns = np.zeros(1, np.int64)
    tau = lib.mxo_step_debug(ctypes.addressof(ins.arr[0]), _ptr(qa), _ptr(da), float(E), _ptr(ns))
    return tau, int(ns[0])


def lens(lens_dict: Dict, q, dl, E: float):
    """One ray through a compound refractive lens, given in the lens frame:
    (ok, position, direction, weight factor) after the stack."""
    lib = _load()
    ins = Instrument({"components": [lens_dict]})
    qa = np.asarray(q, dtype=np.float64)
    da = np.asarray(dl, dtype=np.float64)
    qo, do, w = np.zeros(3), np.zeros(3), np.zeros(1)
    ok = lib.mxo_lens_debug(ctypes.addressof(ins.arr[0]), _ptr(qa), _ptr(da), float(E), _ptr(qo), _ptr(do), _ptr(w))
    return bool(ok), qo, do, float(w[0])


def kn_f(k: float) -> float:
    """Klein-Nishina total cross section over 2 pi r_e^2 at k = E / m_e c^2."""
    return _load().mxo_kn_f(float(k))


def ppnd16(p: float) -> float:
    """Standard normal quantile (Wichura's AS 241)."""
    return _load().mxo_ppnd16(float(p))


def truncnorm(za: float, zb: float, U: float) -> float:
    """Standard normal truncated to [za, zb] by inversion at U."""
    return _load().mxo_truncnorm(float(za), float(zb), float(U))


def proposal_density(source: Dict, gmm, alpha: float, u: float, v: float, E: float):
    """(q, p): the proposal mixture density and the physical source density
    at y = (u, v, E) for a cone-beam source."""
    ins = Instrument({"components": [source]})
    g, gp = _gmm(gmm)
    pp = np.zeros(1)
    q = _load().mxo_proposal_density(ctypes.addressof(ins.arr[0].par), gp, float(alpha), float(u), float(v),
                                     float(E), _ptr(pp))
    return q, float(pp[0])


def proposal_bounds(source: Dict, gmm, alpha: float, n_total: int) -> np.ndarray:
    """The 9 branch boundaries of an n_total-ray proposal run."""
    ins = Instrument({"components": [source]})
    g, gp = _gmm(gmm)
    B = np.zeros(9, np.uint64)
    _load().mxo_proposal_bounds(ctypes.addressof(ins.arr[0].par), gp, float(alpha), int(n_total), _ptr(B))
    return B


def proposal_weight(source: Dict, gmm, alpha: float, n_total: int, y: np.ndarray) -> np.ndarray:
    """p(y) / q(y) of proposal draws y (m x 3: u, v, E) in an n_total-ray run
    (without the stratification cell factor)."""
    lib = _load()
    ins = Instrument({"components": [source]})
    g, gp = _gmm(gmm)
    par = ctypes.addressof(ins.arr[0].par)
    y = np.asarray(y, dtype=np.float64).reshape(-1, 3)
    return np.array([lib.mxo_proposal_weight(par, gp, float(alpha), int(n_total), *row) for row in y])


def trace_after_source(instr: Dict, ids, seed: int, n_total: int, r, d, E, w, purpose: int = 0, job: int = 0):
    """Final states of rays continued from the given states after the source
    (r, d: m x 3; E, w: m) through the rest of the instrument."""
    lib = _load()
    ins = Instrument(instr)
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    n = ids.size
    c = lambda a, shape: np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
    r_in, d_in, E_in, w_in = c(r, (n, 3)), c(d, (n, 3)), c(E, (n,)), c(w, (n,))
    out = {
        "r": np.zeros((n, 3)), "d": np.zeros((n, 3)), "E": np.zeros(n), "w": np.zeros(n),
        "status": np.zeros(n, np.int32), "dead_at": np.zeros(n, np.int32), "bin": np.zeros(n, np.int64),
    }
    lib.mxo_trace_after_source(ctypes.addressof(ins.arr), ins.n, seed, n_total, purpose, job, _ptr(ids), n,
                               _ptr(r_in), _ptr(d_in), _ptr(E_in), _ptr(w_in), _ptr(out["r"]), _ptr(out["d"]),
                               _ptr(out["E"]), _ptr(out["w"]), _ptr(out["status"]), _ptr(out["dead_at"]),
                               _ptr(out["bin"]))
    return out
