"""Error metric of a projection image: which bins carry signal, the 95th
percentile of their relative errors, and the time a run needs to bring it to
1 %.

Host-side FP64 arithmetic on a few arrays per measurement (no part of the
tracing).  The per-bin relative errors themselves come from the library's
batch-means kernel (``batch_means``).

* Flat field: with an empty phantom every ray carries its source weight, so a
  bin's intensity per emitted ray is Omega_pixel / Omega_cone times the
  spectrum's mass in the bin's energy range (point source, plane detector
  normal to the axis: Omega of a pixel [x0, x1] x [y0, y1] at distance D is
  F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0), F = atan(x y / (D r))).
* Signal bins: I_ref / I_flat >= 1e-3, I_ref a high-statistics image: bins
  the object does not darken by more than a factor 1000.
* "1 % per bin": q95 over the signal bins of the relative error <= 0.01.  A
  run of N rays that reaches q95 takes t_per_ray N (q95 / 0.01)^2 to reach
  1 % (the error falls as N^-1/2).
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np


def spectrum_mass(src: Dict, e1: np.ndarray, e2: np.ndarray) -> np.ndarray:
    """Mass of the tube spectrum in [e1, e2): Kramers continuum
    (E0 - E)/E normalised on [emin, emax], plus two Gaussian lines."""
    from math import erf, sqrt
    K = src["e0"] * math.log(src["emax"] / src["emin"]) - (src["emax"] - src["emin"])
    cont = src["f_cont"] * (src["e0"] * np.log(e2 / e1) - (e2 - e1)) / K
    Phi = np.vectorize(lambda z: 0.5 * (1.0 + erf(z / sqrt(2.0))))
    s = src["line_sigma"]
    l1 = src["f_line1"] * (Phi((e2 - src["e_line1"]) / s) - Phi((e1 - src["e_line1"]) / s))
    l2 = src["f_line2"] * (Phi((e2 - src["e_line2"]) / s) - Phi((e1 - src["e_line2"]) / s))
    return cont + l1 + l2


def flat_field(instr: Dict) -> np.ndarray:
    """Per-bin intensity per emitted ray of the projection instrument with an
    empty phantom, flat bin order (iy * nx + ix) * ne + ie."""
    src = instr["components"][0]
    det = instr["components"][-1]
    D = float(det["pos"][2]) - float(src["pos"][2])
    xe = np.linspace(det["xmin"], det["xmax"], det["nx"] + 1)
    ye = np.linspace(det["ymin"], det["ymax"], det["ny"] + 1)
    X, Y = np.meshgrid(xe, ye)
    F = np.arctan(X * Y / (D * np.sqrt(D * D + X * X + Y * Y)))
    om = F[1:, 1:] - F[:-1, 1:] - F[1:, :-1] + F[:-1, :-1]
    cone = 4.0 * math.pi * math.sin(src["half_angle"] / 2.0) ** 2
    edges = np.linspace(det["emin"], det["emax"], det["ne"] + 1)
    spec = spectrum_mass(src, edges[:-1], edges[1:])
    return (om[:, :, None] / cone * spec[None, None, :]).reshape(-1)


def signal_bins(I_ref: np.ndarray, I_flat: np.ndarray, threshold: float = 1e-3) -> np.ndarray:
    return (I_flat > 0) & (I_ref >= threshold * I_flat)


def q95(rel: np.ndarray, mask: np.ndarray) -> float:
    return float(np.percentile(rel[mask], 95.0))


def time_to_1pct(t_per_ray: float, n_rays: float, q: float) -> float:
    return t_per_ray * n_rays * (q / 0.01) ** 2
