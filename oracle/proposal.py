"""Learned-proposal oracle: FP64 MLP, mixture head, truncated-mixture
density, weighted negative log-likelihood and its gradient, Adam.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): tests, the smoke
check and the benchmark's CPU baseline may call it; the product path never
does.  Plain numpy in float64, written from the definitions, no blocking or
fusion.

The proposal learns where the plain cone-beam source should send its rays.
The paper's method traces every ray from a physical source (sections 2-3);
importance sampling keeps the estimator unbiased when rays are drawn from
another density q instead, by weighting each ray with p/q (the Monte Carlo
weight of section 2.2.2 carries exactly this factor).  Here q is a defensive
mixture (Hesterberg 1995) of the plain source and an 8-component diagonal
Gaussian mixture over y = (u, v, E), u = dx/dz, v = dy/dz, truncated to the
box [-t, t]^2 x [emin, emax] (t = tan of the cone half-angle), whose
parameters a small MLP computes from a 6-number context c (focal-spot
position, projection angle as cos/sin, phantom size).

Network (parameters packed in this order, float32 master copy, bfloat16
working copy)::

    W1 (6 x 128), b1 (128), W2 (128 x 128), b2 (128), W3 (128 x 56), b3 (56)
    z1 = c W1 + b1,  h1 = silu(z1),  z2 = h1 W2 + b2,  h2 = silu(z2),
    o = h2 W3 + b3,  silu(z) = z / (1 + exp(-z))

Head: component k reads o[7k] (logit), o[7k+1..7k+3] (mean, raw) and
o[7k+4..7k+6] (width, raw): pi = softmax(logits), mu_d = centre_d + half_d
tanh(raw), sigma_d = half_d (1e-3 + softplus(raw)), half_d the box
half-width.  Loss over a batch: L = -sum_i omega_i log q_gmm(y_i | c_i) /
sum_i omega_i, with log q_gmm = logsumexp_k(log pi_k + sum_d log N(y_d;
mu_kd, sigma_kd)) - log sum_k pi_k Z_k and Z_k the box mass of component k.

Parity pins (tests/test_oracle_proposal.py): central finite differences of
the loss for every parameter block; closed forms at zero weights; the
single-component, wide-box limit against scipy's normal log-density;
Z_k against scipy's normal distribution function.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

N_IN, N_HID, N_OUT, N_COMP = 6, 128, 56, 8
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 24632
SIGMA_FLOOR = 1e-3


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape)
        k += n
    return out


def pack(parts: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float64 holding the exact bfloat16 value."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def box_of(source: Dict) -> Tuple[np.ndarray, np.ndarray]:
    """(lo, hi) of the truncation box of a cone-beam source."""
    t = math.tan(source["half_angle"])
    return np.array([-t, -t, source["emin"]]), np.array([t, t, source["emax"]])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta: np.ndarray, C: np.ndarray) -> Dict[str, np.ndarray]:
    """Layer values for contexts C (n x 6), in float64."""
    P = unpack(theta)
    z1 = C @ P["W1"] + P["b1"]
    h1 = silu(z1)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = silu(z2)
    o = h2 @ P["W3"] + P["b3"]
    return {"z1": z1, "h1": h1, "z2": z2, "h2": h2, "o": o}


def softplus(x):
    return np.logaddexp(0.0, x)


def head(o: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> Dict[str, np.ndarray]:
    """Mixture parameters from the network output o (n x 56)."""
    o = o.reshape(-1, N_COMP, 7)
    centre, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    logits = o[:, :, 0]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    pi = e / e.sum(axis=1, keepdims=True)
    mu = centre + half * np.tanh(o[:, :, 1:4])
    sigma = half * (SIGMA_FLOOR + softplus(o[:, :, 4:7]))
    return {"pi": pi, "mu": mu, "sigma": sigma}


def gmm_table(h: Dict[str, np.ndarray], row: int = 0) -> np.ndarray:
    """The tracer's 56-number table (pi, mu_u, mu_v, mu_E, sigma_u, sigma_v,
    sigma_E per component) of one row."""
    return np.concatenate([h["pi"][row][:, None], h["mu"][row], h["sigma"][row]], axis=1).reshape(56)


def norm_cdf(z):
    from scipy.special import ndtr  # the standard normal distribution function
    return ndtr(z)


def log_q_gmm(y: np.ndarray, h: Dict[str, np.ndarray], lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """log of the truncated mixture density at y (n x 3)."""
    z = (y[:, None, :] - h["mu"]) / h["sigma"]
    comp = np.log(h["pi"]) + np.sum(-0.5 * z * z - np.log(h["sigma"]) - 0.5 * math.log(2 * math.pi), axis=2)
    m = comp.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(comp - m).sum(axis=1))
    za = (lo - h["mu"]) / h["sigma"]
    zb = (hi - h["mu"]) / h["sigma"]
    Z = np.prod(norm_cdf(zb) - norm_cdf(za), axis=2)
    return lse - np.log(np.sum(h["pi"] * Z, axis=1))


def loss(theta, C, Y, omega, lo, hi) -> float:
    h = head(forward(theta, C)["o"], lo, hi)
    return float(-np.sum(omega * log_q_gmm(Y, h, lo, hi)) / np.sum(omega))


def head_grad(o: np.ndarray, Y: np.ndarray, omega: np.ndarray, lo, hi) -> Tuple[float, np.ndarray]:
    """Loss and dL/do (n x 56) by the chain rule through the head."""
    n = o.shape[0]
    O = o.reshape(n, N_COMP, 7)
    h = head(o, lo, hi)
    pi, mu, sigma = h["pi"], h["mu"], h["sigma"]
    W = np.sum(omega)
    a = omega / W  # dL/d(-log q_i)
    z = (Y[:, None, :] - mu) / sigma
    comp = np.log(pi) + np.sum(-0.5 * z * z - np.log(sigma) - 0.5 * math.log(2 * math.pi), axis=2)
    m = comp.max(axis=1, keepdims=True)
    r = np.exp(comp - m)
    r = r / r.sum(axis=1, keepdims=True)  # responsibilities
    za = (lo - mu) / sigma
    zb = (hi - mu) / sigma
    Fd = norm_cdf(zb) - norm_cdf(za)  # per dimension box mass
    Z = np.prod(Fd, axis=2)
    S = np.sum(pi * Z, axis=1)
    s = pi * Z / S[:, None]  # share of the normaliser
    phi = lambda x: np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)
    # -log q = -lse + log S
    # d(-lse)/d mu = -r z / sigma ; d(-lse)/d sigma = -r (z^2 - 1) / sigma
    # d(log S)/d mu_kd = s_k (d Fd/d mu) / Fd ; dFd/dmu = -(phi(zb) - phi(za)) / sigma
    # dFd/dsigma = -(zb phi(zb) - za phi(za)) / sigma
    dFd_mu = -(phi(zb) - phi(za)) / sigma
    dFd_sig = -(zb * phi(zb) - za * phi(za)) / sigma
    g_mu = -r[:, :, None] * z / sigma + s[:, :, None] * dFd_mu / Fd
    g_sig = -r[:, :, None] * (z * z - 1.0) / sigma + s[:, :, None] * dFd_sig / Fd
    # logits: d(-lse)/dlogit_j = -(r_j - pi_j); d(log S)/dlogit_j = s_j - pi_j
    g_logit = -(r - pi) + (s - pi)
    half = 0.5 * (hi - lo)
    g_mu_raw = g_mu * half * (1.0 - np.tanh(O[:, :, 1:4]) ** 2)
    g_sig_raw = g_sig * half / (1.0 + np.exp(-O[:, :, 4:7]))
    G = np.zeros_like(O)
    G[:, :, 0] = g_logit
    G[:, :, 1:4] = g_mu_raw
    G[:, :, 4:7] = g_sig_raw
    G *= a[:, None, None]
    L = float(-np.sum(a * log_q_gmm(Y, h, lo, hi)))
    return L, G.reshape(n, N_OUT)


def loss_grad(theta, C, Y, omega, lo, hi) -> Tuple[float, np.ndarray, Dict[str, np.ndarray]]:
    """Loss, dL/dtheta (packed like theta) and the backward intermediates."""
    P = unpack(theta)
    f = forward(theta, C)
    L, dO = head_grad(f["o"], Y, omega, lo, hi)
    g = {"W3": f["h2"].T @ dO, "b3": dO.sum(axis=0)}
    dH2 = dO @ P["W3"].T
    dZ2 = dH2 * silu_grad(f["z2"])
    g["W2"] = f["h1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2 @ P["W2"].T
    dZ1 = dH1 * silu_grad(f["z1"])
    g["W1"] = C.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return L, pack(g), {"dO": dO, "dZ2": dZ2, "dZ1": dZ1, **f}


def adam(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015), bias-corrected; step >= 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """The seeded initial parameters (shared input generator), as float64."""
    import workloads
    return workloads.init_mlp_params(seed).astype(np.float64)


def gemm_bound(A: np.ndarray, B: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Exact product A B (float64 of bfloat16 operands: every product and a
    sum of at most a few hundred of them is exact to ~1e-16) and Higham's
    bound gamma_K sum |a||b| on a float32 accumulation of it (K = inner
    size, gamma_K = K u / (1 - K u), u = 2^-24)."""
    K = A.shape[1]
    u = 2.0 ** -24
    gamma = K * u / (1.0 - K * u)
    return A @ B, gamma * (np.abs(A) @ np.abs(B))
