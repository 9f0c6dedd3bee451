"""Pins of the learned-proposal oracle against what mathematics fixes:
library quantiles and truncated normals, densities that integrate to one,
the importance-sampling identity E_q[p/q] = 1, unbiased detector images,
finite differences of the loss, closed forms of the network and head, the
network's layers against torch's linear and SiLU layers at random weights,
and Adam against torch's optimizer over several steps.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle
import workloads
from oracle import proposal as P


def cone_source():
    return workloads.edct_projection(workloads.make_phantom(64, 1), workloads.make_mu_tables(1))["components"][0]


def synthetic_gmm(seed, source, sigma_scale=(0.15, 0.8)):
    """A valid 56-number mixture table inside the source's box."""
    rng = np.random.default_rng(seed)
    lo, hi = P.box_of(source)
    pi = rng.dirichlet(np.ones(8))
    mu = lo + (hi - lo) * rng.uniform(0.1, 0.9, size=(8, 3))
    sigma = 0.5 * (hi - lo) * rng.uniform(*sigma_scale, size=(8, 3))
    return np.concatenate([pi[:, None], mu, sigma], axis=1).reshape(56)


# ------------------------------------------------------------ sampler ----

def test_ppnd16_matches_library_quantile():
    ps = np.concatenate([np.logspace(-300, -1, 300), np.linspace(0.01, 0.99, 300), 1 - np.logspace(-16, -1, 80)])
    for p in ps:
        ref = special.ndtri(p)
        assert abs(oracle.ppnd16(p) - ref) <= 2e-15 * max(1.0, abs(ref)), p


@pytest.mark.parametrize("za,zb", [(-1.0, 2.0), (0.5, 3.0), (-4.0, -3.5), (5.0, 9.0), (-30.0, -29.0),
                                   (-0.01, 0.02), (-8.0, 8.0), (2.0, 2.0 + 1e-6)])
def test_truncnorm_matches_library(za, zb):
    for U in (1e-12, 0.01, 0.3, 0.5, 0.77, 0.999, 1 - 1e-12):
        got = oracle.truncnorm(za, zb, U)
        ref = stats.truncnorm.ppf(U, za, zb)
        assert za - 1e-12 <= got <= zb + 1e-12
        # scipy's own accuracy in the far tails is the limiting factor
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref)), (za, zb, U, got, ref)


def gl(n, a, b):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (a + b), 0.5 * (b - a) * w


def test_proposal_density_integrates_to_one():
    """alpha = 0: the truncated mixture over its box (Gauss-Legendre, the
    integrand is smooth there); alpha = 1: the plain density over the cone
    (polar Gauss-Legendre); and q is affine in alpha pointwise."""
    src = cone_source()
    gmm = synthetic_gmm(3, src)
    t = math.tan(src["half_angle"])
    us, wu = gl(40, -t, t)
    Es, wE = gl(24, src["emin"], src["emax"])
    total = 0.0
    for u, a in zip(us, wu):
        for v, b in zip(us, wu):
            for E, c in zip(Es, wE):
                total += a * b * c * oracle.proposal_density(src, gmm, 0.0, u, v, E)[0]
    assert abs(total - 1.0) < 1e-9, total
    rs, wr = gl(24, 0.0, t)
    ps, wp = gl(24, 0.0, 2 * math.pi)
    total = 0.0
    for r, a in zip(rs, wr):
        for ph, b in zip(ps, wp):
            q = oracle.proposal_density(src, gmm, 1.0, r * math.cos(ph), r * math.sin(ph), 85.0)[0]
            total += a * b * r * q * (src["emax"] - src["emin"])
    assert abs(total - 1.0) < 1e-9, total
    rng = np.random.default_rng(4)
    for _ in range(50):
        u, v, E = rng.uniform(-t, t), rng.uniform(-t, t), rng.uniform(20, 150)
        q0 = oracle.proposal_density(src, gmm, 0.0, u, v, E)[0]
        q1 = oracle.proposal_density(src, gmm, 1.0, u, v, E)[0]
        qa = oracle.proposal_density(src, gmm, 0.1, u, v, E)[0]
        assert abs(qa - (0.1 * q1 + 0.9 * q0)) <= 1e-14 * max(q0, q1)


def source_only(src):
    return {"components": [src]}


@pytest.mark.parametrize("alpha", [0.1, 0.5])
def test_importance_weights_have_unit_mean(alpha):
    """E_q[p/q] = integral of p = 1; and for an energy band, E_q[w 1_band] =
    the band's share of the spectrum (closed form)."""
    src = cone_source()
    gmm = synthetic_gmm(5, src)
    n = 400000
    o = oracle.trace_rays(source_only(src), np.arange(n), seed=9, n_total=n, gmm=gmm, alpha=alpha)
    w = o["w"]
    z = (w.mean() - 1.0) / (w.std() / math.sqrt(n))
    assert abs(z) < 5.0, z
    # band [40, 60) keV: continuum (E0 - E)/E / K plus the 59.3 keV line
    lo_e, hi_e = 40.0, 60.0
    E0, emin, emax = src["e0"], src["emin"], src["emax"]
    K = E0 * math.log(emax / emin) - (emax - emin)
    share = src["f_cont"] * (E0 * math.log(hi_e / lo_e) - (hi_e - lo_e)) / K
    share += src["f_line1"] * (stats.norm.cdf(hi_e, src["e_line1"], src["line_sigma"]) -
                               stats.norm.cdf(lo_e, src["e_line1"], src["line_sigma"]))
    band = (o["E"] >= lo_e) & (o["E"] < hi_e)
    x = w * band
    zb = (x.mean() - share) / (x.std() / math.sqrt(n))
    assert abs(zb) < 5.0, (x.mean(), share, zb)
    # draws outside the cone are killed at the source with weight 0
    dead = o["status"] == oracle.STATUS_ABSORBED
    assert np.all(w[dead] == 0.0) and np.all(o["dead_at"][dead] == 0)
    d = o["d"][~dead]
    assert np.all(d[:, 0] ** 2 + d[:, 1] ** 2 <= (math.sin(src["half_angle"]) ** 2) * (1 + 1e-12))


def test_gmm_branch_follows_truncated_normal():
    """alpha = 0 and one component carrying all the mass: u is a truncated
    normal (Kolmogorov-Smirnov against scipy)."""
    src = cone_source()
    lo, hi = P.box_of(src)
    gmm = np.zeros((8, 7))
    gmm[:, 0] = 1e-300
    gmm[:, 1:4] = 0.5 * (lo + hi)
    gmm[:, 4:7] = 0.5 * (hi - lo)
    gmm[2] = [1.0, 0.05, -0.02, 70.0, 0.04, 0.03, 20.0]
    n = 20000
    o = oracle.trace_rays(source_only(src), np.arange(n), seed=2, n_total=n, gmm=gmm.reshape(56), alpha=0.0)
    u = o["d"][:, 0] / o["d"][:, 2]
    a, b = (lo[0] - 0.05) / 0.04, (hi[0] - 0.05) / 0.04
    assert stats.kstest(u, stats.truncnorm(a, b, loc=0.05, scale=0.04).cdf).pvalue > 1e-4
    E = o["E"]
    a, b = (lo[2] - 70.0) / 20.0, (hi[2] - 70.0) / 20.0
    assert stats.kstest(E, stats.truncnorm(a, b, loc=70.0, scale=20.0).cdf).pvalue > 1e-4


def test_proposal_images_are_unbiased():
    """Per-energy-bin detector sums with the proposal agree with the plain
    source within their statistical errors."""
    vol = workloads.make_phantom(64, 1)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), strata=1, nx=32, ny=16, ne=16)
    src = ins["components"][0]
    lo, hi = P.box_of(src)
    # a mixture concentrated on the detector's angular rectangle
    gmm = np.zeros((8, 7))
    for k in range(8):
        gmm[k] = [1 / 8, -0.015 + 0.03 * (k + 0.5) / 8, 0.0, 20 + 130 * (k + 0.5) / 8, 0.006, 0.006, 20.0]
    n = 400000
    plain = oracle.run(ins, n, seed=4)[0]
    prop = oracle.run(ins, n, seed=4, gmm=gmm.reshape(56), alpha=0.1)[0]

    def per_e(t):
        s = t["sum_w"].reshape(16, 32, 16).sum(axis=(0, 1))
        s2 = t["sum_w2"].reshape(16, 32, 16).sum(axis=(0, 1))
        return s / n, np.sqrt(np.maximum(s2 / n - (s / n) ** 2, 0) / n)

    m0, e0 = per_e(plain)
    m1, e1 = per_e(prop)
    z = (m1 - m0) / np.sqrt(e0 ** 2 + e1 ** 2)
    assert np.all(np.abs(z) < 5.0), z
    # and the proposal aims: more detector hits per emitted ray (a plain ray
    # hits this detector with probability ~0.51)
    assert prop["count"].sum() > 1.3 * plain["count"].sum()


# ------------------------------------------------------------ network ----

def box():
    return P.box_of(cone_source())


def test_param_count():
    assert P.N_PARAMS == 24632


def test_zero_weights_closed_form():
    lo, hi = box()
    parts = {name: np.zeros(shape) for name, shape in P.SHAPES}
    parts["b3"] = np.linspace(-1, 1, 56)
    theta = P.pack(parts)
    C = np.random.default_rng(0).normal(size=(5, 6))
    f = P.forward(theta, C)
    assert np.array_equal(f["o"], np.tile(parts["b3"], (5, 1)))
    h = P.head(f["o"], lo, hi)
    logits = parts["b3"].reshape(8, 7)[:, 0]
    assert np.allclose(h["pi"][0], np.exp(logits) / np.exp(logits).sum(), rtol=1e-15, atol=0)
    raw = parts["b3"].reshape(8, 7)
    assert np.allclose(h["mu"][0], 0.5 * (lo + hi) + 0.5 * (hi - lo) * np.tanh(raw[:, 1:4]), rtol=1e-15)
    assert np.allclose(h["sigma"][0], 0.5 * (hi - lo) * (1e-3 + np.log1p(np.exp(raw[:, 4:7]))), rtol=1e-14)


def test_log_q_single_component_wide_box():
    """One component carrying all the mass, far inside a wide box: log q is
    the product of three normal log-densities."""
    lo, hi = np.array([-1e3, -1e3, -1e3]), np.array([1e3, 1e3, 1e3])
    h = {"pi": np.array([[1.0] + [0.0] * 7]), "mu": np.zeros((1, 8, 3)), "sigma": np.ones((1, 8, 3))}
    h["mu"][0, 0] = [0.1, -0.3, 2.0]
    h["sigma"][0, 0] = [0.5, 1.5, 0.7]
    with np.errstate(divide="ignore"):
        y = np.array([[0.2, 0.4, 1.0]])
        got = P.log_q_gmm(y, h, lo, hi)[0]
    ref = sum(stats.norm.logpdf(y[0, d], h["mu"][0, 0, d], h["sigma"][0, 0, d]) for d in range(3))
    assert abs(got - ref) < 1e-13


def test_truncation_mass_matches_library():
    src = cone_source()
    lo, hi = P.box_of(src)
    g = synthetic_gmm(7, src).reshape(8, 7)
    y = np.array([[0.01, -0.02, 80.0]])
    h = {"pi": g[None, :, 0], "mu": g[None, :, 1:4], "sigma": g[None, :, 4:7]}
    Z = np.prod([stats.norm.cdf(hi[d], g[:, 1 + d], g[:, 4 + d]) - stats.norm.cdf(lo[d], g[:, 1 + d], g[:, 4 + d])
                 for d in range(3)], axis=0)
    dens = np.sum(g[:, 0] * np.prod([stats.norm.pdf(y[0, d], g[:, 1 + d], g[:, 4 + d]) for d in range(3)], axis=0))
    ref = math.log(dens / np.sum(g[:, 0] * Z))
    assert abs(P.log_q_gmm(y, h, lo, hi)[0] - ref) < 1e-12
    # the C sampler's density agrees with the numpy one (alpha = 0)
    q, _ = oracle.proposal_density(src, g.reshape(56), 0.0, *y[0])
    assert abs(math.log(q) - ref) < 1e-12


def fd_setup(seed=1, n=7):
    rng = np.random.default_rng(seed)
    lo, hi = box()
    theta = P.init_params(seed) + 0.05 * rng.normal(size=P.N_PARAMS)  # biases non-zero too
    C = rng.normal(size=(n, 6))
    Y = np.stack([rng.uniform(lo[0], hi[0], n), rng.uniform(lo[1], hi[1], n), rng.uniform(lo[2], hi[2], n)], 1)
    omega = rng.uniform(0.1, 2.0, n)
    return theta, C, Y, omega, lo, hi


def test_gradient_matches_finite_differences():
    theta, C, Y, omega, lo, hi = fd_setup()
    L, g, _ = P.loss_grad(theta, C, Y, omega, lo, hi)
    assert abs(L - P.loss(theta, C, Y, omega, lo, hi)) < 1e-12 * abs(L)
    rng = np.random.default_rng(2)
    offsets, k = {}, 0
    for name, shape in P.SHAPES:
        offsets[name] = (k, int(np.prod(shape)))
        k += int(np.prod(shape))
    for name, (k0, n) in offsets.items():
        for idx in rng.choice(n, size=min(n, 12), replace=False):
            i = k0 + idx
            h = 1e-6 * max(1.0, abs(theta[i]))
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            fd = (P.loss(tp, C, Y, omega, lo, hi) - P.loss(tm, C, Y, omega, lo, hi)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3), (name, idx, fd, g[i])


def test_forward_matches_torch_layers():
    """The hidden path at random non-zero weights against torch's own
    linear and SiLU layers in float64.  The parameters are unpacked here from
    the packing the C ABI documents (W1 6 x 128 row-major, b1, W2 128 x 128,
    b2, W3 128 x 56, b3), so a wrong layer order, activation or packing in
    the oracle fails."""
    import torch
    rng = np.random.default_rng(11)
    theta = rng.normal(scale=0.4, size=P.N_PARAMS)
    C = rng.normal(scale=1.5, size=(33, 6))
    sizes = [(6, 128), (128,), (128, 128), (128,), (128, 56), (56,)]
    parts, k = [], 0
    for shp in sizes:
        n = int(np.prod(shp))
        parts.append(torch.from_numpy(theta[k:k + n].reshape(shp).copy()))
        k += n
    assert k == P.N_PARAMS
    W1, b1, W2, b2, W3, b3 = parts
    F = torch.nn.functional
    x = torch.from_numpy(C)
    z1 = F.linear(x, W1.T.contiguous(), b1)
    z2 = F.linear(F.silu(z1), W2.T.contiguous(), b2)
    o = F.linear(F.silu(z2), W3.T.contiguous(), b3)
    f = P.forward(theta, C)
    for name, ref in (("z1", z1), ("z2", z2), ("o", o)):
        ref = ref.numpy()
        assert np.max(np.abs(f[name] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), name
    assert np.max(np.abs(f["h1"] - F.silu(z1).numpy())) <= 1e-13 * max(1.0, float(z1.abs().max()))
    # the hidden layers matter at these weights: the output is far from b3
    assert np.max(np.abs(f["o"] - theta[-56:])) > 1.0


def test_adam_matches_torch_optimizer():
    """Twelve Adam steps with gradients that change size and sign, against
    torch.optim.Adam in float64 (same lr, betas, eps); a wrong bias
    correction (1 - b2 for 1 - b2^t, say) or moment update fails at step 2."""
    import torch
    rng = np.random.default_rng(5)
    n = 257
    theta = rng.normal(size=n)
    m, v = np.zeros(n), np.zeros(n)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=2e-3, betas=(0.85, 0.995), eps=1e-7)
    for step in range(1, 13):
        g = rng.normal(size=n) * 10.0 ** rng.integers(-4, 3, n)
        theta, m, v = P.adam(theta, m, v, g, step, lr=2e-3, b1=0.85, b2=0.995, eps=1e-7)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        ref = p.detach().numpy()
        assert np.max(np.abs(theta - ref)) <= 1e-13, step


def test_adam_first_step_is_sign_step():
    """After one step from zero moments, Adam moves each parameter by lr
    times the sign of its gradient (up to eps)."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    th, m, v = P.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), rtol=1e-15)


def test_bf16_rounding_matches_torch():
    import torch
    x = np.random.default_rng(0).normal(size=10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(-8, 8, 10000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(P.bf16_round(x), ref)


def test_gemm_bound_holds_for_float32_accumulation():
    rng = np.random.default_rng(3)
    A = P.bf16_round(rng.normal(size=(64, 128)))
    B = P.bf16_round(rng.normal(size=(128, 32)))
    exact, bound = P.gemm_bound(A, B)
    acc = np.zeros((64, 32), np.float32)
    for k in range(128):
        acc = (acc + (A[:, k:k + 1] * B[k:k + 1, :]).astype(np.float32)).astype(np.float32)
    assert np.all(np.abs(acc - exact) <= bound)


def test_branch_sizes_follow_the_masses():
    src = cone_source()
    gmm = synthetic_gmm(11, src)
    lo, hi = P.box_of(src)
    g = gmm.reshape(8, 7)
    Z = g[:, 0] * np.prod([stats.norm.cdf(hi[d], g[:, 1 + d], g[:, 4 + d]) - stats.norm.cdf(lo[d], g[:, 1 + d], g[:, 4 + d])
                           for d in range(3)], axis=0)
    for N, alpha in ((10**9, 0.1), (12345, 0.3), (7, 0.5), (1000, 0.0), (1000, 1.0)):
        B = oracle.proposal_bounds(src, gmm, alpha, N).astype(np.int64)
        assert B[0] == int(np.floor(alpha * N + 0.5)) and B[8] == N
        assert np.all(np.diff(B) >= 0)
        want = (N - B[0]) * Z / Z.sum()
        assert np.all(np.abs(np.diff(B) - want) <= 1.0 + 1e-9 * N)


def test_all_plain_split_is_the_plain_source():
    """alpha = 1: every ray takes the plain branch with the plain source's
    strata, uniforms and weight 130 S(E) x cell factor, so the rays equal
    the plain stratified source's, ray by ray."""
    ins = workloads.edct_projection(workloads.make_phantom(64, 1), workloads.make_mu_tables(1), strata=64)
    gmm = synthetic_gmm(12, ins["components"][0])
    n = 20011
    ids = np.arange(n)
    a = oracle.trace_rays(ins, ids, seed=3, n_total=n, gmm=gmm, alpha=1.0)
    b = oracle.trace_rays(ins, ids, seed=3, n_total=n)
    assert np.array_equal(a["status"], b["status"]) and np.array_equal(a["bin"], b["bin"])
    for k in ("d", "E", "w", "r"):
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-12), k


def test_continuing_after_the_source_reproduces_the_trace():
    """The oracle's continuation from a given post-source state, fed its own
    source states, reproduces its full traces bit for bit."""
    ins = workloads.edct_projection(workloads.make_phantom(64, 1), workloads.make_mu_tables(1), strata=16)
    src = ins["components"][0]
    gmm = synthetic_gmm(13, src)
    ids = np.arange(3000)
    full = oracle.trace_rays(ins, ids, seed=5, n_total=3000, job=3, gmm=gmm, alpha=0.1)
    s0 = oracle.trace_rays({"components": [src]}, ids, seed=5, n_total=3000, job=3, gmm=gmm, alpha=0.1)
    live = s0["status"] != oracle.STATUS_ABSORBED
    c = oracle.trace_after_source(ins, ids[live], 5, 3000, s0["r"][live], s0["d"][live], s0["E"][live],
                                  s0["w"][live], job=3)
    for k in ("r", "d", "E", "w", "status", "dead_at", "bin"):
        assert np.array_equal(c[k], full[k][live]), k
    # and the weight function times the stratum factor is the source weight
    y = np.stack([s0["d"][:, 0] / s0["d"][:, 2], s0["d"][:, 1] / s0["d"][:, 2], s0["E"]], 1)[live]
    W = oracle.proposal_weight(src, gmm, 0.1, 3000, y)
    f = s0["w"][live] / W
    assert np.all(f > 0.2) and np.all(f < 5.0)
