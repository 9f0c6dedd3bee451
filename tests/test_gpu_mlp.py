"""The proposal network's HIP kernels against the FP64 oracle, layer by layer.

Every product is checked on the GPU's own bfloat16 operands (read back from
the workspace) against the exact product, within Higham's bound for a
float32 accumulation, |s_hat - s| <= gamma_K sum |a_i b_i| (gamma_K =
K u / (1 - K u), u = 2^-24; one more term for a bias add or a split
reduction).  Elementwise steps are checked against FP64 evaluations of the
same float32 inputs.  The full gradient is compared with the oracle's FP64
gradient at the same weights and inputs, and training must lower the loss.
"""
import numpy as np
import pytest

import workloads
from oracle import proposal as P

from test_gpu_parity import announce

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def gamma(K):
    return K * U / (1 - K * U)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def mxr():
    import paper_2410_08747_amd as m
    return m


def box():
    src = workloads.edct_projection(workloads.make_phantom(64, 1), workloads.make_mu_tables(1))["components"][0]
    return P.box_of(src)


def params(seed=1):
    rng = np.random.default_rng(seed)
    theta = P.init_params(seed) + 0.05 * rng.normal(size=P.N_PARAMS)
    return theta.astype(np.float32)


def data(n, seed=2):
    rng = np.random.default_rng(seed)
    lo, hi = box()
    ctx = rng.normal(size=(n, 6)).astype(np.float32)
    y = np.stack([rng.uniform(lo[d], hi[d], n) for d in range(3)], 1)
    omega = rng.uniform(0.1, 2.0, n)
    return ctx, y, omega


def f64(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def check_product(got, A, B, bias, label, extra=0):
    exact, bound = P.gemm_bound(A, B)
    K = A.shape[1] + extra
    bnd = gamma(K + 1) * (np.abs(A) @ np.abs(B) + (np.abs(bias) if bias is not None else 0.0))
    ref = exact + (bias if bias is not None else 0.0)
    err = np.abs(got - ref)
    bad = err > bnd + 1e-45
    assert not bad.any(), f"{label}: {bad.sum()} entries beyond the bound, worst {np.max(err - bnd):.3e}"


def test_forward_layers(torch_cuda):
    m = mxr()
    n = 1000  # not a multiple of the 16 x 64 tiles
    announce("mlp forward layers n", n)
    theta = params()
    net = m.ProposalNet(theta, batch=n)
    ctx, _, _ = data(n)
    out = net.forward(torch_cuda.tensor(ctx, device="cuda"))
    torch_cuda.cuda.synchronize()
    import torch
    W = P.unpack(f64(net.w))
    assert np.array_equal(f64(net.w), P.bf16_round(theta))  # working copy = bf16 of the master
    X = f64(net.region("X", n, torch.bfloat16, 6))
    assert np.array_equal(X, P.bf16_round(ctx))
    Z1 = f64(net.region("Z1", n, torch.float32, 128))
    H1 = f64(net.region("H1", n, torch.bfloat16, 128))
    Z2 = f64(net.region("Z2", n, torch.float32, 128))
    H2 = f64(net.region("H2", n, torch.bfloat16, 128))
    O = f64(out)
    assert np.array_equal(O, f64(net.region("O", n, torch.float32, 56)))
    check_product(Z1, X, W["W1"], W["b1"], "layer 1")
    check_product(Z2, H1, W["W2"], W["b2"], "layer 2")
    check_product(O, H2, W["W3"], W["b3"], "layer 3")
    # activations: bf16 of a float32 silu of the GPU's own pre-activations
    for Z, H, name in ((Z1, H1, "h1"), (Z2, H2, "h2")):
        s = P.silu(Z)
        assert np.all(np.abs(H - s) <= 2.0 ** -8 * np.abs(s) + 1e-37), name


def test_mixture_params(torch_cuda):
    m = mxr()
    n = 333
    announce("mixture head params")
    net = m.ProposalNet(params(3), batch=n)
    ctx, _, _ = data(n, 4)
    out = net.forward(torch_cuda.tensor(ctx, device="cuda"))
    lo, hi = box()
    g = net.mixture(out, lo, hi)
    torch_cuda.cuda.synchronize()
    h = P.head(f64(out), lo, hi)
    ref = np.concatenate([h["pi"][:, :, None], h["mu"], h["sigma"]], 2).reshape(n, 56)
    got = f64(g)
    assert np.all(np.abs(got - ref) <= 2e-6 * np.abs(ref) + 1e-12), np.max(np.abs(got - ref) / np.abs(ref))
    assert np.allclose(got.reshape(n, 8, 7)[:, :, 0].sum(1), 1.0, rtol=1e-6)


def test_head_gradient_and_loss(torch_cuda):
    """dL/do in float32 against the oracle's FP64 head gradient at the GPU's
    own outputs o: float32 evaluation of ~40 operations whose condition
    numbers stay below ~1e3 gives ~1e-4 of the row's largest entry."""
    m = mxr()
    n = 2500
    announce("head gradient n", n)
    net = m.ProposalNet(params(5), batch=n)
    ctx, y, omega = data(n, 6)
    lo, hi = box()
    import torch
    loss, _ = net.loss_grad(torch.tensor(ctx, device="cuda"), torch.tensor(y, device="cuda"),
                            torch.tensor(omega, device="cuda"), lo, hi)
    torch_cuda.cuda.synchronize()
    O = f64(net.region("O", n, torch.float32, 56))
    L_ref, dO_ref = P.head_grad(O, y, omega, lo, hi)
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * abs(L_ref) + 1e-6
    dO = f64(net.region("DO", n, torch.float32, 56))
    scale = np.max(np.abs(dO_ref), axis=1, keepdims=True)
    err = np.abs(dO - dO_ref) / scale
    assert err.max() <= 3e-4, err.max()
    assert np.array_equal(f64(net.region("DOH", n, torch.bfloat16, 56)), P.bf16_round(dO.astype(np.float32)))


def test_backward_products_and_gradient(torch_cuda):
    m = mxr()
    n = 2500  # three 1024-row splits, the last ragged
    announce("backward products n", n)
    net = m.ProposalNet(params(7), batch=n)
    ctx, y, omega = data(n, 8)
    lo, hi = box()
    import torch
    net.loss_grad(torch.tensor(ctx, device="cuda"), torch.tensor(y, device="cuda"),
                  torch.tensor(omega, device="cuda"), lo, hi)
    torch_cuda.cuda.synchronize()
    W = P.unpack(f64(net.w))
    X = f64(net.region("X", n, torch.bfloat16, 6))
    H1 = f64(net.region("H1", n, torch.bfloat16, 128))
    H2 = f64(net.region("H2", n, torch.bfloat16, 128))
    Z1 = f64(net.region("Z1", n, torch.float32, 128))
    Z2 = f64(net.region("Z2", n, torch.float32, 128))
    dO = f64(net.region("DO", n, torch.float32, 56))
    dOh = f64(net.region("DOH", n, torch.bfloat16, 56))
    dZ2 = f64(net.region("DZ2", n, torch.float32, 128))
    dZ2h = f64(net.region("DZ2H", n, torch.bfloat16, 128))
    dZ1 = f64(net.region("DZ1", n, torch.float32, 128))
    dZ1h = f64(net.region("DZ1H", n, torch.bfloat16, 128))
    # dZ = (dO W^T) * silu'(Z): the product's bound times |silu'|, plus the
    # float32 evaluation of silu'(z) = s (1 + z (1 - s)), whose error is
    # absolute (about 8 u (1 + |z|)), not relative to silu' near its zero
    for got, A, Wt, Z, name in ((dZ2, dOh, W["W3"].T, Z2, "dZ2"), (dZ1, dZ2h, W["W2"].T, Z1, "dZ1")):
        exact, _ = P.gemm_bound(A, Wt)
        sg = P.silu_grad(Z)
        bnd = (gamma(A.shape[1]) * (np.abs(A) @ np.abs(Wt)) * np.abs(sg) + 8 * U * (1 + np.abs(Z)) * np.abs(exact)
               + 2 * U * np.abs(exact * sg) + 1e-40)
        assert np.all(np.abs(got - exact * sg) <= bnd), name
    assert np.array_equal(dZ2h, P.bf16_round(dZ2.astype(np.float32)))
    assert np.array_equal(dZ1h, P.bf16_round(dZ1.astype(np.float32)))
    g = P.unpack(f64(net.grad))
    splits = (n + 1023) // 1024
    # weight gradients: split-K float32 accumulations (K <= 1024) reduced over the splits
    for got, A, B, name in ((g["W3"], H2.T, dOh, "dW3"), (g["W2"], H1.T, dZ2h, "dW2"), (g["W1"], X.T, dZ1h, "dW1")):
        exact, _ = P.gemm_bound(A, B)
        bnd = gamma(1024 + splits) * (np.abs(A) @ np.abs(B)) + 1e-40
        assert np.all(np.abs(got - exact) <= bnd), name
    for got, D, name in ((g["b3"], dO, "db3"), (g["b2"], dZ2, "db2"), (g["b1"], dZ1, "db1")):
        exact = D.sum(axis=0)
        bnd = gamma(1024 + splits) * np.abs(D).sum(axis=0) + 1e-40
        assert np.all(np.abs(got - exact) <= bnd), name
    # against the oracle's FP64 gradient at the same bf16 weights and inputs
    # (activations unrounded there): close in direction and size
    L, g_ref, _ = P.loss_grad(f64(net.w), X, y, omega, lo, hi)
    gg = f64(net.grad)
    cos = gg @ g_ref / (np.linalg.norm(gg) * np.linalg.norm(g_ref))
    rel = np.linalg.norm(gg - g_ref) / np.linalg.norm(g_ref)
    assert cos > 0.999 and rel < 0.05, (cos, rel)


def test_adam_step(torch_cuda):
    m = mxr()
    announce("adam")
    theta = params(9)
    net = m.ProposalNet(theta, batch=16)
    rng = np.random.default_rng(10)
    mth, vth = np.zeros(P.N_PARAMS), np.zeros(P.N_PARAMS)
    th = theta.astype(np.float64)
    for step in range(1, 4):
        g = rng.normal(size=P.N_PARAMS).astype(np.float32) * 10.0 ** rng.integers(-4, 1, P.N_PARAMS)
        net.grad.copy_(torch_cuda.tensor(g))
        net.adam(lr=1e-3)
        th, mth, vth = P.adam(th, mth, vth, g.astype(np.float64), step, lr=1e-3)
    torch_cuda.cuda.synchronize()
    got = f64(net.master)
    assert np.all(np.abs(got - th) <= 1e-6 * np.maximum(np.abs(th), 1e-3)), np.max(np.abs(got - th))
    assert np.array_equal(f64(net.w), P.bf16_round(got.astype(np.float32)))


def test_train_weights(torch_cuda):
    m = mxr()
    announce("training weights")
    rng = np.random.default_rng(11)
    n_bins, n = 5000, 20000
    sum_w = np.where(rng.random(n_bins) < 0.4, 0.0, rng.uniform(0, 3, n_bins))
    sum_w[7] = 1e-9  # a starved bin meets the floor
    live = np.flatnonzero(sum_w > 0)
    bins = rng.choice(live, n)
    w = rng.uniform(0.01, 2, n)
    hits = {"w": torch_cuda.tensor(w, device="cuda"), "bin": torch_cuda.tensor(bins, device="cuda")}
    omega = m.train_weights(hits, n, torch_cuda.tensor(sum_w, device="cuda"), floor_frac=1e-3)
    torch_cuda.cuda.synchronize()
    floor = 1e-3 * sum_w[live].mean()
    ref = w / np.maximum(sum_w[bins], floor)
    assert np.max(np.abs(f64(omega) - ref) / ref) <= 1e-12


def test_training_lowers_the_loss(torch_cuda):
    """Rows drawn from one truncated mixture, contexts random: three epochs
    of Adam lower the loss measured on the same rows."""
    m = mxr()
    announce("training")
    import torch
    rng = np.random.default_rng(12)
    lo, hi = box()
    n = 40000
    centres = np.array([[-0.1, 0.0, 40.0], [0.1, 0.02, 110.0]])
    k = rng.integers(0, 2, n)
    y = centres[k] + rng.normal(size=(n, 3)) * np.array([0.02, 0.01, 8.0])
    y = np.clip(y, lo + 1e-9, hi - 1e-9)
    ctx = rng.normal(size=(n, 6)).astype(np.float32)
    omega = np.ones(n)
    net = m.ProposalNet(P.init_params(13).astype(np.float32), batch=4096)
    tc, ty, tw = (torch.tensor(a, device="cuda") for a in (ctx, y, omega))
    before = float(net.loss_grad(tc[:4096], ty[:4096], tw[:4096], lo, hi)[0].item())
    steps = 3 * ((n + 4095) // 4096)
    log = torch.zeros(steps, dtype=torch.float64, device="cuda")
    net.train(tc, ty, tw, lo, hi, epochs=3, lr=3e-3, seed=5, loss_log=log)
    after = float(net.loss_grad(tc[:4096], ty[:4096], tw[:4096], lo, hi)[0].item())
    torch_cuda.cuda.synchronize()
    lg = f64(log)
    assert np.all(np.isfinite(lg))
    assert after < before - 1.0, (before, after)
    assert lg[-5:].mean() < lg[:5].mean()
    assert net.step == steps


@pytest.mark.parametrize("n", [4096, 65536, 1000, 45])
def test_fused_step_gradient_equals_the_layered_gradient(torch_cuda, n):
    """One training step over a whole batch (epochs = 1, batch = n): the
    fused step's gradient (left in the gradient buffer) against the
    layer-by-layer gradient of mxr_mlp_loss_grad on the same rows and
    weights.  The operands and roundings are the same, only the order of the
    float32 sums differs (strips of 32 rows summed per work-group, then the
    groups in order, against 1024-row splits), so the two agree to float32
    summation noise; the step's loss agrees as well.  Batches that are not a
    multiple of the 32-row strip leave a partial strip."""
    m = mxr()
    import torch
    announce("fused step vs layered gradient", n)
    rng = np.random.default_rng(21 + n)
    lo, hi = box()
    y = np.stack([rng.uniform(lo[d], hi[d], n) for d in range(3)], 1)
    ctx = rng.normal(size=(n, 6)).astype(np.float32)
    omega = rng.uniform(0.1, 2.0, n)
    p0 = P.init_params(3).astype(np.float32) + rng.normal(0, 0.05, 24632).astype(np.float32)
    tc, ty, tw = (torch.tensor(a, device="cuda") for a in (ctx, y, omega))
    ref = m.ProposalNet(p0, batch=n)
    loss_ref, grad_ref = ref.loss_grad(tc, ty, tw, lo, hi)
    g_ref = grad_ref.clone()
    fused = m.ProposalNet(p0, batch=n)
    log = torch.zeros(1, dtype=torch.float64, device="cuda")
    fused.train(tc, ty, tw, lo, hi, epochs=1, lr=1e-3, seed=9, loss_log=log)
    torch.cuda.synchronize()
    g = fused.grad.double().cpu().numpy()
    r = g_ref.double().cpu().numpy()
    rel = np.linalg.norm(g - r) / np.linalg.norm(r)
    cos = float(g @ r / (np.linalg.norm(g) * np.linalg.norm(r)))
    print(f"n={n}: gradient rel. difference {rel:.2e}, cosine {cos:.8f}; loss {float(log[0]):.6f} vs "
          f"{float(loss_ref.item()):.6f}", flush=True)
    assert rel < 2e-3 and cos > 0.99999
    assert abs(float(log[0]) - float(loss_ref.item())) <= 1e-5 * max(1.0, abs(float(loss_ref.item())))
    # the Adam step of the fused path from the same gradient: master - lr sign-ish step
    assert torch.isfinite(fused.master).all()
    assert fused.step == 1
