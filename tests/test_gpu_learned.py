"""What the learned proposal gains, measured on the GPU with the project's own
kernels end to end: hits collected by the plain tracer, the network trained
by the library's forward / backward / Adam kernels (mxr_proposal_train, one
call), the proposal set from one forward (mxr_proposal_apply), and the
per-bin error by batch means over 16 independent replicas.

At equal rays the learned proposal must reach a lower 95th-percentile
per-bin relative error (over the signal bins) than the plain source, and its
image must agree with a high-statistics plain reference (mean z^2 near 1:
the importance weights keep the estimator unbiased).  The one-call training
must give bit for bit the parameters of the separate calls it replaces
(training weights per run, then the training loop).
"""
import numpy as np
import pytest

import workloads

from test_gpu_parity import announce, cpu

pytestmark = pytest.mark.gpu

R = 16


def mxr():
    import paper_2410_08747_amd as m
    return m


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def instr(angle=0.0):
    vol = workloads.make_phantom(64, seed=1)
    return workloads.edct_projection(vol, workloads.make_mu_tables(1), angle=angle, strata=1024, nx=64, ny=16,
                                     ne=32)


def collect(torch, I, n_rays, cap, context):
    hits = I.new_hits(cap)
    tallies = I.new_tallies()
    I.collect(n_rays, seed=1, context=context, hits=hits, purpose=1, tallies=tallies)
    torch.cuda.synchronize()
    n = int(hits["count"].item())
    assert 0 < n <= cap
    return hits, n, tallies[0]["sum_w"]


def replicas(torch, I, n_rays):
    m = mxr()
    per = n_rays // R
    nb = I.new_tallies()[0]["sum_w"].numel()
    sums = torch.zeros(R, nb, dtype=torch.float64, device="cuda")
    for r in range(R):
        t = {"count": torch.zeros(nb, dtype=torch.int64, device="cuda"), "sum_w": sums[r],
             "sum_w2": torch.zeros(nb, dtype=torch.float64, device="cuda")}
        I.run(per, seed=1, purpose=3 + r, tallies=[t])
    torch.cuda.synchronize()
    mean, rel = m.batch_means(sums, per)
    return cpu(mean), cpu(rel)


def test_one_call_training_equals_the_separate_calls(torch_cuda):
    torch = torch_cuda
    m = mxr()
    ins = instr()
    I = m.Instrument(ins)
    ctx = workloads.projection_context(0.0, 64)
    announce("one-call training vs separate calls")
    hits, n, image = collect(torch, I, 3_000_000, 2_000_000, ctx)
    # two runs' worth of rows: the first half weighted by the image, the
    # second half by twice the image (a different run's normalisation)
    half = n // 2
    images = [image, 2.0 * image]
    a = m.ProposalNet(workloads.init_mlp_params(1), batch=4096)
    omega_a = a.train_from_runs(I, hits, [0, half, n], images, epochs=2, lr=1e-3, seed=3)
    b = m.ProposalNet(workloads.init_mlp_params(1), batch=4096)
    parts = [m.train_weights({"w": hits["w"][0:half], "bin": hits["bin"][0:half]}, half, images[0]),
             m.train_weights({"w": hits["w"][half:n], "bin": hits["bin"][half:n]}, n - half, images[1])]
    omega_b = torch.cat(parts)
    lo, hi = I.proposal_box()
    b.train(hits["ctx"][:n], hits["y"][:n], omega_b, lo, hi, epochs=2, lr=1e-3, seed=3)
    torch.cuda.synchronize()
    assert torch.equal(omega_a, omega_b)
    assert torch.equal(a.master, b.master)
    assert torch.equal(a.w, b.w)
    assert a.step == b.step > 0


def test_learned_proposal_gains_at_equal_rays(torch_cuda):
    torch = torch_cuda
    m = mxr()
    from paper_2410_08747_amd import metrics
    ins = instr()
    I = m.Instrument(ins)
    ctx = workloads.projection_context(0.0, 64)
    announce("learned gain: collect, train, apply, replicas")
    hits, n, image = collect(torch, I, 20_000_000, 8_000_000, ctx)
    net = m.ProposalNet(workloads.init_mlp_params(1), batch=65536)
    steps = 5 * ((n + 65535) // 65536)
    log = torch.zeros(steps, dtype=torch.float64, device="cuda")
    net.train_from_runs(I, hits, [0, n], [image], epochs=5, lr=1e-3, seed=1, loss_log=log)
    torch.cuda.synchronize()
    ll = cpu(log)
    assert np.all(np.isfinite(ll)) and ll[-20:].mean() < ll[:20].mean()
    del hits

    # high-statistics plain reference and its signal bins
    n_ref = 400_000_000
    ref = I.run(n_ref, seed=7, purpose=2)[0]
    torch.cuda.synchronize()
    I_ref = cpu(ref["sum_w"]) / n_ref
    var_ref = cpu(ref["sum_w2"]) / n_ref ** 2
    mask = metrics.signal_bins(I_ref, metrics.flat_field(ins))
    assert mask.sum() > 1000

    n_eval = 64_000_000
    _, rel_p = replicas(torch, I, n_eval)
    I.apply_proposal(net, ctx, alpha=0.1)
    mean_l, rel_l = replicas(torch, I, n_eval)
    q_p, q_l = metrics.q95(rel_p, mask), metrics.q95(rel_l, mask)
    z = (mean_l - I_ref)[mask] / np.sqrt((rel_l * mean_l)[mask] ** 2 + var_ref[mask])
    z2 = float(np.mean(z * z))
    print(f"q95 plain {q_p:.4f} learned {q_l:.4f} (gain in rays to equal error {(q_p / q_l) ** 2:.2f}x); "
          f"mean z^2 {z2:.3f}, |z| > 4 in {np.mean(np.abs(z) > 4):.2e} of {mask.sum()} bins; "
          f"loss {ll[:20].mean():.3f} -> {ll[-20:].mean():.3f}", flush=True)
    assert q_l < 0.9 * q_p, f"learned q95 {q_l:.4f} is not below plain {q_p:.4f}"
    # unbiased: the learned image against the reference, within the batch-means
    # and reference errors (a 16-replica variance estimate inflates z^2 a little)
    assert 0.8 < z2 < 1.3
    assert np.mean(np.abs(z) > 5) < 1e-3
