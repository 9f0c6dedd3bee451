"""The batch-means error kernel against numpy, and the error metric of a
small projection: replicas of the plain source give relative errors that
agree with the i.i.d. estimate sqrt(sum w^2 - (sum w)^2 / n) / sum w."""
import numpy as np
import pytest

import workloads
from paper_2410_08747_amd import metrics

from test_gpu_parity import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_batch_means_kernel(torch_cuda):
    import paper_2410_08747_amd as m
    announce("batch means kernel")
    rng = np.random.default_rng(1)
    R, nb, per = 16, 10007, 1000
    sums = rng.gamma(2.0, 1.0, size=(R, nb))
    sums[:, 5] = 0.0  # an empty bin
    mean, rel = m.batch_means(torch_cuda.tensor(sums, device="cuda"), per)
    I = sums / per
    ref_mean = I.mean(0)
    ref_rel = I.std(0, ddof=1) / (np.sqrt(R) * ref_mean)
    g_mean, g_rel = mean.cpu().numpy(), rel.cpu().numpy()
    ok = ref_mean > 0
    assert np.allclose(g_mean, ref_mean, rtol=1e-14, atol=0)
    assert np.allclose(g_rel[ok], ref_rel[ok], rtol=1e-12)
    assert np.isinf(g_rel[5])
    with pytest.raises(m.MxrError):
        m.batch_means(torch_cuda.tensor(sums[:1], device="cuda"), per)


def test_replica_error_matches_iid_estimate(torch_cuda):
    """Unstratified plain runs: batch means and the i.i.d. formula estimate
    the same per-bin error (their ratio scatters around 1 with the
    chi distribution of 15 degrees of freedom)."""
    import paper_2410_08747_amd as m
    announce("replica error vs iid")
    vol = workloads.make_phantom(64, seed=1)
    ins = workloads.edct_projection(vol, workloads.make_mu_tables(1), strata=1, nx=16, ny=8, ne=8)
    I = m.Instrument(ins)
    R, per = 16, 200000
    nb = 16 * 8 * 8
    sums = torch_cuda.zeros(R, nb, dtype=torch_cuda.float64, device="cuda")
    one = I.new_tallies()
    for r in range(R):
        t = [{"count": torch_cuda.zeros(nb, dtype=torch_cuda.int64, device="cuda"), "sum_w": sums[r],
              "sum_w2": torch_cuda.zeros(nb, dtype=torch_cuda.float64, device="cuda")}]
        I.run(per, seed=1, purpose=3 + r, tallies=t)
        I.run(per, seed=1, purpose=3 + r, tallies=one)
    mean, rel = m.batch_means(sums, per)
    torch_cuda.cuda.synchronize()
    n = R * per
    sw, sw2 = one[0]["sum_w"].cpu().numpy(), one[0]["sum_w2"].cpu().numpy()
    iid = np.sqrt(np.maximum(sw2 - sw * sw / n, 0)) / sw
    g = rel.cpu().numpy()
    live = (one[0]["count"].cpu().numpy() > 400)
    ratio = g[live] / iid[live]
    assert abs(np.median(ratio) - 1.0) < 0.05, np.median(ratio)
    assert np.allclose(mean.cpu().numpy(), sw / n, rtol=1e-12, atol=0)
    # the metric helpers on this image
    mask = metrics.signal_bins(mean.cpu().numpy(), metrics.flat_field(ins))
    assert mask.sum() > 0.5 * nb
    q = metrics.q95(g, mask)
    assert 0 < q < 1
