"""The allocation-free network forward (mxr_mlp_forward_noalloc) against the
workspace forward (mxr_mlp_forward), through the C ABI: the same kernels on
the same operands, so the outputs must agree bit for bit -- on two calls in a
row, the second with fewer rows (the static scratch keeps the first call's
values, none of which may leak into the second), and a call above the row
limit is refused."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def mxr():
    import paper_2410_08747_amd as m
    return m


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def contexts(rng, n):
    ang = rng.uniform(0, 2 * np.pi, n)
    c = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), np.cos(ang), np.sin(ang),
                  rng.uniform(0.5, 1.0, n)], 1)
    return c.astype(np.float32)


def test_noalloc_forward_equals_workspace_forward(torch_cuda):
    torch = torch_cuda
    m = mxr()
    print("[gpu case] allocation-free forward vs workspace forward", flush=True)
    rng = np.random.default_rng(11)
    params = np.asarray(workloads.init_mlp_params(1), dtype=np.float32)
    params = params + rng.normal(0, 0.05, params.shape).astype(np.float32)  # non-trivial weights
    net = m.ProposalNet(params, batch=m.MLP_NOALLOC_ROWS)
    for n in (m.MLP_NOALLOC_ROWS, 1000, 1):
        ctx = torch.tensor(contexts(rng, n), device="cuda")
        ref = torch.empty(n, m.MLP_OUT, dtype=torch.float32, device="cuda")
        m.mxr_mlp_forward(net.w.data_ptr(), ctx.data_ptr(), n, ref.data_ptr(), net.ws.data_ptr(), net.ws_bytes)
        out = torch.full((n, m.MLP_OUT), float("nan"), dtype=torch.float32, device="cuda")
        m.mxr_mlp_forward_noalloc(net.w.data_ptr(), ctx.data_ptr(), n, out.data_ptr())
        torch.cuda.synchronize()
        assert torch.isfinite(out).all(), f"n={n}: non-finite outputs"
        assert torch.equal(out, ref), f"n={n}: outputs differ from the workspace forward"
    ctx = torch.zeros(m.MLP_NOALLOC_ROWS + 1, m.MLP_IN, dtype=torch.float32, device="cuda")
    out = torch.empty(m.MLP_NOALLOC_ROWS + 1, m.MLP_OUT, dtype=torch.float32, device="cuda")
    with pytest.raises(m.MxrError):
        m.mxr_mlp_forward_noalloc(net.w.data_ptr(), ctx.data_ptr(), m.MLP_NOALLOC_ROWS + 1, out.data_ptr())
    assert "at most" in m.mxr_last_error()
