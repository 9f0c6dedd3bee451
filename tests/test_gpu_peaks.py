"""The micro-benchmark kernels behind the measured roofline denominators
(mxr_peak_launch): each runs through the C ABI; the atomic kernel's counts
add up exactly to the atomics it reports, the read kernel's partial sums to
the elements it reports, and the arithmetic kernels leave finite sinks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def mxr():
    import paper_2410_08747_amd as m
    return m


@pytest.mark.parametrize("kind", ["fp64_fma", "u32_mulhi", "fp64_exp"])
def test_arithmetic_kernels(torch_cuda, kind):
    groups = 64
    buf = torch_cuda.zeros(groups * 256, dtype=torch_cuda.float64, device="cuda")
    print("[gpu case] peak", kind, flush=True)
    work = mxr().mxr_peak_launch(kind, buf.data_ptr(), buf.numel() * 8, 1, 100, groups)
    torch_cuda.cuda.synchronize()
    assert work > 0 and torch_cuda.isfinite(buf).all()


def test_read_kernel_sums(torch_cuda):
    groups = 32
    sink = groups * 256
    n_doubles = sink + 2 * 1_000_003
    buf = torch_cuda.ones(n_doubles, dtype=torch_cuda.float64, device="cuda")
    buf[:sink] = 0.0
    print("[gpu case] peak read", flush=True)
    work = mxr().mxr_peak_launch("read", buf.data_ptr(), n_doubles * 8, 1, 1, groups)
    torch_cuda.cuda.synchronize()
    assert work == 16 * 1_000_003
    assert buf[:sink].sum().item() == 2 * 1_000_003


@pytest.mark.parametrize("spread", [1, 130, 14400])
def test_atomic_counts(torch_cuda, spread):
    groups = 16
    buf = torch_cuda.zeros(20000, dtype=torch_cuda.float64, device="cuda")
    print("[gpu case] peak atomic", spread, flush=True)
    work = mxr().mxr_peak_launch("atomic_f64", buf.data_ptr(), buf.numel() * 8, spread, 7, groups)
    torch_cuda.cuda.synchronize()
    assert work == groups * 256 * 7
    assert buf[:spread].sum().item() == work and buf[spread:].sum().item() == 0.0


def test_errors(torch_cuda):
    m = mxr()
    buf = torch_cuda.zeros(1024, dtype=torch_cuda.float64, device="cuda")
    with pytest.raises(m.MxrError):
        m.mxr_peak_launch("fp64_fma", buf.data_ptr(), buf.numel() * 8, 1, 10, 64)  # sink too small
    with pytest.raises(m.MxrError):
        m.mxr_peak_launch("atomic_f64", buf.data_ptr(), buf.numel() * 8, 2000, 1, 1)  # spread beyond the buffer
    with pytest.raises(m.MxrError):
        m.mxr_peak_launch("fp64_exp", buf.data_ptr(), buf.numel() * 8, 1, 0, 1)  # no iterations
