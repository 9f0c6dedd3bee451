"""bench.py's host-side contract, checked without a GPU: more than one GPU
is refused with a message (the tracer measures one GPU), the argument
parser knows every workload, and the measured-traffic lookup reads the
committed profile summaries (None when the kernel sources differ from the
ones the counters were taken with)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_workloads_listed():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for w in ("projection", "batch", "learned", "train", "stepping", "crl", "scatter", "peaks", "basic", "beamline"):
        assert w in r.stdout


def test_measured_traffic_lookup(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    for prof in (bench.PROFILE, bench.PROFILE_STEP, bench.PROFILE_CRL, bench.PROFILE_SCATTER):
        assert os.path.exists(os.path.join(ROOT, prof))
        t = bench.measured_traffic(prof)
        assert t is None or t > 0
    # a profile whose source hash does not match gives no traffic
    fake = tmp_path / "p.md"
    fake.write_text("counters: source=0000000000000000 fetch_kib=1 write_kib=1 fetch_scale=2.00 write_scale=1.00\n")
    assert bench.measured_traffic(str(fake)) is None  # an absolute path is used as is


def test_committed_profiles_match_the_kernel_sources():
    """The headline line's measured figures (HBM traffic, VALU issue, FP64
    op classes) come from the committed counters only while their source
    hash is the current kernel sources'; a kernel change without new
    counters would silently turn them into nulls."""
    sys.path.insert(0, ROOT)
    import bench
    for prof in (bench.PROFILE, bench.PROFILE_STEP, bench.PROFILE_CRL, bench.PROFILE_SCATTER):
        assert bench.measured_traffic(prof) is not None, f"{prof}: counters taken on other kernel sources"
    assert bench.measured_valu() is not None
    assert bench.measured_fp64_flop() is not None
