"""Pins of the oracle's counter-based generator.

Philox4x32-10 (Salmon et al., SC'11) is checked word for word against the
engine of the rocRAND headers, an implementation written independently of
the oracle; the uniform mapping and the counter layout (block, ray id,
purpose/job) are checked through the same engine; uniformity by moments and
chi-square.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROCRAND_HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"


@pytest.fixture(scope="module")
def kat_exe(tmp_path_factory):
    if not (os.path.exists(ROCRAND_HEADER) and shutil.which("g++")):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("kat") / "philox_kat")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    os.path.join(HERE, "philox_kat.cpp"), "-o", exe], check=True)
    return exe


def rocrand_words(exe, triples):
    inp = "".join(f"{s} {q} {c}\n" for s, q, c in triples)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    return [[int(x) for x in line.split()] for line in out.strip().splitlines()]


def test_philox_matches_rocrand_engine(kat_exe):
    rng = np.random.default_rng(7)
    triples = [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**62 - 1)]
    for _ in range(300):
        triples.append((int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2)),
                        int(rng.integers(0, 2**63)), int(rng.integers(0, 2**62))))
    ref = rocrand_words(kat_exe, triples)
    for (s, q, c), want in zip(triples, ref):
        ctr = [c & 0xFFFFFFFF, c >> 32, q & 0xFFFFFFFF, q >> 32]
        key = [s & 0xFFFFFFFF, s >> 32]
        assert oracle.philox(ctr, key) == want, (s, q, c)


def test_uniform_counter_layout(kat_exe):
    """uniform(seed, ray, index, purpose, job) uses counter (index // 2, ray
    lo, ray hi, purpose << 24 | job) and words (1:0) / (3:2)."""
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(100):
        seed = int(rng.integers(0, 2**63))
        # the engine's offset is 4 * (index // 2 | ray lo << 32): keep it in 64 bits
        ray = (int(rng.integers(0, 2**20)) << 32) | int(rng.integers(0, 2**29))
        purpose = int(rng.integers(0, 8))
        job = int(rng.integers(0, 2**24))
        idx = int(rng.integers(0, 12))
        cases.append((seed, ray, purpose, job, idx))
    triples = []
    for seed, ray, purpose, job, idx in cases:
        word3 = (purpose << 24) | job
        sub = (ray >> 32) | (word3 << 32)
        ctr = (idx // 2) | ((ray & 0xFFFFFFFF) << 32)
        triples.append((seed, sub, ctr))
    ref = rocrand_words(kat_exe, triples)
    for (seed, ray, purpose, job, idx), w in zip(cases, ref):
        word = (w[1] << 32 | w[0]) if idx % 2 == 0 else (w[3] << 32 | w[2])
        want = ((word >> 12) + 0.5) * 2.0**-52
        got = oracle.uniform(seed, ray, idx, purpose, job)
        assert got == want


def test_uniform_distribution():
    n = 60000
    u = np.array([oracle.uniform(1, r, k) for r in range(n // 6) for k in range(6)])
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    assert abs(u.var() - 1 / 12) < 4 * np.sqrt(1 / 180 / n)
    h, _ = np.histogram(u, bins=100, range=(0, 1))
    assert stats.chisquare(h).pvalue > 1e-4
    # pairs from the same block and from adjacent rays are uncorrelated
    a = np.array([oracle.uniform(3, r, 0) for r in range(20000)])
    b = np.array([oracle.uniform(3, r, 1) for r in range(20000)])
    assert abs(np.corrcoef(a, b)[0, 1]) < 4 / np.sqrt(20000)
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 4 / np.sqrt(20000)


def test_seed_purpose_job_change_stream():
    base = oracle.uniform(1, 5, 0)
    assert oracle.uniform(2, 5, 0) != base
    assert oracle.uniform(1, 6, 0) != base
    assert oracle.uniform(1, 5, 0, purpose=1) != base
    assert oracle.uniform(1, 5, 0, job=3) != base
    assert oracle.uniform(1, 5, 2) != base
