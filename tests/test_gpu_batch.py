"""Batched runs (many angles of phantoms of different size in one captured
launch), through the C ABI.

A batch must give every job's tallies exactly what a separate mxr_run of
that job gives (counts identical, sums within 1e-9 relative: only the order
of the atomic additions differs), for every launch shape, on every replay of
the captured graph; and a job of a batch must match the oracle's run of the
same instrument, seed and RNG job field.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

REL_BIN = 1e-9


def mxr():
    import paper_2410_08747_amd as m
    return m


def announce(*what):
    print("[gpu case]", *what, flush=True)


def cpu(t):
    return t.detach().cpu().numpy()


def same_tally(a, b, label):
    assert np.array_equal(cpu(a["count"]), cpu(b["count"])), f"{label}: counts differ"
    for key in ("sum_w", "sum_w2"):
        g, o = cpu(a[key]), cpu(b[key])
        assert np.array_equal(g == 0, o == 0), f"{label}: {key} zero pattern differs"
        nz = o != 0
        if nz.any():
            err = np.max(np.abs(g[nz] - o[nz]) / np.abs(o[nz]))
            assert err <= REL_BIN, f"{label}: {key} rel err {err:.3e}"


def oracle_tally(gt, ot, label):
    assert np.array_equal(cpu(gt["count"]).astype(np.uint64), ot["count"]), f"{label}: counts differ from oracle"
    for key in ("sum_w", "sum_w2"):
        g, o = cpu(gt[key]), ot[key]
        assert np.array_equal(g == 0, o == 0), f"{label}: {key} zero pattern differs from oracle"
        nz = o != 0
        if nz.any():
            assert np.max(np.abs(g[nz] - o[nz]) / np.abs(o[nz])) <= REL_BIN, f"{label}: {key} vs oracle"


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def edct_jobs():
    """Three phantoms of uneven size (40^3, 48^3, 64^3) at several angles,
    small detectors, ray counts from 1 to 300001 (ragged tails)."""
    mu = workloads.make_mu_tables(1)
    jobs = []
    sizes = [(40, [0.0, 1.3], [1, 70001]), (48, [0.2, 2.9, 4.4], [300001, 257, 4096]), (64, [0.7, 5.5], [200003, 65536])]
    k = 0
    for n, angles, rays in sizes:
        vol = workloads.make_phantom(n, seed=n)
        for ang, nr in zip(angles, rays):
            ins = workloads.edct_projection(vol, mu, angle=ang, strata=16, nx=32, ny=16, ne=32)
            jobs.append((ins, nr, 11 + k, 100 + k))
            k += 1
    return jobs


def build(m, spec, shared):
    out = []
    for ins, nr, seed, job in spec:
        I = m.Instrument(ins, shared=shared)
        out.append((I, nr, seed, job, I.new_tallies()))
    return out


def separate_runs(jobs):
    return [I.run(nr, seed=seed, job=job) for I, nr, seed, job, _ in jobs]


@pytest.mark.parametrize("schedule", [(0, 0, 256, 0), (1, 1, 256, 0), (1, 2, 4096, 0), (1, 8, 65536, 0),
                                      (2, 0, 256, 1), (2, 0, 256, 3)])
def test_batch_equals_separate_runs(torch_cuda, edct_jobs, schedule):
    m = mxr()
    announce("batch vs separate runs", "schedule", schedule, "jobs", len(edct_jobs))
    jobs = build(m, edct_jobs, {})
    ref = separate_runs(jobs)
    B = m.Batch(jobs, schedule=schedule)
    assert B.schedule == schedule
    B.run()
    torch_cuda.cuda.synchronize()
    for k, (j, r) in enumerate(zip(jobs, ref)):
        same_tally(j[4][0], r[0], f"job {k} schedule {schedule}")
    B.close()


def test_batch_job_matches_oracle(torch_cuda, edct_jobs):
    m = mxr()
    announce("batch jobs vs oracle")
    jobs = build(m, edct_jobs, {})
    B = m.Batch(jobs)
    B.run()
    torch_cuda.cuda.synchronize()
    for k in (0, 1, 4, 6):
        ins, nr, seed, job = edct_jobs[k]
        o = oracle.run(ins, nr, seed=seed, job=job)
        oracle_tally(jobs[k][4][0], o[0], f"batch job {k}")


def test_graph_replays(torch_cuda, edct_jobs):
    """Every replay of the captured launch, with eager zeroing and other work
    between replays, gives the first replay's tallies."""
    m = mxr()
    announce("graph replays")
    jobs = build(m, edct_jobs, {})
    B = m.Batch(jobs, schedule=(1, 4, 4096, 0))
    L = m.Batch(jobs, schedule=(2, 0, 0, 2))  # the launches form: its own graph
    first = None
    for rep in range(4):
        for j in jobs:
            for v in j[4][0].values():
                v.zero_()
        (B if rep % 2 == 0 else L).run()
        torch_cuda.cuda.synchronize()
        snap = [{k: v.clone() for k, v in j[4][0].items()} for j in jobs]
        if first is None:
            first = snap
        else:
            for k, (a, b) in enumerate(zip(snap, first)):
                same_tally(a, b, f"replay {rep} job {k}")
        # unrelated eager work between replays
        torch_cuda.ones(1 << 20, device="cuda").sum().item()


def test_schedule_change_and_autotune(torch_cuda, edct_jobs, tmp_path):
    m = mxr()
    announce("autotune")
    jobs = build(m, edct_jobs, {})
    ref = separate_runs(jobs)
    B = m.Batch(jobs)
    cache = str(tmp_path / "tune.txt")
    s1 = B.autotune(0.25, cache)
    assert B.schedule == s1
    f, g, t, br = s1
    assert (f, g, t, br) == (0, 0, 256, 0) or (f == 1 and 1 <= g <= 8 and t % 256 == 0 and br == 0) or \
        (f == 2 and 1 <= br <= 4)
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"\t{f} {g} {t} {br}")
    B.schedule = (0, 0, 256, 0)
    s2 = B.autotune(0.25, cache)  # answered from the cache, nothing timed
    assert s2 == s1 and len(open(cache).read().strip().splitlines()) == 1
    # timing runs added into the tallies: zero, then one production run
    for j in jobs:
        for v in j[4][0].values():
            v.zero_()
    B.run()
    torch_cuda.cuda.synchronize()
    for k, (j, r) in enumerate(zip(jobs, ref)):
        same_tally(j[4][0], r[0], f"tuned job {k}")


def test_shared_upload(torch_cuda, edct_jobs):
    m = mxr()
    shared = {}
    jobs = build(m, edct_jobs, shared)
    # 3 phantom volumes, 1 mu table (same array object)
    assert len([k for k in shared if k[1] == np.dtype(np.uint8).str]) == 3
    assert len([k for k in shared if k[1] == np.dtype(np.float64).str]) == 1


def test_basic_chain_batch(torch_cuda):
    """A batch of the slit + absorber instrument (no phantom) at several seeds."""
    m = mxr()
    announce("basic chain batch")
    ins = workloads.basic_absorber()
    spec = [(ins, n, seed, seed) for n, seed in [(1000, 1), (250007, 2), (1, 3), (99999, 4)]]
    jobs = build(m, spec, {})
    ref = separate_runs(jobs)
    B = m.Batch(jobs)
    B.run()
    torch_cuda.cuda.synchronize()
    for k, (j, r) in enumerate(zip(jobs, ref)):
        same_tally(j[4][0], r[0], f"basic job {k}")
    o = oracle.run(ins, 250007, seed=2, job=2)
    oracle_tally(jobs[1][4][0], o[0], "basic job 1 vs oracle")


def test_batch_errors(torch_cuda, edct_jobs):
    m = mxr()
    announce("batch errors")
    ins, nr, seed, job = edct_jobs[0]
    I = m.Instrument(ins)
    other = m.Instrument(workloads.basic_absorber())
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 0, I.new_tallies()), (other, 10, 1, 0, other.new_tallies())])  # chains differ
    with pytest.raises(m.MxrError):
        m.Batch([(I, 0, 1, 0, I.new_tallies())])  # no rays
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 1 << 24, I.new_tallies())])  # job field too wide
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 0, I.new_tallies())], schedule=(1, 9, 256, 0))
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 0, I.new_tallies())], schedule=(1, 2, 300, 0))
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 0, I.new_tallies())], schedule=(2, 0, 0, 5))
    with pytest.raises(m.MxrError):
        m.Batch([(I, 10, 1, 0, I.new_tallies())], schedule=(3, 0, 0, 0))
    B = m.Batch([(I, 10, 1, 0, I.new_tallies())])
    with pytest.raises(m.MxrError):
        B.autotune(0.0)
    with pytest.raises(m.MxrError):
        B.schedule = (1, 3, 100, 0)
    # a proposal on a job's instrument is refused (batches trace the plain source)
    import torch
    P = m.Instrument(ins)
    g = np.tile([1 / 8, 0.0, 0.0, 80.0, 0.02, 0.02, 30.0], 8)
    P.set_proposal(torch.tensor(g, device="cuda"), 0.1)
    with pytest.raises(m.MxrError):
        m.Batch([(P, 10, 1, 0, P.new_tallies())])
