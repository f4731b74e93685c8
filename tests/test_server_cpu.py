"""The serving scheduler on the CPU (fake executor: no GPU, jobs take a
time proportional to their points): FIFO completion, continuous batching of
small jobs, admission under a small budget, bad jobs failing alone, and the
latency / throughput statistics."""
import time

import numpy as np
import pytest

import paper_2409_10743_amd as dbx


def pts(n, seed=0):
    return np.random.Generator(np.random.PCG64(seed)).random((n, 3)).astype(np.float32)


def test_jobs_complete_and_stats():
    s = dbx.Server(slots=2, fake_us_per_mpoint=2000.0)
    tickets = [s.submit(pts(1000 * (k + 1), k), 0.01, 2) for k in range(20)]
    for t in tickets:
        assert s.wait(t, 10.0) == 0
        assert (s.labels(t) == -1).all()
    st = s.stats()
    assert st["submitted"] == 20 and st["completed"] == 20 and st["failed"] == 0
    assert st["points"] == sum(1000 * (k + 1) for k in range(20))
    assert 0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["mpoints_per_s"] > 0
    s.close()


def test_small_jobs_are_batched_large_ones_are_not():
    # one slot that is busy with a large job while small ones queue up
    s = dbx.Server(slots=1, batch_cut=10000, fake_us_per_mpoint=200000.0)
    big = s.submit(pts(200000), 0.01, 2)
    time.sleep(0.01)
    small = [s.submit(pts(500, k), 0.01, 5) for k in range(30)]
    for t in [big] + small:
        assert s.wait(t, 30.0) == 0
    st = s.stats()
    assert st["batches"] >= 1 and st["batched_jobs"] >= 10
    s.close()


def test_budget_admission_and_too_big():
    one = dbx.load_library().dbscan_scratch_bytes(100000, 2, 1) + 100000 * 16 + 4096
    s = dbx.Server(slots=4, budget_bytes=int(one * 1.5), batch_cut=1,
                   fake_us_per_mpoint=100000.0)
    ts = [s.submit(pts(100000, k), 0.01, 2) for k in range(6)]
    huge = s.submit(pts(1000000, 9), 0.01, 2)
    for t in ts:
        assert s.wait(t, 60.0) == 0
    assert s.wait(huge, 60.0) == -5
    st = s.stats()
    assert st["peak_in_flight_bytes"] <= int(one * 1.5)
    assert st["failed"] == 1 and st["completed"] == 6
    s.close()


def test_invalid_jobs_rejected_at_submit():
    s = dbx.Server(slots=1, fake_us_per_mpoint=10.0)
    with pytest.raises(dbx.DbscanError):
        s.submit(pts(10), float("nan"), 2)
    with pytest.raises(dbx.DbscanError):
        s.submit(pts(10), 0.1, 0)
    ok = s.submit(pts(10), 0.1, 2)
    assert s.wait(ok, 10.0) == 0
    assert s.submit(np.zeros((0, 3), np.float32), 0.1, 2) > 0
    s.close()


def test_fifo_order_for_large_jobs():
    s = dbx.Server(slots=1, batch_cut=1, fake_us_per_mpoint=20000.0)
    ts = [s.submit(pts(20000, k), 0.01, 2) for k in range(8)]
    done = []
    for t in ts:
        s.wait(t, 30.0)
        done.append(s.job_times(t)[1])
    assert done == sorted(done)
    s.close()


def test_budget_bounds_memory_kept_between_jobs():
    """Slots keep their arena and I/O buffers after a job; the budget bounds
    that memory, not only the jobs running: jobs of growing size on four
    slots under a budget of about two of the largest never make the slots
    hold more than the budget (idle slots give memory back), and every job
    completes."""
    lib = dbx.load_library()
    big = lib.dbscan_scratch_bytes(200000, 5, 1) + 200000 * 16
    budget = int(big * 2.2)
    s = dbx.Server(slots=4, budget_bytes=budget, batch_cut=1, fake_us_per_mpoint=20000.0)
    sizes = [20000, 200000, 50000, 200000, 120000, 200000, 10000, 180000, 200000, 90000]
    ts = [s.submit(pts(n, k), 0.01, 5) for k, n in enumerate(sizes)]
    for t in ts:
        assert s.wait(t, 60.0) == 0
    st = s.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0
    assert 0 < st["peak_in_flight_bytes"] <= budget
    s.close()


def test_batches_respect_the_budget():
    """Small jobs are batched only up to what fits the budget (batched
    layout included); none fails."""
    lib = dbx.load_library()
    one = lib.dbscan_scratch_bytes(5000, 2, 1) + 5000 * 16
    s = dbx.Server(slots=1, budget_bytes=one * 6, batch_cut=10000, fake_us_per_mpoint=50000.0)
    first = s.submit(pts(9000, 1), 0.01, 2)
    time.sleep(0.01)
    ts = [s.submit(pts(5000, 10 + k), 0.01, 2) for k in range(40)]
    for t in [first] + ts:
        assert s.wait(t, 60.0) == 0
    st = s.stats()
    assert st["failed"] == 0 and st["batches"] >= 1
    assert st["peak_in_flight_bytes"] <= one * 6
    s.close()
