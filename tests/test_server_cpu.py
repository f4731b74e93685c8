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
