"""GPU serving: jobs of uneven sizes submitted while others run; every
result must be identical to the same job clustered alone (and, for the
smaller ones, to the oracle); a bad job inside a batch fails alone."""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
import paper_2409_10743_amd as dbx  # noqa: E402

pytestmark = pytest.mark.gpu
F32 = np.float32


def test_mixed_trace_alone_equals_in_mix():
    pool = datagen.clumps(1 << 21, 50)
    rng = np.random.Generator(np.random.PCG64(7))
    sizes = np.rint(np.exp(rng.uniform(np.log(100), np.log(1 << 20), 60))).astype(int)
    jobs = []
    for n in sizes:
        start = int(rng.integers(0, pool.shape[0] - n + 1))
        jobs.append((pool[start:start + n], datagen.mean_spacing_eps(int(n)),
                     int(rng.choice([2, 5, 10]))))
    srv = dbx.Server(0, slots=3, batch_cut=1 << 15)
    tickets = [srv.submit(p, float(e), m) for p, e, m in jobs]
    for t in tickets:
        assert srv.wait(t, 120.0) == 0
    st = srv.stats()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["batches"] >= 1  # small jobs were batched
    ctx = dbx.Context(0)
    for t, (p, e, m) in zip(tickets, jobs):
        alone = ctx.cluster(torch.from_numpy(np.ascontiguousarray(p)).cuda(), float(e), m)
        np.testing.assert_array_equal(srv.labels(t), alone.cpu().numpy())
        if p.shape[0] <= 50000:
            np.testing.assert_array_equal(srv.labels(t), oracle.dbscan(p, F32(e), m))
    srv.close()
    ctx.close()


def test_nonfinite_job_fails_alone_in_a_batch():
    srv = dbx.Server(0, slots=1, batch_cut=1 << 20)
    big = datagen.clumps(1 << 20, 3)
    good = [datagen.clumps(2000, 10 + k) for k in range(6)]
    bad = datagen.clumps(2000, 99)
    bad[17, 2] = np.nan
    t_big = srv.submit(big, 0.002, 2)          # keeps the slot busy while the rest queue
    tg = [srv.submit(p, 0.02, 3) for p in good[:3]]
    tb = srv.submit(bad, 0.02, 3)
    tg += [srv.submit(p, 0.02, 3) for p in good[3:]]
    assert srv.wait(t_big, 120.0) == 0
    assert srv.wait(tb, 120.0) == -2
    for t, p in zip(tg, good):
        assert srv.wait(t, 120.0) == 0
        np.testing.assert_array_equal(srv.labels(t), oracle.dbscan(p, F32(0.02), 3))
    srv.close()
