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


def test_trace_segment_every_small_job_against_the_oracle():
    """The serving trace's first 2 seconds (about 400 jobs of the 60 s
    workload: log-uniform sizes, minPts 2/5/10, windows of the clump pools)
    through the continuous-batching server: every job of at most 10^6
    points and 10 random larger ones against the oracle, and 40 random jobs
    identical alone (one slot, no batching) and in the mix."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    jobs = [j for j in datagen.serving_trace() if j.t_arrival < 2.0]
    pools = {}
    for j in jobs:
        if j.pool not in pools:
            pools[j.pool] = datagen.serving_pool(j.pool)
    rng = np.random.default_rng(61)
    sizes = np.array([j.n for j in jobs])
    small = np.flatnonzero(sizes <= 10 ** 6)
    large = rng.choice(np.flatnonzero(sizes > 10 ** 6), 10, replace=False)
    print(f"[serving] {len(jobs)} jobs, {small.size} small, {sizes.sum()} points", flush=True)
    mix = dbx.Server(0, slots=4, budget_bytes=200 * 10 ** 9)
    tickets = [mix.submit(pools[j.pool][j.start:j.start + j.n], float(j.eps), j.min_pts)
               for j in jobs]
    for t in tickets:
        assert mix.wait(t, 300.0) == 0
    assert mix.stats()["batched_jobs"] > 0
    threads = min(16, os.cpu_count() or 1)

    def bad(k):
        j = jobs[k]
        ref = oracle.dbscan(pools[j.pool][j.start:j.start + j.n], j.eps, j.min_pts)
        return int((ref != mix.labels(tickets[k])).sum())

    with ThreadPoolExecutor(max_workers=threads) as ex:
        wrong = list(ex.map(bad, sorted(np.concatenate([small, large]).tolist(),
                                        key=lambda k: -jobs[k].n)))
    assert sum(wrong) == 0
    solo = dbx.Server(0, slots=1, batch_cut=1)
    for k in rng.choice(len(jobs), 40, replace=False):
        j = jobs[k]
        t = solo.submit(pools[j.pool][j.start:j.start + j.n], float(j.eps), j.min_pts)
        assert solo.wait(t, 300.0) == 0
        np.testing.assert_array_equal(solo.labels(t), mix.labels(tickets[k]))
    solo.close()
    mix.close()


def test_tight_budget_releases_idle_slots():
    """Under a budget of about two of the largest jobs, four slots that keep
    their memory between jobs must give it back for each other (idle slots
    free their arenas on the device): every job completes, the slots never
    hold more than the budget, and the labels are the oracle's."""
    lib = dbx.load_library()
    sizes = [300_000, 40_000, 250_000, 5_000, 300_000, 120_000, 60_000, 280_000, 2_000, 200_000]
    jobs = [(datagen.clumps(n, 70 + k), F32(0.004), [2, 5, 10][k % 3]) for k, n in
            enumerate(sizes)]
    big = max(lib.dbscan_scratch_bytes(n, 5, 1) for n in sizes) + max(sizes) * 16
    budget = int(big * 2.3)
    srv = dbx.Server(0, slots=4, budget_bytes=budget, batch_cut=1)
    tickets = [srv.submit(p, float(e), m) for p, e, m in jobs]
    for t in tickets:
        assert srv.wait(t, 120.0) == 0
    st = srv.stats()
    assert st["failed"] == 0 and 0 < st["peak_in_flight_bytes"] <= budget
    for t, (p, e, m) in zip(tickets, jobs):
        np.testing.assert_array_equal(srv.labels(t), oracle.dbscan(p, e, m))
    srv.close()
