"""Host logic of the serving loop, on the CPU with a stand-in executor: batch
formation by class and arrival order, the query cap, memory-based admission,
continuous batching (a request that arrives while a batch runs is served by
another worker without waiting for it), routing of answers, the seeded
Poisson request stream and the latency report."""
import threading
import time

import numpy as np
import pytest

from paper_2510_00566_amd.serving import Request, Scheduler, Server, latency_report, poisson_requests, replay


def _req(rid, index="a", m=4, k=10, nprobe=16, t=0.0, d=8):
    q = np.full((m, d), float(rid), dtype=np.float32)
    q[:, 1] = np.arange(m)
    return Request(rid=rid, index=index, queries=q, k=k, nprobe=nprobe, arrival=t)


def _echo(delay=0.0, log=None):
    """Stand-in for the GPU: each query's answer encodes (request id, row)."""
    def run(wid, b):
        if log is not None:
            log.append((wid, b.bid, b.index, b.k, [r.rid for r in b.requests], time.perf_counter()))
        if delay:
            time.sleep(delay)
        outs = []
        for r in b.requests:
            ids = np.repeat((r.queries[:, 0].astype(np.int64) * 1000 + r.queries[:, 1].astype(np.int64))[:, None],
                            r.k, axis=1)
            outs.append((ids, np.zeros((r.m, r.k), np.float32)))
        return outs
    return run


def test_batches_by_class_in_arrival_order():
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30, max_batch_queries=10)
    reqs = [_req(0, "a", 4, 10, t=0.0), _req(1, "b", 4, 10, t=0.1), _req(2, "a", 4, 100, t=0.2),
            _req(3, "a", 4, 10, t=0.3), _req(4, "a", 4, 10, t=0.4), _req(5, "b", 4, 10, t=0.5)]
    for r in reqs:
        sched.submit(r)
    sched.close()
    got = []
    while True:
        b = sched.next_batch()
        if b is None:
            break
        got.append((b.index, b.k, [r.rid for r in b.requests]))
        sched.finish(b)
    # oldest head first; within a class, arrival order; at most 10 queries
    assert got == [("a", 10, [0, 3]), ("b", 10, [1, 5]), ("a", 100, [2]), ("a", 10, [4])]


def test_admission_keeps_memory_in_flight_within_budget():
    cost = lambda i, nq, k: 100 * nq  # noqa: E731
    sched = Scheduler(cost, budget=5000, max_batch_queries=64)
    srv = Server(sched, _echo(delay=0.01), n_workers=4)
    reqs = [_req(i, "a" if i % 2 else "b", m=1 + (i % 17), t=0.0) for i in range(60)]
    for r in reqs:
        sched.submit(r)
    sched.close()
    srv.start()
    srv.join()
    assert len(srv.completed) == 60
    assert sched.peak_inflight <= 5000
    assert sched.inflight == 0
    assert all(b[4] <= 50 for b in srv.batches)


def test_oversized_request_runs_alone():
    sched = Scheduler(lambda i, nq, k: 100 * nq, budget=500, max_batch_queries=4096)
    srv = Server(sched, _echo(), n_workers=2)
    sched.submit(_req(0, m=20))
    sched.submit(_req(1, m=2))
    sched.close()
    srv.start()
    srv.join()
    assert sorted(len(b) for b in [[r for r in srv.completed if r.batch == x[0]] for x in srv.batches]) == [1, 1]


def test_answers_are_routed_to_their_request():
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30, max_batch_queries=100)
    srv = Server(sched, _echo(), n_workers=3)
    reqs = [_req(i, "ab"[i % 2], m=1 + i % 9, k=(10, 100)[i % 3 == 0], t=0.0) for i in range(40)]
    for r in reqs:
        sched.submit(r)
    sched.close()
    srv.start()
    srv.join()
    assert sorted(r.rid for r in srv.completed) == list(range(40))
    for r in reqs:
        assert r.ids.shape == (r.m, r.k)
        assert (r.ids[:, 0] == r.rid * 1000 + np.arange(r.m)).all()


def test_requests_arriving_during_a_batch_overlap_it():
    log = []
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30, max_batch_queries=100)
    srv = Server(sched, _echo(delay=0.2, log=log), n_workers=2)
    srv.start()
    sched.submit(_req(0, t=time.perf_counter()))
    time.sleep(0.05)
    sched.submit(_req(1, t=time.perf_counter()))
    sched.close()
    srv.join()
    (w0, b0, *_r0, t0), (w1, b1, *_r1, t1) = sorted(log, key=lambda e: e[-1])
    assert w0 != w1
    assert t1 - t0 < 0.2  # the second batch started before the first finished
    r0, r1 = sorted(srv.completed, key=lambda r: r.rid)
    assert r1.start < r0.done


def test_poisson_stream_is_seeded_and_has_the_rate():
    pools = {"a": np.zeros((100, 4), np.float32), "b": np.ones((100, 6), np.float32)}
    s1 = poisson_requests(pools, rate=1000.0, duration=2.0, seed=3)
    s2 = poisson_requests(pools, rate=1000.0, duration=2.0, seed=3)
    assert [(r.index, r.m, r.k, r.nprobe, r.arrival) for r in s1] == [(r.index, r.m, r.k, r.nprobe, r.arrival)
                                                                      for r in s2]
    assert 1800 < len(s1) < 2200
    assert all(1 <= r.m <= 256 and r.k in (10, 100) and r.nprobe in (16, 64) for r in s1)
    assert all(r.queries.shape[1] == (4 if r.index == "a" else 6) for r in s1)
    gaps = np.diff([r.arrival for r in s1])
    assert abs(gaps.mean() - 1e-3) < 1e-4


def test_replay_and_latency_report():
    pools = {"a": np.zeros((50, 4), np.float32)}
    reqs = poisson_requests(pools, rate=400.0, duration=0.25, seed=5, sizes=(1, 8))
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30)
    srv = Server(sched, _echo(delay=0.002), n_workers=2)
    replay(srv, reqs)
    rep = latency_report(reqs)
    assert rep["requests"] == len(reqs)
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs])
    assert (lat > 0).all()
    assert rep["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert rep["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert rep["queries"] == sum(r.m for r in reqs)


def test_failed_batch_does_not_stop_the_server():
    def flaky(wid, b):
        if any(r.rid == 3 for r in b.requests):
            raise RuntimeError("device error")
        return _echo()(wid, b)
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30, max_batch_queries=1)
    srv = Server(sched, flaky, n_workers=2)
    for i in range(6):
        sched.submit(_req(i, m=1))
    sched.close()
    srv.start()
    srv.join()
    assert len(srv.completed) == 6 and len(srv.errors) == 1
    assert [r.ids is None for r in sorted(srv.completed, key=lambda r: r.rid)] == [False] * 3 + [True] + [False] * 2


class _FakeCtxExecutor:
    """Stand-in executor with a context memory model like the library's: a
    batch of cost c grows the worker's resident scratch to at least c (by
    1.25x when it grows) and nothing shrinks it but trim()."""

    def __init__(self, n_workers, cost, delay=0.002):
        self.res = [0] * n_workers
        self.cost = cost
        self.delay = delay
        self.lock = threading.Lock()
        self.samples = []
        self.trims = 0

    def __call__(self, wid, b):
        need = self.cost(b.index, b.nq, b.k)
        with self.lock:
            if need > self.res[wid]:
                self.res[wid] = int(need * 1.25)
            self.samples.append(sum(self.res))
        time.sleep(self.delay)
        return _echo()(wid, b)

    def resident(self, wid):
        return self.res[wid]

    def trim(self, wid):
        with self.lock:
            self.res[wid] = 0
            self.trims += 1


def test_resident_scratch_stays_within_budget():
    """Memory admission counts the scratch the workers' contexts keep after
    their batches: the sum of resident bytes never exceeds the budget."""
    cost = lambda i, nq, k: 1000 * nq  # noqa: E731
    budget = 120_000
    ex = _FakeCtxExecutor(3, cost)
    sched = Scheduler(cost, budget=budget, max_batch_queries=64)
    srv = Server(sched, ex, n_workers=3)
    g = np.random.Generator(np.random.PCG64(5))
    reqs = [_req(i, "a" if i % 3 else "b", m=int(g.integers(1, 60)), t=0.0) for i in range(120)]
    for r in reqs:
        sched.submit(r)
    sched.close()
    srv.start()
    srv.join()
    assert len(srv.completed) == 120 and not srv.errors
    assert max(ex.samples) <= budget
    assert sched.peak_inflight <= budget
    assert sched.busy == 0
    # what the scheduler still charges is what the contexts keep
    assert sched.inflight == sum(ex.res)
    # a worker above its share (budget / 3) trims after its batch
    assert all(r <= budget // 3 for r in ex.res)


def test_full_queue_rejects_at_arrival():
    """max_queued bounds the waiting queries: a request that would exceed it
    is refused at arrival and counted; served requests leave room again."""
    sched = Scheduler(lambda i, nq, k: nq, budget=1 << 30, max_batch_queries=64, max_queued=10)
    a, b, c = _req(0, m=6), _req(1, m=4), _req(2, m=1)
    assert sched.submit(a) and sched.submit(b)
    assert not sched.submit(c) and c.rejected and sched.rejected == 1
    bt = sched.next_batch(0)
    assert [r.rid for r in bt.requests] == [0, 1]
    d = _req(3, m=10)
    assert sched.submit(d) and not d.rejected
    rep = latency_report([a, b, c, d])
    assert rep["rejected"] == 1


def test_request_waiting_for_memory_is_counted_deferred():
    """The head request does not fit beside a batch in flight: it waits (is
    deferred) and runs once that batch finishes and releases its memory."""
    sched = Scheduler(lambda i, nq, k: 100 * nq, budget=1000, max_batch_queries=64, growth=1.0)
    sched.submit(_req(0, m=6))
    first = sched.next_batch(0)
    late = _req(1, m=6)
    sched.submit(late)
    got = []
    t = threading.Thread(target=lambda: got.append(sched.next_batch(1)))
    t.start()
    time.sleep(0.2)
    assert not got and late.deferred and sched.deferred == 1
    sched.finish(first, resident=0)
    t.join(timeout=5)
    assert got and [r.rid for r in got[0].requests] == [1]
    assert latency_report([late])["deferred"] == 1


def test_trim_that_leaves_memory_is_asked_once():
    """A context whose trim cannot release everything (worker 0 keeps 3000
    bytes): when worker 1's batch does not fit beside it, worker 0 is asked to
    trim once, then runs the batch itself (it fits there), instead of being
    asked to trim again and again."""
    sched = Scheduler(lambda i, nq, k: 1000 * nq, budget=10_000, max_batch_queries=64, growth=1.0)
    sched.submit(_req(0, m=3))
    sched.finish(sched.next_batch(0), resident=3000)
    log, got1 = [], []

    def worker0():
        while True:
            b = sched.next_batch(0)
            if b is None:
                return
            if b.trim:
                log.append("trim")
                sched.finish(b, resident=3000)
                if log.count("trim") > 3:
                    sched.close()
                    return
                continue
            log.append(("batch", [r.rid for r in b.requests]))
            sched.finish(b, resident=3000)
            sched.close()
            return

    def worker1():
        # the request arrives and worker 1 looks at it before worker 0 wakes
        with sched._lock:
            sched.submit(_req(1, m=8))
            got1.append(sched.next_batch(1))

    a = threading.Thread(target=worker0, daemon=True)
    a.start()
    for _ in range(500):
        if 0 in sched._idle:
            break
        time.sleep(0.01)
    b = threading.Thread(target=worker1, daemon=True)
    b.start()
    a.join(timeout=10)
    b.join(timeout=10)
    assert log == ["trim", ("batch", [1])]
    assert got1 == [None] and sched.deferred == 1


def test_batch_runs_beside_memory_left_after_trims():
    """Both workers keep 3000 bytes that no trim releases; a 9000-byte batch
    does not fit beside the other's 3000 under a 10000 budget.  Once each
    worker has trimmed, nothing more can be released, so the batch runs
    (over the budget by that memory only) instead of both workers waiting
    for ever."""
    sched = Scheduler(lambda i, nq, k: 1000 * nq, budget=10_000, max_batch_queries=64, growth=1.0)
    for wid in (0, 1):
        sched.submit(_req(wid, m=3))
        sched.finish(sched.next_batch(wid), resident=3000)
    log = []

    def worker(wid):
        while True:
            b = sched.next_batch(wid)
            if b is None:
                return
            if b.trim:
                log.append(("trim", wid))
                sched.finish(b, resident=3000)
                continue
            log.append(("batch", [r.rid for r in b.requests]))
            sched.finish(b, resident=3000)
            sched.close()

    ts = [threading.Thread(target=worker, args=(w,), daemon=True) for w in (0, 1)]
    for t in ts:
        t.start()
    for _ in range(500):
        if sched._idle == {0, 1}:
            break
        time.sleep(0.01)
    sched.submit(_req(2, m=9))
    for t in ts:
        t.join(timeout=10)
    assert not any(t.is_alive() for t in ts), f"workers still waiting: {log}"
    assert [e for e in log if e[0] == "batch"] == [("batch", [2])]
    assert len([e for e in log if e[0] == "trim"]) <= 2
