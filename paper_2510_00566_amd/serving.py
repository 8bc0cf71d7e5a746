"""Serving loop over resident indexes: continuous batching with memory-based
admission.

Requests (a few queries each, with their own k, probe count and index)
arrive at any time.  Worker threads each own a search context (its own HIP
streams and scratch memory), so several batches are on the GPU at once.  A
worker that becomes free forms the next batch at once from the requests
waiting at that moment: the class (index, k) of the oldest waiting request,
then that class's requests in arrival order, up to a query cap and within
the memory budget left by the batches already in flight.  Requests that
arrive while batches run join the next batch formed; no batch waits for a
fixed window.  Probe counts may differ inside a batch (a per-query probe
array), k may not (k sets the result shape).

Memory admission counts what stays allocated, not only what a batch uses: a
worker's context keeps its scratch at the largest size it has needed (grown
by the library's factor of 1.25), so the scheduler charges each worker its
resident scratch, raises the charge when a batch may grow it, and lowers it
only when the worker reports a smaller resident size after trimming its
context.  A worker whose context holds more than its share of the budget
(budget / workers) after a batch trims it.

The search itself is exact at eps = 1, so a request's answer does not depend
on which other requests share its batch; ``tests/test_gpu_serving.py`` checks
that.  Everything here is host-side orchestration (threads, queues,
accounting); each batch is one ``pano_search_ctx`` call.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    index: str
    queries: np.ndarray       # [m, d] float32
    k: int
    nprobe: int
    arrival: float = 0.0      # seconds, on the server clock
    start: float = -1.0       # when its batch was launched
    done: float = -1.0        # when its answer was ready on the host
    ids: np.ndarray | None = None
    dists: np.ndarray | None = None
    batch: int = -1           # id of the batch that served it
    deferred: bool = False    # waited at the head of the queue for memory
    rejected: bool = False    # refused at arrival: the queue was full

    @property
    def m(self) -> int:
        return int(self.queries.shape[0])


@dataclasses.dataclass
class Batch:
    bid: int
    index: str
    k: int
    requests: list
    bytes: int
    worker: int = 0
    prev_charge: int = 0
    trim: bool = False       # no requests: the worker releases its context's memory

    @property
    def nq(self) -> int:
        return sum(r.m for r in self.requests)


class Scheduler:
    """Thread-safe admission and batch formation (no GPU here).

    cost(index, nq, k) -> bytes of device memory a batch of nq queries needs
    while in flight.  Each worker is charged its resident bytes: a batch of
    cost c on worker w raises w's charge to max(charge_w, growth * c), and
    budget caps the sum of the charges of all workers.  finish() sets the
    worker's charge to the resident size it reports (0 after a trim).  A
    single request that cannot fit even when no other batch is in flight is
    still admitted alone (it could never run otherwise), and so is a batch
    that does not fit beside memory the other workers keep after a trim; the
    budget is then exceeded by that batch only.  max_queued (queries, None: no limit)
    bounds the waiting queue: a request that would exceed it is rejected at
    arrival (back-pressure instead of unbounded queueing).  A request that
    reaches the head of the queue but must wait for memory held by other
    batches is counted as deferred."""

    def __init__(self, cost: Callable[[str, int, int], int], budget: int, max_batch_queries: int = 4096,
                 growth: float = 1.25, max_queued: int | None = None):
        self.cost = cost
        self.budget = int(budget)
        self.max_q = int(max_batch_queries)
        self.growth = float(growth)
        self.max_queued = None if max_queued is None else int(max_queued)
        self._queued = 0  # queries waiting
        self.rejected = 0
        self.deferred = 0
        self._lock = threading.Condition()
        self._queues: dict = collections.OrderedDict()  # (index, k) -> deque of Request
        self._charge: dict = {}  # worker id -> bytes charged for its context
        self._busy = 0  # batches in flight
        self._idle: set = set()  # workers waiting in next_batch
        self._pressure = False  # idle workers holding memory should trim
        self._trimmed: set = set()  # workers that trimmed for the current shortage
        self._peak = 0
        self._closed = False
        self._next_bid = 0

    # ---- producer side
    def submit(self, req: Request) -> bool:
        """Queue a request; False (and req.rejected) if the queue is full."""
        with self._lock:
            if self.max_queued is not None and self._queued + req.m > self.max_queued:
                req.rejected = True
                self.rejected += 1
                return False
            self._queued += req.m
            key = (req.index, req.k)
            self._queues.setdefault(key, collections.deque()).append(req)
            self._lock.notify_all()
            return True

    def close(self):
        """No more requests will be submitted; workers drain and stop."""
        with self._lock:
            self._closed = True
            self._lock.notify_all()

    # ---- worker side
    def _oldest_class(self):
        """The class whose first waiting request is the oldest (arrival, rid)."""
        best, best_head = None, None
        for key, q in self._queues.items():
            if q and (best_head is None or (q[0].arrival, q[0].rid) < best_head):
                best, best_head = key, (q[0].arrival, q[0].rid)
        return best

    def _charged_with(self, wid: int, need: int) -> int:
        """Total charge if worker wid runs a batch of cost `need`."""
        mine = max(self._charge.get(wid, 0), int(self.growth * need))
        return sum(v for w, v in self._charge.items() if w != wid) + mine

    def next_batch(self, wid: int = 0) -> Batch | None:
        """Block until a batch can be formed and admitted for worker wid;
        None when closed and drained.  Returns a batch without requests
        (trim=True) when the worker should release its context's memory
        first: another worker's batch does not fit beside the memory that
        idle workers keep."""
        with self._lock:
            self._idle.add(wid)
            try:
                return self._next_locked(wid)
            finally:
                self._idle.discard(wid)

    def _next_locked(self, wid: int) -> Batch | None:
        while True:
            if self._pressure and self._charge.get(wid, 0) > 0 and wid not in self._trimmed:
                # asked to make room: release this context's memory (once
                # per shortage: what a trim leaves, a second one leaves too)
                self._trimmed.add(wid)
                b = Batch(-1, "", 0, [], 0, worker=wid, prev_charge=self._charge[wid], trim=True)
                self._busy += 1
                return b
            key = self._oldest_class()
            if key is None:
                if self._closed:
                    return None
                self._lock.wait()
                continue
            q = self._queues[key]
            index, k = key
            # memory other workers could still release (what is left after a
            # trim stays: waiting for it would wait for ever)
            others_hold = any(v > 0 for w, v in self._charge.items() if w != wid and w not in self._trimmed)
            take, nq = [], 0
            while q and (not take or nq + q[0].m <= self.max_q):
                cand = nq + q[0].m
                need = self.cost(index, cand, k)
                if self._charged_with(wid, need) > self.budget and (take or self._busy > 0 or others_hold):
                    break
                take.append(q.popleft())
                nq = cand
            if not take:
                # the oldest class does not fit beside the memory the other
                # workers hold: idle ones are asked to trim, busy ones may
                # trim when they finish
                if not q[0].deferred:
                    q[0].deferred = True
                    self.deferred += 1
                if any(self._charge.get(w, 0) > 0 for w in self._idle if w != wid and w not in self._trimmed):
                    self._pressure = True
                self._lock.notify_all()
                self._lock.wait()
                continue
            self._pressure = False
            self._trimmed.clear()
            self._queued -= nq
            need = self.cost(index, nq, k)
            prev = self._charge.get(wid, 0)
            self._charge[wid] = max(prev, int(self.growth * need))
            self._busy += 1
            self._peak = max(self._peak, sum(self._charge.values()))
            b = Batch(self._next_bid, index, k, take, need, worker=wid, prev_charge=prev)
            self._next_bid += 1
            return b

    def finish(self, batch: Batch, resident: int | None = None):
        """Batch done; resident: the bytes its worker's context now keeps
        (None: an executor that keeps nothing between batches, so the charge
        returns to what it was before the batch)."""
        with self._lock:
            self._busy -= 1
            self._charge[batch.worker] = int(resident) if resident is not None else batch.prev_charge
            self._lock.notify_all()

    def share(self, n_workers: int) -> int:
        """Resident bytes a worker may keep between batches."""
        return self.budget // max(1, n_workers)

    @property
    def peak_inflight(self) -> int:
        """Largest total charge seen (bytes)."""
        return self._peak

    @property
    def inflight(self) -> int:
        """Current total charge (bytes), resident memory of idle workers included."""
        with self._lock:
            return sum(self._charge.values())

    @property
    def busy(self) -> int:
        return self._busy


class Server:
    """Worker threads that pull batches from a Scheduler and run them with
    execute(worker_id, batch) -> list of (ids, dists) per request.  If the
    executor has resident(wid) and trim(wid), a worker reports its context's
    resident bytes after each batch and trims the context first when it holds
    more than its share of the budget."""

    def __init__(self, scheduler: Scheduler, execute: Callable, n_workers: int = 3,
                 clock: Callable[[], float] = time.perf_counter):
        self.sched = scheduler
        self.execute = execute
        self.clock = clock
        self.n_workers = n_workers
        self.completed: list = []
        self.batches: list = []
        self._lock = threading.Lock()
        self._threads = []
        self.errors: list = []

    def _resident_after(self, wid: int):
        ex = self.execute
        if not (hasattr(ex, "resident") and hasattr(ex, "trim")):
            return None
        r = ex.resident(wid)
        if r > self.sched.share(self.n_workers):
            ex.trim(wid)
            r = ex.resident(wid)
        return r

    def _run(self, wid: int):
        while True:
            b = self.sched.next_batch(wid)
            if b is None:
                return
            if b.trim:
                ex = self.execute
                if hasattr(ex, "trim"):
                    ex.trim(wid)
                self.sched.finish(b, ex.resident(wid) if hasattr(ex, "resident") else 0)
                continue
            t0 = self.clock()
            for r in b.requests:
                r.start = t0
                r.batch = b.bid
            try:
                outs = self.execute(wid, b)
            except Exception as e:  # a failed batch fails its requests, not the server
                with self._lock:
                    self.errors.append((b.bid, repr(e)))
                outs = [(None, None)] * len(b.requests)
            t1 = self.clock()
            for r, (ids, dd) in zip(b.requests, outs):
                r.ids, r.dists, r.done = ids, dd, t1
            self.sched.finish(b, self._resident_after(wid))
            with self._lock:
                self.completed.extend(b.requests)
                self.batches.append((b.bid, wid, b.index, b.k, b.nq, t0, t1))

    def start(self):
        for w in range(self.n_workers):
            t = threading.Thread(target=self._run, args=(w,), daemon=True)
            t.start()
            self._threads.append(t)

    def join(self):
        for t in self._threads:
            t.join()


def poisson_requests(pools: dict, rate: float, duration: float, seed: int, sizes=(1, 256), ks=(10, 100),
                     nprobes=(16, 64)) -> list:
    """Seeded open-loop request stream: Poisson arrivals at `rate` requests/s
    over `duration` s; each request draws an index from `pools`
    (name -> query array), a size uniform in [sizes[0], sizes[1]], a k and a
    probe count uniformly from the given sets, and its queries from the
    pool."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20251001, 77, seed])))
    names = sorted(pools)
    reqs, t, rid = [], 0.0, 0
    while True:
        t += g.exponential(1.0 / rate)
        if t > duration:
            break
        name = names[int(g.integers(len(names)))]
        pool = pools[name]
        m = int(g.integers(sizes[0], sizes[1] + 1))
        rows = g.integers(0, pool.shape[0], size=m)
        reqs.append(Request(rid=rid, index=name, queries=np.ascontiguousarray(pool[rows]),
                            k=int(ks[int(g.integers(len(ks)))]), nprobe=int(nprobes[int(g.integers(len(nprobes)))]),
                            arrival=t))
        rid += 1
    return reqs


def replay(server: Server, reqs: list, clock: Callable[[], float] = time.perf_counter,
           sleep: Callable[[float], None] = time.sleep) -> float:
    """Submit each request at its arrival offset from now (open loop), then
    close the scheduler and wait for the workers.  Arrival times are
    rewritten to the server clock.  Returns the clock value at the start."""
    t0 = clock()
    server.start()
    for r in sorted(reqs, key=lambda r: (r.arrival, r.rid)):
        wait = t0 + r.arrival - clock()
        if wait > 0:
            sleep(wait)
        r.arrival = t0 + r.arrival
        server.sched.submit(r)
    server.sched.close()
    server.join()
    return t0


def latency_report(reqs: list) -> dict:
    """p50 / p99 / mean latency (ms, arrival to answer) and throughput over
    the served requests."""
    lat = np.array([(r.done - r.arrival) * 1e3 for r in reqs if r.done >= 0])
    nq = sum(r.m for r in reqs if r.done >= 0)
    counts = {"rejected": sum(1 for r in reqs if r.rejected), "deferred": sum(1 for r in reqs if r.deferred)}
    if lat.size == 0:
        return {"requests": 0, **counts}
    t_first = min(r.arrival for r in reqs)
    t_last = max(r.done for r in reqs if r.done >= 0)
    span = max(t_last - t_first, 1e-9)
    return {"requests": int(lat.size), "queries": int(nq),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "qps": float(nq / span), "rps": float(lat.size / span), "span_s": float(span), **counts}


# ---------------------------------------------------------------- GPU executor
class GpuExecutor:
    """Runs a batch as one search on the worker's own context and stream.

    indexes: name -> Index; params: name -> search Params (None: library
    defaults).  One Context and one torch stream per worker."""

    def __init__(self, indexes: dict, n_workers: int, device: int = 0, params: dict | None = None,
                 nprobe_max: int = 64):
        import torch
        from .index import Context
        self.indexes = indexes
        self.params = params or {}
        self.ctxs = [Context(device) for _ in range(n_workers)]
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_workers)]
        self.device = device
        self.nprobe_max = int(nprobe_max)

    def cost(self, index: str, nq: int, k: int) -> int:
        idx = self.indexes[index]
        d = idx.d
        io = nq * (d * 4 + 4 + k * 12)  # queries, probe counts, ids + dists
        return int(idx.scratch_bytes(nq, k, nprobe=self.nprobe_max, per_query_nprobe=True,
                                     params=self.params.get(index)) + io)

    def resident(self, wid: int) -> int:
        """Device bytes worker wid's context keeps for search scratch (the
        batch's query and result tensors are charged while it runs)."""
        return int(self.ctxs[wid].scratch_bytes())

    def trim(self, wid: int):
        self.ctxs[wid].trim()

    def __call__(self, wid: int, b: Batch):
        import torch
        idx = self.indexes[b.index]
        st = self.streams[wid]
        q = np.concatenate([r.queries for r in b.requests]).astype(np.float32, copy=False)
        npr = np.concatenate([np.full(r.m, r.nprobe, dtype=np.int32) for r in b.requests])
        with torch.cuda.stream(st):
            qd = torch.from_numpy(q).to(f"cuda:{self.device}", non_blocking=False)
            npd = torch.from_numpy(npr).to(f"cuda:{self.device}", non_blocking=False)
            # batch shapes vary from call to call: launch eagerly rather than
            # capture a graph per shape
            ids, dd = idx.search(qd, b.k, nprobe=npd, ctx=self.ctxs[wid], stream=st, eager=True,
                                 params=self.params.get(b.index), nprobe_max=self.nprobe_max)
            ids_h = ids.cpu().numpy()
            dd_h = dd.cpu().numpy()
        outs, o = [], 0
        for r in b.requests:
            outs.append((ids_h[o:o + r.m].copy(), dd_h[o:o + r.m].copy()))
            o += r.m
        return outs


def main(argv=None):
    import argparse
    import json
    import sys

    import torch

    from . import autotune, synth
    from .index import Context, Index, Transform, ivf_assign

    ap = argparse.ArgumentParser(description="continuous-batching serving loop over two resident indexes")
    ap.add_argument("--qps", type=float, nargs="+", default=[2000.0, 5000.0, 10000.0, 20000.0, 50000.0],
                    help="offered loads in queries per second (Poisson request arrivals, mean request size "
                         "128.5 queries); one JSON line per load")
    ap.add_argument("--duration", type=float, default=60.0, help="seconds of arrivals per load")
    ap.add_argument("--max-queued", type=int, default=262144,
                    help="queries waiting at most; requests beyond are rejected at arrival")
    ap.add_argument("--c4-store", default="bf16", choices=["f32", "bf16"],
                    help="level storage of the embedding-shaped index")
    ap.add_argument("--scale", type=float, default=0.1, help="fraction of each index's N")
    ap.add_argument("--workers", type=int, default=3)
    ap.add_argument("--budget-gib", type=float, default=8.0)
    ap.add_argument("--max-batch", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ctx = Context(0)
    indexes, pools, params = {}, {}, {}
    for name, wname in (("c3", "ivf_zipf_batched"), ("c4", "ivf_embed_bf16")):
        w0 = synth.WORKLOADS[wname]
        w = synth.scaled(w0, n=int(w0.n * args.scale), nq=4096,
                         nlist=max(64, int(w0.nlist * args.scale)),
                         n_clusters=max(64, int(w0.n_clusters * args.scale)) if w0.n_clusters else 0)
        t = time.time()
        data = synth.generate(w)
        xd = torch.from_numpy(data["x"]).cuda()
        cent, assign = ivf_assign(ctx, xd, w.nlist, iters=8, seed=w.cfg_id)
        rows = np.random.Generator(np.random.PCG64(w.cfg_id)).choice(w.n, min(w.n, 65536), replace=False)
        c_np, a_np = cent.cpu().numpy(), assign.cpu().numpy()
        tf = Transform.fit(data["x"][rows] - c_np[a_np[rows]], fit_sample=0, seed=w.cfg_id)
        store = args.c4_store if name == "c4" else "f32"
        # the tuner's choice (search knobs and level width) for the workload
        # this index is shaped like and its storage type
        npv = w0.nprobe_range[1] if w0.nprobe_range else w0.nprobe
        p, width = autotune.lookup(autotune.signature("gfx950", w.d, store, w.n, npv, w0.k))
        if p is not None:
            p.use_bf16 = 1 if store == "bf16" else 0
            params[name] = p
        if width and w.tune_width:
            w.level_width = int(width)
        indexes[name] = Index.build(ctx, tf, xd, cent, assign, w.level_cuts(), store=store)
        pools[name] = data["q"]
        del xd
        torch.cuda.synchronize()
        log(f"[serve] index {name}: n={w.n} d={w.d} nlist={w.nlist} {store} built in {time.time() - t:.1f}s")

    log(f"[serve] search params {params}")
    ex = GpuExecutor(indexes, args.workers, params=params)
    # warm every context on both indexes (first-use allocations)
    warm = poisson_requests(pools, 200.0, 0.05, args.seed + 1000, sizes=(1, 64))
    srv = Server(Scheduler(ex.cost, int(args.budget_gib * 2 ** 30), args.max_batch), ex, n_workers=args.workers)
    replay(srv, warm)
    for qps in args.qps:
        rate = qps / 128.5
        sched = Scheduler(ex.cost, int(args.budget_gib * 2 ** 30), args.max_batch, max_queued=args.max_queued)
        srv = Server(sched, ex, n_workers=args.workers)
        reqs = poisson_requests(pools, rate, args.duration, args.seed)
        log(f"[serve] offered {qps:.0f} q/s: {len(reqs)} requests, {sum(r.m for r in reqs)} queries "
            f"over {args.duration}s")
        replay(srv, reqs)
        rep = latency_report(reqs)
        rep["by_index"] = {n: {k_: v_ for k_, v_ in latency_report([r for r in reqs if r.index == n]).items()
                               if k_ in ("requests", "p50_ms", "p99_ms", "qps")} for n in indexes}
        rep.update({"offered_qps": qps, "workers": args.workers, "rate_rps": rate, "batches": len(srv.batches),
                    "mean_batch_queries": float(np.mean([b[4] for b in srv.batches])) if srv.batches else 0.0,
                    "peak_inflight_gib": sched.peak_inflight / 2 ** 30, "errors": len(srv.errors),
                    "duration_s": args.duration, "max_queued": args.max_queued,
                    "stores": {n: ("bf16" if (n == "c4" and args.c4_store == "bf16") else "f32") for n in indexes},
                    "params": {n: vars(p) for n, p in params.items()},
                    "scale": args.scale, "indexes": {n: {"n": int(ix.info()["n"]), "d": ix.d}
                                                     for n, ix in indexes.items()}})
        print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
