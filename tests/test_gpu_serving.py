"""The serving loop on the GPU: two resident indexes (a d = 128 Zipf-list
index and a d = 768 unit-norm index), requests of mixed index, k and probe
count served by three workers with their own contexts, so batches overlap on
the device.  Each request's answer in the mix must equal the answer of the
same request searched alone (bit for bit), and a sample must equal the
oracle's."""
import sys

import numpy as np
import pytest

from paper_2510_00566_amd import synth

gpu = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@gpu
def test_mixed_requests_equal_their_alone_answers():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Context
    from paper_2510_00566_amd.serving import GpuExecutor, Scheduler, Server, poisson_requests, replay, latency_report

    specs = {
        "c3": synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=20000, nq=256, nlist=32, n_clusters=32),
        "c4": synth.scaled(synth.WORKLOADS["ivf_embed_bf16"], n=12000, nq=256, nlist=24),
    }
    cases, pools = {}, {}
    for name, w in specs.items():
        _log(f"case serving index {name}: n={w.n} d={w.d} nlist={w.nlist}")
        cases[name] = gc.build_case(w)
        pools[name] = cases[name]["data"]["q"]
    indexes = {name: c["idx"] for name, c in cases.items()}
    ex = GpuExecutor(indexes, n_workers=3)
    sched = Scheduler(ex.cost, budget=1 << 30, max_batch_queries=48)
    srv = Server(sched, ex, n_workers=3)
    reqs = poisson_requests(pools, rate=400.0, duration=0.1, seed=11, sizes=(1, 24), nprobes=(4, 8))
    _log(f"{len(reqs)} requests")
    replay(srv, reqs)
    assert not srv.errors, srv.errors
    assert len(srv.completed) == len(reqs)
    rep = latency_report(reqs)
    _log("report", rep, "batches", len(srv.batches))
    # batches ran concurrently on more than one worker
    assert len({b[1] for b in srv.batches}) > 1
    alone_ctx = Context(0)
    for r in reqs:
        qd = torch.from_numpy(r.queries).cuda()
        ids, dd = indexes[r.index].search(qd, r.k, nprobe=r.nprobe, ctx=alone_ctx)
        assert np.array_equal(ids.cpu().numpy(), r.ids), r.rid
        assert np.array_equal(dd.cpu().numpy(), r.dists), r.rid
    for r in reqs[:6]:
        ref_i, ref_d = gc.oracle_answer(cases[r.index], r.queries, r.nprobe, r.k)
        gc.compare(r.ids, r.dists, ref_i, ref_d)
