"""GPU parity of the asynchronous search (PANO_SEARCH_ASYNC): it returns
without waiting, consecutive searches queue on one stream, a query whose
result buffer overflows is answered by the exact fallback on the device, and
a query with a non-finite value gets (-1, +inf) and is reported by the
context's status call.  Every answer is checked against the oracle."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2510_00566_amd import synth

gpu = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _workload(d, k, nlist, nprobe, width, n, nq):
    base = synth.WORKLOADS["flat_sift_like"]
    return dataclasses.replace(base, name=f"async-d{d}", d=d, k=k, nlist=nlist, nprobe=nprobe, level_width=width,
                               n=n, nq=nq, n_clusters=0)


@gpu
@pytest.mark.parametrize("eager", [False, True])
def test_async_batches_queue_on_one_stream(torch_cuda, eager):
    """Four query batches searched back to back without waiting (two of them
    the same size, so the captured graph is replayed, the other two new
    shapes), then one synchronisation: each answer matches the oracle's."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=30000, nq=160, nlist=32, n_clusters=32)
    data = synth.generate(w)
    _log(f"case async batches eager={eager} n=30000 d=128 nlist=32")
    case = gc.build_case(w, data=data)
    q = data["q"]
    cuts = [(0, 40), (40, 80), (80, 150), (150, 160)]
    outs = []
    for a, b in cuts:
        qd = torch_cuda.from_numpy(q[a:b].copy()).cuda()
        ids, dd = case["idx"].search(qd, w.k, nprobe=5, eager=eager, asynchronous=True)
        outs.append((qd, ids, dd))
    torch_cuda.cuda.synchronize()
    assert case["idx"].ctx.status() == 0
    for (a, b), (_, ids, dd) in zip(cuts, outs):
        ref_i, ref_d = gc.oracle_answer(case, q[a:b], 5, w.k)
        gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)


@gpu
def test_async_overflow_takes_device_fallback(torch_cuda):
    """5000 identical rows tie for every query: the band of equal distances
    exceeds the per-query buffer and the device fallback answers with the k
    smallest ids, as the synchronous search's host-driven fallback does."""
    from tests import gpu_cases as gc
    w = _workload(d=24, k=8, nlist=1, nprobe=1, width=8, n=5008, nq=4)
    base = synth.uniform_cube(1, 24, seed=7)
    x = np.repeat(base, 5008, axis=0)
    x[5000:] = synth.uniform_cube(8, 24, seed=8) + 3.0
    q = synth.uniform_cube(4, 24, seed=9) * 0.01 + base
    _log("case async identical rows n=5008 d=24 k=8")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    qd = torch_cuda.from_numpy(q).cuda()
    for eager in (False, True):
        ids, dd = case["idx"].search(qd, 8, nprobe=1, eager=eager, asynchronous=True)
        torch_cuda.cuda.synchronize()
        ids = ids.cpu().numpy()
        assert (ids == np.arange(8)[None, :]).all()
        ref_i, ref_d = gc.oracle_answer(case, q, 1, 8)
        gc.compare(ids, dd.cpu().numpy(), ref_i, ref_d)
    assert case["idx"].ctx.status() == 0


@gpu
def test_async_nonfinite_reported_by_status(torch_cuda):
    """A NaN and an inf query among finite ones: the finite ones are answered
    as the oracle answers them, the others get (-1, +inf), and the status
    call reports two such queries, then none."""
    from tests import gpu_cases as gc
    from paper_2510_00566_amd._lib import PanoError
    w = _workload(d=32, k=5, nlist=4, nprobe=2, width=8, n=800, nq=6)
    x = synth.uniform_cube(800, 32, seed=11)
    q = synth.uniform_cube(6, 32, seed=12)
    _log("case async non-finite n=800 d=32 nlist=4")
    case = gc.build_case(w, data={"x": x, "q": q})
    bad = q.copy()
    bad[1, 7] = np.nan
    bad[4, 0] = np.inf
    ids, dd = case["idx"].search(torch_cuda.from_numpy(bad).cuda(), 5, nprobe=2, asynchronous=True)
    with pytest.raises(PanoError, match=r"non-finite.*\(2\)"):
        case["idx"].ctx.status()
    assert case["idx"].ctx.status() == 0
    ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
    for r in (1, 4):
        assert (ids[r] == -1).all() and np.isinf(dd[r]).all()
    good = [0, 2, 3, 5]
    ref_i, ref_d = gc.oracle_answer(case, q[good], 2, 5)
    gc.compare(ids[good], dd[good], ref_i, ref_d)
    # a synchronous search on the same context afterwards is unaffected
    si, sd = case["idx"].search(torch_cuda.from_numpy(q).cuda(), 5, nprobe=2)
    ref_i, ref_d = gc.oracle_answer(case, q, 2, 5)
    gc.compare(si.cpu().numpy(), sd.cpu().numpy(), ref_i, ref_d)
