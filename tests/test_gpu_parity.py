"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  ids must be bit-exact and distances within 1e-5
relative (they are expected to be bit-equal: both sides use the canonical
recipe for the reported distance)."""
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


def _flat_small():
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=6000, nq=24)
    return w


def _ivf_small():
    # GIST-like shape (d = 960, 16 levels of 60) at a size the oracle checks in seconds
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=20000, nq=24, nlist=32, nprobe=4, n_clusters=32)
    return w


@gpu
def test_flat_parity(torch_cuda):
    from tests import gpu_cases as gc
    w = _flat_small()
    _log("case flat n=6000 d=128 L=8 k=10")
    case = gc.build_case(w)
    q = case["data"]["q"]
    ids, dd = case["idx"].search(torch_cuda.from_numpy(q).cuda(), w.k, nprobe=1)
    ref_i, ref_d = gc.oracle_answer(case, q, 1, w.k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    bi, bd = case["idx"].search_bruteforce(torch_cuda.from_numpy(q).cuda(), w.k, nprobe=1)
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)


@gpu
def test_ivf_gist_shape_parity(torch_cuda):
    from tests import gpu_cases as gc
    w = _ivf_small()
    _log("case ivf n=20000 d=960 nlist=32 nprobe=4 L=16 k=10")
    case = gc.build_case(w)
    q = case["data"]["q"]
    qd = torch_cuda.from_numpy(q).cuda()
    ids, dd = case["idx"].search(qd, w.k, nprobe=w.nprobe, stats=True)
    st = case["idx"].stats()
    _log("stats", {k: st[k] for k in ("candidates", "dims_read", "items", "committed", "band", "fallback_queries")})
    ref_i, ref_d = gc.oracle_answer(case, q, w.nprobe, w.k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    assert st["fallback_queries"] == 0
    assert st["dims_read"] < 0.5 * st["candidates"] * w.d
    bi, bd = case["idx"].search_bruteforce(qd, w.k, nprobe=w.nprobe)
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)


@gpu
def test_graph_replay_matches_eager(torch_cuda):
    """The search is captured into a HIP graph on first use and replayed; every
    replay (with eager work and synchronisation in between) must equal the
    eager result bit for bit."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=12000, nq=20, nlist=16, nprobe=3, n_clusters=16)
    w.d = 200
    w.level_width = 20
    case = gc.build_case(w)
    q = torch_cuda.from_numpy(case["data"]["q"]).cuda()
    ids = torch_cuda.empty((w.nq, w.k), dtype=torch_cuda.int64, device="cuda")
    dd = torch_cuda.empty((w.nq, w.k), dtype=torch_cuda.float32, device="cuda")
    ei, ed = case["idx"].search(q, w.k, nprobe=w.nprobe, eager=True)
    for rep in range(4):
        case["idx"].search(q, w.k, nprobe=w.nprobe, out=(ids, dd))  # graph replay
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(ids, ei) and torch_cuda.equal(dd, ed), rep
        ei2, ed2 = case["idx"].search(q, w.k, nprobe=w.nprobe, eager=True, stats=True)
        assert torch_cuda.equal(ei2, ei)
    ref_i, ref_d = gc.oracle_answer(case, case["data"]["q"], w.nprobe, w.k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)


PARAM_GRID = [
    dict(),
    dict(blocks_per_item=2),
    dict(blocks_per_item=4, dense_min=32),
    dict(blocks_per_item=3, group=8),
    dict(blocks_per_item=8, group=4, seed_pool=256, seed_count=16),
    dict(blocks_per_item=4, dense_min=1 << 30),
    dict(blocks_per_item=2, group=1, grid=7),
    dict(scan_mode=4),
    dict(scan_mode=4, group=4, grid=5, dense_min=1),
    dict(scan_mode=4, blocks_per_item=3, dense_min=1 << 30, arrival_order=1),
    dict(scan_mode=3),
    dict(arrival_order=1),
    dict(walk_lanes=1),
    dict(walk_lanes=2),
    dict(walk_lanes=4, walk_step=1),
]


@gpu
@pytest.mark.parametrize("kw", PARAM_GRID, ids=[str(sorted(k.items())) for k in PARAM_GRID])
def test_parity_across_search_knobs(torch_cuda, kw):
    """Every setting of the search knobs (work-item size, group size, seeding,
    dense-refinement threshold, grid) returns the oracle's answer."""
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Params
    key = "knob_case"
    if not hasattr(test_parity_across_search_knobs, key):
        w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=30000, nq=40, nlist=24, nprobe=5, n_clusters=24)
        w.d = 240
        w.level_width = 24
        case = gc.build_case(w)
        ref = gc.oracle_answer(case, case["data"]["q"], w.nprobe, w.k)
        setattr(test_parity_across_search_knobs, key, (w, case, ref))
    w, case, (ref_i, ref_d) = getattr(test_parity_across_search_knobs, key)
    q = torch_cuda.from_numpy(case["data"]["q"]).cuda()
    p = Params(**kw)
    ids, dd = case["idx"].search(q, w.k, nprobe=w.nprobe, params=p)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    ids2, dd2 = case["idx"].search(q, w.k, nprobe=w.nprobe, params=p, eager=True)
    gc.compare(ids2.cpu().numpy(), dd2.cpu().numpy(), ref_i, ref_d)
    bi, bd = case["idx"].search_bruteforce(q, w.k, nprobe=w.nprobe, params=p)
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)


@gpu
def test_graph_not_reused_across_indexes(torch_cuda):
    """A search graph captured for one index must never be replayed for
    another: free an index, build a new one of the same shape (the host
    allocator may hand out the same handle address) and search with the very
    same query and output buffers; the answer must be the new index's."""
    import dataclasses
    from tests import gpu_cases as gc
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="graph-reuse", d=48, k=10, nlist=4, nprobe=2, level_width=8, n=4000, nq=16,
                            n_clusters=0)
    q = synth.uniform_cube(16, 48, seed=21)
    qd = torch_cuda.from_numpy(q).cuda()
    ids = torch_cuda.empty((16, 10), dtype=torch_cuda.int64, device="cuda")
    dd = torch_cuda.empty((16, 10), dtype=torch_cuda.float32, device="cuda")
    for rnd, seed in enumerate((22, 23, 24)):
        x = synth.uniform_cube(4000, 48, seed=seed)
        case = gc.build_case(w, data={"x": x, "q": q})
        for brute in (False, True):
            fn = case["idx"].search_bruteforce if brute else case["idx"].search
            fn(qd, 10, nprobe=2, out=(ids, dd))
            torch_cuda.cuda.synchronize()
            ref_i, ref_d = gc.oracle_answer(case, q, 2, 10)
            gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
        case["idx"].free()
        del case


@gpu
def test_search_ordered_after_callers_stream(torch_cuda):
    """A search on a caller's stream sees the work queued before it on that
    stream: the queries are written by copies enqueued on a side stream just
    before each search (no host synchronisation in between), and every answer
    must be the oracle's for the queries just written."""
    from tests import gpu_cases as gc
    w = _ivf_small()
    _log("case ivf stream ordering n=20000 d=960 nlist=32 nprobe=4")
    case = gc.build_case(w)
    q = case["data"]["q"]
    qs = [np.ascontiguousarray(q), np.ascontiguousarray(q[::-1])]
    refs = [gc.oracle_answer(case, x, w.nprobe, w.k) for x in qs]
    host = [torch_cuda.from_numpy(x).pin_memory() for x in qs]
    qd = torch_cuda.empty(q.shape, dtype=torch_cuda.float32, device="cuda")
    st = torch_cuda.cuda.Stream()
    for rnd in range(4):
        j = rnd % 2
        with torch_cuda.cuda.stream(st):
            qd.copy_(host[j], non_blocking=True)
            ids, dd = case["idx"].search(qd, w.k, nprobe=w.nprobe, stream=st)
        gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), *refs[j])


@gpu
def test_flat_full_size_config(torch_cuda):
    """The flat configuration at full size: N = 100,000, d = 128 (spectrum
    j^-1.2), 8 levels of 16, all 100 queries, k = 10; ids bit-exact against
    brute force (the C oracle's, pinned bit for bit to the numpy oracle)."""
    from oracle import c_oracle
    from tests import gpu_cases as gc
    w = synth.WORKLOADS["flat_sift_like"]
    _log("case flat full n=100000 d=128 nq=100 L=8 k=10")
    case = gc.build_case(w)
    q = case["data"]["q"]
    qd = torch_cuda.from_numpy(q).cuda()
    ids, dd = case["idx"].search(qd, w.k, nprobe=1, stats=True)
    st = case["idx"].stats()
    c_oracle.build(force=False)
    n = case["x"].shape[0]
    off = np.arange(q.shape[0] + 1, dtype=np.int64) * n
    cand = np.tile(np.arange(n, dtype=np.int64), q.shape[0])
    ref_i, ref_d = c_oracle.knn_lists(q, case["x"], off, cand, w.k, threads=16)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    assert st["fallback_queries"] == 0 and st["candidates"] == n * q.shape[0]
    _log("phi", st["dims_read"] / (st["candidates"] * w.d))
    bi, bd = case["idx"].search_bruteforce(qd, w.k, nprobe=1)
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)
