"""GPU parity on the edge cases of the method and the interface: fewer
candidates than k, a single query with k = 1, exact ties and duplicate rows
(including a tie band larger than the per-query result buffer, which takes
the exact fallback), empty input, non-finite queries, per-query probe counts
on Zipf-sized lists, small ragged blocks, and the relaxed bound (eps < 1)."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import brute
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
    return dataclasses.replace(base, name=f"edge-d{d}", d=d, k=k, nlist=nlist, nprobe=nprobe, level_width=width,
                               n=n, nq=nq, n_clusters=0)


def _run(torch_cuda, case, w, q, nprobe=None, k=None, **kw):
    from tests import gpu_cases as gc
    k = k or w.k
    nprobe = w.nprobe if nprobe is None else nprobe
    qd = torch_cuda.from_numpy(q).cuda()
    npd = torch_cuda.from_numpy(np.asarray(nprobe, dtype=np.int32)).cuda() if np.ndim(nprobe) else int(nprobe)
    ids, dd = case["idx"].search(qd, k, nprobe=npd, stats=True, **kw)
    st = case["idx"].stats()
    ref_i, ref_d = gc.oracle_answer(case, q, nprobe, k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    bi, bd = case["idx"].search_bruteforce(qd, k, nprobe=npd)
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)
    return ids.cpu().numpy(), dd.cpu().numpy(), st


@gpu
def test_fewer_candidates_than_k(torch_cuda):
    """k = 64 over a 40-row flat index: the tail of every answer is (-1, +inf)."""
    from tests import gpu_cases as gc
    w = _workload(d=32, k=64, nlist=1, nprobe=1, width=8, n=40, nq=3)
    x = synth.uniform_cube(40, 32, seed=1)
    q = synth.uniform_cube(3, 32, seed=2)
    _log("case fewer-than-k n=40 d=32 k=64")
    case = gc.build_case(w, data={"x": x, "q": q})
    ids, dd, _ = _run(torch_cuda, case, w, q)
    assert (ids[:, 40:] == -1).all() and np.isinf(dd[:, 40:]).all()
    assert sorted(ids[0, :40].tolist()) == list(range(40))


@gpu
def test_single_query_k1(torch_cuda):
    from tests import gpu_cases as gc
    w = _workload(d=96, k=1, nlist=8, nprobe=2, width=16, n=5000, nq=1)
    x = synth.uniform_cube(5000, 96, seed=3)
    q = synth.uniform_cube(1, 96, seed=4)
    _log("case nq=1 k=1 n=5000 d=96 nlist=8")
    case = gc.build_case(w, data={"x": x, "q": q})
    _run(torch_cuda, case, w, q)
    from paper_2510_00566_amd.index import Params
    # seeding from one or two exact distances (teams spanning wavefronts)
    _run(torch_cuda, case, w, q, params=Params(seed_count=1))
    _run(torch_cuda, case, w, q, k=2, params=Params(seed_count=2))


@gpu
def test_integer_grid_ties(torch_cuda):
    """Small-integer rows: many exact distance ties and duplicate rows; ties
    are ordered by id on both sides."""
    from tests import gpu_cases as gc
    w = _workload(d=16, k=10, nlist=8, nprobe=3, width=4, n=6000, nq=32)
    x = synth.integer_grid(6000, 16, seed=5, span=2)
    q = synth.integer_grid(32, 16, seed=6, span=2)
    _log("case integer grid n=6000 d=16 nlist=8 nprobe=3")
    case = gc.build_case(w, data={"x": x, "q": q})
    _, _, st = _run(torch_cuda, case, w, q)
    _log("fallback queries", st["fallback_queries"])


@gpu
def test_distances_at_float_midpoints(torch_cuda):
    """Integer rows whose squared distances are odd integers just above 2^24,
    exactly halfway between two floats: the canonical value is the
    round-to-nearest-even of the exact sum, so the merge's parallel
    rescoring must fall back to the sequential sum for these rows, and ties
    after rounding are ordered by id."""
    from tests import gpu_cases as gc
    # the margins scale with the row norms (~2^22 here); the other
    # coordinates spread the distances so that the margin band of each work
    # item fits its local top-k
    w = _workload(d=16, k=10, nlist=1, nprobe=1, width=4, n=400, nq=8)
    x = synth.integer_grid(400, 16, seed=21, span=64)
    x[:, 0] = 2048.0
    q = synth.integer_grid(8, 16, seed=22, span=64)
    q[:, 0] = -2048.0
    d2 = ((x[None, :, :].astype(np.float64) - q[:, None, :]) ** 2).sum(-1)
    assert (d2 % 2 == 1).any() and (d2 > 2.0 ** 24).all()
    _log("case float midpoints n=400 d=16 k=10")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    ids, dd, st = _run(torch_cuda, case, w, q)
    assert st["fallback_queries"] == 0
    # the answers include rows whose exact distance was a rounding midpoint
    exact = np.take_along_axis(d2, ids.astype(np.int64), axis=1)
    assert (exact % 2 == 1).any()


@gpu
def test_tie_band_beyond_buffer_takes_fallback(torch_cuda):
    """5000 identical rows tie for every query: the band of equal distances
    exceeds the per-query buffer, the exact fallback runs, and the answer is
    the k smallest ids."""
    from tests import gpu_cases as gc
    w = _workload(d=24, k=8, nlist=1, nprobe=1, width=8, n=5008, nq=4)
    base = synth.uniform_cube(1, 24, seed=7)
    x = np.repeat(base, 5008, axis=0)
    x[5000:] = synth.uniform_cube(8, 24, seed=8) + 3.0
    q = synth.uniform_cube(4, 24, seed=9) * 0.01 + base
    _log("case identical rows n=5008 d=24 k=8")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    ids, _, st = _run(torch_cuda, case, w, q)
    assert (ids == np.arange(8)[None, :]).all()
    assert st["fallback_queries"] == 4


@gpu
def test_merge_of_long_result_buffers(torch_cuda):
    """k = 128 over 64-slot blocks of a flat index with weak pruning: each
    query meets hundreds of work items and its result buffer grows past what
    the merge sorts in LDS, so the merge first cuts it by radix select."""
    from tests import gpu_cases as gc
    w = _workload(d=64, k=128, nlist=1, nprobe=1, width=8, n=30000, nq=8)
    x = synth.uniform_cube(30000, 64, seed=13)
    q = synth.uniform_cube(8, 64, seed=14)
    _log("case long buffers n=30000 d=64 k=128 block=64")
    case = gc.build_case(w, data={"x": x, "q": q}, block=64)
    from paper_2510_00566_amd.index import Params
    # a seed threshold from only k candidates keeps d_k loose for longer
    _, _, st = _run(torch_cuda, case, w, q, params=Params(seed_pool=128, seed_count=128))
    _log("published per query", st["committed"] / w.nq, "fallback", st["fallback_queries"])
    # the merge sorts at most 2048 entries in LDS: on average more than that
    # were published per query, so at least one buffer took the select path
    assert st["committed"] > 2048 * w.nq
    assert st["fallback_queries"] == 0


@gpu
def test_empty_query_batch(torch_cuda):
    from tests import gpu_cases as gc
    w = _workload(d=32, k=5, nlist=1, nprobe=1, width=8, n=500, nq=2)
    x = synth.uniform_cube(500, 32, seed=10)
    case = gc.build_case(w, data={"x": x, "q": x[:2]})
    q = torch_cuda.empty((0, 32), dtype=torch_cuda.float32, device="cuda")
    ids, dd = case["idx"].search(q, 5, nprobe=1)
    assert ids.shape == (0, 5) and dd.shape == (0, 5)


@gpu
def test_nonfinite_query_rejected(torch_cuda):
    from tests import gpu_cases as gc
    from paper_2510_00566_amd._lib import PanoError
    w = _workload(d=32, k=5, nlist=4, nprobe=2, width=8, n=800, nq=3)
    x = synth.uniform_cube(800, 32, seed=11)
    q = synth.uniform_cube(3, 32, seed=12)
    case = gc.build_case(w, data={"x": x, "q": q})
    bad = q.copy()
    bad[1, 7] = np.nan
    with pytest.raises(PanoError, match="non-finite"):
        case["idx"].search(torch_cuda.from_numpy(bad).cuda(), 5, nprobe=2)
    bad[1, 7] = np.inf
    with pytest.raises(PanoError, match="non-finite"):
        case["idx"].search(torch_cuda.from_numpy(bad).cuda(), 5, nprobe=2, eager=True)
    _run(torch_cuda, case, w, q)  # the index is still usable


@gpu
def test_zipf_lists_per_query_nprobe(torch_cuda):
    """Batched IVF shape: Zipf(1.1) cluster sizes, nprobe drawn per query
    (clamped to nlist by both sides), 16-wide levels."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=40000, nq=48, nlist=64, n_clusters=64)
    data = synth.generate(w)
    _log("case zipf n=40000 d=128 nlist=64 per-query nprobe")
    case = gc.build_case(w, data=data)
    npq = np.minimum(data["nprobe"], 64).astype(np.int32)
    ids, _, st = _run(torch_cuda, case, w, data["q"], nprobe=npq)
    _log("zipf stats", {k: st[k] for k in ("candidates", "dims_read", "fallback_queries")})
    assert st["fallback_queries"] == 0
    # a positive nprobe_all bounds the per-query counts (larger ones are
    # clamped to it): the oracle gets the clamped counts
    from tests import gpu_cases as gc
    qd = torch_cuda.from_numpy(data["q"]).cuda()
    npd = torch_cuda.from_numpy(npq).cuda()
    for cap in (16, 64):
        ids, dd = case["idx"].search(qd, w.k, nprobe=npd, nprobe_max=cap)
        ref_i, ref_d = gc.oracle_answer(case, data["q"], np.minimum(npq, cap), w.k)
        gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
        bi, bd = case["idx"].search_bruteforce(qd, w.k, nprobe=npd, nprobe_max=cap)
        gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)


@gpu
@pytest.mark.parametrize("block", [64, 128])
def test_small_ragged_blocks(torch_cuda, block):
    """Blocks of 64 and 128 slots: most lists end in a partly filled block."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=15000, nq=20, nlist=20, nprobe=4, n_clusters=20)
    w.d = 180
    w.level_width = 20
    _log(f"case block={block} n=15000 d=180 nlist=20")
    case = gc.build_case(w, block=block)
    assert case["idx"].info()["block"] == block
    _run(torch_cuda, case, w, case["data"]["q"])


@gpu
def test_relaxed_bound_properties(torch_cuda):
    """eps < 1 (Eq. 4) may drop true neighbours, so its answer is checked by
    what must still hold: every reported distance is the canonical distance
    of the reported id, answers are ordered by (D, id), every id comes from a
    probed list, and no answer beats the exact one; eps = 1 is exact."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=15000, nq=24, nlist=16, nprobe=4, n_clusters=16)
    w.d = 120
    w.level_width = 12
    case = gc.build_case(w)
    q = case["data"]["q"]
    qd = torch_cuda.from_numpy(q).cuda()
    ref_i, ref_d = gc.oracle_answer(case, q, w.nprobe, w.k)
    probes = brute.probe_lists(q, case["cent"], w.nprobe)
    for eps in (0.0, 0.5, 0.9):
        ids, dd = case["idx"].search(qd, w.k, nprobe=w.nprobe, eps=eps)
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
        for i in range(w.nq):
            assert (ids[i] >= 0).all()
            assert len(set(ids[i].tolist())) == w.k
            assert np.isin(case["assign"][ids[i]], probes[i]).all()
            canon = brute.canonical_dist(q[i], case["x"][ids[i]])
            assert np.array_equal(canon.astype(np.float32), dd[i])
            order = np.lexsort((ids[i], dd[i]))
            assert (order == np.arange(w.k)).all()
            assert (dd[i] >= ref_d[i]).all()
    ids, dd = case["idx"].search(qd, w.k, nprobe=w.nprobe, eps=1.0)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)


@gpu
@pytest.mark.parametrize("nlist,nprobe", [(2000, 40), (2000, 100), (5000, 40), (5000, 100)])
def test_many_lists(torch_cuda, nlist, nprobe):
    """The coarse step with many lists: the instance for up to 4096 lists
    (register-resident selects of 64 values per lane) and the general one
    (8-bit radix passes over an LDS histogram beyond 4096 lists), with
    p <= 64 (narrowed through the per-lane minima) and p > 64."""
    from tests import gpu_cases as gc
    w = _workload(d=32, k=10, nlist=nlist, nprobe=nprobe, width=8, n=4 * nlist, nq=16)
    _log(f"case many lists n={4 * nlist} d=32 nlist={nlist} nprobe={nprobe}")
    case = gc.build_case(w)
    _, _, st = _run(torch_cuda, case, w, case["data"]["q"])
    assert st["fallback_queries"] == 0


@gpu
@pytest.mark.parametrize("nlist,nprobe", [(200, 40), (200, 150), (1000, 40), (1000, 300), (3000, 100)])
def test_coarse_band_of_equal_centroid_distances(torch_cuda, nlist, nprobe):
    """Every centroid has the same norm (entries +-1), so a query at the
    origin ties with every list and a query within 1e-6 of it has all its
    list distances inside the coarse error band: the band is the whole list
    set.  Up to 256 band members are ordered in registers and LDS by the fast
    instance; wider bands go whole to the LDS instance.  The probe sets must
    still be the exact (D, list id) order, which the oracle's answer checks."""
    import torch
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Index, Transform
    d = 32
    g = np.random.default_rng(nlist + nprobe)
    cent = np.where(g.random((nlist, d)) < 0.5, -1.0, 1.0).astype(np.float32)
    assign = (np.arange(3 * nlist) % nlist).astype(np.int32)
    x = (cent[assign] + 0.05 * g.standard_normal((3 * nlist, d))).astype(np.float32)
    q = np.zeros((6, d), np.float32)
    q[3:] = (1e-6 * g.standard_normal((3, d))).astype(np.float32)
    w = _workload(d=d, k=10, nlist=nlist, nprobe=nprobe, width=8, n=3 * nlist, nq=6)
    _log(f"case coarse tie band nlist={nlist} nprobe={nprobe} n={3 * nlist} d={d}")
    xd = torch.from_numpy(x).cuda()
    cd, ad = torch.from_numpy(cent).cuda(), torch.from_numpy(assign).cuda()
    tf = Transform.fit(x, seed=1)
    idx = Index.build(gc.ctx(), tf, xd, cd, ad, w.level_cuts())
    case = {"x": x, "cent": cent, "assign": assign, "idx": idx}
    _run(torch_cuda, case, w, q)
    idx.free()


@gpu
def test_out_of_distribution_queries_stay_exact(torch_cuda):
    """Queries whose spectrum is flat in the data's PCA basis (no energy
    compaction, Prop. 5.2's alpha_q -> 0) still get the exact answer."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=20000, nq=24, nlist=32, nprobe=4, n_clusters=32)
    case = gc.build_case(w)
    for qp in (0.0, 0.003):
        q = synth.queries(dataclasses.replace(w, q_spec_p=qp))["q"]
        _log(f"case ood q_spec_p={qp} n=20000 d=960")
        _, _, st = _run(torch_cuda, case, w, q)
        assert st["fallback_queries"] == 0


@gpu
@pytest.mark.parametrize("name,n,nlist", [("ivf_gist_like", 12000, 48), ("ivf_zipf_batched", 40000, 96)])
def test_ivf_assign_final_pass_canonical(torch_cuda, name, n, nlist):
    """The k-means' final pass gives every row the list with the smallest
    (canonical D, list id) key: the oracle's count of rows that are not so
    assigned is zero."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS[name], n=n, nq=1, nlist=nlist, n_clusters=nlist)
    data = synth.generate(w, with_queries=False)
    _log(f"case canonical assignment {name} n={n} nlist={nlist}")
    case = gc.build_case(w, data={"x": data["x"]})
    bad = brute.assignment_mismatches(case["x"], case["cent"], case["assign"])
    _log("assignment mismatches", bad)
    assert bad == 0
