"""GPU parity of the per-wave scan (scan mode 4) and its brute-force
instance against the oracle: flat and IVF shapes, per-query probe counts,
bfloat16 tiles, a tie band past the result buffer (exact fallback), k = 128,
ragged 64-slot blocks."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2510_00566_amd import synth
from paper_2510_00566_amd.index import Params

gpu = pytest.mark.gpu
WAVE = Params(scan_mode=4)


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check(torch_cuda, case, w, q, nprobe, k=None, store_bf16=False, eps=1.0):
    from tests import gpu_cases as gc
    k = k or w.k
    qd = torch_cuda.from_numpy(q).cuda()
    npd = torch_cuda.from_numpy(np.asarray(nprobe, dtype=np.int32)).cuda() if np.ndim(nprobe) else int(nprobe)
    prm = Params(scan_mode=4, use_bf16=1 if store_bf16 else 0)
    ids, dd = case["idx"].search(qd, k, nprobe=npd, params=prm, stats=True, eps=eps)
    st = case["idx"].stats()
    ref_i, ref_d = gc.oracle_answer(case, q, nprobe, k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    ids2, dd2 = case["idx"].search(qd, k, nprobe=npd, params=prm, eps=eps)  # graph replay
    gc.compare(ids2.cpu().numpy(), dd2.cpu().numpy(), ref_i, ref_d)
    bi, bd = case["idx"].search_bruteforce(qd, k, nprobe=npd, params=Params(scan_mode=4))
    gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)
    if store_bf16:
        # the brute-force scan of the bfloat16 tiles (bracketed commits,
        # canonical rescoring from the FP32 rows)
        bi, bd = case["idx"].search_bruteforce(qd, k, nprobe=npd, params=Params(use_bf16=1))
        gc.compare(bi.cpu().numpy(), bd.cpu().numpy(), ref_i, ref_d)
    return st


@gpu
def test_wave_flat(torch_cuda):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=6000, nq=24)
    _log("case wave flat n=6000 d=128")
    case = gc.build_case(w)
    st = _check(torch_cuda, case, w, case["data"]["q"], 1)
    assert st["fallback_queries"] == 0 and st["candidates"] == 6000 * 24


@gpu
def test_wave_gist_shape(torch_cuda):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=20000, nq=24, nlist=32, nprobe=4, n_clusters=32)
    _log("case wave ivf n=20000 d=960 L=16")
    case = gc.build_case(w)
    st = _check(torch_cuda, case, w, case["data"]["q"], w.nprobe)
    assert st["dims_read"] < 0.5 * st["candidates"] * w.d


@gpu
@pytest.mark.parametrize("width", [8, 16, 32])
def test_wave_zipf_per_query_nprobe(torch_cuda, width):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=40000, nq=48, nlist=64, n_clusters=64)
    w.level_width = width
    data = synth.generate(w)
    _log(f"case wave zipf n=40000 width={width}")
    case = gc.build_case(w, data=data)
    _check(torch_cuda, case, w, data["q"], np.minimum(data["nprobe"], 64).astype(np.int32))


@gpu
def test_wave_bf16(torch_cuda):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_embed_bf16"], n=30000, nq=16, nlist=32, nprobe=6)
    _log("case wave bf16 n=30000 d=768 k=100")
    case = gc.build_case(w, store="bf16")
    _check(torch_cuda, case, w, case["data"]["q"], w.nprobe, store_bf16=True)


@gpu
def test_wave_ties_take_fallback(torch_cuda):
    from tests import gpu_cases as gc
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="wave-ties", d=24, k=8, nlist=1, nprobe=1, level_width=8, n=5008, nq=4,
                            n_clusters=0)
    one = synth.uniform_cube(1, 24, seed=7)
    x = np.repeat(one, 5008, axis=0)
    x[5000:] = synth.uniform_cube(8, 24, seed=8) + 3.0
    q = synth.uniform_cube(4, 24, seed=9) * 0.01 + one
    _log("case wave identical rows n=5008 d=24 k=8")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    _check(torch_cuda, case, w, q, 1)


@gpu
@pytest.mark.parametrize("block", [64, 128])
def test_wave_k128_small_blocks(torch_cuda, block):
    from tests import gpu_cases as gc
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="wave-k128", d=40, k=128, nlist=1, nprobe=1, level_width=8, n=9000, nq=6,
                            n_clusters=0)
    _log(f"case wave k=128 block={block} n=9000 d=40")
    case = gc.build_case(w, block=block)
    _check(torch_cuda, case, w, case["data"]["q"], 1)


@gpu
def test_wave_single_level_and_eps(torch_cuda):
    """One level (the level-1 test is the only one) and eps < 1 answers
    that keep their defining properties."""
    from oracle import brute
    from tests import gpu_cases as gc
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="wave-L1", d=48, k=10, nlist=1, nprobe=1, level_width=48, n=3000, nq=8,
                            n_clusters=0)
    case = gc.build_case(w)
    _check(torch_cuda, case, w, case["data"]["q"], 1)
    w2 = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=15000, nq=16, nlist=16, nprobe=4, n_clusters=16)
    w2.d = 120
    w2.level_width = 12
    c2 = gc.build_case(w2)
    q = c2["data"]["q"]
    ref_i, ref_d = gc.oracle_answer(c2, q, w2.nprobe, w2.k)
    for eps in (0.5, 0.9):
        ids, dd = c2["idx"].search(torch_cuda.from_numpy(q).cuda(), w2.k, nprobe=w2.nprobe, eps=eps, params=WAVE)
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
        for i in range(w2.nq):
            assert len(set(ids[i].tolist())) == w2.k
            canon = brute.canonical_dist(q[i], c2["x"][ids[i]])
            assert np.array_equal(canon.astype(np.float32), dd[i])
            assert (dd[i] >= ref_d[i]).all()


@gpu
def test_wave_long_lists_ordered_in_chunks(torch_cuda):
    """2,500 queries probing every one of 4 lists: each list holds 2,500
    queries, which are ordered by their distance to the list in chunks of
    1,024 per workgroup (three chunks per list, the last one ragged); the
    answers of the per-wave scan, the workgroup scan and the brute force stay
    those of the oracle."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=3000, nq=2500, nlist=4, n_clusters=4)
    w = dataclasses.replace(w, d=32, level_width=8, nprobe_range=None, nprobe=4)
    data = synth.generate(w)
    _log("case wave long lists n=3000 d=32 nlist=4 nq=2500")
    case = gc.build_case(w, data=data)
    _check(torch_cuda, case, w, data["q"], 4)
    qd = torch_cuda.from_numpy(data["q"]).cuda()
    ids, dd = case["idx"].search(qd, w.k, nprobe=4, params=Params(scan_mode=0))
    ref_i, ref_d = gc.oracle_answer(case, data["q"], 4, w.k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
