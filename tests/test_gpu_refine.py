"""GPU parity of the point-centric refine (pano_refine) against the oracle's
exact k-NN over each query's candidate ids: random candidate subsets with
empty slots, a first pass's top-k' (the IVF search), identical rows (ties),
a single candidate, rejected ids, eps < 1."""
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


def _cands(n, nq, kp, seed, holes=True):
    g = np.random.Generator(np.random.PCG64(seed))
    c = np.stack([g.permutation(n)[:kp] for _ in range(nq)]).astype(np.int64)
    if holes:
        c[g.random(c.shape) < 0.1] = -1
    return c


@gpu
@pytest.mark.parametrize("kp,k", [(1, 1), (50, 10), (300, 10), (1000, 100)])
def test_refine_random_candidates(torch_cuda, kp, k):
    from oracle import brute
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=12000, nq=20, nlist=16, nprobe=3, n_clusters=16)
    w.d = 240
    w.level_width = 24
    _log(f"case refine n=12000 d=240 kprime={kp} k={k}")
    case = gc.build_case(w)
    q = case["data"]["q"]
    cand = _cands(w.n, w.nq, kp, seed=kp)
    ids, dd = case["idx"].refine(torch_cuda.from_numpy(q).cuda(), k, torch_cuda.from_numpy(cand).cuda())
    ri, rd = brute.knn_candidates(q, case["x"], cand, k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ri, rd)


@gpu
def test_refine_of_first_pass_top_kprime(torch_cuda):
    """A first pass (the IVF search with k' = 100) refined to k = 10 gives
    the first pass's own top 10, which is the oracle's."""
    from oracle import brute
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=40000, nq=32, nlist=64, n_clusters=64)
    _log("case refine zipf first pass k'=100 -> k=10")
    case = gc.build_case(w)
    q = case["data"]["q"]
    qd = torch_cuda.from_numpy(q).cuda()
    fi, _ = case["idx"].search(qd, 100, nprobe=8)
    ids, dd = case["idx"].refine(qd, 10, fi)
    ri, rd = brute.knn_candidates(q, case["x"], fi.cpu().numpy(), 10)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ri, rd)
    si, sd = case["idx"].search(qd, 10, nprobe=8)
    assert torch_cuda.equal(si, ids) and torch_cuda.equal(sd, dd)


@gpu
def test_refine_ties_flat_and_errors(torch_cuda):
    import dataclasses
    from oracle import brute
    from paper_2510_00566_amd._lib import PanoError
    from tests import gpu_cases as gc
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="refine-ties", d=24, k=8, nlist=1, nprobe=1, level_width=8, n=600, nq=4,
                            n_clusters=0)
    one = synth.uniform_cube(1, 24, seed=7)
    x = np.repeat(one, 600, axis=0)
    x[500:] = synth.uniform_cube(100, 24, seed=8)
    q = synth.uniform_cube(4, 24, seed=9) * 0.01 + one
    _log("case refine identical rows n=600 d=24 k=8")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    qd = torch_cuda.from_numpy(q).cuda()
    cand = _cands(600, 4, 400, seed=3)
    ids, dd = case["idx"].refine(qd, 8, torch_cuda.from_numpy(cand).cuda())
    ri, rd = brute.knn_candidates(q, x, cand, 8)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ri, rd)
    # only empty slots: padding
    empty = -np.ones((4, 5), np.int64)
    ids, dd = case["idx"].refine(qd, 3, torch_cuda.from_numpy(empty).cuda())
    assert (ids.cpu().numpy() == -1).all() and np.isinf(dd.cpu().numpy()).all()
    bad = cand.copy()
    bad[2, 7] = 600
    with pytest.raises(PanoError, match="candidate id"):
        case["idx"].refine(qd, 8, torch_cuda.from_numpy(bad).cuda())
    # the index is still usable
    ids, dd = case["idx"].refine(qd, 8, torch_cuda.from_numpy(cand).cuda())
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ri, rd)


@gpu
def test_refine_relaxed_properties(torch_cuda):
    from oracle import brute
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=8000, nq=16)
    case = gc.build_case(w)
    q = case["data"]["q"]
    cand = _cands(w.n, w.nq, 2000, seed=5, holes=False)
    ri, rd = brute.knn_candidates(q, case["x"], cand, w.k)
    for eps in (0.5, 0.8):
        ids, dd = case["idx"].refine(torch_cuda.from_numpy(q).cuda(), w.k, torch_cuda.from_numpy(cand).cuda(), eps=eps)
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
        for i in range(w.nq):
            assert set(ids[i].tolist()) <= set(cand[i].tolist())
            assert np.array_equal(brute.canonical_dist(q[i], case["x"][ids[i]]).astype(np.float32), dd[i])
            assert (dd[i] >= rd[i]).all()
