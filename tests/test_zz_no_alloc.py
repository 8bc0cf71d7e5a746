"""The allocation-free search entry point (pano_search_noalloc, for callers
that cannot allocate) against pano_search: the same ids and distances on two
calls in a row, the second with fewer queries (the fixed scratch keeps the
first call's contents), also when the exact fallback runs; a search larger
than the fixed scratch is rejected with the bytes it needs."""
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


def _same(a, b):
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


@gpu
def test_noalloc_matches_search_on_consecutive_calls(torch_cuda):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=30000, nq=64, nlist=48, n_clusters=48)
    data = synth.generate(w)
    _log("case noalloc zipf n=30000 d=128 nlist=48 nq=64 then 17")
    case = gc.build_case(w, data=data)
    q = torch_cuda.from_numpy(data["q"]).cuda()
    npq = torch_cuda.from_numpy(np.minimum(data["nprobe"], 48).astype(np.int32)).cuda()
    for nq in (64, 17):
        ref = case["idx"].search(q[:nq], w.k, nprobe=npq[:nq], nprobe_max=48)
        got = case["idx"].search_noalloc(q[:nq], w.k, nprobe=npq[:nq], nprobe_max=48)
        torch_cuda.cuda.synchronize()
        _same(got, ref)
        ri, rd = gc.oracle_answer(case, data["q"][:nq], np.minimum(data["nprobe"][:nq], 48), w.k)
        gc.compare(got[0].cpu().numpy(), got[1].cpu().numpy(), ri, rd)
    # a common probe count and eps < 1 (no seeding) through the same array
    for nq, eps in ((40, 1.0), (9, 0.5)):
        ref = case["idx"].search(q[:nq], w.k, nprobe=5, eps=eps)
        got = case["idx"].search_noalloc(q[:nq], w.k, nprobe=5, eps=eps)
        _same(got, ref)


@gpu
def test_noalloc_fallback_and_size_limit(torch_cuda):
    from paper_2510_00566_amd._lib import PanoError
    from tests import gpu_cases as gc
    import dataclasses
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="noalloc-ties", d=24, k=8, nlist=1, nprobe=1, level_width=8, n=5008, nq=4,
                            n_clusters=0)
    one = synth.uniform_cube(1, 24, seed=7)
    x = np.repeat(one, 5008, axis=0)
    x[5000:] = synth.uniform_cube(8, 24, seed=8) + 3.0
    q = synth.uniform_cube(4, 24, seed=9) * 0.01 + one
    _log("case noalloc identical rows n=5008 d=24 k=8 (fallback)")
    case = gc.build_case(w, data={"x": x, "q": q}, transform="identity")
    qd = torch_cuda.from_numpy(q).cuda()
    for nq in (4, 2):
        ref = case["idx"].search(qd[:nq], w.k, nprobe=1)
        got = case["idx"].search_noalloc(qd[:nq], w.k, nprobe=1)
        _same(got, ref)
        assert (got[0].cpu().numpy() == np.arange(8)[None, :]).all()
    # a batch whose scratch exceeds the fixed array: rejected, nothing run
    wz = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=20000, nq=8, nlist=4096, n_clusters=64)
    wz.nlist = 64
    dz = synth.generate(wz)
    cz = gc.build_case(wz, data=dz)
    big = torch_cuda.zeros((40000, wz.d), dtype=torch_cuda.float32, device="cuda")
    with pytest.raises(PanoError, match="bytes of scratch"):
        cz["idx"].search_noalloc(big, 100, nprobe=64)
    # still usable afterwards
    qz = torch_cuda.from_numpy(dz["q"]).cuda()
    _same(cz["idx"].search_noalloc(qz, wz.k, nprobe=6), cz["idx"].search(qz, wz.k, nprobe=6))
