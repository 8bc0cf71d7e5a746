"""GPU parity at the full sizes of the batched Zipf configuration (10M x 128,
4096 Zipf(1.1) lists, nprobe ~ U[8, 128], 10,000 queries, k = 10), the
GIST-like one (1M x 960, 1024 lists, nprobe 32, 1,000 queries) and the
unit-norm embedding one (5M x 768 stored in bfloat16, 4096 lists, nprobe 64,
10,000 queries, k = 100), in the launch configuration the benchmark times:
its stored level width and search knobs, the residual PCA, the whole query
batch in one call.

The oracle recomputes a sample of queries one by one (ids bit-exact,
distances to 1e-5 relative): a seeded random sample plus the queries with
the largest nprobe.  Every other query is checked by a property that holds
at any size: the pruned scan returns exactly the brute-force scan's answer
(both exact at eps = 1)."""
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


def _full_size_case(torch, name, store):
    from tests import gpu_cases as gc
    from paper_2510_00566_amd import autotune
    from paper_2510_00566_amd.index import Index, Transform, ivf_assign
    w = dataclasses.replace(synth.WORKLOADS[name])
    npv = w.nprobe_range[1] if w.nprobe_range else w.nprobe
    prm, width = autotune.lookup(autotune.signature("gfx950", w.d, store, w.n, npv, w.k))
    assert prm is not None, f"no stored search knobs for {name}"
    if width and w.tune_width:
        w.level_width = int(width)
    _log(f"case full size {name}: n={w.n} d={w.d} nq={w.nq} nlist={w.nlist} width={w.level_width} {prm}")
    data = synth.generate(w)
    x, q = data["x"], data["q"]
    xd = torch.from_numpy(x).cuda()
    cent, assign = ivf_assign(gc.ctx(), xd, w.nlist, iters=4, seed=w.cfg_id)
    c_np, a_np = cent.cpu().numpy(), assign.cpu().numpy()
    # residual PCA, as the benchmark fits it
    rows = np.random.Generator(np.random.PCG64(w.cfg_id)).choice(w.n, min(w.n, 131072), replace=False)
    tf = Transform.fit(x[rows] - c_np[a_np[rows]], fit_sample=0, seed=w.cfg_id)
    cuts = np.asarray(list(range(0, w.d, w.level_width)) + [w.d], dtype=np.int32)
    idx = Index.build(gc.ctx(), tf, xd, cent, assign, cuts, store=store)
    del xd
    torch.cuda.synchronize()
    return w, prm, data, c_np, a_np, idx


def _check_full_size(torch, name, sample_n, widest_n, store="f32"):
    from tests import gpu_cases as gc
    from oracle import brute
    w, prm, data, c_np, a_np, idx = _full_size_case(torch, name, store)
    try:
        q = data["q"]
        qd = torch.from_numpy(q).cuda()
        if w.nprobe_range is not None:
            nprobe = data["nprobe"].astype(np.int32)
            npd, np_max = torch.from_numpy(nprobe).cuda(), int(w.nprobe_range[1])
        else:
            nprobe = np.full(w.nq, w.nprobe, dtype=np.int32)
            npd, np_max = w.nprobe, 0
        ids = torch.empty((w.nq, w.k), dtype=torch.int64, device="cuda")
        dd = torch.empty((w.nq, w.k), dtype=torch.float32, device="cuda")
        idx.search(qd, w.k, nprobe=npd, eps=1.0, params=prm, out=(ids, dd), nprobe_max=np_max)
        bi, bd = idx.search_bruteforce(qd, w.k, nprobe=npd, params=prm, nprobe_max=np_max)
        torch.cuda.synchronize()
        gi, gd = ids.cpu().numpy(), dd.cpu().numpy()
        # every query: the pruned answer is the brute-force answer
        assert np.array_equal(gi, bi.cpu().numpy()), "pruned and brute-force ids differ"
        assert np.array_equal(gd, bd.cpu().numpy()), "pruned and brute-force distances differ"
        # a sample: the oracle, query by query
        rs = np.random.Generator(np.random.PCG64(2024))
        widest = np.argsort(-nprobe, kind="stable")[:widest_n]
        sample = np.unique(np.concatenate([rs.choice(w.nq, size=sample_n, replace=False), widest]))
        _log(f"  oracle on {sample.size} queries (nprobe up to {int(nprobe[sample].max())})")
        ri, rd, _ = brute.knn_ivf(q[sample], data["x"], c_np, a_np, nprobe[sample], w.k)
        gc.compare(gi[sample], gd[sample], ri, rd)
    finally:
        idx.free()
        torch.cuda.empty_cache()


@gpu
def test_full_size_zipf_batched(torch_cuda):
    # about 10^6 candidates a query: ten queries keep the oracle near 30 s
    _check_full_size(torch_cuda, "ivf_zipf_batched", 8, 2)


@gpu
def test_full_size_gist_like(torch_cuda):
    _check_full_size(torch_cuda, "ivf_gist_like", 12, 4)


@gpu
def test_full_size_embed_bf16(torch_cuda):
    # bfloat16 level tiles, FP32 rescoring: the answer is still the exact one
    _check_full_size(torch_cuda, "ivf_embed_bf16", 10, 0, store="bf16")
