"""GPU parity of the bfloat16 scan: level slices read in bfloat16 under a
certified margin, the boundary band rescored canonically from the FP32 rows
in the merge.  Its answer must equal the
oracle's exactly like the FP32 scan's (ids bit-exact, distances within 1e-5
relative), on the unit-norm embedding shape (d = 768, 32-wide levels,
k = 100) and on the GIST shape across the search knobs."""
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


_CASES = {}


def _embed_case():
    if "embed" not in _CASES:
        from tests import gpu_cases as gc
        w = synth.scaled(synth.WORKLOADS["ivf_embed_bf16"], n=24000, nq=24, nlist=32, nprobe=6)
        _log("case embed n=24000 d=768 nlist=32 nprobe=6 L=24 k=100 store=bf16")
        case = gc.build_case(w, store="bf16")
        ref = gc.oracle_answer(case, case["data"]["q"], w.nprobe, w.k)
        _CASES["embed"] = (w, case, ref)
    return _CASES["embed"]


@gpu
def test_bf16_embed_parity(torch_cuda):
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Params
    w, case, (ref_i, ref_d) = _embed_case()
    q = torch_cuda.from_numpy(case["data"]["q"]).cuda()
    idx = case["idx"]
    assert idx.info()["has_bf16"] == 1
    ids, dd = idx.search(q, w.k, nprobe=w.nprobe, params=Params(use_bf16=1), stats=True)
    st_b = idx.stats()
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    fi, fd = idx.search(q, w.k, nprobe=w.nprobe, stats=True)
    st_f = idx.stats()
    gc.compare(fi.cpu().numpy(), fd.cpu().numpy(), ref_i, ref_d)
    assert torch_cuda.equal(ids, fi) and torch_cuda.equal(dd, fd)
    _log("bf16 bytes", st_b["scan_bytes"], "f32 bytes", st_f["scan_bytes"],
         "bf16 dims", st_b["dims_read"], "f32 dims", st_f["dims_read"])
    assert st_b["fallback_queries"] == 0
    # graph replay of the bfloat16 search returns the same answer
    gi, gd = idx.search(q, w.k, nprobe=w.nprobe, params=Params(use_bf16=1))
    assert torch_cuda.equal(gi, ids) and torch_cuda.equal(gd, dd)


BF16_GRID = [
    dict(use_bf16=1),
    dict(use_bf16=1, blocks_per_item=2),
    dict(use_bf16=1, blocks_per_item=4, dense_min=32),
    dict(use_bf16=1, blocks_per_item=3, group=8, dense_min=1 << 30),
    dict(use_bf16=1, group=1, seed_pool=256, seed_count=16, grid=5),
    dict(use_bf16=1, scan_mode=4),
    dict(use_bf16=1, scan_mode=4, dense_min=1 << 30, group=8),
]


@gpu
@pytest.mark.parametrize("kw", BF16_GRID, ids=[str(sorted(k.items())) for k in BF16_GRID])
def test_bf16_gist_shape_knobs(torch_cuda, kw):
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Params
    if "gist" not in _CASES:
        w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=30000, nq=40, nlist=24, nprobe=5, n_clusters=24)
        w.d = 240
        w.level_width = 24
        _log("case gist-shape n=30000 d=240 nlist=24 nprobe=5 L=10 k=10 store=bf16")
        case = gc.build_case(w, store="bf16")
        ref = gc.oracle_answer(case, case["data"]["q"], w.nprobe, w.k)
        _CASES["gist"] = (w, case, ref)
    w, case, (ref_i, ref_d) = _CASES["gist"]
    q = torch_cuda.from_numpy(case["data"]["q"]).cuda()
    ids, dd = case["idx"].search(q, w.k, nprobe=w.nprobe, params=Params(**kw))
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
    si, sd = case["idx"].search(q, w.k, nprobe=w.nprobe, params=Params(**kw), stats=True)
    gc.compare(si.cpu().numpy(), sd.cpu().numpy(), ref_i, ref_d)
    st = case["idx"].stats()
    _log("bf16", kw, "fallback queries", st["fallback_queries"], "band", st["band"])
    if kw == dict(use_bf16=1):
        # the local top-k holds the widened band: no query needs the fallback
        assert st["fallback_queries"] == 0
    ei, ed = case["idx"].search(q, w.k, nprobe=w.nprobe, params=Params(**kw), eager=True)
    gc.compare(ei.cpu().numpy(), ed.cpu().numpy(), ref_i, ref_d)


@gpu
def test_bf16_needs_bf16_index(torch_cuda):
    """A search asking for bfloat16 slices on an FP32-only index is rejected."""
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import Params
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=3000, nq=4)
    case = gc.build_case(w)
    q = torch_cuda.from_numpy(case["data"]["q"]).cuda()
    with pytest.raises(Exception, match="PANO_BF16"):
        case["idx"].search(q, w.k, nprobe=1, params=Params(use_bf16=1))
    # the FP32 search on the same index still works afterwards
    ids, dd = case["idx"].search(q, w.k, nprobe=1)
    ref_i, ref_d = gc.oracle_answer(case, case["data"]["q"], 1, w.k)
    gc.compare(ids.cpu().numpy(), dd.cpu().numpy(), ref_i, ref_d)
