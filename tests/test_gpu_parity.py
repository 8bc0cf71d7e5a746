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
