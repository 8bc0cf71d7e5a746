"""GPU bound audit: the per-level certified bounds the GPU computes for
sampled (query, row) pairs, from the index's own tiles, tails and query
constants with the scans' bound functions, must bracket the exact
stored-frame distance ||y_q - y_x||^2 (the bounds of Section 5 with the
margins of the floating-point analysis): lower <= D <= upper after every
level, in both the coordinate-difference and the dot-product form, for
FP32 and bfloat16 tiles.  D is computed here in FP64 from the FP32 values
the GPU used (exact up to a relative 1e-13).  Near pairs (each query's
nearest rows, where the bounds are tightest) and random pairs are both
sampled; the bounds must also be tight at the last level."""
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


def _pairs(x, q, n_rand, seed):
    g = np.random.default_rng(seed)
    near = []
    for qi in range(q.shape[0]):
        d = ((x.astype(np.float64) - q[qi].astype(np.float64)) ** 2).sum(1)
        near += [(qi, int(r)) for r in np.argsort(d)[:8]]
    rnd = [(int(g.integers(q.shape[0])), int(g.integers(x.shape[0]))) for _ in range(n_rand)]
    pq, pr = zip(*(near + rnd))
    return np.asarray(pq, np.int32), np.asarray(pr, np.int64)


def _audit(torch_cuda, idx, q, pq, pr, bf16):
    qd = torch_cuda.from_numpy(q).cuda()
    out, rows = idx.audit_bounds(qd, pq, pr, bf16=bf16)
    b = out.cpu().numpy().astype(np.float64)
    rw = rows.cpu().numpy().astype(np.float64)
    D = ((rw[:, 0] - rw[:, 1]) ** 2).sum(1)
    slack = 1e-13 * D + 1e-30
    for form, (lo, hi) in (("difference", (0, 1)), ("dot", (2, 3))):
        low, up = b[:, :, lo], b[:, :, hi]
        bad_lo = np.argwhere(low > D[:, None] + slack[:, None])
        bad_hi = np.argwhere(up < D[:, None] - slack[:, None])
        assert bad_lo.size == 0, f"{form} lower bound above D at (pair, level) {bad_lo[:3].tolist()}"
        assert bad_hi.size == 0, f"{form} upper bound below D at (pair, level) {bad_hi[:3].tolist()}"
        # not vacuous: at the last level the bracket is the head's rounding only
        width = (up[:, -1] - low[:, -1]) / np.maximum(D, 1e-30)
        _log(f"{form}: relative width at the last level: median {np.median(width):.2e}, max {width.max():.2e}; "
             f"min lower/D after level 1 {np.min(low[:, 0] / np.maximum(D, 1e-30)):.3f}")
        assert np.all(np.isfinite(low)) and np.all(np.isfinite(up))
        assert np.median(width) < (0.05 if bf16 else 1e-3)
    return b, D


@gpu
@pytest.mark.parametrize("name,n,nlist,width", [("ivf_gist_like", 6000, 16, 60), ("ivf_zipf_batched", 30000, 64, 32),
                                                ("flat_sift_like", 8000, 1, 16)])
def test_bounds_bracket_the_exact_distance(torch_cuda, name, n, nlist, width):
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS[name], n=n, nq=24, nlist=nlist,
                     n_clusters=nlist if synth.WORKLOADS[name].n_clusters else 0)
    w = dataclasses.replace(w, level_width=width)
    _log(f"case audit {name} n={n} d={w.d} nlist={nlist} width={width}")
    case = gc.build_case(w)
    pq, pr = _pairs(case["x"], case["data"]["q"], 3000, seed=n)
    _audit(torch_cuda, case["idx"], case["data"]["q"], pq, pr, bf16=False)


@gpu
def test_bfloat16_bounds_bracket_the_fp32_row_distance(torch_cuda):
    """bfloat16 tiles of unit-norm embedding-like rows: the widened bracket
    holds against the distance to the FP32 row, and the FP32 audit of the
    same index holds too."""
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_embed_bf16"], n=12000, nq=16, nlist=32, n_clusters=32)
    _log("case audit bf16 n=12000 d=768 nlist=32")
    case = gc.build_case(w, store="bf16")
    pq, pr = _pairs(case["x"], case["data"]["q"], 2000, seed=4)
    for bf in (True, False):
        _audit(torch_cuda, case["idx"], case["data"]["q"], pq, pr, bf16=bf)


@gpu
def test_out_of_distribution_queries_and_errors(torch_cuda):
    """Queries with a flat spectrum in the data's basis (their tails stay
    large) are bracketed too; pair indices out of range are refused."""
    from paper_2510_00566_amd._lib import PanoError
    from tests import gpu_cases as gc
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=6000, nq=12, nlist=16, n_clusters=16)
    case = gc.build_case(w)
    q = synth.queries(dataclasses.replace(w, q_spec_p=0.0))["q"]
    _log("case audit ood n=6000 d=960")
    pq, pr = _pairs(case["x"], q, 1000, seed=9)
    _audit(torch_cuda, case["idx"], q, pq, pr, bf16=False)
    qd = torch_cuda.from_numpy(q).cuda()
    with pytest.raises(PanoError, match="out of range"):
        case["idx"].audit_bounds(qd, np.array([0], np.int32), np.array([w.n], np.int64))
    with pytest.raises(PanoError, match="bfloat16"):
        case["idx"].audit_bounds(qd, np.array([0], np.int32), np.array([0], np.int64), bf16=True)
