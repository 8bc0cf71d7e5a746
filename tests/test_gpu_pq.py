"""GPU parity of the IVFPQ search (Section 4.2 shaping, Section 6.2 the PQ
scan) against the oracle: ids and distances bit-exact at eps = 1 (pruned and
brute-force scans), on the GIST-like and SIFT-like shapes, k = 1, 10 and 100,
per-query probe counts, a band of equal distances wider than the buffers
(the exact fallback), the relaxed bound, and a non-finite query.  The oracle
takes the index's trained quantizer (shaped transform, codebooks, codes)
and its coarse lists, since k-means has no pinned result; the codes are
checked against the oracle's own nearest-codeword rule softly."""
import dataclasses
import sys

import numpy as np
import pytest

from oracle import pq
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


def build_pq_case(w, data, dsub, kappa=2.0, iters=6, sample=8192, transform="pca"):
    import torch
    from tests import gpu_cases as gc
    from paper_2510_00566_amd.index import PQIndex, Transform, ivf_assign
    x = data["x"]
    xd = torch.from_numpy(x).cuda()
    cuts = w.level_cuts()
    if transform == "pca":
        tf = Transform.fit(x, seed=w.cfg_id).shape(cuts, kappa, isotropize=True, seed=5)
    else:
        tf = Transform.identity(w.d)
    cent, assign = ivf_assign(gc.ctx(), xd, w.nlist, iters=3 if w.nlist > 1 else 0, seed=w.cfg_id)
    idx = PQIndex.build(gc.ctx(), tf, xd, cent, assign, cuts, dsub, iters=iters, sample=sample, seed=7)
    torch.cuda.synchronize()
    mu, t, _, _ = tf.get()
    cb, codes = idx.export()
    return {"x": x, "xd": xd, "tf": tf, "mu": mu, "t": t, "cent": cent.cpu().numpy(),
            "assign": assign.cpu().numpy(), "idx": idx, "cb": cb, "codes": codes, "cuts": cuts, "dsub": dsub}


def oracle_pq(case, q, nprobe, k):
    return pq.pq_knn_ivf(q, case["mu"], case["t"], case["cb"], case["codes"], case["cent"], case["assign"],
                         nprobe, k)


def run_and_compare(torch_cuda, case, q, nprobe, k, **kw):
    qd = torch_cuda.from_numpy(np.ascontiguousarray(q)).cuda()
    npd = torch_cuda.from_numpy(np.asarray(nprobe, dtype=np.int32)).cuda() if np.ndim(nprobe) else int(nprobe)
    ri, rd = oracle_pq(case, q, nprobe, k)
    out = {}
    for brute in (False, True):
        ids, dd = case["idx"].search(qd, k, nprobe=npd, brute=brute, stats=True, **kw)
        st = case["idx"].stats()
        gi, gd = ids.cpu().numpy(), dd.cpu().numpy()
        bad = np.nonzero((gi != ri).any(axis=1))[0]
        assert bad.size == 0, f"brute={brute}: {bad.size} queries differ; first {bad[:3]}: {gi[bad[0]]} vs {ri[bad[0]]}"
        assert np.array_equal(gd, rd), f"brute={brute}: distances differ"
        out[brute] = st
    _log("phi", round(out[False]["phi"], 4), "fallback", out[False]["fallback_queries"])
    assert out[True]["phi"] == 1.0
    return out


@gpu
def test_pq_sift_like_shape(torch_cuda):
    """d = 128, dsub = 4 (M = 32), 8 levels of 16, Zipf lists, k = 10."""
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=20000, nq=40, nlist=32, n_clusters=32)
    w = dataclasses.replace(w, level_width=16, nprobe_range=None, nprobe=4)
    data = synth.generate(w)
    _log("case pq sift-like n=20000 d=128 dsub=4 nlist=32")
    case = build_pq_case(w, data, dsub=4)
    st = run_and_compare(torch_cuda, case, data["q"], 4, 10)
    assert st[False]["phi"] < 1.0
    # the codes: nearest codewords (FP32 on the GPU), softly against FP64
    y = pq.shaped_query(case["x"][:2000], case["mu"], case["t"])
    yc = pq.shaped_query(case["cent"], case["mu"], case["t"])
    mism = (pq.encode(y - yc[case["assign"][:2000]], case["cb"]) != case["codes"][:2000]).mean()
    _log("code mismatches vs the FP64 rule", mism)
    assert mism < 1e-3


@gpu
def test_pq_gist_like_shape(torch_cuda):
    """d = 960, dsub = 8 (M = 120: the table fills 120 KB of LDS), 12 levels of
    80 coordinates, 1024-wide clusters scaled down."""
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=8000, nq=12, nlist=16, nprobe=3, n_clusters=16)
    w = dataclasses.replace(w, level_width=80)
    data = synth.generate(w)
    _log("case pq gist-like n=8000 d=960 dsub=8 nlist=16")
    case = build_pq_case(w, data, dsub=8, sample=4096, iters=4)
    run_and_compare(torch_cuda, case, data["q"], 3, 10)


@gpu
@pytest.mark.parametrize("k", [1, 100])
def test_pq_k_extremes_and_per_query_nprobe(torch_cuda, k):
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=12000, nq=24, nlist=16, n_clusters=16)
    w = dataclasses.replace(w, level_width=32, nprobe_range=(1, 16))
    data = synth.generate(w)
    _log(f"case pq k={k} per-query nprobe n=12000 d=128 dsub=8")
    case = build_pq_case(w, data, dsub=8)
    npq = np.minimum(data["nprobe"], 16).astype(np.int32)
    run_and_compare(torch_cuda, case, data["q"], npq, k, nprobe_max=16)


@gpu
def test_pq_flat_ragged_and_fewer_than_k(torch_cuda):
    """One list of 300 rows (a ragged second block), k = 128 > rows in reach
    for no query, and a 40-row index where k = 64 pads with (-1, +inf)."""
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="pq-flat", n=300, nq=5, d=64, level_width=16, nlist=1, nprobe=1)
    data = synth.generate(w)
    _log("case pq flat n=300 d=64 dsub=4")
    case = build_pq_case(w, data, dsub=4, sample=300)
    run_and_compare(torch_cuda, case, data["q"], 1, 128)


@gpu
def test_pq_equal_codes_take_the_fallback(torch_cuda):
    """3000 identical rows share one code, so their distances tie exactly: the
    band exceeds the per-wave buffers, the exact fallback answers with the
    smallest ids, as the oracle does."""
    base = synth.WORKLOADS["flat_sift_like"]
    w = dataclasses.replace(base, name="pq-ties", n=3400, nq=4, d=32, level_width=8, nlist=1, nprobe=1)
    g = np.random.default_rng(3)
    x = (g.standard_normal((3400, 32)) * 3).astype(np.float32)
    x[:3000] = x[0]
    q = (x[0] + 0.01 * g.standard_normal((4, 32))).astype(np.float32)
    _log("case pq equal codes n=3400 d=32 dsub=2")
    case = build_pq_case(w, {"x": x, "q": q}, dsub=2, sample=3400)
    st = run_and_compare(torch_cuda, case, q, 1, 8)
    assert st[False]["fallback_queries"] == 4


@gpu
def test_pq_relaxed_bound_and_nonfinite(torch_cuda):
    """eps < 1: every returned distance is a true table distance of the
    returned id and no answer beats the exact one; a NaN query is refused."""
    import torch
    from paper_2510_00566_amd._lib import PanoError
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=12000, nq=16, nlist=16, n_clusters=16)
    w = dataclasses.replace(w, level_width=16, nprobe_range=None, nprobe=3)
    data = synth.generate(w)
    _log("case pq eps<1 n=12000 d=128 dsub=4")
    case = build_pq_case(w, data, dsub=4)
    q = data["q"]
    qd = torch.from_numpy(q).cuda()
    ri, rd = oracle_pq(case, q, 3, 10)
    ids, dd = case["idx"].search(qd, 10, nprobe=3, eps=0.5)
    gi, gd = ids.cpu().numpy(), dd.cpu().numpy()
    y = pq.shaped_query(q, case["mu"], case["t"])
    yc = pq.shaped_query(case["cent"], case["mu"], case["t"])
    for qi in range(q.shape[0]):
        ok = gi[qi] >= 0
        for r in np.nonzero(ok)[0]:
            tab = pq.lut(y[qi] - yc[case["assign"][gi[qi][r]]], case["cb"])
            assert pq.adc(tab, case["codes"][gi[qi][r:r + 1]])[0] == gd[qi][r]
        assert (gd[qi][ok] >= rd[qi][ok]).all()
    bad = q.copy()
    bad[2, 5] = np.nan
    with pytest.raises(PanoError, match="non-finite"):
        case["idx"].search(torch.from_numpy(bad).cuda(), 10, nprobe=3)
    run_and_compare(torch_cuda, case, q, 3, 10)  # still usable
