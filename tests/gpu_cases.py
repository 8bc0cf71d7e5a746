"""Shared set-up for the GPU parity tests: build an index through the C ABI
from a seeded synthetic workload and compute the oracle's answer for the
same inputs (the oracle takes the index's centroids and assignment, since
k-means has no pinned result)."""
from __future__ import annotations

import numpy as np

from oracle import brute
from paper_2510_00566_amd import synth
from paper_2510_00566_amd.index import Context, Index, Transform, ivf_assign

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = Context(0)
    return _CTX


def build_case(w: synth.Workload, iters: int = 4, block: int = 256, store: str = "f32", data=None,
               transform: str = "pca", fit_sample: int = 0):
    import torch
    data = data if data is not None else synth.generate(w)
    x = data["x"]
    xd = torch.from_numpy(x).cuda()
    if transform == "pca":
        tf = Transform.fit(x, fit_sample=fit_sample, seed=w.cfg_id)
    else:
        tf = Transform.identity(w.d)
    cent, assign = ivf_assign(ctx(), xd, w.nlist, iters=iters if w.nlist > 1 else 0, seed=w.cfg_id)
    idx = Index.build(ctx(), tf, xd, cent, assign, w.level_cuts(), block=block, store=store)
    torch.cuda.synchronize()
    return {"data": data, "x": x, "xd": xd, "tf": tf, "cent": cent.cpu().numpy(),
            "assign": assign.cpu().numpy(), "idx": idx}


def oracle_answer(case, q: np.ndarray, nprobe, k: int):
    x = case["x"]
    if case["cent"].shape[0] == 1:
        ids, dd = brute.knn_flat(q, x, k)
        return ids, dd
    ids, dd, _ = brute.knn_ivf(q, x, case["cent"], case["assign"], nprobe, k)
    return ids, dd


def compare(ids_gpu, d_gpu, ids_ref, d_ref):
    """ids bit-exact; distances within 1e-5 relative (and +inf padding equal)."""
    ids_gpu = np.asarray(ids_gpu)
    d_gpu = np.asarray(d_gpu)
    assert ids_gpu.shape == ids_ref.shape
    bad = np.nonzero((ids_gpu != ids_ref).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} queries differ; first {bad[:5]}: gpu {ids_gpu[bad[0]]} ref {ids_ref[bad[0]]}"
    fin = np.isfinite(d_ref)
    assert np.array_equal(np.isfinite(d_gpu), fin)
    rel = np.abs(d_gpu[fin].astype(np.float64) - d_ref[fin]) / np.maximum(np.abs(d_ref[fin].astype(np.float64)), 1e-30)
    assert rel.size == 0 or rel.max() <= 1e-5, rel.max()
