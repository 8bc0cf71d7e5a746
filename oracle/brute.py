"""Oracle O1/O2: brute-force exact k-NN, written as the plain definition.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.

Problem 1 (kNN refinement, Section 3) asks for the k candidates nearest to the
query in Euclidean distance.  The paper fixes neither the precision nor the
summation order of the "exact distance", so the oracle uses one canonical
recipe (a reading of the paper, listed in the design notes):

    d64(q, x) = sum_{j=0}^{d-1} ((double)q_j - (double)x_j)^2

accumulated sequentially in j, every product and every sum rounded to FP64
(no fused multiply-add), then D(q, x) = (float32) d64 (round to nearest even).
The answer is the first k candidates in ascending order of the key (D, id);
fewer than k candidates are padded with id -1 and distance +inf.

Problem 2 (ANN index) yields the candidate set.  For IVF, the probe set of a
query is the first nprobe list ids in ascending order of (D(q, c_l), l) with
raw-space centroids, and the candidate set is every vector assigned to a probed
list ("exact at probe").
"""
from __future__ import annotations

import numpy as np


def canonical_dist(q: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """D(q, x) for one query q [d] against rows xs [n, d]; returns float32 [n].

    numpy's subtract/multiply/add ufuncs round each elementwise operation
    separately, so the loop over j reproduces the sequential FP64 recipe.
    """
    q64 = np.asarray(q, dtype=np.float32).astype(np.float64)
    x64 = np.asarray(xs, dtype=np.float32).astype(np.float64)
    s = np.zeros(x64.shape[0], dtype=np.float64)
    for j in range(q64.shape[0]):
        t = q64[j] - x64[:, j]
        s = s + t * t
    return s.astype(np.float32)


def canonical_dist_many(qs: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """D for every (query, row) pair: float32 [nq, n].  Same recipe as above."""
    q64 = np.asarray(qs, dtype=np.float32).astype(np.float64)
    x64 = np.asarray(xs, dtype=np.float32).astype(np.float64)
    s = np.zeros((q64.shape[0], x64.shape[0]), dtype=np.float64)
    for j in range(q64.shape[1]):
        t = q64[:, j, None] - x64[None, :, j]
        s = s + t * t
    return s.astype(np.float32)


def topk_by_key(dist: np.ndarray, ids: np.ndarray, k: int):
    """First k entries in ascending (dist, id) order, padded with (-1, +inf)."""
    order = np.lexsort((ids, dist))[:k]
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float32)
    out_i[: order.size] = ids[order]
    out_d[: order.size] = dist[order]
    return out_i, out_d


def knn_flat(qs: np.ndarray, xs: np.ndarray, k: int, chunk: int = 1 << 15):
    """O1: exact k-NN of every query over all rows.  Returns ids [nq,k] int64,
    dists [nq,k] float32."""
    qs = np.atleast_2d(qs)
    nq = qs.shape[0]
    n = xs.shape[0]
    ids_all = np.arange(n, dtype=np.int64)
    out_i = np.full((nq, k), -1, dtype=np.int64)
    out_d = np.full((nq, k), np.inf, dtype=np.float32)
    for qi in range(nq):
        best_d = np.empty(0, dtype=np.float32)
        best_i = np.empty(0, dtype=np.int64)
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            dd = canonical_dist(qs[qi], xs[s:e])
            cd = np.concatenate([best_d, dd])
            ci = np.concatenate([best_i, ids_all[s:e]])
            ti, td = topk_by_key(cd, ci, k)
            keep = ti >= 0
            best_i, best_d = ti[keep], td[keep]
        out_i[qi, : best_i.size] = best_i
        out_d[qi, : best_d.size] = best_d
    return out_i, out_d


def probe_lists(qs: np.ndarray, centroids: np.ndarray, nprobe) -> list:
    """The probe set of each query: the first nprobe list ids by (D(q,c_l), l).
    nprobe is an int or a per-query array; it is clamped to [1, nlist]."""
    qs = np.atleast_2d(qs)
    nlist = centroids.shape[0]
    npv = np.broadcast_to(np.asarray(nprobe), (qs.shape[0],))
    dd = canonical_dist_many(qs, centroids)
    lids = np.arange(nlist, dtype=np.int64)
    out = []
    for qi in range(qs.shape[0]):
        p = int(min(max(int(npv[qi]), 1), nlist))
        order = np.lexsort((lids, dd[qi]))[:p]
        out.append(lids[order])
    return out


def knn_ivf(qs: np.ndarray, xs: np.ndarray, centroids: np.ndarray, assign: np.ndarray,
            nprobe, k: int):
    """O2: exact k-NN over the vectors of each query's probed lists."""
    qs = np.atleast_2d(qs)
    assign = np.asarray(assign)
    probes = probe_lists(qs, centroids, nprobe)
    members = {}
    order = np.argsort(assign, kind="stable")
    bounds = np.searchsorted(assign[order], np.arange(centroids.shape[0] + 1))
    for l in range(centroids.shape[0]):
        members[l] = order[bounds[l]:bounds[l + 1]].astype(np.int64)
    out_i = np.full((qs.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((qs.shape[0], k), np.inf, dtype=np.float32)
    for qi in range(qs.shape[0]):
        cand = np.concatenate([members[int(l)] for l in probes[qi]]) if len(probes[qi]) else np.empty(0, np.int64)
        if cand.size == 0:
            continue
        dd = canonical_dist(qs[qi], xs[cand])
        out_i[qi], out_d[qi] = topk_by_key(dd, cand, k)
    return out_i, out_d, probes


def assignment_mismatches(xs: np.ndarray, centroids: np.ndarray, assign: np.ndarray, chunk: int = 4096) -> int:
    """Soft check: how many rows are not assigned to their (D, l)-nearest centroid."""
    bad = 0
    lids = np.arange(centroids.shape[0])
    for s in range(0, xs.shape[0], chunk):
        dd = canonical_dist_many(xs[s:s + chunk], centroids)
        for r in range(dd.shape[0]):
            best = np.lexsort((lids, dd[r]))[0]
            bad += int(best != assign[s + r])
    return bad


def knn_candidates(qs: np.ndarray, xs: np.ndarray, cand: np.ndarray, k: int):
    """Refine (Section 6.4): exact k-NN of each query among its own candidate
    ids cand [nq][k'] (a first pass's top-k'; -1 marks an empty slot), by the
    (D, id) key.  Returns ids [nq,k] int64, dists [nq,k] float32."""
    qs = np.atleast_2d(qs)
    cand = np.atleast_2d(np.asarray(cand, dtype=np.int64))
    out_i = np.full((qs.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((qs.shape[0], k), np.inf, dtype=np.float32)
    for qi in range(qs.shape[0]):
        ids = np.unique(cand[qi][cand[qi] >= 0])
        if ids.size == 0:
            continue
        out_i[qi], out_d[qi] = topk_by_key(canonical_dist(qs[qi], xs[ids]), ids, k)
    return out_i, out_d
