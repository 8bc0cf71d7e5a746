"""Seeded synthetic workloads shaped like the paper's datasets.

This module only draws random inputs: it holds none of the search method's
arithmetic (no transform fit, no distances, no pruning).  Both the CPU oracle
and the HIP path are fed from it, so every parity comparison sees the same
bytes.

Data law (per workload): x = c + Q (sqrt(lambda) * z), z ~ N(0, I), where Q is
a Haar-random rotation (QR of a Gaussian matrix with the diagonal sign fix of
Mezzadri, "How to generate random matrices from the classical compact groups",
2007), lambda_1 = 1 and the decay law is given per workload, and the centers
c (if any) are N(0, center_var * I).  Queries follow the same law.

Random streams: each workload draws from
Generator(PCG64(SeedSequence([20251001, cfg_id, stream]))) with streams
0 rotation, 1 centers, 2 database, 3 queries, 4 per-query nprobe,
5 k-means init, 6 PCA fit sample, 7 serving arrivals.

The paper's own datasets (Deep, SIFT, arXiv, GIST, Ada, Large) are not
available; these synthetic workloads stand in for them with matching N and d
(the GIST-like d=960 and the SIFT/Deep-like d=128 shapes).
"""
from __future__ import annotations

import dataclasses
import numpy as np

BASE_SEED = 20251001
STREAM_ROTATION, STREAM_CENTERS, STREAM_DB, STREAM_QUERIES = 0, 1, 2, 3
STREAM_NPROBE, STREAM_KMEANS, STREAM_PCA, STREAM_SERVING = 4, 5, 6, 7


def rng(cfg_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, cfg_id, stream])))


def haar_rotation(d: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal d x d matrix (float64)."""
    a = g.standard_normal((d, d))
    qm, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return qm * s[None, :]


def spectrum(kind: str, d: int, p: float) -> np.ndarray:
    j = np.arange(1, d + 1, dtype=np.float64)
    if kind == "power":
        return j ** (-p)
    if kind == "exp":
        return np.exp(-p * (j - 1))
    raise ValueError(kind)


def zipf_sizes(n: int, n_clusters: int, s: float) -> np.ndarray:
    """Cluster sizes proportional to c^-s (c = 1..n_clusters), summing to n,
    every cluster non-empty; rounding by largest remainder."""
    w = np.arange(1, n_clusters + 1, dtype=np.float64) ** (-s)
    w /= w.sum()
    raw = w * n
    sizes = np.maximum(np.floor(raw).astype(np.int64), 1)
    rem = n - int(sizes.sum())
    if rem > 0:
        order = np.argsort(-(raw - np.floor(raw)), kind="stable")
        sizes[order[:rem]] += 1
    elif rem < 0:
        order = np.argsort(-sizes, kind="stable")
        i = 0
        while rem < 0:
            sizes[order[i % n_clusters]] -= 1
            rem += 1
            i += 1
    return sizes


@dataclasses.dataclass
class Workload:
    name: str
    cfg_id: int
    n: int
    d: int
    nq: int
    k: int
    spec_kind: str
    spec_p: float
    n_clusters: int = 0          # 0: a single zero-mean Gaussian
    center_var: float = 4.0
    zipf_s: float = 0.0          # 0: equal cluster sizes
    normalize: bool = False
    nlist: int = 1
    nprobe: int = 1
    nprobe_range: tuple | None = None   # per-query nprobe ~ U{lo..hi}
    level_width: int = 16
    tune_width: bool = False     # the level width is the tuner's choice (else fixed by the configuration)
    q_spec_p: float | None = None  # out-of-distribution queries: their own decay law parameter (None = the data's)
    pq_dsub: int = 0             # IVFPQ: coordinates per sub-quantizer (0: not a PQ workload)
    pq_kappa: float = 0.0        # IVFPQ: the energy cap of the spectrum shaping (Section 4.2)
    note: str = ""

    @property
    def L(self) -> int:
        return (self.d + self.level_width - 1) // self.level_width

    def level_cuts(self) -> np.ndarray:
        m = list(range(0, self.d, self.level_width)) + [self.d]
        return np.asarray(m, dtype=np.int32)


# Full-size workloads (the five configurations of the headline benchmark).
WORKLOADS = {
    "flat_sift_like": Workload("flat_sift_like", 1, 100_000, 128, 100, 10, "power", 1.2,
                               level_width=16, note="flat exact kNN, one list, 8 levels x 16 dims"),
    "ivf_gist_like": Workload("ivf_gist_like", 2, 1_000_000, 960, 1000, 10, "exp", 0.01,
                              n_clusters=1024, nlist=1024, nprobe=32, level_width=60,
                              note="IVFFlat exact-at-probe, 16 levels x 60 dims"),
    "ivf_zipf_batched": Workload("ivf_zipf_batched", 3, 10_000_000, 128, 10_000, 10, "power", 1.0,
                                 n_clusters=4096, zipf_s=1.1, nlist=4096, nprobe=68,
                                 nprobe_range=(8, 128), level_width=16, tune_width=True,
                                 note="batched IVFFlat, Zipf(1.1) list sizes, nprobe ~ U[8,128]"),
    "ivf_embed_bf16": Workload("ivf_embed_bf16", 4, 5_000_000, 768, 10_000, 100, "power", 0.8,
                               normalize=True, nlist=4096, nprobe=64, level_width=32, tune_width=True,
                               note="unit-normed embeddings, BF16 levels + FP32 rescoring"),
    # IVFPQ over the GIST-like data (the same rows and queries as
    # ivf_gist_like): 120 sub-quantizers of 8 coordinates, 12 levels of 80
    "ivfpq_gist_like": Workload("ivfpq_gist_like", 2, 1_000_000, 960, 1000, 10, "exp", 0.01,
                                n_clusters=1024, nlist=1024, nprobe=32, level_width=80, pq_dsub=8, pq_kappa=2.0,
                                note="IVFPQ (M=120, 8 bits), shaped PCA (kappa 2), 12 levels x 80 dims"),
}


def scaled(w: Workload, n: int, nq: int, nlist: int | None = None, nprobe: int | None = None,
           n_clusters: int | None = None) -> Workload:
    """A reduced-size variant of a workload: same law, fewer points."""
    nw = dataclasses.replace(w, n=n, nq=nq)
    if nlist is not None:
        nw.nlist = nlist
    if nprobe is not None:
        nw.nprobe = nprobe
    if n_clusters is not None:
        nw.n_clusters = n_clusters
    nw.name = f"{w.name}@{n}"
    return nw


def _cluster_labels(w: Workload, g: np.random.Generator, count: int, sizes: np.ndarray | None) -> np.ndarray:
    if w.n_clusters == 0:
        return np.zeros(count, dtype=np.int64)
    if sizes is not None:
        lab = np.repeat(np.arange(w.n_clusters, dtype=np.int64), sizes)
        g.shuffle(lab)
        return lab
    if w.zipf_s > 0:
        p = np.arange(1, w.n_clusters + 1, dtype=np.float64) ** (-w.zipf_s)
        p /= p.sum()
        return g.choice(w.n_clusters, size=count, p=p)
    return g.integers(0, w.n_clusters, size=count)


def _draw(w: Workload, count: int, labels: np.ndarray, centers: np.ndarray | None,
          rot: np.ndarray, sq: np.ndarray, g: np.random.Generator, chunk: int = 1 << 16) -> np.ndarray:
    out = np.empty((count, w.d), dtype=np.float32)
    rot32 = rot.T.astype(np.float32)
    sq32 = sq.astype(np.float32)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        z = g.standard_normal((e - s, w.d), dtype=np.float32)
        z *= sq32[None, :]
        v = z @ rot32
        if centers is not None:
            v += centers[labels[s:e]]
        if w.normalize:
            nrm = np.sqrt(np.einsum("ij,ij->i", v, v, dtype=np.float64)).astype(np.float32)
            nrm[nrm == 0] = 1.0
            v /= nrm[:, None]
        out[s:e] = v
    return out


def generate(w: Workload, with_queries: bool = True):
    """Return dict(x [n,d] f32, q [nq,d] f32, labels [n], qlabels [nq], nprobe [nq] int32)."""
    rot = haar_rotation(w.d, rng(w.cfg_id, STREAM_ROTATION))
    lam = spectrum(w.spec_kind, w.d, w.spec_p)
    sq = np.sqrt(lam)
    centers = None
    if w.n_clusters > 0:
        gc = rng(w.cfg_id, STREAM_CENTERS)
        centers = (gc.standard_normal((w.n_clusters, w.d)) * np.sqrt(w.center_var)).astype(np.float32)
    gdb = rng(w.cfg_id, STREAM_DB)
    sizes = None
    if w.n_clusters > 0:
        if w.zipf_s > 0:
            sizes = zipf_sizes(w.n, w.n_clusters, w.zipf_s)
        else:
            sizes = np.full(w.n_clusters, w.n // w.n_clusters, dtype=np.int64)
            sizes[: w.n - int(sizes.sum())] += 1
    labels = _cluster_labels(w, gdb, w.n, sizes)
    x = _draw(w, w.n, labels, centers, rot, sq, gdb)
    out = {"x": x, "labels": labels, "lambda": lam}
    if with_queries:
        out.update(queries(w, rot=rot, centers=centers))
    return out


def queries(w: Workload, rot: np.ndarray | None = None, centers: np.ndarray | None = None):
    """The workload's queries alone: dict(q [nq,d] f32, qlabels [nq], nprobe
    [nq] int32).  They follow the data's law (same rotation and centres), with
    the spectrum of q_spec_p when it is set (scaled to the same total energy):
    a slower decay spreads a query's energy over more principal directions of
    the data (out-of-distribution queries whose tail energy decays at a rate
    of their own)."""
    if rot is None:
        rot = haar_rotation(w.d, rng(w.cfg_id, STREAM_ROTATION))
    if centers is None and w.n_clusters > 0:
        gc = rng(w.cfg_id, STREAM_CENTERS)
        centers = (gc.standard_normal((w.n_clusters, w.d)) * np.sqrt(w.center_var)).astype(np.float32)
    lam = spectrum(w.spec_kind, w.d, w.spec_p)
    if w.q_spec_p is not None:
        # the queries' own decay, scaled to the data's total energy so that
        # only how the energy spreads over the directions differs
        lq = spectrum(w.spec_kind, w.d, w.q_spec_p)
        lam = lq * (lam.sum() / lq.sum())
    sq = np.sqrt(lam)
    gq = rng(w.cfg_id, STREAM_QUERIES)
    qlab = _cluster_labels(w, gq, w.nq, None)
    out = {"q": _draw(w, w.nq, qlab, centers, rot, sq, gq), "qlabels": qlab}
    if w.nprobe_range is not None:
        lo, hi = w.nprobe_range
        out["nprobe"] = rng(w.cfg_id, STREAM_NPROBE).integers(lo, hi + 1, size=w.nq).astype(np.int32)
    else:
        out["nprobe"] = np.full(w.nq, w.nprobe, dtype=np.int32)
    return out


def uniform_cube(n: int, d: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Small helper for property tests: uniform float32 points."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 99, seed])))
    return g.uniform(lo, hi, size=(n, d)).astype(np.float32)


def integer_grid(n: int, d: int, seed: int, span: int = 4) -> np.ndarray:
    """Small-integer points: many exact distance ties and duplicates."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, 98, seed])))
    return g.integers(-span, span + 1, size=(n, d)).astype(np.float32)
