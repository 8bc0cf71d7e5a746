"""Oracle O3: a plain serial version of the paper's pruned scan, in FP64.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.

What it follows:
  * Section 4.1: T is the PCA basis, rows = eigenvectors of the empirical
    covariance sorted by descending eigenvalue.  The fit is centred: vectors
    are mapped to T (v - mu) (a translation plus a rotation preserves every
    distance, so the bounds stay sound).  Eigenvector signs are fixed so that
    the largest-magnitude entry of each row is positive.
  * Eq. 1: ||q - x||^2 = ||Tq||^2 + ||Tx||^2 - 2 <Tq, Tx>.
  * Eq. 2: partial products p^(0,l) and tail energies R^(l,d) over the level
    cuts 0 = m_0 < m_1 < ... < m_L = d.
  * Eq. 3 / Eq. 4: LB_eps^l = A^l - 2 eps C^l with A^l = R_q^(0,d) + R_x^(0,d)
    - 2 p^(0,l) and C^l = sqrt(R_q^(l,d) R_x^(l,d)); eps = 1 is the exact
    Cauchy-Schwarz lower bound.  The upper bound A^l + 2 C^l is the other side
    of the same inequality (the paper names it but never writes it).
  * Algorithm 1: a heap H seeded with the exact distances of the first k
    candidates, then batches of B candidates; within a batch the threshold d_k
    is frozen, every candidate advances one level at a time and is pruned as
    soon as LB_eps^l > d_k (strict); survivors' exact distances are pushed to H,
    which is cropped to k.

Readings (where the paper is silent):
  * The "exact distance" pushed to H is the canonical D of oracle.brute
    (sequential FP64 over the raw rows, rounded to FP32); ties at equal D are
    broken by the smaller id, and exactly k results are returned.
  * Candidates are visited in the order given (probe rank, then list
    position); the first k seed H and the batches cover the rest.
  * The pruning test carries a slack 2^-22 d_k + 1e-11 (R_q + R_x) so that FP64
    rounding of LB and the FP32 rounding of D can never prune a candidate whose
    canonical D equals or beats d_k.
"""
from __future__ import annotations

import math
import numpy as np

from .brute import canonical_dist, topk_by_key


def pca_fit(xs: np.ndarray, sample: np.ndarray | None = None):
    """Centred PCA in FP64.  Returns mu [d], T [d, d] (rows = eigenvectors,
    descending eigenvalue), lam [d]."""
    x64 = np.asarray(xs if sample is None else xs[sample], dtype=np.float64)
    mu = x64.mean(axis=0)
    xc = x64 - mu
    cov = (xc.T @ xc) / x64.shape[0]
    lam, vec = np.linalg.eigh(cov)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    t = vec[:, order].T.copy()
    piv = np.argmax(np.abs(t), axis=1)
    sgn = np.sign(t[np.arange(t.shape[0]), piv])
    sgn[sgn == 0] = 1.0
    t *= sgn[:, None]
    return mu, t, lam


def apply_transform(mu: np.ndarray, t: np.ndarray, v: np.ndarray) -> np.ndarray:
    """T (v - mu) in FP64 for rows v [n, d] (or one vector)."""
    v64 = np.asarray(v, dtype=np.float64)
    return (v64 - mu) @ t.T


def tail_energies(y: np.ndarray, m) -> np.ndarray:
    """R^(l,d) = sum_{j > m_l} y_j^2 for l = 0..L (Eq. 2); shape [..., L+1]."""
    m = list(m)
    y = np.asarray(y, dtype=np.float64)
    sq = y * y
    out = [sq[..., m[l]:].sum(axis=-1) for l in range(len(m))]
    return np.stack(out, axis=-1)


def energy_profile(lam: np.ndarray) -> np.ndarray:
    """E(m) = sum_{j>m} lam_j / sum_j lam_j for m = 0..d (Section 4.1)."""
    lam = np.asarray(lam, dtype=np.float64)
    tail = np.concatenate([np.cumsum(lam[::-1])[::-1], [0.0]])
    return tail / tail[0]


def alpha_fit(lam: np.ndarray) -> float:
    """Least-squares fit (through the origin) of log E(m) ~ -alpha m / d over
    the levels where E(m) >= 1e-3, i.e. the range a pruning threshold can use."""
    e = energy_profile(lam)
    d = lam.shape[0]
    mm = np.arange(d + 1, dtype=np.float64)
    ok = (e >= 1e-3) & (mm < d)
    x = mm[ok] / d
    y = np.log(e[ok])
    return float(-(x @ y) / (x @ x))


def bounds_trace(q: np.ndarray, x: np.ndarray, mu, t, m, eps: float = 1.0) -> dict:
    """Per-level quantities of Eq. 3/4 for one (query, candidate) pair, l = 0..L.
    Level 0 reads no coordinate (p = 0)."""
    m = list(m)
    tq = apply_transform(mu, t, q)
    tx = apply_transform(mu, t, x)
    rq = tail_energies(tq, m)
    rx = tail_energies(tx, m)
    L = len(m) - 1
    p = np.zeros(L + 1)
    for l in range(1, L + 1):
        p[l] = p[l - 1] + float(tq[m[l - 1]:m[l]] @ tx[m[l - 1]:m[l]])
    a = rq[0] + rx[0] - 2.0 * p
    c = np.sqrt(rq * rx)
    return {"A": a, "C": c, "LB": a - 2.0 * eps * c, "UB": a + 2.0 * c, "p": p,
            "Rq": rq, "Rx": rx, "tq": tq, "tx": tx}


def panorama_knn(q: np.ndarray, xs: np.ndarray, ids: np.ndarray, mu, t, m, k: int,
                 batch: int = 1024, eps: float = 1.0):
    """Algorithm 1 over the candidates xs [n, d] (raw rows) with ids [n], in the
    given order.  Returns (ids [k], dists [k], rho [n]) where rho is the number
    of dimensions read per candidate (d for the seed and for survivors)."""
    m = [int(v) for v in m]
    L = len(m) - 1
    d = m[-1]
    n = xs.shape[0]
    ids = np.asarray(ids, dtype=np.int64)
    rho = np.zeros(n, dtype=np.int64)
    # Precompute for the query: T(q), ||T(q)||^2 and every tail R_q^(l,d).
    tq = apply_transform(mu, t, q)
    rq = tail_energies(tq, m)

    # Seed the heap with the exact distances of the first k candidates.
    s = min(k, n)
    h_d = canonical_dist(q, xs[:s]).astype(np.float32)
    h_i = ids[:s].copy()
    rho[:s] = d
    h_i, h_d = _crop(h_d, h_i, k)
    dk = float(h_d[k - 1]) if h_i.size >= k else math.inf

    for b0 in range(s, n, batch):
        b1 = min(n, b0 + batch)
        tx = apply_transform(mu, t, xs[b0:b1])
        rx = tail_energies(tx, m)
        active = np.ones(b1 - b0, dtype=bool)
        p = np.zeros(b1 - b0)
        slack = 2.0 ** -22 * dk + 1e-11 * (rq[0] + rx[:, 0])
        for l in range(1, L + 1):
            lo, hi = m[l - 1], m[l]
            act = np.nonzero(active)[0]
            p[act] += tx[act, lo:hi] @ tq[lo:hi]
            lb = relaxed_lower_bound(rq[0], rx[act, 0], p[act], rq[l], rx[act, l], eps)
            pruned = lb > dk + slack[act]
            rho[b0 + act[pruned]] = hi
            active[act[pruned]] = False
        surv = np.nonzero(active)[0]
        rho[b0 + surv] = d
        if surv.size:
            dd = canonical_dist(q, xs[b0 + surv])
            # Push every survivor, then crop H to k and refresh d_k.
            h_d = np.concatenate([h_d, dd])
            h_i = np.concatenate([h_i, ids[b0 + surv]])
            h_i, h_d = _crop(h_d, h_i, k)
            dk = float(h_d[k - 1]) if h_i.size >= k else math.inf
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float32)
    out_i[: h_i.size] = h_i
    out_d[: h_d.size] = h_d
    return out_i, out_d, rho


def relaxed_lower_bound(rq0, rx0, p, rql, rxl, eps):
    """Eq. 4: LB_eps = A - 2 eps C, A = R_q^(0,d) + R_x^(0,d) - 2 p^(0,l),
    C = sqrt(R_q^(l,d) R_x^(l,d)); eps = 1 gives Eq. 3."""
    a = rq0 + rx0 - 2.0 * p
    c = np.sqrt(rql * rxl)
    return a - 2.0 * eps * c


def _crop(dist, ids, k):
    order = np.lexsort((ids, dist))[:k]
    return ids[order], dist[order]


def panorama_refine(q: np.ndarray, xs: np.ndarray, cand: np.ndarray, mu, t, m, k: int, eps: float = 1.0):
    """Refine with the point-centric form of Algorithm 1 (Table of the two
    modes: B = 1; Section 6.4): the query's candidate ids in their given order
    (-1 entries skipped), each early-abandoned at its first level whose bound
    exceeds the running d_k, which every survivor updates."""
    cand = np.asarray(cand, dtype=np.int64)
    ids = cand[cand >= 0]
    return panorama_knn(q, xs[ids], ids, mu, t, m, k, batch=1, eps=eps)


def ivf_candidates(probes, assign: np.ndarray) -> np.ndarray:
    """Candidate order for the IVF scan: probe rank, then position in the list
    (ascending row id)."""
    assign = np.asarray(assign)
    parts = [np.nonzero(assign == int(l))[0] for l in probes]
    return np.concatenate(parts).astype(np.int64) if parts else np.empty(0, np.int64)


def panorama_knn_ivf(qs, xs, centroids, assign, nprobe, mu, t, m, k, batch=1024, eps=1.0):
    """Algorithm 1 over each query's probed lists.  Returns ids, dists, and the
    fraction of dimensions read (phi) per query."""
    from .brute import probe_lists
    qs = np.atleast_2d(qs)
    probes = probe_lists(qs, centroids, nprobe)
    out_i = np.full((qs.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((qs.shape[0], k), np.inf, dtype=np.float32)
    phi = np.zeros(qs.shape[0])
    d = xs.shape[1]
    for qi in range(qs.shape[0]):
        cand = ivf_candidates(probes[qi], assign)
        if cand.size == 0:
            continue
        out_i[qi], out_d[qi], rho = panorama_knn(qs[qi], xs[cand], cand, mu, t, m, k, batch, eps)
        phi[qi] = rho.sum() / (cand.size * d)
    return out_i, out_d, phi
