"""Oracle O4: the IVFPQ form of the method (Section 4.2 spectrum shaping,
Section 6.2 the PQ scan), in FP64.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.

What it follows:
  * Section 4.2, Procedure 1 (inter-level shaping): the coordinates of the PCA
    frame carry expected variances v (at first the eigenvalues).  Level
    energies E_l are the sums of v over each level; the cap is tau = kappa *
    mean(E_l).  Levels are visited front to back; a level over the cap is
    rotated together with the fewest following coordinates s >= 1 for which
    its expected energy after a Haar rotation of that block, b_l / (b_l + s)
    times the block's total, is at most tau (s stops at the last coordinate;
    "at most" allows a relative 1e-9 for rounding).
    After the rotation every coordinate of the block carries the block's mean
    variance.  The plan is the ordered list of rotated blocks.
  * Section 4.2, Procedure 2 (intra-level isotropization): one Haar rotation
    per level's coordinates.  The combined transform is U R T_PCA.
  * Section 6.2 (IVFPQ): each vector's residual against its list centroid,
    in the shaped frame, is split into M sub-vectors of dsub coordinates, each
    coded by one of 256 codewords; per probed list the query's look-up table
    holds the squared distance of each sub-vector of the query's residual
    against that list's centroid to each codeword, and a candidate's distance
    is the sum of its M table entries (asymmetric distance computation).
  * The bound of Eq. 3/4 applied to the reconstruction xhat: after the
    levels 1..l the partial sum P_l of the table entries is the head term,
    and LB = P_l + (a - b)^2 + 2 (1 - eps) a b with a, b the norms of the query
    and of xhat beyond level l (the same closed form as for flat vectors).
  * Algorithm 1 with these quantities: a heap seeded by the exact distances of
    the first k candidates, then batches whose candidates advance one level at
    a time and are dropped once LB exceeds the frozen d_k.

Readings (where the paper is silent):
  * The query in the shaped frame is y_i = sum_j T_ij (q_j - mu_j), summed
    sequentially in j in FP64 with every operation rounded separately.
  * A table entry is float32 of the sequential FP64 sum over the sub-vector's
    coordinates of (y_j - c_j)^2; the distance ADC(q, x) is float32 of the
    sequential FP64 sum of the candidate's M entries in sub-quantizer order.
  * The answer is the first k candidates by (ADC, id) over the probed lists
    (probe sets as in oracle.brute); the PQ codes are not re-ranked.
  * Residual codes, as IVFPQ stores them: a vector of list l is coded as
    T (x - mu) - y_c(l), with y_c(l) = T (c_l - mu) by the same sequential
    FP64 recipe as the queries; the query's residual for list l is
    z = y - y_c(l) (FP64 differences), and its tail norms beyond each level are
    those of z.
"""
from __future__ import annotations

import math
import numpy as np

from .brute import probe_lists


# ------------------------------------------------------------------ shaping
def robin_hood_plan(lam, cuts, kappa: float):
    """Procedure 1 on expected variances.  Returns (blocks, v): blocks is a
    list of (start, length) coordinate ranges, rotated in this order; v the
    expected per-coordinate variances afterwards."""
    # every sum is taken in coordinate order (Python's sum adds left to right)
    v = [float(x) for x in np.asarray(lam, dtype=np.float64)]
    m = [int(c) for c in cuts]
    L = len(m) - 1
    d = m[-1]
    # an energy within a relative 1e-9 of the cap counts as within it, so that
    # rounding alone never asks for a rotation
    tau = kappa * sum(v) / L
    cap = tau * (1.0 + 1e-9)
    blocks = []
    for l in range(L):
        lo, hi = m[l], m[l + 1]
        b = hi - lo
        if sum(v[lo:hi]) <= cap:
            continue
        s = 1
        while hi + s < d and b / (b + s) * sum(v[lo:hi + s]) > cap:
            s += 1
        s = min(s, d - hi)
        if s == 0:
            continue
        mean = sum(v[lo:hi + s]) / (b + s)
        v[lo:hi + s] = [mean] * (b + s)
        blocks.append((lo, b + s))
    return blocks, np.asarray(v)


def level_energies(v, cuts) -> np.ndarray:
    m = [int(c) for c in cuts]
    return np.array([np.asarray(v)[m[l]:m[l + 1]].sum() for l in range(len(m) - 1)])


def shaped_transform(t_pca: np.ndarray, cuts, blocks, block_rots, level_rots) -> np.ndarray:
    """U R T_PCA: R rotates each plan block (block_rots[i] is its orthogonal
    matrix) in plan order; U applies level_rots[l] to level l's coordinates
    (None: identity)."""
    t = np.array(t_pca, dtype=np.float64)
    for (s, n), q in zip(blocks, block_rots):
        t[s:s + n] = q @ t[s:s + n]
    m = [int(c) for c in cuts]
    for l, q in enumerate(level_rots):
        if q is not None:
            t[m[l]:m[l + 1]] = q @ t[m[l]:m[l + 1]]
    return t


# ------------------------------------------------------------------ queries and tables
def shaped_query(qs: np.ndarray, mu: np.ndarray, t: np.ndarray) -> np.ndarray:
    """y = T (q - mu) per row, each coordinate a sequential FP64 sum over j."""
    q64 = np.atleast_2d(np.asarray(qs, dtype=np.float32)).astype(np.float64)
    qc = q64 - np.asarray(mu, dtype=np.float64)[None, :]
    t = np.asarray(t, dtype=np.float64)
    y = np.zeros((qc.shape[0], t.shape[0]))
    for j in range(t.shape[1]):
        y = y + t[None, :, j] * qc[:, j, None]
    return y


def lut(y: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """Table of one query: float32 [M, 256]; entry (m, c) = sum over the
    sub-vector's coordinates of (y_j - C[m, c, j])^2, sequential in FP64."""
    cb = np.asarray(codebooks, dtype=np.float32).astype(np.float64)
    M, K, dsub = cb.shape
    ys = np.asarray(y, dtype=np.float64).reshape(M, 1, dsub)
    s = np.zeros((M, K))
    for j in range(dsub):
        t = ys[:, :, j] - cb[:, :, j]
        s = s + t * t
    return s.astype(np.float32)


def adc(tab: np.ndarray, codes: np.ndarray) -> np.ndarray:
    """ADC of rows with codes [n, M] (uint8) under one query's table [M, 256]:
    float32 of the sequential FP64 sum over m."""
    codes = np.atleast_2d(np.asarray(codes))
    s = np.zeros(codes.shape[0])
    for mm in range(codes.shape[1]):
        s = s + tab[mm, codes[:, mm]].astype(np.float64)
    return s.astype(np.float32)


def reconstruct(codes: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """xhat in the shaped frame, FP64 [n, M * dsub]."""
    cb = np.asarray(codebooks, dtype=np.float32).astype(np.float64)
    codes = np.atleast_2d(np.asarray(codes))
    M = cb.shape[0]
    return np.concatenate([cb[mm, codes[:, mm]] for mm in range(M)], axis=1)


def tails(v: np.ndarray, cuts) -> np.ndarray:
    """Norms beyond each level, sqrt(sum_{j >= m_l} v_j^2) for l = 0..L, of
    rows v [n, d] (FP64)."""
    m = [int(c) for c in cuts]
    sq = np.asarray(v, dtype=np.float64) ** 2
    return np.stack([np.sqrt(sq[:, m[l]:].sum(axis=1)) for l in range(len(m))], axis=1)


def encode(y: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """Nearest codeword per sub-vector by (squared distance in FP64, code)."""
    cb = np.asarray(codebooks, dtype=np.float32).astype(np.float64)
    M, K, dsub = cb.shape
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    out = np.empty((y.shape[0], M), dtype=np.uint8)
    for mm in range(M):
        sub = y[:, mm * dsub:(mm + 1) * dsub]
        dd = ((sub[:, None, :] - cb[mm][None, :, :]) ** 2).sum(axis=2)
        out[:, mm] = np.argmin(dd, axis=1)  # first minimum: the smaller code
    return out


# ------------------------------------------------------------------ searches
def _members(assign, nlist):
    order = np.argsort(assign, kind="stable")
    bounds = np.searchsorted(np.asarray(assign)[order], np.arange(nlist + 1))
    return [order[bounds[l]:bounds[l + 1]] for l in range(nlist)]


def _topk(dist, ids, k):
    order = np.lexsort((ids, dist))[:k]
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float32)
    out_i[:order.size] = ids[order]
    out_d[:order.size] = dist[order]
    return out_i, out_d


def pq_knn_ivf(qs, mu, t, codebooks, codes, centroids, assign, nprobe, k):
    """O-PQ1: first k by (ADC, id) over each query's probed lists (brute force
    over the codes, each list with its own table).  Returns ids [nq, k] int64,
    dists [nq, k] float32."""
    qs = np.atleast_2d(qs)
    probes = probe_lists(qs, centroids, nprobe)
    mem = _members(assign, centroids.shape[0])
    y = shaped_query(qs, mu, t)
    yc = shaped_query(centroids, mu, t)
    out_i = np.full((qs.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((qs.shape[0], k), np.inf, dtype=np.float32)
    for qi in range(qs.shape[0]):
        ids, dist = [], []
        for l in probes[qi]:
            mm = mem[int(l)]
            if mm.size:
                ids.append(mm.astype(np.int64))
                dist.append(adc(lut(y[qi] - yc[int(l)], codebooks), codes[mm]))
        if ids:
            out_i[qi], out_d[qi] = _topk(np.concatenate(dist), np.concatenate(ids), k)
    return out_i, out_d


def pq_lower_bound(p, a, b, eps):
    """LB = P + (a - b)^2 + 2 (1 - eps) a b (Eq. 3/4 with the head term P)."""
    return p + (a - b) ** 2 + 2.0 * (1.0 - eps) * a * b


def panorama_pq_knn(zs, tabs, which, codes, xt, ids, sub_cuts, k, batch=1024, eps=1.0):
    """Algorithm 1 over one query's candidates in the given order.  zs [p, d]
    the query's residuals against its p probed lists, tabs [p, M, 256] their
    tables, which [n] the list (index into zs) of each candidate, codes [n, M],
    xt [n, L+1] the norms of xhat beyond each level, sub_cuts the level cuts in
    sub-quantizer units.  Returns (ids [k], dists [k], subs_read [n])."""
    sub_cuts = [int(c) for c in sub_cuts]
    L = len(sub_cuts) - 1
    M = sub_cuts[-1]
    dsub = zs.shape[1] // M
    n = codes.shape[0]
    ids = np.asarray(ids, dtype=np.int64)
    which = np.asarray(which, dtype=np.int64)
    zt = tails(zs, [c * dsub for c in sub_cuts])  # [p, L+1]
    read = np.zeros(n, dtype=np.int64)

    def full(rows):
        out = np.zeros(rows.size, dtype=np.float32)
        for w in np.unique(which[rows]):
            sel = which[rows] == w
            out[sel] = adc(tabs[w], codes[rows[sel]])
        return out

    s = min(k, n)
    h_d = full(np.arange(s))
    h_i = ids[:s].copy()
    read[:s] = M
    h_i, h_d = _crop(h_d, h_i, k)
    dk = float(h_d[k - 1]) if h_i.size >= k else math.inf
    for b0 in range(s, n, batch):
        b1 = min(n, b0 + batch)
        active = np.ones(b1 - b0, dtype=bool)
        p = np.zeros(b1 - b0)
        for l in range(1, L + 1):
            act = np.nonzero(active)[0]
            wl = which[b0 + act]
            for mm in range(sub_cuts[l - 1], sub_cuts[l]):
                p[act] += tabs[wl, mm, codes[b0 + act, mm]].astype(np.float64)
            read[b0 + act] = sub_cuts[l]
            if l == L:
                break
            a = zt[wl, l]
            lb = pq_lower_bound(p[act], a, xt[b0 + act, l], eps)
            # slack for the FP32 rounding of the table entries and of ADC
            pruned = lb > dk + 2.0 ** -20 * (dk + p[act] + (a + xt[b0 + act, l]) ** 2)
            active[act[pruned]] = False
        surv = np.nonzero(active)[0]
        if surv.size:
            dd = full(b0 + surv)
            h_d = np.concatenate([h_d, dd])
            h_i = np.concatenate([h_i, ids[b0 + surv]])
            h_i, h_d = _crop(h_d, h_i, k)
            dk = float(h_d[k - 1]) if h_i.size >= k else math.inf
    out_i = np.full(k, -1, dtype=np.int64)
    out_d = np.full(k, np.inf, dtype=np.float32)
    out_i[:h_i.size] = h_i
    out_d[:h_d.size] = h_d
    return out_i, out_d, read


def _crop(dist, ids, k):
    order = np.lexsort((ids, dist))[:k]
    return ids[order], dist[order]


def panorama_pq_knn_ivf(qs, mu, t, codebooks, codes, centroids, assign, nprobe, k, sub_cuts,
                        batch=1024, eps=1.0):
    """Algorithm 1 over each query's probed lists (probe rank, then ascending
    row id).  Returns ids, dists and the fraction of table look-ups done."""
    qs = np.atleast_2d(qs)
    probes = probe_lists(qs, centroids, nprobe)
    mem = _members(assign, centroids.shape[0])
    y = shaped_query(qs, mu, t)
    yc = shaped_query(centroids, mu, t)
    cb = np.asarray(codebooks)
    M, _, dsub = cb.shape
    xt = tails(reconstruct(codes, cb), [c * dsub for c in sub_cuts])
    out_i = np.full((qs.shape[0], k), -1, dtype=np.int64)
    out_d = np.full((qs.shape[0], k), np.inf, dtype=np.float32)
    frac = np.zeros(qs.shape[0])
    for qi in range(qs.shape[0]):
        parts = [mem[int(l)] for l in probes[qi]]
        cand = np.concatenate(parts).astype(np.int64)
        if cand.size == 0:
            continue
        which = np.concatenate([np.full(pp.size, i, np.int64) for i, pp in enumerate(parts)])
        zs = np.stack([y[qi] - yc[int(l)] for l in probes[qi]])
        tabs = np.stack([lut(z, cb) for z in zs])
        out_i[qi], out_d[qi], rd = panorama_pq_knn(zs, tabs, which, codes[cand], xt[cand], cand, sub_cuts, k,
                                                   batch, eps)
        frac[qi] = rd.sum() / (cand.size * M)
    return out_i, out_d, frac
