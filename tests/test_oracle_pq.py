"""Pins of the IVFPQ oracle (oracle/pq.py) against what the paper and the
mathematics fix: hand-worked plans of Section 4.2's Procedure 1, the order of
the shaped transform's composition, closed forms of the table and its
distance, the bound below the distance at every level, Algorithm 1 equal to
the brute force at eps = 1, and planted mistakes that must fail.  CPU only."""
import math

import numpy as np
import pytest

from oracle import brute, pq


# ------------------------------------------------------------------ Procedure 1
def test_plan_hand_example_full_equalization():
    """lambda = (8, 4, 2, 1, 1, 0, 0, 0), four levels of two: mean level
    energy 4.  With kappa = 1 (tau = 4) level 1 (energy 12) needs every
    following coordinate: 2/(2+s) * 16 <= 4 first holds at s = 6."""
    blocks, v = pq.robin_hood_plan([8, 4, 2, 1, 1, 0, 0, 0], [0, 2, 4, 6, 8], 1.0)
    assert blocks == [(0, 8)]
    assert np.array_equal(v, np.full(8, 2.0))


def test_plan_hand_example_kappa_two():
    """kappa = 2 (tau = 8): level 1 with two more coordinates gives
    2/4 * 15 = 7.5 <= 8 (one more gives 2/3 * 14 = 9.33 > 8); levels 2-4 then
    hold 7.5, 1 and 0."""
    blocks, v = pq.robin_hood_plan([8, 4, 2, 1, 1, 0, 0, 0], [0, 2, 4, 6, 8], 2.0)
    assert blocks == [(0, 4)]
    assert np.allclose(v, [3.75, 3.75, 3.75, 3.75, 1, 0, 0, 0], rtol=0, atol=0)
    assert np.allclose(pq.level_energies(v, [0, 2, 4, 6, 8]), [7.5, 7.5, 1, 0])


def test_plan_second_level_rotated():
    """A plan with two blocks: lambda = (5, 5, 5, 5, 0, 0, 0, 0), kappa = 1
    (tau = 5).  Level 1 (10) takes two coordinates (2/4 * 20 = 10 > 5 fails
    at s = 2, 2/5 * 20 = 8 at s = 3, 2/6 * 20 = 6.67 at s = 4, 2/7 * 20 = 5.71
    at s = 5, 2/8 * 20 = 5 at s = 6)."""
    blocks, v = pq.robin_hood_plan([5, 5, 5, 5, 0, 0, 0, 0], [0, 2, 4, 6, 8], 1.0)
    assert blocks == [(0, 8)]
    assert np.allclose(v, 2.5)
    # unequal levels: the first level of three coordinates
    blocks, v = pq.robin_hood_plan([6, 3, 3, 3, 0, 0], [0, 3, 4, 6], 1.0)
    # tau = 15/3 = 5: level 1 has 12: s = 1 gives 3/4 * 15 = 11.25, s = 2:
    # 3/5 * 15 = 9, s = 3: 3/6 * 15 = 7.5 and s stops at the end (6 - 3 = 3)
    assert blocks == [(0, 6)]
    assert np.allclose(v, 2.5)


@pytest.mark.parametrize("kappa", [1.0, 1.5, 2.0, 4.0])
def test_plan_caps_and_minimality(kappa):
    """Every rotated level ends at or below the cap, no shorter block would
    do, and levels already under the cap are left alone."""
    d, L = 96, 8
    cuts = list(range(0, d + 1, d // L))
    lam = np.exp(-0.08 * np.arange(d))
    blocks, v = pq.robin_hood_plan(lam, cuts, kappa)
    tau = kappa * sum(lam.tolist()) / L
    cap = tau * (1 + 1e-9)
    e = pq.level_energies(v, cuts)
    assert (e <= cap).all() or blocks[-1][0] + blocks[-1][1] == d
    # rounding alone asks for no rotation: a level is rotated at most once
    assert len({s0 for s0, _ in blocks}) == len(blocks)
    # replay: each block is the shortest that meets the cap
    w = [float(x) for x in lam]
    for s0, n in blocks:
        lvl = cuts.index(s0)
        b = cuts[lvl + 1] - s0
        assert sum(w[s0:s0 + b]) > cap
        assert b / n * sum(w[s0:s0 + n]) <= cap or s0 + n == d
        if n - 1 > b:
            assert b / (n - 1) * sum(w[s0:s0 + n - 1]) > cap
        w[s0:s0 + n] = [sum(w[s0:s0 + n]) / n] * n
    assert np.allclose(w, v, rtol=0, atol=0)
    # total energy is preserved
    assert math.isclose(v.sum(), lam.sum(), rel_tol=1e-12)


def test_plan_flat_spectrum_untouched():
    lam = np.ones(32)
    blocks, v = pq.robin_hood_plan(lam, list(range(0, 33, 8)), 1.0)
    assert blocks == [] and np.array_equal(v, lam)


# ------------------------------------------------------------------ composition
def test_shaped_transform_composition_order():
    """R acts first (plan order), then the level rotations; both left-multiply
    the rows they own."""
    t = np.eye(4)
    swap = np.array([[0.0, 1.0], [-1.0, 0.0]])
    out = pq.shaped_transform(t, [0, 2, 4], [(1, 2)], [swap], [None, None])
    assert np.array_equal(out, np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, -1, 0, 0], [0, 0, 0, 1]], float))
    out2 = pq.shaped_transform(t, [0, 2, 4], [(1, 2)], [swap], [swap, None])
    # level 1 (rows 0, 1) rotated after the block rotation
    assert np.array_equal(out2[:2], swap @ out[:2])
    assert np.array_equal(out2[2:], out[2:])


# ------------------------------------------------------------------ tables and distances
def test_shaped_query_hand_and_order():
    t = np.array([[1.0, 2.0], [3.0, 4.0]])
    y = pq.shaped_query(np.array([[2.0, 3.0]], np.float32), np.array([1.0, 1.0]), t)
    assert np.array_equal(y, [[5.0, 11.0]])
    # the sum runs in coordinate order: ((0 + 1) + 1e-16) - 1 = 0 in FP64
    t3 = np.array([[1.0, 1e-16, -1.0]])
    y3 = pq.shaped_query(np.array([[1.0, 1.0, 1.0]], np.float32), np.zeros(3), t3)
    assert y3[0, 0] == 0.0


def test_lut_closed_form():
    """dsub = 2, M = 2, y = (1, 2, 3, 4); codewords C[0][c] = (c, 0),
    C[1][c] = (0, c): entries (1 - c)^2 + 4 and 9 + (4 - c)^2."""
    cb = np.zeros((2, 256, 2), np.float32)
    c = np.arange(256, dtype=np.float32)
    cb[0, :, 0] = c
    cb[1, :, 1] = c
    tab = pq.lut(np.array([1.0, 2.0, 3.0, 4.0]), cb)
    assert np.array_equal(tab[0], ((1 - c) ** 2 + 4).astype(np.float32))
    assert np.array_equal(tab[1], (9 + (4 - c) ** 2).astype(np.float32))


def test_adc_sums_in_fp64_then_rounds():
    """Entries (2^24, 1, 1): the FP64 sum 2^24 + 2 is a float; an FP32 running
    sum would give 2^24."""
    tab = np.zeros((3, 256), np.float32)
    tab[0, 5] = 2.0 ** 24
    tab[1, 7] = 1.0
    tab[2, 9] = 1.0
    v = pq.adc(tab, np.array([[5, 7, 9]], np.uint8))
    assert v[0] == np.float32(16777218.0)


def test_adc_equals_exact_distance_when_codewords_are_the_rows():
    """Identity transform, integer rows whose sub-vectors are codewords: the
    table distance is the exact squared distance (small integers), equal to
    the canonical distance of oracle.brute."""
    g = np.random.default_rng(7)
    n, d, dsub = 40, 8, 2
    M = d // dsub
    x = g.integers(-5, 6, size=(n, d)).astype(np.float32)
    qv = g.integers(-5, 6, size=(3, d)).astype(np.float32)
    cb = np.zeros((M, 256, dsub), np.float32)
    codes = np.zeros((n, M), np.uint8)
    for m in range(M):
        sub = x[:, m * dsub:(m + 1) * dsub]
        uniq, inv = np.unique(sub, axis=0, return_inverse=True)
        cb[m, :uniq.shape[0]] = uniq
        cb[m, uniq.shape[0]:] = 100.0
        codes[:, m] = inv.reshape(-1)
    y = pq.shaped_query(qv, np.zeros(d), np.eye(d))
    for qi in range(3):
        got = pq.adc(pq.lut(y[qi], cb), codes)
        assert np.array_equal(got, brute.canonical_dist(qv[qi], x))
    assert np.array_equal(pq.reconstruct(codes, cb), x.astype(np.float64))


def test_tails_and_encode():
    g = np.random.default_rng(3)
    v = g.standard_normal((5, 6))
    t = pq.tails(v, [0, 2, 6])
    assert np.allclose(t[:, 0], np.linalg.norm(v, axis=1))
    assert np.allclose(t[:, 1], np.linalg.norm(v[:, 2:], axis=1))
    assert np.array_equal(t[:, 2], np.zeros(5))
    cb = g.standard_normal((3, 256, 2)).astype(np.float32)
    y = g.standard_normal((7, 6))
    codes = pq.encode(y, cb)
    for r in range(7):
        for m in range(3):
            dd = [((y[r, 2 * m:2 * m + 2] - cb[m, c].astype(np.float64)) ** 2).sum() for c in range(256)]
            assert codes[r, m] == int(np.argmin(dd))


def test_pq_lower_bound_closed_form():
    assert pq.pq_lower_bound(1.0, 3.0, 1.0, 1.0) == 5.0
    assert pq.pq_lower_bound(1.0, 3.0, 1.0, 0.5) == 8.0
    assert pq.pq_lower_bound(2.0, 1.0, 1.0, 1.0) == 2.0


def _random_pq(seed, n=600, d=32, dsub=4):
    g = np.random.default_rng(seed)
    M = d // dsub
    lam = np.exp(-0.3 * np.arange(d))
    x = (g.standard_normal((n, d)) * np.sqrt(lam)).astype(np.float32)
    cb = (g.standard_normal((M, 256, dsub)) * np.sqrt(lam.reshape(M, dsub))[:, None, :]).astype(np.float32)
    y = pq.shaped_query(x, np.zeros(d), np.eye(d))
    codes = pq.encode(y, cb)
    qs = (g.standard_normal((6, d)) * np.sqrt(lam)).astype(np.float32)
    return x, qs, cb, codes


def test_lower_bound_below_distance_every_level():
    """LB (eps = 1) <= the table distance at every level, for every candidate
    (Eq. 3 with the head term given by the table)."""
    x, qs, cb, codes = _random_pq(11)
    d = x.shape[1]
    M, _, dsub = cb.shape
    sub_cuts = [0, 2, 4, 6, 8]
    xt = pq.tails(pq.reconstruct(codes, cb), [c * dsub for c in sub_cuts])
    for qi in range(qs.shape[0]):
        y = pq.shaped_query(qs[qi:qi + 1], np.zeros(d), np.eye(d))[0]
        tab = pq.lut(y, cb)
        full = pq.adc(tab, codes).astype(np.float64)
        yt = pq.tails(y[None, :], [c * dsub for c in sub_cuts])[0]
        p = np.zeros(codes.shape[0])
        for l in range(1, len(sub_cuts)):
            for m in range(sub_cuts[l - 1], sub_cuts[l]):
                p += tab[m, codes[:, m]].astype(np.float64)
            lb = pq.pq_lower_bound(p, yt[l], xt[:, l], 1.0)
            assert (lb <= full * (1 + 1e-6) + 1e-9).all()
            assert (pq.pq_lower_bound(p, yt[l], xt[:, l], 0.5) >= lb).all()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_panorama_pq_equals_brute_at_eps_one(seed):
    x, qs, cb, codes = _random_pq(seed)
    d = x.shape[1]
    cent = np.zeros((1, d), np.float32)
    assign = np.zeros(x.shape[0], np.int64)
    ri, rd = pq.pq_knn_ivf(qs, np.zeros(d), np.eye(d), cb, codes, cent, assign, 1, 10)
    for batch in (1, 16, 1024):
        gi, gd, frac = pq.panorama_pq_knn_ivf(qs, np.zeros(d), np.eye(d), cb, codes, cent, assign, 1, 10,
                                              [0, 2, 4, 6, 8], batch=batch)
        assert np.array_equal(gi, ri) and np.array_equal(gd, rd)
        assert (frac <= 1.0).all() and (frac > 0).all()
    # pruning happens on this spectrum
    assert frac.mean() < 0.99


def test_planted_bound_mistakes_fail(monkeypatch):
    """A plausible slip in the bound (the tail term's sign, or a dropped head
    term) breaks equality with the brute-force answer or LB <= distance."""
    x, qs, cb, codes = _random_pq(5)
    d = x.shape[1]
    cent = np.zeros((1, d), np.float32)
    assign = np.zeros(x.shape[0], np.int64)
    ri, rd = pq.pq_knn_ivf(qs, np.zeros(d), np.eye(d), cb, codes, cent, assign, 1, 10)
    good = pq.pq_lower_bound
    for bad in (lambda p, a, b, e: p + (a + b) ** 2 + 2 * (1 - e) * a * b,
                lambda p, a, b, e: 2 * p + (a - b) ** 2):
        monkeypatch.setattr(pq, "pq_lower_bound", bad)
        gi, gd, _ = pq.panorama_pq_knn_ivf(qs, np.zeros(d), np.eye(d), cb, codes, cent, assign, 1, 10,
                                           [0, 2, 4, 6, 8], batch=16)
        assert not np.array_equal(gi, ri)
    monkeypatch.setattr(pq, "pq_lower_bound", good)


def test_pq_knn_ivf_probes_and_ties():
    """Two lists, probe one: only its members answer; equal codes tie and are
    ordered by id."""
    d, dsub = 4, 2
    cb = np.zeros((2, 256, 2), np.float32)
    cb[0, :, 0] = np.arange(256)
    cb[1, :, 1] = np.arange(256)
    codes = np.array([[3, 3], [1, 1], [1, 1], [0, 2], [9, 9]], np.uint8)
    assign = np.array([0, 0, 0, 1, 1])
    cent = np.array([[0, 0, 0, 0], [50, 50, 50, 50]], np.float32)
    q = np.zeros((1, d), np.float32)
    ids, dd = pq.pq_knn_ivf(q, np.zeros(d), np.eye(d), cb, codes, cent, assign, 1, 4)
    # distances: row 0: 9 + 9, rows 1, 2: 1 + 1 (tie, by id)
    assert ids[0].tolist() == [1, 2, 0, -1]
    assert dd[0, :3].tolist() == [2.0, 2.0, 18.0] and np.isinf(dd[0, 3])


def test_residual_table_hand_example():
    """A member of list 1 (centroid (10, 10, 10, 10)) coded (1, 1) with
    codewords C[0][1] = (1, 0) and C[1][1] = (0, 1) is reconstructed as
    (11, 10, 10, 11); for q = (10, 10, 10, 10) the residual is 0 and the
    distance is 1 + 1."""
    cb = np.full((2, 256, 2), 50.0, np.float32)
    cb[0, 1] = (1.0, 0.0)
    cb[1, 1] = (0.0, 1.0)
    cent = np.array([[0, 0, 0, 0], [10, 10, 10, 10]], np.float32)
    codes = np.array([[0, 0], [1, 1]], np.uint8)
    assign = np.array([0, 1])
    q = np.full((1, 4), 10.0, np.float32)
    ids, dd = pq.pq_knn_ivf(q, np.zeros(4), np.eye(4), cb, codes, cent, assign, 1, 2)
    assert ids[0].tolist() == [1, -1] and dd[0, 0] == 2.0
    ids, dd = pq.pq_knn_ivf(q, np.zeros(4), np.eye(4), cb, codes, cent, assign, 2, 2)
    # row 0 (list 0, centroid 0, codewords (50, 50) twice): 4 * 40^2
    assert ids[0].tolist() == [1, 0] and dd[0].tolist() == [2.0, 6400.0]


@pytest.mark.parametrize("seed", [4, 9])
def test_panorama_pq_residual_lists_equal_brute(seed):
    """Four clusters with their own centroids, residual codes, two probed
    lists: Algorithm 1 with per-list tables equals the brute force at eps = 1,
    and LB <= distance for every candidate at every level."""
    g = np.random.default_rng(seed)
    d, dsub, n = 32, 4, 800
    M = d // dsub
    cent = (g.standard_normal((4, d)) * 6).astype(np.float32)
    assign = g.integers(0, 4, size=n)
    lam = np.exp(-0.2 * np.arange(d))
    x = (cent[assign] + g.standard_normal((n, d)) * np.sqrt(lam)).astype(np.float32)
    qs = (cent[g.integers(0, 4, size=5)] + g.standard_normal((5, d)) * np.sqrt(lam)).astype(np.float32)
    mu, t = np.zeros(d), np.eye(d)
    yc = pq.shaped_query(cent, mu, t)
    resid = pq.shaped_query(x, mu, t) - yc[assign]
    cb = (g.standard_normal((M, 256, dsub)) * np.sqrt(lam.reshape(M, dsub))[:, None, :]).astype(np.float32)
    codes = pq.encode(resid, cb)
    sub_cuts = [0, 2, 4, 6, 8]
    ri, rd = pq.pq_knn_ivf(qs, mu, t, cb, codes, cent, assign, 2, 10)
    gi, gd, frac = pq.panorama_pq_knn_ivf(qs, mu, t, cb, codes, cent, assign, 2, 10, sub_cuts, batch=32)
    assert np.array_equal(gi, ri) and np.array_equal(gd, rd)
    assert frac.mean() < 1.0
    # the bound on every candidate of every list
    xt = pq.tails(pq.reconstruct(codes, cb), [c * dsub for c in sub_cuts])
    y = pq.shaped_query(qs, mu, t)
    for qi in range(qs.shape[0]):
        for l in range(4):
            mm = np.nonzero(assign == l)[0]
            z = y[qi] - yc[l]
            tab = pq.lut(z, cb)
            full = pq.adc(tab, codes[mm]).astype(np.float64)
            zt = pq.tails(z[None, :], [c * dsub for c in sub_cuts])[0]
            p = np.zeros(mm.size)
            for lv in range(1, 5):
                for m in range(sub_cuts[lv - 1], sub_cuts[lv]):
                    p += tab[m, codes[mm, m]].astype(np.float64)
                assert (pq.pq_lower_bound(p, zt[lv], xt[mm, lv], 1.0) <= full * (1 + 1e-6) + 1e-9).all()
