"""The plain C oracle (used to time the CPU baseline) agrees with the numpy
oracle, which is pinned in test_oracle_pins.py."""
import numpy as np

from oracle import brute, panorama
from paper_2510_00566_amd import synth


def _ivf_case(n=5000, d=40, nc=16, nq=6, seed_cfg=2):
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=n, nq=nq, n_clusters=nc)
    w.d = d
    w.level_width = 8
    data = synth.generate(w)
    x, q = data["x"], data["q"]
    cent = np.stack([x[data["labels"] == c].mean(axis=0) for c in range(nc)]).astype(np.float32)
    assign = np.argmin(brute.canonical_dist_many(x, cent), axis=1).astype(np.int32)
    return w, x, q, cent, assign


def test_c_canonical_distance_bit_equal(c_oracle):
    x = synth.uniform_cube(200, 33, 3, -5, 5)
    q = synth.uniform_cube(1, 33, 4, -5, 5)[0]
    ref = brute.canonical_dist(q, x)
    lib = c_oracle.lib()
    import ctypes as C
    for i in range(x.shape[0]):
        v = lib.orc_canonical_dist(q.ctypes.data_as(C.c_void_p), x[i].ctypes.data_as(C.c_void_p), 33)
        assert np.float32(v) == ref[i]


def test_c_probe_and_knn_match_numpy(c_oracle):
    w, x, q, cent, assign = _ivf_case()
    pr_c = c_oracle.probe(q, cent, 5)
    pr_n = brute.probe_lists(q, cent, 5)
    for a, b in zip(pr_c, pr_n):
        assert np.array_equal(a, b)
    mem = c_oracle.list_members(assign, cent.shape[0])
    off, cand = c_oracle.candidates_csr(pr_c, mem)
    ic, dc = c_oracle.knn_lists(q, x, off, cand, 10)
    i_n, d_n, _ = brute.knn_ivf(q, x, cent, assign, 5, 10)
    assert np.array_equal(ic, i_n) and np.array_equal(dc, d_n)


def test_c_panorama_matches_numpy_and_brute(c_oracle):
    w, x, q, cent, assign = _ivf_case()
    mu, t, _ = panorama.pca_fit(x)
    m = w.level_cuts()
    ys, R = c_oracle.prepare(x, mu, t, m)
    assert np.allclose(ys, panorama.apply_transform(mu, t, x), atol=1e-9)
    pr = c_oracle.probe(q, cent, 5)
    mem = c_oracle.list_members(assign, cent.shape[0])
    off, cand = c_oracle.candidates_csr(pr, mem)
    ic, dc, dims = c_oracle.panorama(q, x, ys, R, mu, t, m, off, cand, 10, batch=256)
    i_n, d_n, phi = panorama.panorama_knn_ivf(q, x, cent, assign, 5, mu, t, m, 10, batch=256)
    assert np.array_equal(ic, i_n) and np.array_equal(dc, d_n)
    phi_c = dims / ((off[1:] - off[:-1]) * x.shape[1])
    assert np.allclose(phi_c, phi, rtol=1e-12)
    ib, db = c_oracle.knn_lists(q, x, off, cand, 10)
    assert np.array_equal(ic, ib)
