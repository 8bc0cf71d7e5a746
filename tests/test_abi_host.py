"""CPU-side checks of the C ABI library: it loads, exports every entry point
declared in include/panorama.h, and its host-only FP64 PCA fit (Section 4.1)
is correct.  No GPU call is made here."""
import os
import re

import numpy as np
import pytest

from paper_2510_00566_amd import _lib as L
from paper_2510_00566_amd import synth
from paper_2510_00566_amd.index import Transform

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "panorama.h")).read()
    return sorted(set(re.findall(r"\b(pano_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2510_00566_amd import build
        build.build()
    return L.lib()


def test_every_declared_symbol_is_exported(lib):
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(L.exported_symbols())


def test_invalid_arguments_are_rejected_without_gpu(lib):
    import ctypes as C
    h = C.c_void_p()
    assert lib.pano_transform_identity(0, C.byref(h)) == L.PANO_EINVAL
    assert b"bad" in lib.pano_last_error()
    x = np.zeros((1, 3), np.float32)
    st = lib.pano_build_transform(x.ctypes.data_as(C.c_void_p), 1, 3, 0, 0, C.byref(h))
    assert st == L.PANO_EINVAL
    x = np.ones((4, 3), np.float32)
    x[2, 1] = np.nan
    st = lib.pano_build_transform(x.ctypes.data_as(C.c_void_p), 4, 3, 0, 0, C.byref(h))
    assert st == L.PANO_EINVAL and b"non-finite" in lib.pano_last_error()


@pytest.mark.parametrize("d,n", [(5, 400), (33, 3000), (128, 20000)])
def test_pca_fit_matches_numpy(lib, d, n):
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=n, nq=1)
    w.d = d
    x = synth.generate(w, with_queries=False)["x"]
    tf = Transform.fit(x, fit_sample=0, seed=1)
    mu, t, lam, alpha = tf.get()
    x64 = x.astype(np.float64)
    mu_ref = x64.mean(axis=0)
    cov = (x64 - mu_ref).T @ (x64 - mu_ref) / n
    lam_ref = np.linalg.eigvalsh(cov)[::-1]
    assert np.allclose(mu, mu_ref, atol=1e-12)
    assert np.abs(t @ t.T - np.eye(d)).max() < 1e-11
    assert np.allclose(lam, lam_ref, rtol=1e-9, atol=1e-12 * lam_ref[0])
    assert np.all(np.diff(lam) <= 1e-14 * lam[0])
    # rows are eigenvectors: T cov T^t is diagonal with lambda on it
    dd = t @ cov @ t.T
    assert np.abs(dd - np.diag(lam)).max() < 1e-9 * lam[0]
    piv = np.abs(t).argmax(axis=1)
    assert np.all(t[np.arange(d), piv] > 0)
    # Ky Fan: tail energy of the transformed fit data = trailing eigen-sum
    y = (x64 - mu) @ t.T
    for m in (0, d // 3, d - 1):
        assert abs((y[:, m:] ** 2).sum(axis=1).mean() - lam[m:].sum()) < 1e-9 * lam.sum()


def test_pca_fit_sample_is_seeded(lib):
    x = synth.uniform_cube(5000, 16, 3)
    a = Transform.fit(x, fit_sample=1000, seed=7).get()
    b = Transform.fit(x, fit_sample=1000, seed=7).get()
    c = Transform.fit(x, fit_sample=1000, seed=8).get()
    assert np.array_equal(a[1], b[1]) and not np.array_equal(a[0], c[0])


def test_transform_from_rejects_non_orthonormal(lib):
    with pytest.raises(L.PanoError):
        Transform.from_matrix(np.zeros(3), np.ones((3, 3)))
    tf = Transform.from_matrix(np.zeros(2), np.array([[0.6, 0.8], [-0.8, 0.6]]))
    assert np.allclose(tf.get()[1], [[0.6, 0.8], [-0.8, 0.6]])


def test_build_levels_rejects_bad_geometry_without_gpu(lib):
    """Block sizes outside {0, 64, 128, 256}, a first level wider than 64
    dimensions and padded widths summing past 4096 are rejected before any
    handle is used."""
    import ctypes as C
    h = C.c_void_p()

    def build(block, m):
        m = np.ascontiguousarray(m, dtype=np.int32)
        return lib.pano_build_levels(None, None, None, 10, int(m[-1]), None, None, 1,
                                     m.ctypes.data_as(C.c_void_p), m.size - 1, block, L.PANO_F32, C.byref(h), None)

    assert build(512, [0, 8, 16]) == L.PANO_EINVAL and b"block" in lib.pano_last_error()
    assert build(96, [0, 8, 16]) == L.PANO_EINVAL
    assert build(256, [0, 68, 80]) == L.PANO_EINVAL and b"first level" in lib.pano_last_error()
    assert build(256, [0, 64, 4097]) == L.PANO_EINVAL and b"4096" in lib.pano_last_error()
    assert build(256, [0, 8, 8]) == L.PANO_EINVAL and b"increase" in lib.pano_last_error()
    # a valid geometry gets as far as the null handles
    assert build(0, [0, 8, 16]) == L.PANO_EINVAL and b"null" in lib.pano_last_error()
    assert build(128, [0, 64, 4096]) == L.PANO_EINVAL and b"null" in lib.pano_last_error()


def test_ctx_calls_reject_null_without_gpu(lib):
    import ctypes as C
    out = C.c_int64()
    assert lib.pano_ctx_scratch_bytes(None, C.byref(out)) == L.PANO_EINVAL
    assert lib.pano_ctx_trim(None) == L.PANO_EINVAL
