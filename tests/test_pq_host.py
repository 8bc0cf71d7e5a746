"""The library's host-side shaping (Section 4.2: Procedure 1's plan, Haar
rotations and the shaped transform U R T) against the oracle and the
properties the paper fixes.  CPU only: these entry points never touch the
GPU."""
import math

import numpy as np
import pytest

from oracle import pq


def _lib_or_skip():
    from paper_2510_00566_amd import _lib
    try:
        _lib.lib()
    except RuntimeError as e:
        pytest.skip(str(e))


@pytest.mark.parametrize("kind,p", [("exp", 0.05), ("exp", 0.01), ("power", 1.0), ("power", 0.5)])
@pytest.mark.parametrize("kappa", [1.0, 1.3, 2.0, 8.0])
def test_library_plan_matches_oracle(kind, p, kappa):
    _lib_or_skip()
    from paper_2510_00566_amd import synth
    from paper_2510_00566_amd.index import shape_plan
    for d, cuts in ((128, list(range(0, 129, 16))), (960, list(range(0, 961, 80))), (96, [0, 8, 24, 48, 96])):
        lam = synth.spectrum(kind, d, p)
        assert shape_plan(lam, cuts, kappa) == pq.robin_hood_plan(lam, cuts, kappa)[0]


def test_library_shaped_transform_properties():
    """Orthogonal; with no cap (huge kappa) and no isotropization it is the
    PCA basis itself; isotropization alone mixes rows only within levels and
    keeps each level's energy; the expected variances it reports are the
    plan's, evened out within levels."""
    _lib_or_skip()
    from paper_2510_00566_amd import synth
    from paper_2510_00566_amd.index import Transform
    w = synth.scaled(synth.WORKLOADS["flat_sift_like"], n=4000, nq=1)
    x = synth.generate(w, with_queries=False)["x"]
    tf = Transform.fit(x, seed=1)
    mu, t0, lam, _ = tf.get()
    cuts = np.arange(0, 129, 16)
    same = tf.shape(cuts, 1e9, isotropize=False, seed=3).get()
    assert np.array_equal(same[1], t0)
    iso = tf.shape(cuts, 1e9, isotropize=True, seed=3)
    _, t1, v1, _ = iso.get()
    assert np.abs(t1 @ t1.T - np.eye(128)).max() < 1e-12
    mix = t1 @ t0.T
    off = np.ones((128, 128), bool)
    for l in range(8):
        off[cuts[l]:cuts[l + 1], cuts[l]:cuts[l + 1]] = False
    assert np.abs(mix[off]).max() < 1e-12
    cov = np.diag(lam)
    e_iso = np.diag(mix @ cov @ mix.T)
    for l in range(8):
        assert math.isclose(e_iso[cuts[l]:cuts[l + 1]].sum(), lam[cuts[l]:cuts[l + 1]].sum(), rel_tol=1e-9)
    shaped = tf.shape(cuts, 1.5, isotropize=True, seed=3)
    _, t2, v2, _ = shaped.get()
    assert np.abs(t2 @ t2.T - np.eye(128)).max() < 1e-12
    blocks, v = pq.robin_hood_plan(lam, cuts, 1.5)
    assert len(blocks) >= 1
    ev = np.array([v[cuts[l]:cuts[l + 1]].mean() for l in range(8)]).repeat(16)
    assert np.allclose(v2, ev, rtol=1e-12)
    # a different seed gives a different rotation, the same seed the same
    assert np.array_equal(tf.shape(cuts, 1.5, seed=3).get()[1], t2)
    assert not np.array_equal(tf.shape(cuts, 1.5, seed=4).get()[1], t2)
