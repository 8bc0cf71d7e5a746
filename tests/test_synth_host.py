"""The seeded input generators (no method arithmetic): queries drawn alone
equal those of the full draw, and out-of-distribution queries keep the data's
total energy while spreading it over more directions."""
import dataclasses

import numpy as np

from paper_2510_00566_amd import synth


def test_queries_alone_equal_full_draw():
    w = synth.scaled(synth.WORKLOADS["ivf_zipf_batched"], n=5000, nq=7, nlist=16, n_clusters=16)
    a = synth.generate(w)
    b = synth.queries(w)
    for key in ("q", "qlabels", "nprobe"):
        assert np.array_equal(a[key], b[key])


def test_out_of_distribution_queries():
    w = synth.scaled(synth.WORKLOADS["ivf_gist_like"], n=2000, nq=4000, n_clusters=8)
    w = dataclasses.replace(w, d=96)
    lam = synth.spectrum(w.spec_kind, w.d, w.spec_p)
    rot = synth.haar_rotation(w.d, synth.rng(w.cfg_id, synth.STREAM_ROTATION))
    gc = synth.rng(w.cfg_id, synth.STREAM_CENTERS)
    centers = (gc.standard_normal((w.n_clusters, w.d)) * np.sqrt(w.center_var)).astype(np.float32)
    for qp in (None, 0.0):
        wq = dataclasses.replace(w, q_spec_p=qp)
        qd = synth.queries(wq)
        r = qd["q"].astype(np.float64) - centers[qd["qlabels"]]
        # same total energy as the data's law
        assert abs((r * r).sum(1).mean() / lam.sum() - 1.0) < 0.05
        # energy along the data's principal directions (columns of rot)
        y = r @ rot
        share = (y * y).mean(0) / (y * y).mean(0).sum()
        want = lam[:10].sum() / lam.sum() if qp is None else 10 / w.d  # the data's law / flat
        assert abs(share[:10].sum() - want) < 0.01
