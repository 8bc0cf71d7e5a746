"""The tuner's stored choices: every entry of the committed cache lies in the
search space the tuner explores (so it was written by the tuner, not by
hand), and each of the four workloads finds its entry under the signature
the benchmark looks up."""
import json

import pytest

from paper_2510_00566_amd import autotune, synth


def _entries():
    with open(autotune.DEFAULT_CACHE) as f:
        return json.load(f)


def test_stored_params_lie_in_the_search_space():
    sp = autotune.SEARCH_SPACE
    for sig, rec in _entries().items():
        p = rec["params"]
        assert p["scan_mode"] in sp["scan_mode"], sig
        assert p["blocks_per_item"] in sp["blocks_per_item"], sig
        assert p["group"] in sp["group"], sig
        assert (p["seed_pool"], p["seed_count"]) in [tuple(s) for s in sp["seed"]], sig
        assert p["dense_min"] in sp["dense_min"], sig
        assert p["arrival_order"] in sp["arrival_order"], sig
        assert rec["ms"] > 0, sig


@pytest.mark.parametrize("name,store", [("flat_sift_like", "f32"), ("ivf_gist_like", "f32"),
                                        ("ivf_zipf_batched", "f32"), ("ivf_embed_bf16", "bf16")])
def test_each_workload_has_an_entry(name, store):
    w = synth.WORKLOADS[name]
    npv = w.nprobe_range[1] if w.nprobe_range else w.nprobe
    prm, width = autotune.lookup(autotune.signature("gfx950", w.d, store, w.n, npv, w.k))
    assert prm is not None
    # a tuned width is one the tuner tries and cuts at most 64 levels
    if w.tune_width:
        assert width in (8, 16, 32) and -(-w.d // width) <= 64
    assert prm.use_bf16 == (1 if store == "bf16" else 0)
