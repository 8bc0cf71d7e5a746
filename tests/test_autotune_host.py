"""The tuner, on the CPU: every entry of the committed cache lies in the
search space the tuner explores (so it was written by the tuner, not by
hand) and each of the four workloads finds its entry under the signature
the benchmark looks up; with a stand-in index and clock, the coordinate
descent reaches the optimum of a separable cost, the width tuner keeps the
fastest width and frees every trial index, and the cache round-trips."""
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


class _FakeIndex:
    """Stand-in for an index: search() records the knobs it was called with;
    the fake clock prices them with a separable cost."""

    def __init__(self, width=0):
        self.width = width
        self.last = None
        self.freed = False

    def search(self, q, k, nprobe=1, params=None, nprobe_max=0):
        self.last = params

    def free(self):
        self.freed = True


_BEST = {"scan_mode": 4, "blocks_per_item": 4, "group": 16, "seed": (1024, 64), "dense_min": 256,
         "arrival_order": 1}


def _cost(p, width=0):
    c = 10.0 + abs(width - 16) * 0.5
    c += 0.0 if p.scan_mode == _BEST["scan_mode"] else 3.0
    c += abs(p.blocks_per_item - _BEST["blocks_per_item"]) * 0.3
    c += 0.0 if p.group == _BEST["group"] else 1.0
    c += 0.0 if (p.seed_pool, p.seed_count) == _BEST["seed"] else 0.7
    c += 0.0 if p.dense_min == _BEST["dense_min"] else 0.2
    c += 0.0 if p.arrival_order == _BEST["arrival_order"] else 0.1
    return c


def _fake_clock(idxs):
    def timer(fn, reps):
        fn()
        ix = next(i for i in idxs if i.last is not None)
        t = _cost(ix.last, ix.width)
        ix.last = None
        return t
    return timer


def test_coordinate_descent_finds_a_separable_optimum(monkeypatch):
    idx = _FakeIndex(width=16)
    monkeypatch.setattr(autotune, "_time", _fake_clock([idx]))
    best, t = autotune.tune_search(idx, None, 10, 8, use_bf16=1)
    got = {"scan_mode": best.scan_mode, "blocks_per_item": best.blocks_per_item, "group": best.group,
           "seed": (best.seed_pool, best.seed_count), "dense_min": best.dense_min,
           "arrival_order": best.arrival_order}
    assert got == _BEST and best.use_bf16 == 1
    assert t == pytest.approx(10.0)


def test_level_width_tuner_keeps_the_fastest_width(monkeypatch):
    built = []

    def build(width):
        built.append(_FakeIndex(width))
        return built[-1]

    monkeypatch.setattr(autotune, "_time", _fake_clock(built))
    w, prm, results = autotune.tune_level_width(build, None, 10, 8, widths=(8, 16, 32))
    assert w == 16 and sorted(results) == [8, 16, 32]
    assert all(ix.freed for ix in built)  # every trial index is released
    assert prm.scan_mode == _BEST["scan_mode"]


def test_cache_round_trip_and_signature_buckets(tmp_path):
    path = str(tmp_path / "cache.json")
    p = autotune.Params(group=8, blocks_per_item=2, seed_pool=256, seed_count=32, scan_mode=3)
    sig = autotune.signature("gfx950", 128, "f32", 10_000_000, [3, 100, 7], 10)
    # rows round up to a power of 4, probes (the largest requested) to a power of 2
    assert sig == "gfx950|d128|f32|N16777216|np128|k10"
    assert autotune.signature("gfx950", 128, "f32", 16_777_216, 128, 10) == sig
    assert autotune.lookup(sig, path) == (None, None)
    autotune.store(sig, p, 32, 0.0125, path)
    got, width = autotune.lookup(sig, path)
    assert got == p and width == 32
    assert autotune.load_cache(path)[sig]["ms"] == pytest.approx(12.5)
