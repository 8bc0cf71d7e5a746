"""Project autotuner for the pruned scan.

Search-time knobs (the scan kernel: workgroup or per-wave; blocks per work
item, queries per group, seeding pool and count, the density at which a
level is refined on the matrix cores, the order of each list's queries, and
whether to prune at all: where the bounds prune too little the brute-force
scan of the same candidates is faster and gives the same answer) are swept
by timing real searches on a sample of the workload's queries; the level
width is a build-time knob (it changes the packed layout), tuned by building
one index per candidate width on a subsample of the data.  Results are cached
in a JSON file keyed by (GPU architecture, d, storage dtype, N bucket, nprobe
bucket, k).
"""
from __future__ import annotations

import itertools
import json
import os
import time
from dataclasses import asdict

from .index import Params

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

SEARCH_SPACE = {
    "scan_mode": [0, 4, 3],
    "blocks_per_item": [1, 2, 4, 8],
    "group": [16, 8],
    "seed": [(512, 32), (1024, 64), (256, 32)],
    "dense_min": [64, 256, 1, 1 << 30],
    "arrival_order": [0, 1],
}


def signature(arch: str, d: int, store: str, n: int, nprobe, k: int) -> str:
    nb = 1
    while nb < n:
        nb <<= 2
    npb = 1
    npv = int(nprobe) if not hasattr(nprobe, "__len__") else int(max(nprobe))
    while npb < npv:
        npb <<= 1
    return f"{arch}|d{d}|{store}|N{nb}|np{npb}|k{k}"


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tune_search(idx, q_dev, k: int, nprobe, reps: int = 5, space: dict | None = None, log=None,
                use_bf16: int = 0, nprobe_max: int = 0) -> tuple[Params, float]:
    """Coordinate-wise sweep of the search knobs; returns the best Params and
    its time per search (seconds).  nprobe_max bounds per-query probe counts."""
    space = space or SEARCH_SPACE
    best = Params()
    cur = {"scan_mode": 0, "blocks_per_item": 1, "group": 16, "seed": (512, 32), "dense_min": 64,
           "arrival_order": 0}

    def mk(cfg):
        return Params(group=cfg["group"], blocks_per_item=cfg["blocks_per_item"],
                      seed_pool=cfg["seed"][0], seed_count=cfg["seed"][1], dense_min=cfg["dense_min"],
                      use_bf16=use_bf16, scan_mode=cfg["scan_mode"],
                      arrival_order=cfg["arrival_order"])

    def run(cfg):
        p = mk(cfg)
        if log:
            log(f"[autotune] trying {cfg}")
        return _time(lambda: idx.search(q_dev, k, nprobe=nprobe, params=p, nprobe_max=nprobe_max), reps)

    best_t = run(cur)
    for _ in range(2):  # two passes of coordinate descent
        for key, vals in space.items():
            for v in vals:
                if v == cur[key]:
                    continue
                trial = dict(cur)
                trial[key] = v
                t = run(trial)
                if log:
                    log(f"[autotune] {trial} {t * 1e3:.3f} ms")
                if t < best_t:
                    best_t, cur = t, trial
    best = mk(cur)
    return best, best_t


def tune_level_width(build_index, q_dev, k: int, nprobe, widths=(8, 16, 32), reps: int = 5, log=None,
                     nprobe_max: int = 0, use_bf16: int = 0):
    """Build one index per level width (build_index(width) -> Index) and keep
    the width whose tuned search is fastest."""
    results = {}
    for wdt in widths:
        idx = build_index(wdt)
        p, t = tune_search(idx, q_dev, k, nprobe, reps=reps, log=log, nprobe_max=nprobe_max, use_bf16=use_bf16)
        results[wdt] = (p, t)
        if log:
            log(f"[autotune] width {wdt}: {t * 1e3:.3f} ms with {p}")
        idx.free()
    wbest = min(results, key=lambda w: results[w][1])
    return wbest, results[wbest][0], results


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(sig: str, params: Params, width: int | None, t: float, path: str = DEFAULT_CACHE):
    cache = load_cache(path)
    rec = asdict(params)
    cache[sig] = {"params": rec, "level_width": width, "ms": t * 1e3}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def lookup(sig: str, path: str = DEFAULT_CACHE):
    rec = load_cache(path).get(sig)
    if rec is None:
        return None, None
    return Params(**rec["params"]), rec.get("level_width")
