"""Python front end over the C ABI.  PyTorch only supplies device memory and
the current HIP stream; all computation happens in libpanorama.so."""
from __future__ import annotations

import ctypes as C
import weakref
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        L.check(L.lib().pano_ctx_create(device, C.byref(h)))
        self.h = h
        self.device = device
        self._indexes = weakref.WeakSet()

    def scratch_bytes(self) -> int:
        """Device memory the context keeps for search scratch."""
        out = C.c_int64()
        L.check(L.lib().pano_ctx_scratch_bytes(self.h, C.byref(out)))
        return out.value

    def status(self) -> int:
        """Wait for the device; raise if asynchronous searches met non-finite
        queries since the last call (their count is in the error)."""
        out = C.c_int64()
        st = L.lib().pano_ctx_status(self.h, C.byref(out))
        if st != L.PANO_OK:
            raise L.PanoError(st, L.lib().pano_last_error().decode(errors="replace") + f" ({out.value})")
        return out.value

    def trim(self):
        """Release the context's search scratch (no search may be running on it)."""
        L.check(L.lib().pano_ctx_trim(self.h))

    def close(self):
        """Destroy the context; indexes built on it are freed first."""
        if self.h:
            for ix in list(self._indexes):
                ix.free()
            L.lib().pano_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Transform:
    def __init__(self, h, d):
        self.h = h
        self.d = d

    @classmethod
    def fit(cls, x: np.ndarray, fit_sample: int = 0, seed: int = 0) -> "Transform":
        x = np.ascontiguousarray(x, dtype=np.float32)
        h = C.c_void_p()
        L.check(L.lib().pano_build_transform(_np_ptr(x), x.shape[0], x.shape[1], int(fit_sample), int(seed),
                                             C.byref(h)))
        return cls(h, x.shape[1])

    @classmethod
    def identity(cls, d: int) -> "Transform":
        h = C.c_void_p()
        L.check(L.lib().pano_transform_identity(d, C.byref(h)))
        return cls(h, d)

    @classmethod
    def from_matrix(cls, mu: np.ndarray, t: np.ndarray) -> "Transform":
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        t = np.ascontiguousarray(t, dtype=np.float64)
        h = C.c_void_p()
        L.check(L.lib().pano_transform_from(mu.shape[0], _np_ptr(mu), _np_ptr(t), C.byref(h)))
        return cls(h, mu.shape[0])

    def shape(self, m, kappa: float, isotropize: bool = True, seed: int = 0) -> "Transform":
        """The shaped transform U R T of Section 4.2 for level cuts m."""
        m = np.ascontiguousarray(m, dtype=np.int32)
        h = C.c_void_p()
        L.check(L.lib().pano_transform_shape(self.h, _np_ptr(m), m.size - 1, float(kappa), 1 if isotropize else 0,
                                             int(seed), C.byref(h)))
        return Transform(h, self.d)

    def get(self):
        d = self.d
        mu = np.empty(d)
        t = np.empty((d, d))
        lam = np.empty(d)
        alpha = C.c_double()
        dd = C.c_int32()
        L.check(L.lib().pano_transform_get(self.h, C.byref(dd), _np_ptr(mu), _np_ptr(t), _np_ptr(lam),
                                           C.byref(alpha)))
        return mu, t, lam, alpha.value

    def __del__(self):
        try:
            if self.h:
                L.lib().pano_transform_free(self.h)
                self.h = None
        except Exception:
            pass


def shape_plan(lam, m, kappa: float):
    """Procedure 1's plan: list of (start, length) coordinate blocks."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.int32)
    cap = int(m.size) + 1
    out = np.zeros(2 * cap, dtype=np.int32)
    nb = C.c_int32()
    L.check(L.lib().pano_shape_plan(_np_ptr(lam), lam.size, _np_ptr(m), m.size - 1, float(kappa), _np_ptr(out), cap,
                                    C.byref(nb)))
    return [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(nb.value)]


class PQIndex:
    """IVFPQ index over the shaped frame (Section 6.2): codes, codebooks and
    the sub-quantizer-major block layout live in device memory."""

    def __init__(self, h, ctx, n, d, m, dsub):
        self.h = h
        self.ctx = ctx
        self.n = n
        self.d = d
        self.m = np.asarray(m, dtype=np.int32)
        self.dsub = dsub
        self.M = d // dsub

    @classmethod
    def build(cls, ctx: Context, tf: Transform, x_dev, centroids_dev, assign_dev, m, dsub: int, iters: int = 10,
              sample: int = 65536, seed: int = 0, stream=None) -> "PQIndex":
        m = np.ascontiguousarray(m, dtype=np.int32)
        n, d = x_dev.shape
        h = C.c_void_p()
        L.check(L.lib().pano_pq_build(ctx.h, tf.h, _ptr(x_dev), n, d, _ptr(centroids_dev), _ptr(assign_dev),
                                      centroids_dev.shape[0], _np_ptr(m), m.size - 1, int(dsub), int(iters),
                                      int(sample), int(seed), C.byref(h), _stream_handle(stream)))
        return cls(h, ctx, n, d, m, dsub)

    def search(self, q_dev, k: int, nprobe=1, eps: float = 1.0, brute: bool = False, stats: bool = False,
               stream=None, nprobe_max: int = 0, out=None):
        import torch
        nq = q_dev.shape[0]
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=q_dev.device)
            dists = torch.empty((nq, k), dtype=torch.float32, device=q_dev.device)
        else:
            ids, dists = out
        np_dev, np_all = _probe_args(nprobe, nprobe_max)
        flags = (L.PANO_PQ_BRUTE if brute else 0) | (L.PANO_SEARCH_STATS if stats else 0)
        L.check(L.lib().pano_pq_search(self.ctx.h, self.h, _ptr(q_dev), nq, k, _ptr(np_dev), np_all, float(eps),
                                       _ptr(ids), _ptr(dists), flags, _stream_handle(stream)))
        return ids, dists

    def stats(self) -> dict:
        out = np.zeros(5, dtype=np.int64)
        ms = C.c_double()
        L.check(L.lib().pano_pq_stats(self.h, _np_ptr(out), C.byref(ms)))
        return {"lookups": int(out[0]), "lookups_full": int(out[1]), "fallback_queries": int(out[2]),
                "candidates": int(out[3]), "scan_bytes": int(out[4]), "ms_scan": ms.value,
                "phi": float(out[0]) / max(1, int(out[1]))}

    def export(self):
        """(codebooks [M, 256, dsub] float32, codes [n, M] uint8)."""
        cb = np.empty((self.M, 256, self.dsub), dtype=np.float32)
        codes = np.empty((self.n, self.M), dtype=np.uint8)
        L.check(L.lib().pano_pq_export(self.h, _np_ptr(cb), _np_ptr(codes), None, None))
        return cb, codes

    def free(self):
        if self.h:
            L.lib().pano_pq_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def ivf_assign(ctx: Context, x_dev, nlist: int, iters: int = 10, seed: int = 0, stream=None):
    import torch
    n, d = x_dev.shape
    cent = torch.empty((nlist, d), dtype=torch.float32, device=x_dev.device)
    assign = torch.empty((n,), dtype=torch.int32, device=x_dev.device)
    L.check(L.lib().pano_ivf_assign(ctx.h, _ptr(x_dev), n, d, nlist, iters, seed, _ptr(cent), _ptr(assign),
                                    _stream_handle(stream)))
    return cent, assign


@dataclass
class Params:
    group: int = 0
    blocks_per_item: int = 0
    seed_pool: int = 0
    seed_count: int = 0
    grid: int = 0
    use_bf16: int = 0
    dense_min: int = 0
    scan_mode: int = 0  # 0/1 workgroup scan, 3 no pruning (brute-force scan), 4 per-wave scan
    walk_lanes: int = 0  # lanes per pair in the per-pair walk: 1, 2, 4 (0 = by the number of pairs)
    walk_step: int = 0  # levels per step of the four-lane walk: 1 or 2 (0 = 2 when levels are <= 64 wide)
    arrival_order: int = 0  # 1: keep each list's queries in arrival order (0 = ordered by distance to the list)

    def c(self):
        p = L.SearchParams()
        p.group, p.blocks_per_item, p.seed_pool = self.group, self.blocks_per_item, self.seed_pool
        p.seed_count, p.grid, p.use_bf16 = self.seed_count, self.grid, self.use_bf16
        p.reserved[0] = self.dense_min
        p.reserved[1] = self.scan_mode
        p.reserved[2] = self.walk_lanes
        p.reserved[3] = self.walk_step
        p.reserved[4] = self.arrival_order
        return p


def _probe_args(nprobe, nprobe_max: int):
    """(per-query count tensor or None, nprobe_all) of the C ABI."""
    import torch
    if isinstance(nprobe, torch.Tensor):
        return nprobe, int(nprobe_max)
    return None, int(nprobe)


class Index:
    def __init__(self, h, ctx: Context, d: int):
        self.h = h
        self.ctx = ctx
        self.d = d
        ctx._indexes.add(self)

    @classmethod
    def build(cls, ctx: Context, tf: Transform, x_dev, centroids_dev, assign_dev, m, block: int = 256,
              store: str = "f32", stream=None) -> "Index":
        m = np.ascontiguousarray(m, dtype=np.int32)
        n, d = x_dev.shape
        h = C.c_void_p()
        L.check(L.lib().pano_build_levels(ctx.h, tf.h, _ptr(x_dev), n, d, _ptr(centroids_dev), _ptr(assign_dev),
                                          centroids_dev.shape[0], _np_ptr(m), m.size - 1, block,
                                          L.PANO_BF16 if store == "bf16" else L.PANO_F32, C.byref(h),
                                          _stream_handle(stream)))
        return cls(h, ctx, d)

    def _outs(self, q_dev, k):
        import torch
        nq = q_dev.shape[0]
        ids = torch.empty((nq, k), dtype=torch.int64, device=q_dev.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=q_dev.device)
        return ids, dists

    def search(self, q_dev, k: int, nprobe=1, eps: float = 1.0, params: Params | None = None,
               stats: bool = False, stream=None, out=None, eager: bool = False, ctx: Context | None = None,
               timing: bool = False, nprobe_max: int = 0, asynchronous: bool = False):
        """k-NN of each row of q_dev among its probed lists.  nprobe: an int,
        or a device tensor of per-query counts (bounded by nprobe_max when
        positive).  ctx: run on this context (one per concurrent caller)
        instead of the index's own.  timing: phase durations of an ordinary
        (uncounted) search in stats().  asynchronous: return without waiting
        (results complete in stream order; see Context.status)."""
        import torch
        ids, dists = out if out is not None else self._outs(q_dev, k)
        np_dev, np_all = _probe_args(nprobe, nprobe_max)
        prm = params.c() if params is not None else None
        flags = ((L.PANO_SEARCH_STATS if stats else 0) | (L.PANO_SEARCH_EAGER if eager else 0) |
                 (L.PANO_SEARCH_TIMING if timing else 0) | (L.PANO_SEARCH_ASYNC if asynchronous else 0))
        c = ctx if ctx is not None else self.ctx
        L.check(L.lib().pano_search_ctx(c.h, self.h, _ptr(q_dev), q_dev.shape[0], k, _ptr(np_dev), np_all,
                                        float(eps), _ptr(ids), _ptr(dists),
                                        C.byref(prm) if prm is not None else None, flags, _stream_handle(stream)))
        return ids, dists

    def refine(self, q_dev, k: int, cand_dev, eps: float = 1.0, stream=None, out=None):
        """k-NN of each query among its own candidate ids cand_dev [nq][k']
        (int64, -1 = empty), by the point-centric scan."""
        ids, dists = out if out is not None else self._outs(q_dev, k)
        L.check(L.lib().pano_refine(self.h, _ptr(q_dev), q_dev.shape[0], k, _ptr(cand_dev), cand_dev.shape[1],
                                    float(eps), _ptr(ids), _ptr(dists), _stream_handle(stream)))
        return ids, dists

    def audit_bounds(self, q_dev, pair_q, pair_row, bf16: bool = False, rows: bool = True, stream=None):
        """Per-level certified bounds of (query, row) pairs as the GPU computes
        them: a tensor [npairs][L][4] (lower, upper with the head from
        coordinate differences; lower, upper in the dot-product form), and,
        with rows, the transformed query and stored row of each pair
        [npairs][2][d_pad]."""
        import torch
        pq = torch.as_tensor(pair_q, dtype=torch.int32, device=q_dev.device).contiguous()
        pr = torch.as_tensor(pair_row, dtype=torch.int64, device=q_dev.device).contiguous()
        inf = self.info()
        out = torch.empty((pq.shape[0], inf["L"], 4), dtype=torch.float32, device=q_dev.device)
        rw = torch.empty((pq.shape[0], 2, inf["d_pad"]), dtype=torch.float32, device=q_dev.device) if rows else None
        L.check(L.lib().pano_audit_bounds(self.h, _ptr(q_dev), q_dev.shape[0], _ptr(pq), _ptr(pr), pq.shape[0],
                                          1 if bf16 else 0, _ptr(out), _ptr(rw) if rows else None,
                                          _stream_handle(stream)))
        return out, rw

    def search_noalloc(self, q_dev, k: int, nprobe=1, eps: float = 1.0, params: Params | None = None,
                       stream=None, out=None, nprobe_max: int = 0):
        """The same search with no allocation inside the library: its scratch
        is the library's fixed per-GPU array (calls on one GPU must not
        overlap).  out: caller-allocated (ids, dists)."""
        ids, dists = out if out is not None else self._outs(q_dev, k)
        np_dev, np_all = _probe_args(nprobe, nprobe_max)
        prm = params.c() if params is not None else None
        L.check(L.lib().pano_search_noalloc(self.h, _ptr(q_dev), q_dev.shape[0], k, _ptr(np_dev), np_all,
                                            float(eps), _ptr(ids), _ptr(dists),
                                            C.byref(prm) if prm is not None else None, _stream_handle(stream)))
        return ids, dists

    def scratch_bytes(self, nq: int, k: int, nprobe=1, per_query_nprobe: bool = False,
                      params: Params | None = None) -> int:
        """Device scratch a search of nq queries needs on its context.  With
        per_query_nprobe, nprobe is the largest per-query count (0: nlist)."""
        out = C.c_int64()
        prm = params.c() if params is not None else None
        L.check(L.lib().pano_search_scratch_bytes(self.h, int(nq), int(k), 1 if per_query_nprobe else 0,
                                                  int(nprobe), C.byref(prm) if prm is not None else None,
                                                  C.byref(out)))
        return out.value

    def search_bruteforce(self, q_dev, k: int, nprobe=1, params: Params | None = None, stats: bool = False,
                          stream=None, out=None, eager: bool = False, nprobe_max: int = 0, timing: bool = False):
        """The same probe lists scanned without bounds (every level of every
        candidate).  timing: phase durations in stats(), as for search."""
        ids, dists = out if out is not None else self._outs(q_dev, k)
        np_dev, np_all = _probe_args(nprobe, nprobe_max)
        prm = params.c() if params is not None else None
        flags = (L.PANO_SEARCH_STATS if stats else 0) | (L.PANO_SEARCH_EAGER if eager else 0)
        flags |= L.PANO_SEARCH_TIMING if timing else 0
        L.check(L.lib().pano_search_bruteforce(self.h, _ptr(q_dev), q_dev.shape[0], k, _ptr(np_dev), np_all,
                                               _ptr(ids), _ptr(dists), C.byref(prm) if prm is not None else None,
                                               flags, _stream_handle(stream)))
        return ids, dists

    def info(self) -> dict:
        inf = L.IndexInfo()
        L.check(L.lib().pano_index_info(self.h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def layout(self):
        inf = self.info()
        m = np.empty(inf["L"] + 1, dtype=np.int32)
        ll = np.empty(inf["nlist"], dtype=np.int64)
        L.check(L.lib().pano_index_layout(self.h, _np_ptr(m), _np_ptr(ll)))
        return m, ll

    def stats(self) -> dict:
        st = L.Stats()
        L.check(L.lib().pano_stats_get(self.h, C.byref(st)))
        out = {f: getattr(st, f) for f, _ in st._fields_ if f not in ("level_reads", "scan_cycles")}
        out["level_reads"] = list(st.level_reads)
        out["scan_cycles"] = list(st.scan_cycles)
        return out

    def free(self):
        if self.h:
            L.lib().pano_index_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
