"""ctypes front end of the plain C oracle (oracle/c/pano_oracle.c).

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline leg).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "c", "pano_oracle.c")
LIB = os.path.join(HERE, "c", "libpano_oracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        _lib.orc_canonical_dist.restype = C.c_float
        _lib.orc_canonical_dist.argtypes = [P, P, i32]
        _lib.orc_max_threads.restype = i32
        _lib.orc_probe.argtypes = [P, i64, P, i32, i32, P, i32, P, i32]
        _lib.orc_knn_lists.argtypes = [P, i64, P, i32, P, P, i32, P, P, i32]
        _lib.orc_transform.argtypes = [P, P, P, i64, i32, P, i32]
        _lib.orc_tails.argtypes = [P, i64, i32, P, i32, P, i32]
        _lib.orc_panorama.argtypes = [P, i64, P, P, P, i32, P, P, P, i32, P, P, i32, i32, dbl,
                                      P, P, P, i32]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def max_threads() -> int:
    return int(lib().orc_max_threads())


def probe(qs, centroids, nprobe, threads=0):
    qs = _c(np.atleast_2d(qs), np.float32)
    cent = _c(centroids, np.float32)
    npv = _c(np.broadcast_to(np.asarray(nprobe), (qs.shape[0],)), np.int32)
    maxp = int(min(max(int(npv.max()), 1), cent.shape[0]))
    out = np.empty((qs.shape[0], maxp), dtype=np.int32)
    lib().orc_probe(_p(qs), qs.shape[0], _p(cent), cent.shape[0], qs.shape[1], _p(npv), maxp,
                    _p(out), threads)
    return [row[row >= 0].astype(np.int64) for row in out]


def list_members(assign, nlist):
    assign = np.asarray(assign)
    order = np.argsort(assign, kind="stable").astype(np.int64)
    bounds = np.searchsorted(assign[order], np.arange(nlist + 1))
    return [order[bounds[l]:bounds[l + 1]] for l in range(nlist)]


def candidates_csr(probes, members):
    parts = [np.concatenate([members[int(l)] for l in pr]) if len(pr) else np.empty(0, np.int64)
             for pr in probes]
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    off[1:] = np.cumsum([p.size for p in parts])
    ids = np.concatenate(parts) if parts else np.empty(0, np.int64)
    return off, _c(ids, np.int64)


def knn_lists(qs, xs, off, cand, k, threads=0):
    qs = _c(np.atleast_2d(qs), np.float32)
    xs = _c(xs, np.float32)
    ids = np.empty((qs.shape[0], k), dtype=np.int64)
    dd = np.empty((qs.shape[0], k), dtype=np.float32)
    lib().orc_knn_lists(_p(qs), qs.shape[0], _p(xs), xs.shape[1], _p(_c(off, np.int64)),
                        _p(_c(cand, np.int64)), k, _p(ids), _p(dd), threads)
    return ids, dd


def prepare(xs, mu, t, m, threads=0):
    """Build-time part of the CPU scan: FP64 transformed rows and tails."""
    xs = _c(xs, np.float32)
    n, d = xs.shape
    ys = np.empty((n, d), dtype=np.float64)
    lib().orc_transform(_p(_c(mu, np.float64)), _p(_c(t, np.float64)), _p(xs), n, d, _p(ys), threads)
    m32 = _c(m, np.int32)
    L = m32.size - 1
    R = np.empty((n, L + 1), dtype=np.float64)
    lib().orc_tails(_p(ys), n, d, _p(m32), L, _p(R), threads)
    return ys, R


def panorama(qs, xs, ys, R, mu, t, m, off, cand, k, batch=1024, eps=1.0, threads=0):
    qs = _c(np.atleast_2d(qs), np.float32)
    xs = _c(xs, np.float32)
    m32 = _c(m, np.int32)
    L = m32.size - 1
    nq, d = qs.shape
    ids = np.empty((nq, k), dtype=np.int64)
    dd = np.empty((nq, k), dtype=np.float32)
    dims = np.empty(nq, dtype=np.int64)
    lib().orc_panorama(_p(qs), nq, _p(xs), _p(_c(ys, np.float64)), _p(_c(R, np.float64)), d,
                       _p(_c(mu, np.float64)), _p(_c(t, np.float64)), _p(m32), L,
                       _p(_c(off, np.int64)), _p(_c(cand, np.int64)), k, batch, float(eps),
                       _p(ids), _p(dd), _p(dims), threads)
    return ids, dd, dims
