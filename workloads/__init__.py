"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Nothing in this package computes PageRank or any step of the update method:
it only draws graphs and edge batches.  The heavy draws (R-MAT, duplicate
removal, the temporal stream) run in ``gen.c`` through ctypes; batch sampling
uses numpy's PCG64 with an explicit seed.

Shapes follow the paper's workloads: R-MAT graphs with a self-loop added on
every vertex downstream (Sections 5.1.3 and 5.2.2), uniform 80/20
insert/delete batches sized as a fraction of |E| (Section 5.2.2), and a
preferential-attachment temporal stream replayed in insertion-only batches
standing in for the SNAP temporal graphs of Table 1 (Sections 5.1.3-5.1.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lock = threading.Lock()
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = False) -> str:
    """Compile gen.c into libgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            lib.gen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_uint64, P, P, P]
            lib.gen_rmat.restype = None
            lib.gen_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, P]
            lib.gen_permutation.restype = None
            lib.gen_dedupe.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P]
            lib.gen_dedupe.restype = ctypes.c_int64
            lib.gen_temporal.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_uint64, P, P, P]
            lib.gen_temporal.restype = ctypes.c_int64
            _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    perm = np.empty(n, dtype=np.int32)
    lib.gen_permutation(n, seed, _ptr(perm))
    return perm


def rmat_raw(scale: int, n_draws: int, seed: int, n_limit: int | None = None, permute: bool = True,
             abc=RMAT_ABC):
    """Raw R-MAT draws (duplicates and self-draws included), relabelled when permute."""
    lib = _load()
    n = (1 << scale) if n_limit is None else int(n_limit)
    perm = permutation(n, seed ^ 0x5EED) if permute else None
    src = np.empty(n_draws, dtype=np.int32)
    dst = np.empty(n_draws, dtype=np.int32)
    a, b, c = abc
    lib.gen_rmat(scale, n_draws, n, a, b, c, seed, _ptr(perm), _ptr(src), _ptr(dst))
    return n, src, dst


def dedupe(n: int, src: np.ndarray, dst: np.ndarray):
    """Distinct non-self pairs sorted by (src, dst)."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    os_ = np.empty(max(m, 1), dtype=np.int32)
    od = np.empty(max(m, 1), dtype=np.int32)
    k = lib.gen_dedupe(n, m, _ptr(src), _ptr(dst), _ptr(os_), _ptr(od))
    if k < 0:
        raise MemoryError("gen_dedupe: allocation failed")
    return os_[:k].copy(), od[:k].copy()


def rmat_graph(scale: int, edge_factor: float = 16, seed: int = 1, n_limit: int | None = None,
               permute: bool = True, abc=RMAT_ABC):
    """R-MAT graph: (n, src, dst) with duplicates and self-draws removed.

    Self-loops are NOT included; the library and the oracle add one per vertex.
    """
    n = (1 << scale) if n_limit is None else int(n_limit)
    draws = int(round(edge_factor * n))
    n, src, dst = rmat_raw(scale, draws, seed, n_limit=n, permute=permute, abc=abc)
    s, d = dedupe(n, src, dst)
    return n, s, d


def temporal_stream(n: int, total: int, mean_deg: float = 20.0, p_repeat: float = 0.10, seed: int = 7,
                    permute: bool = True):
    """Preferential-attachment temporal edge stream (time order), as int32 arrays."""
    lib = _load()
    perm = permutation(n, seed ^ 0x7E3A) if permute else None
    src = np.empty(total, dtype=np.int32)
    dst = np.empty(total, dtype=np.int32)
    k = lib.gen_temporal(n, total, mean_deg, p_repeat, seed, _ptr(perm), _ptr(src), _ptr(dst))
    if k < 0:
        raise MemoryError("gen_temporal: allocation failed")
    return src[:k], dst[:k]


def _keys(n: int, src, dst):
    return src.astype(np.int64) * np.int64(n) + dst.astype(np.int64)


def batch_8020(n: int, src: np.ndarray, dst: np.ndarray, frac: float, seed: int,
               insert_share: float = 0.8):
    """One random batch of round(frac * |E|) edges, |E| counting one self-loop per vertex.

    80% are distinct uniform pairs (u != v) not already in the graph; 20% are
    distinct existing non-self-loop edges chosen uniformly.  `src`/`dst` must
    be the duplicate-free edge list sorted by (src, dst) (as rmat_graph gives).
    Returns (del_src, del_dst, ins_src, ins_dst) as int32 arrays.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m_total = src.shape[0] + n
    b = max(1, int(round(frac * m_total)))
    b_ins = int(round(insert_share * b))
    b_del = min(b - b_ins, src.shape[0])
    keys = _keys(n, src, dst)
    # insertions: distinct uniform pairs, u != v, not present
    ins = np.empty(0, dtype=np.int64)
    while ins.shape[0] < b_ins:
        need = b_ins - ins.shape[0]
        u = rng.integers(0, n, size=need + need // 8 + 8, dtype=np.int64)
        v = rng.integers(0, n, size=u.shape[0], dtype=np.int64)
        k = u * n + v
        k = k[u != v]
        if keys.shape[0]:
            pos = np.searchsorted(keys, k)
            pos = np.minimum(pos, keys.shape[0] - 1)
            k = k[keys[pos] != k]
        k = np.concatenate([ins, k])
        _, first = np.unique(k, return_index=True)
        k = k[np.sort(first)]
        ins = k[:b_ins]
        if n < 2:
            break
    # deletions: distinct uniform existing edges
    sel = np.empty(0, dtype=np.int64)
    while sel.shape[0] < b_del:
        need = b_del - sel.shape[0]
        cand = rng.integers(0, src.shape[0], size=need + need // 8 + 8, dtype=np.int64)
        cand = np.concatenate([sel, cand])
        _, first = np.unique(cand, return_index=True)
        sel = cand[np.sort(first)][:b_del]
    ins_src = (ins // n).astype(np.int32)
    ins_dst = (ins % n).astype(np.int32)
    return src[sel].copy(), dst[sel].copy(), ins_src, ins_dst


def random_digraph(n: int, p: float, seed: int):
    """Erdos-Renyi style directed graph for small tests: (src, dst), no self-loops."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mask = rng.random((n, n)) < p
    np.fill_diagonal(mask, False)
    s, d = np.nonzero(mask)
    return s.astype(np.int32), d.astype(np.int32)


def random_edit_batch(n: int, src: np.ndarray, dst: np.ndarray, n_ins: int, n_del: int, seed: int,
                      messy: bool = True):
    """Small adversarial batch for tests: may repeat pairs, include self-loops,
    delete absent edges, insert existing edges and both insert and delete a pair."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ins_s = rng.integers(0, n, size=n_ins).astype(np.int32)
    ins_d = rng.integers(0, n, size=n_ins).astype(np.int32)
    del_s = rng.integers(0, n, size=n_del).astype(np.int32)
    del_d = rng.integers(0, n, size=n_del).astype(np.int32)
    if messy and src.shape[0] and n_del:
        k = min(n_del, src.shape[0])
        pick = rng.integers(0, src.shape[0], size=k)
        half = k // 2 + 1
        del_s[:half] = src[pick[:half]]
        del_d[:half] = dst[pick[:half]]
        if n_ins > 2:
            ins_s[0], ins_d[0] = del_s[0], del_d[0]          # insert + delete of one pair
            ins_s[1], ins_d[1] = ins_s[2], ins_d[2]          # repeated insert
            ins_s[-1] = ins_d[-1]                             # self-loop insert
        if n_del > 2:
            del_s[-1] = del_d[-1]                             # self-loop delete
    return del_s, del_d, ins_s, ins_d
