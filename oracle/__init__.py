"""Plain FP64 CPU oracle for Static / ND / DF / DF-P PageRank (arXiv 2401.15870).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never does.  The arithmetic lives in
``oracle.c`` (plain C, FP64, no FMA contraction); this module only marshals
numpy arrays through ctypes.

Passages followed:
  * Equation 1 (PageRank with damping alpha, C0 = (1-alpha)/|V|) and the
    self-loop on every vertex (Sections 3.1, 5.1.3, 5.1.4).
  * Batch semantics Delta- = E^{t-1} \\ E^t, Delta+ = E^t \\ E^{t-1} (Section 3.2).
  * Algorithm 1 with Sections 4.1.1-4.1.2: initial marking, expansion when the
    relative change exceeds tau_f, pruning (DF-P) when it is <= tau_p, the
    closed-loop rank of Equation 2 (derived in Appendix A.1), L-inf stop.
  * Static from 1/|V| (Section 3.1); Naive-dynamic from R^{t-1} (Section 3.3.1).
  * Parameters alpha = 0.85, tau = 1e-10, MAX_ITERATIONS = 500 (Section 5.1.2);
    tau_f = tau_p = 1e-6 (Sections 4.2, 4.3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

STATIC, ND, DF, DFP = 0, 1, 2, 3
MODES = {"static": STATIC, "nd": ND, "df": DF, "dfp": DFP}
# frontier measure compared with tau_f / tau_p (Section 4.2)
CRITERIA = {"relative": 0, "absolute": 1, "contrib": 2}

ALPHA, TOL, TOL_F, TOL_P, MAX_ITERS = 0.85, 1e-10, 1e-6, 1e-6, 500

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c with gcc into a shared library."""
    stale = not os.path.exists(out) or any(
        os.path.getmtime(out) < os.path.getmtime(f) for f in (src, _HDR))
    if force or stale:
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-I", _HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def _declare(lib):
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.orc_canonical.argtypes = [i32, i64, P, P, P, P]
    lib.orc_canonical.restype = i64
    lib.orc_csr.argtypes = [i32, i64, P, P, ctypes.c_int, P, P]
    lib.orc_csr.restype = None
    lib.orc_apply.argtypes = [i32, i64, P, P, i64, P, P, i64, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_apply.restype = ctypes.c_int
    lib.orc_rank.argtypes = [i32, i32, P, P, P, P, P, P, i64, P, P, i64, P, P, P,
                             f64, f64, f64, f64, i32, i32, P, P, P, P]
    lib.orc_rank.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it when missing).  `path` loads another
    build of the same source, which the mutation tests use."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            build()
            _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class Graph:
    """A snapshot: canonical edge set (sorted pairs, one self-loop per vertex) + CSRs."""
    n: int
    esrc: np.ndarray
    edst: np.ndarray
    out_off: np.ndarray
    out_idx: np.ndarray
    in_off: np.ndarray
    in_idx: np.ndarray

    @property
    def m(self) -> int:
        return int(self.esrc.shape[0])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.out_off)


def _from_canonical(n, es, ed, lib) -> Graph:
    m = es.shape[0]
    oo = np.empty(n + 1, np.int32); oi = np.empty(max(m, 1), np.int32)
    io = np.empty(n + 1, np.int32); ii = np.empty(max(m, 1), np.int32)
    lib.orc_csr(n, m, _p(es), _p(ed), 0, _p(oo), _p(oi))
    lib.orc_csr(n, m, _p(es), _p(ed), 1, _p(io), _p(ii))
    return Graph(n, es, ed, oo, oi[:m], io, ii[:m])


def graph(n: int, src, dst, lib=None) -> Graph:
    """Canonical graph of an edge list: duplicates dropped, self-loop on every vertex."""
    lib = lib or load()
    src, dst = _i32(src), _i32(dst)
    m = src.shape[0]
    es = np.empty(m + n, np.int32); ed = np.empty(m + n, np.int32)
    k = lib.orc_canonical(n, m, _p(src), _p(dst), _p(es), _p(ed))
    if k == -1:
        raise ValueError("vertex id out of range")
    if k < 0:
        raise MemoryError("oracle allocation failed")
    return _from_canonical(n, es[:k].copy(), ed[:k].copy(), lib)


@dataclass
class Batch:
    """Effective batch: Delta- and Delta+ as sorted pair lists, plus counts."""
    dm_src: np.ndarray
    dm_dst: np.ndarray
    dp_src: np.ndarray
    dp_dst: np.ndarray
    info: dict


def apply(g: Graph, del_src, del_dst, ins_src, ins_dst, lib=None):
    """Apply a batch: returns (G^t, effective Batch)."""
    lib = lib or load()
    ds, dd, is_, id_ = _i32(del_src), _i32(del_dst), _i32(ins_src), _i32(ins_dst)
    nd, ni = ds.shape[0], is_.shape[0]
    cap = g.m + ni
    ns = np.empty(max(cap, 1), np.int32); nds = np.empty(max(cap, 1), np.int32)
    dms = np.empty(max(nd, 1), np.int32); dmd = np.empty(max(nd, 1), np.int32)
    dps = np.empty(max(ni, 1), np.int32); dpd = np.empty(max(ni, 1), np.int32)
    m_new = ctypes.c_int64(0); n_dm = ctypes.c_int64(0); n_dp = ctypes.c_int64(0)
    info = np.zeros(5, np.int64)
    rc = lib.orc_apply(g.n, g.m, _p(g.esrc), _p(g.edst), nd, _p(ds), _p(dd), ni, _p(is_), _p(id_),
                       _p(ns), _p(nds), ctypes.byref(m_new), _p(dms), _p(dmd), ctypes.byref(n_dm),
                       _p(dps), _p(dpd), ctypes.byref(n_dp), _p(info))
    if rc == -1:
        raise ValueError("vertex id out of range")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    k = m_new.value
    g2 = _from_canonical(g.n, ns[:k].copy(), nds[:k].copy(), lib)
    b = Batch(dms[:n_dm.value].copy(), dmd[:n_dm.value].copy(), dps[:n_dp.value].copy(),
              dpd[:n_dp.value].copy(),
              dict(zip(["ins_in", "ins_effective", "del_in", "del_effective", "self_loop_dels_ignored"],
                       info.tolist())))
    return g2, b


@dataclass
class Result:
    ranks: np.ndarray
    iterations: int
    converged: int
    ever_affected: int
    vertex_updates: int
    edges_pulled: int
    last_delta: float
    frontier: np.ndarray


EMPTY = np.zeros(1, np.int32)


def rank(mode, g: Graph, r_prev=None, g_prev: Graph | None = None, batch: Batch | None = None,
         alpha=ALPHA, tol=TOL, tol_f=TOL_F, tol_p=TOL_P, max_iters=MAX_ITERS, criterion="relative",
         lib=None) -> Result:
    """Run Static / ND / DF / DF-P (Algorithm 1) on G^t; DF/DF-P need G^{t-1} and the batch."""
    lib = lib or load()
    mode = MODES.get(mode, mode) if isinstance(mode, str) else int(mode)
    n = g.n
    if mode == STATIC:
        rp = np.zeros(max(n, 1), np.float64)
    else:
        rp = np.ascontiguousarray(r_prev, dtype=np.float64)
        assert rp.shape[0] == n
    if mode in (DF, DFP):
        assert g_prev is not None and batch is not None
        po, pi = g_prev.out_off, g_prev.out_idx
        dms, dmd, dps, dpd = batch.dm_src, batch.dm_dst, batch.dp_src, batch.dp_dst
    else:
        po = pi = None
        dms = dmd = dps = dpd = EMPTY[:0]
    out = np.empty(max(n, 1), np.float64)
    stats = np.zeros(5, np.int64)
    last = ctypes.c_double(0.0)
    frontier = np.zeros(max_iters, np.int32)
    rc = lib.orc_rank(n, mode, _p(po), _p(pi), _p(g.out_off), _p(g.out_idx), _p(g.in_off),
                      _p(g.in_idx), dms.shape[0], _p(dms if dms.size else EMPTY), _p(dmd if dmd.size else EMPTY),
                      dps.shape[0], _p(dps if dps.size else EMPTY), _p(dpd if dpd.size else EMPTY), _p(rp),
                      alpha, tol, tol_f, tol_p, CRITERIA.get(criterion, criterion), max_iters, _p(out),
                      _p(stats), ctypes.byref(last),
                      _p(frontier))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    it = int(stats[0])
    return Result(out[:n].copy(), it, int(stats[1]), int(stats[2]), int(stats[3]), int(stats[4]),
                  last.value, frontier[:it].copy())


def num_threads() -> int:
    return int(load().orc_num_threads())
