"""Dynamic Frontier PageRank (DF / DF-P) on MI355X: Python binding of libdfpr.

Thin marshalling over the C ABI declared in include/dfpr.h: every step of the
update (batch sort and CSR rebuild, marking, pull iterations, expansion and
pruning, the L-inf reduction) runs in the library's HIP kernels.  torch is used
only for device memory (rank vectors, device-resident edge arrays) and streams.

    import paper_2401_15870_amd as dfpr
    g = dfpr.Graph.from_coo(n, src, dst)                 # numpy or torch int32
    info = g.apply_batch(del_src, del_dst, ins_src, ins_dst)
    r, st = g.update_ranks("dfp", r_prev)                 # torch float64 on the GPU
"""
from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from collections.abc import Sequence

import numpy as np

from . import _capi
from ._capi import BatchInfo, Params, Stats

MODES = {"static": _capi.STATIC, "nd": _capi.ND, "df": _capi.DF, "dfp": _capi.DFP}
ERRORS = {_capi.DFPR_EINVAL: "EINVAL", _capi.DFPR_ERANGE: "ERANGE", _capi.DFPR_ENOMEM: "ENOMEM",
          _capi.DFPR_EHIP: "EHIP", _capi.DFPR_ESTATE: "ESTATE"}


class DfprError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def lib():
    return _capi.load()


def _check(rc):
    if rc != _capi.DFPR_OK:
        raise DfprError(rc, lib().dfpr_last_error().decode(errors="replace"))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ids(a):
    """(pointer, count, where, keepalive) for an int32 edge array (numpy/list or torch)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if a.dtype != torch.int32:
                a = a.to(torch.int32)
            a = a.contiguous()
            return ctypes.c_void_p(a.data_ptr()), a.numel(), (_capi.DEVICE if a.is_cuda else _capi.HOST), a
    except ImportError:
        pass
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return ctypes.c_void_p(arr.ctypes.data if arr.size else 0), arr.size, _capi.HOST, arr


# Handles still open when the interpreter starts to exit are destroyed by an
# atexit hook, which runs before interpreter finalisation, while torch (whose
# HIP runtime the library is bound to) is still intact: servers first (they
# own graphs and lane threads), then graphs.  Destructors that Python runs
# later, during finalisation, do nothing: a destroy there could reach a HIP
# runtime that is already being torn down, and the process is ending anyway.
_live_servers: "weakref.WeakSet" = weakref.WeakSet()
_live_graphs: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_all():
    for objs in (_live_servers, _live_graphs):
        for o in list(objs):
            try:
                o.close()
            except Exception:  # noqa: BLE001 - best effort at exit
                pass


def default_params() -> Params:
    p = Params()
    lib().dfpr_params_default(ctypes.byref(p))
    return p


class Graph:
    """A graph held in device memory (canonical in- and out-CSR, self-loop on every vertex)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n
        _live_graphs.add(self)

    @classmethod
    def from_coo(cls, n, src, dst, edge_capacity=0, keep_ids=False, row_slack=0, stream=None):
        """keep_ids: keep the caller's vertex numbering inside the library
        (default: internal numbering by decreasing degree, invisible outside).
        row_slack: free slots after every CSR row (see set_row_slack)."""
        ps, ms, ws, ks = _ids(src)
        pd, md, wd, kd = _ids(dst)
        if ms != md or ws != wd:
            raise ValueError("src and dst must have the same length and location")
        h = ctypes.c_void_p()
        flags = _capi.CREATE_KEEP_IDS if keep_ids else 0
        _check(lib().dfpr_graph_create(int(n), int(ms), ps, pd, ws, int(edge_capacity), flags, _stream_ptr(stream),
                                       ctypes.byref(h)))
        g = cls(h, int(n))
        if row_slack:
            g.set_row_slack(row_slack, stream=stream)
        return g

    def close(self):
        if self._h:
            lib().dfpr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def m(self) -> int:
        n = ctypes.c_int32()
        m = ctypes.c_int64()
        _check(lib().dfpr_graph_size(self._h, ctypes.byref(n), ctypes.byref(m)))
        return int(m.value)

    def export(self, in_csr=False, stream=None):
        """Canonical CSR as numpy arrays (offsets[n+1], indices[m])."""
        off = np.empty(self.n + 1, np.int32)
        idx = np.empty(max(self.m, 1), np.int32)
        _check(lib().dfpr_graph_export(self._h, 1 if in_csr else 0, ctypes.c_void_p(off.ctypes.data),
                                       ctypes.c_void_p(idx.ctypes.data), _capi.HOST, _stream_ptr(stream)))
        return off, idx[: self.m]

    def apply_batch(self, del_src=(), del_dst=(), ins_src=(), ins_dst=(), stream=None) -> dict:
        a, nds, w1, k1 = _ids(del_src)
        b, ndd, w2, k2 = _ids(del_dst)
        c, nis, w3, k3 = _ids(ins_src)
        d, nid, w4, k4 = _ids(ins_dst)
        if nds != ndd or nis != nid:
            raise ValueError("src/dst length mismatch")
        wheres = {w for w, k in ((w1, nds), (w3, nis)) if k}
        if len(wheres) > 1:
            raise ValueError("deletions and insertions must live in the same memory")
        where = wheres.pop() if wheres else _capi.HOST
        info = BatchInfo()
        _check(lib().dfpr_apply_batch(self._h, nds, a, b, nis, c, d, where, _stream_ptr(stream), ctypes.byref(info)))
        return info.as_dict()

    def apply_batch_noalloc(self, del_src=(), del_dst=(), ins_src=(), ins_dst=(), stream=None) -> dict:
        """apply_batch through the allocation-free entry point (at most
        NOALLOC_MAX_PAIRS pairs, within the edge capacity reserved at create)."""
        a, nds, w1, k1 = _ids(del_src)
        b, ndd, w2, k2 = _ids(del_dst)
        c, nis, w3, k3 = _ids(ins_src)
        d, nid, w4, k4 = _ids(ins_dst)
        if nds != ndd or nis != nid:
            raise ValueError("src/dst length mismatch")
        wheres = {w for w, k in ((w1, nds), (w3, nis)) if k}
        if len(wheres) > 1:
            raise ValueError("deletions and insertions must live in the same memory")
        where = wheres.pop() if wheres else _capi.HOST
        info = BatchInfo()
        _check(lib().dfpr_apply_batch_noalloc(self._h, nds, a, b, nis, c, d, where, _stream_ptr(stream),
                                              ctypes.byref(info)))
        return info.as_dict()

    def update_ranks(self, mode, r_prev=None, out=None, stream=None, timing=False, asynchronous=False, **kw):
        """Run Static / ND / DF / DF-P.  r_prev and out are float64 CUDA tensors of n entries.
        asynchronous: DF/DF-P update ranks in place during each iteration (not bit-reproducible)."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        p = default_params()
        for k, v in kw.items():
            setattr(p, k, _capi.CRITERIA.get(v, v) if k == "criterion" else v)
        if timing:
            p.flags |= _capi.FLAG_TIMING
        if asynchronous:
            p.flags |= _capi.FLAG_ASYNC
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        for t in (out, r_prev):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != self.n):
                raise ValueError("rank vectors must be contiguous float64 CUDA tensors of n entries")
        st = Stats()
        rp = ctypes.c_void_p(r_prev.data_ptr()) if r_prev is not None else None
        _check(lib().dfpr_update_ranks(self._h, m, ctypes.byref(p), rp, ctypes.c_void_p(out.data_ptr()),
                                       _stream_ptr(stream), ctypes.byref(st)))
        return out, st.as_dict()

    def set_tuning(self, bounds):
        """In-degree bin limits of the pull kernel (5 non-decreasing ints >= 1)."""
        arr = (ctypes.c_int32 * 5)(*[int(x) for x in bounds])
        _check(lib().dfpr_set_tuning(self._h, arr))

    def get_tuning(self):
        arr = (ctypes.c_int32 * 5)()
        _check(lib().dfpr_get_tuning(self._h, arr))
        return list(arr)

    def autotune(self, stream=None):
        """Time candidate bin thresholds on this graph and install the best; returns (bounds, ms)."""
        arr = (ctypes.c_int32 * 5)()
        ms = ctypes.c_double()
        _check(lib().dfpr_autotune(self._h, _stream_ptr(stream), arr, ctypes.byref(ms)))
        return list(arr), ms.value

    def set_fused_limit(self, max_edges):
        """Edge count up to which a rank update runs in one cooperative launch (0: never)."""
        _check(lib().dfpr_set_fused_limit(self._h, int(max_edges)))

    def set_row_slack(self, slack, stream=None):
        """Lay both CSRs out again with `slack` free slots after every row, so
        that small batches merge into the rows they touch (0: packed rows)."""
        _check(lib().dfpr_set_row_slack(self._h, int(slack), _stream_ptr(stream)))

    def set_two_phase(self, on=True):
        """Dense-form DF/DF-P iterations through the two-phase pull (exact
        sums, streamed phases) instead of the gathering pull; off frees its layout."""
        _check(lib().dfpr_set_two_phase(self._h, 1 if on else 0))

    def set_timing(self, on=True):
        _check(lib().dfpr_set_timing(self._h, 1 if on else 0))


class _Records(Sequence):
    """Per-member results of a batch call, one dict per member, made when read
    (a batch of hundreds of members returns without building them all)."""

    __slots__ = ("_arr",)

    def __init__(self, arr):
        self._arr = arr

    def __len__(self):
        return len(self._arr)

    def __getitem__(self, k):
        if isinstance(k, slice):
            return [self._arr[i].as_dict() for i in range(*k.indices(len(self._arr)))]
        return self._arr[k].as_dict()


def _ptr_array(items):
    """(void* array, where, keepalive) for a list of int32 id arrays (numpy or torch)."""
    parts = [_ids(a) for a in items]
    wheres = {w for _, k, w, _ in parts if k}
    if len(wheres) > 1:
        raise ValueError("all member arrays must live in the same memory")
    arr = (ctypes.c_void_p * max(len(parts), 1))(*[p for p, _, _, _ in parts])
    return arr, [k for _, k, _, _ in parts], (wheres.pop() if wheres else _capi.HOST), parts


class BatchGraph(Graph):
    """Many independent graphs in one device arena, updated together.

    Member k owns arena vertices [base_k, base_k + n_k); rank vectors span the
    arena.  Each member converges on its own (per-member constant term,
    L-inf change, iteration count)."""

    def __init__(self, handle, n, bases, sizes):
        super().__init__(handle, n)
        self.bases = bases
        self.sizes = sizes

    @property
    def count(self) -> int:
        return len(self.sizes)

    @classmethod
    def from_coo(cls, graphs, keep_ids=False, row_slack=0, stream=None):
        """graphs: list of (n_k, src_k, dst_k) with member-local ids."""
        count = len(graphs)
        ns = (ctypes.c_int32 * count)(*[int(g[0]) for g in graphs])
        srcs, ms, w1, k1 = _ptr_array([g[1] for g in graphs])
        dsts, md, w2, k2 = _ptr_array([g[2] for g in graphs])
        if ms != md:
            raise ValueError("src and dst must have the same length per member")
        if any(ms) and w1 != w2:
            raise ValueError("src and dst must live in the same memory")
        mm = (ctypes.c_int64 * count)(*ms)
        h = ctypes.c_void_p()
        flags = _capi.CREATE_KEEP_IDS if keep_ids else 0
        _check(lib().dfpr_batch_create(count, ns, mm, srcs, dsts, w1, flags, _stream_ptr(stream), ctypes.byref(h)))
        bases, sizes = [], []
        for k in range(count):
            b, n = ctypes.c_int32(), ctypes.c_int32()
            _check(lib().dfpr_batch_member(h, k, ctypes.byref(b), ctypes.byref(n)))
            bases.append(b.value)
            sizes.append(n.value)
        g = cls(h, sum(sizes), bases, sizes)
        if row_slack:
            g.set_row_slack(row_slack, stream=stream)
        return g

    def member(self, r, k):
        """Member k's slice of an arena rank vector."""
        return r[self.bases[k]: self.bases[k] + self.sizes[k]]

    def apply_batch_many(self, batches, stream=None):
        """batches: list (one per member) of (del_src, del_dst, ins_src, ins_dst), member-local ids."""
        if len(batches) != self.count:
            raise ValueError("one batch per member")
        ds, nds, wa, ka = _ptr_array([b[0] for b in batches])
        dd, ndd, wb, kb = _ptr_array([b[1] for b in batches])
        is_, nis, wc, kc = _ptr_array([b[2] for b in batches])
        id_, nid, wd, kd = _ptr_array([b[3] for b in batches])
        if nds != ndd or nis != nid:
            raise ValueError("src/dst length mismatch")
        wheres = {w for w, cnt in ((wa, sum(nds)), (wc, sum(nis))) if cnt}
        if len(wheres) > 1:
            raise ValueError("deletions and insertions must live in the same memory")
        where = wheres.pop() if wheres else _capi.HOST
        info = (BatchInfo * self.count)()
        _check(lib().dfpr_apply_batch_many(self._h, (ctypes.c_int64 * self.count)(*nds), ds, dd,
                                           (ctypes.c_int64 * self.count)(*nis), is_, id_, where,
                                           _stream_ptr(stream), info))
        return _Records(info)

    def update_ranks_many(self, mode, r_prev=None, out=None, stream=None, timing=False, **kw):
        """Update every member; returns (arena ranks, total stats, per-member stats)."""
        import torch
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        p = default_params()
        for k, v in kw.items():
            setattr(p, k, _capi.CRITERIA.get(v, v) if k == "criterion" else v)
        if timing:
            p.flags |= _capi.FLAG_TIMING
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        for t in (out, r_prev):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != self.n):
                raise ValueError("rank vectors must be contiguous float64 CUDA tensors over the arena")
        st = Stats()
        per = (Stats * self.count)()
        rp = ctypes.c_void_p(r_prev.data_ptr()) if r_prev is not None else None
        _check(lib().dfpr_update_ranks_many(self._h, m, ctypes.byref(p), rp, ctypes.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream), ctypes.byref(st), per))
        return out, st.as_dict(), _Records(per)


class Server:
    """Request loop over graphs resident in HBM (see include/dfpr.h, serving form).

    srv = Server(heap_bytes=8 << 30, lanes=4)
    gid = srv.add_graph(Graph.from_coo(n, src, dst))      # the handle moves into the server
    t = srv.submit(gid, del_src, del_dst, ins_src, ins_dst, want_ranks=True)
    ranks, st, info, latency_ms, queue_ms = srv.wait(t)
    """

    def __init__(self, heap_bytes, lanes=4, mode="dfp", **kw):
        p = default_params()
        for k, v in kw.items():
            setattr(p, k, _capi.CRITERIA.get(v, v) if k == "criterion" else v)
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        h = ctypes.c_void_p()
        _check(lib().dfpr_server_create(int(heap_bytes), int(lanes), m, ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self._n = {}
        self._keep = {}
        _live_servers.add(self)

    def close(self):
        if self._h:
            lib().dfpr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add_graph(self, graph, r0=None) -> int:
        """Move `graph` (a plain Graph) into the server; r0: float64 CUDA tensor or None (Static)."""
        gid = ctypes.c_int32()
        rp = ctypes.c_void_p(r0.data_ptr()) if r0 is not None else None
        _check(lib().dfpr_server_add_graph(self._h, graph._h, rp, ctypes.byref(gid)))
        self._n[gid.value] = graph.n
        graph._h = None  # owned by the server now
        return gid.value

    def submit(self, gid, del_src=(), del_dst=(), ins_src=(), ins_dst=(), want_ranks=False) -> int:
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in (del_src, del_dst, ins_src, ins_dst)]
        if arrs[0].size != arrs[1].size or arrs[2].size != arrs[3].size:
            raise ValueError("src/dst length mismatch")
        ptr = [ctypes.c_void_p(a.ctypes.data if a.size else 0) for a in arrs]
        out = np.empty(self._n[gid], np.float64) if want_ranks else None
        t = ctypes.c_int64()
        _check(lib().dfpr_server_submit(self._h, int(gid), arrs[0].size, ptr[0], ptr[1], arrs[2].size, ptr[2], ptr[3],
                                        ctypes.c_void_p(out.ctypes.data) if out is not None else None,
                                        ctypes.byref(t)))
        self._keep[t.value] = out
        return t.value

    def wait(self, ticket):
        """(ranks or None, stats, batch info, latency ms, queue ms); raises DfprError on a failed request."""
        st, info = Stats(), BatchInfo()
        lat, qms = ctypes.c_double(), ctypes.c_double()
        rc = lib().dfpr_server_wait(self._h, int(ticket), ctypes.byref(st), ctypes.byref(info), ctypes.byref(lat),
                                    ctypes.byref(qms))
        out = self._keep.pop(ticket, None)
        _check(rc)
        return out, st.as_dict(), info.as_dict(), lat.value, qms.value

    def ranks(self, gid):
        out = np.empty(self._n[gid], np.float64)
        _check(lib().dfpr_server_ranks(self._h, int(gid), ctypes.c_void_p(out.ctypes.data), _capi.HOST))
        return out

    def set_active_lanes(self, k):
        _check(lib().dfpr_server_set_active_lanes(self._h, int(k)))

    def stats(self) -> dict:
        s = _capi.ServerStats()
        _check(lib().dfpr_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()


def version() -> str:
    return lib().dfpr_version().decode()
