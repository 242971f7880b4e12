"""ctypes declarations of the dfpr C ABI (include/dfpr.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfpr.so")

DFPR_OK, DFPR_EINVAL, DFPR_ERANGE, DFPR_ENOMEM, DFPR_EHIP, DFPR_ESTATE = 0, -1, -2, -3, -4, -5
STATIC, ND, DF, DFP = 0, 1, 2, 3
HOST, DEVICE = 0, 1
FLAG_TIMING = 1
FLAG_ASYNC = 2
NOALLOC_MAX_PAIRS = 1 << 19
CRITERIA = {"relative": 0, "absolute": 1, "contrib": 2}
CREATE_KEEP_IDS = 1

# Every exported function declared in include/dfpr.h.
EXPORTS = ("dfpr_params_default", "dfpr_graph_create", "dfpr_graph_destroy", "dfpr_graph_size",
           "dfpr_graph_export", "dfpr_apply_batch", "dfpr_apply_batch_noalloc", "dfpr_update_ranks", "dfpr_set_tuning",
           "dfpr_get_tuning", "dfpr_autotune", "dfpr_set_timing", "dfpr_set_fused_limit",
           "dfpr_set_row_slack", "dfpr_set_two_phase", "dfpr_batch_create", "dfpr_batch_count",
           "dfpr_batch_member", "dfpr_apply_batch_many", "dfpr_update_ranks_many", "dfpr_server_create",
           "dfpr_server_destroy", "dfpr_server_add_graph", "dfpr_server_submit", "dfpr_server_wait",
           "dfpr_server_ranks", "dfpr_server_graph_size", "dfpr_server_get_stats", "dfpr_server_set_active_lanes",
           "dfpr_last_error",
           "dfpr_version")


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tol", ctypes.c_double), ("frontier_tol", ctypes.c_double),
                ("prune_tol", ctypes.c_double), ("dense_switch", ctypes.c_double), ("max_iters", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("criterion", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("ins_in", ctypes.c_int64), ("ins_effective", ctypes.c_int64), ("del_in", ctypes.c_int64),
                ("del_effective", ctypes.c_int64), ("self_loop_dels_ignored", ctypes.c_int64),
                ("m_after", ctypes.c_int64), ("ms_total", ctypes.c_double), ("ms_sort", ctypes.c_double),
                ("ms_rebuild", ctypes.c_double * 2), ("row_local", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return _as_dict(self)


def _as_dict(rec, drop=("reserved", "reserved2", "reserved3")):
    """Fields of a ctypes struct as a dict (arrays as lists), reserved fields left out."""
    cls = type(rec)
    names = cls.__dict__.get("_names")
    if names is None:  # per class, once: (field, is_array)
        names = tuple((k, hasattr(t, "_length_")) for k, t in cls._fields_ if k not in drop)
        cls._names = names
    return {k: (list(getattr(rec, k)) if arr else getattr(rec, k)) for k, arr in names}


BINS = 6


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("last_delta", ctypes.c_double),
                ("ever_affected", ctypes.c_int64), ("vertex_updates", ctypes.c_int64),
                ("edges_pulled", ctypes.c_int64), ("bin_vertices", ctypes.c_int64 * BINS),
                ("bin_edges", ctypes.c_int64 * BINS), ("ms_total", ctypes.c_double), ("ms_pull", ctypes.c_double),
                ("pull_launches", ctypes.c_int32), ("reserved", ctypes.c_int32), ("ms_commit", ctypes.c_double),
                ("ms_bin", ctypes.c_double), ("ms_mark", ctypes.c_double), ("pull_bytes", ctypes.c_double),
                ("dense_iterations", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("ms_two_phase", ctypes.c_double), ("two_phase_bytes", ctypes.c_double),
                ("two_phase_passes", ctypes.c_int32), ("reserved3", ctypes.c_int32)]

    def as_dict(self):
        return _as_dict(self)


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("peak_in_flight", ctypes.c_int64), ("in_flight", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("lanes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("heap_bytes", ctypes.c_int64), ("heap_used", ctypes.c_int64), ("heap_peak", ctypes.c_int64)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out.pop("reserved", None)
        return out


def declare(lib):
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.dfpr_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.dfpr_params_default.restype = None
    lib.dfpr_graph_create.argtypes = [i32, i64, P, P, ctypes.c_int, i64, i32, P, ctypes.POINTER(P)]
    lib.dfpr_graph_create.restype = ctypes.c_int
    lib.dfpr_graph_destroy.argtypes = [P]
    lib.dfpr_graph_destroy.restype = ctypes.c_int
    lib.dfpr_graph_size.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.dfpr_graph_size.restype = ctypes.c_int
    lib.dfpr_graph_export.argtypes = [P, ctypes.c_int, P, P, ctypes.c_int, P]
    lib.dfpr_graph_export.restype = ctypes.c_int
    lib.dfpr_apply_batch.argtypes = [P, i64, P, P, i64, P, P, ctypes.c_int, P, ctypes.POINTER(BatchInfo)]
    lib.dfpr_apply_batch.restype = ctypes.c_int
    lib.dfpr_apply_batch_noalloc.argtypes = [P, i64, P, P, i64, P, P, ctypes.c_int, P, ctypes.POINTER(BatchInfo)]
    lib.dfpr_apply_batch_noalloc.restype = ctypes.c_int
    lib.dfpr_update_ranks.argtypes = [P, ctypes.c_int, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(Stats)]
    lib.dfpr_update_ranks.restype = ctypes.c_int
    lib.dfpr_set_tuning.argtypes = [P, ctypes.POINTER(i32)]
    lib.dfpr_set_tuning.restype = ctypes.c_int
    lib.dfpr_get_tuning.argtypes = [P, ctypes.POINTER(i32)]
    lib.dfpr_get_tuning.restype = ctypes.c_int
    lib.dfpr_autotune.argtypes = [P, P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.dfpr_autotune.restype = ctypes.c_int
    lib.dfpr_set_fused_limit.argtypes = [P, i64]
    lib.dfpr_set_fused_limit.restype = ctypes.c_int
    lib.dfpr_set_row_slack.argtypes = [P, i32, P]
    lib.dfpr_set_row_slack.restype = ctypes.c_int
    lib.dfpr_set_two_phase.argtypes = [P, ctypes.c_int]
    lib.dfpr_set_two_phase.restype = ctypes.c_int
    lib.dfpr_set_timing.argtypes = [P, ctypes.c_int]
    lib.dfpr_set_timing.restype = ctypes.c_int
    PP = ctypes.POINTER(P)
    lib.dfpr_batch_create.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i64), PP, PP, ctypes.c_int, i32, P,
                                      ctypes.POINTER(P)]
    lib.dfpr_batch_create.restype = ctypes.c_int
    lib.dfpr_batch_count.argtypes = [P, ctypes.POINTER(i32)]
    lib.dfpr_batch_count.restype = ctypes.c_int
    lib.dfpr_batch_member.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.dfpr_batch_member.restype = ctypes.c_int
    lib.dfpr_apply_batch_many.argtypes = [P, ctypes.POINTER(i64), PP, PP, ctypes.POINTER(i64), PP, PP, ctypes.c_int,
                                          P, ctypes.POINTER(BatchInfo)]
    lib.dfpr_apply_batch_many.restype = ctypes.c_int
    lib.dfpr_update_ranks_many.argtypes = [P, ctypes.c_int, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(Stats),
                                           ctypes.POINTER(Stats)]
    lib.dfpr_update_ranks_many.restype = ctypes.c_int
    D = ctypes.POINTER(ctypes.c_double)
    lib.dfpr_server_create.argtypes = [ctypes.c_size_t, i32, ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(P)]
    lib.dfpr_server_create.restype = ctypes.c_int
    lib.dfpr_server_destroy.argtypes = [P]
    lib.dfpr_server_destroy.restype = ctypes.c_int
    lib.dfpr_server_add_graph.argtypes = [P, P, P, ctypes.POINTER(i32)]
    lib.dfpr_server_add_graph.restype = ctypes.c_int
    lib.dfpr_server_submit.argtypes = [P, i32, i64, P, P, i64, P, P, P, ctypes.POINTER(i64)]
    lib.dfpr_server_submit.restype = ctypes.c_int
    lib.dfpr_server_wait.argtypes = [P, i64, ctypes.POINTER(Stats), ctypes.POINTER(BatchInfo), D, D]
    lib.dfpr_server_wait.restype = ctypes.c_int
    lib.dfpr_server_ranks.argtypes = [P, i32, P, ctypes.c_int]
    lib.dfpr_server_ranks.restype = ctypes.c_int
    lib.dfpr_server_graph_size.argtypes = [P, i32, ctypes.POINTER(i32)]
    lib.dfpr_server_graph_size.restype = ctypes.c_int
    lib.dfpr_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.dfpr_server_get_stats.restype = ctypes.c_int
    lib.dfpr_server_set_active_lanes.argtypes = [P, i32]
    lib.dfpr_server_set_active_lanes.restype = ctypes.c_int
    lib.dfpr_last_error.argtypes = []
    lib.dfpr_last_error.restype = ctypes.c_char_p
    lib.dfpr_version.argtypes = []
    lib.dfpr_version.restype = ctypes.c_char_p
    return lib


_lib = None


def load(path: str | None = None):
    """Load the built HIP library.  Raises if it is missing: there is no fallback."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"dfpr HIP library not built: {p} is missing (run __graft_entry__.build())")
    # One HIP runtime per process: torch carries its own copy of the runtime
    # (same soname); loading it first lets the library bind to that copy
    # instead of pulling in a second runtime, which would then see no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = declare(ctypes.CDLL(p))
    if path is None:
        _lib = lib
    return lib
