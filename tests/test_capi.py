"""The C-ABI library loads and exports every symbol include/dfpr.h declares;
argument checks that return before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2401_15870_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dfpr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfpr_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_capi.LIB_PATH):
        from paper_2401_15870_amd import build
        build.build()
    return _capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    assert set(names) == set(_capi.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_params_default(lib):
    p = _capi.Params()
    lib.dfpr_params_default(ctypes.byref(p))
    assert (p.alpha, p.tol, p.frontier_tol, p.prune_tol, p.max_iters, p.flags) == (0.85, 1e-10, 1e-6, 1e-6, 500, 0)
    assert p.dense_switch == 1.0 and p.criterion == 0 and p.reserved == 0


def test_invalid_arguments_rejected_before_device_work(lib):
    h = ctypes.c_void_p()
    assert lib.dfpr_graph_create(0, 0, None, None, 0, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_graph_create(5, 3, None, None, 0, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_graph_create(5, -1, None, None, 0, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_graph_create(5, 0, None, None, 0, 0, 8, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert b"invalid" in lib.dfpr_last_error()
    st = _capi.Stats()
    assert lib.dfpr_update_ranks(None, 3, None, None, None, None, ctypes.byref(st)) == _capi.DFPR_EINVAL
    assert lib.dfpr_set_tuning(None, (ctypes.c_int32 * 5)(4, 8, 16, 32, 64)) == _capi.DFPR_EINVAL
    assert lib.dfpr_set_fused_limit(None, -1) == _capi.DFPR_EINVAL
    assert lib.dfpr_set_fused_limit(None, 5) == _capi.DFPR_EINVAL
    assert lib.dfpr_apply_batch(None, -1, None, None, 0, None, None, 0, None, None) == _capi.DFPR_EINVAL
    assert lib.dfpr_graph_destroy(None) == _capi.DFPR_OK
    # batched form
    n1 = (ctypes.c_int32 * 1)(5)
    m1 = (ctypes.c_int64 * 1)(0)
    pp = (ctypes.c_void_p * 1)()
    assert lib.dfpr_batch_create(0, n1, m1, pp, pp, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    n0 = (ctypes.c_int32 * 1)(0)
    assert lib.dfpr_batch_create(1, n0, m1, pp, pp, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    m3 = (ctypes.c_int64 * 1)(3)
    assert lib.dfpr_batch_create(1, n1, m3, pp, pp, 0, 0, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert b"member 0" in lib.dfpr_last_error()
    assert lib.dfpr_batch_create(1, n1, m1, pp, pp, 0, 2, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    cnt = ctypes.c_int32()
    assert lib.dfpr_batch_count(None, ctypes.byref(cnt)) == _capi.DFPR_EINVAL
    b, n = ctypes.c_int32(), ctypes.c_int32()
    assert lib.dfpr_batch_member(None, 0, ctypes.byref(b), ctypes.byref(n)) == _capi.DFPR_EINVAL
    assert lib.dfpr_apply_batch_many(None, None, None, None, None, None, None, 0, None, None) == _capi.DFPR_EINVAL
    assert lib.dfpr_update_ranks_many(None, 3, None, None, None, None, None, None) == _capi.DFPR_EINVAL
    assert lib.dfpr_set_row_slack(None, 2, None) == _capi.DFPR_EINVAL
    # serving form
    assert lib.dfpr_server_create(0, 4, 3, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_server_create(1 << 20, 0, 3, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_server_create(1 << 20, 4, 9, None, ctypes.byref(h)) == _capi.DFPR_EINVAL
    assert lib.dfpr_server_destroy(None) == _capi.DFPR_OK
    t = ctypes.c_int64()
    assert lib.dfpr_server_submit(None, 0, 0, None, None, 0, None, None, None, ctypes.byref(t)) == _capi.DFPR_EINVAL
    assert lib.dfpr_server_wait(None, 1, None, None, None, None) == _capi.DFPR_EINVAL
    assert lib.dfpr_server_add_graph(None, None, None, None) == _capi.DFPR_EINVAL
    ss = _capi.ServerStats()
    assert lib.dfpr_server_get_stats(None, ctypes.byref(ss)) == _capi.DFPR_EINVAL
    assert lib.dfpr_version().startswith(b"dfpr")


def test_struct_layouts_match_header():
    # field counts and sizes of the ABI structs as declared in include/dfpr.h
    assert ctypes.sizeof(_capi.Params) == 5 * 8 + 4 * 4
    assert ctypes.sizeof(_capi.BatchInfo) == 6 * 8 + 4 * 8 + 2 * 4
    assert ctypes.sizeof(_capi.Stats) == 4 + 4 + 8 + 3 * 8 + 12 * 8 + 8 + 8 + 4 + 4 + 3 * 8 + 8 + 4 + 4 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(_capi.ServerStats) == 5 * 8 + 4 * 4 + 3 * 8


def test_per_member_records_and_struct_dicts():
    """Per-member results of batch calls: one dict per member, made when read,
    arrays as lists, reserved fields left out."""
    import paper_2401_15870_amd as m
    info = (_capi.BatchInfo * 3)()
    for k in range(3):
        info[k].ins_in = 10 + k
        info[k].ms_rebuild[1] = 0.5 * k
        info[k].row_local = k % 2
    rec = m._Records(info)
    assert len(rec) == 3
    assert rec[1]["ins_in"] == 11 and rec[1]["row_local"] == 1 and rec[2]["ms_rebuild"] == [0.0, 1.0]
    assert rec[-1]["ins_in"] == 12
    assert [r["ins_in"] for r in rec] == [10, 11, 12]
    assert [r["ins_in"] for r in rec[1:]] == [11, 12]
    assert "reserved" not in rec[0]
    st = _capi.Stats()
    st.iterations = 7
    st.bin_edges[5] = 9
    d = st.as_dict()
    assert d["iterations"] == 7 and d["bin_edges"] == [0, 0, 0, 0, 0, 9]
    assert "reserved" not in d and "reserved2" not in d and "reserved3" not in d
