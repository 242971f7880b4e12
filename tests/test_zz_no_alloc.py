"""The allocation-free apply entry point (dfpr_apply_batch_noalloc) against
dfpr_apply_batch: the same batches on two handles of the same graph give the
same effective counts, the same CSRs bit for bit and, from the same previous
ranks, the same DF-P ranks bit for bit; two calls in a row, the second with a
smaller batch (the scratch array keeps the first call's contents)."""
import numpy as np
import pytest

import workloads as W
from gpu_common import dfpr, rmat, torch_cuda

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _same_csr(a, b):
    for in_csr in (False, True):
        oa, ia = a.export(in_csr=in_csr)
        ob, ib = b.export(in_csr=in_csr)
        assert np.array_equal(oa, ob) and np.array_equal(ia, ib), in_csr


@pytest.mark.parametrize("device_input", [False, True])
def test_noalloc_matches_apply(device_input):
    torch = torch_cuda()
    m = dfpr()
    n, s, d = rmat(13, seed=71)
    ref = m.Graph.from_coo(n, s, d)
    got = m.Graph.from_coo(n, s, d)
    r0, _ = ref.update_ranks("static", None)
    torch.cuda.synchronize()
    # first call: a large batch (near the pair limit's order at this size), then a smaller one
    for k, frac in enumerate((5e-2, 2e-3)):
        ds, dd, is_, id_ = W.batch_8020(n, s, d, frac, seed=720 + k)
        if k == 1:  # messy entries too: repeats, self pairs, absent deletions
            ds = np.concatenate([ds, ds[:3], [5], [7]]).astype(np.int32)
            dd = np.concatenate([dd, dd[:3], [5], [int(d[0])]]).astype(np.int32)
            is_ = np.concatenate([is_, is_[:4], [9]]).astype(np.int32)
            id_ = np.concatenate([id_, id_[:4], [9]]).astype(np.int32)
        args = (ds, dd, is_, id_)
        if device_input:
            args = tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in args)
        ia = ref.apply_batch(*args)
        ib = got.apply_batch_noalloc(*args)
        _print(f"noalloc call {k} ({len(ds) + len(is_)} pairs, device={device_input}): {ib}")
        for key in ("ins_in", "ins_effective", "del_in", "del_effective", "self_loop_dels_ignored", "m_after"):
            assert ia[key] == ib[key], (k, key, ia[key], ib[key])
        _same_csr(ref, got)
        ra, sa = ref.update_ranks("dfp", r0)
        rb, sb = got.update_ranks("dfp", r0)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb) and sa["iterations"] == sb["iterations"], k
        r0 = ra.clone()
    ref.close()
    got.close()


def test_noalloc_limits():
    torch_cuda()
    m = dfpr()
    n, s, d = rmat(10, seed=73)
    g = m.Graph.from_coo(n, s, d, edge_capacity=len(s) + n)  # no room for growth
    off0, idx0 = g.export()
    big = np.zeros(m._capi.NOALLOC_MAX_PAIRS + 1, np.int32)
    with pytest.raises(m.DfprError) as e:
        g.apply_batch_noalloc([], [], big, big)
    assert e.value.code == m._capi.DFPR_EINVAL
    ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-2, seed=74)
    with pytest.raises(m.DfprError) as e:
        g.apply_batch_noalloc([], [], is_, id_)  # insertions beyond the reserved capacity
    assert e.value.code == m._capi.DFPR_ENOMEM
    off1, idx1 = g.export()
    assert np.array_equal(off0, off1) and np.array_equal(idx0, idx1)
    info = g.apply_batch_noalloc(ds, dd, [], [])  # deletions only: fits
    assert info["del_effective"] == len(ds)
    g.close()
