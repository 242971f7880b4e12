"""Rows with free slots (dfpr_set_row_slack): small batches merge into the rows
they touch, a row without room lays every row out again, large batches take
the usual rebuild.  Whatever the layout, the exported CSRs equal the oracle's
bit for bit (Section 3.2 batch semantics), and the ranks equal those of the
same graph with packed rows bit for bit (the rank kernels read only the
neighbours of a row) and the oracle's within the parity bar."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import LINF, Pair, assert_csr_equal, assert_info_equal, dfpr, hub_graph, rmat, torch_cuda

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


class Twin:
    """One graph three ways: packed rows, rows with free slots, the oracle."""

    def __init__(self, n, s, d, slack, keep_ids=False):
        self.packed = Pair(n, s, d, keep_ids=keep_ids)
        self.slack = Pair(n, s, d, keep_ids=keep_ids, row_slack=slack)
        self.n = n

    def apply(self, ds, dd, is_, id_, device=False):
        self.packed.apply(ds, dd, is_, id_, device=device)
        info = self.slack.apply(ds, dd, is_, id_, device=device)
        assert_csr_equal(self.slack.g, self.slack.og)
        return info

    def rank(self, mode, r_prev, **kw):
        r1, st1, ref = self.slack.rank(mode, r_prev, **kw)
        r0, st0, _ = self.packed.rank(mode, r_prev, **kw)
        assert np.array_equal(r1, r0), (mode, float(np.abs(r1 - r0).max()))
        assert st1["iterations"] == st0["iterations"] and st1["ever_affected"] == st0["ever_affected"]
        err = float(np.abs(r1 - ref.ranks).max())
        assert err <= LINF, (mode, err)
        return r1, st1, ref


@pytest.mark.parametrize("keep_ids", [False, True])
@pytest.mark.parametrize("slack", [1, 3])
def test_slack_layout_export_and_static(slack, keep_ids):
    torch_cuda()
    n, s, d = rmat(12, ef=12, seed=31)
    t = Twin(n, s, d, slack, keep_ids=keep_ids)
    _print("slack layout", slack, "keep_ids", keep_ids, "n", n, "m", t.slack.og.m)
    assert_csr_equal(t.slack.g, t.slack.og)
    assert t.slack.g.m == t.slack.og.m
    t.rank("static", None)


@pytest.mark.parametrize("keep_ids", [False, True])
def test_slack_row_local_chain(keep_ids):
    """Chained small 80/20 batches: row-local while every touched row has room,
    a re-layout when one has none, row-local again afterwards."""
    torch_cuda()
    n, s, d = rmat(13, ef=10, seed=32)
    t = Twin(n, s, d, 2, keep_ids=keep_ids)
    r = O.rank("static", t.slack.og).ranks
    paths = []
    for step in range(8):
        og = t.slack.og
        ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 2e-4, seed=700 + step)
        info = t.apply(ds, dd, is_, id_, device=bool(step % 2))
        paths.append(info["row_local"])
        mode = ("df", "dfp")[step % 2]
        r, st, ref = t.rank(mode, r)
        r = ref.ranks
    _print("row-local per step", paths)
    assert paths[0] == 1 and sum(paths) >= 4


def test_slack_full_row_relays_out():
    """Slack 1 and two insertions into one row: no room, so every row is laid
    out again with one free slot; the next small batch merges in place."""
    torch_cuda()
    n, s, d = rmat(11, ef=8, seed=33)
    t = Twin(n, s, d, 1, keep_ids=True)
    og = t.slack.og
    u = 5
    outs = set(og.out_idx[og.out_off[u]:og.out_off[u + 1]].tolist())
    new = [v for v in range(n) if v not in outs and v != u][:3]
    info = t.apply([], [], [u] * len(new), new)
    assert info["row_local"] == 0 and info["ins_effective"] == 3
    r0 = O.rank("static", t.slack.og).ranks
    info = t.apply([], [], [u], [[v for v in range(n) if v not in outs and v != u][5]])
    assert info["row_local"] == 1
    t.rank("dfp", r0)


def test_slack_deletions_and_insertions_in_one_row():
    """One hub row loses and gains neighbours in one batch (more than a
    workgroup's worth of old neighbours, so the merge loops), plus a batch
    of deletions only; then a large batch that takes the usual rebuild."""
    torch_cuda()
    n, s, d = hub_graph(3000, 900, 1200, 6000, seed=34)
    t = Twin(n, s, d, 4)
    og = t.slack.og
    hub_out = og.out_idx[og.out_off[0]:og.out_off[1]]
    dels = hub_out[1::50][:8]
    cand = np.setdiff1d(np.arange(1, n), hub_out)[:3]
    info = t.apply(np.zeros(len(dels), np.int32), dels, np.zeros(len(cand), np.int32), cand)
    assert info["row_local"] == 1
    r = O.rank("static", t.slack.og).ranks
    t.rank("dfp", r)
    og = t.slack.og
    k = np.arange(0, og.esrc.shape[0], 97)
    keep = og.esrc[k] != og.edst[k]
    info = t.apply(og.esrc[k][keep][:20], og.edst[k][keep][:20], [], [])
    assert info["row_local"] == 1
    og = t.slack.og
    ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 5e-2, seed=35)
    info = t.apply(ds, dd, is_, id_)
    assert info["row_local"] == 0  # more than one pair per 256 slots: the usual rebuild
    r = O.rank("static", t.slack.og).ranks
    og = t.slack.og
    ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 1e-3, seed=36)
    t.apply(ds, dd, is_, id_)
    t.rank("dfp", r)


def test_slack_set_and_clear():
    torch_cuda()
    m = dfpr()
    n, s, d = rmat(10, ef=8, seed=37)
    p = Pair(n, s, d)
    for slack in (5, 0, 2):
        p.g.set_row_slack(slack)
        assert_csr_equal(p.g, p.og)
    og = p.og
    ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 1e-3, seed=38)
    info = p.apply(ds, dd, is_, id_)
    assert_csr_equal(p.g, p.og)
    p.g.set_row_slack(0)
    assert_csr_equal(p.g, p.og)
    for bad in (-1, (1 << 16) + 1):
        with pytest.raises(m.DfprError) as e:
            p.g.set_row_slack(bad)
        assert e.value.code == -1
    assert_csr_equal(p.g, p.og)
    _print("set/clear slack: last batch row_local", info["row_local"])


def test_slack_noalloc_apply():
    """The allocation-free apply on rows with free slots: same CSRs and ranks
    as the allocating apply on a twin graph."""
    torch = torch_cuda()
    m = dfpr()
    n, s, d = rmat(12, ef=10, seed=39)
    a = m.Graph.from_coo(n, s, d, row_slack=2)
    b = m.Graph.from_coo(n, s, d, row_slack=2)
    og = O.graph(n, s, d)
    r0 = torch.from_numpy(O.rank("static", og).ranks).cuda()
    for step in range(3):
        ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 3e-4, seed=800 + step)
        ia = a.apply_batch(ds, dd, is_, id_)
        ib = b.apply_batch_noalloc(ds, dd, is_, id_)
        og, _ = O.apply(og, ds, dd, is_, id_)
        assert ia["row_local"] == ib["row_local"]
        for in_csr in (False, True):
            oa, xa = a.export(in_csr=in_csr)
            ob, xb = b.export(in_csr=in_csr)
            assert np.array_equal(oa, ob) and np.array_equal(xa, xb)
        ra, _ = a.update_ranks("dfp", r0.clone())
        rb, _ = b.update_ranks("dfp", r0.clone())
        assert torch.equal(ra, rb)
        r0 = ra
    a.close()
    b.close()


def test_slack_batched_members():
    torch = torch_cuda()
    m = dfpr()
    members = [rmat(sc, ef=10, seed=50 + sc) for sc in (8, 10, 9)]
    bg = m.BatchGraph.from_coo(members, row_slack=2)
    plain = [m.Graph.from_coo(n, s, d) for n, s, d in members]
    ogs = [O.graph(n, s, d) for n, s, d in members]
    r, _, _ = bg.update_ranks_many("static", None)
    r_prev = r.clone()
    batches = [W.batch_8020(n, og.esrc, og.edst, 2e-3, seed=60 + k) for k, ((n, _, _), og) in
               enumerate(zip(members, ogs))]
    infos = bg.apply_batch_many(batches)
    _print("batched slack: row_local", [i.get("row_local") for i in infos])
    off, idx = bg.export()
    for k, ((n, _, _), og) in enumerate(zip(members, ogs)):
        og2, ob = O.apply(og, *batches[k])
        assert_info_equal(infos[k], ob)
        base = bg.bases[k]
        o = off[base: base + n + 1].astype(np.int64)
        assert np.array_equal(o - o[0], og2.out_off) and np.array_equal(idx[o[0]: o[-1]] - base, og2.out_idx)
    r, _, per = bg.update_ranks_many("dfp", r_prev)
    for k, g in enumerate(plain):
        g.apply_batch(*batches[k])
        rk, st = g.update_ranks("dfp", bg.member(r_prev, k).clone())
        assert torch.equal(bg.member(r, k), rk), k


def test_slack_long_rows_in_chunks():
    """A hub row longer than one merge work item (4096 neighbours) in both
    CSRs: changed in place, then past its free slots (re-laid out)."""
    torch_cuda()
    n, s, d = hub_graph(20000, 9000, 10000, 20000, seed=40)
    t = Twin(n, s, d, 2)
    og = t.slack.og
    hub_out = og.out_idx[og.out_off[0]:og.out_off[1]]
    hub_in = og.in_idx[og.in_off[0]:og.in_off[1]]
    assert len(hub_out) > 2 * 4096 and len(hub_in) > 2 * 4096
    new_out = np.setdiff1d(np.arange(1, n), hub_out)[[3, 500, 9000]]
    new_in = np.setdiff1d(np.arange(1, n), hub_in)[[7, 800]]
    ds = np.concatenate([np.zeros(4, np.int32), hub_in[[100, 5000, 8000]]])
    dd = np.concatenate([hub_out[[50, 4100, 4097, 9999]], np.zeros(3, np.int32)])
    is_ = np.concatenate([np.zeros(3, np.int32), new_in])
    id_ = np.concatenate([new_out, np.zeros(2, np.int32)])
    info = t.apply(ds, dd, is_, id_)
    assert info["row_local"] == 1
    r = O.rank("static", t.slack.og).ranks
    t.rank("dfp", r)
    og = t.slack.og
    hub_out = og.out_idx[og.out_off[0]:og.out_off[1]]
    new_out = np.setdiff1d(np.arange(1, n), hub_out)[[1, 2, 4000, 7000, 9000]]
    info = t.apply([0], [hub_out[6000]], np.zeros(5, np.int32), new_out, device=True)
    assert info["row_local"] == 0  # 4 net insertions, 2 free slots: laid out again
    t.rank("dfp", r)
    og = t.slack.og
    hub_in = og.in_idx[og.in_off[0]:og.in_off[1]]
    info = t.apply([], [], np.setdiff1d(np.arange(1, n), hub_in)[[11, 12]], np.zeros(2, np.int32))
    assert info["row_local"] == 1  # fresh free slots after the re-layout
    t.rank("df", r)


def test_slack_power_of_two_vertex_count():
    """n a power of two: the pad id n needs one id bit more than the vertices.
    Rows next to rows that lose their edge to vertex 0 in a large batch (the
    general rebuild, which keys pads like entries) keep their pads, and later
    small batches and large batches still give the oracle's CSRs."""
    torch_cuda()
    n, s, d = hub_graph(4096, 900, 1200, 8000, seed=41)
    t = Twin(n, s, d, 2)
    og = t.slack.og
    to0 = og.in_idx[og.in_off[0]:og.in_off[1]]
    to0 = to0[to0 > 0][:60]
    for step in range(3):
        og = t.slack.og
        ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 3e-2, seed=42 + step)
        if step == 0:
            ds = np.concatenate([ds, to0]).astype(np.int32)
            dd = np.concatenate([dd, np.zeros(len(to0), np.int32)])
        info = t.apply(ds, dd, is_, id_)
        assert info["row_local"] == 0
        og = t.slack.og
        ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 2e-4, seed=52 + step)
        t.apply(ds, dd, is_, id_)
    r = O.rank("static", t.slack.og).ranks
    og = t.slack.og
    ds, dd, is_, id_ = W.batch_8020(n, og.esrc, og.edst, 1e-3, seed=60)
    t.apply(ds, dd, is_, id_)
    t.rank("dfp", r)
