"""Serving form: graphs resident in a server, requests (graph, batch) applied
and ranked concurrently on several lanes.  Every request's result must be the
same as when its graph's requests run alone through the plain entry points
(bit for bit: same kernels, same thresholds), and within L-inf 1e-9 of the
oracle from the same previous ranks."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import LINF, dfpr, hub_graph, rmat, torch_cuda

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _graphs(seed):
    rng = np.random.default_rng(seed)
    gs = [rmat(10, seed=seed), rmat(12, seed=seed + 1), rmat(13, ef=8, seed=seed + 2), rmat(11, ef=24, seed=seed + 3)]
    n = 600
    s, d = W.random_digraph(n, 0.02, seed=seed)
    gs.append((n, s, d))
    gs.append(hub_graph(5000, 1500, 2500, 20000, seed=seed))
    gs.append((1, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    rng.shuffle(gs)
    return gs


def _chains(graphs, steps, seed):
    out = []
    for k, (n, s, d) in enumerate(graphs):
        ch = []
        for t in range(steps):
            if len(s) and t % 2 == 0:
                ch.append(W.batch_8020(n, s, d, 5e-3, seed=seed * 100 + k * 10 + t))
            else:
                ch.append(W.random_edit_batch(n, s, d, 6, 3, seed=seed * 100 + k * 10 + t))
        out.append(ch)
    return out


def _alone(graphs, chains, fused_limit=None):
    """Each graph's chain through a plain handle: the reference results."""
    torch = torch_cuda()
    m = dfpr()
    res = []
    for (n, s, d), ch in zip(graphs, chains):
        g = m.Graph.from_coo(n, s, d)
        if fused_limit is not None:
            g.set_fused_limit(fused_limit)
        r, _ = g.update_ranks("static", None)
        seq = [r.cpu().numpy()]
        for b in ch:
            g.apply_batch(*b)
            r, _ = g.update_ranks("dfp", r, out=r)
            torch.cuda.synchronize()
            seq.append(r.cpu().numpy())
        res.append(seq)
        g.close()
    return res


def _handle(m, n, s, d, fused_limit, row_slack=0):
    g = m.Graph.from_coo(n, s, d, row_slack=row_slack)
    if fused_limit is not None:
        g.set_fused_limit(fused_limit)
    return g


def _serve(graphs, chains, heap_bytes, lanes, fused_limit=None, row_slack=0):
    m = dfpr()
    srv = m.Server(heap_bytes, lanes=lanes)
    gids = [srv.add_graph(_handle(m, n, s, d, fused_limit, row_slack)) for n, s, d in graphs]
    resident = srv.stats()["heap_used"]  # the graphs' CSRs live in the heap
    r0 = [srv.ranks(g) for g in gids]
    tickets = []
    steps = len(chains[0])
    for t in range(steps):  # interleave the graphs: every graph has a request in flight
        for k, gid in enumerate(gids):
            tickets.append((k, t, srv.submit(gid, *chains[k][t], want_ranks=True)))
    out = [[r0[k]] + [None] * steps for k in range(len(graphs))]
    lat = []
    local = 0
    for k, t, tk in tickets:
        r, st, info, ms, qms = srv.wait(tk)
        out[k][t + 1] = r
        lat.append(ms)
        local += info["row_local"]
    stats = srv.stats()
    stats["resident_bytes"] = resident
    stats["row_local_applies"] = local
    final = [srv.ranks(g) for g in gids]
    srv.close()
    return out, stats, final, lat


def test_serving_alone_vs_mix():
    torch_cuda()
    graphs = _graphs(1)
    chains = _chains(graphs, 4, seed=1)
    ref = _alone(graphs, chains)
    _print("serving: mix of", len(graphs), "graphs x", len(chains[0]), "requests, 4 lanes")
    got, stats, final, lat = _serve(graphs, chains, heap_bytes=256 << 20, lanes=4)
    _print("  stats", stats, "p50 latency ms", float(np.median(lat)))
    assert stats["completed"] == stats["submitted"] == len(graphs) * len(chains[0])
    assert stats["failed"] == 0 and stats["heap_used"] == stats["resident_bytes"]
    assert stats["peak_in_flight"] > 1  # requests really overlapped
    for k in range(len(graphs)):
        for t in range(len(chains[k]) + 1):
            assert np.array_equal(got[k][t], ref[k][t]), (k, t, float(np.abs(got[k][t] - ref[k][t]).max()))
        assert np.array_equal(final[k], ref[k][-1])


def test_serving_alone_vs_mix_multilaunch():
    """The same with every update on the launch-per-iteration path (single
    launch disabled, as for graphs above its edge limit): the lanes' pull,
    commit and binning kernels then run concurrently on different streams, and
    each result must still equal its graph's requests run alone, bit for bit."""
    torch_cuda()
    graphs = _graphs(4)
    chains = _chains(graphs, 4, seed=4)
    ref = _alone(graphs, chains, fused_limit=0)
    _print("serving (launch per iteration): mix of", len(graphs), "graphs x", len(chains[0]), "requests, 4 lanes")
    got, stats, final, lat = _serve(graphs, chains, heap_bytes=256 << 20, lanes=4, fused_limit=0)
    _print("  stats", stats, "p50 latency ms", float(np.median(lat)))
    assert stats["completed"] == stats["submitted"] == len(graphs) * len(chains[0])
    assert stats["failed"] == 0 and stats["heap_used"] == stats["resident_bytes"]
    assert stats["peak_in_flight"] > 1
    for k in range(len(graphs)):
        for t in range(len(chains[k]) + 1):
            assert np.array_equal(got[k][t], ref[k][t]), (k, t, float(np.abs(got[k][t] - ref[k][t]).max()))
        assert np.array_equal(final[k], ref[k][-1])


def test_serving_alone_vs_mix_row_slack():
    """Served graphs laid out with free slots per row: small batches merge
    into the rows they touch (in the heap-held CSRs, saving old neighbours in
    the request's borrowed targets); results equal the packed plain handles'
    bit for bit."""
    torch_cuda()
    graphs = _graphs(5)
    chains = _chains(graphs, 4, seed=5)
    ref = _alone(graphs, chains)
    got, stats, final, lat = _serve(graphs, chains, heap_bytes=256 << 20, lanes=4, row_slack=2)
    _print("  serving with row slack: stats", stats)
    assert stats["completed"] == stats["submitted"] == len(graphs) * len(chains[0])
    assert stats["failed"] == 0 and stats["heap_used"] == stats["resident_bytes"]
    assert stats["row_local_applies"] > 0
    for k in range(len(graphs)):
        for t in range(len(chains[k]) + 1):
            assert np.array_equal(got[k][t], ref[k][t]), (k, t, float(np.abs(got[k][t] - ref[k][t]).max()))
        assert np.array_equal(final[k], ref[k][-1])


def test_serving_matches_oracle():
    torch_cuda()
    graphs = _graphs(2)[:4]
    chains = _chains(graphs, 3, seed=2)
    got, stats, _, _ = _serve(graphs, chains, heap_bytes=128 << 20, lanes=3)
    for k, (n, s, d) in enumerate(graphs):
        og = O.graph(n, s, d)
        for t, b in enumerate(chains[k]):
            og2, ob = O.apply(og, *b)
            ref = O.rank("dfp", og2, got[k][t], og, ob)
            err = float(np.abs(got[k][t + 1] - ref.ranks).max())
            assert err <= LINF, (k, t, err)
            og = og2


def test_serving_small_heap_queues_instead_of_failing():
    torch_cuda()
    graphs = _graphs(3)
    chains = _chains(graphs, 3, seed=3)
    ref = _alone(graphs, chains)
    # the most any single request needs, measured with one lane
    _, st1, _, _ = _serve(graphs, chains, heap_bytes=256 << 20, lanes=1)
    need = st1["heap_peak"]
    assert st1["peak_in_flight"] == 1
    # room for about one request beside the resident CSRs, plus headroom for
    # fragmentation (a request's blocks each need a contiguous free range)
    got, st, _, _ = _serve(graphs, chains, heap_bytes=need + (need - st1["resident_bytes"]) // 2, lanes=4)
    _print("  single-request peak", need, "stats", st)
    assert st["failed"] == 0 and st["heap_peak"] <= st["heap_bytes"]
    for k in range(len(graphs)):
        for t in range(len(chains[k]) + 1):
            assert np.array_equal(got[k][t], ref[k][t]), (k, t)


def test_serving_errors():
    torch_cuda()
    m = dfpr()
    n_big, sb, db = rmat(14, seed=5)
    # 3 MiB: holds the graphs' CSRs (~2.3 MB for the scale-14 graph), not a
    # request on the scale-14 graph besides (scratch ~1.7 MB + targets ~2.3 MB)
    srv = m.Server(3 << 20, lanes=2)
    small = srv.add_graph(m.Graph.from_coo(50, *W.random_digraph(50, 0.1, seed=5)))
    big = srv.add_graph(m.Graph.from_coo(n_big, sb, db))
    before = srv.ranks(small)
    t_bad = srv.submit(small, [], [], [0], [50])  # id outside [0, 50)
    t_big = srv.submit(big, [], [], [0], [1])
    t_ok = srv.submit(small, [], [], [0], [1], want_ranks=True)
    with pytest.raises(m.DfprError) as e:
        srv.wait(t_bad)
    assert e.value.code == -2
    with pytest.raises(m.DfprError) as e:
        srv.wait(t_big)
    assert e.value.code == -3
    r, st, info, _, _ = srv.wait(t_ok)
    assert info["ins_in"] == 1 and r.shape == (50,)
    assert st["converged"] == 1
    if info["ins_effective"] == 0:  # (0, 1) already present: nothing marked, ranks unchanged
        assert np.array_equal(r, before)
    with pytest.raises(m.DfprError):
        srv.submit(7, [], [], [], [])
    with pytest.raises(m.DfprError):
        srv.wait(t_ok)  # collected already
    st = srv.stats()
    assert st["failed"] == 2 and st["completed"] == 3
    srv.close()
