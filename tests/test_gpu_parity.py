"""GPU path against the CPU oracle through the C ABI: canonical CSRs bit-exact,
effective batch counts equal, ranks within L-inf 1e-9 from the same R_prev bits
(bit-exact when every vertex is in the one-lane-per-vertex bin)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import LINF, Pair, assert_csr_equal, hub_graph, rmat, torch_cuda

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ graph store
@pytest.mark.parametrize("keep_ids", [False, True])
@pytest.mark.parametrize("case", ["single_vertex", "no_edges", "dups_and_selfs", "rmat10", "rmat14", "hub"])
def test_create_csr_bitexact(case, keep_ids):
    torch_cuda()
    _print("create", case)
    if case == "single_vertex":
        n, s, d = 1, np.zeros(0, np.int32), np.zeros(0, np.int32)
    elif case == "no_edges":
        n, s, d = 37, np.zeros(0, np.int32), np.zeros(0, np.int32)
    elif case == "dups_and_selfs":
        n = 300
        rng = np.random.default_rng(3)
        s = rng.integers(0, n, 5000).astype(np.int32)
        d = rng.integers(0, n, 5000).astype(np.int32)
        d[::7] = s[::7]
    elif case == "rmat10":
        n, s, d = rmat(10, seed=2)
    elif case == "rmat14":
        n, s, d = rmat(14, seed=3)
    else:
        n, s, d = hub_graph(30000, 9000, 12000, 60000, seed=4)
    p = Pair(n, s, d, keep_ids=keep_ids)
    assert p.g.m == p.og.m
    assert_csr_equal(p.g, p.og)


def test_apply_messy_batches_chained():
    """Repeated pairs, self-loop deletes, absent deletes, existing inserts, a pair
    both inserted and deleted: every step matches the oracle bit for bit."""
    torch_cuda()
    rng = np.random.default_rng(7)
    for trial in range(12):
        n = int(rng.integers(2, 400))
        s, d = W.random_digraph(n, float(rng.uniform(0.002, 0.05)), seed=trial)
        p = Pair(n, s, d, keep_ids=bool(trial % 2))
        for step in range(4):
            ds, dd, is_, id_ = W.random_edit_batch(n, p.og.esrc, p.og.edst, int(rng.integers(0, 60)),
                                                   int(rng.integers(0, 60)), seed=trial * 10 + step)
            _print("apply", trial, step, n, len(ds), len(is_))
            p.apply(ds, dd, is_, id_, device=(step % 2 == 1))
            assert_csr_equal(p.g, p.og)


@pytest.mark.parametrize("frac", [1e-5, 1e-3, 1e-1])
def test_apply_8020_rmat14(frac):
    """Batches below and above the one-block sort size; the inverse batch restores G0."""
    torch_cuda()
    n, s, d = rmat(14, seed=5)
    p = Pair(n, s, d)
    g0 = (p.og.out_off.copy(), p.og.out_idx.copy())
    ds, dd, is_, id_ = W.batch_8020(n, s, d, frac, seed=6)
    _print("apply8020", frac, len(ds), len(is_))
    p.apply(ds, dd, is_, id_)
    assert_csr_equal(p.g, p.og)
    p.apply(is_, id_, ds, dd)  # inverse: delete what was inserted, insert what was deleted
    assert_csr_equal(p.g, p.og)
    assert np.array_equal(p.og.out_off, g0[0]) and np.array_equal(p.og.out_idx, g0[1])


def test_apply_hub_rows():
    torch_cuda()
    n, s, d = hub_graph(20000, 7000, 9000, 40000, seed=8)
    p = Pair(n, s, d)
    rng = np.random.default_rng(9)
    # delete half of the hub's in-edges and add new ones to and from the hub
    hub_in = p.og.in_idx[p.og.in_off[0]:p.og.in_off[1]]
    dels = hub_in[hub_in != 0][::2]
    new = rng.integers(1, n, 3000).astype(np.int32)
    p.apply(dels, np.zeros_like(dels), np.concatenate([new, np.zeros(3000, np.int32)]),
            np.concatenate([np.zeros(3000, np.int32), new]))
    assert_csr_equal(p.g, p.og)


def _pairs_not_in(rng, og, count, u_range, v_range, taken):
    """`count` distinct non-self pairs with u, v in the given ranges, absent from the graph and `taken`."""
    existing = set(zip(og.esrc.tolist(), og.edst.tolist()))
    out = []
    while len(out) < count:
        u = int(rng.integers(*u_range))
        v = int(rng.integers(*v_range))
        if u != v and (u, v) not in existing and (u, v) not in taken:
            taken.add((u, v))
            out.append((u, v))
    return out


@pytest.mark.parametrize("extra", [0, 1])
def test_apply_run_and_group_paths(extra):
    """Raw batch sizes on both sides of the switch between the run-by-run copy
    (at most one raw entry per 256 edges) and the merge of touched groups."""
    torch_cuda()
    n, s, d = rmat(12, seed=61)
    p = Pair(n, s, d)
    rng = np.random.default_rng(62)
    nk = p.og.m // 256 + extra
    n_del = nk // 5
    nonself = np.flatnonzero(p.og.esrc != p.og.edst)
    pick = rng.choice(nonself, n_del, replace=False)
    ins = _pairs_not_in(rng, p.og, nk - n_del, (0, n), (0, n), set())
    _print("apply paths", nk, p.og.m)
    p.apply(p.og.esrc[pick], p.og.edst[pick], np.array([u for u, _ in ins], np.int32),
            np.array([v for _, v in ins], np.int32))
    assert_csr_equal(p.g, p.og)


def test_apply_runs_in_one_row():
    """Run-by-run copy with all the cuts in one row: a small batch (below one
    raw entry per 256 edges) that inserts 300 new out-neighbours of vertex 7
    and deletes 100 of its existing ones, so consecutive runs are empty or one
    element long."""
    torch_cuda()
    n, s, d = rmat(15, seed=81)
    p = Pair(n, s, d, keep_ids=True)
    og = p.og
    rng = np.random.default_rng(82)
    row = og.out_idx[og.out_off[7]:og.out_off[8]]
    row = row[row != 7]
    dels = rng.choice(row, min(100, len(row)), replace=False).astype(np.int32)
    cand = np.setdiff1d(np.arange(n, dtype=np.int32), np.concatenate([row, [7]]))
    ins = rng.choice(cand, 300, replace=False).astype(np.int32)
    assert len(dels) + len(ins) <= og.m // 256
    _print("runs in one row", len(dels), len(ins), og.m)
    info = p.apply(np.full(len(dels), 7, np.int32), dels, np.full(300, 7, np.int32), ins)
    assert info["ins_effective"] == 300 and info["del_effective"] == len(dels)
    assert_csr_equal(p.g, p.og)


@pytest.mark.parametrize("side", ["out", "in"])
@pytest.mark.parametrize("scale,step", [(14, 1024), (15, 16384)])
def test_apply_entries_at_copy_chunk_edges(side, scale, step):
    """Run-by-run copy where the cuts sit on the copy workgroups' chunk edges
    (1024 positions of the new index array on a graph under 2M edges): the
    batch inserts the edges that end up at positions q-1 and q of every
    step-th position q (and the first and last positions) of the out- or
    in-CSR, and deletes, at every other such q, an extra edge that sorts just
    before position q, so a deletion's cut, an empty run and an insertion meet
    there.  Cuts every 1024 positions make short runs (under 4096 on average:
    one wavefront per run); every 16384, long ones (runs walked per chunk).
    Caller ids are kept, so the positions are those of the canonical CSR."""
    torch_cuda()
    n, s, d = rmat(scale, seed=91)
    full = O.graph(n, s, d)  # the graph after the batch
    m = full.m
    off, idx = (full.out_off, full.out_idx) if side == "out" else (full.in_off, full.in_idx)
    row_of = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    edges = list(range(step, m, step))
    pos = sorted({p for q in edges + [0, m - 1] for p in (q - 1, q) if 0 <= p < m and row_of[p] != idx[p]})
    extra = []
    for q in edges[::2]:
        r = int(row_of[q])
        lo = int(idx[q - 1]) + 1 if row_of[q - 1] == r else 0
        cand = [c for c in range(lo, int(idx[q])) if c != r]
        if cand:
            extra.append((r, cand[0]))
    assert len(extra) > len(edges) // 4
    keep = np.ones(m, bool)
    keep[pos] = False
    rows = np.concatenate([row_of[keep], [r for r, _ in extra]]).astype(np.int32)
    cols = np.concatenate([idx[keep], [c for _, c in extra]]).astype(np.int32)
    xr = np.array([r for r, _ in extra], np.int32)
    xc = np.array([c for _, c in extra], np.int32)
    if side == "out":
        src, dst, ins_src, ins_dst, del_src, del_dst = rows, cols, row_of[pos], idx[pos], xr, xc
    else:
        src, dst, ins_src, ins_dst, del_src, del_dst = cols, rows, idx[pos], row_of[pos], xc, xr
    p = Pair(n, src, dst, keep_ids=True)
    assert len(pos) + len(extra) <= p.og.m // 256  # the run-by-run copy
    assert (p.og.m < 4096 * (len(pos) + len(extra))) == (step == 1024)  # short runs, or long ones
    _print("chunk edges", side, scale, step, len(pos), len(extra), p.og.m)
    info = p.apply(del_src, del_dst, ins_src.astype(np.int32), ins_dst.astype(np.int32))
    assert info["ins_effective"] == len(pos) and info["del_effective"] == len(extra)
    assert_csr_equal(p.g, p.og)
    assert np.array_equal(p.og.out_idx, full.out_idx) and np.array_equal(p.og.in_idx, full.in_idx)


@pytest.mark.parametrize("k", [63, 64, 65])
def test_apply_group_entries_at_lane_count(k):
    """Merge of touched groups: rows 0..63 (one group; caller ids kept inside)
    get exactly 63, 64 or 65 effective entries, a third of them deletions; up
    to 63 are held in the lanes, from 64 on they are searched in memory.  The
    rest of the batch (rows >= 64) makes it large enough for the merge path."""
    torch_cuda()
    n, s, d = rmat(12, seed=63)
    p = Pair(n, s, d, keep_ids=True)
    og = p.og
    rng = np.random.default_rng(64)
    in_group = np.flatnonzero((og.esrc < 64) & (og.esrc != og.edst))
    dels = rng.choice(in_group, k // 3, replace=False)
    taken = set()
    ins = _pairs_not_in(rng, og, k - k // 3, (0, 64), (0, n), taken)
    pad = _pairs_not_in(rng, og, og.m // 256 + 1, (64, n), (0, n), taken)
    ins_src = np.array([u for u, _ in ins + pad], np.int32)
    ins_dst = np.array([v for _, v in ins + pad], np.int32)
    _print("group entries", k, len(ins_src) + len(dels), og.m)
    info = p.apply(og.esrc[dels], og.edst[dels], ins_src, ins_dst)
    assert info["ins_effective"] == len(ins_src) and info["del_effective"] == len(dels)
    assert_csr_equal(p.g, p.og)


# ------------------------------------------------------------------ ranks
def _setup(scale=12, frac=1e-3, seed=1, ef=16, keep_ids=False):
    n, s, d = rmat(scale, ef=ef, seed=seed)
    p = Pair(n, s, d, keep_ids=keep_ids)
    r0 = O.rank("static", p.og).ranks
    ds, dd, is_, id_ = W.batch_8020(n, s, d, frac, seed=seed + 100)
    p.apply(ds, dd, is_, id_)
    return p, r0


@pytest.mark.parametrize("keep_ids", [False, True])
@pytest.mark.parametrize("mode", ["static", "nd", "df", "dfp"])
@pytest.mark.parametrize("scale,frac", [(10, 1e-2), (14, 1e-3)])
def test_ranks_parity(mode, scale, frac, keep_ids):
    p, r0 = _setup(scale, frac, seed=scale, keep_ids=keep_ids)
    _print("ranks", mode, scale, frac)
    r, st, ref = p.rank(mode, r0)
    err = float(np.abs(r - ref.ranks).max())
    _print(f"  linf={err:.3e} it gpu={st['iterations']} oracle={ref.iterations} "
           f"ever gpu={st['ever_affected']} oracle={ref.ever_affected}")
    assert err <= LINF
    assert st["converged"] == ref.converged == 1
    assert abs(st["iterations"] - ref.iterations) <= 1
    assert (r >= (1 - 0.85) / p.n).all()


@pytest.mark.parametrize("fused", [False, True])
def test_dense_form_long_runs(fused):
    """A long dense run (the dense form copies an unprocessed vertex over only
    when the previous iteration processed it, by the iteration stamps it keeps
    in the ever array, 254 values in turn): with a rank tolerance of 1e-300 and
    frontier and prune thresholds near the rounding level, DF-P runs until its
    frontier dies out or for 300 iterations, pruning and re-marking vertices
    all along; the dense form (in one launch, or per iteration) gives the
    frontier form's bits and statistics."""
    torch = torch_cuda()
    p, r0 = _setup(11, 1e-2, seed=93)
    kw = dict(tol=1e-300, max_iters=300, frontier_tol=1e-15, prune_tol=1e-15)
    outs = {}
    for sw in (float("inf"), 0.0):
        p2 = Pair(p.n, p.og_prev.esrc, p.og_prev.edst, fused=fused and sw != 0.0)
        p2.apply(p.batch.dm_src, p.batch.dm_dst, p.batch.dp_src, p.batch.dp_dst)
        rp = torch.from_numpy(np.ascontiguousarray(r0)).cuda()
        r, st = p2.g.update_ranks("dfp", rp, dense_switch=sw, **kw)
        outs[sw] = (r.cpu().numpy(), st)
    (rd, sd), (rf, sf) = outs[float("inf")], outs[0.0]
    _print("long runs: iterations", sd["iterations"], "ever", sd["ever_affected"], "updates", sd["vertex_updates"])
    assert sd["iterations"] == sf["iterations"] >= 100
    for key in ("ever_affected", "vertex_updates", "edges_pulled"):
        assert sd[key] == sf[key], key
    assert np.array_equal(rd, rf)


@pytest.mark.parametrize("frac", [1e-3, 1e-1])
@pytest.mark.parametrize("mode", ["df", "dfp"])
def test_dense_and_frontier_forms_agree(mode, frac):
    """The dense form (every vertex reads its in-neighbours' expand flags) and the
    frontier form (marks pushed to out-neighbours) give bit-identical ranks and
    frontier statistics, and both match the oracle; the default switches between
    them by the cost rule (dense_switch: infinity always dense, 0 never)."""
    torch = torch_cuda()
    p, r0 = _setup(13, frac, seed=91)
    outs = {}
    inf = float("inf")
    for sw in (inf, 1.0, 0.0):
        p2 = Pair(p.n, p.og_prev.esrc, p.og_prev.edst)
        p2.apply(p.batch.dm_src, p.batch.dm_dst, p.batch.dp_src, p.batch.dp_dst)
        r, st, ref = p2.rank(mode, r0, dense_switch=sw)
        outs[sw] = (r, st)
        assert np.abs(r - ref.ranks).max() <= LINF
        assert abs(st["iterations"] - ref.iterations) <= 1
    for key in ("iterations", "ever_affected", "vertex_updates", "edges_pulled"):
        assert outs[inf][1][key] == outs[1.0][1][key] == outs[0.0][1][key], key
    assert outs[inf][1]["dense_iterations"] == outs[inf][1]["iterations"]
    assert outs[0.0][1]["dense_iterations"] == 0
    assert np.array_equal(outs[inf][0], outs[0.0][0]) and np.array_equal(outs[1.0][0], outs[0.0][0])


@pytest.mark.parametrize("mode", ["df", "dfp"])
def test_hub_frontier_stays_in_frontier_form(mode):
    """A preferential-attachment graph whose batch reaches a few hubs (many
    in-edges, few out-edges): the default keeps such a frontier in the frontier
    form (its expanding vertices have few out-edges to mark, while the dense
    form would scan the flags of almost every in-edge); forcing the dense form
    gives the same bits and statistics, and both match the oracle."""
    torch_cuda()
    n = 20000
    src, dst = W.temporal_stream(n, 400000, seed=93)
    k0 = 360000
    s0, d0 = W.dedupe(n, src[:k0], dst[:k0])
    outs = {}
    inf = float("inf")
    for sw in (1.0, inf):
        p = Pair(n, s0, d0)
        r0 = O.rank("static", p.og).ranks
        p.apply([], [], src[k0:k0 + 400], dst[k0:k0 + 400])
        r, st, ref = p.rank(mode, r0, dense_switch=sw)
        assert np.abs(r - ref.ranks).max() <= LINF
        assert st["ever_affected"] == ref.ever_affected
        outs[sw] = (r, st)
    _print(f"hub frontier {mode}: dense iterations {outs[1.0][1]['dense_iterations']} of "
           f"{outs[1.0][1]['iterations']} (default), edges pulled {outs[1.0][1]['edges_pulled']}")
    assert outs[1.0][1]["dense_iterations"] < outs[1.0][1]["iterations"]
    assert outs[inf][1]["dense_iterations"] == outs[inf][1]["iterations"]
    for key in ("iterations", "ever_affected", "vertex_updates", "edges_pulled"):
        assert outs[1.0][1][key] == outs[inf][1][key], key
    assert np.array_equal(outs[1.0][0], outs[inf][0])


@pytest.mark.parametrize("mode", ["static", "nd", "df", "dfp"])
def test_ranks_bitexact_lane_bin(mode):
    """With every vertex in the one-lane bin the sums run in the oracle's order:
    ranks, iteration counts and frontier statistics are identical."""
    p, r0 = _setup(13, 1e-3, seed=21, keep_ids=True)
    maxdeg = int(np.diff(p.og.in_off).max())
    p.g.set_tuning([maxdeg] * 5)
    r, st, ref = p.rank(mode, r0)
    assert np.array_equal(r, ref.ranks)
    assert st["iterations"] == ref.iterations
    assert st["vertex_updates"] == ref.vertex_updates
    assert st["edges_pulled"] == ref.edges_pulled
    assert st["ever_affected"] == ref.ever_affected


@pytest.mark.parametrize("bounds", [[1, 2, 3, 4, 5], [1, 1, 1, 2, 3], [2, 4, 8, 16, 32]])
@pytest.mark.parametrize("mode", ["static", "dfp", "df"])
def test_all_bins(mode, bounds):
    """Small thresholds push vertices into every bin, the chunked one included."""
    p, r0 = _setup(12, 1e-2, seed=31)
    p.g.set_tuning(bounds)
    assert p.g.get_tuning() == bounds
    r, st, ref = p.rank(mode, r0, dense_switch=0.0)  # frontier form: the worklist bins are used
    assert np.abs(r - ref.ranks).max() <= LINF
    assert st["bin_vertices"][5] > 0 and st["bin_vertices"][3] > 0
    if mode != "static":
        p, r0 = _setup(12, 1e-2, seed=31)  # the update consumed the batch marks: same batch again
        p.g.set_tuning(bounds)
        r2, st2, _ = p.rank(mode, r0, dense_switch=float("inf"))  # dense form over the all-vertex bins
        assert np.array_equal(r, r2) and st2["dense_iterations"] == st2["iterations"]


@pytest.mark.parametrize("mode", ["static", "df", "dfp"])
def test_hub_graph_ranks(mode):
    """A vertex with thousands of in- and out-edges: chunked pull (several
    chunks per row) and chunked marking of its out-row."""
    n, s, d = hub_graph(30000, 9000, 12000, 90000, seed=41)
    p = Pair(n, s, d)
    r0 = O.rank("static", p.og).ranks
    p.apply([], [], [0, 5], [77, 0])  # touches the hub as a source and as a target
    r, st, ref = p.rank(mode, r0)
    assert np.abs(r - ref.ranks).max() <= LINF
    if mode != "static":
        assert st["ever_affected"] == ref.ever_affected


def test_autotune_keeps_parity():
    p, r0 = _setup(13, 1e-3, seed=97)
    bounds, ms = p.g.autotune()
    assert bounds == p.g.get_tuning() and ms > 0
    assert bounds[0] >= 1 and all(bounds[i] <= bounds[i + 1] for i in range(4))
    r, st, ref = p.rank("dfp", r0)  # the pending marks of the batch survived tuning
    assert np.abs(r - ref.ranks).max() <= LINF
    assert st["ever_affected"] == ref.ever_affected


def test_empty_and_noop_batches():
    n, s, d = rmat(10, seed=51)
    p = Pair(n, s, d)
    r0b = O.rank("static", p.og).ranks
    ex = (p.og.esrc[p.og.esrc != p.og.edst][:3], p.og.edst[p.og.esrc != p.og.edst][:3])
    p.apply([4, 4], [4, 4], ex[0], ex[1])  # self-loop deletes + existing inserts
    assert len(p.batch.dm_src) == 0 and len(p.batch.dp_src) == 0
    for mode in ("df", "dfp"):
        r, st, ref = p.rank(mode, r0b)
        assert st["iterations"] == 1 and st["converged"] == 1 and st["ever_affected"] == 0
        assert np.array_equal(r, r0b)
    # marks accumulate over applies until the next DF/DF-P update consumes them
    have = set(zip(p.og.esrc.tolist(), p.og.edst.tolist()))
    u, v = next((a, b) for a in range(n) for b in range(n) if a != b and (a, b) not in have)
    p.apply([], [], [u], [v])
    r, st, ref = p.rank("dfp", r0b)
    assert st["ever_affected"] == ref.ever_affected > 0
    r, st, _ = p.rank("dfp", r0b)
    assert st["ever_affected"] == 0 and np.array_equal(r, r0b)


def test_rank_alias_and_determinism():
    torch = torch_cuda()
    p, r0 = _setup(12, 1e-3, seed=61)
    p.g.update_ranks("static")  # a full solve discards the setup batch's pending marks
    outs = []
    for _ in range(2):
        p.apply(*W.batch_8020(p.n, p.og.esrc[p.og.esrc != p.og.edst], p.og.edst[p.og.esrc != p.og.edst], 1e-3,
                              seed=62))
        p.apply(p.batch.dp_src, p.batch.dp_dst, p.batch.dm_src, p.batch.dm_dst)  # back to the same graph
        p.apply(*W.batch_8020(p.n, p.og.esrc[p.og.esrc != p.og.edst], p.og.edst[p.og.esrc != p.og.edst], 1e-3,
                              seed=62))
        rp = torch.from_numpy(r0.copy()).cuda()
        r, st = p.g.update_ranks("dfp", rp, out=rp)  # r_out aliases r_prev
        torch.cuda.synchronize()
        outs.append((r.cpu().numpy().copy(), st["iterations"], st["ever_affected"]))
        p.apply(p.batch.dp_src, p.batch.dp_dst, p.batch.dm_src, p.batch.dm_dst)
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]


def test_errors_leave_graph_unchanged():
    torch = torch_cuda()
    import paper_2401_15870_amd as dfpr
    p, r0 = _setup(10, 1e-2, seed=71)
    with pytest.raises(dfpr.DfprError) as e:
        p.g.apply_batch([0, 1], [2, p.n], [], [])
    assert e.value.code == -2
    assert_csr_equal(p.g, p.og)
    rp = torch.from_numpy(r0).cuda()
    with pytest.raises(dfpr.DfprError) as e:
        p.g.update_ranks("dfp", rp, alpha=1.5)
    assert e.value.code == -1
    with pytest.raises(dfpr.DfprError):
        p.g.set_tuning([10, 5, 20, 30, 40])
    # the pending marks survived the failed calls: DF-P still matches the oracle
    r, st, ref = p.rank("dfp", r0)
    assert np.abs(r - ref.ranks).max() <= LINF
    # iteration cap is not an error
    r, st, ref = p.rank("static", None, max_iters=3)
    assert st["converged"] == 0 and st["iterations"] == 3 == ref.iterations
    assert np.abs(r - ref.ranks).max() <= LINF


def test_temporal_chain():
    """Insertion-only batches replayed in time order, each step from the
    oracle's previous ranks (many inserts are repeats: no-ops)."""
    torch_cuda()
    src, dst = W.temporal_stream(4000, 60000, seed=81)
    n = 4000
    k0 = int(0.9 * len(src))
    p = Pair(n, src[:k0], dst[:k0])
    r = O.rank("static", p.og).ranks
    B = (len(src) - k0) // 5
    for i in range(5):
        lo = k0 + i * B
        p.apply([], [], src[lo:lo + B], dst[lo:lo + B])
        assert_csr_equal(p.g, p.og)
        gr, st, ref = p.rank("dfp", r)
        assert np.abs(gr - ref.ranks).max() <= LINF
        r = ref.ranks


# ------------------------------------------------------------------ single-launch loop
def _fused_pair_case(case):
    if case == "rmat12":
        return rmat(12, seed=21)
    if case == "rmat14":
        return rmat(14, seed=22)
    if case == "hub":
        return hub_graph(20000, 9000, 12000, 60000, seed=23)
    if case == "tiny":
        s, d = W.random_digraph(40, 0.1, seed=24)
        return 40, s, d
    return 1, np.zeros(0, np.int32), np.zeros(0, np.int32)


@pytest.mark.parametrize("bounds", [None, [1, 2, 3, 4, 5]])
@pytest.mark.parametrize("mode", ["static", "nd", "df", "dfp"])
@pytest.mark.parametrize("case", ["rmat12", "rmat14", "hub", "tiny", "single"])
def test_fused_loop_matches_launch_loop(case, mode, bounds):
    """One cooperative launch per update gives the same bits as the
    launch-per-iteration loop (same kernels, same work split), and the oracle's
    ranks within the bar."""
    torch_cuda()
    n, s, d = _fused_pair_case(case)
    res = []
    for fused in (False, True):
        p = Pair(n, s, d, fused=fused)
        if bounds:
            p.g.set_tuning(bounds)
        r0 = O.rank("static", p.og).ranks
        if len(s):
            ds, dd, is_, id_ = W.batch_8020(n, s, d, 2e-3, seed=25)
        else:
            ds = dd = np.zeros(0, np.int32)
            is_ = id_ = np.zeros(0, np.int32)
        p.apply(ds, dd, is_, id_)
        r, st, ref = p.rank(mode, None if mode == "static" else r0)
        assert np.abs(r - ref.ranks).max() <= LINF
        res.append((r, st))
    (r1, s1), (r2, s2) = res
    assert np.array_equal(r1, r2), float(np.abs(r1 - r2).max())
    for k in ("iterations", "converged", "last_delta", "ever_affected", "vertex_updates", "edges_pulled"):
        assert s1[k] == s2[k], (k, s1[k], s2[k])
    assert s2["pull_launches"] == 1


def test_single_launch_bins_after_failed_and_chained_applies():
    """Single-launch updates after a batch rejected once its rebuild had run
    (the cached all-vertex bins must be those of the unchanged graph) and
    after two applies in a row (those of the last graph).  Thresholds
    [1, 2, 3, 4, 5] put most vertices in the chunked bin, so the bins of two
    graphs differ."""
    torch_cuda()
    import paper_2401_15870_amd as dfpr
    n, s, d = rmat(12, seed=27)
    p = Pair(n, s, d, fused=True)
    p.g.set_tuning([1, 2, 3, 4, 5])
    r0 = O.rank("static", p.og).ranks
    p.apply(*W.batch_8020(n, s, d, 1e-2, seed=28))
    with pytest.raises(dfpr.DfprError) as e:
        p.g.apply_batch([0, 1], [2, n], [5, 6], [7, 8])
    assert e.value.code == -2
    assert_csr_equal(p.g, p.og)
    r, st, ref = p.rank("dfp", r0)
    assert np.abs(r - ref.ranks).max() <= LINF
    assert st["pull_launches"] == 1
    p.apply(*W.batch_8020(n, s, d, 1e-2, seed=29))
    p.apply(*W.batch_8020(n, s, d, 3e-2, seed=30))
    assert_csr_equal(p.g, p.og)
    r, st, ref = p.rank("static", None)
    assert np.abs(r - ref.ranks).max() <= LINF
    assert st["pull_launches"] == 1 and st["iterations"] == ref.iterations


@pytest.mark.parametrize("mode", ["static", "dfp"])
def test_fused_loop_iteration_cap(mode):
    """Stopping at max_iters (not converged) happens at the same iteration on both paths."""
    torch_cuda()
    n, s, d = rmat(12, seed=26)
    out = []
    for fused in (False, True):
        p = Pair(n, s, d, fused=fused)
        r0 = O.rank("static", p.og).ranks
        ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-2, seed=27)
        p.apply(ds, dd, is_, id_)
        r, st, ref = p.rank(mode, None if mode == "static" else r0, max_iters=3)
        assert st["iterations"] == ref.iterations == 3 and st["converged"] == ref.converged == 0
        assert np.abs(r - ref.ranks).max() <= LINF
        out.append(r)
    assert np.array_equal(out[0], out[1])


def test_library_loaded_before_torch_initialises():
    """A fresh process that loads the library before torch has touched the GPU
    still finds the device (one HIP runtime per process)."""
    import subprocess
    import sys
    import os
    code = ("import numpy as np, paper_2401_15870_amd as m; m.lib(); "
            "g = m.Graph.from_coo(4, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32)); "
            "print('edges', g.m)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "edges 7" in out.stdout


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("mode", ["df", "dfp"])
@pytest.mark.parametrize("criterion,tf", [("absolute", 1e-12), ("contrib", 1e-13), ("relative", 1e-6)])
def test_frontier_criteria(criterion, tf, mode, fused):
    """The three change measures of Section 4.2 against the oracle (the
    tolerances of the absolute measures sit in the range the paper sweeps)."""
    torch_cuda()
    n, s, d = rmat(12, seed=41)
    p = Pair(n, s, d, fused=fused)
    r0 = O.rank("static", p.og).ranks
    ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-3, seed=42)
    p.apply(ds, dd, is_, id_)
    r, st, ref = p.rank(mode, r0, criterion=criterion, frontier_tol=tf, prune_tol=tf)
    err = float(np.abs(r - ref.ranks).max())
    _print(f"criterion {criterion} tf {tf:g} {mode} fused={fused}: linf {err:.2e} it {st['iterations']}/"
           f"{ref.iterations} ever {st['ever_affected']}/{ref.ever_affected}")
    assert err <= LINF
    assert st["ever_affected"] == ref.ever_affected
    assert abs(st["iterations"] - ref.iterations) <= 1


def _eq1_residual_l1(og, x, alpha=0.85):
    """||x - F(x)||_1 with F(x)_v = (1 - alpha)/N + alpha * sum_{u in in(v)} x_u/|out(u)|
    (Equation 1 applied to every vertex of G^t)."""
    n = og.n
    dout = np.diff(og.out_off).astype(np.float64)
    contrib = x / dout
    rows = np.repeat(np.arange(n), np.diff(og.in_off))
    fx = (1 - alpha) / n + alpha * np.bincount(rows, weights=contrib[og.in_idx], minlength=n)
    return float(np.abs(x - fx).sum())


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("mode", ["df", "dfp"])
def test_asynchronous_mode(mode, fused):
    """In-place (asynchronous) DF/DF-P (Section 4.4: one rank vector, vertices
    processed later in an iteration read the values already updated in it).
    The result depends on the device's execution order, so it is accepted by a
    bound that holds for every processing order, not by parity.

    Bound (stated before any run).  P^T is column-stochastic, so
    ||(I - alpha P^T)^-1||_1 <= 1/(1 - alpha) and, for any vector x,
    ||x - r*||_1 <= ||x - F(x)||_1 / (1 - alpha), F being Equation 1 on G^t and
    r* its fixed point.  With pruning off and expansion on every change
    (tau_p = -1, tau_f = 0; Equation 2 also leaves a processed vertex at its
    Equation-1 value for the in-neighbour values it read) every vertex whose
    in-neighbours changed is processed again, so at the stop the residual comes
    from (a) the changes of the last iteration, each at most tau, weighted by
    alpha and column sums of 1: at most alpha*N*tau in L1, whatever the order;
    and (b) the vertices never processed, which keep R_prev, a Static solve of
    G^{t-1} stopped at tau: again at most alpha*N*tau.  So both the synchronous
    and the asynchronous result must satisfy ||x - F(x)||_1 <= 2 alpha N tau
    and ||x - r*||_1 <= 2 alpha N tau / (1 - alpha).

    At the default tau_f = tau_p = 1e-6 the pruning error is not bounded by tau
    (for either execution), so there the test checks convergence and the
    exact lower bound x >= (1 - alpha)/N, and reports the iteration counts and
    errors of both executions as data."""
    torch_cuda()
    alpha, tau = 0.85, 1e-10
    n, s, d = rmat(14, seed=51)
    p = Pair(n, s, d, fused=fused)
    r0 = O.rank("static", p.og).ranks
    ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-3, seed=52)
    p.apply(ds, dd, is_, id_)
    exact = O.rank("static", p.og, tol=1e-15, max_iters=500).ranks
    res_bound = 2 * alpha * n * tau
    ra, sta, ref = p.rank(mode, r0, asynchronous=True, frontier_tol=0.0, prune_tol=-1.0)
    for name, x, st in (("async", ra, sta), ("sync oracle", ref.ranks, {"converged": ref.converged})):
        res = _eq1_residual_l1(p.og, x, alpha)
        err = float(np.abs(x - exact).sum())
        _print(f"async test {mode} fused={fused} no pruning, {name}: residual L1 {res:.2e} (bound {res_bound:.2e}), "
               f"error L1 {err:.2e} (bound {res_bound / (1 - alpha):.2e})")
        assert st["converged"] == 1
        assert res <= res_bound
        assert err <= res_bound / (1 - alpha)
        assert x.min() >= (1 - alpha) / n
    _print(f"  iterations no pruning: async {sta['iterations']}, sync {ref.iterations}")
    # default thresholds: convergence, lower bound, data
    ra, sta, ref = p.rank(mode, r0, asynchronous=True)
    e_async = float(np.abs(ra - exact).max())
    e_sync = float(np.abs(ref.ranks - exact).max())
    _print(f"  defaults: iterations async {sta['iterations']} sync {ref.iterations}; linf vs r* async {e_async:.2e} "
           f"sync {e_sync:.2e}; async vs sync {float(np.abs(ra - ref.ranks).max()):.2e}")
    assert sta["converged"] == 1
    assert ra.min() >= (1 - alpha) / n
