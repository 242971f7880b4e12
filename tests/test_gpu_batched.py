"""Batched form: many graphs in one arena, updated together.  Every member must
equal its plain-handle result (bit-exact with the same thresholds and create
flags; the members converge on their own) and the oracle's (L-inf 1e-9)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import LINF, assert_info_equal, dfpr, rmat, torch_cuda

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _members(seed):
    """Mixed sizes, including the degenerate ones (one vertex, no edges)."""
    rng = np.random.default_rng(seed)
    out = [(1, np.zeros(0, np.int32), np.zeros(0, np.int32)),
           (23, np.zeros(0, np.int32), np.zeros(0, np.int32))]
    for k, scale in enumerate((8, 11, 9, 12, 10)):
        out.append(rmat(scale, ef=float(rng.uniform(8, 32)), seed=seed * 10 + k))
    n = 700
    s, d = W.random_digraph(n, 0.01, seed=seed)
    out.append((n, s, d))
    return out


def _member_csr(off, idx, base, n):
    o = off[base: base + n + 1].astype(np.int64)
    return (o - o[0]).astype(np.int32), (idx[o[0]: o[-1]] - base).astype(np.int32)


class Batched:
    """A batch handle, a plain handle per member and an oracle graph per member."""

    def __init__(self, members, keep_ids=False, fused=True):
        """fused=False runs the batch handle's updates on the launch-per-iteration
        loop instead of its default single launch (both give the same bits)."""
        m = dfpr()
        self.members = members
        self.bg = m.BatchGraph.from_coo(members, keep_ids=keep_ids)
        if not fused:
            self.bg.set_fused_limit(0)
        self.plain = [m.Graph.from_coo(n, s, d, keep_ids=keep_ids) for n, s, d in members]
        self.og = [O.graph(n, s, d) for n, s, d in members]
        self.og_prev = [None] * len(members)
        self.ob = [None] * len(members)

    def check_csr(self):
        for in_csr in (False, True):
            off, idx = self.bg.export(in_csr=in_csr)
            for k, og in enumerate(self.og):
                mo, mi = _member_csr(off, idx, self.bg.bases[k], self.bg.sizes[k])
                ref_off, ref_idx = (og.in_off, og.in_idx) if in_csr else (og.out_off, og.out_idx)
                assert np.array_equal(mo, ref_off) and np.array_equal(mi, ref_idx), (k, in_csr)

    def apply(self, batches, device=False):
        torch = torch_cuda()
        if device:
            batches = [tuple(torch.as_tensor(np.asarray(a, np.int32)).cuda() for a in b) for b in batches]
        infos = self.bg.apply_batch_many(batches)
        for k, b in enumerate(batches):
            pinfo = self.plain[k].apply_batch(*b)
            og2, ob = O.apply(self.og[k], *[np.asarray(a.cpu() if hasattr(a, "cpu") else a) for a in b])
            assert_info_equal(infos[k], ob)
            assert_info_equal(pinfo, ob)
            assert infos[k]["m_after"] == og2.m == pinfo["m_after"]
            self.og_prev[k], self.og[k], self.ob[k] = self.og[k], og2, ob
        return infos

    def arena(self, parts):
        return np.concatenate([np.asarray(p, np.float64) for p in parts])

    def rank(self, mode, r_prev_parts, oracle=True, **kw):
        torch = torch_cuda()
        rp = None
        if r_prev_parts is not None:
            rp = torch.from_numpy(self.arena(r_prev_parts)).cuda()
        r, tot, per = self.bg.update_ranks_many(mode, rp, **kw)
        torch.cuda.synchronize()
        r = r.cpu().numpy()
        results = []
        for k, (n, _, _) in enumerate(self.members):
            rpk = None if r_prev_parts is None else torch.from_numpy(np.asarray(r_prev_parts[k], np.float64)).cuda()
            rk, stk = self.plain[k].update_ranks(mode, rpk, **kw)
            rk = rk.cpu().numpy()
            mine = self.bg.member(r, k)
            assert np.array_equal(mine, rk), (mode, k, float(np.abs(mine - rk).max()))
            assert per[k]["iterations"] == stk["iterations"], (k, per[k], stk)
            assert per[k]["converged"] == stk["converged"]
            assert per[k]["last_delta"] == stk["last_delta"]
            assert per[k]["ever_affected"] == stk["ever_affected"], (k, per[k]["ever_affected"], stk["ever_affected"])
            if oracle:
                okw = {k2: v for k2, v in kw.items() if k2 in ("alpha", "tol", "max_iters")}
                rpo = None if r_prev_parts is None else np.asarray(r_prev_parts[k], np.float64)
                if mode in ("df", "dfp"):
                    ref = O.rank(mode, self.og[k], rpo, self.og_prev[k], self.ob[k], **okw)
                else:
                    ref = O.rank(mode, self.og[k], rpo, **okw)
                err = float(np.abs(mine - ref.ranks).max())
                assert err <= LINF, (mode, k, err)
                assert abs(per[k]["iterations"] - ref.iterations) <= 1
            results.append(mine.copy())
        assert tot["iterations"] == max(p["iterations"] for p in per)
        assert tot["converged"] == int(all(p["converged"] for p in per))
        assert tot["ever_affected"] == sum(p["ever_affected"] for p in per)
        return results, tot, per


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("keep_ids", [False, True])
def test_batched_create_csr_and_static(keep_ids, fused):
    torch_cuda()
    b = Batched(_members(1), keep_ids=keep_ids, fused=fused)
    _print("batched create", [m[0] for m in b.members])
    assert b.bg.count == len(b.members)
    assert b.bg.sizes == [m[0] for m in b.members]
    b.check_csr()
    parts, tot, per = b.rank("static", None)
    its = [p["iterations"] for p in per]
    _print("  static iterations per member", its)
    assert len(set(its)) > 1  # members really converge at different iterations


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("keep_ids", [False, True])
@pytest.mark.parametrize("mode", ["nd", "df", "dfp"])
def test_batched_update_matches_plain(mode, keep_ids, fused):
    torch_cuda()
    members = _members(2)
    b = Batched(members, keep_ids=keep_ids, fused=fused)
    r0 = [O.rank("static", og).ranks for og in b.og]
    rng = np.random.default_rng(5)
    batches = []
    for k, (n, s, d) in enumerate(members):
        frac = float(np.exp(rng.uniform(np.log(1e-3), np.log(5e-2))))
        if k == 3:  # one member with an empty batch
            batches.append((np.zeros(0, np.int32),) * 4)
        else:
            batches.append(W.batch_8020(n, s, d, frac, seed=100 + k) if len(s) else
                           W.random_edit_batch(n, s, d, 5, 2, seed=100 + k))
    b.apply(batches)
    b.check_csr()
    _print("batched", mode, "members", len(members))
    b.rank(mode, r0)


@pytest.mark.parametrize("dense_switch", [float("inf"), 0.0])
def test_batched_dense_and_frontier_forms(dense_switch):
    torch_cuda()
    members = _members(3)
    b = Batched(members, fused=False)  # the per-iteration loop, where the two forms are chosen
    r0 = [O.rank("static", og).ranks for og in b.og]
    batches = [W.batch_8020(n, s, d, 1e-2, seed=200 + k) if len(s) else (np.zeros(0, np.int32),) * 4
               for k, (n, s, d) in enumerate(members)]
    b.apply(batches, device=True)
    _print("batched dense_switch", dense_switch)
    b.rank("dfp", r0, oracle=False, dense_switch=dense_switch)


def test_batched_chained_updates_and_timing():
    torch_cuda()
    members = [rmat(s, seed=40 + s) for s in (9, 10, 11, 12)]
    b = Batched(members)
    r = [O.rank("static", og).ranks for og in b.og]
    for step in range(3):
        batches = [W.random_edit_batch(n, og.esrc, og.edst, 40, 10, seed=step * 10 + k)
                   for k, ((n, _, _), og) in enumerate(zip(members, b.og))]
        b.apply(batches, device=bool(step % 2))
        _print("chained step", step)
        r, tot, per = b.rank("dfp", r, timing=(step == 1))
        if step == 1:
            assert tot["ms_total"] > 0


def test_batched_many_small_graphs():
    """Hundreds of tiny members: the arena path with a long member table."""
    torch_cuda()
    rng = np.random.default_rng(9)
    members = []
    for k in range(300):
        n = int(rng.integers(1, 60))
        s, d = W.random_digraph(n, float(rng.uniform(0.02, 0.3)), seed=1000 + k)
        members.append((n, s, d))
    b = Batched(members)
    b.check_csr()
    r0 = [O.rank("static", og).ranks for og in b.og]
    batches = [W.random_edit_batch(n, s, d, 3, 2, seed=2000 + k) for k, (n, s, d) in enumerate(members)]
    b.apply(batches)
    _print("many small: members", len(members))
    b.rank("dfp", r0)
    b.rank("df", r0, oracle=False)


def test_batched_errors():
    torch_cuda()
    m = dfpr()
    members = _members(4)[:4]
    b = Batched(members)
    off0, idx0 = b.bg.export()
    bad = [(np.zeros(0, np.int32),) * 4 for _ in members]
    n3 = members[3][0]
    bad[3] = (np.zeros(0, np.int32), np.zeros(0, np.int32), np.array([0], np.int32), np.array([n3], np.int32))
    with pytest.raises(m.DfprError) as e:
        b.bg.apply_batch_many(bad)
    assert e.value.code == -2  # ERANGE: an id beyond its member, even though the arena has room
    off1, idx1 = b.bg.export()
    assert np.array_equal(off0, off1) and np.array_equal(idx0, idx1)
    with pytest.raises(m.DfprError) as e:
        b.bg.apply_batch([0], [1], [], [])
    assert e.value.code == -1  # the plain apply is refused on a batch handle
    with pytest.raises(m.DfprError) as e:
        m.BatchGraph.from_coo([(3, np.array([0], np.int32), np.array([5], np.int32))])
    assert e.value.code == -2
