"""Parity at the full sizes of the benchmark configurations, in the launch
configuration the benchmark times (autotuned thresholds): CSRs compared in full,
ranks compared in full against the oracle run from the same previous ranks.

  * one large R-MAT graph: scale 24, edge factor 16: Static, then one 80/20
    batch applied to the initial graph at 1e-7, 1e-5, 1e-4, 1e-3 and 1e-1 |E|
    (DF-P) and at 1e-4 |E| (DF, ND), each from the oracle's Static ranks;
  * the temporal stream: 2M vertices, 40M edges, first 90 % as the initial
    graph, insertion-only batches of 40,000 in time order (first three);
  * the small-graph configuration: R-MAT scale 14, batches of 1e-3|E| each
    applied to the same initial graph from the same ranks (Static, ND, DF, DF-P);
  * the batched configuration's member distribution (64 of its graphs): every
    member bit-identical to its plain-handle result and within the parity bar
    of the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import LINF, Pair, assert_csr_equal, dfpr, torch_cuda

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _print(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rmat24():
    """The scale-24 graph on the host and its oracle Static ranks (shared by the
    scale-24 cases; each case builds its own device graph and applies its batch
    to this initial graph)."""
    n, s, d = W.rmat_graph(24, 16, seed=1)
    _print("rmat24: n", n, "edges", len(s))
    og = O.graph(n, s, d)
    ref0 = O.rank("static", og)
    return n, s, d, og, ref0


def _device_pair(n, s, d, og):
    torch = torch_cuda()
    p = Pair.__new__(Pair)
    p.dfpr, p.og, p.og_prev, p.batch, p.n, p.kw = dfpr(), og, None, None, n, {}
    p.g = p.dfpr.Graph.from_coo(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return p


def test_fullsize_rmat24_static(rmat24):
    n, s, d, og, ref0 = rmat24
    p = _device_pair(n, s, d, og)
    assert_csr_equal(p.g, p.og)
    bounds, _ = p.g.autotune()
    _print("  autotuned", bounds)
    r_gpu, st, _ = p.rank("static", None)
    err0 = float(np.abs(r_gpu - ref0.ranks).max())
    _print("  static linf", err0, "it", st["iterations"], ref0.iterations)
    assert err0 <= LINF and st["iterations"] == ref0.iterations
    p.g.close()


# DF-P across the batch sizes of the random-batch experiment (Section 5.2.2):
# small batches run the frontier form, large ones the dense form, so both sides
# of the switch are compared at full size; DF and ND at the default batch size.
@pytest.mark.parametrize("mode,frac", [("dfp", 1e-7), ("dfp", 1e-5), ("dfp", 1e-4), ("dfp", 1e-3), ("dfp", 1e-1),
                                       ("df", 1e-4), ("nd", 1e-4)])
def test_fullsize_rmat24_update(rmat24, mode, frac):
    n, s, d, og, ref0 = rmat24
    p = _device_pair(n, s, d, og)
    p.g.autotune()
    ds, dd, is_, id_ = W.batch_8020(n, s, d, frac, seed=1001 + int(round(-np.log10(frac))))
    p.apply(ds, dd, is_, id_, device=True)
    assert_csr_equal(p.g, p.og)
    r, st, ref = p.rank(mode, ref0.ranks)
    err = float(np.abs(r - ref.ranks).max())
    _print(f"  {mode} f={frac:g}: batch {len(ds) + len(is_)}, linf {err:.3e} it {st['iterations']}/{ref.iterations} "
           f"ever {st['ever_affected']}/{ref.ever_affected} dense its {st['dense_iterations']}")
    assert err <= LINF
    assert abs(st["iterations"] - ref.iterations) <= 1
    p.g.close()


def test_fullsize_temporal():
    torch_cuda()
    n, total = 2_000_000, 40_000_000
    src, dst = W.temporal_stream(n, total, seed=7)
    k0 = int(0.9 * len(src))
    p = Pair(n, src[:k0], dst[:k0])
    _print("temporal: n", n, "initial edges", p.og.m)
    assert_csr_equal(p.g, p.og)
    p.g.autotune()
    r = O.rank("static", p.og).ranks
    B = 40_000
    for i in range(3):
        lo = k0 + i * B
        info = p.apply([], [], src[lo:lo + B], dst[lo:lo + B])
        assert_csr_equal(p.g, p.og)
        gr, st, ref = p.rank("dfp", r)
        err = float(np.abs(gr - ref.ranks).max())
        _print(f"  batch {i}: effective {info['ins_effective']} of {B}, linf {err:.3e}, it {st['iterations']}")
        assert err <= LINF
        r = ref.ranks


@pytest.mark.parametrize("mode", ["static", "nd", "df", "dfp"])
def test_fullsize_small_graph(mode):
    torch_cuda()
    n, s, d = W.rmat_graph(14, 16, seed=3)
    og0 = O.graph(n, s, d)
    r0 = O.rank("static", og0).ranks
    worst = 0.0
    for k in range(12):
        p = Pair(n, s, d)
        ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-3, seed=500 + k)
        p.apply(ds, dd, is_, id_)
        r, st, ref = p.rank(mode, r0)
        worst = max(worst, float(np.abs(r - ref.ranks).max()))
        assert st["converged"] == ref.converged == 1
    _print(f"small graph {mode}: worst linf over 12 batches {worst:.3e}")
    assert worst <= LINF


def test_fullsize_batched_members():
    torch = torch_cuda()
    m = dfpr()
    rng = np.random.Generator(np.random.PCG64(11))
    members, fracs = [], []
    for k in range(64):
        n = int(round(np.exp(rng.uniform(np.log(1e3), np.log(1e6)))))
        ef = float(rng.uniform(8, 32))
        scale = int(np.ceil(np.log2(n)))
        _, s, d = W.rmat_graph(scale, ef, seed=9000 + k, n_limit=n)
        members.append((n, s, d))
        fracs.append(float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2)))))
    _print("batched: 64 members,", sum(len(s) for _, s, _ in members), "edges")
    bg = m.BatchGraph.from_coo(members)
    bounds, _ = bg.autotune()
    plain = [m.Graph.from_coo(n, s, d) for n, s, d in members]
    for g in plain:
        g.set_tuning(bounds)
    r, _, _ = bg.update_ranks_many("static", None)
    r_prev = r.clone()
    batches = [W.batch_8020(n, s, d, f, seed=9500 + k) for k, ((n, s, d), f) in enumerate(zip(members, fracs))]
    bg.apply_batch_many(batches)
    r, tot, per = bg.update_ranks_many("dfp", r_prev)
    torch.cuda.synchronize()
    for k, g in enumerate(plain):
        g.apply_batch(*batches[k])
        rk, st = g.update_ranks("dfp", bg.member(r_prev, k).clone())
        assert torch.equal(bg.member(r, k), rk), k
        assert per[k]["iterations"] == st["iterations"]
    worst = 0.0
    for k in range(len(members)):  # every member against the oracle
        n, s, d = members[k]
        og = O.graph(n, s, d)
        og2, ob = O.apply(og, *batches[k])
        rp = bg.member(r_prev, k).cpu().numpy()
        ref = O.rank("dfp", og2, rp, og, ob)
        err = float(np.abs(bg.member(r, k).cpu().numpy() - ref.ranks).max())
        worst = max(worst, err)
        assert err <= LINF, (k, err)
    _print(f"  batched members vs oracle: worst linf {worst:.3e} over {len(members)} members")


def test_batched_multipart_single_launch():
    """A batch whose arena spans two pull parts (parts hold whole members of
    about 8M vertices), updated in its default single launch, where the parts'
    pulls run concurrently: each part keeps its own chunk partial sums and
    arrival counters.  Small thresholds put long rows of every part in the
    chunked bin.  Every member bit-identical to its plain handle (launch per
    iteration at this size), and within the parity bar of the oracle."""
    torch = torch_cuda()
    m = dfpr()
    members = [W.rmat_graph(22, 6, seed=9700 + k) for k in range(3)]
    bounds = [4, 16, 128, 1024, 4096]
    bg = m.BatchGraph.from_coo(members)
    bg.set_fused_limit(1 << 40)  # the single launch at any arena size
    bg.set_tuning(bounds)
    plain = [m.Graph.from_coo(n, s, d) for n, s, d in members]
    for g in plain:
        g.set_tuning(bounds)
    _print("multipart batch: members", [n for n, _, _ in members], "edges", bg.m)
    r, _, _ = bg.update_ranks_many("static", None)
    r_prev = r.clone()
    for k, g in enumerate(plain):
        rk, _ = g.update_ranks("static", None)
        assert torch.equal(bg.member(r, k), rk), ("static", k)
    batches = [W.batch_8020(n, s, d, 1e-4, seed=9800 + k) for k, (n, s, d) in enumerate(members)]
    bg.apply_batch_many(batches)
    r, tot, per = bg.update_ranks_many("dfp", r_prev)
    torch.cuda.synchronize()
    for k, g in enumerate(plain):
        g.apply_batch(*batches[k])
        rk, st = g.update_ranks("dfp", bg.member(r_prev, k).clone())
        assert torch.equal(bg.member(r, k), rk), ("dfp", k, float((bg.member(r, k) - rk).abs().max()))
        assert per[k]["iterations"] == st["iterations"]
    n, s, d = members[0]
    og = O.graph(n, s, d)
    og2, ob = O.apply(og, *batches[0])
    ref = O.rank("dfp", og2, bg.member(r_prev, 0).cpu().numpy(), og, ob)
    err = float(np.abs(bg.member(r, 0).cpu().numpy() - ref.ranks).max())
    _print(f"  member 0 vs oracle: linf {err:.3e}")
    assert err <= LINF
