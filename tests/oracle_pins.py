"""Pins for the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each pin takes the oracle library handle, so the same checks run against the
real oracle (tests/test_oracle.py) and against deliberately broken builds of it
(tests/test_oracle_mutants.py), which shows that a plausible mistake anywhere
in the oracle fails at least one pin.

Sources of truth used here:
  * Python set arithmetic for canonical graphs and batch semantics
    (Section 3.2 defines Delta- = E^{t-1} \\ E^t, Delta+ = E^t \\ E^{t-1});
  * numpy.linalg.solve of (I - alpha P^T) r = (1 - alpha)/N 1, the fixed point
    of Equation 1 with a self-loop on every vertex;
  * hand-derived closed forms (derivations in the docstrings);
  * the one-step exactness of Equation 2 when in-neighbours are fixed
    (Appendix A.1);
  * exact invariants: r >= (1 - alpha)/N at every iterate, sum r = 1 for Static.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle as O
import workloads as W

ALPHA = 0.85


# ----------------------------------------------------------------- helpers
def set_canonical(n, src, dst):
    return sorted(set(zip(map(int, src), map(int, dst))) | {(v, v) for v in range(n)})


def dense_pagerank(n, edges, alpha=ALPHA):
    """Exact PageRank of Equation 1 by a dense linear solve (self-loops included in `edges`)."""
    deg = np.zeros(n)
    for u, _ in edges:
        deg[u] += 1
    P = np.zeros((n, n))
    for u, v in edges:
        P[u, v] = 1.0 / deg[u]
    A = np.eye(n) - alpha * P.T
    return np.linalg.solve(A, np.full(n, (1 - alpha) / n))


def small_graphs(count, nmax=8, seed=0):
    rng = np.random.default_rng(seed)
    for k in range(count):
        n = int(rng.integers(1, nmax + 1))
        p = float(rng.uniform(0.05, 0.7))
        s, d = W.random_digraph(n, p, seed * 1000 + k)
        yield n, s, d


# -------------------------------------------------------- graph and batches
def pin_canonical(lib):
    """Canonical edge set and CSRs equal the set definition (bit-exact)."""
    for n, s, d in small_graphs(60, seed=1):
        # add duplicates and self pairs to the input
        s2 = np.concatenate([s, s[: len(s) // 2], np.arange(n, dtype=np.int32)[: n // 2]])
        d2 = np.concatenate([d, d[: len(d) // 2], np.arange(n, dtype=np.int32)[: n // 2]])
        g = O.graph(n, s2, d2, lib=lib)
        want = set_canonical(n, s2, d2)
        assert list(zip(g.esrc.tolist(), g.edst.tolist())) == want
        for v in range(n):
            out_row = g.out_idx[g.out_off[v]:g.out_off[v + 1]].tolist()
            in_row = g.in_idx[g.in_off[v]:g.in_off[v + 1]].tolist()
            assert out_row == sorted(b for a, b in want if a == v)
            assert in_row == sorted(a for a, b in want if b == v)


def pin_apply(lib):
    """Batch application equals the paper's set definitions of Delta+ and Delta-."""
    for k, (n, s, d) in enumerate(small_graphs(80, seed=2)):
        g = O.graph(n, s, d, lib=lib)
        ds, dd, is_, id_ = W.random_edit_batch(n, s, d, n_ins=int(3 + k % 5), n_del=int(3 + k % 4), seed=k)
        old = set(zip(g.esrc.tolist(), g.edst.tolist()))
        ins = {(int(a), int(b)) for a, b in zip(is_, id_) if a != b}
        dele = {(int(a), int(b)) for a, b in zip(ds, dd) if a != b}
        new = (old - dele) | ins
        g2, b = O.apply(g, ds, dd, is_, id_, lib=lib)
        assert list(zip(g2.esrc.tolist(), g2.edst.tolist())) == sorted(new)
        assert list(zip(b.dp_src.tolist(), b.dp_dst.tolist())) == sorted(new - old)
        assert list(zip(b.dm_src.tolist(), b.dm_dst.tolist())) == sorted(old - new)
        assert b.info["ins_effective"] == len(new - old)
        assert b.info["del_effective"] == len(old - new)
        assert b.info["self_loop_dels_ignored"] == len({(int(a), int(c)) for a, c in zip(ds, dd) if a == c})
        assert b.info["ins_in"] == len(is_) and b.info["del_in"] == len(ds)


# ------------------------------------------------------------------ Static
def pin_static_dense(lib):
    """Static (cold start 1/N, Equation 1) reaches the dense-solve fixed point."""
    for n, s, d in small_graphs(60, nmax=12, seed=3):
        g = O.graph(n, s, d, lib=lib)
        edges = list(zip(g.esrc.tolist(), g.edst.tolist()))
        exact = dense_pagerank(n, edges)
        r = O.rank("static", g, lib=lib)
        assert r.converged == 1
        # L-inf stop at tau = 1e-10: the remaining error is at most
        # tau * alpha/(1-alpha) in the max-norm-contractive sense; 1e-9 bounds it.
        assert np.abs(r.ranks - exact).max() <= 1e-9
        r2 = O.rank("static", g, tol=1e-15, lib=lib)
        assert np.abs(r2.ranks - exact).max() <= 1e-13
        assert abs(r2.ranks.sum() - 1.0) <= 1e-12


def pin_static_closed_forms(lib):
    """Closed forms of Equation 1 with self-loops (derived by hand).

    * 2 vertices, edge 0->1: d(0)=2, d(1)=1, C0=0.075.  r0 = C0 + a r0/2 gives
      r0 = 3/23; r1 = C0 + a (r0/2 + r1) gives r1 = 20/23.
    * bidirected star, centre c and 4 leaves: d(c)=5, d(leaf)=2, C0=0.03;
      with r_c + 4 r_l = 1, 0.83 r_c = 0.03 + 1.7 r_l gives r_c = 91/251, r_l = 40/251.
    * path 0->1->2->3: r0 = C0/(1-a/2), r_i = (C0 + a r_{i-1}/2)/(1-a/2) for
      the interior, r3 = (C0 + a r2/2)/(1-a); r0 = 3/46.
    * directed cycle and complete digraph: every rank is 1/n by symmetry.
    """
    tol = 1e-15
    r = O.rank("static", O.graph(2, [0], [1], lib=lib), tol=tol, lib=lib).ranks
    assert np.allclose(r, [3 / 23, 20 / 23], rtol=0, atol=1e-14)
    g = O.graph(5, [0, 0, 0, 0, 1, 2, 3, 4], [1, 2, 3, 4, 0, 0, 0, 0], lib=lib)
    r = O.rank("static", g, tol=tol, lib=lib).ranks
    assert np.allclose(r, [91 / 251] + [40 / 251] * 4, rtol=0, atol=1e-14)
    a, C0 = ALPHA, (1 - ALPHA) / 4
    r0 = C0 / (1 - a / 2)
    r1 = (C0 + a * r0 / 2) / (1 - a / 2)
    r2 = (C0 + a * r1 / 2) / (1 - a / 2)
    r3 = (C0 + a * r2 / 2) / (1 - a)
    r = O.rank("static", O.graph(4, [0, 1, 2], [1, 2, 3], lib=lib), tol=tol, lib=lib).ranks
    assert np.allclose(r, [r0, r1, r2, r3], rtol=0, atol=1e-14)
    assert abs(r0 - 3 / 46) < 1e-16
    for n in (3, 7, 16):
        cyc = O.graph(n, np.arange(n), (np.arange(n) + 1) % n, lib=lib)
        assert np.abs(O.rank("static", cyc, tol=tol, lib=lib).ranks - 1 / n).max() < 1e-14
        s, d = np.nonzero(~np.eye(n, dtype=bool))
        comp = O.graph(n, s, d, lib=lib)
        assert np.abs(O.rank("static", comp, tol=tol, lib=lib).ranks - 1 / n).max() < 1e-14


def pin_nd_is_static_warm(lib):
    """Naive-dynamic from the exact previous ranks converges to the new exact ranks,
    and ND from 1/N equals Static bit-for-bit (same iteration from the same start)."""
    for n, s, d in small_graphs(25, nmax=10, seed=4):
        g = O.graph(n, s, d, lib=lib)
        st = O.rank("static", g, lib=lib)
        nd = O.rank("nd", g, np.full(n, 1.0 / n), lib=lib)
        assert np.array_equal(st.ranks, nd.ranks) and st.iterations == nd.iterations
        ds, dd, is_, id_ = W.random_edit_batch(n, s, d, 3, 2, seed=n)
        g2, _ = O.apply(g, ds, dd, is_, id_, lib=lib)
        exact2 = dense_pagerank(n, list(zip(g2.esrc.tolist(), g2.edst.tolist())))
        exact1 = dense_pagerank(n, list(zip(g.esrc.tolist(), g.edst.tolist())))
        r = O.rank("nd", g2, exact1, lib=lib)
        assert np.abs(r.ranks - exact2).max() <= 1e-9


# ------------------------------------------------------------- DF and DF-P
def _path_insert_all(n, lib):
    g0 = O.graph(n, [], [], lib=lib)
    g1, b = O.apply(g0, [], [], np.arange(n - 1), np.arange(1, n), lib=lib)
    return g0, g1, b


def pin_dfp_closed_loop(lib):
    """Equation 2 is exact in one step once in-neighbours are final (Appendix A.1).

    On a self-looped directed path built by one insert batch (every vertex is
    marked), DF-P with no pruning makes vertex i final in iteration i+1, so it
    stops after n+1 iterations with the exact ranks; DF (Equation 1) needs the
    self-loop recursion and many more iterations.
    """
    for n in (2, 3, 6, 9):
        g0, g1, b = _path_insert_all(n, lib)
        exact = dense_pagerank(n, list(zip(g1.esrc.tolist(), g1.edst.tolist())))
        r = O.rank("dfp", g1, np.full(n, 1.0 / n), g0, b, tol_f=-1, tol_p=-1, lib=lib)
        assert r.iterations == n + 1
        assert np.abs(r.ranks - exact).max() < 1e-15
        rdf = O.rank("df", g1, np.full(n, 1.0 / n), g0, b, tol_f=-1, tol_p=-1, lib=lib)
        assert rdf.iterations >= 2 * (n + 1) + 10
        assert np.abs(rdf.ranks - exact).max() < 1e-9
    # 2 vertices with defaults: (3/23, 20/23) after two rank-changing iterations
    g0, g1, b = _path_insert_all(2, lib)
    r = O.rank("dfp", g1, np.array([0.5, 0.5]), g0, b, lib=lib)
    assert r.iterations == 3 and r.converged == 1
    assert np.abs(r.ranks - [3 / 23, 20 / 23]).max() < 1e-15


def pin_dynamic_bruteforce(lib):
    """Every single-edge insert or delete on small random graphs: DF and DF-P with
    tau_f = 0 (expand on any change) and no pruning, started from the exact ranks
    of G^{t-1}, reach the exact ranks of G^t.  A vertex whose rank must change but
    is never marked would stay at its old value and fail this."""
    worst = 0.0
    for n, s, d in small_graphs(14, nmax=6, seed=5):
        if n < 2:
            continue
        g = O.graph(n, s, d, lib=lib)
        old = set(zip(g.esrc.tolist(), g.edst.tolist()))
        exact1 = dense_pagerank(n, sorted(old))
        for u, v in itertools.product(range(n), range(n)):
            if u == v:
                continue
            if (u, v) in old:
                g2, b = O.apply(g, [u], [v], [], [], lib=lib)
            else:
                g2, b = O.apply(g, [], [], [u], [v], lib=lib)
            exact2 = dense_pagerank(n, list(zip(g2.esrc.tolist(), g2.edst.tolist())))
            for mode in ("df", "dfp"):
                r = O.rank(mode, g2, exact1, g, b, tol_f=0.0, tol_p=-1.0, lib=lib)
                err = np.abs(r.ranks - exact2).max()
                worst = max(worst, err)
                assert err <= 1e-9, (n, u, v, mode, err)
    return worst


def pin_dynamic_special_cases(lib):
    """Empty effective batch: one iteration, ranks returned bit-exact.  All vertices
    marked: DF never unmarks, so it equals ND bit-for-bit."""
    for n, s, d in small_graphs(20, nmax=10, seed=6):
        g = O.graph(n, s, d, lib=lib)
        r0 = O.rank("static", g, lib=lib).ranks
        # no-op batch: re-insert existing edges, delete absent ones, self-loops
        if len(s):
            ins_s, ins_d = s[:2], d[:2]
        else:
            ins_s, ins_d = np.zeros(0, np.int32), np.zeros(0, np.int32)
        absent = [(a, b) for a in range(n) for b in range(n)
                  if a != b and (a, b) not in set(zip(s.tolist(), d.tolist()))][:2]
        del_s = [a for a, _ in absent] + [0]
        del_d = [b for _, b in absent] + [0]
        g2, b = O.apply(g, del_s, del_d, ins_s, ins_d, lib=lib)
        assert len(b.dm_src) == 0 and len(b.dp_src) == 0
        for mode in ("df", "dfp"):
            r = O.rank(mode, g2, r0, g, b, lib=lib)
            assert r.iterations == 1 and r.converged == 1 and r.ever_affected == 0
            assert np.array_equal(r.ranks, r0)
        # every vertex marked: toggle u -> u+1 for every u, so every u is the
        # source of an effective change and out(u) holds u itself
        if n >= 2:
            have = set(zip(s.tolist(), d.tolist()))
            tog = [(u, (u + 1) % n) for u in range(n)]
            dl = [e for e in tog if e in have]
            il = [e for e in tog if e not in have]
            g3, b3 = O.apply(g, [a for a, _ in dl], [c for _, c in dl], [a for a, _ in il],
                             [c for _, c in il], lib=lib)
            assert len(set(b3.dm_src.tolist()) | set(b3.dp_src.tolist())) == n
            df = O.rank("df", g3, r0, g, b3, lib=lib)
            nd = O.rank("nd", g3, r0, lib=lib)
            assert np.array_equal(df.ranks, nd.ranks) and df.iterations == nd.iterations


def pin_relative_criterion(lib):
    """The expansion test uses dr / max(previous, current rank) (Section 4.2).

    3 vertices, G^{t-1} = {1->2}, insert 0->1, R_prev = (0.1, 0.3, 0.6), DF with
    tau_f = 0.3.  Marked: out(0) = {0, 1}.  Iteration 1, vertex 1 (in(1) = {0, 1},
    d = 2 for both): c = 0.1/2 + 0.3/2 = 0.2, r = 0.05 + 0.85*0.2 = 0.22,
    dr = 0.08; dr/max = 0.08/0.3 = 0.267 <= 0.3 (no expansion), whereas dr/min
    would be 0.364 > 0.3.  Vertex 0: r = 0.05 + 0.85*0.05 = 0.0925, rel 0.075.
    Later changes only shrink, so vertex 2 is never processed and keeps 0.6."""
    g0 = O.graph(3, [1], [2], lib=lib)
    g1, b = O.apply(g0, [], [], [0], [1], lib=lib)
    r = O.rank("df", g1, np.array([0.1, 0.3, 0.6]), g0, b, tol_f=0.3, lib=lib)
    assert r.ever_affected == 2
    assert r.ranks[2] == 0.6
    # with a threshold below 0.267 vertex 1 expands and vertex 2 is processed
    r = O.rank("df", g1, np.array([0.1, 0.3, 0.6]), g0, b, tol_f=0.25, lib=lib)
    assert r.ever_affected == 3 and r.ranks[2] != 0.6


def pin_other_criteria(lib):
    """The two other measures of Section 4.2 on the same example: vertex 1 has
    dr = 0.08 and out-degree 2, vertex 0 dr = 0.0075 (see pin_relative_criterion).
    Rank change dr: expands at tau_f = 0.06 (vertex 2 then processed), not at 0.1.
    Contribution-factor change dr/d = 0.04: no expansion at tau_f = 0.06, but
    expansion at tau_f = 0.03."""
    g0 = O.graph(3, [1], [2], lib=lib)
    g1, b = O.apply(g0, [], [], [0], [1], lib=lib)
    rp = np.array([0.1, 0.3, 0.6])
    r = O.rank("df", g1, rp, g0, b, tol_f=0.06, criterion="absolute", lib=lib)
    assert r.ever_affected == 3 and r.ranks[2] != 0.6
    # at tau_f = 0.1 the rank change (0.08) stays below while the relative one (0.267) would not
    r = O.rank("df", g1, rp, g0, b, tol_f=0.1, criterion="absolute", lib=lib)
    assert r.ever_affected == 2 and r.ranks[2] == 0.6
    r = O.rank("df", g1, rp, g0, b, tol_f=0.06, criterion="contrib", lib=lib)
    assert r.ever_affected == 2 and r.ranks[2] == 0.6
    r = O.rank("df", g1, rp, g0, b, tol_f=0.03, criterion="contrib", lib=lib)
    assert r.ever_affected == 3
    # DF-P prunes with the same measure: with tau_p above every change the
    # marked vertices are processed once and dropped
    r = O.rank("dfp", g1, rp, g0, b, tol_f=1.0, tol_p=1.0, criterion="absolute", lib=lib)
    assert r.iterations == 2 and r.vertex_updates == 2


def pin_lower_bound(lib):
    """Every iterate of every mode satisfies r >= (1-alpha)/N (all terms are
    non-negative and the Equation 2 factor 1/(1-alpha/d) is >= 1)."""
    for n, s, d in small_graphs(12, nmax=12, seed=7):
        if n < 2:
            continue
        g = O.graph(n, s, d, lib=lib)
        r0 = O.rank("static", g, lib=lib).ranks
        ds, dd, is_, id_ = W.random_edit_batch(n, s, d, 4, 3, seed=n + 11)
        g2, b = O.apply(g, ds, dd, is_, id_, lib=lib)
        for its in (1, 2, 3, 5, 500):
            for mode in ("static", "nd", "df", "dfp"):
                r = O.rank(mode, g2, r0, g, b, max_iters=its, lib=lib)
                assert r.ranks.min() >= (1 - ALPHA) / n
                if mode == "static":
                    assert abs(r.ranks.sum() - 1.0) <= 1e-12


def pin_threshold_strictness(lib):
    """Algorithm 1 prunes when the relative change is at most tau_p and expands
    when it exceeds tau_f.  With alpha = 1/2, |V| = 4 (C0 = 1/8) and dyadic
    ranks every quantity below is exact in binary floating point, so the
    thresholds can be set to a vertex's computed change itself.

    Expansion (DF, Equation 1).  G^{t-1} = {1->2} (+ self-loops), insert 0->1,
    R_prev = (1/4, 1/2, 1/2, 1/4).  Marked: out(0) = {0, 1}; |out(0)| =
    |out(1)| = 2.  Vertex 1: c = 1/8 + 1/4, r = 1/8 + c/2 = 5/16, change 3/16,
    relative 3/16 / (1/2) = 3/8.  Vertex 0: r = 1/8 + 1/16 = 3/16, relative
    1/4.  Both then shrink towards the fixed point (1/6, 2/9).  With tau_f = 3/8
    nothing expands, so vertex 2 is never processed and keeps 1/2 exactly; a
    non-strict test would expand vertex 1 and process vertex 2.

    Pruning (DF-P, Equation 2).  G^{t-1} = {0->2, 1->2}, delete 0->2,
    R_prev = (1/4, 1/2, 3/8, 1/4).  Marked: {0, 2}; afterwards |out(0)| =
    |out(2)| = 1, so the factor 1/(1 - alpha/1) is 2.  Vertex 0: r = 2(1/8 +
    (1/4 - 1/4)/2) = 1/4, change 0.  Vertex 2: in(2) = {1, 2}, c - R[2] = 1/4,
    r = 2(1/8 + 1/8) = 1/2, change 1/8, relative 1/8 / (1/2) = 1/4.  With
    tau_p = 1/4 (tau_f = 1: nothing expands) both are pruned after the first
    iteration: the second processes nothing, 2 vertex updates in all.  A strict
    test would keep vertex 2 for a second iteration (3 updates)."""
    g0 = O.graph(4, [1], [2], lib=lib)
    g1, b = O.apply(g0, [], [], [0], [1], lib=lib)
    rp = np.array([0.25, 0.5, 0.5, 0.25])
    r = O.rank("df", g1, rp, g0, b, alpha=0.5, tol_f=0.375, tol_p=0.375, lib=lib)
    assert r.ever_affected == 2 and r.ranks[2] == 0.5
    assert abs(r.ranks[0] - 1 / 6) < 1e-10 and abs(r.ranks[1] - 2 / 9) < 1e-10
    # just below the computed change, vertex 1 expands and vertex 2 is processed
    r = O.rank("df", g1, rp, g0, b, alpha=0.5, tol_f=np.nextafter(0.375, 0.0), tol_p=0.375, lib=lib)
    assert r.ever_affected == 3 and r.ranks[2] != 0.5

    g0 = O.graph(4, [0, 1], [2, 2], lib=lib)
    g1, b = O.apply(g0, [0], [2], [], [], lib=lib)
    rp = np.array([0.25, 0.5, 0.375, 0.25])
    r = O.rank("dfp", g1, rp, g0, b, alpha=0.5, tol_f=1.0, tol_p=0.25, lib=lib)
    assert list(r.frontier) == [2, 0] and r.vertex_updates == 2 and r.iterations == 2
    assert r.ranks.tolist() == [0.25, 0.5, 0.5, 0.25]
    r = O.rank("dfp", g1, rp, g0, b, alpha=0.5, tol_f=1.0, tol_p=np.nextafter(0.25, 0.0), lib=lib)
    assert list(r.frontier) == [2, 1] and r.vertex_updates == 3


def pin_marks_win_over_prunes(lib):
    """A vertex pruned in an iteration is processed again in the next one when
    an in-neighbour expanded in the same iteration (the expansion marks all of
    its out-neighbours, Algorithm 1).

    alpha = 1/2, |V| = 4, G^{t-1} = {1->2}, insert 0->2, R_prev = (1/2, 1/2,
    3/4, 1/4), DF-P with tau_f = tau_p = 1/10.  Marked: out(0) = {0, 2};
    |out(0)| = |out(1)| = 2, |out(2)| = 1.
      iteration 1: vertex 0 (in(0) = {0}): r = C0/(1 - alpha/2) = 1/6, relative
        change (1/2 - 1/6)/(1/2) = 2/3: kept and expands, marking {0, 2}.
        Vertex 2: r = 2(1/8 + (1/4 + 1/4)/2) = 3/4, change 0: pruned, but
        re-marked by vertex 0.
      iteration 2: vertex 0: r = 1/6 again, change 0: pruned, no expansion.
        Vertex 2: r = 2(1/8 + (1/12 + 1/4)/2) = 7/12, relative change
        (1/6)/(3/4) = 2/9: kept and expands (marks itself).
      iteration 3: vertex 2: r = 7/12, change 0.  Stop.
    So 3 iterations, frontier sizes 2, 2, 1, and R[2] = 7/12.  If prunes won,
    vertex 2 would stay at 3/4."""
    g0 = O.graph(4, [1], [2], lib=lib)
    g1, b = O.apply(g0, [], [], [0], [2], lib=lib)
    rp = np.array([0.5, 0.5, 0.75, 0.25])
    r = O.rank("dfp", g1, rp, g0, b, alpha=0.5, tol_f=0.1, tol_p=0.1, lib=lib)
    assert r.iterations == 3 and r.converged == 1
    assert list(r.frontier) == [2, 2, 1] and r.vertex_updates == 5 and r.ever_affected == 2
    assert abs(r.ranks[2] - 7 / 12) < 1e-15 and abs(r.ranks[0] - 1 / 6) < 1e-15
    assert r.ranks[1] == 0.5 and r.ranks[3] == 0.25


ALL_PINS = [pin_canonical, pin_apply, pin_static_dense, pin_static_closed_forms, pin_nd_is_static_warm,
            pin_dfp_closed_loop, pin_dynamic_bruteforce, pin_dynamic_special_cases, pin_relative_criterion,
            pin_other_criteria, pin_lower_bound, pin_threshold_strictness,
            pin_marks_win_over_prunes]
