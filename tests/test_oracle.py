"""The CPU oracle against its pins (no GPU)."""
import numpy as np
import pytest

import oracle as O
import oracle_pins as P


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=[p.__name__ for p in P.ALL_PINS])
def test_oracle_pin(orc, pin):
    pin(orc)


def test_bruteforce_worst_error_reported(orc):
    worst = P.pin_dynamic_bruteforce(orc)
    assert worst < 1e-9


def test_out_of_range_ids_rejected(orc):
    with pytest.raises(ValueError):
        O.graph(3, [0, 3], [1, 1], lib=orc)
    g = O.graph(3, [0], [1], lib=orc)
    with pytest.raises(ValueError):
        O.apply(g, [], [], [0], [-1], lib=orc)


def test_max_iters_cap_reports_not_converged(orc):
    g = O.graph(4, [0, 1, 2], [1, 2, 3], lib=orc)
    r = O.rank("static", g, max_iters=3, lib=orc)
    assert r.iterations == 3 and r.converged == 0 and r.last_delta > 1e-10


def test_default_tolerance_error_is_small(orc):
    """At the paper's tau_f = tau_p = 1e-6, DF and DF-P stay close to the exact
    ranks on a small R-MAT graph (reported bound, not the parity gate)."""
    import workloads as W
    n, s, d = W.rmat_graph(9, 8, seed=3)
    g = O.graph(n, s, d, lib=orc)
    r0 = O.rank("static", g, tol=1e-14, lib=orc).ranks
    ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-2, seed=5)
    g2, b = O.apply(g, ds, dd, is_, id_, lib=orc)
    ref = O.rank("static", g2, tol=1e-14, lib=orc).ranks
    for mode in ("df", "dfp"):
        r = O.rank(mode, g2, r0, g, b, lib=orc)
        assert r.converged == 1
        assert np.abs(r.ranks - ref).max() / ref.max() < 1e-4
        assert 0 < r.ever_affected <= n
