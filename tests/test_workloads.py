"""Seeded input generators: determinism and the shapes the workloads promise."""
import numpy as np

import workloads as W


def test_rmat_deterministic_and_clean():
    n, s, d = W.rmat_graph(12, 16, seed=5)
    n2, s2, d2 = W.rmat_graph(12, 16, seed=5)
    assert n == n2 == 4096 and np.array_equal(s, s2) and np.array_equal(d, d2)
    assert (s != d).all()
    keys = s.astype(np.int64) * n + d
    assert (np.diff(keys) > 0).all()  # sorted, no duplicates
    assert 0.7 * 16 * n < s.shape[0] <= 16 * n
    # skew: the hottest vertex receives far more than the mean in-degree
    assert np.bincount(d, minlength=n).max() > 20 * (s.shape[0] / n)
    _, s3, _ = W.rmat_graph(12, 16, seed=6)
    assert not np.array_equal(s, s3[: s.shape[0]])


def test_rmat_limit_redraws():
    n, s, d = W.rmat_graph(10, 8, seed=2, n_limit=700)
    assert n == 700 and s.max() < 700 and d.max() < 700


def test_batch_8020_shape():
    n, s, d = W.rmat_graph(11, 16, seed=1)
    ds, dd, is_, id_ = W.batch_8020(n, s, d, 1e-2, seed=9)
    m_total = s.shape[0] + n
    b = round(1e-2 * m_total)
    assert is_.shape[0] == round(0.8 * b) and ds.shape[0] == b - round(0.8 * b)
    have = set(zip(s.tolist(), d.tolist()))
    assert all(e in have for e in zip(ds.tolist(), dd.tolist()))
    assert not any(e in have for e in zip(is_.tolist(), id_.tolist()))
    assert (is_ != id_).all()
    assert len(set(zip(is_.tolist(), id_.tolist()))) == is_.shape[0]
    assert len(set(zip(ds.tolist(), dd.tolist()))) == ds.shape[0]
    again = W.batch_8020(n, s, d, 1e-2, seed=9)
    assert all(np.array_equal(x, y) for x, y in zip(again, (ds, dd, is_, id_)))


def test_temporal_stream():
    s, d = W.temporal_stream(20000, 400000, seed=3)
    assert s.shape[0] == 400000 and (s != d).all()
    keys = s.astype(np.int64) * 20000 + d
    rep = 1.0 - np.unique(keys).shape[0] / keys.shape[0]
    # 10% exact repeats plus urn collisions on hubs; Table 1's temporal graphs
    # keep 42-64% of their temporal edges as distinct static edges
    assert 0.1 < rep < 0.7
    indeg = np.bincount(d, minlength=20000)
    assert indeg.max() > 50 * indeg.mean()  # preferential attachment skew
