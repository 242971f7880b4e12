"""Golden fixtures under tests/golden/.

closed_forms.txt holds exact Static ranks of small graphs (Equation 1 with a
self-loop on every vertex, solved by hand): the oracle reaches them to 1e-13,
and so does the library on the GPU.  oracle_dfp_rmat8.txt holds the oracle's
Static and DF-P results on a seeded graph and batch, written by
tests/golden/make_golden.py: the oracle must still produce them bit for bit
(an unintended change to its arithmetic fails here), and the library's DF-P
from the stored Static ranks must be within the parity tolerance of them."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def closed_forms():
    cases, cur = [], None
    for line in open(os.path.join(HERE, "closed_forms.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *rest = line.split()
        if key == "case":
            cur = {"name": rest[0], "n": int(rest[1])}
            cases.append(cur)
        elif key == "edges":
            cur["src"] = np.array([int(e.split("-")[0]) for e in rest], np.int32)
            cur["dst"] = np.array([int(e.split("-")[1]) for e in rest], np.int32)
        elif key == "ranks":
            cur["ranks"] = np.array([float(Fraction(x)) for x in rest])
    return cases


def regression():
    kv = {}
    for line in open(os.path.join(HERE, "oracle_dfp_rmat8.txt")):
        if line.startswith("#"):
            continue
        key, *rest = line.split()
        kv[key] = rest
    return kv


@pytest.mark.parametrize("case", closed_forms(), ids=lambda c: c["name"])
def test_closed_forms_oracle(case):
    g = O.graph(case["n"], case["src"], case["dst"])
    r = O.rank("static", g, tol=1e-15).ranks
    assert np.abs(r - case["ranks"]).max() <= 1e-13
    assert abs(case["ranks"].sum() - 1.0) <= 1e-15


def test_oracle_regression_bit_exact():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    kv = regression()
    n, g0, g1, r0, r1 = mg.compute()
    assert n == int(kv["n"][0]) and g0.m == int(kv["m0"][0]) and g1.m == int(kv["m1"][0])
    assert r0.iterations == int(kv["static_iterations"][0]) and r1.iterations == int(kv["dfp_iterations"][0])
    assert r1.ever_affected == int(kv["dfp_ever_affected"][0])
    assert np.array_equal(r0.ranks, np.array([float(x) for x in kv["static"]]))
    assert np.array_equal(r1.ranks, np.array([float(x) for x in kv["dfp"]]))


@pytest.mark.gpu
@pytest.mark.parametrize("case", closed_forms(), ids=lambda c: c["name"])
def test_closed_forms_gpu(case):
    from gpu_common import dfpr, torch_cuda
    torch_cuda()
    g = dfpr().Graph.from_coo(case["n"], case["src"], case["dst"])
    r, st = g.update_ranks("static", None, tol=1e-15, max_iters=500)
    assert np.abs(r.cpu().numpy() - case["ranks"]).max() <= 1e-13
    g.close()


@pytest.mark.gpu
def test_regression_fixture_gpu():
    import workloads as W
    from gpu_common import dfpr, torch_cuda
    torch = torch_cuda()
    kv = regression()
    n, s, d = W.rmat_graph(8, 16, seed=3)
    g = dfpr().Graph.from_coo(n, s, d)
    g.apply_batch(*W.batch_8020(n, s, d, 1e-2, seed=4))
    r0 = torch.from_numpy(np.array([float(x) for x in kv["static"]])).cuda()
    r, st = g.update_ranks("dfp", r0)
    assert np.abs(r.cpu().numpy() - np.array([float(x) for x in kv["dfp"]])).max() <= 1e-9
    assert st["ever_affected"] == int(kv["dfp_ever_affected"][0])
    g.close()
