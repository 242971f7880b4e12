"""Writes tests/golden/oracle_dfp_rmat8.txt: the oracle's Static ranks of a
seeded R-MAT scale-8 graph, then its DF-P update after one seeded 80/20 batch
(Algorithm 1 with the defaults of Section 5.1.2).  It calls only the oracle
and the seeded input generators; the stored values pin the oracle against
unintended change (the tests recompute them bit for bit).

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

SCALE, GRAPH_SEED, FRAC, BATCH_SEED = 8, 3, 1e-2, 4
OUT = os.path.join(HERE, "oracle_dfp_rmat8.txt")


def compute():
    n, s, d = W.rmat_graph(SCALE, 16, seed=GRAPH_SEED)
    g0 = O.graph(n, s, d)
    r0 = O.rank("static", g0)
    batch = W.batch_8020(n, s, d, FRAC, seed=BATCH_SEED)
    g1, eff = O.apply(g0, *batch)
    r1 = O.rank("dfp", g1, r0.ranks, g0, eff)
    return n, g0, g1, r0, r1


def main():
    n, g0, g1, r0, r1 = compute()
    with open(OUT, "w") as f:
        f.write("# Oracle golden values, written by tests/golden/make_golden.py (oracle and seeded generators only)\n")
        f.write(f"# R-MAT scale {SCALE}, edge factor 16, seed {GRAPH_SEED}; 80/20 batch of {FRAC:g}*|E|, seed {BATCH_SEED}\n")
        f.write("# alpha 0.85, tol 1e-10, tau_f = tau_p = 1e-6 (Section 5.1.2); Static from 1/|V|, then DF-P (Algorithm 1)\n")
        f.write(f"n {n}\nm0 {g0.m}\nm1 {g1.m}\n")
        f.write(f"static_iterations {r0.iterations}\ndfp_iterations {r1.iterations}\n")
        f.write(f"dfp_ever_affected {r1.ever_affected}\n")
        f.write("static " + " ".join(repr(float(x)) for x in r0.ranks) + "\n")
        f.write("dfp " + " ".join(repr(float(x)) for x in r1.ranks) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
