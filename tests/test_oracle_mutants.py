"""Plant plausible mistakes in copies of the oracle (on the CPU) and check that
the pins catch every one.  This is what makes the pins a check on the oracle
rather than a restatement of it."""
import os
import shutil
import subprocess

import pytest

import oracle as O
import oracle_pins as P

HERE = os.path.dirname(os.path.abspath(O.__file__))

MUTANTS = {
    "no_damping_on_sum": ("r = C0 + alpha * c;", "r = C0 + c;"),
    "dfp_self_term_kept": ("(C0 + alpha * (c - R[v] / d))", "(C0 + alpha * c)"),
    "dfp_factor_dropped": ("r = (1.0 / (1.0 - alpha / d)) * (C0 + alpha * (c - R[v] / d));",
                           "r = (C0 + alpha * (c - R[v] / d));"),
    "in_degree_as_divisor": ("c = c + R[u] / (double)(out_off[u + 1] - out_off[u]);",
                             "c = c + R[u] / (double)(in_off[u + 1] - in_off[u]);"),
    "pull_over_out_edges": ("for (int32_t p = in_off[v]; p < in_off[v + 1]; p++) {\n        int32_t u = in_idx[p];",
                            "for (int32_t p = out_off[v]; p < out_off[v + 1]; p++) {\n        int32_t u = out_idx[p];"),
    "mark_current_snapshot_only": ("for (int32_t p = prev_off[u]; p < prev_off[u + 1]; p++) A[prev_idx[p]] = 1;", ""),
    "delete_wins_over_insert": ("b++; /* also inserted: keep once */\n      else {",
                                "b++; /* also inserted: keep once */\n      {"),
    "c0_wrong_vertex_count": ("const double C0 = (1.0 - alpha) / (double)n;",
                              "const double C0 = (1.0 - alpha) / (double)(n + 1);"),
    "iteration_count_off_by_one": ("if (dR <= tol) { converged = 1; it++; break; }",
                                   "if (dR <= tol) { converged = 1; break; }"),
    "df_also_prunes": ("An[v] = (mode == ORC_DFP && rel <= tol_p) ? 0 : 1;", "An[v] = (rel <= tol_p) ? 0 : 1;"),
    "static_warm_start": ("R[v] = (mode == ORC_STATIC) ? 1.0 / (double)n : r_prev[v];", "R[v] = r_prev[v];"),
    "self_loop_replaced": ("{ fill[v] = start[v]; rows[fill[v]++] = v; }",
                           "{ fill[v] = start[v]; rows[fill[v]++] = (v + 1) % n; }"),
    "in_csr_keyed_by_source": ("const int32_t* key = by_dst ? edst : esrc;", "const int32_t* key = esrc;"),
    "relative_change_over_min": ("else rel = dr / fmax(r, R[v]);", "else rel = dr / fmin(r, R[v]);"),
    "expand_before_commit_lost": ("if (rel > tol_f) X[v] = 1;", "if (rel > tol_f && mode == ORC_DFP) X[v] = 1;"),
    "absolute_measure_relative": ("if (criterion == ORC_CRIT_ABSOLUTE) rel = dr;",
                                  "if (criterion == ORC_CRIT_ABSOLUTE) rel = dr / fmax(r, R[v]);"),
    "contrib_measure_times_degree": ("else if (criterion == ORC_CRIT_CONTRIB) rel = dr / d;",
                                     "else if (criterion == ORC_CRIT_CONTRIB) rel = dr * d;"),
    "prune_strict_less": ("An[v] = (mode == ORC_DFP && rel <= tol_p) ? 0 : 1;",
                          "An[v] = (mode == ORC_DFP && rel < tol_p) ? 0 : 1;"),
    "expand_non_strict": ("if (rel > tol_f) X[v] = 1;", "if (rel >= tol_f) X[v] = 1;"),
    "prunes_win_over_marks": ("#pragma omp atomic write\n          An[out_idx[p]] = 1;",
                              "if (!A[out_idx[p]]) An[out_idx[p]] = 1;"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(os.path.join(HERE, "oracle.c")).read()
    assert src.count(old) == 1, name
    d = tmp_path / name
    d.mkdir()
    shutil.copy(os.path.join(HERE, "oracle.h"), d / "oracle.h")
    (d / "oracle.c").write_text(src.replace(old, new))
    so = d / "liboracle_mut.so"
    subprocess.check_call(["gcc", *O.CFLAGS, "-I", str(d), "-o", str(so), str(d / "oracle.c"), "-lm"])
    return O.load(str(so))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmp_path, name, old, new)
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(lib)
        except Exception:  # noqa: BLE001 - an assertion or a crash both count as caught
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passed every pin"
