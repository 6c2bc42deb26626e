"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/dfpr_oracle.c``, plants one plausible mistake (a
dropped term, a wrong index, a wrong comparison, a transposed operand ...),
builds it on the CPU and runs the pin suite against it in a child process;
the suite has to fail.  The real oracle is untouched.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dfpr_oracle.c")

MUTANTS = {
    "teleport_dropped": ("return alpha * sum + (1.0 - alpha) / (double)g->n;",
                         "return alpha * sum;"),
    "outdeg_from_in_csr": ("sum += R[u] / (double)(g->out_off[u + 1] - g->out_off[u]);",
                           "sum += R[u] / (double)(g->in_off[u + 1] - g->in_off[u]);"),
    "gather_wrong_vertex": ("sum += R[u] / (double)", "sum += R[v] / (double)"),
    "damping_inside_wrong": ("return alpha * sum + (1.0 - alpha) / (double)g->n;",
                             "return sum + (1.0 - alpha) / (double)g->n;"),
    "no_self_loops": ("g->keys[m + v] = KEY(v, v);", "g->keys[m + v] = KEY(0, 0);"),
    "linf_not_max": ("linf = d > linf ? d : linf;", "linf = d;"),
    "change_signed": ("const double d = fabs(r - cur[v]);", "const double d = r - cur[v];"),
    "frontier_not_strict": ("affected[v] && dr[v] > frontier_tol",
                            "affected[v] && dr[v] >= frontier_tol"),
    "deleted_target_unmarked": ("for (int64_t i = 0; i < n_del; i++) flags[del_dst[i]] = 1;",
                                ";"),
    "insertion_source_unmarked": ("for (int64_t i = 0; i < n_ins; i++) is_source[ins_src[i]] = 1;",
                                  ";"),
    "self_loop_deletable": ("if (del_src[i] != del_dst[i]) dk[nd++]", "if (1) dk[nd++]"),
    "second_buffer_not_prev": ("memcpy(B, prev, (size_t)n * sizeof(double));",
                               "memset(B, 0, (size_t)n * sizeof(double));"),
    "marks_not_kept": ("memcpy(next, affected, (size_t)n);", "memset(next, 0, (size_t)n);"),
    "df_sweeps_every_vertex": ("sweep(g, marks, cur, nxt, change, alpha)",
                               "sweep(g, NULL, cur, nxt, change, alpha)"),
    "df_loose_convergence": (
        "        if (w.linf <= tol) { s.converged = 1; break; }\n    }\n    memcpy(ranks_out, cur, "
        "(size_t)n * sizeof(double));\n    for",
        "        if (w.linf <= tol * 1e6) { s.converged = 1; break; }\n    }\n    memcpy(ranks_out, "
        "cur, (size_t)n * sizeof(double));\n    for"),
    "loose_convergence": ("        if (w.linf <= tol) { s.converged = 1; break; }\n    }\n    if (cur != R)",
                          "        if (w.linf <= tol * 1e6) { s.converged = 1; break; }\n    }\n    if (cur != R)"),
    "in_csr_transposed": ("g->in_idx[cursor[v]++] = u;", "g->in_idx[cursor[v]++] = v;"),
    "insert_duplicates": ("else { nk[w++] = g->keys[a++]; b++; }",
                          "else { nk[w++] = g->keys[a++]; nk[w++] = ik[b++]; }"),
    "uniform_start_wrong": ("ranks_out[v] = 1.0 / (double)g->n;", "ranks_out[v] = 1.0;"),
    "dt_deleted_edges_ignored": ("for (int64_t j = lo; j < n_del && del[j] / n == x; j++) {",
                                 "for (int64_t j = lo; j < lo; j++) {"),
    "dt_stops_after_first_level": (
        "if (!flags[w]) { flags[w] = 1; queue[tail++] = w; }\n        }\n        /* deleted",
        "if (!flags[w]) { flags[w] = 1; }\n        }\n        /* deleted"),
    "dt_iterates_every_vertex": ("sweep(g, aff, cur, nxt, NULL, alpha)",
                                 "sweep(g, NULL, cur, nxt, NULL, alpha)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    work = tmp_path / "oracle"
    work.mkdir()
    shutil.copy(os.path.join(ROOT, "oracle", "dfpr_oracle.h"), work)
    (work / "dfpr_oracle.c").write_text(text.replace(old, new))
    so = work / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o",
                           str(so), str(work / "dfpr_oracle.c"), "-lm"])
    env = dict(os.environ, DFPR_ORACLE_LIB=str(so), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
