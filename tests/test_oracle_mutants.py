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
    "teleport_dropped": ("double r = (1.0 - alpha) / (double)g->n;", "double r = 0.0;"),
    "outdeg_from_in_csr": ("(double)(g->out_off[u + 1] - g->out_off[u])",
                           "(double)(g->in_off[u + 1] - g->in_off[u])"),
    "gather_wrong_vertex": ("r += alpha * R[u] / outdeg;", "r += alpha * R[v] / outdeg;"),
    "no_self_loops": ("g->keys[m + v] = KEY(v, v);", "g->keys[m + v] = KEY(0, 0);"),
    "linf_not_max": ("            if (d > dR) dR = d;\n            edges",
                     "            dR = d;\n            edges"),
    "df_linf_not_max": ("            dr[v] = d;\n            if (d > dR) dR = d;",
                        "            dr[v] = d;\n            dR = d;"),
    "frontier_not_strict": ("affected[v] && dr[v] > frontier_tol",
                            "affected[v] && dr[v] >= frontier_tol"),
    "deleted_target_unmarked": ("if (i < n_del) flags[del_dst[i]] = 1;", ";"),
    "self_loop_deletable": ("if (del_src[i] != del_dst[i]) dk[nd++]", "if (1) dk[nd++]"),
    "second_buffer_not_prev": (
        "memcpy(Rn, prev, (size_t)n * sizeof(double));\n    oracle_stats s = {0};\n"
        "    for (int32_t v = 0; v < n; v++) s.affected_initial += aff[v];\n    if (affected_initial)",
        "memset(Rn, 0, (size_t)n * sizeof(double));\n    oracle_stats s = {0};\n"
        "    for (int32_t v = 0; v < n; v++) s.affected_initial += aff[v];\n    if (affected_initial)"),
    "marks_not_kept": ("memcpy(next, affected, (size_t)n);", "memset(next, 0, (size_t)n);"),
    "loose_convergence": ("        if (dR <= tol) { s.converged = 1; break; }\n    }\n    if (cur != R)",
                          "        if (dR <= tol * 1e6) { s.converged = 1; break; }\n    }\n    if (cur != R)"),
    "in_csr_transposed": ("g->in_idx[cursor[v]++] = u;", "g->in_idx[cursor[v]++] = v;"),
    "insert_duplicates": ("else { nk[w++] = g->keys[a++]; b++; }",
                          "else { nk[w++] = g->keys[a++]; nk[w++] = ik[b++]; }"),
    "uniform_start_wrong": ("ranks_out[v] = 1.0 / (double)g->n;", "ranks_out[v] = 1.0;"),
    "dt_deleted_edges_ignored": ("for (int64_t j = lo; j < n_del && del[j] / n == x; j++) {",
                                 "for (int64_t j = lo; j < lo; j++) {"),
    "dt_stops_after_first_level": (
        "if (!flags[w]) { flags[w] = 1; queue[tail++] = w; }\n        }\n        /* deleted",
        "if (!flags[w]) { flags[w] = 1; }\n        }\n        /* deleted"),
    "dt_iterates_every_vertex": ("v < n; v++) {\n            if (!aff[v]) continue;",
                                 "v < n; v++) {\n            if (0) continue;"),
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
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o",
                           str(so), str(work / "dfpr_oracle.c"), "-lm"])
    env = dict(os.environ, DFPR_ORACLE_LIB=str(so), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
