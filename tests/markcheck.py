"""Comparison of final Dynamic Frontier marks with the oracle's, shared by
the GPU parity tests."""
import sys

import numpy as np


def say(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


def check_final_marks(fg, f1, ch, in_off, in_idx, ftol, what="", iters_equal=True):
    """Final Dynamic Frontier marks (fg, the library's; f1, the oracle's)
    compared as sets.  A vertex expands when its largest rank change in a
    sweep exceeds ftol, a comparison the two sides may take differently only
    when that change lies within rounding of ftol (ch: the oracle's largest
    change per vertex).  Such vertices are ambiguous.  With none, the sets
    must be equal; otherwise their symmetric difference must stay within 1%
    of the oracle's set, and every vertex in it must have an in-neighbour
    that is ambiguous or itself in the difference (a mark that hinges on a
    comparison at ftol, or follows from one).  When the two sides ran a
    different number of iterations, any vertex marked on both may have
    expanded in the iteration only one of them ran."""
    fg = np.asarray(fg, bool)
    f1 = np.asarray(f1, bool)
    margin = max(1e-2 * ftol, 4e-17)
    amb = np.abs(ch - ftol) <= margin
    if not iters_equal:
        amb = amb | (fg & f1)
    diff = fg ^ f1
    nd = int(diff.sum())
    say(f"final marks {what}: {int(f1.sum())} oracle, {int(fg.sum())} library, "
         f"{nd} differ, {int(amb.sum())} ambiguous")
    if not amb.any():
        assert nd == 0, f"final marks differ at {np.flatnonzero(diff)[:10]}"
        return
    assert nd <= max(1, int(f1.sum()) // 100)
    for w in np.flatnonzero(diff):
        row = in_idx[in_off[w]:in_off[w + 1]]
        assert (amb[row] | diff[row]).any(), f"unexplained mark difference at {w}"
