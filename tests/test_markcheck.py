"""Host logic of the final-mark comparison used by the GPU parity tests."""
import numpy as np
import pytest

from markcheck import check_final_marks

# in-CSR of a path 0 -> 1 -> 2 -> 3 with self-loops: in(v) = {v-1, v}
IN_OFF = np.array([0, 1, 3, 5, 7])
IN_IDX = np.array([0, 0, 1, 1, 2, 2, 3])
FTOL = 1e-13


def test_equal_sets_pass():
    f = np.array([1, 1, 0, 0], np.uint8)
    check_final_marks(f, f, np.array([0.0, 5e-13, 0, 0]), IN_OFF, IN_IDX, FTOL)


def test_difference_without_ambiguity_fails():
    f1 = np.array([1, 1, 0, 0], np.uint8)
    fg = np.array([1, 1, 1, 0], np.uint8)
    with pytest.raises(AssertionError):
        check_final_marks(fg, f1, np.array([0.0, 5e-13, 0, 0]), IN_OFF, IN_IDX, FTOL)


def test_difference_explained_by_a_change_at_the_tolerance():
    # vertex 1's largest change sits on tau_f: whether 2 is marked hinges on it
    f1 = np.array([1, 1, 0, 0] * 50, np.uint8)
    fg = f1.copy()
    fg[2] = 1
    off = np.concatenate([IN_OFF[:-1] + 7 * k for k in range(50)] + [[350]])
    idx = np.concatenate([IN_IDX + 4 * k for k in range(50)])
    ch = np.zeros(200)
    ch[1] = FTOL * (1 + 1e-4)
    check_final_marks(fg, f1, ch, off, idx, FTOL)
    ch[1] = 2 * FTOL           # clearly above: the difference is unexplained
    with pytest.raises(AssertionError):
        check_final_marks(fg, f1, ch, off, idx, FTOL)
