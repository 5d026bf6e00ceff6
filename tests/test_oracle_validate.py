"""Pins of the oracle's input check against the input conditions of Sec. 3.

The generator of Sec. 3 takes n weights w_0 >= w_1 >= ... >= w_{n-1} >= 0 and
S = sum w (Alg. 1 divides by S).  The reading used throughout (the same on the
GPU side) adds: weights finite, S finite and positive, S >= w_0 (so every
w_u / S <= 1), w_0 either 0 or at least 2^-960 (so 2^32 / w_0 is finite), and
n < 2^32 (node ids are 32-bit).  Each condition is broken on its own here and
must give its own status; the precedence between two broken conditions is
non-finite, then negative, then unsorted, then the conditions on S.
"""
import ctypes

import numpy as np
import pytest

import oracle as O

OK, INVALID, UNSORTED, NEGATIVE, NONFINITE, TOO_LARGE = 0, -1, -2, -3, -4, -5


def code(w, S):
    return O.validate(np.asarray(w, dtype=np.float64), S)


def test_valid_inputs_pass():
    assert code([], 1.0) == OK                          # empty graph
    assert code([3.0, 2.0, 2.0, 0.0], 7.0) == OK        # ties and zero weights
    assert code([0.0, 0.0, 0.0], 1.0) == OK             # all zero: no edges, but valid
    assert code([5.0], 5.0) == OK                       # S == w_0 is allowed
    assert code([2.0 ** -960, 2.0 ** -961], 1.0) == OK  # smallest allowed head
    assert code([1.0, -0.0], 1.0) == OK                 # -0.0 compares equal to 0: not negative


@pytest.mark.parametrize("w", [[np.nan, 1.0], [3.0, np.nan], [np.inf, 1.0], [2.0, 1.0, -np.inf],
                               [1.0, np.inf]])
def test_nonfinite_weight(w):
    assert code(w, 10.0) == NONFINITE


@pytest.mark.parametrize("w", [[2.0, 1.0, -0.5], [-1.0, -2.0], [1.0, -5e-324]])
def test_negative_weight(w):
    assert code(w, 10.0) == NEGATIVE


@pytest.mark.parametrize("w", [[1.0, 2.0], [3.0, 2.0, 2.0, 2.5], [1.0, 0.0, 5e-324]])
def test_unsorted_weights(w):
    assert code(w, 10.0) == UNSORTED


@pytest.mark.parametrize("S", [0.0, -1.0, np.inf, np.nan])
def test_bad_weight_sum(S):
    assert code([1.0, 0.5], S) == INVALID


def test_sum_below_the_head_weight():
    assert code([5.0, 1.0], 4.0) == INVALID
    assert code([5.0, 1.0], np.nextafter(5.0, 0.0)) == INVALID


def test_head_weight_too_small_for_the_quantisation():
    assert code([2.0 ** -961, 2.0 ** -962], 1.0) == INVALID
    assert code([5e-324], 1.0) == INVALID


def test_too_many_nodes():
    # n is checked before any weight is read, so a one-element buffer is enough
    w = np.ones(1)
    L = O.lib()
    got = L.orc_validate(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1 << 32, 1.0)
    assert got == TOO_LARGE
    got = L.orc_validate(w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), (1 << 32) + 5, 1.0)
    assert got == TOO_LARGE


def test_precedence_between_broken_conditions():
    assert code([1.0, np.nan, -1.0, 5.0], 10.0) == NONFINITE   # all three broken
    assert code([1.0, 2.0, -1.0], 10.0) == NEGATIVE            # unsorted and negative
    assert code([4.0, 5.0], 1.0) == UNSORTED                   # unsorted and S < w_0
    assert code([4.0, -1.0], 1.0) == NEGATIVE                  # negative and S < w_0


def test_every_generation_entry_refuses_invalid_input():
    """The oracle's generator and partition return the check's status."""
    bad = np.array([1.0, 2.0])
    with pytest.raises(O.OracleError) as e:
        O.generate(bad, 10.0, 1)
    assert e.value.code == UNSORTED
    with pytest.raises(O.OracleError) as e:
        O.partition(np.array([2.0, -1.0]), 10.0, 4)
    assert e.value.code == NEGATIVE
