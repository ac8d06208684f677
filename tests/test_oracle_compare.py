"""Pins of the oracle's comparison measures (every parity verdict goes through
them): hand-computed values, so that a plausible slip -- dividing by the
wrong norm, dropping the square root, accumulating in FP32, swapping the
arguments -- fails one case.
"""
import math

import numpy as np
import pytest

import oracle


def test_rel_l2_hand_cases():
    # ||(0,1)|| / ||(1,0)|| = 1; dividing by ||a|| = sqrt(2) would give 0.707.
    assert oracle.rel_l2([1.0, 1.0], [1.0, 0.0]) == 1.0
    # ||(3,-1)|| / ||(0,5)|| = sqrt(10)/5.
    assert math.isclose(oracle.rel_l2([3.0, 4.0], [0.0, 5.0]), math.sqrt(10.0) / 5.0, rel_tol=1e-15)
    # Without the square roots this would be 4, not 2.
    assert oracle.rel_l2([3.0, 0.0], [1.0, 0.0]) == 2.0
    # Not symmetric in its arguments: the reference scales.
    assert oracle.rel_l2([2.0, 0.0], [1.0, 0.0]) == 1.0
    assert oracle.rel_l2([1.0, 0.0], [2.0, 0.0]) == 0.5
    # Equal inputs.
    assert oracle.rel_l2(np.arange(7.0), np.arange(7.0)) == 0.0


def test_rel_l2_zero_reference_is_the_absolute_norm():
    assert oracle.rel_l2([3.0, 4.0], [0.0, 0.0]) == 5.0
    assert oracle.rel_l2([0.0, 0.0], [0.0, 0.0]) == 0.0


def test_rel_l2_accumulates_fp32_inputs_in_fp64():
    # Squares of 1e30 overflow FP32 and squares of 1e-30 underflow it; in
    # FP64 both are exact enough: ||(0, 1e30)|| / ||(1e30, 1e30)|| = 1/sqrt(2).
    for s in (1e30, 1e-30):
        ref = np.array([s, s], dtype=np.float32)
        a = np.array([s, 2 * s], dtype=np.float32)
        got = oracle.rel_l2(a, ref)
        want = float(np.float32(2 * s) - np.float32(s)) / (math.sqrt(2.0) * float(np.float32(s)))
        assert math.isclose(got, want, rel_tol=1e-12), (s, got, want)
    # An irrational ratio from FP32 inputs: FP64 arithmetic gives 1/sqrt(2)
    # to the last bits, FP32 arithmetic only to about 1e-8.
    a = np.array([1.0, 1.0, 1.0], dtype=np.float32)
    ref = np.array([1.0, 1.0, 0.0], dtype=np.float32)
    assert math.isclose(oracle.rel_l2(a, ref), 1.0 / math.sqrt(2.0), rel_tol=1e-15)


def test_rel_l2_flattens_any_shape():
    ref = np.arange(24.0).reshape(2, 3, 4) + 1.0
    a = ref.copy()
    a[1, 2, 3] += 2.0
    assert math.isclose(oracle.rel_l2(a, ref), 2.0 / math.sqrt(float(np.sum(ref ** 2))), rel_tol=1e-15)
    with pytest.raises(ValueError):
        oracle.rel_l2(np.zeros(3), np.zeros(4))


def test_max_rel_hand_cases():
    # Largest pointwise deviation 3 against the largest |ref| 5 (not 4).
    assert oracle.max_rel([1.0, -2.0, 5.0], [4.0, -5.0, 5.0]) == 0.6
    # The sign of the deviation and of the reference does not matter.
    assert oracle.max_rel([-1.0, 0.0], [1.0, 0.0]) == 2.0
    # A single wrong point out of a million: invisible to a loose global
    # norm, exact here.
    ref = np.ones(1 << 20)
    a = ref.copy()
    a[12345] = 1.5
    assert oracle.max_rel(a, ref) == 0.5
    assert oracle.rel_l2(a, ref) < 1e-3
    assert oracle.max_rel([3.0, 4.0], [0.0, 0.0]) == 4.0
    assert oracle.max_rel([], []) == 0.0
    with pytest.raises(ValueError):
        oracle.max_rel(np.zeros(3), np.zeros(4))


def test_max_rel_fp32_inputs_in_fp64():
    # 16777217 is not an FP32 value; the difference of the FP32 inputs
    # 16777218 and 16777216 is 2 exactly.
    a = np.array([16777218.0], dtype=np.float32)
    ref = np.array([16777216.0], dtype=np.float32)
    assert oracle.max_rel(a, ref) == 2.0 / 16777216.0
