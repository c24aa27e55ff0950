"""Pins of the oracle's comparison metrics on hand-computed values (CPU).

Every GPU parity test grades through ``ritz_rel_err`` (reading C-7: the
largest relative error over the leading r Ritz values, both sorted in
descending order) and ``orth_error`` (||Q^T Q - I||_2), so these are
checked against numbers worked out by hand, not against their own
formulas.  ``sin_theta`` (section 3.1) is pinned in test_oracle_extract.
"""
import math

import numpy as np

import oracle


def test_ritz_rel_err_hand_values():
    # |10 - 10.01| / 10.01 = 9.99e-4 beats |2.0002 - 2| / 2 = 1e-4
    assert math.isclose(oracle.ritz_rel_err([10.0, 5.0, 2.0002], [10.01, 5.0, 2.0]), 0.01 / 10.01,
                        rel_tol=1e-12)
    # the reference is the denominator, not the GPU value
    assert math.isclose(oracle.ritz_rel_err([3.0], [2.0]), 0.5, rel_tol=1e-15)
    assert math.isclose(oracle.ritz_rel_err([2.0], [3.0]), 1.0 / 3.0, rel_tol=1e-15)
    # negative reference values use their magnitude
    assert math.isclose(oracle.ritz_rel_err([-3.9], [-4.0]), 0.025, rel_tol=1e-12)


def test_ritz_rel_err_only_leading_r():
    g = [20.0, 10.0, 1.0, 0.5]
    r_ = [20.0, 10.0, 1.5, 0.1]
    assert oracle.ritz_rel_err(g, r_, 2) == 0.0
    assert math.isclose(oracle.ritz_rel_err(g, r_, 3), 0.5 / 1.5, rel_tol=1e-15)
    assert math.isclose(oracle.ritz_rel_err(g, r_), 4.0, rel_tol=1e-15)   # |0.5 - 0.1| / 0.1


def test_ritz_rel_err_is_not_blind_to_one_bad_value():
    ref = np.linspace(20.0, 1.0, 64)
    got = ref.copy()
    got[63] *= 1.0 + 3e-5                      # only the smallest wanted value is off
    assert math.isclose(oracle.ritz_rel_err(got, ref, 64), 3e-5, rel_tol=1e-9)
    assert oracle.ritz_rel_err(got, ref, 63) == 0.0


def test_orth_error_hand_values():
    # Q = [[1, e], [0, 1]]: Q^T Q - I = [[0, e], [e, e^2]], whose largest
    # eigenvalue magnitude is (e^2 + e sqrt(e^2 + 4)) / 2
    e = 0.1
    Q = np.array([[1.0, e], [0.0, 1.0]])
    assert math.isclose(oracle.orth_error(Q), (e * e + e * math.sqrt(e * e + 4.0)) / 2.0, rel_tol=1e-12)
    # columns of norm 2 and orthogonal: Q^T Q - I = 3 I
    Q = np.zeros((5, 3))
    Q[0, 0] = Q[2, 1] = Q[4, 2] = 2.0
    assert math.isclose(oracle.orth_error(Q), 3.0, rel_tol=1e-15)
    # two equal unit columns: Q^T Q - I = [[0, 1], [1, 0]], norm 1
    v = np.array([0.6, 0.8, 0.0])
    assert math.isclose(oracle.orth_error(np.stack([v, v], axis=1)), 1.0, rel_tol=1e-15)


def test_orth_error_of_a_rotation_is_rounding():
    c, s = math.cos(0.3), math.sin(0.3)
    Q = np.array([[c, -s], [s, c], [0.0, 0.0]])
    assert oracle.orth_error(Q) < 1e-15
