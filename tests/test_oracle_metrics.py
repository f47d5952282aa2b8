"""Pins of the oracle's field-comparison metrics (Schrijver et al. 2006 definitions, as used for the
paper's Table 1) against values that follow from the definitions by hand: identical, scaled,
reversed and orthogonal fields, and a two-vector case worked out on paper."""
import math

import numpy as np
import pytest

import oracle


def test_identical_scaled_reversed_and_orthogonal_fields():
    rng = np.random.default_rng(71)
    B = rng.normal(size=(3, 50))
    m = oracle.schrijver_metrics(B, B)
    assert m == pytest.approx(dict(C_vec=1.0, C_cs=1.0, E_n=1.0, E_m=1.0, eps=1.0), abs=1e-14)
    m = oracle.schrijver_metrics(B, 2.0 * B)      # |b - B| = |B|: E' = 0; energy ratio 4
    assert m == pytest.approx(dict(C_vec=1.0, C_cs=1.0, E_n=0.0, E_m=0.0, eps=4.0), abs=1e-14)
    m = oracle.schrijver_metrics(B, -B)           # |b - B| = 2|B|
    assert m == pytest.approx(dict(C_vec=-1.0, C_cs=-1.0, E_n=-1.0, E_m=-1.0, eps=1.0), abs=1e-14)
    b = np.cross(B.T, rng.normal(size=(50, 3))).T  # orthogonal to B point by point
    m = oracle.schrijver_metrics(B, b)
    assert abs(m["C_vec"]) < 1e-14 and abs(m["C_cs"]) < 1e-14


def test_two_vectors_by_hand():
    # B = (1,0,0), (0,2,0); b = (1,1,0), (0,2,0)
    B = np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0]])
    b = np.array([[1.0, 0.0], [1.0, 2.0], [0.0, 0.0]])
    m = oracle.schrijver_metrics(B, b)
    # sum B.b = 1 + 4 = 5; sum|B|^2 = 5; sum|b|^2 = 2 + 4 = 6
    assert m["C_vec"] == pytest.approx(5.0 / math.sqrt(5.0 * 6.0), rel=1e-15)
    # per point cosines 1/sqrt(2) and 1
    assert m["C_cs"] == pytest.approx((1.0 / math.sqrt(2.0) + 1.0) / 2.0, rel=1e-15)
    # |b - B| = 1, 0; sum|B| = 3; per point 1/1 and 0/2
    assert m["E_n"] == pytest.approx(1.0 - 1.0 / 3.0, rel=1e-15)
    assert m["E_m"] == pytest.approx(1.0 - 0.5, rel=1e-15)
    assert m["eps"] == pytest.approx(6.0 / 5.0, rel=1e-15)
