"""Pins of the oracle's error measures and of its quantised-input mode.

The GPU parity tests gate on ``oracle.normwise_rel`` and report
``oracle.error_report``, so both are checked here against values computed
by hand: a dropped square root, a norm taken over datapoints instead of
replica columns, a mean instead of a maximum, or a zero column that counts
as agreement would each change one of the expected numbers below.

The quantised-input gradient ``dis_grad_quantized`` is pinned by two facts
of its definition: in FP64 mode the power-of-two scale cancels exactly, so
it equals the plain gradient; with integer inputs every stored operand is
exact in bfloat16, so it equals the plain gradient bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1909_10547_amd import synth


# ---------------------------------------------------------------------------
# normwise_rel: max over replica columns of ||y - y*||_2 / ||y*||_2
# ---------------------------------------------------------------------------

def test_normwise_rel_hand_case():
    # rows are datapoints, columns replicas
    yref = np.array([[3.0, 1.0],
                     [4.0, 0.0]])
    y = np.array([[3.0, 1.5],
                  [4.5, 0.0]])
    # column 0: ||(0, 0.5)|| / ||(3, 4)|| = 0.5 / 5 = 0.1
    # column 1: ||(0.5, 0)|| / ||(1, 0)|| = 0.5
    # (over rows it would be 0.5/sqrt(10) = 0.158; without the square
    # roots 0.25; as a mean over columns 0.3)
    assert oracle.normwise_rel(y, yref) == pytest.approx(0.5, rel=1e-15)
    assert oracle.normwise_rel(y[:, :1], yref[:, :1]) == pytest.approx(0.1, rel=1e-15)


def test_normwise_rel_one_dimensional_and_scale_invariant():
    # a vector is one replica column
    assert oracle.normwise_rel(np.array([3.0, 4.5]), np.array([3.0, 4.0])) == pytest.approx(0.1, rel=1e-15)
    # relative: scaling both arguments by 2^k leaves it unchanged exactly
    rng = np.random.default_rng(60)
    y, r = rng.normal(size=(7, 3)), rng.normal(size=(7, 3))
    assert oracle.normwise_rel(8.0 * y, 8.0 * r) == oracle.normwise_rel(y, r)
    # the last axis is the replica axis whatever the rank
    y3, r3 = rng.normal(size=(2, 5, 4)), rng.normal(size=(2, 5, 4))
    assert oracle.normwise_rel(y3, r3) == oracle.normwise_rel(y3.reshape(10, 4), r3.reshape(10, 4))


def test_normwise_rel_zero_column_rule_and_empty():
    yref = np.array([[1.0, 0.0],
                     [0.0, 0.0]])
    assert oracle.normwise_rel(yref.copy(), yref) == 0.0
    y = yref.copy()
    y[1, 1] = 1e-30
    assert oracle.normwise_rel(y, yref) == np.inf
    assert oracle.normwise_rel(np.zeros((0, 3)), np.zeros((0, 3))) == 0.0


def test_error_report_hand_case():
    yref = np.array([[1000.0], [2.0], [4.0], [0.1]])
    y = np.array([[1000.0], [2.2], [4.0], [0.5]])
    rep = oracle.error_report(y, yref)
    assert rep["normwise"] == oracle.normwise_rel(y, yref)
    # elementwise over |y*| >= 1e-3 * max|y*| = 1: rows 0-2, errors (0, 0.1, 0);
    # row 3 (relative error 4) is below the threshold and must not count
    assert rep["elem_max"] == pytest.approx(0.1, rel=1e-12)
    assert rep["elem_p50"] == 0.0
    assert rep["elem_p99"] == pytest.approx(0.098, rel=1e-12)


# ---------------------------------------------------------------------------
# dis_grad_quantized: g = sum_i Q(FK_i / s_i) Q(gbar_i s_i)
# ---------------------------------------------------------------------------

def test_dis_grad_quantized_fp64_mode_is_the_plain_gradient():
    rng = np.random.default_rng(61)
    t = synth.draw_dis_table(rng, synth.xgrid_geom(1e-5, 0.9, 12), 30, 6)
    s, _ = oracle.dis_stored(t.fk, "f64")
    assert np.any(s != 1.0)  # the scales do not cancel trivially
    gbar = rng.normal(size=(30, 4))
    g = oracle.dis_grad_quantized(t.mask, t.fk, gbar, "f64")
    assert oracle.normwise_rel(g, oracle.dis_grad(t.mask, t.fk, gbar)) < 1e-14


def test_dis_grad_quantized_integer_inputs_are_exact_in_bf16():
    rng = np.random.default_rng(62)
    t = synth.integer_dis_table(rng, 6, 5, ndata=9, nactive=4)
    gbar = rng.integers(-16, 17, size=(9, 3)).astype(np.float64)
    s, _ = oracle.dis_stored(t.fk, "bf16")
    assert np.all(s > 1.0)
    np.testing.assert_array_equal(oracle.dis_grad_quantized(t.mask, t.fk, gbar, "bf16"),
                                  oracle.dis_grad(t.mask, t.fk, gbar))
