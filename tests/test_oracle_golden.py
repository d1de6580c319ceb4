"""Hand-derived closed-form cases (tests/golden/hand_cases.json)."""
import json
import os

import numpy as np

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def test_dis_hand_case():
    c = GOLD["dis"]
    T = oracle.dis(np.array(c["mask"], np.uint8), np.array(c["fk"], float), np.array(c["pdf"], float))
    np.testing.assert_array_equal(T, c["expected"])
    g = oracle.dis_grad(np.array(c["mask"], np.uint8), np.array(c["fk"], float), np.array(c["gbar"], float))
    np.testing.assert_array_equal(g[:, :, 0], c["expected_grad_r0"])


def test_had_hand_case():
    c = GOLD["had"]
    m, fk, f = np.array(c["mask"], np.uint8), np.array(c["fk"], float), np.array(c["pdf"], float)
    np.testing.assert_array_equal(oracle.had(m, fk, f), c["expected"])
    g = oracle.had_grad(m, fk, f, np.array(c["gbar"], float))
    np.testing.assert_array_equal(g, c["expected_grad"])


def test_chi2_hand_case():
    c = GOLD["chi2"]
    L = oracle.cholesky(np.array(c["cov"], float))
    np.testing.assert_array_equal(L, c["chol"])
    chi, d = oracle.chi2([L], np.array(c["sigma"], float), np.array(c["data"], float))
    np.testing.assert_allclose(chi, c["expected_chi2"], rtol=1e-15)
    np.testing.assert_allclose(d, c["expected_grad"], rtol=1e-15)
