"""Pins of the oracle's network PDF and its gradient (Sections 2 and 3: the
fit parametrises the PDF with a neural network on the x-grid and trains it
by gradient descent through the convolution).

* Closed forms: with zero input weights the network is constant in x, so
  f = x^alpha (1-x)^beta (W3 tanh(b2 + W2 tanh(b1)) + b3), worked by hand for
  a one-unit network; with beta > 0 the PDF vanishes at x = 1.
* Finite differences in FP64 on every parameter of small networks, for the
  gradient of a linear functional of f.
* The chain of a fit step, loss(params) = chi2(sigma(f(params))) with DIS and
  hadronic tables: mlp_pdf_grad of the convolution adjoints of dchi2/dsigma
  against central differences of the composed loss.
"""
import numpy as np
import pytest

import oracle
from paper_1909_10547_amd import synth


def test_mlp_closed_form_one_unit():
    # h1 = h2 = 1, one flavour: W1 = 0, b1 = 0.3, W2 = 0.8, b2 = -0.1,
    # W3 = 2, b3 = 0.5: out = 2 tanh(-0.1 + 0.8 tanh(0.3)) + 0.5
    x = np.array([1e-3, 0.1, 0.5, 1.0])
    p = np.array([[0.0, 0.0, 0.3, 0.8, -0.1, 2.0, 0.5]])
    assert oracle.mlp_nparams(1, 1, 1) == 7
    f = oracle.mlp_pdf(p, x, [0.5], [2.0], 1, 1)
    t1 = 0.2913126124515909   # tanh(0.3)
    out = 2.0 * np.tanh(-0.1 + 0.8 * t1) + 0.5
    want = x ** 0.5 * (1 - x) ** 2 * out
    assert f.shape == (1, 4, 1)
    assert np.allclose(f[0, :, 0], want, rtol=1e-14, atol=0)
    assert f[0, 3, 0] == 0.0  # x = 1 with beta > 0


def test_mlp_inputs_are_x_and_log_x():
    # one unit reading only ln x (W1 = [0, 1]), identity-like small slope:
    # out = tanh(tanh(ln x)) with W2 = W3 = 1, biases 0, no preprocessing
    x = np.array([0.2, 0.7])
    p = np.array([[0.0, 1.0, 0.0, 1.0, 0.0, 1.0, 0.0]])
    f = oracle.mlp_pdf(p, x, [0.0], [0.0], 1, 1)
    assert np.allclose(f[0, :, 0], np.tanh(np.tanh(np.log(x))), rtol=1e-14, atol=0)
    p2 = np.array([[1.0, 0.0, 0.0, 1.0, 0.0, 1.0, 0.0]])
    f2 = oracle.mlp_pdf(p2, x, [0.0], [0.0], 1, 1)
    assert np.allclose(f2[0, :, 0], np.tanh(np.tanh(x)), rtol=1e-14, atol=0)


@pytest.mark.parametrize("F,h1,h2,X,R", [(3, 4, 3, 5, 2), (2, 2, 5, 7, 1)])
def test_mlp_gradient_finite_differences(F, h1, h2, X, R):
    rng = np.random.default_rng([F, h1, h2])
    x = synth.xgrid_geom(1e-5, 0.9, X)
    P = oracle.mlp_nparams(F, h1, h2)
    params = rng.normal(scale=0.7, size=(R, P))
    pa, pb = rng.uniform(-0.3, 0.5, F), rng.uniform(1, 4, F)
    gpdf = rng.normal(size=(F, X, R))
    g = oracle.mlp_pdf_grad(params, x, pa, pb, h1, h2, gpdf)

    def loss(p):
        return float(np.sum(gpdf * oracle.mlp_pdf(p, x, pa, pb, h1, h2)))

    h = 1e-6
    fd = np.empty_like(params)
    for r in range(R):
        for k in range(P):
            e = np.zeros_like(params)
            e[r, k] = h
            fd[r, k] = (loss(params + e) - loss(params - e)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_fit_chain_gradient_finite_differences():
    """d chi2(sigma(f(params))) / d params through DIS and hadronic tables."""
    rng = np.random.default_rng(41)
    X, F, h1, h2, R = 6, 4, 3, 3, 2
    x = synth.xgrid_geom(1e-4, 0.9, X)
    td = synth.draw_dis_table(rng, x, 5, nactive=3, nflav=F)
    th = synth.draw_general_had_table(rng, x, 4, npairs=5, nflav=F)
    P = oracle.mlp_nparams(F, h1, h2)
    params = rng.normal(scale=0.5, size=(R, P))
    pa, pb = rng.uniform(-0.2, 0.4, F), rng.uniform(1, 3, F)
    Ns = [5, 4]
    Cs = []
    for n in Ns:
        A = rng.normal(size=(n, n))
        Cs.append(A @ A.T + n * np.eye(n))
    Ls = [oracle.cholesky(C) for C in Cs]
    D = rng.normal(size=sum(Ns))

    def sigma(f):
        return np.concatenate([oracle.dis(td.mask, td.fk, f), oracle.had(th.mask, th.fk, f)])

    def loss(p):
        c, _ = oracle.chi2(Ls, sigma(oracle.mlp_pdf(p, x, pa, pb, h1, h2)), D, want_grad=False)
        return float(np.sum(c))

    f = oracle.mlp_pdf(params, x, pa, pb, h1, h2)
    _, dsig = oracle.chi2(Ls, sigma(f), D)
    gpdf = oracle.dis_grad(td.mask, td.fk, dsig[:5], F, X) + oracle.had_grad(th.mask, th.fk, f, dsig[5:])
    g = oracle.mlp_pdf_grad(params, x, pa, pb, h1, h2, gpdf)
    h = 1e-6
    fd = np.empty_like(params)
    for r in range(R):
        for k in range(P):
            e = np.zeros_like(params)
            e[r, k] = h
            fd[r, k] = (loss(params + e) - loss(params - e)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))
