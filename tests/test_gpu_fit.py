"""The fit step on the device: a network PDF on the x-grid, the DIS and
hadronic convolutions, the FP64 chi2, both adjoints, the reverse pass
through the network and a gradient-descent update (Sections 2 and 3),
against the oracle's network and chain.

* Network forward and reverse pass: FP32 against FP64, normwise <= 1e-5,
  on the workload's network (14 flavours, 50 grid points, 25 + 20 units)
  and on edge shapes (one unit, one grid point, 256 grid points).
* Chain: d chi2 / d params through every kernel, against the oracle's
  composed gradient (FP32 tables: normwise <= 1e-4, the FP32 chain's
  rounding through chi2 and two adjoints; BF16 tables: <= 5e-3).
* Gradient descent lowers chi2.
* Full size: the global-fit workload (30 datasets, 10590 datapoints, R = 100)
  in the configuration bench.py times.
"""
import functools
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1909_10547_amd import fkconv, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("F,X,h1,h2,R", [(14, 50, 25, 20, 16), (1, 1, 1, 1, 1), (3, 256, 4, 5, 3),
                                         (14, 50, 25, 20, 100)])
def test_network_forward_and_reverse_pass(F, X, h1, h2, R):
    rng = np.random.default_rng([F, X, h1, h2, R])
    x = synth.xgrid_geom(1e-7, 1.0, X) if X > 1 else np.array([0.5])
    pa, pb = synth.mlp_preprocessing_exponents(F)
    params = synth.mlp_init(R, F, h1, h2)
    gpdf = rng.normal(size=(F, X, R)).astype(np.float32)
    say(f"case F={F} X={X} h1={h1} h2={h2} R={R}")
    with fkconv.Context(0) as c:
        m, P = fkconv.fk_mlp_create(c.ctx, x, h1, h2, pa, pb)
        assert P == oracle.mlp_nparams(F, h1, h2)
        pd = dev(params)
        f = fkconv.fk_mlp_forward(c.ctx, m, pd, F, X)
        g = fkconv.fk_mlp_backward(c.ctx, m, pd, dev(gpdf))
        torch.cuda.synchronize()
        f, g = f.double().cpu().numpy(), g.double().cpu().numpy()
        fkconv.fk_mlp_destroy(c.ctx, m)
    fr = oracle.mlp_pdf(params.astype(np.float64), x, pa, pb, h1, h2)
    gr = oracle.mlp_pdf_grad(params.astype(np.float64), x, pa, pb, h1, h2, gpdf.astype(np.float64))
    ef = oracle.normwise_rel(f, fr)
    eg = oracle.normwise_rel(g.T, gr.T)
    say(f"  pdf {ef:.2e}, parameter gradient {eg:.2e}")
    assert ef <= 1e-5 and eg <= 1e-5


def fit_case(scale_dis, scale_had, R):
    fit = synth.global_fit_workload(1.0)
    wd, wh = synth.dis_fit_workload(scale_dis), synth.had_fit_workload(scale_had)
    dis_t = [wd.table(d) for d in range(len(wd.ndata))]
    had_t = [wh.table(d) for d in range(len(wh.ndata))]
    x = wd.xgrid
    pa, pb = synth.mlp_preprocessing_exponents()
    params = synth.mlp_init(R)
    cen = fit.central_pdf()
    centrals = [oracle.dis(t.mask, t.fk, cen)[:, 0] for t in dis_t] + \
               [oracle.had(t.mask, t.fk, cen)[:, 0] for t in had_t]
    Cs, Ds = fit.covariances(centrals)
    return dict(dis_t=dis_t, had_t=had_t, x=x, pa=pa, pb=pb, params=params, Cs=Cs, D=np.concatenate(Ds))


def gpu_chain(c, case, fmt, steps=0, lr=0.0):
    """(chi2 [R], d chi2/d params [R][P]) after ``steps`` descent steps."""
    dis_t, had_t, x = case["dis_t"], case["had_t"], case["x"]
    hd = [c.load(t, fmt) for t in dis_t]
    hh = [c.load(t, fmt) for t in had_t]
    gd, gh = fkconv.fk_group_create(c.ctx, hd), fkconv.fk_group_create(c.ctx, hh)
    cv = fkconv.fk_load_covariance(c.ctx, case["Cs"])
    m, P = fkconv.fk_mlp_create(c.ctx, x, synth.MLP_H1, synth.MLP_H2, case["pa"], case["pb"])
    params = dev(case["params"])
    D = torch.from_numpy(case["D"]).cuda()
    Nd = sum(t.ndata for t in dis_t)
    R = params.shape[0]
    sig = torch.empty((Nd + sum(t.ndata for t in had_t), R), device="cuda")
    gpdf = torch.empty((14, len(x), R), device="cuda")
    gpar = torch.empty_like(params)
    hist = []
    for k in range(steps + 1):
        f = fkconv.fk_mlp_forward(c.ctx, m, params, 14, len(x))
        fkconv.fk_conv_dis(c.ctx, gd, f, out=sig[:Nd])
        fkconv.fk_conv_had(c.ctx, gh, f, out=sig[Nd:])
        chi, dchi = fkconv.fk_chi2(c.ctx, cv, sig, D)
        fkconv.fk_conv_backward(c.ctx, gd, None, dchi[:Nd].contiguous(), grad_pdf=gpdf)
        fkconv.fk_conv_backward(c.ctx, gh, f, dchi[Nd:].contiguous(), grad_pdf=gpdf, accumulate=True)
        fkconv.fk_mlp_backward(c.ctx, m, params, gpdf, grad_params=gpar)
        hist.append(chi.cpu().numpy().copy())
        if k < steps:
            fkconv.fk_sgd_update(c.ctx, params, gpar, lr)
    torch.cuda.synchronize()
    out = (hist, gpar.double().cpu().numpy(), params.double().cpu().numpy())
    fkconv.fk_mlp_destroy(c.ctx, m)
    fkconv.fk_unload_covariance(c.ctx, cv)
    for h in (gd, gh, *hd, *hh):
        fkconv.fk_unload_table(c.ctx, h)
    return out


def oracle_chain(case, params):
    x, pa, pb = case["x"], case["pa"], case["pb"]
    dis_t, had_t = case["dis_t"], case["had_t"]
    f = oracle.mlp_pdf(params, x, pa, pb, synth.MLP_H1, synth.MLP_H2)
    sig = np.concatenate([oracle.dis(t.mask, t.fk, f) for t in dis_t] + [oracle.had(t.mask, t.fk, f) for t in had_t])
    Ls = [oracle.cholesky(C) for C in case["Cs"]]
    chi, dsig = oracle.chi2(Ls, sig, case["D"])
    gpdf = np.zeros_like(f)
    off = 0
    for t in dis_t:
        gpdf += oracle.dis_grad(t.mask, t.fk, dsig[off:off + t.ndata], 14, len(x))
        off += t.ndata
    for t in had_t:
        gpdf += oracle.had_grad(t.mask, t.fk, f, dsig[off:off + t.ndata])
        off += t.ndata
    return chi, oracle.mlp_pdf_grad(params, x, pa, pb, synth.MLP_H1, synth.MLP_H2, gpdf)


@pytest.mark.parametrize("fmt,tol", [("f32", 1e-4), ("bf16", 5e-3)])
def test_fit_step_gradient_against_oracle(fmt, tol):
    case = fit_case(0.1, 0.05, 8)
    say(f"case fit step {fmt}: {sum(t.ndata for t in case['dis_t'])} DIS + "
        f"{sum(t.ndata for t in case['had_t'])} hadronic datapoints, R=8")
    with fkconv.Context(0) as c:
        hist, g, _ = gpu_chain(c, case, fmt)
    chi_r, g_r = oracle_chain(case, case["params"].astype(np.float64))
    ec = float(np.max(np.abs(hist[0] - chi_r) / chi_r))
    eg = oracle.normwise_rel(g.T, g_r.T)
    say(f"  chi2 {ec:.2e}, d chi2 / d params {eg:.2e}")
    assert ec <= tol and eg <= tol


def test_gradient_descent_lowers_chi2():
    """Ten descent steps whose first step moves no parameter by more than
    1e-3 lower every replica's chi2 at every step."""
    case = fit_case(0.1, 0.05, 4)
    with fkconv.Context(0) as c:
        _, g0, _ = gpu_chain(c, case, "f32")
        lr = 1e-3 / float(np.max(np.abs(g0)))
        hist, _, _ = gpu_chain(c, case, "f32", steps=10, lr=lr)
    h = np.array(hist)
    say(f"learning rate {lr:.3e}; chi2 per replica {np.array2string(h[0], precision=4)} -> "
        f"{np.array2string(h[-1], precision=4)}")
    assert np.all(np.isfinite(h))
    assert np.all(np.diff(h, axis=0) < 0)


def test_fit_step_full_size():
    """Global fit (20 DIS + 10 hadronic datasets, 10590 datapoints), R = 100."""
    t0 = time.time()
    case = fit_case(1.0, 1.0, 100)
    say(f"case full-size fit step: workload generated in {time.time() - t0:.1f}s")
    with fkconv.Context(0) as c:
        res = {fmt: gpu_chain(c, case, fmt) for fmt in ("f32", "bf16")}
    t0 = time.time()
    chi_r, g_r = oracle_chain(case, case["params"].astype(np.float64))
    for fmt, tol in (("f32", 1e-4), ("bf16", 5e-3)):
        hist, g, _ = res[fmt]
        ec = float(np.max(np.abs(hist[0] - chi_r) / chi_r))
        eg = oracle.normwise_rel(g.T, g_r.T)
        say(f"  {fmt}: chi2 {ec:.2e}, d chi2 / d params {eg:.2e} (oracle {time.time() - t0:.1f}s)")
        assert ec <= tol and eg <= tol


def test_autograd_chain_equals_explicit_calls():
    """network -> convolutions -> chi2 through torch.autograd gives the
    parameter gradient of the explicit chain of entry points (to FP32
    rounding: torch adds the two convolutions' PDF gradients itself)."""
    from paper_1909_10547_amd import autograd
    case = fit_case(0.1, 0.05, 4)
    with fkconv.Context(0) as c:
        _, g_explicit, _ = gpu_chain(c, case, "f32")
        dis_t, had_t, x = case["dis_t"], case["had_t"], case["x"]
        hd = [c.load(t, "f32") for t in dis_t]
        hh = [c.load(t, "f32") for t in had_t]
        gd, gh = fkconv.fk_group_create(c.ctx, hd), fkconv.fk_group_create(c.ctx, hh)
        cv = fkconv.fk_load_covariance(c.ctx, case["Cs"])
        m, _ = fkconv.fk_mlp_create(c.ctx, x, synth.MLP_H1, synth.MLP_H2, case["pa"], case["pb"])
        params = dev(case["params"]).requires_grad_(True)
        f = autograd.mlp_pdf(c.ctx, m, params, 14, len(x))
        sig = torch.cat([autograd.fk_conv(c.ctx, gd, f), autograd.fk_conv(c.ctx, gh, f)])
        chi = autograd.fk_chi2(c.ctx, cv, sig, torch.from_numpy(case["D"]).cuda())
        chi.sum().backward()
        torch.cuda.synchronize()
        g_auto = params.grad.double().cpu().numpy()
        fkconv.fk_mlp_destroy(c.ctx, m)
        fkconv.fk_unload_covariance(c.ctx, cv)
        for h in (gd, gh, *hd, *hh):
            fkconv.fk_unload_table(c.ctx, h)
    e = oracle.normwise_rel(g_auto.T, g_explicit.T)
    say(f"autograd chain vs explicit calls: {e:.2e}")
    assert e <= 1e-6
