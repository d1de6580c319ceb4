"""Parity at the full sizes of the workloads, in the launch configuration
bench.py times (every dataset of a workload in one group launch, R = 100).

* Hadronic global fit (10 datasets, 4327 datapoints, 60 pairs, X = 50):
  every datapoint of every dataset against the FP64 oracle.  Gates per
  dataset: BF16 normwise <= 5e-3, FP32 normwise <= 1e-5, and per element
  the rounding bounds |y - y*| <= c sum|terms| (FP32: gamma_n with n the
  longest accumulation chain; BF16: 2u + u^2 for the two rounded factors
  of every term, u = 2^-8, plus gamma_n).  Whole datasets also against the
  stored-operand mode (same rounded operands: kernel arithmetic only).
* Hadronic adjoint at full size: the whole table streams; gbar is nonzero
  on a sample of datapoints only (the adjoint is linear in gbar), so the
  oracle evaluates just those rows.
* DIS global fit (20 datasets, 6263 datapoints, X = 50): every datapoint.
* Fit (both workloads, 30 covariance blocks, R = 100): chi2 against the
  oracle, dchi2/dsigma against the oracle at the GPU's sigma, and the
  gradient d chi2/d f projected on a random direction per replica against
  the oracle's five-point difference quotient, which is exact for chi2(t)
  (a polynomial of degree four in the step t).
* The DIS bandwidth set (FP32 tables of 2 GiB): sampled datapoints at the
  replica counts bench.py times.
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

U32 = 2.0 ** -24
U_BF16 = 2.0 ** -8


def gamma(n, u=U32):
    return n * u / (1 - n * u)


def comp(got, ref, absterms):
    """max over elements of |got - ref| / sum|terms| (an all-zero term sum
    must give an exact result)."""
    err = np.abs(got - ref)
    r = np.where(absterms > 0, err / np.where(absterms > 0, absterms, 1.0), np.where(err > 0, np.inf, 0.0))
    return float(np.max(r))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@functools.lru_cache(maxsize=None)
def had_tables():
    t0 = time.time()
    w = synth.had_fit_workload()
    tabs = [w.table(d) for d in range(len(w.ndata))]
    say(f"hadronic workload: {sum(t.ndata for t in tabs)} datapoints generated in {time.time() - t0:.1f}s")
    return w, tabs


@functools.lru_cache(maxsize=None)
def dis_tables():
    w = synth.dis_fit_workload()
    return w, [w.table(d) for d in range(len(w.ndata))]


def run_group(c, tabs, fmt, fn, pdfs, gbar=None):
    """Load ``tabs`` in ``fmt`` as one group, convolve every PDF of ``pdfs``
    (a list) and, with ``gbar``, run the adjoint of the first one."""
    hs = [c.load(t, fmt) for t in tabs]
    g = fkconv.fk_group_create(c.ctx, hs)
    outs, grad = [], None
    for k, pdf in enumerate(pdfs):
        x = dev(pdf)
        outs.append(fn(c.ctx, g, x).double().cpu().numpy())
        if gbar is not None and k == 0:
            grad = fkconv.fk_conv_backward(c.ctx, g, x, dev(gbar)).double().cpu().numpy()
    torch.cuda.synchronize()
    fkconv.fk_unload_table(c.ctx, g)
    for h in hs:
        fkconv.fk_unload_table(c.ctx, h)
    return outs, grad


# ---------------------------------------------------------------------------
# hadronic workload
# ---------------------------------------------------------------------------

ADJ_EVERY = 11  # adjoint: gbar nonzero on every 11th datapoint


@pytest.fixture(scope="module")
def had_full():
    w, tabs = had_tables()
    pdf = w.pdf(100).astype(np.float32).astype(np.float64)
    Ntot = sum(t.ndata for t in tabs)
    rows = np.zeros(Ntot, bool)
    rows[::ADJ_EVERY] = True
    gbar = np.where(rows[:, None], np.random.default_rng(5).normal(size=(Ntot, 100)), 0.0)
    gbar = gbar.astype(np.float32).astype(np.float64)
    outs, grads = {}, {}
    with fkconv.Context(0) as c:
        for fmt in ("bf16", "f32"):
            t0 = time.time()
            o, grads[fmt] = run_group(c, tabs, fmt, fkconv.fk_conv_had, [pdf], gbar)
            outs[fmt] = o[0]
            say(f"hadronic {fmt}: loaded, convolved and adjoint in {time.time() - t0:.1f}s")
    offs = np.cumsum([0] + [t.ndata for t in tabs])
    return dict(w=w, tabs=tabs, pdf=pdf, outs=outs, grads=grads, offs=offs, gbar=gbar, rows=rows)


# longest accumulation chain of one hadronic output: the MFMA product over a
# row's partners (<= F X), the epilogue over (a, alpha) (<= F X), the partial
# sums of the items, and the rounding of the stored FP32 operand
N_HAD = 2 * 14 * 50 + 16


@pytest.mark.parametrize("d", range(10))
def test_had_full_size_every_datapoint(had_full, d):
    tabs, pdf, outs, offs = had_full["tabs"], had_full["pdf"], had_full["outs"], had_full["offs"]
    t = tabs[d]
    sl = slice(offs[d], offs[d + 1])
    ref = oracle.had(t.mask, t.fk, pdf)
    absterms = oracle.had(t.mask, np.abs(t.fk), np.abs(pdf))
    eb = oracle.error_report(outs["bf16"][sl], ref)
    ef = oracle.error_report(outs["f32"][sl], ref)
    cf = comp(outs["f32"][sl], ref, absterms)
    cb = comp(outs["bf16"][sl], ref, absterms)
    say(f"hadronic dataset {d} (N={t.ndata}, all rows x 100 replicas): bf16 {eb['normwise']:.3e} "
        f"(elem p99 {eb.get('elem_p99', 0):.2e}), fp32 {ef['normwise']:.3e}; per element / sum|terms|: "
        f"fp32 {cf:.2e} (bound {gamma(N_HAD):.2e}), bf16 {cb:.2e} (bound {2 * U_BF16 + U_BF16 ** 2 + gamma(N_HAD):.2e})")
    assert eb["normwise"] <= 5e-3
    assert ef["normwise"] <= 1e-5
    assert cf <= gamma(N_HAD)
    assert cb <= 2 * U_BF16 + U_BF16 ** 2 + gamma(N_HAD)


@pytest.mark.parametrize("d", [7, 2, 1])
def test_had_full_size_whole_dataset_stored_operands(had_full, d):
    # same rounded operands as the kernel: only FP32 accumulation differs
    tabs, pdf, outs, offs = had_full["tabs"], had_full["pdf"], had_full["outs"], had_full["offs"]
    t = tabs[d]
    got = outs["bf16"][offs[d]:offs[d + 1]]
    q = oracle.had_quantized(t.mask, t.fk, pdf, "bf16")
    absterms = oracle.had(t.mask, np.abs(t.fk), np.abs(pdf))
    en = oracle.normwise_rel(got, q)
    ce = comp(got, q, absterms)
    say(f"hadronic dataset {d} bf16 vs stored operands (all {t.ndata} rows): normwise {en:.3e}, "
        f"per element {ce:.2e} of sum|terms|")
    assert en <= 1e-5
    assert ce <= gamma(N_HAD)


def test_had_full_size_adjoint(had_full):
    tabs, pdf, grads, offs = had_full["tabs"], had_full["pdf"], had_full["grads"], had_full["offs"]
    gbar, rows = had_full["gbar"], had_full["rows"]
    t0 = time.time()
    ref = np.zeros_like(pdf)
    for d, t in enumerate(tabs):
        sel = np.nonzero(rows[offs[d]:offs[d + 1]])[0]
        if len(sel):
            ref += oracle.had_grad(t.mask, t.fk[sel], pdf, gbar[offs[d] + sel])
    ef = oracle.normwise_rel(grads["f32"], ref)
    eb = oracle.normwise_rel(grads["bf16"], ref)
    say(f"hadronic adjoint, full tables, gbar on {int(rows.sum())} datapoints: fp32 {ef:.3e}, bf16 {eb:.3e} "
        f"(oracle {time.time() - t0:.1f}s)")
    assert ef <= 1e-5
    assert eb <= 5e-3


# ---------------------------------------------------------------------------
# DIS global workload
# ---------------------------------------------------------------------------

def test_dis_global_full_size_every_datapoint():
    w, tabs = dis_tables()
    pdf = w.pdf(100).astype(np.float32).astype(np.float64)
    with fkconv.Context(0) as c:
        outs = {fmt: run_group(c, tabs, fmt, fkconv.fk_conv_dis, [pdf])[0][0] for fmt in ("bf16", "f32")}
    n_dis = 9 * 50 + 4
    off = 0
    worst = {"bf16": 0.0, "f32": 0.0, "q": 0.0}
    for d, t in enumerate(tabs):
        sl = slice(off, off + t.ndata)
        off += t.ndata
        ref = oracle.dis(t.mask, t.fk, pdf)
        absterms = oracle.dis(t.mask, np.abs(t.fk), np.abs(pdf))
        q = oracle.dis_quantized(t.mask, t.fk, pdf, "bf16")
        eb, ef = oracle.normwise_rel(outs["bf16"][sl], ref), oracle.normwise_rel(outs["f32"][sl], ref)
        eq = oracle.normwise_rel(outs["bf16"][sl], q)
        cf = comp(outs["f32"][sl], ref, absterms)
        worst = {"bf16": max(worst["bf16"], eb), "f32": max(worst["f32"], ef), "q": max(worst["q"], eq)}
        assert eb <= 5e-3, (d, eb)
        assert ef <= 1e-5, (d, ef)
        assert eq <= 1e-5, (d, eq)
        assert cf <= gamma(n_dis), (d, cf)
    say(f"DIS global, {off} datapoints x 100 replicas, 20 datasets: worst dataset bf16 {worst['bf16']:.3e}, "
        f"fp32 {worst['f32']:.3e}, bf16 vs stored operands {worst['q']:.3e}")


# ---------------------------------------------------------------------------
# fit: both workloads, FP64 chi2, gradient
# ---------------------------------------------------------------------------

def test_fit_full_size_chi2_and_gradient():
    wh, had_t = had_tables()
    wd, dis_t = dis_tables()
    fit = synth.global_fit_workload()
    R = 100
    pdf = fit.pdf().astype(np.float32).astype(np.float64)
    cen = fit.central_pdf()
    t0 = time.time()
    centrals = [oracle.dis(t.mask, t.fk, cen)[:, 0] for t in dis_t] + \
               [oracle.had(t.mask, t.fk, cen)[:, 0] for t in had_t]
    Cs, Ds = fit.covariances(centrals)
    D = np.concatenate(Ds)
    Nd = sum(t.ndata for t in dis_t)
    rng = np.random.default_rng(9)
    v = pdf * rng.normal(size=pdf.shape)  # a direction per replica, on the scale of f

    with fkconv.Context(0) as c:
        hd = [c.load(t, "f32") for t in dis_t]
        hh = [c.load(t, "f32") for t in had_t]
        gd = fkconv.fk_group_create(c.ctx, hd)
        gh = fkconv.fk_group_create(c.ctx, hh)
        cv = fkconv.fk_load_covariance(c.ctx, Cs)
        x = dev(pdf)
        sig = torch.cat([fkconv.fk_conv_dis(c.ctx, gd, x), fkconv.fk_conv_had(c.ctx, gh, x)])
        chi, dchi = fkconv.fk_chi2(c.ctx, cv, sig, torch.from_numpy(D).cuda())
        g = fkconv.fk_conv_backward(c.ctx, gd, None, dchi[:Nd].contiguous())
        fkconv.fk_conv_backward(c.ctx, gh, x, dchi[Nd:].contiguous(), grad_pdf=g, accumulate=True)
        torch.cuda.synchronize()
        chi, dchi, g = chi.cpu().numpy(), dchi.double().cpu().numpy(), g.double().cpu().numpy()
        sig_gpu = sig.double().cpu().numpy()
        for h in (gd, gh, *hd, *hh):
            fkconv.fk_unload_table(c.ctx, h)
        fkconv.fk_unload_covariance(c.ctx, cv)
    say(f"fit: GPU chain done; {len(Cs)} covariance blocks, {D.shape[0]} datapoints")

    Ls = [oracle.cholesky(C) for C in Cs]

    def sigma(f):
        return np.concatenate([oracle.dis(t.mask, t.fk, f) for t in dis_t] +
                              [oracle.had(t.mask, t.fk, f) for t in had_t])

    c_ref, _ = oracle.chi2(Ls, sigma(pdf), D, want_grad=False)
    _, d_at_gpu = oracle.chi2(Ls, sig_gpu, D)
    ec = float(np.max(np.abs(chi - c_ref) / c_ref))
    ed = oracle.normwise_rel(dchi, d_at_gpu)
    # chi2 along f + t v is a quartic in t: the five-point quotient is exact
    h = 1e-3
    vals = {k: oracle.chi2(Ls, sigma(pdf + k * h * v), D, want_grad=False)[0] for k in (-2, -1, 1, 2)}
    dd = (-vals[2] + 8 * vals[1] - 8 * vals[-1] + vals[-2]) / (12 * h)
    proj = np.einsum("axr,axr->r", g, v)
    erel = np.abs(proj - dd) / np.abs(dd)
    say(f"fit (FP32 tables, R={R}): chi2 rel err {ec:.2e}, dchi2/dsigma {ed:.2e}, directional derivative "
        f"per replica max rel err {erel.max():.2e} (median {np.median(erel):.2e}); oracle {time.time() - t0:.1f}s")
    assert ec <= 1e-4
    assert ed <= 1e-6
    assert erel.max() <= 1e-4


# ---------------------------------------------------------------------------
# DIS bandwidth set (2 GiB of FP32 tables)
# ---------------------------------------------------------------------------

def test_dis_bandwidth_set_sampled_rows():
    base = synth.dis_fit_workload()
    scale = 2.0 * (1 << 30) / (9 * 50 * 4 * sum(base.ndata))
    w = synth.dis_fit_workload(scale)
    t0 = time.time()
    tabs = [w.table(d) for d in range(len(w.ndata))]
    N = sum(t.ndata for t in tabs)
    say(f"DIS bandwidth set: {N} datapoints generated in {time.time() - t0:.1f}s")
    sels, off = [], 0
    for t in tabs:
        sels.append(off + np.unique(np.linspace(0, t.ndata - 1, 100).astype(int)))
        off += t.ndata
    allsel = np.concatenate(sels)
    offs = np.cumsum([0] + [t.ndata for t in tabs])
    with fkconv.Context(0) as c:
        for fmt, Rs, tol in (("f32", (1,), 1e-5), ("bf16", (1, 100), 5e-3)):
            pdfs = [w.pdf(R).astype(np.float32).astype(np.float64) for R in Rs]
            outs = run_group(c, tabs, fmt, fkconv.fk_conv_dis, pdfs)[0]
            for R, pdf, got in zip(Rs, pdfs, outs):
                ref = np.concatenate([oracle.dis(t.mask, t.fk[s - s0], pdf)
                                      for t, s, s0 in zip(tabs, sels, offs)])
                e = oracle.normwise_rel(got[allsel], ref)
                say(f"DIS bandwidth set {fmt} R={R}: {len(allsel)} sampled datapoints, normwise {e:.3e}")
                assert e <= tol
