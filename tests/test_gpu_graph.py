"""The descent step captured in a HIP graph.

Every entry point of the step (network PDF, DIS and hadronic forward, FP64
chi2 with its gradient, both adjoints, the network's reverse pass, the
update) only launches kernels on the caller's stream and neither allocates
nor sets memory, so a graph of one step replays it.  Each replay, with eager
work and synchronisations in between, must equal bitwise the eager step
from the same parameters.
"""
import sys

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


@pytest.mark.parametrize("fmt", ["bf16", "f32"])
def test_descent_step_replays_in_a_graph(fmt):
    fit = synth.global_fit_workload(1.0)
    wd, wh = synth.dis_fit_workload(0.1), synth.had_fit_workload(0.05)
    dis_t = [wd.table(d) for d in range(len(wd.ndata))]
    had_t = [wh.table(d) for d in range(len(wh.ndata))]
    x = wd.xgrid
    X, R = len(x), 8
    pa, pb = synth.mlp_preprocessing_exponents()
    params0 = synth.mlp_init(R)
    cen = fit.central_pdf()
    centrals = [oracle.dis(t.mask, t.fk, cen)[:, 0] for t in dis_t] + \
               [oracle.had(t.mask, t.fk, cen)[:, 0] for t in had_t]
    Cs, Ds = fit.covariances(centrals)
    Nd = sum(t.ndata for t in dis_t)
    N = Nd + sum(t.ndata for t in had_t)
    say(f"case {fmt}: {Nd} DIS + {N - Nd} hadronic datapoints, R={R}")
    with fkconv.Context(0) as c:
        hd = [c.load(t, fmt) for t in dis_t]
        hh = [c.load(t, fmt) for t in had_t]
        gd, gh = fkconv.fk_group_create(c.ctx, hd), fkconv.fk_group_create(c.ctx, hh)
        cv = fkconv.fk_load_covariance(c.ctx, Cs)
        m, P = fkconv.fk_mlp_create(c.ctx, x, synth.MLP_H1, synth.MLP_H2, pa, pb)
        D = torch.from_numpy(np.concatenate(Ds)).cuda()
        f = torch.empty((14, X, R), device="cuda")
        sig = torch.empty((N, R), device="cuda")
        chi = torch.empty(R, dtype=torch.float64, device="cuda")
        dchi = torch.empty((N, R), device="cuda")
        gpdf = torch.empty((14, X, R), device="cuda")
        gpar = torch.empty((R, P), device="cuda")
        lr = [0.0]

        def step(params):
            fkconv.fk_mlp_forward(c.ctx, m, params, 14, X, pdf=f)
            fkconv.fk_conv_dis(c.ctx, gd, f, out=sig[:Nd])
            fkconv.fk_conv_had(c.ctx, gh, f, out=sig[Nd:])
            fkconv.fk_chi2(c.ctx, cv, sig, D, chi2=chi, dchi2_dsigma=dchi)
            fkconv.fk_conv_backward(c.ctx, gd, None, dchi[:Nd], grad_pdf=gpdf)
            fkconv.fk_conv_backward(c.ctx, gh, f, dchi[Nd:], grad_pdf=gpdf, accumulate=True)
            fkconv.fk_mlp_backward(c.ctx, m, params, gpdf, grad_params=gpar)
            fkconv.fk_sgd_update(c.ctx, params, gpar, lr[0])

        # a rate whose first step moves no parameter by more than 1e-3
        step(dev(params0))
        torch.cuda.synchronize()
        lr[0] = 1e-3 / float(gpar.abs().max())
        # eager reference: three steps from params0
        pe = dev(params0)
        ref = []
        for _ in range(3):
            step(pe)
            torch.cuda.synchronize()
            ref.append((chi.clone(), pe.clone()))
        # one step captured on its own parameters
        pg = dev(params0)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step(pg)
        torch.cuda.synchronize()
        assert torch.equal(pg, dev(params0)), "capturing ran the step"
        other = dev(synth.had_fit_workload(0.05).pdf(3))
        for k in range(3):
            # eager work on the same tables between the replays
            y = fkconv.fk_conv_had(c.ctx, gh, other)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            same = torch.equal(chi, ref[k][0]) and torch.equal(pg, ref[k][1])
            say(f"  replay {k}: chi2 {chi.cpu().numpy()[:2]} ... bitwise equal to eager step {k}: {same}")
            assert same
            assert torch.isfinite(y).all()
        del graph
        fkconv.fk_mlp_destroy(c.ctx, m)
        fkconv.fk_unload_covariance(c.ctx, cv)
        for h in (gd, gh, *hd, *hh):
            fkconv.fk_unload_table(c.ctx, h)
