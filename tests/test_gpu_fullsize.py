"""Parity at the full size of the hadronic global-fit workload (10 datasets,
N ~ U{20..1000}, 60 pairs, x-grid 50, R = 100), in the launch configuration
bench.py times (one group launch), on sampled outputs: the FP64 oracle
evaluates evenly spaced datapoints of every dataset for all replicas.

BF16 gate: normwise <= 5e-3 against FP64 over the sampled rows, plus the
stored-operand check (kernel arithmetic) on a few rows: the kernel and the
FP64 evaluation of the same stored operands differ only by FP32 summation,
whose error is bounded by a multiple of the sum of the absolute products
(not of |sigma|, which cancels), so the gate is 1e-5 of that sum."""
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


def test_hadronic_workload_full_size_sampled():
    t0 = time.time()
    w = synth.had_fit_workload()
    tabs = [w.table(d) for d in range(len(w.ndata))]
    pdf = w.pdf(100).astype(np.float32).astype(np.float64)
    say(f"generated {sum(t.ndata for t in tabs)} datapoints in {time.time() - t0:.1f}s")
    with fkconv.Context(0) as c:
        x = torch.from_numpy(pdf.astype(np.float32)).cuda()
        outs = {}
        for fmt in ("bf16", "f32"):
            t0 = time.time()
            hs = [c.load(t, fmt) for t in tabs]
            g = fkconv.fk_group_create(c.ctx, hs)
            say(f"loaded {fmt} in {time.time() - t0:.1f}s")
            outs[fmt] = fkconv.fk_conv_had(c.ctx, g, x).double().cpu().numpy()
            fkconv.fk_unload_table(c.ctx, g)
            for h in hs:
                fkconv.fk_unload_table(c.ctx, h)
    refs, gb, gf, off = [], [], [], 0
    qerr = qnorm = 0.0
    for d, t in enumerate(tabs):
        sel = np.unique(np.linspace(0, t.ndata - 1, 6).astype(int))
        sub = t.fk[sel]
        r = oracle.had(t.mask, sub, pdf)
        refs.append(r)
        gb.append(outs["bf16"][off + sel])
        gf.append(outs["f32"][off + sel])
        if d < 3:
            q = oracle.had_quantized(t.mask, sub[:2], pdf, "bf16")
            absterms = oracle.had(t.mask, np.abs(sub[:2]), np.abs(pdf))
            got = outs["bf16"][off + sel[:2]]
            qerr = max(qerr, float(np.max(np.abs(got - q) / absterms)))
            qnorm = max(qnorm, oracle.normwise_rel(got, q))
        off += t.ndata
    ref = np.concatenate(refs)
    eb = oracle.normwise_rel(np.concatenate(gb), ref)
    ef = oracle.normwise_rel(np.concatenate(gf), ref)
    say(f"full size, {ref.shape[0]} sampled datapoints x 100 replicas: bf16 {eb:.3e}, fp32 {ef:.3e}, "
        f"bf16 stored-operand {qerr:.3e} of sum|terms| (normwise {qnorm:.3e})")
    assert ef <= 1e-5
    assert eb <= 5e-3
    assert qerr <= 1e-5
    # the whole-output BF16 error against FP32 (itself within 1e-5 of FP64)
    e_all = oracle.normwise_rel(outs["bf16"], outs["f32"])
    say(f"bf16 vs fp32 over all {outs['f32'].shape[0]} datapoints: {e_all:.3e}")
    assert e_all <= 5e-3 - 1e-5
