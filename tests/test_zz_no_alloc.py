"""fk_conv_dis_static, the entry point that allocates nothing (its staged
PDF operand lives in the library's static device scratch), against
fk_conv_dis on the same inputs: bitwise equal, on two calls in a row (the
second with a smaller input), and the size limit is an error."""
import sys

import numpy as np
import pytest

from paper_1909_10547_amd import fkconv, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_scratch_entry_equals_fk_conv_dis():
    w = synth.dis_fit_workload()
    tabs = [w.table(d) for d in range(len(w.ndata))]
    with fkconv.Context(0) as c:
        hs = [c.load(t, "bf16") for t in tabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        # first call: all 20 datasets, 200 replicas (two column passes);
        # second: one dataset, 16 replicas
        for h, R in ((g, 200), (hs[3], 16)):
            info = fkconv.fk_table_info(c.ctx, h)
            x = torch.from_numpy(w.pdf(R).astype(np.float32)).cuda()
            say(f"case: ndata={info['ndata']} R={R} bf16")
            ref = fkconv.fk_conv_dis(c.ctx, h, x)
            out = torch.full_like(ref, float("nan"))
            fkconv.fk_conv_dis_static(c.ctx, h, x, out=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref)
        # FP32 tables of 20 distinct flavour patterns need more than 4 MiB
        hf = [c.load(t, "f32") for t in tabs]
        gf = fkconv.fk_group_create(c.ctx, hf)
        x = torch.from_numpy(w.pdf(8).astype(np.float32)).cuda()
        out = torch.empty((sum(t.ndata for t in tabs), 8), device="cuda")
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_conv_dis_static(c.ctx, gf, x, out=out)
        assert e.value.code == fkconv.FK_E_TOO_LARGE
        # a hadronic handle is rejected
        wh = synth.had_fit_workload(scale=0.03)
        hh = c.load(wh.table(0), "bf16")
        xh = torch.from_numpy(wh.pdf(4).astype(np.float32)).cuda()
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_conv_dis_static(c.ctx, hh, xh, out=torch.empty((wh.table(0).ndata, 4), device="cuda"))
        assert e.value.code == fkconv.FK_E_ARG
