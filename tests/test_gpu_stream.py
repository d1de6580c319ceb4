"""The streaming hadronic forward kernel against the persistent one and the
oracle.  The two kernels split the x index over different numbers of waves,
so they sum in different orders: each must be within the FP32 summation
bound of the stored-operand oracle, and the stream kernel must be
deterministic and give every member table bitwise its rows of a group.  The
persistent kernel is selected with the context option FK_OPT_KERNELS.  The cases use the hadronic fit shape (x-grid of 50, groups of at
least two k-steps), where the stream kernel applies, over replica counts
that select every column-tile count."""
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


def kernels(c, stream):
    fkconv.fk_set_option(c.ctx, fkconv.FK_OPT_KERNELS,
                         fkconv.FK_KERNELS_STREAM if stream else fkconv.FK_KERNELS_ITEM)


def run(c, h, x, stream):
    kernels(c, stream)
    try:
        y = fkconv.fk_conv_had(c.ctx, h, x)
        torch.cuda.synchronize()
    finally:
        kernels(c, True)
    return y


@pytest.mark.parametrize("fmt", ["bf16", "f32", "e4m3"])
@pytest.mark.parametrize("R", [1, 16, 100, 200])
def test_stream_equals_persistent_and_oracle(fmt, R):
    w = synth.had_fit_workload(scale=0.12)
    tabs = [w.table(d) for d in range(len(w.ndata))]
    pdf = w.pdf(R).astype(np.float32).astype(np.float64)
    say(f"case fmt={fmt} R={R} ndata={[t.ndata for t in tabs]}")
    with fkconv.Context(0) as c:
        hs = [c.load(t, fmt) for t in tabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        x = torch.from_numpy(pdf.astype(np.float32)).cuda()
        ys = run(c, g, x, True)
        yp = run(c, g, x, False)
        assert torch.equal(run(c, g, x, True), ys), "stream kernel is not deterministic"
        # every member alone equals its rows of the group
        off = 0
        for t, h in zip(tabs, hs):
            y1 = run(c, h, x, True)
            assert torch.equal(y1, ys[off:off + t.ndata])
            off += t.ndata
        fkconv.fk_unload_table(c.ctx, g)
        for h in hs:
            fkconv.fk_unload_table(c.ctx, h)
    q = np.concatenate([oracle.had_quantized(t.mask, t.fk, pdf, fmt)
                        for t in tabs])
    absterms = np.concatenate([oracle.had(t.mask, np.abs(t.fk), np.abs(pdf)) for t in tabs])
    # FP32 summation bound, as for the other stored-operand gates; the FP8
    # MFMA gets the looser gate of the FP8 forward tests
    tol = 1e-4 if fmt == "e4m3" else 1e-5
    for name, y in (("stream", ys), ("persistent", yp)):
        e = float(np.max(np.abs(y.double().cpu().numpy() - q) / absterms))
        say(f"  {name}: stored-operand error {e:.2e} of sum|terms|")
        assert e <= tol, name


@pytest.mark.parametrize("fmt", ["bf16", "f32", "e4m3"])
@pytest.mark.parametrize("R", [1, 16, 100, 200])
def test_dis_stream_against_partial_sum_kernel_and_oracle(fmt, R):
    """DIS: the stream kernel (one accumulation chain per row, written
    directly) against the partial-sum kernel and the stored-operand oracle."""
    w = synth.dis_fit_workload(scale=0.15)
    tabs = [w.table(d) for d in range(len(w.ndata))]
    pdf = w.pdf(R).astype(np.float32).astype(np.float64)
    say(f"case DIS fmt={fmt} R={R} ndata={[t.ndata for t in tabs]}")
    with fkconv.Context(0) as c:
        hs = [c.load(t, fmt) for t in tabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        x = torch.from_numpy(pdf.astype(np.float32)).cuda()

        def dis(h, stream):
            kernels(c, stream)
            try:
                y = fkconv.fk_conv_dis(c.ctx, h, x)
                torch.cuda.synchronize()
            finally:
                kernels(c, True)
            return y

        ys = dis(g, True)
        yp = dis(g, False)
        assert torch.equal(dis(g, True), ys), "DIS stream kernel is not deterministic"
        off = 0
        for t, h in zip(tabs, hs):
            assert torch.equal(dis(h, True), ys[off:off + t.ndata])
            off += t.ndata
        fkconv.fk_unload_table(c.ctx, g)
        for h in hs:
            fkconv.fk_unload_table(c.ctx, h)
    q = np.concatenate([oracle.dis_quantized(t.mask, t.fk, pdf, fmt) for t in tabs])
    absterms = np.concatenate([oracle.dis(t.mask, np.abs(t.fk), np.abs(pdf)) for t in tabs])
    tol = 1e-4 if fmt == "e4m3" else 1e-5
    for name, y in (("stream", ys), ("partial-sum", yp)):
        e = float(np.max(np.abs(y.double().cpu().numpy() - q) / np.where(absterms > 0, absterms, 1.0)))
        say(f"  {name}: stored-operand error {e:.2e} of sum|terms|")
        assert e <= tol, name


def test_timing_kinds_name_the_kernel_that_ran():
    """Kernel timing books the stream kernels under their own kinds, so a
    timing read says which forward kernel a call used."""
    w = synth.had_fit_workload(scale=0.05)
    t = w.table(0)
    wd = synth.dis_fit_workload(scale=0.05)
    td = wd.table(0)
    R = 16
    with fkconv.Context(0) as c:
        h = c.load(t, "bf16")
        hd = c.load(td, "bf16")
        x = torch.from_numpy(w.pdf(R).astype(np.float32)).cuda()
        xd = torch.from_numpy(wd.pdf(R).astype(np.float32)).cuda()
        for stream in (True, False):
            kernels(c, stream)
            try:
                fkconv.fk_timing_read(c.ctx)
                fkconv.fk_timing_enable(c.ctx, True)
                fkconv.fk_conv_had(c.ctx, h, x)
                fkconv.fk_conv_dis(c.ctx, hd, xd)
                torch.cuda.synchronize()
                fkconv.fk_timing_enable(c.ctx, False)
                kt = fkconv.fk_timing_read(c.ctx)
            finally:
                kernels(c, True)
            say(f"stream={stream}: {({k: v[1] for k, v in kt.items() if v[1]})}")
            assert kt["stage"][1] == 2
            if stream:
                assert kt["had_stream"][1] == 1 and kt["had_fwd"][1] == 0
                assert kt["dis_stream"][1] == 1 and kt["dis_fwd"][1] == 0
                assert kt["fwd_reduce"][1] == 1  # the hadronic items' partial sums
            else:
                assert kt["had_fwd"][1] == 1 and kt["had_stream"][1] == 0
                assert kt["dis_fwd"][1] == 1 and kt["dis_stream"][1] == 0
                assert kt["fwd_reduce"][1] == 2
        fkconv.fk_unload_table(c.ctx, h)
        fkconv.fk_unload_table(c.ctx, hd)


def run_adj(c, h, x, gbar, stream):
    kernels(c, stream)
    try:
        g = fkconv.fk_conv_backward(c.ctx, h, x, gbar)
        torch.cuda.synchronize()
    finally:
        kernels(c, True)
    return g


@pytest.mark.parametrize("fmt", ["bf16", "f32", "e4m3"])
@pytest.mark.parametrize("R", [1, 16, 100, 200])
def test_adjoint_stream_against_item_kernel_and_oracle(fmt, R):
    """Hadronic adjoint: the stream kernel (gradient rows in registers, one
    record per block pair) against the per-item kernel and the oracle's
    gradient of the stored operands, on a group of tables with partial last
    blocks and odd block counts."""
    w = synth.had_fit_workload(scale=0.12)
    tabs = [w.table(d) for d in range(len(w.ndata))]
    pdf = w.pdf(R).astype(np.float32).astype(np.float64)
    N = sum(t.ndata for t in tabs)
    gbar = np.random.default_rng(R).normal(size=(N, R)).astype(np.float32).astype(np.float64)
    say(f"case fmt={fmt} R={R} ndata={[t.ndata for t in tabs]}")
    with fkconv.Context(0) as c:
        hs = [c.load(t, fmt) for t in tabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        x = torch.from_numpy(pdf.astype(np.float32)).cuda()
        gb = torch.from_numpy(gbar.astype(np.float32)).cuda()
        fkconv.fk_timing_read(c.ctx)
        fkconv.fk_timing_enable(c.ctx, True)
        gs = run_adj(c, g, x, gb, True)
        fkconv.fk_timing_enable(c.ctx, False)
        kt = fkconv.fk_timing_read(c.ctx)
        gp = run_adj(c, g, x, gb, False)
        assert torch.equal(run_adj(c, g, x, gb, True), gs), "stream adjoint is not deterministic"
        fkconv.fk_unload_table(c.ctx, g)
        for h in hs:
            fkconv.fk_unload_table(c.ctx, h)
    used = "stream" if kt["had_adj_stream"][1] else "per-item"
    say(f"  default path: {used} kernel")
    if fmt != "e4m3":
        assert kt["had_adj_stream"][1] > 0, "the stream adjoint should apply to these tables"
    q = np.zeros_like(pdf)
    absterms = np.zeros_like(pdf)
    off = 0
    for t in tabs:
        q += oracle.had_grad_quantized(t.mask, t.fk, pdf, gbar[off:off + t.ndata], fmt)
        absterms += oracle.had_grad(t.mask, np.abs(t.fk), np.abs(pdf), np.abs(gbar[off:off + t.ndata]))
        off += t.ndata
    tol = 1e-4 if fmt == "e4m3" else 1e-5
    scale = np.where(absterms > 0, absterms, 1.0)
    for name, y in (("stream", gs), ("per-item", gp)):
        e = float(np.max(np.abs(y.double().cpu().numpy() - q) / scale))
        say(f"  {name}: stored-operand error {e:.2e} of sum|terms|")
        assert e <= tol, name


@pytest.mark.parametrize("X,expect_adj_stream", [(8, None), (20, None), (64, True), (72, False)])
def test_stream_kernels_across_grid_sizes(X, expect_adj_stream):
    """Forward and adjoint at x-grids of 8 (each wave one x index), 20, 64
    (the most gradient rows a wave keeps in registers) and 72 (the adjoint
    falls back to the per-item kernel): stored-operand oracle, and, where
    the grid decides it, the path that ran (read from the kernel timing
    kinds; at 8 and 20 it depends on the group sizes)."""
    rng = np.random.default_rng(X)
    xg = synth.xgrid_geom(1e-6, 0.95, X)
    N, R = 53, 16
    # many ordered pairs, so that every group lasts the ring's eight k-steps
    t = synth.draw_general_had_table(rng, xg, N, npairs=120)
    f = synth.sample_pdf(synth.draw_pdf_params(rng), xg, R, 0.05, rng).astype(np.float32).astype(np.float64)
    gbar = rng.normal(size=(N, R)).astype(np.float32).astype(np.float64)
    say(f"case X={X} N={N} R={R} pairs={int(t.mask.sum())}")
    with fkconv.Context(0) as c:
        h = c.load(t, "bf16")
        x = torch.from_numpy(f.astype(np.float32)).cuda()
        gb = torch.from_numpy(gbar.astype(np.float32)).cuda()
        fkconv.fk_timing_read(c.ctx)
        fkconv.fk_timing_enable(c.ctx, True)
        y = fkconv.fk_conv_had(c.ctx, h, x)
        g = fkconv.fk_conv_backward(c.ctx, h, x, gb)
        torch.cuda.synchronize()
        fkconv.fk_timing_enable(c.ctx, False)
        kt = fkconv.fk_timing_read(c.ctx)
        fkconv.fk_unload_table(c.ctx, h)
    say(f"  kernels: {({k: v[1] for k, v in kt.items() if v[1]})}")
    assert (kt["had_adj_stream"][1] > 0) != (kt["had_adj"][1] > 0)
    if expect_adj_stream is not None:
        assert (kt["had_adj_stream"][1] > 0) == expect_adj_stream
    qy = oracle.had_quantized(t.mask, t.fk, f, "bf16")
    ay = oracle.had(t.mask, np.abs(t.fk), np.abs(f))
    ey = float(np.max(np.abs(y.double().cpu().numpy() - qy) / np.where(ay > 0, ay, 1.0)))
    qg = oracle.had_grad_quantized(t.mask, t.fk, f, gbar, "bf16")
    ag = oracle.had_grad(t.mask, np.abs(t.fk), np.abs(f), np.abs(gbar))
    eg = float(np.max(np.abs(g.double().cpu().numpy() - qg) / np.where(ag > 0, ag, 1.0)))
    say(f"  forward {ey:.2e}, adjoint {eg:.2e} of sum|terms|")
    assert ey <= 1e-5 and eg <= 1e-5
