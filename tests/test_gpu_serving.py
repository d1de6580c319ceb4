"""Serving loop: continuous batching of requests with mixed tables and
replica counts.  Every request's result must be bitwise the same as the
same request run alone through fk_conv_*, and match the FP64 oracle within
its format's tolerance; FP32 requests on a BF16 table are routed to the
linked FP32 table, and so are BF16 requests once the table's probe error is
above its tolerance.  Direct calls may overlap served passes on the same
table, and a pass waits for the stream that produced its PDF."""
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


def test_mixed_requests_equal_alone_runs():
    wd = synth.dis_fit_workload(scale=0.15)
    wh = synth.had_fit_workload(scale=0.04)
    cat = [("dis", wd.table(0)), ("dis", wd.table(1)), ("had", wh.table(0)), ("had", wh.table(1)),
           ("had", wh.table(2))]
    rng = np.random.default_rng(4)
    with fkconv.Context(0) as c:
        hb = [c.load(t, "bf16") for _, t in cat]
        hf = [c.load(t, "f32") for _, t in cat]
        for b, f in zip(hb, hf):
            fkconv.fk_table_set_fallback(c.ctx, b, f)
        fkconv.fk_serve_start(c.ctx, nslots=24, nstreams=3, request_budget_bytes=48 << 20)
        reqs = []
        for k in range(160):
            ti = int(rng.integers(0, len(cat)))
            R = int(rng.choice([1, 4, 16, 100]))
            prec = fkconv.FK_F32 if rng.random() < 0.2 else fkconv.FK_BF16
            pdf = synth.sample_pdf(synth.draw_pdf_params(np.random.default_rng([4, k])), wd.xgrid, R,
                                   0.05 if R > 1 else 0.0, np.random.default_rng([5, k]))
            x = torch.from_numpy(pdf.astype(np.float32)).cuda()
            out = torch.full((cat[ti][1].ndata, R), float("nan"), device="cuda")
            reqs.append((ti, R, prec, x, out))
        torch.cuda.synchronize()
        tickets = [fkconv.fk_submit(c.ctx, hb[ti], x, out, precision=prec) for ti, R, prec, x, out in reqs]
        t0 = time.time()
        pending = set(range(len(tickets)))
        while pending and time.time() - t0 < 60:
            for i in list(pending):
                st = fkconv.fk_poll(c.ctx, tickets[i])
                assert st != fkconv.FK_FAILED
                if st == fkconv.FK_DONE:
                    pending.discard(i)
        assert not pending, f"{len(pending)} requests not done"
        lat = []
        for t in tickets:
            a, b, d = fkconv.fk_ticket_times(c.ctx, t)
            assert a <= b <= d
            lat.append((d - a) * 1e-6)
        say(f"served {len(tickets)} requests in {time.time() - t0:.2f}s; latency p50 {np.percentile(lat, 50):.2f} ms "
            f"p99 {np.percentile(lat, 99):.2f} ms")
        fkconv.fk_serve_stop(c.ctx)
        nchk = 0
        for (ti, R, prec, x, out) in reqs:
            kind, tab = cat[ti]
            h = hf[ti] if prec == fkconv.FK_F32 else hb[ti]
            fn = fkconv.fk_conv_had if kind == "had" else fkconv.fk_conv_dis
            alone = fn(c.ctx, h, x)
            torch.cuda.synchronize()
            assert torch.equal(alone, out), f"request on table {ti} R={R} differs from its alone run"
            if nchk < 40:
                # FP32: the FP64 definition; BF16: the oracle on the same
                # rounded operands (kernel arithmetic)
                pdf32 = x.double().cpu().numpy()
                if prec == fkconv.FK_F32:
                    ref = (oracle.had if kind == "had" else oracle.dis)(tab.mask, tab.fk, pdf32)
                else:
                    ref = (oracle.had_quantized if kind == "had" else oracle.dis_quantized)(
                        tab.mask, tab.fk, pdf32, "bf16")
                e = oracle.normwise_rel(out.double().cpu().numpy(), ref)
                assert e <= 1e-5, (kind, R, prec, e)
                nchk += 1
        say("every request equals its alone run bitwise")


def test_serving_errors():
    w = synth.dis_fit_workload(scale=0.1)
    t = w.table(0)
    with fkconv.Context(0) as c:
        h = c.load(t, "bf16")
        x = torch.zeros((14, 50, 4), device="cuda")
        out = torch.zeros((t.ndata, 4), device="cuda")
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_submit(c.ctx, h, x, out)
        assert e.value.code == fkconv.FK_E_STATE
        fkconv.fk_serve_start(c.ctx, nslots=4, nstreams=2, request_budget_bytes=1 << 20)
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_submit(c.ctx, 987654, x, out)
        assert e.value.code == fkconv.FK_E_HANDLE
        big = torch.zeros((14, 50, 4000), device="cuda")
        bigo = torch.zeros((t.ndata, 4000), device="cuda")
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_submit(c.ctx, h, big, bigo)
        assert e.value.code == fkconv.FK_E_TOO_LARGE
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_unload_table(c.ctx, 987654)
        assert e.value.code == fkconv.FK_E_HANDLE
        fkconv.fk_serve_stop(c.ctx)


def _wait(c, tickets, limit=60.0):
    t0 = time.time()
    pending = set(tickets)
    while pending and time.time() - t0 < limit:
        for t in list(pending):
            st = fkconv.fk_poll(c.ctx, t)
            assert st != fkconv.FK_FAILED
            if st == fkconv.FK_DONE:
                pending.discard(t)
    assert not pending, f"{len(pending)} requests not done"


def test_direct_calls_overlap_serving_on_the_same_table():
    """Served passes run on scratch of their own: direct calls on the same
    table, issued while its requests are in flight, and the requests
    themselves both equal their alone runs bitwise."""
    wh = synth.had_fit_workload(scale=0.08)
    tab = wh.table(0)
    with fkconv.Context(0) as c:
        h = c.load(tab, "bf16")
        xs = [torch.from_numpy(wh.pdf(R).astype(np.float32)).cuda() for R in (16, 100, 4, 100)]
        alone = [fkconv.fk_conv_had(c.ctx, h, x).clone() for x in xs]
        torch.cuda.synchronize()
        say(f"case: table N={tab.ndata}, {len(xs)} PDF batches, serving + direct calls")
        fkconv.fk_serve_start(c.ctx, nslots=32, nstreams=4, request_budget_bytes=64 << 20)
        outs, tickets = [], []
        for k in range(48):
            x = xs[k % len(xs)]
            o = torch.full((tab.ndata, x.shape[2]), float("nan"), device="cuda")
            outs.append((k % len(xs), o))
            tickets.append(fkconv.fk_submit(c.ctx, h, x, o))
            # a direct call on the same table between the submissions
            y = fkconv.fk_conv_had(c.ctx, h, xs[(k + 1) % len(xs)])
            torch.cuda.synchronize()
            assert torch.equal(y, alone[(k + 1) % len(xs)]), f"direct call {k} differs"
        _wait(c, tickets)
        for i, o in outs:
            assert torch.equal(o, alone[i]), "served request differs from its alone run"
        fkconv.fk_serve_stop(c.ctx)
        say("direct calls and served requests equal their alone runs")


def test_request_waits_for_the_stream_that_produced_its_pdf():
    """The PDF is written on the caller's stream after a long kernel, and the
    request is submitted at once: the pass must wait for the recorded event."""
    wd = synth.dis_fit_workload(scale=0.2)
    tab = wd.table(0)
    R = 16
    with fkconv.Context(0) as c:
        h = c.load(tab, "bf16")
        src = torch.from_numpy(wd.pdf(R).astype(np.float32)).cuda()
        ref = fkconv.fk_conv_dis(c.ctx, h, src).clone()
        fkconv.fk_serve_start(c.ctx, nslots=8, nstreams=2, request_budget_bytes=16 << 20)
        x = torch.full_like(src, float("nan"))
        out = torch.full((tab.ndata, R), float("nan"), device="cuda")
        a = torch.randn(2048, 2048, device="cuda")
        torch.cuda.synchronize()
        say("case: DIS request submitted behind 20 GEMMs on the producing stream")
        for _ in range(20):  # keep the producing stream busy for a while
            a = torch.tanh(a @ a * 1e-3)
        x.copy_(src)
        t = fkconv.fk_submit(c.ctx, h, x, out)
        _wait(c, [t])
        assert torch.equal(out, ref)
        fkconv.fk_serve_stop(c.ctx)


def test_probe_routes_requests_to_the_fallback():
    """fk_table_probe measures the BF16 table against its FP32 fallback on the
    device; above the tolerance, BF16 requests are served by the fallback."""
    wh = synth.had_fit_workload(scale=0.05)
    tab = wh.table(1)
    R = 16
    with fkconv.Context(0) as c:
        hb = c.load(tab, "bf16")
        hf = c.load(tab, "f32")
        x = torch.from_numpy(wh.pdf(R).astype(np.float32)).cuda()
        with pytest.raises(fkconv.FKError) as e:
            fkconv.fk_table_probe(c.ctx, hb, x)
        assert e.value.code == fkconv.FK_E_STATE
        fkconv.fk_table_set_fallback(c.ctx, hb, hf)
        yb = fkconv.fk_conv_had(c.ctx, hb, x).clone()
        yf = fkconv.fk_conv_had(c.ctx, hf, x).clone()
        torch.cuda.synchronize()
        host = oracle.normwise_rel(yb.double().cpu().numpy(), yf.double().cpu().numpy())
        fkconv.fk_serve_start(c.ctx, nslots=8, nstreams=2, request_budget_bytes=16 << 20)
        for tol, want in ((1.0, yb), (0.0, yf)):
            err = fkconv.fk_table_probe(c.ctx, hb, x, tol=tol)
            say(f"probe tol={tol}: device error {err:.6e}, host {host:.6e}")
            assert abs(err - host) <= 1e-6 * host
            out = torch.full_like(yb, float("nan"))
            t = fkconv.fk_submit(c.ctx, hb, x, out)
            _wait(c, [t])
            assert torch.equal(out, want)
        fkconv.fk_serve_stop(c.ctx)
