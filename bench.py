#!/usr/bin/env python3
"""Throughput of the hadronic FK-table convolution on one MI355X.

Workload: the hadronic global-fit shape (10 datasets, N ~ U{20..1000}, 60
active ordered flavour pairs from a symmetric mask, x-grid of 50 points,
R = 100 PDF replicas), seeded synthetic tables and PDFs.  One step is one
convolution of all datasets (Eq. (1) of the paper, one group launch) with
the tables stored in BF16; the same step with FP32 tables is timed beside
it.  Tables and PDFs are resident in HBM before the timed region.

The JSON line carries the headline metric (datapoint*replicas/s, BF16), the
FP32 figure, per-step latency percentiles, errors, the roofline of the
dominant kernel (timed with HIP events on its launch stream by the library's
timing hook), the FP64 CPU oracle's throughput on a bounded sample, and the
timings of the other steps of the path (DIS convolution, adjoints, FP64
chi2, a full fit step).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "hadronic FK-conv datapoint·replicas/s bf16 vs fp32 @rel≤5e-3; p50/p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2516.6
COUNTERS = os.path.join(ROOT, "profiles", "had_fwd_bf16_had_fit_counters.json")
DIS_COUNTERS = os.path.join(ROOT, "profiles", "dis_fwd_dis_bandwidth_counters.json")
# the kernel source and the planner that hands it its work lists
KERNEL_SRC = [os.path.join(ROOT, "paper_1909_10547_amd", "csrc", f)
              for f in ("conv_kernels.hip", "runtime.cpp")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def counters():
    """The committed rocprofv3 counter summary of the forward kernel, if it
    was taken on the current kernel source and planner; else None."""
    try:
        d = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d


def traffic_from_counters():
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated), or None."""
    d = counters()
    return d.get("hbm_bytes_per_launch") if d else None


def mfma_from_counters():
    """MFMA busy fraction of the forward kernel from SQ_VALU_MFMA_BUSY_CYCLES
    (summed over SIMDs) / (GRBM_GUI_ACTIVE of one XCD x SIMDs), or None."""
    d = counters()
    return d.get("mfma") if d else None


def time_steps(fn, steps, warmup, torch):
    """Wall-clock ms per step over ``steps`` back-to-back steps (synchronized
    on both sides), then the per-step latencies of a second pass in which
    each step is bracketed by its own pair of events (the event records
    themselves separate the steps, so that pass is not the timed one)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in ev])
    return wall / steps * 1e3, per


def kernel_times(c, fn, steps, torch, fkconv):
    fkconv.fk_timing_read(c.ctx)
    fkconv.fk_timing_enable(c.ctx, True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    fkconv.fk_timing_enable(c.ctx, False)
    return fkconv.fk_timing_read(c.ctx)


FWD_KERNELS = {"had": (("had_stream", "had_stream_kernel"), ("had_fwd", "had_fwd_kernel")),
               "dis": (("dis_stream", "dis_stream_kernel"), ("dis_fwd", "dis_fwd_kernel"))}


def fwd_kernel(kt, kind):
    """(total ms, launches, kernel name) of the forward MFMA kernel that ran
    (the stream form, or the persistent/partial-sum form as fallback)."""
    for key, name in FWD_KERNELS[kind]:
        if kt[key][1]:
            return kt[key][0], kt[key][1], name
    return 0.0, 0, FWD_KERNELS[kind][0][1]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="shrink dataset sizes (quick checks only; the metric uses 1.0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip DIS/adjoint/chi2 rows")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving rows")
    ap.add_argument("--serve-quick", action="store_true",
                    help="serving: 2k requests at 2 rates (default: 10k requests at each of 6 rates)")
    ap.add_argument("--no-rsweep", action="store_true", help="skip the replica-count sweep")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured HBM-copy and BF16-GEMM ceilings")
    ap.add_argument("--no-dis-hbm", action="store_true",
                    help="skip the large DIS set used for the HBM-bandwidth rows")
    ap.add_argument("--dis-hbm-gib", type=float, default=2.0,
                    help="FP32 table size of the large DIS set")
    ap.add_argument("--no-table3", action="store_true", help="skip the Table 3 shape rows")
    ap.add_argument("--profile-bf16", action="store_true",
                    help="only load the BF16 tables and run the BF16 step (for profiler runs)")
    ap.add_argument("--profile-adj", action="store_true",
                    help="only load the BF16 tables and run the BF16 hadronic adjoint (for profiler runs)")
    ap.add_argument("--profile-dis", action="store_true",
                    help="only the DIS bandwidth set, BF16 (FP32 with --profile-f32), R=1 (for profiler runs)")
    ap.add_argument("--profile-nrep", type=int, default=0,
                    help="replica count of the --profile-bf16/--profile-adj runs (default: the workload's)")
    ap.add_argument("--profile-f32", action="store_true",
                    help="with --profile-bf16/--profile-adj/--profile-dis: load and run the FP32 tables instead")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain device copy of 1 GiB three times (HBM byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the workload shards by dataset, see DESIGN.md)", file=sys.stderr)
        return 2

    import torch

    import paper_1909_10547_amd  # noqa: F401
    from paper_1909_10547_amd import fkconv, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4}))
        return 0
    if args.profile_dis:
        base = synth.dis_fit_workload()
        scale = args.dis_hbm_gib * (1 << 30) / (9 * 50 * 4 * sum(base.ndata))
        wd = synth.dis_fit_workload(scale)
        c = fkconv.Context(0)
        hs = [c.load(wd.table(d), "f32" if args.profile_f32 else "bf16") for d in range(len(wd.ndata))]
        g = fkconv.fk_group_create(c.ctx, hs)
        x = torch.from_numpy(wd.pdf(1).astype(np.float32)).cuda()
        for _ in range(args.warmup + args.steps):
            fkconv.fk_conv_dis(c.ctx, g, x)
        torch.cuda.synchronize()
        print(json.dumps({"profile_dis_steps": args.warmup + args.steps}))
        return 0
    t_start = time.perf_counter()
    w = synth.had_fit_workload(args.scale)
    R = w.nrep
    log(f"generating hadronic tables: ndata={w.ndata}")
    tabs = []
    for d in range(len(w.ndata)):
        tabs.append(w.table(d))
    log(f"  generated in {time.perf_counter() - t_start:.1f}s")
    pdf64 = w.pdf(R).astype(np.float32).astype(np.float64)
    c = fkconv.Context(0)
    t0 = time.perf_counter()
    if args.profile_bf16 or args.profile_adj:
        fmt = "f32" if args.profile_f32 else "bf16"
        hb = [c.load(t, fmt) for t in tabs]
        if args.profile_nrep:
            R = args.profile_nrep
            pdf64 = w.pdf(R).astype(np.float32).astype(np.float64)
    else:
        hb = [c.load(t, "bf16") for t in tabs]
    gb = fkconv.fk_group_create(c.ctx, hb)
    if args.profile_bf16:
        x = torch.from_numpy(pdf64.astype(np.float32)).cuda()
        for _ in range(args.warmup + args.steps):
            fkconv.fk_conv_had(c.ctx, gb, x)
        torch.cuda.synchronize()
        print(json.dumps({"profile_bf16_steps": args.warmup + args.steps}))
        return 0
    if args.profile_adj:
        x = torch.from_numpy(pdf64.astype(np.float32)).cuda()
        Nt = sum(t.ndata for t in tabs)
        gbar = torch.ones((Nt, R), dtype=torch.float32, device="cuda")
        for _ in range(args.warmup + args.steps):
            fkconv.fk_conv_backward(c.ctx, gb, x, gbar)
        torch.cuda.synchronize()
        print(json.dumps({"profile_adj_steps": args.warmup + args.steps}))
        return 0
    hf = [c.load(t, "f32") for t in tabs]
    gf = fkconv.fk_group_create(c.ctx, hf)
    log(f"  packed and loaded bf16 + fp32 in {time.perf_counter() - t0:.1f}s")
    Ntot = sum(t.ndata for t in tabs)
    npairs = [int(t.mask.sum()) for t in tabs]
    X = tabs[0].fk.shape[-1]
    elems = sum(t.ndata * p * X * X for t, p in zip(tabs, npairs))
    # the forward streams the symmetric part over unordered pairs (a <= b)
    upper = [int(np.triu((t.mask | t.mask.T) != 0).sum()) for t in tabs]
    elems_fwd = sum(t.ndata * u * X * X for t, u in zip(tabs, upper))
    x = torch.from_numpy(pdf64.astype(np.float32)).cuda()
    out_b = torch.empty((Ntot, R), dtype=torch.float32, device="cuda")
    out_f = torch.empty_like(out_b)

    def step_b():
        fkconv.fk_conv_had(c.ctx, gb, x, out=out_b)

    def step_f():
        fkconv.fk_conv_had(c.ctx, gf, x, out=out_f)

    log("timing bf16 / fp32 steps")
    ms_b, per_b = time_steps(step_b, args.steps, args.warmup, torch)
    ms_f, per_f = time_steps(step_f, args.steps, args.warmup, torch)
    kt_b = kernel_times(c, step_b, args.steps, torch, fkconv)
    kt_f = kernel_times(c, step_f, args.steps, torch, fkconv)
    value_b = Ntot * R / (ms_b * 1e-3)
    value_f = Ntot * R / (ms_f * 1e-3)
    yb = out_b.double().cpu().numpy()
    yf = out_f.double().cpu().numpy()

    def normwise(y, r):
        num = np.sqrt(((y - r) ** 2).sum(axis=0))
        den = np.sqrt((r ** 2).sum(axis=0))
        return float(np.max(num / den))

    err_b_vs_f = normwise(yb, yf)
    had_ms, had_n, had_name = fwd_kernel(kt_b, "had")
    kern_ms = had_ms / max(had_n, 1)
    bytes_alg = elems_fwd * 2 + pdf64.size * 4 + Ntot * R * 4
    flops_alg = 2.0 * elems_fwd * R
    achieved = bytes_alg / (kern_ms * 1e-3) / 1e9
    traffic = traffic_from_counters()
    hadf_ms, hadf_n, _ = fwd_kernel(kt_f, "had")
    kern_f_ms = hadf_ms / max(hadf_n, 1)
    result = {
        "metric": METRIC,
        "value": value_b,
        "unit": "datapoint*replicas/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_b,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic: seeded FK tables and PDF replicas with the shapes of the hadronic global-fit workload",
        "config": {
            "workload": f"hadronic FK convolution, Eq. (1): {len(tabs)} datasets, {Ntot} datapoints, "
                        f"{npairs[0]} active flavour pairs, x-grid {X}, R={R} replicas",
            "datasets": len(tabs), "ndata": Ntot, "nrep": R, "nx": X,
            "active_pairs": npairs, "fk_elements": elems,
            "forward_stored_blocks": upper, "forward_stored_elements": elems_fwd, "scale": args.scale,
            "parallelism": "single GPU",
        },
        "latency_ms": {"p50": float(np.percentile(per_b, 50)), "p99": float(np.percentile(per_b, 99)),
                       "fp32_p50": float(np.percentile(per_f, 50)), "fp32_p99": float(np.percentile(per_f, 99))},
        "fp32": {"value": value_f, "ms_per_step": ms_f, "kernel_ms": kern_f_ms,
                 "tflops": flops_alg / (kern_f_ms * 1e-3) / 1e12},
        "speedup_bf16_over_fp32": value_b / value_f,
        "error": {"bf16_vs_fp32_normwise": err_b_vs_f,
                  "note": "fp32 is within 1e-5 of the FP64 oracle (tests); FP64 errors on the CPU sample below"},
        "roofline": {
            "kernel": f"{had_name}<bf16>",
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_alg,
            "kernel_ms": kern_ms,
            "mfma_tflops": flops_alg / (kern_ms * 1e-3) / 1e12,
            "mfma_frac_algorithmic": flops_alg / (kern_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS,
            "mfma_counters": mfma_from_counters(),
        },
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kt_b.items() if v[1]},
        # device memory held by the loaded tables (the analogue of the
        # paper's Table 2): forward copy over unordered pairs + the adjoint's
        # full rows + per-table plan scratch, per storage format
        "memory_bytes": {
            "bf16_tables": sum(fkconv.fk_table_info(c.ctx, h)["device_bytes"] for h in hb),
            "fp32_tables": sum(fkconv.fk_table_info(c.ctx, h)["device_bytes"] for h in hf),
            "context_total": fkconv.fk_memory(c.ctx)[0],
        },
    }

    # outputs of the rows below that the CPU-baseline leg checks against FP64
    checks = []
    if not args.no_peaks:
        log("measured ceilings: HBM copy, BF16 GEMM")
        pk = measured_peaks(torch)
        pk["mfma_bf16_register_tflops"] = fkconv.fk_measure_mfma_peak(c.ctx)
        pk["note"] += "; register-only v_mfma_f32_16x16x32_bf16 loop (fk_measure_mfma_peak)"
        result["measured_peaks"] = pk
        result["roofline"]["mfma_frac_of_register_peak"] = (result["roofline"]["mfma_tflops"] /
                                                            pk["mfma_bf16_register_tflops"])
        result["roofline"]["frac_of_measured"] = achieved / pk["hbm_copy_gbs"]
    if not args.no_rsweep:
        log("replica sweep")
        result.setdefault("rows", {})["had_bf16_rsweep"] = rsweep(c, w, gb, elems_fwd, Ntot, args, torch,
                                                                  fkconv)
    if not args.no_extras:
        log("extra rows: DIS, adjoints, chi2, fit step")
        result.setdefault("rows", {}).update(extras(c, w, tabs, gb, gf, x, out_b, R, args, torch, fkconv,
                                                    synth, checks))
    if not args.no_table3:
        log("Table 3 shapes (flattened form)")
        result.setdefault("rows", {})["table3"] = table3(c, args, torch, fkconv, synth, checks)
    if not args.no_serve:
        log("serving")
        result.setdefault("rows", {})["serving"] = serving(c, w, tabs, args, torch, fkconv, synth, checks)
    if not args.no_dis_hbm:
        log("large DIS set for HBM bandwidth")
        result.setdefault("rows", {})["dis_hbm"] = dis_hbm(c, args, torch, fkconv, synth)

    # The CPU-baseline leg: the FP64 oracle timed on the host (every datapoint
    # of the headline workload) and every error against FP64 in this line.
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline: the FP64 oracle on every datapoint (errors per dataset)")
        # calibrate on two datapoints; the whole workload when it fits in
        # about four times the sample budget, else evenly spaced rows
        t0 = time.perf_counter()
        oracle.had(tabs[0].mask, tabs[0].fk[:2], pdf64)
        per_dp = (time.perf_counter() - t0) / 2
        whole = per_dp * Ntot <= 4 * args.cpu_seconds
        k = Ntot if whole else max(1, int(args.cpu_seconds / per_dp / len(tabs)))
        refs, sels, nsamp, off = [], [], 0, 0
        per_ds = []
        t0 = time.perf_counter()
        for d, t in enumerate(tabs):
            sel = np.arange(t.ndata) if whole else np.unique(np.linspace(0, t.ndata - 1, min(k, t.ndata)).astype(int))
            sels.append(sel)
            ref = oracle.had(t.mask, t.fk[sel], pdf64)
            refs.append(ref)
            per_ds.append({"dataset": d, "ndata": t.ndata, "rows": int(len(sel)),
                           "bf16": normwise(yb[off + sel], ref), "fp32": normwise(yf[off + sel], ref)})
            nsamp += len(sel)
            off += t.ndata
        passes = 1
        # when the sample finished early, repeat it
        while time.perf_counter() - t0 < 0.8 * args.cpu_seconds:
            for t, sel in zip(tabs, sels):
                oracle.had(t.mask, t.fk[sel], pdf64)
            passes += 1
        el = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": passes * nsamp * R / el, "unit": "datapoint*replicas/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"all {Ntot} datapoints" if whole else f"{nsamp} of {Ntot} datapoints (evenly spaced in "
                       "every dataset)") + f" x {R} replicas, FP64, {passes} pass(es) in {el:.1f}s",
        }
        # the same oracle on one thread, on the first datasets' rows
        nth = oracle.num_threads()
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        n1 = 0
        for t, sel in zip(tabs, sels):
            sel1 = sel[: max(1, len(sel) // 32)]
            oracle.had(t.mask, t.fk[sel1], pdf64)
            n1 += len(sel1)
            if time.perf_counter() - t0 > 0.5 * args.cpu_seconds:
                break
        el1 = time.perf_counter() - t0
        oracle.set_num_threads(nth)
        result["cpu_baseline"]["value_1thread"] = n1 * R / el1
        result["cpu_baseline"]["sample_1thread"] = f"{n1} datapoints x {R} replicas, FP64, 1 thread, {el1:.1f}s"
        gotb = np.concatenate([yb[o + s_] for o, s_ in zip(np.cumsum([0] + [t.ndata for t in tabs]), sels)])
        gotf = np.concatenate([yf[o + s_] for o, s_ in zip(np.cumsum([0] + [t.ndata for t in tabs]), sels)])
        ref = np.concatenate(refs)
        worst_b = max(e["bf16"] for e in per_ds)
        result["error"].update({
            "rows_vs_fp64": "all rows" if whole else "evenly spaced rows of every dataset",
            "bf16_vs_fp64_normwise_all": normwise(gotb, ref),
            "fp32_vs_fp64_normwise_all": normwise(gotf, ref),
            "bf16_vs_fp64_max_over_datasets": worst_b,
            "fp32_vs_fp64_max_over_datasets": max(e["fp32"] for e in per_ds),
            "per_dataset": per_ds,
            "elementwise_bf16": oracle.error_report(gotb, ref),
            "elementwise_fp32": oracle.error_report(gotf, ref),
            "elementwise_note": "relative error of the outputs with |y*| >= 1e-3 max|y*|: p50, p99, max",
            "gate": "normwise per replica column, max over columns, per dataset: bf16 <= 5e-3, fp32 <= 1e-5",
            "gate_met": bool(worst_b <= 5e-3 and max(e["fp32"] for e in per_ds) <= 1e-5),
        })
        try:
            result["cpu_baseline"]["cpu_model"] = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                                                   if l.startswith("model name")][0]
        except (OSError, IndexError):
            pass
        # every other row's outputs against FP64
        fp64_checks(result, checks, oracle, normwise)

    fkconv.fk_unload_table(c.ctx, gb)
    fkconv.fk_unload_table(c.ctx, gf)
    c.close()
    result["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(result), flush=True)
    return 0


def fp64_checks(result, checks, oracle, normwise):
    """Errors against the FP64 oracle of the rows that appended their outputs
    to ``checks`` (part of the CPU-baseline leg)."""
    rows = result.get("rows", {})

    def gradwise(g, ref):
        # normwise over (flavour, x) per replica column, max over columns
        F, X, R = ref.shape
        return normwise(g.reshape(F * X, R), ref.reshape(F * X, R))

    for ck in checks:
        if ck["type"] == "dis":
            refs = [oracle.dis(m, fk, ck["pdf"]) for m, fk in ck["tables"]]
            gref = sum(oracle.dis_grad(m, fk, gb, ck["pdf"].shape[0], ck["pdf"].shape[1])
                       for (m, fk), gb in zip(ck["tables"],
                                              np.split(ck["gbar"], np.cumsum([fk.shape[0] for _, fk in ck["tables"]])[:-1])))
            offs = np.cumsum([0] + [r.shape[0] for r in refs])
            for fmt, y in ck["out"].items():
                per = [normwise(y[o:o + r.shape[0]], r) for o, r in zip(offs, refs)]
                rows[f"dis_{fmt}"]["error_vs_fp64"] = {
                    "rows": "all", "max_over_datasets": max(per), "all": normwise(y, np.concatenate(refs)),
                    "adjoint_normwise": gradwise(ck["grad"][fmt], gref),
                    "adjoint_weights": "seeded normal weights on every datapoint"}
        elif ck["type"] == "had_grad":
            gref = sum(oracle.had_grad(m, fk, ck["pdf"], gb) for (m, fk), gb in zip(ck["tables"], ck["gbar"]))
            for fmt, g in ck["grad"].items():
                rows[f"had_adjoint_{fmt}"]["error_vs_fp64"] = {
                    "normwise": gradwise(g, gref),
                    "weights": "seeded normal weights on 12 evenly spaced rows of every dataset, zero elsewhere"}
        elif ck["type"] == "chi2":
            Ls = [oracle.cholesky(C) for C in ck["C"]]
            ref, dref = oracle.chi2(Ls, ck["sigma"], ck["D"])
            rows["chi2_fp64"]["error_vs_fp64"] = {
                "chi2_max_rel": float(np.max(np.abs(ck["chi2"] - ref) / np.abs(ref))),
                "gradient_normwise": normwise(ck["grad"], dref),
                "note": "gradient returned in FP32"}
        elif ck["type"] == "flat":
            ref = oracle.flat_conv(ck["fk"], oracle.luminosity(ck["mask"], ck["pdf"]))
            rows["table3"][ck["index"]]["error_vs_fp64"] = {
                "sampled_outputs": list(ck["y"].shape),
                "max_abs_over_max_ref": float(np.max(np.abs(ck["y"] - ref)) / np.max(np.abs(ref)))}
        elif ck["type"] == "serving":
            err = 0.0
            for kind, m, fk, pdf, y in ck["items"]:
                ref = oracle.had(m, fk, pdf) if kind == "had" else oracle.dis(m, fk, pdf)
                err = max(err, oracle.normwise_rel(y, ref))
            rows["serving"]["error"]["fp32_reference_vs_fp64_max_normwise"] = err


def serving(c, w, had_tabs, args, torch, fkconv, synth, checks):
    """Continuous batching: the table catalogue of the serving workload (the
    20 DIS and 10 hadronic datasets plus two DIS and two hadronic tables with
    N = 2000), BF16 with FP32 fallback copies; each BF16 table is probed
    against its fallback on a 100-replica batch and routed to it when the
    error is above 5e-3; requests pick a table uniformly and R uniformly
    from {1, 4, 16, 100}; 20% ask for FP32.  Capacity is measured
    closed-loop (everything submitted at once), then Poisson streams at
    fractions of it; latency = submit -> completion seen by the loop.
    Afterwards every request of the last stream is re-run alone (bitwise
    equality is required) and its error is measured (against FP64 in the
    CPU-baseline leg, from the data this function appends to ``checks``)."""
    sw = synth.serving_workload(1.0)
    cat = list(sw.catalogue())
    hb, hf = [], []
    for kind, t in cat:
        hb.append(c.load(t, "bf16"))
        hf.append(c.load(t, "f32"))
        fkconv.fk_table_set_fallback(c.ctx, hb[-1], hf[-1])
    nd = [t.ndata for _, t in cat]
    kinds = [k for k, _ in cat]
    pools = {R: [torch.from_numpy(sw.request_pdf(R, k).astype(np.float32)).cuda() for k in range(4)]
             for R in sw.rep_choices}
    probe = [fkconv.fk_table_probe(c.ctx, h, pools[100][0], tol=5e-3) for h in hb]
    routed = [i for i, e in enumerate(probe) if e > 5e-3]
    fkconv.fk_serve_start(c.ctx, nslots=256, nstreams=4, request_budget_bytes=512 << 20)
    rng = np.random.default_rng(4)

    def run(nreq, rate):
        t_arr, tab, Rs, pseed = sw.requests(nreq, rate if rate else 1.0, len(cat))
        prec = np.where(rng.random(nreq) < 0.2, fkconv.FK_F32, fkconv.FK_BF16)
        outs = [torch.empty((nd[tab[i]], int(Rs[i])), dtype=torch.float32, device="cuda")
                for i in range(nreq)]
        torch.cuda.synchronize()
        tickets = [0] * nreq
        t0 = time.perf_counter()
        for i in range(nreq):
            if rate:
                dt = t_arr[i] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            x = pools[int(Rs[i])][int(pseed[i]) % 4]
            while True:
                try:
                    tickets[i] = fkconv.fk_submit(c.ctx, hb[tab[i]], x, outs[i], precision=int(prec[i]))
                    break
                except fkconv.FKError as e:
                    if e.code != fkconv.FK_E_QUEUE_FULL:
                        raise
                    time.sleep(1e-4)
        pend = set(range(nreq))
        while pend:
            for i in list(pend):
                st = fkconv.fk_poll(c.ctx, tickets[i])
                if st == fkconv.FK_FAILED:
                    raise RuntimeError(f"serving request {i} failed")
                if st == fkconv.FK_DONE:
                    pend.discard(i)
        wall = time.perf_counter() - t0
        lat = np.array([(lambda a, b, d: (d - a) * 1e-6)(*fkconv.fk_ticket_times(c.ctx, t)) for t in tickets])
        dprep = float(sum(nd[tab[i]] * Rs[i] for i in range(nreq)))
        return {"requests": nreq, "wall_s": wall, "req_per_s": nreq / wall, "dp_rep_per_s": dprep / wall,
                "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99))}, \
            (tab, Rs, prec, outs, pseed)

    res = {"probe": {"tol": 5e-3, "max_err": float(max(probe)), "routed_to_fp32": len(routed),
                     "tables": len(cat)}}
    nreq = 2000 if args.serve_quick else 10000
    cap, sample = run(nreq, None)
    res["closed_loop"] = cap
    fracs = (0.5, 0.9) if args.serve_quick else (0.25, 0.5, 0.75, 0.9, 1.0, 1.2)
    for f in fracs:
        r, sample = run(nreq, f * cap["req_per_s"])
        res[f"rate_{f:g}x"] = r
    fkconv.fk_serve_stop(c.ctx)

    # every request of the last stream: alone run (bitwise) and error.  The
    # reference of a request is its FP32 alone run on the GPU; the FP32
    # runs of every distinct (table, PDF batch) are checked against the FP64
    # oracle (DIS: every row; hadronic: 16 evenly spaced rows).
    tab, Rs, prec, outs, pseed = sample
    ref32, alone = {}, {}
    differ = 0
    err_b, err_f = [], []
    for i in range(len(outs)):
        key = (int(tab[i]), int(Rs[i]), int(pseed[i]) % 4)
        x = pools[key[1]][key[2]]
        fn = fkconv.fk_conv_had if kinds[key[0]] == "had" else fkconv.fk_conv_dis
        if key not in ref32:
            ref32[key] = fn(c.ctx, hf[key[0]], x)
            alone[key] = fn(c.ctx, hb[key[0]] if key[0] not in routed else hf[key[0]], x)
        want = ref32[key] if prec[i] == fkconv.FK_F32 else alone[key]
        differ += int(not torch.equal(want, outs[i]))
        r = ref32[key]
        num = ((outs[i].double() - r.double()) ** 2).sum(0).sqrt()
        den = (r.double() ** 2).sum(0).sqrt()
        e = float((num / den).max())
        (err_f if prec[i] == fkconv.FK_F32 else err_b).append(e)
    if differ:
        raise RuntimeError(f"serving: {differ} of {len(outs)} requests differ from their alone runs")
    items = []
    for (ti, R, k), y in ref32.items():
        t = cat[ti][1]
        pdf = pools[R][k].double().cpu().numpy()
        sel = (np.unique(np.linspace(0, t.ndata - 1, 16).astype(int)) if kinds[ti] == "had"
               else np.arange(t.ndata))
        items.append((kinds[ti], t.mask, t.fk[sel], pdf, y.double().cpu().numpy()[sel]))
    checks.append({"type": "serving", "items": items})
    res["alone_equals_mix"] = f"all {len(outs)} requests of the last stream bitwise equal to their alone runs"
    res["error"] = {
        "bf16_requests_max_normwise": float(max(err_b)) if err_b else None,
        "bf16_requests_over_5e-3": int(sum(e > 5e-3 for e in err_b)),
        "fp32_requests_max_normwise": float(max(err_f)) if err_f else None,
        "requests": len(outs),
        "reference": "each request's FP32 alone run; FP32 vs the FP64 oracle over every distinct "
                     "(table, PDF batch): DIS every row, hadronic 16 evenly spaced rows",
        "fp32_reference_vs_fp64_max_normwise": None,
    }
    for h in hb + hf:
        fkconv.fk_unload_table(c.ctx, h)
    return res


# Table 3 of the paper: (K, R) of the PDF matrix, (N, K) of the FK table, and
# the printed times in seconds (TensorFlow CPU, AVX, TensorFlow GPU, OpenCL;
# None where the table prints "~1"), which include the transfer to the GPU.
TABLE3 = [
    (35721, 1, 8, (1.10e-2, 1.57e-4, 4.14e-1, None)),
    (10 ** 6, 1, 8, (4.70e-2, 5.00e-3, 4.49e-1, None)),
    (10 ** 7, 1, 8, (3.20e-1, 5.70e-2, 7.90e-1, 1.38)),
    (10 ** 8, 1, 8, (2.90, 5.70e-1, 4.21, 6.31)),
    (35721, 100, 8, (6.90e-2, 1.60e-2, 4.31e-1, None)),
    (35721, 1000, 8, (1.50e-1, 1.69e-1, 5.63e-1, None)),
    (35721, 10 ** 4, 8, (1.12, 1.73, 1.92, 1.76)),
    (35721, 5 * 10 ** 4, 10, (5.33, 8.93, 7.83, 5.80)),
    (35721, 1, 100, (2.80e-2, 2.43e-3, 4.24e-1, None)),
    (35721, 1, 1000, (1.30e-1, 2.14e-2, 5.60e-1, None)),
    (35721, 1, 10 ** 4, (1.14, 2.16e-1, 1.93, 1.76)),
    (35721, 100, 100, (6.20e-2, 1.86e-1, 4.32e-1, None)),
    (35721, 1000, 1000, (3.00e-1, 21.61, 7.19e-1, 5.25)),
    (35721, 2000, 2000, (5.06, 86.13, 1.38, 15.97)),
]


def table3(c, args, torch, fkconv, synth, checks):
    """Every row of Table 3 in the flattened form the paper times: FK [N][K]
    against a PDF matrix [K][R].  For K = 35721 the matrix is the luminosity
    of 49 flavour pairs on 27 grid points, formed on the device from the PDF;
    the toy rows (K = 1e6 .. 1e8) use a seeded positive matrix.  Times (s):
    ``resident`` = the kernels alone (luminosity + product) on resident
    inputs; ``with_h2d`` = the paper's measurement: copy FK and the K x R
    matrix from pinned host memory, multiply, copy the result back;
    ``with_h2d_pdf`` (K = 35721) = copy FK and the PDF only and form the
    luminosity on the device.  Median of 5 after a warm-up."""
    rows = []
    mask = synth.table3_mask()
    s = torch.cuda.current_stream()

    def med(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts))

    for K, R, N, paper in TABLE3:
        lumi = K == 35721
        fk_h = torch.from_numpy(synth.table3_fk(N, K)).pin_memory()
        fk_d = torch.empty_like(fk_h, device="cuda")
        fk_d.copy_(fk_h)
        out_d = torch.empty((N, R), dtype=torch.float32, device="cuda")
        out_h = torch.empty((N, R), dtype=torch.float32).pin_memory()
        nw = fkconv.fk_flat_conv_workspace(c.ctx, N, K, R)
        work = torch.empty(max(nw // 4, 1), dtype=torch.float32, device="cuda")
        L_d = torch.empty((K, R), dtype=torch.float32, device="cuda")
        if lumi:
            pdf_h = torch.from_numpy(synth.table3_pdf(R).astype(np.float32)).pin_memory()
            pdf_d = pdf_h.cuda()
            fkconv.fk_luminosity(c.ctx, mask, pdf_d, lum=L_d)
            L_h = torch.empty((K, R), dtype=torch.float32).pin_memory()
            L_h.copy_(L_d)
        else:
            L_h = torch.from_numpy(synth.table3_matrix(K, R)).pin_memory()
            L_d.copy_(L_h)
        torch.cuda.synchronize()

        def resident():
            if lumi:
                fkconv.fk_luminosity(c.ctx, mask, pdf_d, lum=L_d)
            fkconv.fk_flat_conv(c.ctx, fk_d, L_d, out=out_d, work=work)

        def with_h2d():
            fk_d.copy_(fk_h, non_blocking=True)
            L_d.copy_(L_h, non_blocking=True)
            fkconv.fk_flat_conv(c.ctx, fk_d, L_d, out=out_d, work=work)
            out_h.copy_(out_d, non_blocking=True)

        def with_h2d_pdf():
            fk_d.copy_(fk_h, non_blocking=True)
            pdf_d.copy_(pdf_h, non_blocking=True)
            fkconv.fk_luminosity(c.ctx, mask, pdf_d, lum=L_d)
            fkconv.fk_flat_conv(c.ctx, fk_d, L_d, out=out_d, work=work)
            out_h.copy_(out_d, non_blocking=True)

        t_res = med(resident)
        t_h2d = med(with_h2d)
        row = {"pdf": [K, R], "fk": [N, K], "resident_s": t_res, "with_h2d_s": t_h2d,
               "kernel": "mfma" if (N > 16 and R > 16) else "stream",
               "flop": 2.0 * N * K * R, "bytes_resident": 4.0 * (N * K + K * R + N * R),
               "paper_s": {"tf_cpu": paper[0], "avx": paper[1], "tf_gpu": paper[2], "opencl": paper[3],
                           "note": "Table 3, including the transfer to the GPU; None = printed as ~1"}}
        if lumi:
            row["with_h2d_pdf_s"] = med(with_h2d_pdf)
        best = min(v for v in paper if v is not None)
        row["paper_best_over_with_h2d"] = best / t_h2d
        if lumi:
            # sampled outputs for the FP64 check (16 rows x 8 columns at most)
            resident()
            rr = np.unique(np.linspace(0, N - 1, min(N, 16)).astype(int))
            cc = np.unique(np.linspace(0, R - 1, min(R, 8)).astype(int))
            checks.append({"type": "flat", "index": len(rows), "mask": mask, "fk": fk_h.numpy()[rr],
                           "pdf": pdf_h.numpy()[:, :, cc], "y": out_d.double().cpu().numpy()[np.ix_(rr, cc)]})
        rows.append(row)
        log(f"  Table 3 row PDF {K}x{R} FK {N}x{K}: resident {t_res * 1e3:.3f} ms, with H2D "
            f"{t_h2d * 1e3:.3f} ms (paper best {best:.3g} s)")
        del fk_h, fk_d, out_d, out_h, work, L_d, L_h
        if lumi:
            del pdf_h, pdf_d
        torch.cuda.empty_cache()
    return rows


def measured_peaks(torch):
    """Ceilings measured on this GPU with library kernels: a 4 GiB device copy
    (HBM read + write) and an 8192^3 BF16 GEMM (hipBLASLt)."""
    n = 1 << 30
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * 4 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    m = 8192
    x = torch.randn((m, m), dtype=torch.bfloat16, device="cuda")
    y = torch.randn((m, m), dtype=torch.bfloat16, device="cuda")
    for _ in range(3):
        z = x @ y
    torch.cuda.synchronize()
    e0.record()
    for _ in range(20):
        z = x @ y
    e1.record()
    torch.cuda.synchronize()
    tflops = 20 * 2.0 * m ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del x, y, z
    torch.cuda.empty_cache()
    return {"hbm_copy_gbs": copy_gbs, "bf16_gemm_tflops": tflops,
            "note": "4 GiB float32 device copy counted as read + write; torch.matmul BF16 8192^3"}


def rsweep(c, w, gb, elems_fwd, Ntot, args, torch, fkconv):
    """The hadronic BF16 step at one replica (the table-streaming bound:
    HBM GB/s of algorithmic bytes, and from the FETCH/WRITE counters when
    they were taken on the current source) and at more replicas (passes of
    128 columns, each streaming the table once)."""
    out = {}
    cnt = counters()
    for R in (1, 256, 512, 1024):
        x = torch.from_numpy(w.pdf(R).astype(np.float32)).cuda()
        y = torch.empty((Ntot, R), dtype=torch.float32, device="cuda")
        fn = lambda: fkconv.fk_conv_had(c.ctx, gb, x, out=y)
        ms, per = time_steps(fn, max(5, args.steps // 2), 3, torch)
        kt = kernel_times(c, fn, max(5, args.steps // 2), torch, fkconv)
        kms = fwd_kernel(kt, "had")[0] / max(5, args.steps // 2)  # all passes of one step
        tfl = 2.0 * elems_fwd * R / (kms * 1e-3) / 1e12
        out[f"R{R}"] = {"ms_per_step": ms, "value": Ntot * R / (ms * 1e-3),
                        "had_fwd_ms_per_step": kms, "passes": (R + 127) // 128,
                        "mfma_tflops": tfl, "mfma_frac": tfl / PEAK_BF16_TFLOPS}
        if R == 1:
            byt = elems_fwd * 2 + x.numel() * 4 + Ntot * 4
            out["R1"]["achieved_gbs"] = byt / (kms * 1e-3) / 1e9
            r1 = (cnt or {}).get("forward_bf16_R1")
            if r1:
                out["R1"]["hbm_bytes_from_counters"] = r1["hbm_bytes_per_launch"]
                out["R1"]["hbm_gbs_from_counters"] = r1["hbm_bytes_per_launch"] / (kms * 1e-3) / 1e9
    return out


def dis_hbm(c, args, torch, fkconv, synth):
    """The global-DIS recipe (20 datasets, 9 of 14 flavours, 50 x-points) with
    every N scaled so the FP32 tables reach --dis-hbm-gib; 20 tables of
    1e5 datapoints each are far larger than the 256 MB last-level cache, so
    every step streams from HBM.  Reports GB/s of algorithmic table bytes."""
    base = synth.dis_fit_workload()
    per_dp = 9 * 50 * 4
    scale = args.dis_hbm_gib * (1 << 30) / (per_dp * sum(base.ndata))
    w = synth.dis_fit_workload(scale)
    tabs = [w.table(d) for d in range(len(w.ndata))]
    N = sum(t.ndata for t in tabs)
    elems = sum(t.fk.size for t in tabs)
    out = {"ndata": N, "fk_elements": elems, "peak_gbs": PEAK_HBM_GBS}
    try:
        dis_counters = json.load(open(DIS_COUNTERS))
        if dis_counters.get("kernel_sha256_16") != kernel_hash():
            dis_counters = None
    except (OSError, ValueError):
        dis_counters = None
    for fmt, nbytes in (("f32", 4), ("bf16", 2)):
        hs = [c.load(t, fmt) for t in tabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        for R in (1, 100):
            if fmt == "f32" and R == 100:
                continue
            x = torch.from_numpy(w.pdf(R).astype(np.float32)).cuda()
            y = torch.empty((N, R), dtype=torch.float32, device="cuda")
            fn = lambda: fkconv.fk_conv_dis(c.ctx, g, x, out=y)
            ms, _ = time_steps(fn, max(5, args.steps // 2), 2, torch)
            kt = kernel_times(c, fn, max(5, args.steps // 2), torch, fkconv)
            dms, dn, dname = fwd_kernel(kt, "dis")
            kms = dms / max(dn, 1)
            byt = elems * nbytes + N * R * 4
            out[f"{fmt}_R{R}"] = {"ms_per_step": ms, "kernel_ms": kms, "kernel": dname,
                                  "achieved_gbs": byt / (kms * 1e-3) / 1e9,
                                  "frac": byt / (kms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                                  "value": N * R / (ms * 1e-3)}
            if R == 1 and dis_counters:
                # HBM bytes per launch from FETCH_SIZE + WRITE_SIZE (calibrated),
                # over this run's kernel time
                hb = dis_counters["rows"][fmt]["hbm_bytes_per_launch"]
                out[f"{fmt}_R{R}"]["hbm_bytes_from_counters"] = hb
                out[f"{fmt}_R{R}"]["hbm_gbs_from_counters"] = hb / (kms * 1e-3) / 1e9
        fkconv.fk_unload_table(c.ctx, g)
        for h in hs:
            fkconv.fk_unload_table(c.ctx, h)
    return out


def extras(c, w, tabs, gb, gf, x, out_b, R, args, torch, fkconv, synth, checks):
    """Rows beyond the headline; the outputs that the CPU-baseline leg checks
    against FP64 are appended to ``checks``."""
    rows = {}
    # DIS global-like workload (20 datasets, R=100)
    w1 = synth.dis_fit_workload(args.scale)
    dtabs = [w1.table(d) for d in range(len(w1.ndata))]
    Nd = sum(t.ndata for t in dtabs)
    x1 = torch.from_numpy(w1.pdf(R).astype(np.float32)).cuda()
    dis_centrals = []
    dis_out, dis_grad = {}, {}
    for fmt in ("bf16", "f32"):
        hs = [c.load(t, fmt) for t in dtabs]
        g = fkconv.fk_group_create(c.ctx, hs)
        out = torch.empty((Nd, R), dtype=torch.float32, device="cuda")
        # microsecond-scale steps: ten times the step count (1000 by default)
        ms, per = time_steps(lambda: fkconv.fk_conv_dis(c.ctx, g, x1, out=out), 10 * args.steps, args.warmup,
                             torch)
        kt = kernel_times(c, lambda: fkconv.fk_conv_dis(c.ctx, g, x1, out=out), args.steps, torch, fkconv)
        gout = torch.ones((Nd, R), dtype=torch.float32, device="cuda")
        msb, _ = time_steps(lambda: fkconv.fk_conv_backward(c.ctx, g, None, gout), args.steps, args.warmup, torch)
        rows[f"dis_{fmt}"] = {"ndata": Nd, "ms_per_step": ms, "p50_ms": float(np.median(per)),
                              "p99_ms": float(np.percentile(per, 99)),
                              "kernel_ms": fwd_kernel(kt, "dis")[0] / max(fwd_kernel(kt, "dis")[1], 1),
                              "kernel": fwd_kernel(kt, "dis")[2],
                              "value": Nd * R / (ms * 1e-3), "adjoint_ms": msb}
        # outputs and gradients (seeded weights) for the FP64 check
        gw = torch.from_numpy(np.random.default_rng(11).standard_normal((Nd, R)).astype(np.float32)).cuda()
        dis_out[fmt] = out.double().cpu().numpy()
        dis_grad[fmt] = fkconv.fk_conv_backward(c.ctx, g, None, gw).double().cpu().numpy()
        dis_gw = gw.double().cpu().numpy()
        if fmt == "f32":
            cen = fkconv.fk_conv_dis(c.ctx, g, x1[:, :, :1].contiguous())[:, 0].double().cpu().numpy()
            off = 0
            for t in dtabs:
                dis_centrals.append(cen[off:off + t.ndata])
                off += t.ndata
        fkconv.fk_unload_table(c.ctx, g)
        for h in hs:
            fkconv.fk_unload_table(c.ctx, h)
    checks.append({"type": "dis", "tables": [(t.mask, t.fk) for t in dtabs],
                   "pdf": x1.double().cpu().numpy(), "out": dis_out, "grad": dis_grad, "gbar": dis_gw})
    # hadronic forward with FP8 (e4m3) tables: half the bytes of BF16, but
    # three mantissa bits, so outside the 5e-3 accuracy gate
    h8 = [c.load(t, "e4m3") for t in tabs]
    g8 = fkconv.fk_group_create(c.ctx, h8)
    out8 = torch.empty_like(out_b)
    ms8, per8 = time_steps(lambda: fkconv.fk_conv_had(c.ctx, g8, x, out=out8), args.steps, args.warmup, torch)
    kt8 = kernel_times(c, lambda: fkconv.fk_conv_had(c.ctx, g8, x, out=out8), args.steps, torch, fkconv)
    yb8 = out8.double().cpu().numpy()
    yref = out_b.double().cpu().numpy()
    num = np.sqrt(((yb8 - yref) ** 2).sum(axis=0))
    den = np.sqrt((yref ** 2).sum(axis=0))
    rows["had_fp8"] = {"ms_per_step": ms8, "value": out_b.shape[0] * R / (ms8 * 1e-3),
                       "kernel_ms": fwd_kernel(kt8, "had")[0] / max(fwd_kernel(kt8, "had")[1], 1),
                       "kernel": fwd_kernel(kt8, "had")[2],
                       "normwise_vs_bf16": float(np.max(num / den)),
                       "note": "e4m3 tables (OCP, per-datapoint power-of-two scale); fails the 5e-3 gate"}
    fkconv.fk_unload_table(c.ctx, g8)
    for h in h8:
        fkconv.fk_unload_table(c.ctx, h)
    # hadronic adjoint
    Ntot = out_b.shape[0]
    gbar = torch.ones((Ntot, R), dtype=torch.float32, device="cuda")
    # the adjoint streams the full symmetric rows: every ordered active pair
    elems_full = sum(int(t.fk.size) for t in tabs)
    for fmt, g in (("bf16", gb), ("f32", gf)):
        ms, _ = time_steps(lambda: fkconv.fk_conv_backward(c.ctx, g, x, gbar), args.steps, args.warmup, torch)
        kt = kernel_times(c, lambda: fkconv.fk_conv_backward(c.ctx, g, x, gbar), args.steps, torch, fkconv)
        kn = "had_adj_stream" if kt["had_adj_stream"][1] else "had_adj"
        rows[f"had_adjoint_{fmt}"] = {"ms_per_step": ms,
                                      "kernel_ms": kt[kn][0] / max(kt[kn][1], 1),
                                      "kernel": {"had_adj_stream": "had_stream_kernel<adjoint>",
                                                 "had_adj": "had_adj_kernel"}[kn],
                                      "table_bytes": elems_full * (2 if fmt == "bf16" else 4),
                                      "achieved_gbs": elems_full * (2 if fmt == "bf16" else 4)
                                      / (kt[kn][0] / max(kt[kn][1], 1) * 1e-3) / 1e9}
    # gradient of 12 evenly spaced rows of every dataset (seeded weights on
    # those rows, zero elsewhere) for the FP64 check
    rng = np.random.default_rng(12)
    gs = np.zeros((Ntot, R), dtype=np.float32)
    sels, off = [], 0
    for t in tabs:
        sel = np.unique(np.linspace(0, t.ndata - 1, 12).astype(int))
        gs[off + sel] = rng.standard_normal((len(sel), R)).astype(np.float32)
        sels.append(sel)
        off += t.ndata
    gsd = torch.from_numpy(gs).cuda()
    offs = np.cumsum([0] + [t.ndata for t in tabs])
    checks.append({"type": "had_grad", "tables": [(t.mask, t.fk[sel]) for t, sel in zip(tabs, sels)],
                   "gbar": [gs[o + sel].astype(np.float64) for o, sel in zip(offs, sels)],
                   "pdf": x.double().cpu().numpy(),
                   "grad": {fmt: fkconv.fk_conv_backward(c.ctx, g, x, gsd).double().cpu().numpy()
                            for fmt, g in (("bf16", gb), ("f32", gf))}})
    # FP64 chi2 over the datasets of both workloads (block-diagonal covariance)
    had_c = fkconv.fk_conv_had(c.ctx, gf, x[:, :, :1].contiguous())
    blocks, centrals, off = [], [], 0
    for t in tabs:
        centrals.append(had_c[off:off + t.ndata, 0].double().cpu().numpy())
        off += t.ndata
    fit = synth.global_fit_workload(args.scale)
    Cs, Ds = fit.covariances(dis_centrals + centrals)
    cv = fkconv.fk_load_covariance(c.ctx, Cs)
    D = torch.from_numpy(np.concatenate(Ds)).cuda()
    Nall = sum(C.shape[0] for C in Cs)
    sig = torch.randn((Nall, R), dtype=torch.float32, device="cuda")
    ms, _ = time_steps(lambda: fkconv.fk_chi2(c.ctx, cv, sig, D), args.steps, args.warmup, torch)
    rows["chi2_fp64"] = {"ndata": Nall, "blocks": len(Cs), "ms_per_step": ms}
    chi_g, dchi_g = fkconv.fk_chi2(c.ctx, cv, sig, D)
    checks.append({"type": "chi2", "C": Cs, "D": np.concatenate(Ds), "sigma": sig.double().cpu().numpy(),
                   "chi2": chi_g.cpu().numpy(), "grad": dchi_g.double().cpu().numpy()})
    # full fit step: DIS + hadronic forward (bf16), chi2, both adjoints
    hs = [c.load(t, "bf16") for t in dtabs]
    gd = fkconv.fk_group_create(c.ctx, hs)
    x1c = x  # both workloads share the x-grid [1e-7, 1] of 50 points
    sig_all = torch.empty((Nall, R), dtype=torch.float32, device="cuda")
    gpdf = torch.empty_like(x)

    def fit_step():
        Nd = sum(t.ndata for t in dtabs)
        fkconv.fk_conv_dis(c.ctx, gd, x1c, out=sig_all[:Nd])
        fkconv.fk_conv_had(c.ctx, gb, x1c, out=sig_all[Nd:])
        _, dchi = fkconv.fk_chi2(c.ctx, cv, sig_all, D)
        fkconv.fk_conv_backward(c.ctx, gd, None, dchi[:Nd].contiguous(), grad_pdf=gpdf)
        fkconv.fk_conv_backward(c.ctx, gb, x1c, dchi[Nd:].contiguous(), grad_pdf=gpdf, accumulate=True)

    ms, per = time_steps(fit_step, args.steps, args.warmup, torch)
    rows["fit_step_bf16"] = {"ms_per_step": ms, "p50_ms": float(np.median(per)),
                             "p99_ms": float(np.percentile(per, 99)),
                             "note": "DIS + hadronic forward, FP64 chi2 with gradient, both adjoints"}
    # the whole descent step on the device: network PDF on the x-grid, the
    # step above, the reverse pass through the network, the update
    pa, pb = synth.mlp_preprocessing_exponents()
    m, P = fkconv.fk_mlp_create(c.ctx, w.xgrid, synth.MLP_H1, synth.MLP_H2, pa, pb)
    params = torch.from_numpy(synth.mlp_init(R)).cuda()
    gpar = torch.empty_like(params)
    fnet = torch.empty_like(x)

    lr = [0.0]

    def descent_step():
        Nd = sum(t.ndata for t in dtabs)
        fkconv.fk_mlp_forward(c.ctx, m, params, fnet.shape[0], fnet.shape[1], pdf=fnet)
        fkconv.fk_conv_dis(c.ctx, gd, fnet, out=sig_all[:Nd])
        fkconv.fk_conv_had(c.ctx, gb, fnet, out=sig_all[Nd:])
        _, dchi = fkconv.fk_chi2(c.ctx, cv, sig_all, D)
        fkconv.fk_conv_backward(c.ctx, gd, None, dchi[:Nd].contiguous(), grad_pdf=gpdf)
        fkconv.fk_conv_backward(c.ctx, gb, fnet, dchi[Nd:].contiguous(), grad_pdf=gpdf, accumulate=True)
        fkconv.fk_mlp_backward(c.ctx, m, params, gpdf, grad_params=gpar)
        fkconv.fk_sgd_update(c.ctx, params, gpar, lr[0])

    # a rate whose first step moves no parameter by more than 1e-3
    descent_step()
    lr[0] = 1e-3 / float(gpar.abs().max())
    ms, per = time_steps(descent_step, args.steps, args.warmup, torch)
    rows["descent_step_bf16"] = {"ms_per_step": ms, "p50_ms": float(np.median(per)),
                                 "p99_ms": float(np.percentile(per, 99)), "replicas": R,
                                 "network": f"(x, ln x) -> {synth.MLP_H1} tanh -> {synth.MLP_H2} tanh -> 14, "
                                            f"{P} parameters per replica",
                                 "note": "network PDF, DIS + hadronic forward (BF16 tables), FP64 chi2, both "
                                         "adjoints, reverse pass through the network, gradient-descent update"}
    # the same step captured once in a HIP graph and replayed (every entry
    # point of the step only launches kernels: no allocation, no memset)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        descent_step()
    ms_g, per_g = time_steps(graph.replay, args.steps, args.warmup, torch)
    rows["descent_step_bf16"].update({"graph_ms_per_step": ms_g, "graph_p50_ms": float(np.median(per_g)),
                                      "graph_note": "one step captured in a HIP graph, replayed back to back"})
    del graph
    fkconv.fk_mlp_destroy(c.ctx, m)
    fkconv.fk_unload_table(c.ctx, gd)
    for h in hs:
        fkconv.fk_unload_table(c.ctx, h)
    fkconv.fk_unload_covariance(c.ctx, cv)
    return rows


if __name__ == "__main__":
    sys.exit(main())
