"""bench.py's host logic on the CPU: the one-GPU contract and the FP64 error
report of the rows (the checks that its CPU-baseline leg runs on the
outputs the GPU rows hand over)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_1909_10547_amd import synth  # noqa: E402


def normwise(y, r):
    num = np.sqrt(((y - r) ** 2).sum(axis=0))
    den = np.sqrt((r ** 2).sum(axis=0))
    return float(np.max(num / den))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr or "single GPU" in p.stderr or "1 GPU" in p.stderr


def _checks(eps):
    """Outputs of every row kind equal to the oracle's times (1 + eps) in
    one replica column (so each normwise error is eps)."""
    R = 4
    bump = np.ones(R)
    bump[2] += eps
    w = synth.dis_fit_workload(0.02)
    dt = [w.table(d) for d in range(3)]
    pdf = w.pdf(R).astype(np.float32).astype(np.float64)
    y = np.concatenate([oracle.dis(t.mask, t.fk, pdf) for t in dt])
    Nd = y.shape[0]
    gbar = np.random.default_rng(1).standard_normal((Nd, R))
    offs = np.cumsum([0] + [t.ndata for t in dt])
    g = sum(oracle.dis_grad(t.mask, t.fk, gbar[o:o + t.ndata], pdf.shape[0], pdf.shape[1])
            for t, o in zip(dt, offs))
    hw = synth.had_fit_workload(0.02)
    ht = [hw.table(d) for d in range(2)]
    hp = hw.pdf(R).astype(np.float32).astype(np.float64)
    sels = [np.arange(min(3, t.ndata)) for t in ht]
    gbs = [np.random.default_rng(2 + k).standard_normal((len(s), R)) for k, s in enumerate(sels)]
    hg = sum(oracle.had_grad(t.mask, t.fk[s], hp, b) for t, s, b in zip(ht, sels, gbs))
    C = [np.eye(4) * 2.0 + 0.1, np.eye(3) * 3.0]
    sig = np.random.default_rng(3).standard_normal((7, R))
    D = np.linspace(-1, 1, 7)
    c2, d2 = oracle.chi2([oracle.cholesky(c) for c in C], sig, D)
    mask = synth.table3_mask()
    fk3 = synth.table3_fk(4, 35721)[:2]
    p3 = synth.table3_pdf(R)
    y3 = oracle.flat_conv(fk3, oracle.luminosity(mask, p3))
    checks = [
        {"type": "dis", "tables": [(t.mask, t.fk) for t in dt], "pdf": pdf,
         "out": {"bf16": y * bump, "f32": y}, "grad": {"bf16": g * bump, "f32": g}, "gbar": gbar},
        {"type": "had_grad", "tables": [(t.mask, t.fk[s]) for t, s in zip(ht, sels)], "gbar": gbs,
         "pdf": hp, "grad": {"bf16": hg * bump, "f32": hg}},
        {"type": "chi2", "C": C, "D": D, "sigma": sig, "chi2": c2 * bump, "grad": d2 * bump},
        {"type": "flat", "index": 0, "mask": mask, "fk": fk3, "pdf": p3, "y": y3 * bump},
        {"type": "serving", "items": [("dis", dt[0].mask, dt[0].fk, pdf, y[:dt[0].ndata] * bump)]},
    ]
    result = {"rows": {"dis_bf16": {}, "dis_f32": {}, "had_adjoint_bf16": {}, "had_adjoint_f32": {},
                       "chi2_fp64": {}, "table3": [{}], "serving": {"error": {}}}}
    return result, checks


@pytest.mark.parametrize("eps", [0.0, 1e-3])
def test_fp64_report_of_every_row(eps):
    result, checks = _checks(eps)
    bench.fp64_checks(result, checks, oracle, normwise)
    r = result["rows"]
    tol = 1e-12
    assert abs(r["dis_bf16"]["error_vs_fp64"]["max_over_datasets"] - eps) <= tol
    assert abs(r["dis_bf16"]["error_vs_fp64"]["all"] - eps) <= tol
    assert abs(r["dis_bf16"]["error_vs_fp64"]["adjoint_normwise"] - eps) <= tol
    assert r["dis_f32"]["error_vs_fp64"]["max_over_datasets"] <= tol
    assert abs(r["had_adjoint_bf16"]["error_vs_fp64"]["normwise"] - eps) <= tol
    assert r["had_adjoint_f32"]["error_vs_fp64"]["normwise"] <= tol
    assert abs(r["chi2_fp64"]["error_vs_fp64"]["chi2_max_rel"] - eps) <= tol
    assert abs(r["chi2_fp64"]["error_vs_fp64"]["gradient_normwise"] - eps) <= tol
    # the Table 3 measure is max |err| / max |ref| over the sampled outputs:
    # one column scaled by 1 + eps gives at most eps
    t3 = r["table3"][0]["error_vs_fp64"]["max_abs_over_max_ref"]
    assert t3 <= eps + tol and (eps == 0.0 or t3 > 0.0)
    assert abs(r["serving"]["error"]["fp32_reference_vs_fp64_max_normwise"] - eps) <= tol
