"""The oracle pins catch planted mistakes.

Each case plants one plausible slip in a copy of the oracle (on the CPU, in
a temporary directory) and runs the pin and golden tests against it in a
fresh process: they must fail.

* C mutants: a copy of fkoracle.c is built with gcc and loaded through
  FK_ORACLE_LIB.
* Python mutants: the oracle package (with a slip in ``__init__.py``), the
  input generators and the pin tests are copied into a scratch tree, which
  the tests then import instead of the repository's.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.abspath(os.path.dirname(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "fkoracle.c")).read()
PYSRC = open(os.path.join(ROOT, "oracle", "__init__.py")).read()
PIN_TESTS = ["test_oracle_golden.py", "test_oracle_pins.py", "test_oracle_measures.py",
             "test_oracle_mlp.py"]

MUTANTS = {
    "dis_flavour_map": ("pdf[IDX3(flav[c], al, r, X, R)]", "pdf[IDX3(c, al, r, X, R)]"),
    "dis_replica_stride": ("pdf[IDX3(flav[c], al, r, X, R)]", "pdf[IDX3(flav[c], al, 0, X, R)]"),
    "had_alpha_beta_swap": ("acc += blk[(size_t)al * X + be] * fa", "acc += blk[(size_t)be * X + al] * fa"),
    "had_a_b_swap": ("double fa = pdfl[IDX3(pa[c], al, r, X, R)];", "double fa = pdfl[IDX3(pb[c], al, r, X, R)];"),
    "had_dropped_pair": ("for (int c = 0; c < np; ++c) {\n      const double *blk = fk + ((size_t)i * np + c) * X * X;\n      for (int al",
                         "for (int c = 0; c + 1 < np; ++c) {\n      const double *blk = fk + ((size_t)i * np + c) * X * X;\n      for (int al"),
    "grad_missing_transpose_term": ("if (pb[c] == a) /*", "if (0) /*"),
    "grad_column_index": ("s += blk[(size_t)ap * X + al]", "s += blk[(size_t)al * X + ap]"),
    "grad_sign": ("acc += gi * s;", "acc -= gi * s;"),
    "cholesky_sign": ("for (int k = 0; k < j; ++k) s -= L", "for (int k = 0; k < j; ++k) s += L"),
    "chi2_factor_two": ("= 2.0 * y[i];", "= y[i];"),
    "chi2_back_subst_transpose": ("s -= L[(size_t)j * n + i] * y[j];", "s -= L[(size_t)i * n + j] * y[j];"),
}

# slips in oracle/__init__.py: (text, replacement, count of replacements)
PY_MUTANTS = {
    "normwise_no_sqrt": ("num = np.sqrt(np.sum((y2 - r2) ** 2, axis=0))\n    den = np.sqrt(np.sum(r2 ** 2, axis=0))",
                         "num = np.sum((y2 - r2) ** 2, axis=0)\n    den = np.sum(r2 ** 2, axis=0)"),
    "normwise_over_rows": ("num = np.sqrt(np.sum((y2 - r2) ** 2, axis=0))\n    den = np.sqrt(np.sum(r2 ** 2, axis=0))",
                           "num = np.sqrt(np.sum((y2 - r2) ** 2, axis=1))\n    den = np.sqrt(np.sum(r2 ** 2, axis=1))"),
    "normwise_mean_not_max": ("return float(np.max(rel))", "return float(np.mean(rel))"),
    "normwise_zero_column_passes": ("np.where(num > 0, np.inf, 0.0)", "np.where(num > 0, 0.0, 0.0)"),
    "error_report_threshold": ("thr = 1e-3 * float(np.max(np.abs(yref)))", "thr = 1e-5 * float(np.max(np.abs(yref)))"),
    "dis_grad_quantized_drops_scale": ("quantize(_f64(gbar) * s[:, None], fmt))", "quantize(_f64(gbar), fmt))"),
    "upper_form_no_diagonal_half": ("U[:, (sa == sb)[keep]] *= 0.5", "U[:, (sa == sb)[keep]] *= 1.0"),
    "symmetric_part_no_transpose": ("S[:, c] += np.transpose(fk[:, idx[pb, pa]], (0, 2, 1))",
                                    "S[:, c] += fk[:, idx[pb, pa]]"),
    "bf16_one_bit_short": ('"bf16": (7, -126', '"bf16": (6, -126'),
    "luminosity_a_b_swap": ("L[c] = pdf[a[c]][:, None, :] * pdf[b[c]][None, :, :]",
                            "L[c] = pdf[b[c]][:, None, :] * pdf[a[c]][None, :, :]"),
    "mlp_no_tanh_derivative": ("d2 = (dout @ W3) * (1.0 - a2 ** 2)", "d2 = (dout @ W3)"),
    "mlp_first_layer_derivative": ("d1 = (d2 @ W2) * (1.0 - a1 ** 2)", "d1 = (d2 @ W2) * (1.0 - a1)"),
    "mlp_grad_no_preprocessing": ("dout = (gpdf[:, :, r] * pre).T", "dout = gpdf[:, :, r].T"),
    "mlp_grad_bias_dropped": ("d2.sum(axis=0), (dout.T @ a2).ravel()", "0 * d2.sum(axis=0), (dout.T @ a2).ravel()"),
    "mlp_preprocessing_beta_sign": ("(1.0 - x[None, :]) ** _f64(pre_beta)[:, None]",
                                    "(1.0 + x[None, :]) ** _f64(pre_beta)[:, None]"),
    "mlp_second_layer_no_tanh": ("a2 = np.tanh(a1 @ W2.T + b2)   # [X][h2]", "a2 = a1 @ W2.T + b2   # [X][h2]"),
}


def _run_pins(cwd, env):
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           *[os.path.join(cwd, "tests", t) for t in PIN_TESTS]],
                          cwd=cwd, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mut.c"
    src.write_text(SRC.replace(old, new, 1))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(src), "-lm"])
    env = dict(os.environ, FK_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = _run_pins(ROOT, env)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


def _scratch_tree(dst, init_text):
    """Copy of the oracle, the input generators and the pin tests, with the
    oracle's __init__.py replaced by ``init_text``."""
    os.makedirs(os.path.join(dst, "oracle"))
    shutil.copy(os.path.join(ROOT, "oracle", "fkoracle.c"), os.path.join(dst, "oracle"))
    with open(os.path.join(dst, "oracle", "__init__.py"), "w") as f:
        f.write(init_text)
    os.makedirs(os.path.join(dst, "paper_1909_10547_amd"))
    for fn in ("__init__.py", "synth.py"):
        shutil.copy(os.path.join(ROOT, "paper_1909_10547_amd", fn), os.path.join(dst, "paper_1909_10547_amd"))
    os.makedirs(os.path.join(dst, "tests"))
    for fn in PIN_TESTS + ["conftest.py"]:
        shutil.copy(os.path.join(ROOT, "tests", fn), os.path.join(dst, "tests"))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)


def test_scratch_tree_of_the_unchanged_oracle_passes(tmp_path):
    # the harness itself: an unmodified copy passes the pins
    dst = str(tmp_path / "tree")
    _scratch_tree(dst, PYSRC)
    r = _run_pins(dst, dict(os.environ, OMP_NUM_THREADS="2"))
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_pins_catch_python_mutant(name, tmp_path):
    old, new = PY_MUTANTS[name]
    assert PYSRC.count(old) == 1, f"mutation site for {name} not found exactly once"
    dst = str(tmp_path / "tree")
    _scratch_tree(dst, PYSRC.replace(old, new, 1))
    env = dict(os.environ, OMP_NUM_THREADS="2")
    env.pop("FK_ORACLE_LIB", None)
    r = _run_pins(dst, env)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
