"""The oracle pins catch planted mistakes.

Each case copies fkoracle.c, plants one plausible slip (on the CPU, in a
temporary directory), builds it with gcc and runs the pin and golden tests
against it in a fresh process: they must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = open(os.path.join(ROOT, "oracle", "fkoracle.c")).read()

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


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mut.c"
    src.write_text(SRC.replace(old, new, 1))
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(src), "-lm"])
    env = dict(os.environ, FK_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_golden.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
