"""Host code under the sanitizers (CPU only): the table packer of the
library, driven by tests/host/pack_driver.cpp, and the FP64 oracle's C
loops (running the oracle pins), built with AddressSanitizer and
UndefinedBehaviorSanitizer.  An out-of-bounds access, a use after free or
undefined behaviour makes the run fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_10547_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _gxx():
    g = shutil.which("g++")
    if not g:
        pytest.skip("g++ not available")
    return g


def test_packer_under_asan_ubsan(tmp_path):
    exe = tmp_path / "pack_driver"
    cmd = [_gxx(), *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "pack_driver.cpp"), os.path.join(CSRC, "pack.cpp"),
           "-o", str(exe), "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "pack driver OK" in r.stdout


def test_oracle_loops_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    lib = tmp_path / "liboracle_san.so"
    r = subprocess.run([gcc, *SAN, "-fPIC", "-shared", "-fopenmp", "-o", str(lib),
                        os.path.join(ROOT, "oracle", "fkoracle.c"), "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run([gcc, "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not found")
    env = dict(os.environ, FK_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2",
               LD_PRELOAD=":".join(p for p in (asan, ubsan) if os.path.isabs(p)),
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_golden.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
