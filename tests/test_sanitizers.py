"""AddressSanitizer + UndefinedBehaviorSanitizer builds of host code, on the CPU.

* the C oracle (``oracle/oracle.c``), every function on small inputs, with the
  NDFT route of eq. Fourier_sum checked against the pairwise definition;
* the library's host logic (argument validation of every entry point, error
  strings, the FP64 Lanczos quadrature of ``nfftgp_slq_logquad`` against the
  exact b^T log(A) b at full Krylov dimension).

The GPU half (the whole ABI with a sanitized host build) is
``tests/test_gpu_sanitizer.py``.
"""
import os
import subprocess

import pytest

from sanitize import build_san

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_c_under_sanitizers(tmp_path):
    exe = build_san.build_oracle(str(tmp_path / "oracle_san"))
    r = _run(exe)
    assert r.returncode == 0 and "oracle sanitizer run ok" in r.stdout


def test_library_host_paths_under_sanitizers(tmp_path):
    exe = build_san.build_abi(str(tmp_path / "abi_san"), gpu=False)
    r = _run(exe)
    assert r.returncode == 0 and "abi sanitizer run ok" in r.stdout
