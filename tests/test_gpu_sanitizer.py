"""The whole C ABI on the GPU with the library's host code under
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged): plan
creation with the rule's and a caller's scaling, FP32 and FP64, m = 4 and 6,
applies, CG, column dots, window information, the kernel-form description,
the autotuner, kernel timing, the AAFN preconditioner and preconditioned CG
(tests/sanitize/abi_gpu_main.cpp).  The driver is built by
__graft_entry__.build(); leak detection is off here (the HIP runtime keeps
allocations until exit), on in the CPU half (tests/test_sanitizers.py)."""
import os
import subprocess

import pytest

from sanitize import build_san

pytestmark = pytest.mark.gpu


def test_abi_on_gpu_under_sanitizers():
    exe = build_san.GPU_DRIVER
    assert os.path.exists(exe), "sanitizer driver missing: run __graft_entry__.build()"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    print("[case] abi_gpu_san", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=240)
    print(r.stdout[-3000:], r.stderr[-6000:], flush=True)
    assert r.returncode == 0 and "abi gpu sanitizer run ok" in r.stdout
