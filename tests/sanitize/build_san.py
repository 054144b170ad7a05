"""Builds of the test drivers under AddressSanitizer and UndefinedBehaviorSanitizer.

* oracle: ``oracle/oracle.c`` with ``oracle_main.c``, gcc, host only.
* abi: the library's host-logic sources (``api.hip``, ``precond_api.hip``,
  ``noalloc.hip``) compiled with the sanitizers on their host code only
  (``-Xarch_host`` before every ``-fsanitize=``; device code unchanged),
  linked with the kernel objects of the regular build and a driver:
  ``abi_main.cpp`` (paths that need no GPU) or ``abi_gpu_main.cpp`` (the whole
  C ABI on a GPU).

Test infrastructure: only ``tests/`` and ``__graft_entry__.build()`` use it.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2504_00480_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HOST_SOURCES = ["api.hip", "precond_api.hip", "noalloc.hip"]
GPU_DRIVER = os.path.join(HERE, "abi_gpu_san")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:2])} failed:\n{r.stderr[-4000:]}")


def build_oracle(out: str) -> str:
    _run(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_main.c"),
          os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", out])
    return out


def build_abi(out: str, gpu: bool) -> str:
    """Needs the regular build's kernel objects (paper_2504_00480_amd/_build)."""
    from paper_2504_00480_amd import build as pkg_build
    kobjs = [os.path.join(pkg_build.BUILD, os.path.splitext(s)[0] + ".o")
             for s in pkg_build.SOURCES if s not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in kobjs):
        pkg_build.build()
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        procs = []
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            cmd = [HIPCC, f"--offload-arch={pkg_build.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
                   "-I", pkg_build.INCLUDE, "-I", pkg_build.CSRC, *HOST_SAN,
                   "-c", os.path.join(pkg_build.CSRC, src), "-o", obj]
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True), src))
            objs.append(obj)
        for p, src in procs:
            _, err = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{err[-4000:]}")
        drv = os.path.join(tmp, "driver.o")
        if gpu:
            _run([HIPCC, "-O1", "-g", "-std=c++17", "-I", pkg_build.INCLUDE, *HOST_SAN, "-c",
                  os.path.join(HERE, "abi_gpu_main.cpp"), "-o", drv])
        else:
            _run(["g++", "-O1", "-g", "-std=c++17", "-I", pkg_build.INCLUDE, "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all", "-c", os.path.join(HERE, "abi_main.cpp"), "-o", drv])
        _run([HIPCC, f"--offload-arch={pkg_build.ARCH}", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", *objs, drv, *kobjs, "-o", out + ".tmp"])
        os.replace(out + ".tmp", out)
    return out
