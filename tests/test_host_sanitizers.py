"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with the sanitizers on its host half only (the
device code is built as usual; GPU sanitizers are not used), and the C
program abi_check.c drives, through the C ABI, every argument check that
rejects a call on the host, the host-only entry points and an engine set-up
that fails at its first device call on a machine without a GPU.  Leak
detection is on.  Needs no GPU; takes about a minute to build.
"""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_14652_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
CHECKS = ("address", "undefined")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
@pytest.mark.timeout(600)
def test_abi_host_paths_under_asan_and_ubsan():
    os.makedirs(OUT, exist_ok=True)
    host_san = [f for c in CHECKS for f in ("-Xarch_host", f"-fsanitize={c}")]
    flags = ["--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-g", "-Xarch_host", "-fno-omit-frame-pointer", *host_san,
             f"-I{INCLUDE}", f"-I{CSRC}"]

    def compile_one(src):
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        _run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(2) as ex:
        objs = list(ex.map(compile_one, ("hmc_engine.hip", "hmc_kernels.hip")))
    lib = os.path.join(OUT, "libhmc_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs])
    # the host half really is instrumented
    syms = _run(["nm", "-D", "--undefined-only", lib]).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms
    exe = os.path.join(OUT, "abi_check")
    _run([CLANG, "-g", "-O1", "-fno-omit-frame-pointer", f"-fsanitize={','.join(CHECKS)}",
          f"-I{INCLUDE}", os.path.join(ROOT, "tests", "abi_check.c"), "-o", exe, lib, f"-Wl,-rpath,{OUT}", "-lm"])
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "abi_check ok" in r.stdout, f"rc {r.returncode}\n{r.stdout}\n{r.stderr[-6000:]}"
    shutil.rmtree(OUT, ignore_errors=True)
