"""Builds libhmc.so (the gfx950 kernels and the C-ABI engine) in-tree with hipcc.

Each translation unit is compiled to an object in parallel, then linked.
Packed-FP32 instructions are disabled for the device code.  The compiler's
per-kernel resource report (VGPRs, scratch, occupancy) is written to
_build/kernel_resources.txt; a kernel that needs scratch memory (private
arrays the compiler could not keep in registers, or spills) is reported on
stderr, since it runs far below its register-resident speed.
"""

from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhmc.so")
SOURCES = ("hmc_kernels.hip", "hmc_engine.hip")
ARCH = os.environ.get("HMC_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f"-I{INCLUDE}", f"-I{CSRC}"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *_flags(), "-Rpass-analysis=kernel-resource-usage", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj, r.stderr

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        res = list(ex.map(compile_one, SOURCES))
    objs = [o for o, _ in res]
    rows = _resources("".join(e for _, e in res))
    with open(os.path.join(BUILD, "kernel_resources.txt"), "w") as f:
        f.write("kernel\tvgprs\tscratch_bytes_per_lane\twaves_per_simd\n")
        for k, v in rows.items():
            f.write(f"{k}\t{v.get('VGPRs', '?')}\t{v.get('ScratchSize [bytes/lane]', '?')}\t"
                    f"{v.get('Occupancy [waves/SIMD]', '?')}\n")
    for k, v in rows.items():
        if int(v.get("ScratchSize [bytes/lane]", "0")) > 0:
            print(f"build: kernel {k} uses {v['ScratchSize [bytes/lane]']} bytes of scratch per lane",
                  file=sys.stderr)
    tmp = LIB + ".tmp"
    r = subprocess.run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def _resources(remarks: str) -> dict:
    """Per-kernel figures from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([^:]+?):\s+(\S+)\s+\[-Rpass-analysis", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
