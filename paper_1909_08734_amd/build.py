"""Build the gfx950 shared library ``libcpm.so`` in-tree with hipcc.

Usage: python -m paper_1909_08734_amd.build   (or call build()).
Every call recompiles all sources.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libcpm.so")

ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result"]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Host set-up: plain IEEE evaluation of the stated formulas (no contraction).
HOST = ["-x", "c++", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]

HOST_SOURCES = ["setup_band.cpp", "setup_partition.cpp", "abi.cpp"]
DEVICE_SOURCES = ["device.hip"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="cpm_build_") as tmp:
        objs = []
        jobs = []
        for src in HOST_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            jobs.append([hipcc, *COMMON, *HOST, "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        for src in DEVICE_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            jobs.append([hipcc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj])
            objs.append(obj)
        procs = [(cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for cmd in jobs]
        for cmd, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                raise RuntimeError("compile failed: " + " ".join(cmd) + "\n" + text)
            if verbose and text.strip():
                print(text)
        tmp_lib = LIB + ".tmp"
        link = [hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp_lib, "-lpthread"]
        r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
