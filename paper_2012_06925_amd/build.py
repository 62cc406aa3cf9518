"""Build libbldtt.so (gfx950 HIP kernels + C++17 host engine + C ABI) in-tree.

    python -m paper_2012_06925_amd.build

Host translation units that decide trees and interaction lists are compiled
with -ffp-contract=off so their arithmetic rounds exactly as written.  All
HIP code is compiled with the packed-FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbldtt.so")
OBJ = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]
# MFMA operands and results in VGPRs: the vector ALUs read the results directly
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mllvm", "-amdgpu-mfma-vgpr-form"]
HOST_EXACT = ["-ffp-contract=off", "-fno-fast-math"]

HIP_HOST = ["-D__HIP_PLATFORM_AMD__"]

# (source, flags, object name); the batch kernel's instantiations are split
# over six objects so they compile in parallel.
UNITS = [
    ("kernels.hip", DEVICE, "kernels"),
    ("mlp.hip", DEVICE, "mlp"),
    ("walk.hip", DEVICE + HOST_EXACT, "walk"),
    ("treebuild.hip", DEVICE + HOST_EXACT, "treebuild"),
] + [("batch.hip", DEVICE + [f"-DBATCH_PART={k}"], f"batch{k}") for k in range(6)] + [
    ("degree.cpp", HOST_EXACT + HIP_HOST, "degree"),
    ("tree.cpp", HOST_EXACT, "tree"),
    ("traverse.cpp", HOST_EXACT, "traverse"),
    ("capi.cpp", HOST_EXACT + HIP_HOST, "capi"),
    ("batch_host.cpp", HOST_EXACT + HIP_HOST, "batch_host"),
    ("tune.cpp", [], "tune"),
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    objs = []
    for src, extra, name in UNITS:
        obj = os.path.join(OBJ, name + ".o")
        objs.append(obj)
        cmd = [HIPCC, "-c"] + COMMON + extra + ["-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"libbldtt build failed:\n{msg}")
    link = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs + \
        ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
