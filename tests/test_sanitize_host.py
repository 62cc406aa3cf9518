"""The host engine and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

The library's host translation units (validation, tree build, traversal,
list packing, the batch forest, the degree policy and tuner glue) are compiled
with the sanitizers and linked with the device objects of the normal build
(left uninstrumented) into tests/sanitize/host_engine_check.cpp, which drives
every host-only entry point of the C ABI; the oracle's C source is compiled
with the sanitizers into tests/sanitize/oracle_check.c.  Any memory error,
leak or undefined behaviour aborts the program and fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_06925_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-g", "-O1"]
HOST_UNITS = ("capi", "batch_host", "tree", "traverse", "degree", "tune")
DEVICE_OBJECTS = ("kernels", "mlp", "walk", "treebuild") + tuple(f"batch{k}" for k in range(6))
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(cmds):
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True) for c in cmds]
    for c, p in zip(cmds, procs):
        out, _ = p.communicate()
        assert p.returncode == 0, f"{' '.join(c)}\n{out}"


def _env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env.pop("LD_PRELOAD", None)
    return env


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not present")
def test_host_engine_under_sanitizers(tmp_path):
    build_dir = os.path.join(ROOT, "_build")
    if not all(os.path.exists(os.path.join(build_dir, d + ".o")) for d in DEVICE_OBJECTS):
        from paper_2012_06925_amd import build
        build.build()
    cmds = []
    objs = []
    for u in HOST_UNITS:
        o = str(tmp_path / f"{u}.o")
        objs.append(o)
        cmds.append([CLANG, "-c", "-std=c++17", "-fPIC", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                     "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include")] + SAN +
                    ["-o", o, os.path.join(CSRC, u + ".cpp")])
    drv = str(tmp_path / "host_engine_check.o")
    cmds.append([CLANG, "-c", "-std=c++17", "-I" + os.path.join(ROOT, "include")] + SAN +
                ["-o", drv, os.path.join(ROOT, "tests", "sanitize", "host_engine_check.cpp")])
    _run(cmds)
    exe = str(tmp_path / "host_engine_check")
    _run([[CLANG] + SAN + ["-o", exe, drv] + objs + [os.path.join(build_dir, d + ".o") for d in DEVICE_OBJECTS] +
          ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"]])
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not present")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run([["gcc", "-fopenmp", "-ffp-contract=off"] + SAN +
          ["-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
           os.path.join(ROOT, "oracle", "bldtt_oracle.c"), "-lm"]])
    env = _env()
    env["OMP_NUM_THREADS"] = "4"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
