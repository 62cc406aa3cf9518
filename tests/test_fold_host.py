"""The symmetric passes' fold on the host (CPU only): tests/host/fold_check.cpp
builds trees, lists, symmetric work and folds with the library's own host
code (tree.cpp, traverse.cpp, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer) and checks that the fold gives every particle and
every proxy exactly its own terms, reads every slot once, and keeps each
output's parts in item order."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2012_06925_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not present")
def test_fold_gives_every_output_its_terms_once(tmp_path):
    exe = str(tmp_path / "fold_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I" + os.path.join(ROOT, "include"), "-o", exe,
           os.path.join(ROOT, "tests", "host", "fold_check.cpp"), os.path.join(CSRC, "tree.cpp"),
           os.path.join(CSRC, "traverse.cpp"), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ)
    env.pop("LD_PRELOAD", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout
