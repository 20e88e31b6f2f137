"""Race detection on the oracle's OpenMP paths (CPU only).

The oracle may run the trials of one (colour, sub-colour) set, and its
energy and pair-count sums, on several threads; those trials never
interact and the sums are integers, so every thread count must give the
same bits.  Here the oracle is built with ThreadSanitizer and LLVM's OpenMP
race detector (Archer), on lattices whose sets are large enough to run
threaded, and a driver (tests/tsan/oracle_threads.c) compares one thread
against four.  A copy of the oracle with a race planted in its sweep loop
(the per-set energy and accept sums left shared) must be reported, which
shows the detector is active.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LLVM = "/opt/rocm/lib/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")
DRIVER = os.path.join(ROOT, "tests", "tsan", "oracle_threads.c")
ORACLE = os.path.join(ROOT, "oracle", "smcx_oracle.c")

pytestmark = pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                                reason="needs ROCm's clang with ThreadSanitizer and libarcher")

RACE_EXIT = 66


def build(tmp, oracle_src):
    exe = os.path.join(tmp, "tsan_oracle")
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c99", "-fsanitize=thread", "-fopenmp", "-ffp-contract=off",
                           "-I", os.path.join(ROOT, "oracle"), "-o", exe, DRIVER, oracle_src, "-lm"])
    return exe


def run(exe):
    env = dict(os.environ)
    env.update({"OMP_TOOL_LIBRARIES": ARCHER,
                "LD_LIBRARY_PATH": os.path.join(LLVM, "lib") + ":" + env.get("LD_LIBRARY_PATH", ""),
                "TSAN_OPTIONS": f"halt_on_error=1 exitcode={RACE_EXIT} ignore_noninstrumented_modules=1"})
    return subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)


def test_threaded_oracle_has_no_data_race(tmp_path):
    r = run(build(str(tmp_path), ORACLE))
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.count(": same") == 2


def test_planted_race_is_reported(tmp_path):
    src = open(ORACLE).read()
    needle = "reduction(+ : dE_set, acc_set) "
    assert src.count(needle) == 1
    bad = os.path.join(str(tmp_path), "smcx_oracle.c")
    with open(bad, "w") as f:
        f.write(src.replace(needle, ""))
    shutil.copy(os.path.join(ROOT, "oracle", "smcx_oracle.h"), str(tmp_path))
    r = run(build(str(tmp_path), bad))
    assert r.returncode == RACE_EXIT and "data race" in r.stderr, (r.returncode, r.stderr[-2000:])
