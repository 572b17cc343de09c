"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The FP64 oracle (C) and the solve server's scheduler (the host-only build of
serve_core.h, C++) are compiled with -fsanitize=address,undefined into a
temporary directory, and their CPU tests run against those builds in a child
process (the sanitizer runtime preloaded, any report fatal).  The HIP library's
host code is not covered: it needs the HIP runtime, which is not built with
the sanitizers."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_and_scheduler_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    orc = str(tmp_path / "liboracle_san.so")
    sched = str(tmp_path / "libsched_san.so")
    subprocess.check_call(["gcc"] + SAN + ["-fopenmp", "-fPIC", "-shared", "-std=c99",
                                           "-fno-fast-math", "-ffp-contract=off",
                                           os.path.join(ROOT, "oracle", "gpspca_oracle.c"),
                                           "-o", orc, "-lm"])
    subprocess.check_call(["g++"] + SAN + ["-std=c++17", "-fPIC", "-shared",
                                           os.path.join(ROOT, "paper_1312_6182_amd", "csrc",
                                                        "serve_sim.cpp"), "-o", sched])
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": asan,
        # Python itself is not instrumented: its allocations are not leaks of ours
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "GPSPCA_ORACLE_LIB": orc,
        "GPSPCA_SCHED_LIB": sched,
        "OMP_NUM_THREADS": "4",
    })
    tests = ["tests/test_oracle_pins.py", "tests/test_oracle_quant_pins.py",
             "tests/test_oracle_deflation_pins.py", "tests/test_oracle_bl1x_pins.py",
             "tests/test_serve_sched.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + tests, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert " passed" in r.stdout, out
