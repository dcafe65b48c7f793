"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle is rebuilt with -fsanitize=address,undefined (no recovery) and
its pin suites run against that build in a child interpreter that preloads
the ASan runtime; the served form's arena allocator check runs as a
sanitized executable.  Any sanitizer report aborts the child, so the test
fails on a non-zero exit status and shows the report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ORACLE_PINS = ["tests/test_oracle.py", "tests/test_oracle_resolve.py", "tests/test_oracle_features.py",
               "tests/test_oracle_configs.py"]


def _asan_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("the ASan runtime of this gcc is not installed")
    return path


def _show(proc):
    return (proc.stdout or "")[-6000:] + (proc.stderr or "")[-6000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    runtime = _asan_runtime()
    lib = tmp_path / "libfsz_oracle_san.so"
    subprocess.run(["gcc", "-std=c11", *SAN, "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                    "-shared", "-Wall", "-Wextra", os.path.join(ROOT, "oracle", "fsz_oracle.c"), "-o", str(lib),
                    "-lm"], check=True)
    env = dict(os.environ, FSZO_LIB=str(lib), LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    # -s: a sanitizer report goes straight to stderr before the child exits
    proc = subprocess.run([sys.executable, "-m", "pytest", *ORACLE_PINS, "-q", "-x", "-s", "-m", "not gpu",
                           "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)
    assert proc.returncode == 0, _show(proc)
    assert "passed" in proc.stdout and "AddressSanitizer" not in proc.stderr, _show(proc)


def test_arena_allocator_under_asan_ubsan(tmp_path):
    _asan_runtime()
    exe = tmp_path / "arena_check_san"
    subprocess.run(["g++", "-std=c++17", *SAN, "-Wall", "-I", os.path.join(ROOT, "paper_2607_15413_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", str(exe)], check=True)
    for seed in (1, 2, 3, 4):
        proc = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=300,
                              env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        assert proc.returncode == 0 and proc.stdout.startswith("ok"), _show(proc)
