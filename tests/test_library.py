"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from paper_2607_15413_amd import fsz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "fsz.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsz_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fsz.load_library()
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert set(declared) == set(fsz.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_bound_matches_format_arithmetic():
    def ref(n):
        nb = -(-n // 32)
        nt = -(-n // 256)
        return 32 + (nb + 15) // 16 * 16 + 4 * nt + 128 * nb
    for n in (0, 1, 31, 32, 33, 255, 256, 257, 1 << 20, 25_000_000, 1 << 27, (1 << 33) + 5):
        assert fsz.fsz_compressed_bound(n) == ref(n)


def test_status_strings():
    for s in range(10):
        assert isinstance(fsz.fsz_status_string(s), str)
        assert fsz.fsz_status_string(s) != "unknown status"
    assert fsz.fsz_status_string(0) == "ok"


def test_invalid_arguments_rejected_on_host():
    # argument checks happen before any device work, so they run without a GPU
    st, _ = fsz.fsz_compress(0, 10, 0, 1e-3, 0, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 5, 1e-3, 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 1, float("nan"), 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 10, 1, -1.0, 16, 1000, None)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(18, 10, 1, 1e-3, 16, 1000, None)  # misaligned input
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_compress(16, 1000, 1, 1e-3, 16, 40, None)  # below the rate header size
    assert st == fsz.FSZ_ERR_CAPACITY
    assert fsz.fsz_decompress(16, 8, 16, 10, None) == fsz.FSZ_ERR_CORRUPT
    assert fsz.fsz_decompress(0, 100, 16, 10, None) == fsz.FSZ_ERR_INVALID_ARG
    # allocation-free compression: fields beyond its fixed scratch (2^30 elements)
    big = (1 << 30) + 1
    assert fsz.fsz_compress_noalloc_async(16, big, 1, 1e-3, None, 16, fsz.fsz_compressed_bound(big), 16,
                                          None) == fsz.FSZ_ERR_TOO_LARGE
    assert fsz.fsz_compress_noalloc_async(16, 10, 1, 1e-3, None, 16, 1000, None, None) == fsz.FSZ_ERR_INVALID_ARG
    # random access: a buffer shorter than the rate header of n elements is
    # rejected before the range pass reads any rate byte (1000 elements: 32 + 32 bytes)
    assert fsz.fsz_decompress_range_async(16, 63, 1000, 0, 10, 16, 16, None) == fsz.FSZ_ERR_CORRUPT
    assert fsz.fsz_decompress_range_async(16, 40, 1000, 500, 990, 16, 16, None) == fsz.FSZ_ERR_CORRUPT


def test_batch_invalid_jobs_rejected_on_host():
    # every job is validated before any device work; explicit shapes avoid device queries
    T = (4, 0)
    ok_c = fsz.compress_job(16, 1000, fsz.FSZ_REL, 1e-3, 16, fsz.fsz_compressed_bound(1000), 16)
    ok_d = fsz.decompress_job(16, 64, 16, 1000, 16)
    lib = fsz.load_library()
    assert lib.fsz_batch_async(None, 3, None, None) == fsz.FSZ_ERR_INVALID_ARG
    bad_op = fsz.FszJob(7, 16, 0, 16, 4096, 10, 1, 1e-3, 16)
    assert fsz.fsz_batch_async([ok_c, bad_op], T) == fsz.FSZ_ERR_INVALID_ARG
    no_result = fsz.compress_job(16, 1000, fsz.FSZ_REL, 1e-3, 16, 4096, 0)
    assert fsz.fsz_batch_async([ok_d, no_result], T) == fsz.FSZ_ERR_INVALID_ARG
    small = fsz.compress_job(16, 1000, fsz.FSZ_REL, 1e-3, 16, 40, 16)
    assert fsz.fsz_batch_async([ok_c, small], T) == fsz.FSZ_ERR_CAPACITY
    short = fsz.decompress_job(16, 31, 16, 1000, 16)
    assert fsz.fsz_batch_async([ok_c, short], T) == fsz.FSZ_ERR_CORRUPT
    bad_bound = fsz.compress_job(16, 1000, fsz.FSZ_REL, float("inf"), 16, 4096, 16)
    assert fsz.fsz_batch_async([bad_bound], T) == fsz.FSZ_ERR_INVALID_ARG
    misaligned = fsz.decompress_job(16, 64, 18, 1000, 16)
    assert fsz.fsz_batch_async([misaligned], T) == fsz.FSZ_ERR_INVALID_ARG
    for shape in ((3, 0), (16, 0), (4, -1), (4, 9)):
        assert fsz.fsz_batch_async([ok_c], shape) == fsz.FSZ_ERR_INVALID_ARG
    st, plan = fsz.fsz_plan_create([ok_c, small], T)
    assert st == fsz.FSZ_ERR_CAPACITY and plan is None
    assert fsz.fsz_plan_launch(None) == fsz.FSZ_ERR_INVALID_ARG
    st, _ = fsz.fsz_autotune([ok_c], reps=0)
    assert st == fsz.FSZ_ERR_INVALID_ARG


def test_arena_allocator_against_brute_force(tmp_path):
    # the served form's admission allocator, compiled for the host and run
    # against a unit-map first-fit model with invariant checks after every op
    import subprocess
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I",
                    os.path.join(ROOT, "paper_2607_15413_amd", "csrc"),
                    os.path.join(ROOT, "tests", "arena_check.cpp"), "-o", str(exe)], check=True)
    for seed in (1, 2, 3):
        r = subprocess.run([str(exe), str(seed)], capture_output=True, text=True)
        assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout


def test_server_invalid_config_rejected_on_host():
    lib = fsz.load_library()
    cfg = fsz.FszServerConfig(0, 16, 2, 0, fsz.FszTuning(4, 0))
    h = ctypes.c_void_p(None)
    assert lib.fsz_server_create(ctypes.byref(cfg), ctypes.byref(h)) == fsz.FSZ_ERR_INVALID_ARG
    for jobs, rounds, tuning in ((0, 2, (4, 0)), (16, 0, (4, 0)), (16, 17, (4, 0)), (16, 2, (3, 0))):
        cfg = fsz.FszServerConfig(1 << 20, jobs, rounds, 0, fsz.FszTuning(*tuning))
        assert lib.fsz_server_create(ctypes.byref(cfg), ctypes.byref(h)) == fsz.FSZ_ERR_INVALID_ARG
    assert lib.fsz_server_create(None, ctypes.byref(h)) == fsz.FSZ_ERR_INVALID_ARG
    req = fsz.compress_request(16, 10, fsz.FSZ_REL, 1e-3, 0, 0)
    assert fsz.fsz_server_submit(None, [req]) == fsz.FSZ_ERR_INVALID_ARG
    assert fsz.fsz_server_poll(None) == []
    assert fsz.fsz_server_release(None, 16) == fsz.FSZ_ERR_INVALID_ARG
    assert fsz.fsz_server_now_ns() > 0


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU: --gpus N > 1 exits with status 2 and
    says why, before it imports torch or touches a device."""
    for n in (2, 8):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 2, (n, r.returncode, r.stderr)
        assert "exactly one GPU" in r.stderr and f"--gpus {n}" in r.stderr
        assert r.stdout == ""
