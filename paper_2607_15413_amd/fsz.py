"""Thin ctypes binding of libfsz.so (the C ABI declared in include/fsz.h).

The functions named fsz_* marshal arguments 1:1 onto the C entry points:
device pointers are integers (e.g. ``tensor.data_ptr()``), streams are
hipStream_t handles as integers (``torch.cuda.current_stream().cuda_stream``)
or None for the default stream.  Every step of compression and
decompression runs in the library's HIP kernels; if the built library is
missing this module raises instead of falling back to anything else.

The helpers ``compress`` / ``decompress`` / ``field_stats`` only add PyTorch
device-memory plumbing around those calls.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfsz.so")

FSZ_ABS = 0
FSZ_REL = 1

FSZ_OK = 0
FSZ_ERR_INVALID_ARG = 1
FSZ_ERR_NONFINITE = 2
FSZ_ERR_EB_TOO_SMALL = 3
FSZ_ERR_CAPACITY = 4
FSZ_ERR_CORRUPT = 5
FSZ_ERR_SIZE_MISMATCH = 6
FSZ_ERR_DEVICE = 7
FSZ_ERR_EB_TOO_LARGE = 8
FSZ_ERR_TOO_LARGE = 9

# names of every C entry point declared in include/fsz.h
EXPORTS = (
    "fsz_compressed_bound",
    "fsz_status_string",
    "fsz_field_stats",
    "fsz_compress",
    "fsz_compress_ex",
    "fsz_decompress",
    "fsz_compress_async",
    "fsz_compress_noalloc_async",
    "fsz_decompress_async",
    "fsz_decompress_prezero_async",
    "fsz_decompress_range_async",
    "fsz_compress_features_async",
    "fsz_compress_five_read_async",
    "fsz_compressed_bound_config",
    "fsz_compress_config_async",
    "fsz_decompress_config_async",
    "fsz_batch_async",
    "fsz_autotune",
    "fsz_plan_create",
    "fsz_plan_launch",
    "fsz_plan_get_tuning",
    "fsz_plan_destroy",
    "fsz_server_now_ns",
    "fsz_server_create",
    "fsz_server_submit",
    "fsz_server_poll",
    "fsz_server_release",
    "fsz_server_get_stats",
    "fsz_server_destroy",
)

# feature switches (fsz_compress_features_async)
FSZ_FEAT_CROSS_BLOCK = 1
FSZ_FEAT_CENTERING = 2
FSZ_FEAT_LZ2 = 4
FSZ_FEATURES_ALL = 7

FSZ_OP_COMPRESS = 0
FSZ_OP_DECOMPRESS = 1


class FszError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {fsz_status_string(status)} (status {status})")
        self.status = status


class FszStats(ctypes.Structure):
    _fields_ = [("xmin", ctypes.c_float), ("xmax", ctypes.c_float), ("maxabs", ctypes.c_float),
                ("flags", ctypes.c_uint32)]


class FszResult(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint64), ("status", ctypes.c_uint32), ("epoch", ctypes.c_uint32)]


class FszJob(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("d_src", ctypes.c_void_p), ("src_size", ctypes.c_size_t),
                ("d_dst", ctypes.c_void_p), ("dst_capacity", ctypes.c_size_t), ("n", ctypes.c_size_t),
                ("mode", ctypes.c_int), ("value", ctypes.c_double), ("d_result", ctypes.c_void_p)]


class FszTuning(ctypes.Structure):
    _fields_ = [("waves_per_group", ctypes.c_int), ("groups_per_cu", ctypes.c_int)]


class FszServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_jobs_per_round", ctypes.c_int),
                ("rounds_in_flight", ctypes.c_int), ("auto_release", ctypes.c_int), ("tuning", FszTuning)]


class FszRequest(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("d_src", ctypes.c_void_p), ("src_size", ctypes.c_size_t),
                ("n", ctypes.c_size_t), ("mode", ctypes.c_int), ("value", ctypes.c_double),
                ("tag", ctypes.c_uint64), ("arrival_ns", ctypes.c_uint64)]


class FszCompletion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_uint32), ("op", ctypes.c_uint32),
                ("size", ctypes.c_uint64), ("d_out", ctypes.c_void_p), ("arrival_ns", ctypes.c_uint64),
                ("admit_ns", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64), ("complete_ns", ctypes.c_uint64)]


class FszServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("max_jobs_in_round", ctypes.c_uint64), ("max_rounds_overlapping", ctypes.c_uint64),
                ("hbm_in_use", ctypes.c_size_t), ("hbm_peak", ctypes.c_size_t)]


_lib = None


def load_library():
    """Load libfsz.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    sz, vp = ctypes.c_size_t, ctypes.c_void_p
    lib.fsz_compressed_bound.argtypes = [sz]
    lib.fsz_compressed_bound.restype = sz
    lib.fsz_status_string.argtypes = [ctypes.c_int]
    lib.fsz_status_string.restype = ctypes.c_char_p
    lib.fsz_field_stats.argtypes = [vp, sz, vp, vp]
    lib.fsz_field_stats.restype = ctypes.c_int
    lib.fsz_compress.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, sz,
                                 ctypes.POINTER(sz), vp]
    lib.fsz_compress.restype = ctypes.c_int
    lib.fsz_compress_ex.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, vp, sz,
                                    ctypes.POINTER(sz), vp]
    lib.fsz_compress_ex.restype = ctypes.c_int
    lib.fsz_decompress.argtypes = [vp, sz, vp, sz, vp]
    lib.fsz_decompress.restype = ctypes.c_int
    lib.fsz_compress_async.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, vp, sz, vp, vp]
    lib.fsz_compress_async.restype = ctypes.c_int
    lib.fsz_compress_noalloc_async.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, vp, sz, vp, vp]
    lib.fsz_compress_noalloc_async.restype = ctypes.c_int
    lib.fsz_compress_features_async.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, ctypes.c_uint, vp, sz,
                                                vp, vp]
    lib.fsz_compress_features_async.restype = ctypes.c_int
    lib.fsz_compress_five_read_async.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, vp, sz, vp, vp]
    lib.fsz_compress_five_read_async.restype = ctypes.c_int
    lib.fsz_decompress_range_async.argtypes = [vp, sz, sz, sz, sz, vp, vp, vp]
    lib.fsz_decompress_range_async.restype = ctypes.c_int
    lib.fsz_compressed_bound_config.argtypes = [sz, ctypes.c_int, ctypes.c_int]
    lib.fsz_compressed_bound_config.restype = sz
    lib.fsz_compress_config_async.argtypes = [vp, sz, ctypes.c_int, ctypes.c_double, vp, ctypes.c_int,
                                              ctypes.c_int, vp, sz, vp, vp]
    lib.fsz_compress_config_async.restype = ctypes.c_int
    lib.fsz_decompress_config_async.argtypes = [vp, sz, vp, sz, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.fsz_decompress_config_async.restype = ctypes.c_int
    lib.fsz_decompress_async.argtypes = [vp, sz, vp, sz, vp, vp]
    lib.fsz_decompress_async.restype = ctypes.c_int
    lib.fsz_decompress_prezero_async.argtypes = [vp, sz, vp, sz, vp, vp]
    lib.fsz_decompress_prezero_async.restype = ctypes.c_int
    jp, tp = ctypes.POINTER(FszJob), ctypes.POINTER(FszTuning)
    lib.fsz_batch_async.argtypes = [jp, sz, tp, vp]
    lib.fsz_batch_async.restype = ctypes.c_int
    lib.fsz_autotune.argtypes = [jp, sz, ctypes.c_int, vp, tp]
    lib.fsz_autotune.restype = ctypes.c_int
    lib.fsz_plan_create.argtypes = [jp, sz, tp, ctypes.POINTER(vp)]
    lib.fsz_plan_create.restype = ctypes.c_int
    lib.fsz_plan_launch.argtypes = [vp, vp]
    lib.fsz_plan_launch.restype = ctypes.c_int
    lib.fsz_plan_get_tuning.argtypes = [vp, tp]
    lib.fsz_plan_get_tuning.restype = ctypes.c_int
    lib.fsz_plan_destroy.argtypes = [vp]
    lib.fsz_plan_destroy.restype = None
    lib.fsz_server_now_ns.argtypes = []
    lib.fsz_server_now_ns.restype = ctypes.c_uint64
    lib.fsz_server_create.argtypes = [ctypes.POINTER(FszServerConfig), ctypes.POINTER(vp)]
    lib.fsz_server_create.restype = ctypes.c_int
    lib.fsz_server_submit.argtypes = [vp, ctypes.POINTER(FszRequest), sz]
    lib.fsz_server_submit.restype = ctypes.c_int
    lib.fsz_server_poll.argtypes = [vp, ctypes.POINTER(FszCompletion), sz, ctypes.c_int]
    lib.fsz_server_poll.restype = sz
    lib.fsz_server_release.argtypes = [vp, vp]
    lib.fsz_server_release.restype = ctypes.c_int
    lib.fsz_server_get_stats.argtypes = [vp, ctypes.POINTER(FszServerStats)]
    lib.fsz_server_get_stats.restype = ctypes.c_int
    lib.fsz_server_destroy.argtypes = [vp]
    lib.fsz_server_destroy.restype = None
    _lib = lib
    return lib


# ----------------------------------------------------------------- C ABI


def fsz_compressed_bound(n: int) -> int:
    return int(load_library().fsz_compressed_bound(n))


def fsz_status_string(status: int) -> str:
    return load_library().fsz_status_string(status).decode()


def fsz_field_stats(d_in: int, n: int, d_stats: int, stream=None) -> int:
    return load_library().fsz_field_stats(d_in, n, d_stats, stream)


def fsz_compress(d_in: int, n: int, mode: int, value: float, d_out: int, out_capacity: int,
                 stream=None):
    """Returns (status, out_size)."""
    size = ctypes.c_size_t(0)
    st = load_library().fsz_compress(d_in, n, mode, value, d_out, out_capacity,
                                     ctypes.byref(size), stream)
    return st, size.value


def fsz_compress_ex(d_in: int, n: int, mode: int, value: float, d_stats: int, d_out: int,
                    out_capacity: int, stream=None):
    """Returns (status, out_size)."""
    size = ctypes.c_size_t(0)
    st = load_library().fsz_compress_ex(d_in, n, mode, value, d_stats, d_out, out_capacity,
                                        ctypes.byref(size), stream)
    return st, size.value


def fsz_decompress(d_cmp: int, cmp_size: int, d_out: int, n: int, stream=None) -> int:
    return load_library().fsz_decompress(d_cmp, cmp_size, d_out, n, stream)


def fsz_compress_async(d_in: int, n: int, mode: int, value: float, d_stats, d_out: int,
                       out_capacity: int, d_result: int, stream=None) -> int:
    """Enqueue only; the outcome lands in the device fsz_result at d_result."""
    return load_library().fsz_compress_async(d_in, n, mode, value, d_stats, d_out, out_capacity,
                                             d_result, stream)


def fsz_decompress_prezero_async(d_cmp: int, cmp_size: int, d_out: int, n: int, d_result: int,
                                 stream=None) -> int:
    """Decompression into an output cleared first; all-zero tile groups are skipped (enqueue only)."""
    return load_library().fsz_decompress_prezero_async(d_cmp, cmp_size, d_out, n, d_result, stream)


def fsz_compress_noalloc_async(d_in: int, n: int, mode: int, value: float, d_stats, d_out: int,
                               out_capacity: int, d_result: int, stream=None) -> int:
    """As fsz_compress_async, with the library's scratch in a fixed device array (allocates nothing)."""
    return load_library().fsz_compress_noalloc_async(d_in, n, mode, value, d_stats, d_out, out_capacity,
                                                     d_result, stream)


def fsz_decompress_range_async(d_cmp: int, cmp_size: int, n: int, begin: int, end: int, d_out: int,
                               d_result: int, stream=None) -> int:
    """Elements [begin, end) of the stream's field into d_out (enqueue only)."""
    return load_library().fsz_decompress_range_async(d_cmp, cmp_size, n, begin, end, d_out, d_result, stream)


def fsz_compress_features_async(d_in: int, n: int, mode: int, value: float, d_stats, features: int,
                                d_out: int, out_capacity: int, d_result: int, stream=None) -> int:
    """Compression with a subset of the prediction features (enqueue only)."""
    return load_library().fsz_compress_features_async(d_in, n, mode, value, d_stats, features, d_out,
                                                      out_capacity, d_result, stream)


def fsz_compress_five_read_async(d_in: int, n: int, mode: int, value: float, d_stats, d_out: int,
                                 out_capacity: int, d_result: int, stream=None) -> int:
    """The five-read baseline (enqueue only); same stream as fsz_compress_async."""
    return load_library().fsz_compress_five_read_async(d_in, n, mode, value, d_stats, d_out, out_capacity,
                                                       d_result, stream)


def fsz_compressed_bound_config(n: int, block: int, tile_blocks: int) -> int:
    return int(load_library().fsz_compressed_bound_config(n, block, tile_blocks))


def fsz_compress_config_async(d_in: int, n: int, mode: int, value: float, d_stats, block: int,
                              tile_blocks: int, d_out: int, out_capacity: int, d_result: int, stream=None) -> int:
    """Compression with a (block, tile_blocks) tile configuration (enqueue only)."""
    return load_library().fsz_compress_config_async(d_in, n, mode, value, d_stats, block, tile_blocks, d_out,
                                                    out_capacity, d_result, stream)


def fsz_decompress_config_async(d_cmp: int, cmp_size: int, d_out: int, n: int, block: int, tile_blocks: int,
                                d_result: int, stream=None) -> int:
    """Decode a stream of a (block, tile_blocks) tile configuration (enqueue only)."""
    return load_library().fsz_decompress_config_async(d_cmp, cmp_size, d_out, n, block, tile_blocks, d_result,
                                                      stream)


def fsz_decompress_async(d_cmp: int, cmp_size: int, d_out: int, n: int, d_result: int,
                         stream=None) -> int:
    return load_library().fsz_decompress_async(d_cmp, cmp_size, d_out, n, d_result, stream)


def _job_array(jobs):
    arr = (FszJob * max(len(jobs), 1))()
    for k, j in enumerate(jobs):
        arr[k] = j
    return arr


def _tuning_ptr(tuning):
    if tuning is None:
        return None
    return ctypes.byref(FszTuning(*tuning))


def fsz_batch_async(jobs, tuning=None, stream=None) -> int:
    """jobs: sequence of FszJob; tuning: None or (waves_per_group, groups_per_cu)."""
    arr = _job_array(jobs)
    return load_library().fsz_batch_async(arr, len(jobs), _tuning_ptr(tuning), stream)


def fsz_autotune(jobs, reps: int = 3, stream=None):
    """Returns (status, (waves_per_group, groups_per_cu))."""
    arr = _job_array(jobs)
    best = FszTuning(0, 0)
    st = load_library().fsz_autotune(arr, len(jobs), reps, stream, ctypes.byref(best))
    return st, (best.waves_per_group, best.groups_per_cu)


def fsz_plan_create(jobs, tuning=None):
    """Returns (status, plan handle or None)."""
    arr = _job_array(jobs)
    h = ctypes.c_void_p(None)
    st = load_library().fsz_plan_create(arr, len(jobs), _tuning_ptr(tuning), ctypes.byref(h))
    return st, (h.value if st == FSZ_OK else None)


def fsz_plan_launch(plan, stream=None) -> int:
    return load_library().fsz_plan_launch(plan, stream)


def fsz_plan_get_tuning(plan):
    t = FszTuning(0, 0)
    st = load_library().fsz_plan_get_tuning(plan, ctypes.byref(t))
    return st, (t.waves_per_group, t.groups_per_cu)


def fsz_plan_destroy(plan) -> None:
    load_library().fsz_plan_destroy(plan)


def fsz_server_now_ns() -> int:
    return int(load_library().fsz_server_now_ns())


def fsz_server_create(hbm_budget: int, max_jobs_per_round: int = 256, rounds_in_flight: int = 2,
                      auto_release: bool = False, tuning=(0, 0)):
    """Returns (status, server handle or None)."""
    cfg = FszServerConfig(hbm_budget, max_jobs_per_round, rounds_in_flight, int(auto_release),
                          FszTuning(*tuning))
    h = ctypes.c_void_p(None)
    st = load_library().fsz_server_create(ctypes.byref(cfg), ctypes.byref(h))
    return st, (h.value if st == FSZ_OK else None)


def fsz_server_submit(server, requests) -> int:
    arr = (FszRequest * max(len(requests), 1))()
    for k, r in enumerate(requests):
        arr[k] = r
    return load_library().fsz_server_submit(server, arr, len(requests))


def request_table(count: int):
    """numpy structured array laid out as fsz_request[count] (for large
    submissions: fill columns vectorized, then fsz_server_submit_table)."""
    import numpy as np
    dt = np.dtype({"names": [f[0] for f in FszRequest._fields_],
                   "formats": [np.int32, np.uint64, np.uint64, np.uint64, np.int32, np.float64, np.uint64,
                               np.uint64],
                   "offsets": [getattr(FszRequest, f[0]).offset for f in FszRequest._fields_],
                   "itemsize": ctypes.sizeof(FszRequest)})
    return np.zeros(count, dtype=dt)


def fsz_server_submit_table(server, table) -> int:
    """Submit a request_table() array in one call."""
    ptr = ctypes.cast(table.ctypes.data, ctypes.POINTER(FszRequest))
    return load_library().fsz_server_submit(server, ptr, len(table))


def fsz_server_poll(server, max_count: int = 1024, wait_ms: int = 0):
    """List of FszCompletion (possibly empty)."""
    arr = (FszCompletion * max_count)()
    k = load_library().fsz_server_poll(server, arr, max_count, wait_ms)
    return [arr[i] for i in range(k)]


def fsz_server_release(server, d_out: int) -> int:
    return load_library().fsz_server_release(server, d_out)


def fsz_server_get_stats(server) -> FszServerStats:
    st = FszServerStats()
    load_library().fsz_server_get_stats(server, ctypes.byref(st))
    return st


def fsz_server_destroy(server) -> None:
    load_library().fsz_server_destroy(server)


def compress_request(d_in: int, n: int, mode: int, value: float, tag: int, arrival_ns: int) -> FszRequest:
    return FszRequest(FSZ_OP_COMPRESS, d_in, 0, n, mode, value, tag, arrival_ns)


def decompress_request(d_cmp: int, cmp_size: int, n: int, tag: int, arrival_ns: int) -> FszRequest:
    return FszRequest(FSZ_OP_DECOMPRESS, d_cmp, cmp_size, n, 0, 0.0, tag, arrival_ns)


def compress_job(d_in: int, n: int, mode: int, value: float, d_out: int, capacity: int,
                 d_result: int) -> FszJob:
    return FszJob(FSZ_OP_COMPRESS, d_in, 0, d_out, capacity, n, mode, value, d_result)


def decompress_job(d_cmp: int, cmp_size: int, d_out: int, n: int, d_result: int) -> FszJob:
    return FszJob(FSZ_OP_DECOMPRESS, d_cmp, cmp_size, d_out, 0, n, 0, 0.0, d_result)


def read_result(result_tensor):
    """(size, status, epoch) from a 16-byte device tensor holding an fsz_result."""
    raw = result_tensor.cpu().numpy().tobytes()[:16]
    r = FszResult.from_buffer_copy(raw)
    return r.size, r.status, r.epoch


# ----------------------------------------------------------------- torch plumbing


def _stream_handle(torch, device):
    return torch.cuda.current_stream(device).cuda_stream


def compress(x, mode: int, value: float, out=None, check: bool = True):
    """Compress a contiguous float32 CUDA tensor; returns (uint8 tensor view, status)."""
    import torch
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    n = x.numel()
    if out is None:
        out = torch.empty(fsz_compressed_bound(n), dtype=torch.uint8, device=x.device)
    st, size = fsz_compress(x.data_ptr(), n, mode, value, out.data_ptr(), out.numel(),
                            _stream_handle(torch, x.device))
    if check and st != FSZ_OK:
        raise FszError(st, "fsz_compress")
    return (out[:size] if st == FSZ_OK else out), st


def compress_features(x, mode: int, value: float, features: int, out=None, check: bool = True):
    """Compress a contiguous float32 CUDA tensor with a feature subset; returns
    (uint8 tensor view, status).  Synchronizes the stream to read the size."""
    import torch
    assert x.dtype == torch.float32 and x.is_cuda and x.is_contiguous()
    n = x.numel()
    if out is None:
        out = torch.empty(fsz_compressed_bound(n), dtype=torch.uint8, device=x.device)
    res = torch.zeros(2, dtype=torch.int64, device=x.device)  # fsz_result {u64 size; u32 status, epoch}
    stream = _stream_handle(torch, x.device)
    st = fsz_compress_features_async(x.data_ptr(), n, mode, value, None, features, out.data_ptr(),
                                     out.numel(), res.data_ptr(), stream)
    if st == FSZ_OK:
        torch.cuda.current_stream(x.device).synchronize()
        r = res.cpu()
        size, st = int(r[0]), int(r[1]) & 0xFFFFFFFF
    if check and st != FSZ_OK:
        raise FszError(st, "fsz_compress_features_async")
    return (out[:size] if st == FSZ_OK else out), st


def decompress(stream_bytes, n: int, out=None, check: bool = True):
    """Decompress a uint8 CUDA tensor holding one stream; returns (float32 tensor, status)."""
    import torch
    assert stream_bytes.dtype == torch.uint8 and stream_bytes.is_cuda
    if out is None:
        out = torch.empty(max(n, 1), dtype=torch.float32, device=stream_bytes.device)[:n]
    st = fsz_decompress(stream_bytes.data_ptr(), stream_bytes.numel(), out.data_ptr(), n,
                        _stream_handle(torch, stream_bytes.device))
    if check and st != FSZ_OK:
        raise FszError(st, "fsz_decompress")
    return out, st


class _DeviceBuffer:
    """A raw device range exposed through the CUDA array interface."""

    def __init__(self, ptr: int, nbytes: int):
        self.__cuda_array_interface__ = {"shape": (nbytes,), "typestr": "|u1", "data": (ptr, False),
                                         "version": 2}


def device_view(ptr: int, nbytes: int, dtype=None):
    """A torch tensor viewing nbytes of device memory at ptr (no copy), e.g.
    a served request's output; reinterpreted as dtype when given."""
    import torch
    t = torch.as_tensor(_DeviceBuffer(ptr, nbytes), device="cuda")
    return t if dtype is None or dtype == torch.uint8 else t.view(dtype)


def field_stats(x, out=None):
    """Enqueue the value-range pass; returns a 16-byte device tensor holding fsz_stats."""
    import torch
    if out is None:
        out = torch.empty(4, dtype=torch.int32, device=x.device)
    st = fsz_field_stats(x.data_ptr(), x.numel(), out.data_ptr(), _stream_handle(torch, x.device))
    if st != FSZ_OK:
        raise FszError(st, "fsz_field_stats")
    return out
