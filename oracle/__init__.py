"""FSZ oracle: ctypes front end of the plain C reference compressor.

TEST INFRASTRUCTURE ONLY.  Imported by the tests, the smoke check and the
benchmark's CPU-baseline leg; the product package never imports it.
"""
import ctypes
import os

import numpy as np

from .build import LIB
from .build import build as build_library

OK = 0
ERR_INVALID_ARG = 1
ERR_NONFINITE = 2
ERR_EB_TOO_SMALL = 3
ERR_CAPACITY = 4
ERR_CORRUPT = 5
ERR_SIZE_MISMATCH = 6
ERR_EB_TOO_LARGE = 8

ABS = 0
REL = 1

# feature switches of the ablation (Sec. VI-B); 0 = LZ1 on independent blocks
FEAT_CROSS_BLOCK = 1
FEAT_CENTERING = 2
FEAT_LZ2 = 4
FEATURES_ALL = 7

# tile configurations (Sec. VI-C, Table V): block size B, blocks per tile T
DEFAULT_CONFIG = (32, 8)
CONFIGS = [(32, 4), (32, 8), (32, 16), (64, 4), (64, 8), (64, 16)]

_lib = None


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"oracle {what} failed with status {status}")
        self.status = status


def _load():
    global _lib
    if _lib is None:
        # FSZO_LIB: another build of the same source (the sanitizer test loads
        # an AddressSanitizer / UBSan build this way)
        path = os.environ.get("FSZO_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build_library()
        lib = ctypes.CDLL(path)
        u64 = ctypes.c_uint64
        p = ctypes.c_void_p
        lib.fszo_bound.argtypes = [u64]
        lib.fszo_bound.restype = u64
        lib.fszo_resolve.argtypes = [p, u64, ctypes.c_int, ctypes.c_double, p, p, p]
        lib.fszo_resolve.restype = ctypes.c_int
        lib.fszo_compress.argtypes = [p, u64, ctypes.c_int, ctypes.c_double, p, u64, p]
        lib.fszo_compress.restype = ctypes.c_int
        lib.fszo_compress_features.argtypes = [p, u64, ctypes.c_int, ctypes.c_double, ctypes.c_uint32, p,
                                               u64, p]
        lib.fszo_compress_features.restype = ctypes.c_int
        lib.fszo_tile_eval_features.argtypes = [p, ctypes.c_int, ctypes.c_float, ctypes.c_uint32, p, p, p, p, p]
        lib.fszo_tile_eval_features.restype = ctypes.c_int
        lib.fszo_bound_config.argtypes = [u64, ctypes.c_int, ctypes.c_int]
        lib.fszo_bound_config.restype = u64
        lib.fszo_compress_config.argtypes = [p, u64, ctypes.c_int, ctypes.c_double, ctypes.c_uint32,
                                             ctypes.c_int, ctypes.c_int, p, u64, p]
        lib.fszo_compress_config.restype = ctypes.c_int
        lib.fszo_tile_eval_config.argtypes = [p, ctypes.c_int, ctypes.c_float, ctypes.c_uint32, ctypes.c_int,
                                              ctypes.c_int, p, p, p, p, p]
        lib.fszo_tile_eval_config.restype = ctypes.c_int
        lib.fszo_decompress.argtypes = [p, u64, p, u64]
        lib.fszo_decompress.restype = ctypes.c_int
        lib.fszo_set_threads.argtypes = [ctypes.c_int]
        lib.fszo_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1))


def set_threads(n: int) -> int:
    """Host threads for the oracle's tile loops (1 = serial); returns the previous count."""
    return int(_load().fszo_set_threads(n))


def bound(n: int) -> int:
    return int(_load().fszo_bound(n))


def bound_config(n: int, block: int, tile_blocks: int) -> int:
    return int(_load().fszo_bound_config(n, block, tile_blocks))


def resolve(x, mode: int, value: float):
    """Return (status, E, inv, flags)."""
    x = _f32(x)
    E = ctypes.c_float()
    inv = ctypes.c_float()
    flags = ctypes.c_uint32()
    st = _load().fszo_resolve(x.ctypes.data, x.size, mode, value, ctypes.byref(E),
                              ctypes.byref(inv), ctypes.byref(flags))
    return st, E.value, inv.value, flags.value


def compress_status(x, mode: int, value: float, capacity=None, features: int = FEATURES_ALL,
                    config=DEFAULT_CONFIG):
    """Return (status, stream bytes or None).  config = (B, T)."""
    x = _f32(x)
    B, T = config
    cap = (bound(x.size) if config == DEFAULT_CONFIG else bound_config(x.size, B, T)) \
        if capacity is None else capacity
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    size = ctypes.c_uint64()
    if tuple(config) != DEFAULT_CONFIG:
        st = _load().fszo_compress_config(x.ctypes.data, x.size, mode, value, features, B, T,
                                          out.ctypes.data, cap, ctypes.byref(size))
    elif features == FEATURES_ALL:
        st = _load().fszo_compress(x.ctypes.data, x.size, mode, value, out.ctypes.data, cap,
                                   ctypes.byref(size))
    else:
        st = _load().fszo_compress_features(x.ctypes.data, x.size, mode, value, features,
                                            out.ctypes.data, cap, ctypes.byref(size))
    if st != OK:
        return st, None
    return st, out[: size.value].tobytes()


def compress(x, mode: int, value: float, features: int = FEATURES_ALL, config=DEFAULT_CONFIG) -> bytes:
    st, s = compress_status(x, mode, value, features=features, config=config)
    if st != OK:
        raise OracleError(st, "compress")
    return s


def decompress_status(stream, n: int):
    buf = np.frombuffer(bytes(stream), dtype=np.uint8)
    if buf.size == 0:
        buf = np.zeros(1, dtype=np.uint8)
        size = 0
    else:
        size = buf.size
    out = np.zeros(max(n, 1), dtype=np.float32)
    st = _load().fszo_decompress(buf.ctypes.data, size, out.ctypes.data, n)
    return st, (out[:n] if st == OK else None)


def decompress(stream, n: int) -> np.ndarray:
    st, out = decompress_status(stream, n)
    if st != OK:
        raise OracleError(st, "decompress")
    return out


def tile_eval(x, inv: float):
    """Four-way evaluation of one tile: (mu, centre_ok, cost[4], rates[4][8])."""
    x = _f32(x)
    lib = _load()
    if not hasattr(lib, "_tile_eval_ready"):
        lib.fszo_tile_eval.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
        lib.fszo_tile_eval.restype = ctypes.c_int
        lib._tile_eval_ready = True
    mu = ctypes.c_int32()
    ok = ctypes.c_int()
    cost = np.zeros(4, dtype=np.uint32)
    rates = np.zeros((4, 8), dtype=np.uint32)
    st = lib.fszo_tile_eval(x.ctypes.data, x.size, inv, ctypes.byref(mu), ctypes.byref(ok),
                            cost.ctypes.data, rates.ctypes.data)
    if st != OK:
        raise OracleError(st, "tile_eval")
    return mu.value, bool(ok.value), cost, rates


def tile_eval_features(x, inv: float, features: int):
    """Evaluation of one tile under a feature subset:
    (mu, centre_ok, cost[4], rates[4][8], selected variant)."""
    x = _f32(x)
    mu = ctypes.c_int32()
    ok = ctypes.c_int()
    best = ctypes.c_int()
    cost = np.zeros(4, dtype=np.uint32)
    rates = np.zeros((4, 8), dtype=np.uint32)
    st = _load().fszo_tile_eval_features(x.ctypes.data, x.size, inv, features, ctypes.byref(mu),
                                         ctypes.byref(ok), cost.ctypes.data, rates.ctypes.data,
                                         ctypes.byref(best))
    if st != OK:
        raise OracleError(st, "tile_eval_features")
    return mu.value, bool(ok.value), cost, rates, best.value


def tile_eval_config(x, inv: float, features: int, block: int, tile_blocks: int):
    """Evaluation of one tile of a (B, T) configuration:
    (mu, centre_ok, cost[4], rates[4][T], selected variant)."""
    x = _f32(x)
    mu = ctypes.c_int32()
    ok = ctypes.c_int()
    best = ctypes.c_int()
    cost = np.zeros(4, dtype=np.uint32)
    rates = np.zeros((4, tile_blocks), dtype=np.uint32)
    st = _load().fszo_tile_eval_config(x.ctypes.data, x.size, inv, features, block, tile_blocks,
                                       ctypes.byref(mu), ctypes.byref(ok), cost.ctypes.data, rates.ctypes.data,
                                       ctypes.byref(best))
    if st != OK:
        raise OracleError(st, "tile_eval_config")
    return mu.value, bool(ok.value), cost, rates, best.value
