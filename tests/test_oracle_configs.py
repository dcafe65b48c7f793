"""Pins of the oracle's tile configurations (Sec. VI-C, Table V): block size
B in {32, 64}, blocks per tile T in {4, 8, 16}.

Checked against facts outside the oracle: a brute-force Python evaluation
of every variant (four full residual passes, 64-bit words built by Python
integers), an independent Python encoder, the reconstruction (which
depends on the quantized values alone, so it is the same closed form under
every configuration), and relations between configurations that follow
from the definitions: a 64-element block's rate is the larger of the rates
of its two 32-element halves (the bit length of a maximum is the maximum of
the bit lengths) when both cover the same tile, and a longer tile's first
blocks see the same uncentred residuals as a shorter tile's (the prediction
chain starts at the same tile start).
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import workloads
from tests import fsz_format as fmt
from tests.test_oracle import _fields, unit_grid

CONFIGS = oracle.CONFIGS
NONDEFAULT = [c for c in CONFIGS if c != oracle.DEFAULT_CONFIG]


def _tiles(rng, tile):
    """Small integer tiles of every kind, ragged lengths included."""
    for _ in range(60):
        m = int(rng.choice([1, 2, 3, 31, 32, 33, 63, 64, 65, tile // 2 + 7, tile - 1, tile]))
        m = min(m, tile)
        kind = rng.integers(0, 5)
        i = np.arange(m)
        if kind == 0:
            q = rng.integers(-3, 4, m)
        elif kind == 1:
            q = np.cumsum(rng.integers(-2, 3, m)) + rng.integers(-3000, 3000)
        elif kind == 2:
            q = rng.integers(-50, 50) + rng.integers(-5, 6) * i + rng.integers(-2, 3, m)
        elif kind == 3:
            q = np.full(m, rng.integers(-5000, 5000)) + rng.integers(-1, 2, m)
        else:
            q = rng.integers(-2 ** 12, 2 ** 12, m)
        yield np.asarray(q, dtype=np.int64)


@pytest.mark.parametrize("config", CONFIGS)
def test_config_bruteforce_tiles(config):
    B, T = config
    rng = np.random.default_rng(100 + B + T)
    for q in _tiles(rng, B * T):
        x, eb, E, inv = unit_grid(q)
        for features in (oracle.FEATURES_ALL, 0, oracle.FEAT_CROSS_BLOCK | oracle.FEAT_LZ2):
            mu_bf, ok_bf, cost_bf, rates_bf, best_bf = fmt.brute_force_tile(x, inv, features, B, T)
            mu, ok, cost, rates, best = oracle.tile_eval_config(x, inv, features, B, T)
            assert (mu, ok) == (mu_bf, ok_bf)
            assert list(cost) == cost_bf
            assert rates.tolist() == rates_bf
            assert best == best_bf


@pytest.mark.parametrize("config", CONFIGS)
def test_config_stream_matches_python_encoder(config):
    B, T = config
    rng = np.random.default_rng(200 + B + T)
    for n in (1, 33, 65, B * T, B * T + 1, 3 * B * T - 5):
        for features in (oracle.FEATURES_ALL, 0):
            q = np.cumsum(rng.integers(-4, 5, n)) + rng.integers(-300, 300)
            x, eb, E, inv = unit_grid(q)
            choices = []
            for t in range(fmt.ceil_div(n, B * T)):
                mu, _, _, _, best = fmt.brute_force_tile(x[t * B * T:(t + 1) * B * T], inv, features, B, T)
                choices.append((best & 1, best >> 1, mu))
            flags = 0 if features & fmt.CROSS_BLOCK else 2
            ref = fmt.encode_stream(x, E, inv, oracle.ABS, eb, flags, choices, B, T)
            s = oracle.compress(x, oracle.ABS, eb, features=features, config=config)
            assert s == ref, (config, n, features)
            assert fmt.header_config(fmt.parse_header(s)["flags"]) == config
            assert np.array_equal(oracle.decompress(s, n).view(np.uint32),
                                  fmt.closed_form(x, E, inv).view(np.uint32))


@pytest.mark.parametrize("name,x", list(_fields()))
def test_configs_reconstruct_the_same_field(name, x):
    """Sec. IV-B: the reconstruction is the quantized value times the step,
    whatever the encoding, so every configuration decodes to the same bits
    (and within the bound); sizes follow the tile costs."""
    for rel in (1e-2, 1e-4):
        st, E, inv, _ = oracle.resolve(x, oracle.REL, rel)
        if st == oracle.ERR_EB_TOO_SMALL:
            continue
        ref = fmt.closed_form(x, E, inv)
        for config in CONFIGS:
            B, T = config
            s = oracle.compress(x, oracle.REL, rel, config=config)
            y = oracle.decompress(s, x.size)
            assert np.array_equal(y.view(np.uint32), ref.view(np.uint32)), (name, rel, config)
            assert len(s) == fmt.data_start(x.size, B) + sum(fmt.tile_sizes(s, x.size, B, T))
            assert len(s) <= oracle.bound_config(x.size, B, T)


def test_default_config_call_is_the_plain_stream():
    lib = oracle._load()
    for name, x in list(_fields())[:4]:
        exp = oracle.compress(x, oracle.REL, 1e-3)
        cap = oracle.bound(x.size)
        out = np.zeros(cap, dtype=np.uint8)
        size = ctypes.c_uint64()
        st = lib.fszo_compress_config(x.ctypes.data, x.size, oracle.REL, 1e-3, oracle.FEATURES_ALL, 32, 8,
                                      out.ctypes.data, cap, ctypes.byref(size))
        assert st == oracle.OK
        assert out[:size.value].tobytes() == exp, name
        assert oracle.bound_config(x.size, 32, 8) == cap


@pytest.mark.parametrize("small,large", [((32, 8), (64, 4)), ((32, 16), (64, 8))])
def test_block64_rate_is_max_of_its_halves(small, large):
    """Same tile (B*T equal): the 64-element block k covers the 32-element
    blocks 2k and 2k+1 with the same residuals, so its rate is their
    maximum under every variant, the mean is the same, and its cost is
    8 + 8r instead of two 4 + 4r."""
    (b1, t1), (b2, t2) = small, large
    assert b1 * t1 == b2 * t2
    rng = np.random.default_rng(7 + t2)
    for q in _tiles(rng, b1 * t1):
        x, eb, E, inv = unit_grid(q)
        mu1, ok1, _, r32, _ = oracle.tile_eval_config(x, inv, oracle.FEATURES_ALL, b1, t1)
        mu2, ok2, cost64, r64, _ = oracle.tile_eval_config(x, inv, oracle.FEATURES_ALL, b2, t2)
        assert (mu1, ok1) == (mu2, ok2)
        assert np.array_equal(r64, np.maximum(r32[:, 0::2], r32[:, 1::2]))
        for v in range(4):
            assert cost64[v] == sum(0 if r == 0 else 8 + 8 * int(r) for r in r64[v]) + (4 if v >> 1 else 0)


@pytest.mark.parametrize("short,long", [((32, 4), (32, 8)), ((32, 8), (32, 16)), ((64, 4), (64, 8)),
                                        ((64, 8), (64, 16))])
def test_longer_tile_extends_the_chain(short, long):
    """The first T_short blocks of a longer tile hold the same uncentred
    residuals as the shorter tile over the same elements; the blocks after
    them continue the chain instead of restarting it, so their LZ1 rate is
    the bit length of the plain first differences."""
    (B, ts), (_, tl) = short, long
    rng = np.random.default_rng(3 + tl)
    for q in _tiles(rng, B * tl):
        x, eb, E, inv = unit_grid(q)
        _, _, _, r_short, _ = oracle.tile_eval_config(x[:B * ts], inv, oracle.FEATURES_ALL, B, ts)
        _, _, _, r_long, _ = oracle.tile_eval_config(x, inv, oracle.FEATURES_ALL, B, tl)
        assert np.array_equal(r_long[:2, :ts], r_short[:2, :])
        d = np.abs(np.diff(np.asarray(q, dtype=np.int64)))
        for b in range(ts, fmt.ceil_div(q.size, B)):
            seg = d[b * B - 1:min((b + 1) * B, q.size) - 1]
            assert r_long[0, b] == fmt.bitlen(int(seg.max()))


def test_config_header_bits_and_rejections():
    x = workloads.sinusoid_field(5000, 3)
    for config in CONFIGS:
        s = oracle.compress(x, oracle.REL, 1e-3, config=config)
        flags = fmt.parse_header(s)["flags"]
        assert flags & ~0x1F == 0 and fmt.header_config(flags) == config
        # the reserved tile code and the bits above it are rejected
        for bad in ((flags & ~0x18) | 0x18, flags | 0x20, flags | 0x80):
            c = bytearray(s)
            c[7] = bad
            assert oracle.decompress_status(bytes(c), x.size)[0] == oracle.ERR_CORRUPT
    for B, T in ((16, 8), (32, 2), (32, 32), (128, 4), (64, 0)):
        assert oracle.compress_status(x, oracle.REL, 1e-3, config=(B, T), capacity=10 ** 6)[0] \
            == oracle.ERR_INVALID_ARG
        assert oracle.bound_config(x.size, B, T) == 0


@pytest.mark.parametrize("config", NONDEFAULT)
def test_config_worst_case_fits_the_bound(config):
    """Incompressible input at a tiny bound: the stream stays within the
    configuration's bound (every block at the rate the bound allows)."""
    B, T = config
    rng = np.random.default_rng(5)
    for n in (1, 100, B * T * 3 + 17):
        x = rng.uniform(-1, 1, n).astype(np.float32)
        s = oracle.compress(x, oracle.REL, 1e-6, config=config)
        assert len(s) <= oracle.bound_config(n, B, T)
        st, _ = oracle.compress_status(x, oracle.REL, 1e-6, capacity=len(s) - 1, config=config)
        assert st == oracle.ERR_CAPACITY


@pytest.mark.parametrize("config", CONFIGS)
def test_tile_sizes_array_form(config):
    """The array form of the per-tile size sum (used on streams of millions
    of tiles) agrees with the per-tile form and with the stream's length."""
    B, T = config
    for n, seed in ((1, 1), (B * T + 1, 2), (40000, 3)):
        x = workloads.sinusoid_field(n, seed)
        s = oracle.compress(x, oracle.REL, 1e-4, config=config)
        sizes = fmt.tile_sizes_np(s, n, B, T)
        assert sizes.tolist() == fmt.tile_sizes(s, n, B, T)
        assert fmt.data_start(n, B) + int(sizes.sum()) == len(s)
