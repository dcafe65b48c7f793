"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: the checks are the paper's
worked examples (tests/golden), the pointwise error bound, the cancellation
identity Eq. (4), brute-force four-pass variant choice, closed-form sizes and
exact round trips on constant / linear / quadratic inputs, the rate-header
compression cap, an independent Python encoder whose streams (with arbitrary
variant choices) the decoder must invert, and rejection of corrupt streams.
"""
import json
import os
import struct

import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import workloads
from tests import fsz_format as fmt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def unit_grid(q):
    """Floats equal to integers q, with an ABS bound whose step E is ~1.

    Returns (x, eb, E, inv) after checking that quantization recovers q.
    """
    x = np.asarray(q, dtype=np.float32)
    # a bound just above 1/2 plus the 4-ulp tightening of the step gives E = 1 + O(1e-6)
    eb = 0.5 + 4 * float(np.spacing(np.abs(x).max())) + 1e-6
    st, E, inv, _ = oracle.resolve(x, oracle.ABS, eb)
    assert st == oracle.OK and 1.0 <= E < 1.00001
    assert np.array_equal(fmt.quantize(x, inv), np.asarray(q, dtype=np.int64))
    return x, eb, E, inv


# ---------------------------------------------------------------- figures


def test_fig2_cross_block_state():
    g = golden("fig2_cross_block.json")
    q = np.concatenate([g["start"][b] + np.arange(32) // g["step"][b] for b in range(8)])
    x, _, _, inv = unit_grid(q)
    _, _, _, rates = oracle.tile_eval(x, inv)
    for k, b in enumerate(g["blocks_checked"]):
        assert q[32 * b] == g["boundary_values"][k]
        # cross-block state (Eq. (2)): LZ1 rate of the block
        assert rates[0][b] == g["cross_block_rate"]
        # independent blocks (Eq. (1)): the raw boundary value is the first residual
        blk = q[32 * b:32 * b + 32]
        indep = max([abs(int(blk[0]))] + [abs(int(d)) for d in np.diff(blk)])
        assert fmt.bitlen(indep) == g["independent_rates"][k]
    worst = max(fmt.block_cost(r) for r in g["independent_rates"])
    assert worst - fmt.block_cost(g["cross_block_rate"]) == g["max_saving_bytes"]


def test_fig3_lz1_vs_lz2():
    g = golden("fig3_lz1_vs_lz2.json")
    q = g["offset"] + g["stride"] * np.arange(256)
    x, _, _, inv = unit_grid(q)
    _, _, _, rates = oracle.tile_eval(x, inv)
    b = g["block"]
    assert rates[0][b] == g["lz1_rate"] and fmt.block_cost(rates[0][b]) == g["lz1_cost_bytes"]
    assert rates[1][b] == g["lz2_rate"] and fmt.block_cost(rates[1][b]) == g["lz2_cost_bytes"]


def test_fig4_centering():
    g = golden("fig4_centering.json")
    q = g["base"] + np.array(g["pattern"] * 64)
    x, eb, _, inv = unit_grid(q)
    mu, ok, cost, rates = oracle.tile_eval(x, inv)
    assert ok and mu == g["mu"]
    assert q[0] - mu == g["centred_first_residual"]
    assert rates[0][0] == g["uncentred_block0_rate"]
    assert fmt.block_cost(rates[0][0]) == g["uncentred_block0_bytes"]
    assert rates[2][0] == g["centred_block0_rate"]
    centred = fmt.block_cost(rates[2][0]) + 4
    assert centred == g["centred_block0_bytes_with_mu"]
    assert g["uncentred_block0_bytes"] / centred == pytest.approx(g["saving_factor"])
    # the rest of the tile is identical under centering (Eq. (4))
    assert cost[0] - cost[2] == g["uncentred_block0_bytes"] - centred
    # the whole tile selects LZ1 + centering
    s = oracle.compress(x, oracle.ABS, eb)
    order2, cen, _ = fmt.tile_choices(s, x.size)[0]
    assert (order2, cen) == (0, 1)


# ---------------------------------------------------------------- bound


def _fields():
    rng = np.random.default_rng(11)
    n = 1 << 16
    yield "uniform", rng.uniform(-1, 1, n).astype(np.float32)
    yield "normal", rng.normal(0, 3, n).astype(np.float32)
    yield "offset", (1000 + rng.uniform(0, 1, n)).astype(np.float32)
    yield "lognormal", (rng.lognormal(0, 4, n) * rng.choice([-1, 1], n)).astype(np.float32)
    yield "sinusoid", workloads.sinusoid_field(n, 5)
    yield "grf", workloads.grf_field((32, 32, 64), 7)
    yield "pwq", workloads.piecewise_quadratic((8, 40, 200), 9)


@pytest.mark.parametrize("mode,value", [(1, 1e-2), (1, 1e-3), (1, 1e-4), (1, 1e-5), (0, 1e-3),
                                        (0, 0.25)])
def test_pointwise_bound(mode, value):
    for name, x in _fields():
        st, s = oracle.compress_status(x, mode, value)
        if st == oracle.ERR_EB_TOO_SMALL:
            continue
        assert st == oracle.OK, name
        y = oracle.decompress(s, x.size)
        x64 = x.astype(np.float64)
        eb = value if mode == 0 else value * (x64.max() - x64.min())
        err = np.abs(x64 - y.astype(np.float64)).max()
        assert err <= eb, (name, err, eb)


def test_literal_quantizer_breaks_bound():
    """Why the step is tightened: fl32 arithmetic with E = 2 eb misses the bound."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 1 << 20).astype(np.float32)
    eb = 1e-4 * (float(x.max()) - float(x.min()))
    E = np.float32(2 * eb)
    inv = np.float32(1) / E
    y = fmt.quantize(x, inv).astype(np.float32) * E
    assert (np.abs(x.astype(np.float64) - y.astype(np.float64)) > eb).sum() > 0


# ---------------------------------------------------------------- Eq. (4)


def test_cancellation_identity():
    rng = np.random.default_rng(5)
    for _ in range(200):
        q = rng.integers(-2 ** 20, 2 ** 20, 256)
        mu = int(rng.integers(-2 ** 20, 2 ** 20))
        for order2, k in ((0, 1), (1, 2)):
            a = fmt.residuals(q, order2, 0)
            b = fmt.residuals(q, order2, mu)
            assert np.array_equal(a[k:], b[k:])
            # zero state before the tile: exactly the first k residuals move
            assert b[0] == a[0] - mu
            if order2:
                assert b[1] == a[1] + mu


def one_pass_rates(q, mu):
    """The one-read evaluation that Eq. (4) licenses (and the kernels use):
    plain LZ1 / LZ2 residuals once; a block without a prediction restart has
    one rate per order for all four variants; block 0 of each variant is
    rated from its inner residuals plus its first one (LZ1) or two (LZ2)
    residuals, moved by the tile mean for a centred variant."""
    m = len(q)
    l1 = fmt.residuals(q, 0, 0)
    l2 = fmt.residuals(q, 1, 0)
    nb = fmt.ceil_div(m, 32)
    rates = [[0] * 8 for _ in range(4)]
    for b in range(nb):
        blk1 = [abs(int(v)) for v in l1[32 * b:32 * b + 32]]
        blk2 = [abs(int(v)) for v in l2[32 * b:32 * b + 32]]
        for v in range(4):
            order2, cen = v & 1, v >> 1
            if b > 0:
                a = max(blk2 if order2 else blk1)
            else:
                c = mu if cen else 0
                inner = blk2[2:] if order2 else blk1[1:]
                first = [abs(int(q[0]) - c)]
                if order2 and m >= 2:
                    first.append(abs(int(l2[1]) + c))
                a = max(inner + first)
            rates[v][b] = fmt.bitlen(a)
    cost = [sum(fmt.block_cost(r) for r in rates[v]) + 4 * (v >> 1) for v in range(4)]
    return rates, cost


def test_one_pass_evaluation_equals_plain_definition():
    """Eq. (4) as a property: the one-read four-way evaluation gives the
    oracle's per-variant rates and costs, which it forms from four full
    residual passes."""
    rng = np.random.default_rng(9)
    for q in _tiny_tiles(rng):
        x, eb, E, inv = unit_grid(q)
        mu, ok, cost, rates = oracle.tile_eval(x, inv)
        r1, c1 = one_pass_rates(q, mu)
        assert rates.tolist() == r1
        assert list(cost) == c1


# ---------------------------------------------------------------- brute force


def _tiny_tiles(rng):
    for _ in range(300):
        m = int(rng.choice([1, 2, 3, 31, 32, 33, 64, 100, 200, 255, 256]))
        kind = rng.integers(0, 6)
        i = np.arange(m)
        if kind == 0:
            q = rng.integers(-3, 4, m)
        elif kind == 1:
            q = np.cumsum(rng.integers(-2, 3, m)) + rng.integers(-3000, 3000)
        elif kind == 2:
            q = rng.integers(-50, 50) + rng.integers(-5, 6) * i + rng.integers(-2, 3, m)
        elif kind == 3:
            q = np.full(m, rng.integers(-5000, 5000)) + rng.integers(-1, 2, m)
        elif kind == 4:
            q = rng.integers(-20, 20) * i * i // 64 + rng.integers(-9, 9) * i
        else:
            q = rng.integers(-2 ** 12, 2 ** 12, m)
        yield np.asarray(q, dtype=np.int64)


def test_bruteforce_variant_choice():
    rng = np.random.default_rng(21)
    for q in _tiny_tiles(rng):
        x, eb, E, inv = unit_grid(q)
        mu_bf, ok_bf, cost_bf, rates_bf, best = fmt.brute_force_tile(x, inv)
        mu, ok, cost, rates = oracle.tile_eval(x, inv)
        assert ok == ok_bf
        assert mu == mu_bf
        assert list(cost) == cost_bf
        assert rates.tolist() == rates_bf
        s = oracle.compress(x, oracle.ABS, eb)
        order2, cen, r = fmt.tile_choices(s, x.size)[0]
        assert (order2 + 2 * cen) == best
        assert r == rates_bf[best]
        assert fmt.tile_sizes(s, x.size)[0] == cost_bf[best]


def test_bruteforce_multi_tile_stream_matches_python_encoder():
    """The oracle's bytes equal an independent encoder fed the brute-force choices."""
    rng = np.random.default_rng(8)
    for n in (1, 37, 256, 300, 513, 1000, 2048 + 77):
        q = np.cumsum(rng.integers(-4, 5, n)) + rng.integers(-100, 100)
        x, eb, E, inv = unit_grid(q)
        choices = []
        for t in range(fmt.ceil_div(n, 256)):
            mu, ok, _, _, best = fmt.brute_force_tile(x[t * 256:(t + 1) * 256], inv)
            choices.append((best & 1, best >> 1, mu))
        ref = fmt.encode_stream(x, E, inv, oracle.ABS, eb, 0, choices)
        assert oracle.compress(x, oracle.ABS, eb) == ref


def test_centering_disabled_on_nonfinite_mean():
    x = np.full(256, 3.0e38, dtype=np.float32)
    x[::2] = 2.9e38
    st, E, inv, _ = oracle.resolve(x, oracle.ABS, 1e35)
    assert st == oracle.OK
    mu, ok, cost, _ = oracle.tile_eval(x, inv)
    assert not ok and mu == 0
    s = oracle.compress(x, oracle.ABS, 1e35)
    assert fmt.tile_choices(s, 256)[0][1] == 0
    y = oracle.decompress(s, 256)
    assert np.abs(x.astype(np.float64) - y).max() <= 1e35


# ---------------------------------------------------------------- closed forms


def _on_grid(q, eb):
    """x = fl32(q * E) for the oracle's step E at this eb (checked stable)."""
    q = np.asarray(q, dtype=np.int64)
    x = q.astype(np.float32)
    E = None
    for _ in range(8):  # E depends on max|x| through the ulp tightening: iterate to a fixed point
        st, E2, inv2, _ = oracle.resolve(x, oracle.ABS, eb)
        assert st == oracle.OK
        if E2 == E:
            break
        E = E2
        x = (q.astype(np.float32) * np.float32(E)).astype(np.float32)
    assert E2 == E
    assert np.array_equal(fmt.quantize(x, inv2), q)
    return x, E, inv2


def test_zero_field_size():
    n = 4096
    x = np.zeros(n, dtype=np.float32)
    s = oracle.compress(x, oracle.ABS, 1e-3)
    assert len(s) == 32 + fmt.pad16(n // 32)
    assert np.array_equal(oracle.decompress(s, n), x)


@pytest.mark.parametrize("c", [1013.25, -7.5, 3.0e-20])
def test_constant_field_rel(c):
    n = 256 * 17
    x = np.full(n, c, dtype=np.float32)
    s = oracle.compress(x, oracle.REL, 1e-3)
    h = fmt.parse_header(s)
    assert h["flags"] == 1 and h["E"] == abs(np.float32(c))
    assert len(s) == 32 + fmt.pad16(n // 32) + 4 * (n // 256)
    rb = fmt.rate_bytes(s, n)
    assert all(rb[0::8] == 0x40) and not rb.reshape(-1, 8)[:, 1:].any()
    assert np.array_equal(oracle.decompress(s, n), x)


def test_constant_field_abs_grid():
    n = 256 * 9
    x, E, inv = _on_grid(np.full(n, 4321), 0.01)
    s = oracle.compress(x, oracle.ABS, 0.01)
    assert len(s) == 32 + fmt.pad16(n // 32) + 4 * (n // 256)
    assert np.array_equal(oracle.decompress(s, n), x)


def test_linear_field_exact():
    n = 256 * 8
    q = -700 + 5 * np.arange(n)
    x, E, inv = _on_grid(q, 0.02)
    s = oracle.compress(x, oracle.ABS, 0.02)
    for order2, cen, rates in fmt.tile_choices(s, n):
        assert order2 == 1 and rates[1:] == [0] * 7
    assert np.array_equal(oracle.decompress(s, n), x)


def test_quadratic_field_exact():
    n = 256 * 3
    i = np.arange(n)
    c = 2
    q = c * (i - n // 2) ** 2 + 7 * i - 11
    x, E, inv = _on_grid(q, 100.0)
    s = oracle.compress(x, oracle.ABS, 100.0)
    for order2, cen, rates in fmt.tile_choices(s, n):
        assert order2 == 1 and rates[1:] == [fmt.bitlen(2 * c)] * 7
    assert np.array_equal(oracle.decompress(s, n), x)


def test_compression_ratio_cap():
    for name, x in _fields():
        s = oracle.compress(x, oracle.REL, 1e-2)
        assert len(s) >= 32 + fmt.pad16(fmt.ceil_div(x.size, 32))
        assert 4 * x.size / len(s) < 128


def test_reconstruction_closed_form():
    for name, x in _fields():
        for mode, value in ((1, 1e-3), (0, 1e-2)):
            st, s = oracle.compress_status(x, mode, value)
            if st == oracle.ERR_EB_TOO_SMALL:  # the lognormal field at ABS 1e-2
                continue
            st, E, inv, _ = oracle.resolve(x, mode, value)
            assert np.array_equal(oracle.decompress(s, x.size), fmt.closed_form(x, E, inv)), name


def test_offsets_are_exclusive_scan():
    x = workloads.piecewise_quadratic((4, 30, 90), 3)
    s = oracle.compress(x, oracle.REL, 1e-3)
    n = x.size
    sizes = fmt.tile_sizes(s, n)
    st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
    off = fmt.data_start(n)
    for t, (order2, cen, _) in enumerate(fmt.tile_choices(s, n)):
        if cen:
            mu = struct.unpack_from("<i", s, off)[0]
            assert mu == fmt.pairwise_mean(x[t * 256:(t + 1) * 256], inv)[1]
        off += sizes[t]
    assert off == len(s)


# ---------------------------------------------------------------- decoder


def test_decoder_accepts_any_variant():
    rng = np.random.default_rng(4)
    for n in (5, 256, 700, 1500):
        x = workloads.sinusoid_field(n, int(rng.integers(1000)))
        st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
        choices = [(int(rng.integers(2)), int(rng.integers(2)), int(rng.integers(-5000, 5000)))
                   for _ in range(fmt.ceil_div(n, 256))]
        s = fmt.encode_stream(x, E, inv, oracle.REL, 1e-3, 0, choices)
        assert np.array_equal(oracle.decompress(s, n), fmt.closed_form(x, E, inv))


@pytest.mark.parametrize("n", [1, 2, 31, 33, 255, 257, 511, 1000, 4097])
def test_ragged_round_trip(n):
    x = workloads.sinusoid_field(n, n)
    s = oracle.compress(x, oracle.REL, 1e-3)
    y = oracle.decompress(s, n)
    st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
    assert np.array_equal(y, fmt.closed_form(x, E, inv))


def test_empty_stream():
    s = oracle.compress(np.zeros(0, np.float32), oracle.REL, 1e-3)
    assert len(s) == 32 and fmt.parse_header(s)["n"] == 0
    assert oracle.decompress(s, 0).size == 0


# ---------------------------------------------------------------- status codes


def test_status_codes():
    x = workloads.sinusoid_field(1000, 1)
    bad = x.copy()
    bad[17] = np.nan
    assert oracle.compress_status(bad, oracle.REL, 1e-3)[0] == oracle.ERR_NONFINITE
    bad[17] = np.inf
    assert oracle.compress_status(bad, oracle.ABS, 1e-3)[0] == oracle.ERR_NONFINITE
    assert oracle.compress_status(x, oracle.ABS, 1e-9)[0] == oracle.ERR_EB_TOO_SMALL
    assert oracle.compress_status(x, 2, 1e-3)[0] == oracle.ERR_INVALID_ARG
    assert oracle.compress_status(x, oracle.REL, 0.0)[0] == oracle.ERR_INVALID_ARG
    assert oracle.compress_status(x, oracle.REL, float("nan"))[0] == oracle.ERR_INVALID_ARG
    assert oracle.compress_status(x, oracle.REL, 1e-3, capacity=100)[0] == oracle.ERR_CAPACITY
    big = np.full(10, 3.3e38, dtype=np.float32)
    big[0] = -1.0
    assert oracle.compress_status(big, oracle.ABS, 1e37)[0] == oracle.ERR_EB_TOO_LARGE
    sub = np.full(10, 1e-40, dtype=np.float32)
    assert oracle.compress_status(sub, oracle.REL, 1e-3)[0] == oracle.ERR_EB_TOO_SMALL


def _mutations(s, n):
    d0 = fmt.data_start(n)
    b = bytearray(s)

    def m(f):
        c = bytearray(b)
        f(c)
        return bytes(c)

    yield "magic", m(lambda c: c.__setitem__(0, ord("G"))), oracle.ERR_CORRUPT
    yield "version", m(lambda c: c.__setitem__(4, 2)), oracle.ERR_CORRUPT
    yield "mode", m(lambda c: c.__setitem__(6, 2)), oracle.ERR_CORRUPT
    yield "flags", m(lambda c: c.__setitem__(7, 0x20)), oracle.ERR_CORRUPT
    yield "tile code", m(lambda c: c.__setitem__(7, 0x18)), oracle.ERR_CORRUPT
    yield "n", m(lambda c: struct.pack_into("<Q", c, 8, n + 1)), oracle.ERR_SIZE_MISMATCH
    yield "E nan", m(lambda c: struct.pack_into("<f", c, 16, float("nan"))), oracle.ERR_CORRUPT
    yield "E zero", m(lambda c: struct.pack_into("<f", c, 16, 0.0)), oracle.ERR_CORRUPT
    yield "total", m(lambda c: struct.pack_into("<Q", c, 24, len(s) + 4)), oracle.ERR_CORRUPT
    yield "reserved0", m(lambda c: c.__setitem__(32, c[32] | 0x20)), oracle.ERR_CORRUPT
    yield "reserved1", m(lambda c: c.__setitem__(33, c[33] | 0x80)), oracle.ERR_CORRUPT
    yield "rate+1", m(lambda c: c.__setitem__(34, (c[34] & 0xE0) | min(31, (c[34] & 0x1F) + 1))), \
        oracle.ERR_CORRUPT
    if d0 > 32 + fmt.ceil_div(n, 32):
        yield "padding", m(lambda c: c.__setitem__(d0 - 1, 1)), oracle.ERR_CORRUPT


def test_corrupt_streams_rejected():
    n = 1000
    x = workloads.sinusoid_field(n, 2)
    s = oracle.compress(x, oracle.REL, 1e-4)
    assert oracle.decompress_status(s, n)[0] == oracle.OK
    for name, c, want in _mutations(s, n):
        assert oracle.decompress_status(c, n)[0] == want, name
    assert oracle.decompress_status(s[:-4], n)[0] == oracle.ERR_CORRUPT
    assert oracle.decompress_status(s[:20], n)[0] == oracle.ERR_CORRUPT


@pytest.mark.parametrize("config", oracle.CONFIGS)
def test_threaded_oracle_writes_the_serial_bytes(config):
    """The CPU baseline's parallel mode (tiles over host threads) writes the
    same stream and decodes to the same floats as the serial oracle."""
    x = workloads.piecewise_quadratic((6, 50, 70), 4)[:20_993]
    old = oracle.set_threads(1)
    try:
        feats = (oracle.FEATURES_ALL, 0, oracle.FEAT_CENTERING)
        serial = [oracle.compress(x, oracle.REL, 1e-3, features=f, config=config) for f in feats]
        dec = [oracle.decompress(s, x.size) for s in serial]
        oracle.set_threads(5)
        for f, s, y in zip(feats, serial, dec):
            assert oracle.compress(x, oracle.REL, 1e-3, features=f, config=config) == s
            assert np.array_equal(oracle.decompress(s, x.size), y)
    finally:
        oracle.set_threads(old)


def test_tile_mean_is_pairwise_binary32():
    """mu follows the index-order pairwise binary32 tree (a sequential sum differs)."""
    rng = np.random.default_rng(17)
    inv = float(np.float32(2.0 ** 20))
    differs = 0
    for _ in range(400):
        m = int(rng.choice([256, 255, 130]))
        xt = (rng.uniform(-1, 1, m) * 10.0 ** rng.integers(-3, 3, m)).astype(np.float32)
        mu, ok, _, _ = oracle.tile_eval(xt, inv)
        ok_ref, mu_ref = fmt.pairwise_mean(xt, inv)
        assert ok and ok_ref and mu == mu_ref
        seq = np.float32(0)
        for v in xt:
            seq = np.float32(seq + v)
        mu_seq = int(np.rint(np.float32(np.float32(seq * np.float32(0.00390625)) * np.float32(inv))))
        differs += mu_seq != mu
    assert differs > 0  # the test data is sensitive to the summation order


def test_bound_large_uniform_sample():
    """2^20 uniform samples at tight REL bounds: the regime where an untightened step fails."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, 1 << 20).astype(np.float32)
    for rel in (1e-3, 1e-4, 1e-5):
        s = oracle.compress(x, oracle.REL, rel)
        y = oracle.decompress(s, x.size).astype(np.float64)
        eb = rel * (float(x.max()) - float(x.min()))
        assert np.abs(x.astype(np.float64) - y).max() <= eb
