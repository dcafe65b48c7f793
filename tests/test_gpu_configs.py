"""GPU parity of the tile configurations (Sec. VI-C, Table V): block size B
in {32, 64}, T in {4, 8, 16} blocks per tile.  For every configuration the
HIP streams equal the oracle's byte for byte (aligned and unaligned inputs,
ragged tails, several chunks), the configuration decoder reconstructs the
oracle's streams bit for bit, the default configuration through these entry
points gives the plain stream, and errors are reported as the oracle
reports them.  At the benchmark's size (the 512^3 field) the decode is
checked against the closed form over the whole field and the first tiles'
bytes against the oracle's stream of the same elements.  Every case prints
its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests import fsz_format as fmt
from tests.test_gpu_parity import _fuzz_field, announce, first_diff, gpu_compress

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CONFIGS = oracle.CONFIGS


def _dev():
    return torch.device("cuda:0")


def _stream():
    return torch.cuda.current_stream(_dev()).cuda_stream


def gpu_compress_config(x, mode, value, config, in_offset=0, capacity=None, device_x=None):
    """Returns (status, stream bytes or None)."""
    B, T = config
    n = x.size if device_x is None else device_x.numel()
    if device_x is None:
        xd = torch.zeros(n + in_offset + 4, dtype=torch.float32, device=_dev())
        if n:
            xd[in_offset:in_offset + n] = torch.from_numpy(x).to(_dev())
        ptr = xd.data_ptr() + 4 * in_offset
    else:
        ptr = device_x.data_ptr()
    cap = fsz.fsz_compressed_bound_config(n, B, T) if capacity is None else capacity
    out = torch.zeros(max(cap, 1), dtype=torch.uint8, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    st = fsz.fsz_compress_config_async(ptr, n, mode, value, None, B, T, out.data_ptr(), cap, res.data_ptr(),
                                       _stream())
    if st != fsz.FSZ_OK:
        return st, None
    torch.cuda.synchronize()
    r = res.cpu()
    size, st = int(r[0]), int(r[1]) & 0xFFFFFFFF
    if st != fsz.FSZ_OK:
        return st, None
    return st, out[:size].cpu().numpy().tobytes()


def gpu_decompress_config(stream_bytes, n, config, out_offset=0):
    """Returns (status, float32 array or None); checks nothing is written
    outside the n outputs."""
    B, T = config
    buf = torch.from_numpy(np.frombuffer(stream_bytes, dtype=np.uint8).copy()).to(_dev())
    guard = 8
    out = torch.full((n + out_offset + 2 * guard,), float("nan"), dtype=torch.float32, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    st = fsz.fsz_decompress_config_async(buf.data_ptr(), len(stream_bytes), out.data_ptr() + 4 * (guard + out_offset),
                                         n, B, T, res.data_ptr(), _stream())
    if st != fsz.FSZ_OK:
        return st, None
    torch.cuda.synchronize()
    st = int(res.cpu()[1]) & 0xFFFFFFFF
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[:guard + out_offset])) and np.all(np.isnan(o[guard + out_offset + n:]))
    return st, (o[guard + out_offset:guard + out_offset + n] if st == fsz.FSZ_OK else None)


def _fields():
    yield "sinusoid 1", workloads.sinusoid_field(1, 3)
    yield "sinusoid 1000", workloads.sinusoid_field(1000, 4)
    yield "pwq 8x40x200 (64000)", workloads.piecewise_quadratic((8, 40, 200), 5)
    yield "grf 64x64x80 (40 chunks)", workloads.grf_field((64, 64, 80), 6)
    yield "pwq 5x301x181 (ragged tail, 272405)", workloads.piecewise_quadratic((5, 301, 181), 7)


@pytest.mark.parametrize("config", CONFIGS)
def test_config_streams_match_oracle(config):
    for name, x in _fields():
        for rel in (1e-2, 1e-4):
            exp = oracle.compress(x, oracle.REL, rel, config=config)
            for off in (0, 1):
                announce(f"config {config} {name} REL {rel:g} input offset {off}")
                st, got = gpu_compress_config(x, oracle.REL, rel, config, in_offset=off)
                assert st == fsz.FSZ_OK
                assert got == exp, first_diff(got, exp)
            y_ref = oracle.decompress(exp, x.size)
            for off in (0, 1):
                announce(f"config {config} decode {name} REL {rel:g} output offset {off}")
                st, y = gpu_decompress_config(exp, x.size, config, out_offset=off)
                assert st == fsz.FSZ_OK
                assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32))


@pytest.mark.parametrize("config", CONFIGS)
def test_config_edge_sizes(config):
    """Sizes around a block (B), a tile (B T), a wave (64 segments of 32) and
    a chunk (32768 elements) of the configuration kernels: streams byte for
    byte, decodes bit for bit against the oracle."""
    B, T = config
    te = B * T
    sizes = sorted({1, 2, 3, 31, 32, 33, B - 1, B, B + 1, te - 1, te, te + 1, 2 * te + 5, 2047, 2048, 2049,
                    32767, 32768, 32769, 3 * 32768 + te - 1})
    for n in sizes:
        x = workloads.sinusoid_field(n, n + 11)
        st_ref, exp = oracle.compress_status(x, oracle.REL, 1e-3, config=config)
        announce(f"config {config} edge size n={n}")
        st, got = gpu_compress_config(x, oracle.REL, 1e-3, config)
        assert st == st_ref, (n, st, st_ref)  # n = 2: a range below the bound's resolution
        if st != fsz.FSZ_OK:
            continue
        assert got == exp, (n, first_diff(got, exp))
        st, y = gpu_decompress_config(exp, n, config)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), oracle.decompress(exp, n).view(np.uint32)), n


@pytest.mark.parametrize("config", CONFIGS)
def test_config_special_fields(config):
    """Zeros, constants, subnormals, values near the largest float, a bound
    too large or too small, NaN and -Inf: the oracle's status and bytes."""
    n = 1024 * 9 + 5
    big = np.full(700, 3.0e38, np.float32)
    big[::2] = 2.9e38
    too_large = np.full(10, 3.3e38, np.float32)
    too_large[0] = -1
    x = workloads.sinusoid_field(5000, 9)
    nan = x.copy()
    nan[4321] = np.nan
    inf = x.copy()
    inf[4321] = -np.inf
    cases = [("zeros-abs", np.zeros(n, np.float32), oracle.ABS, 1e-3),
             ("zeros-rel", np.zeros(n, np.float32), oracle.REL, 1e-3),
             ("constant-neg-rel", np.full(n, -7.5, np.float32), oracle.REL, 1e-2),
             ("subnormal-constant", np.full(n, 1e-40, np.float32), oracle.REL, 1e-3),
             ("subnormal-ramp", (np.arange(n, dtype=np.float32) * np.float32(1e-41)), oracle.ABS, 1e-38),
             ("huge-values", big, oracle.ABS, 1e35), ("eb-too-large", too_large, oracle.ABS, 1e37),
             ("eb-too-small", x, oracle.ABS, 1e-9), ("nan", nan, oracle.REL, 1e-3), ("inf", inf, oracle.ABS, 1e-3)]
    for name, f, mode, value in cases:
        st_ref, exp = oracle.compress_status(f, mode, value, config=config)
        announce(f"config {config} special field {name}")
        st, got = gpu_compress_config(f, mode, value, config)
        assert st == st_ref, (name, st, st_ref)
        if st != fsz.FSZ_OK:
            continue
        assert got == exp, (name, first_diff(got, exp))
        st, y = gpu_decompress_config(exp, f.size, config)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), oracle.decompress(exp, f.size).view(np.uint32)), name


def test_config_fuzz():
    """Random fields (seven kinds), sizes, bound modes, bounds and
    configurations, with unaligned inputs and outputs now and then: statuses,
    streams and decodes against the oracle."""
    rng = np.random.default_rng(4321)
    for case in range(48):
        config = CONFIGS[int(rng.integers(0, len(CONFIGS)))]
        n = int(rng.choice([int(rng.integers(1, 1100)), int(rng.integers(1, 70_000)),
                            int(rng.integers(1, 1 << 20))]))
        name, x = _fuzz_field(rng, n)
        mode = int(rng.integers(0, 2))
        value = float(10.0 ** rng.uniform(-5, -1)) if mode == 1 else float(10.0 ** rng.uniform(-4, 0))
        off = int(rng.integers(0, 2))
        st_ref, exp = oracle.compress_status(x, mode, value, config=config)
        announce(f"config fuzz {case}: {config} {name} n={n} mode={mode} value={value:.3g} offset {off}")
        st, got = gpu_compress_config(x, mode, value, config, in_offset=off)
        assert st == st_ref, (case, st, st_ref)
        if st != fsz.FSZ_OK:
            continue
        assert got == exp, (case, first_diff(got, exp))
        st, y = gpu_decompress_config(exp, n, config, out_offset=off)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), oracle.decompress(exp, n).view(np.uint32)), case


@pytest.mark.parametrize("config", [(32, 4), (64, 8)])
def test_config_decoder_high_rates(config):
    """Rates up to 31 in a configuration's stream (tiles centred on means
    far from their data), next to tiles of low rates."""
    B, T = config
    rng = np.random.default_rng(79)
    for n in (3000, 20_001):
        announce(f"config {config} python-encoded high rates n={n}")
        x = workloads.sinusoid_field(n, int(rng.integers(1000)))
        st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
        lim = (1 << 31) - (1 << 23)
        choices = []
        for t in range(fmt.ceil_div(n, B * T)):
            far = t == 0 or rng.random() < 0.5
            mu = int(rng.integers(-lim, lim)) if far else int(rng.integers(-5000, 5000))
            choices.append((int(rng.integers(2)), 1 if far else int(rng.integers(2)), mu))
        s = fmt.encode_stream(x, E, inv, oracle.REL, 1e-3, 0, choices, B=B, T=T)
        assert max(b & 31 for b in fmt.rate_bytes(s, n, B)) >= 25
        st, y = gpu_decompress_config(s, n, config)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), fmt.closed_form(x, E, inv).view(np.uint32))
        assert np.array_equal(y.view(np.uint32), oracle.decompress(s, n).view(np.uint32))


def test_default_config_is_the_plain_stream():
    x = workloads.grf_field((64, 64, 64), 9)
    for rel in (1e-2, 1e-3):
        announce(f"config (32, 8) through the configuration entry point vs fsz_compress, REL {rel:g}")
        st, got = gpu_compress_config(x, oracle.REL, rel, (32, 8))
        assert st == fsz.FSZ_OK
        st, plain = gpu_compress(x, oracle.REL, rel)
        assert st == fsz.FSZ_OK
        assert got == plain == oracle.compress(x, oracle.REL, rel)


def test_config_empty_and_constant():
    for config in ((32, 4), (64, 16)):
        announce(f"config {config}: empty field, constant field")
        st, got = gpu_compress_config(np.zeros(0, dtype=np.float32), oracle.REL, 1e-3, config)
        assert st == fsz.FSZ_OK and got == oracle.compress(np.zeros(0, dtype=np.float32), oracle.REL, 1e-3,
                                                           config=config)
        st, y = gpu_decompress_config(got, 0, config)
        assert st == fsz.FSZ_OK
        c = np.full(3000, 2.5, dtype=np.float32)
        st, got = gpu_compress_config(c, oracle.REL, 1e-3, config)
        assert st == fsz.FSZ_OK and got == oracle.compress(c, oracle.REL, 1e-3, config=config)
        st, y = gpu_decompress_config(got, c.size, config)
        assert st == fsz.FSZ_OK and np.array_equal(y, c)


def test_config_errors_match_oracle():
    x = workloads.sinusoid_field(20000, 2)
    n = x.size
    announce("config: unsupported configurations")
    st, _ = gpu_compress_config(x, oracle.REL, 1e-3, (32, 32), capacity=1 << 20)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    st, _ = gpu_compress_config(x, oracle.REL, 1e-3, (16, 8), capacity=1 << 20)
    assert st == fsz.FSZ_ERR_INVALID_ARG
    assert fsz.fsz_compressed_bound_config(n, 128, 8) == 0
    for config in ((64, 8), (32, 16)):
        B, T = config
        assert fsz.fsz_compressed_bound_config(n, B, T) == oracle.bound_config(n, B, T)
        s = oracle.compress(x, oracle.REL, 1e-3, config=config)
        announce(f"config {config}: capacity one byte short, bound too small, NaN")
        st, _ = gpu_compress_config(x, oracle.REL, 1e-3, config, capacity=len(s) - 1)
        assert st == fsz.FSZ_ERR_CAPACITY == oracle.compress_status(x, oracle.REL, 1e-3, capacity=len(s) - 1,
                                                                    config=config)[0]
        st, _ = gpu_compress_config(x, oracle.ABS, 1e-12, config)
        assert st == fsz.FSZ_ERR_EB_TOO_SMALL
        xn = x.copy()
        xn[777] = np.nan
        st, _ = gpu_compress_config(xn, oracle.REL, 1e-3, config)
        assert st == fsz.FSZ_ERR_NONFINITE
        announce(f"config {config}: stream given to the default decoder and to another configuration")
        buf = torch.from_numpy(np.frombuffer(s, dtype=np.uint8).copy()).to(_dev())
        out = torch.zeros(n, dtype=torch.float32, device=_dev())
        assert fsz.fsz_decompress(buf.data_ptr(), len(s), out.data_ptr(), n, _stream()) == fsz.FSZ_ERR_CORRUPT
        other = (32, 8) if config != (32, 8) else (64, 4)
        assert gpu_decompress_config(s, n, other)[0] == fsz.FSZ_ERR_CORRUPT
        announce(f"config {config}: corrupt streams")
        nb = fmt.ceil_div(n, B)
        d0 = fmt.data_start(n, B)
        cases = {
            "reserved rate bit (block 0)": (32, 0x20),
            "reserved rate bit (block 1)": (33, 0x80),
            "reserved tile code": (7, 0x18),
            "rate + 1": (34, None),
            "n": (8, None),
        }
        for name, (pos, bits) in cases.items():
            c = bytearray(s)
            if name == "rate + 1":
                c[pos] = (c[pos] & 0xE0) | min(31, (c[pos] & 0x1F) + 1)
            elif name == "n":
                c[8] ^= 1
            else:
                c[pos] |= bits
            want = oracle.decompress_status(bytes(c), n)[0]
            assert want != oracle.OK, name
            assert gpu_decompress_config(bytes(c), n, config)[0] == want, name
        if d0 > 32 + nb:
            c = bytearray(s)
            c[32 + nb] = 1  # nonzero rate-header padding
            assert gpu_decompress_config(bytes(c), n, config)[0] == oracle.ERR_CORRUPT


@pytest.mark.parametrize("n", [(3 << 20) + 5, (1 << 23) + 77])
@pytest.mark.parametrize("config", [(32, 4), (64, 8), (64, 16)])
def test_config_prepass_decoder_and_corrupt_streams(config, n):
    """Fields above 2^21 elements decode in 16-wave lookback chunks, fields of
    2^23 elements and more with chunk offsets from a pre-pass over the rate
    header: bit-exact decoding, and the oracle's status for corrupt streams
    (header fields, reserved rate bits, a rate that no longer matches the
    sizes, padding, a stream cut short)."""
    B, T = config
    old = oracle.set_threads(8)
    try:
        x = workloads.sinusoid_field(n, 21)
        s = oracle.compress(x, oracle.REL, 1e-4, config=config)
        announce(f"config {config} large-field decode n={n}: clean stream")
        st, y = gpu_decompress_config(s, n, config)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), oracle.decompress(s, n).view(np.uint32))
        nb = fmt.ceil_div(n, B)
        d0 = fmt.data_start(n, B)
        cases = {
            "magic": lambda c: c.__setitem__(0, ord("G")),
            "mode": lambda c: c.__setitem__(6, 2),
            "reserved tile code": lambda c: c.__setitem__(7, c[7] | 0x18),
            "n": lambda c: c.__setitem__(8, c[8] ^ 1),
            "E zero": lambda c: c.__setitem__(slice(16, 20), bytes(4)),
            "total": lambda c: c.__setitem__(24, c[24] ^ 4),
            "reserved rate bit (block 0)": lambda c: c.__setitem__(32, c[32] | 0x20),
            "reserved rate bit (block 1)": lambda c: c.__setitem__(33, c[33] | 0x80),
            "rate + 1": lambda c: c.__setitem__(34, (c[34] & 0xE0) | min(31, (c[34] & 0x1F) + 1)),
            "last rate + 1": lambda c: c.__setitem__(32 + nb - 1, (c[32 + nb - 1] & 0xE0) |
                                                     min(31, (c[32 + nb - 1] & 0x1F) + 1)),
        }
        if d0 > 32 + nb:
            cases["padding"] = lambda c: c.__setitem__(32 + nb, 1)
        for name, f in cases.items():
            announce(f"config {config} large-field decode n={n}: {name}")
            c = bytearray(s)
            f(c)
            want = oracle.decompress_status(bytes(c), n)[0]
            assert want != oracle.OK, name
            assert gpu_decompress_config(bytes(c), n, config)[0] == want, name
        announce(f"config {config} large-field decode n={n}: stream cut short")
        assert gpu_decompress_config(s[:-4], n, config)[0] == oracle.decompress_status(s[:-4], n)[0]
    finally:
        oracle.set_threads(old)


@pytest.mark.parametrize("config", [(32, 16), (64, 8)])
def test_config_full_size_grf_512(config):
    """The 512^3 field in the launch configuration the benchmark times: the
    decode equals the closed form fl(q E) over the whole field, the stream
    size equals the sum of the tile sizes its rate header gives, and the
    first tiles' rate bytes and data equal the oracle's stream of the same
    elements."""
    B, T = config
    x = workloads.grf_field((512, 512, 512), 1)
    n = x.size
    rel = 1e-3
    st, E, inv, _ = oracle.resolve(x, oracle.REL, rel)
    assert st == oracle.OK
    xd = torch.from_numpy(x).to(_dev())
    announce(f"config {config} full size 512^3 REL {rel:g}")
    st, s = gpu_compress_config(x, oracle.REL, rel, config, device_x=xd)
    assert st == fsz.FSZ_OK
    hdr = fmt.parse_header(s)
    assert hdr["total"] == len(s) and fmt.header_config(hdr["flags"]) == config
    d0 = fmt.data_start(n, B)
    sizes = np.asarray(fmt.tile_sizes(s, n, B, T), dtype=np.int64)
    assert d0 + int(sizes.sum()) == len(s)
    # the first tiles against the oracle's stream of the same elements: an
    # ABS bound of E/2 + 4 ulp(max|prefix|) resolves to the same step E
    # (the tightening subtracts exactly that ulp term), hence the same
    # quantization and tile means
    m = 1024 * B * T
    u = float(np.spacing(np.float32(np.abs(x[:m]).max())))
    pre = oracle.compress(x[:m], oracle.ABS, float(hdr["E"]) / 2 + 4 * u, config=config)
    assert fmt.parse_header(pre)["E"] == hdr["E"]
    assert s[32:32 + m // B] == pre[32:32 + m // B]
    body = int(sizes[:1024].sum())
    assert s[d0:d0 + body] == pre[fmt.data_start(m, B):fmt.data_start(m, B) + body]
    announce(f"config {config} full size 512^3 decode")
    buf = torch.from_numpy(np.frombuffer(s, dtype=np.uint8).copy()).to(_dev())
    del xd
    out = torch.empty(n, dtype=torch.float32, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    assert fsz.fsz_decompress_config_async(buf.data_ptr(), len(s), out.data_ptr(), n, B, T, res.data_ptr(),
                                           _stream()) == fsz.FSZ_OK
    torch.cuda.synchronize()
    assert int(res.cpu()[1]) & 0xFFFFFFFF == fsz.FSZ_OK
    y = out.cpu().numpy()
    assert np.array_equal(y.view(np.uint32), fmt.closed_form(x, E, inv).view(np.uint32))


def test_config_stream_beyond_4gib():
    """64-bit sizes and offsets in the configuration kernels: 2^31 + 4099
    uniform values at REL 1e-6 in 64 x 16 tiles give a stream of about 5.7
    GB.  The rate header sums to the stream's size; the first and the last
    1024 tiles (the last ones stored beyond 2^32 bytes) equal the oracle's
    streams of the same elements; the decode equals the closed form
    fl(rint(fl(x * inv)) * E) over the whole field."""
    B, T = 64, 16
    n = (1 << 31) + 4099
    rng = np.random.default_rng(19)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    rel = 1e-6
    announce(f"config {(B, T)} stream beyond 4 GiB: uniform n={n} REL {rel:g}")
    xd = torch.from_numpy(x).to(_dev())
    st, s = gpu_compress_config(x, oracle.REL, rel, (B, T), device_x=xd)
    assert st == fsz.FSZ_OK and len(s) > (1 << 32)
    hdr = fmt.parse_header(s)
    assert hdr["total"] == len(s) and fmt.header_config(hdr["flags"]) == (B, T)
    E = float(hdr["E"])
    sizes = fmt.tile_sizes_np(s, n, B, T)
    d0 = fmt.data_start(n, B)
    assert d0 + int(sizes.sum()) == len(s)
    te = B * T
    nt = sizes.size
    for first in (0, nt - 1024):
        lo, hi = first * te, min(n, (first + 1024) * te)
        xs = x[lo:hi]
        # an ABS bound of E/2 + 4 ulp(max|xs|) resolves to the same step E
        u = float(np.spacing(np.float32(np.abs(xs).max())))
        ref = oracle.compress(xs, oracle.ABS, E / 2 + 4 * u, config=(B, T))
        assert fmt.parse_header(ref)["E"] == hdr["E"]
        nb = fmt.ceil_div(hi - lo, B)
        assert s[32 + lo // B:32 + lo // B + nb] == ref[32:32 + nb], f"rate bytes of tiles from {first}"
        at = d0 + int(sizes[:first].sum())
        body = int(sizes[first:first + 1024].sum())
        if first:
            assert at > (1 << 32)
        ds = fmt.data_start(hi - lo, B)
        assert len(ref) == ds + body
        assert s[at:at + body] == ref[ds:], f"data of tiles from {first}"
    announce(f"config {(B, T)} stream beyond 4 GiB: decode of {len(s)} bytes")
    buf = torch.from_numpy(np.frombuffer(s, dtype=np.uint8).copy()).to(_dev())
    del s
    y = torch.empty(n, dtype=torch.float32, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    assert fsz.fsz_decompress_config_async(buf.data_ptr(), buf.numel(), y.data_ptr(), n, B, T, res.data_ptr(),
                                           _stream()) == fsz.FSZ_OK
    torch.cuda.synchronize()
    assert int(res.cpu()[1]) & 0xFFFFFFFF == fsz.FSZ_OK
    del buf
    inv = np.float32(1) / np.float32(E)
    q = torch.round(xd * float(inv)).to(torch.int32)  # zero as +0 whatever the product's sign
    del xd
    expect = q.to(torch.float32) * E
    del q
    step = 1 << 28
    for k in range(0, n, step):
        a = y[k:k + step].view(torch.int32)
        b = expect[k:k + step].view(torch.int32)
        bad = (a != b).nonzero()
        if bad.numel():
            i = k + int(bad[0])
            raise AssertionError(f"{bad.numel()} of the elements [{k}, {k + a.numel()}) differ; first at {i}: "
                                 f"decoded {float(y[i])} expected {float(expect[i])} (x = {float(x[i])})")
