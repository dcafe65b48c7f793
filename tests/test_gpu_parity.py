"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Compressed streams must be byte-identical and reconstructions bit-identical
(integer work after one binary32 quantization step, no FMA contraction).
Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests import fsz_format as fmt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    return torch.device("cuda:0")


def _stream():
    return torch.cuda.current_stream(_dev()).cuda_stream


def announce(name):
    print(f"\n[case] {name}", flush=True)


def gpu_compress(x, mode, value, capacity=None, in_offset=0, out_offset=0):
    """Compress numpy float32 x on the GPU; returns (status, bytes or None).
    in_offset / out_offset shift the input / output pointers by that many
    4-byte words from a 256-byte aligned allocation."""
    n = x.size
    xd = torch.zeros(n + in_offset + 4, dtype=torch.float32, device=_dev())
    if n:
        xd[in_offset:in_offset + n] = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n) if capacity is None else capacity
    out = torch.zeros(max(cap, 1) + 4 * out_offset, dtype=torch.uint8, device=_dev())
    st, size = fsz.fsz_compress(xd.data_ptr() + 4 * in_offset, n, mode, value, out.data_ptr() + 4 * out_offset,
                                cap, _stream())
    if st != fsz.FSZ_OK:
        return st, None
    return st, out[4 * out_offset:4 * out_offset + size].cpu().numpy().tobytes()


def gpu_decompress(stream_bytes, n, out_offset=0):
    buf = torch.from_numpy(np.frombuffer(stream_bytes, dtype=np.uint8).copy()).to(_dev())
    out = torch.full((n + out_offset + 4,), float("nan"), dtype=torch.float32, device=_dev())
    st = fsz.fsz_decompress(buf.data_ptr(), len(stream_bytes), out.data_ptr() + 4 * out_offset, n,
                            _stream())
    if st != fsz.FSZ_OK:
        return st, None
    return st, out[out_offset:out_offset + n].cpu().numpy()


def first_diff(a: bytes, b: bytes):
    if len(a) != len(b):
        return f"lengths {len(a)} vs {len(b)}"
    for i in range(len(a)):
        if a[i] != b[i]:
            return f"byte {i}: {a[i]:#04x} vs {b[i]:#04x}"
    return "equal"


def check_round_trip(name, x, mode, value, in_offset=0, out_offset=0):
    announce(f"{name} n={x.size} mode={mode} value={value} in_off={in_offset} out_off={out_offset}")
    st_ref, ref = oracle.compress_status(x, mode, value)
    st, got = gpu_compress(x, mode, value, in_offset=in_offset)
    assert st == st_ref, (name, st, st_ref)
    if st != fsz.FSZ_OK:
        return None
    assert got == ref, f"{name}: stream differs from the oracle ({first_diff(got, ref)})"
    st, y = gpu_decompress(got, x.size, out_offset=out_offset)
    assert st == fsz.FSZ_OK
    y_ref = oracle.decompress(ref, x.size)
    assert np.array_equal(y.view(np.uint32), y_ref.view(np.uint32)), f"{name}: reconstruction differs"
    return ref


# ----------------------------------------------------------------- configs


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_sinusoid_2pow20(rel):
    x = workloads.sinusoid_field(1 << 20, 0)
    check_round_trip("sinusoid-2^20", x, fsz.FSZ_REL, rel)


def test_piecewise_quadratic_full():
    x = workloads.piecewise_quadratic((100, 500, 500), 2)
    for rel in (1e-2, 1e-3, 1e-4):
        check_round_trip("pwq-100x500x500", x, fsz.FSZ_REL, rel)


def test_grf_small():
    x = workloads.grf_field((64, 64, 64), 1)
    for rel in (1e-2, 1e-3, 1e-4):
        check_round_trip("grf-64^3", x, fsz.FSZ_REL, rel)


def test_grf_512_full_size_bench_launch():
    """The benchmark's field (512^3 k^-3 GRF, seed 1) at full size, in the
    benchmark's launch configuration (one range pass, then the asynchronous
    compress per bound on the persistent pipelined kernel, decompress on the
    persistent decoder): every byte and every reconstructed value against the
    oracle."""
    x = workloads.grf_field((512, 512, 512), 1)
    n = x.size
    announce("grf-512^3 full size, bench launch configuration")
    xd = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    out = torch.zeros(cap, dtype=torch.uint8, device=_dev())
    y = torch.zeros(n, dtype=torch.float32, device=_dev())
    stats = torch.zeros(4, dtype=torch.int32, device=_dev())
    r1 = torch.zeros(4, dtype=torch.int32, device=_dev())
    r2 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_field_stats(xd.data_ptr(), n, stats.data_ptr(), _stream()) == fsz.FSZ_OK
    for rel in (1e-2, 1e-3, 1e-4):
        announce(f"grf-512^3 REL {rel:g}")
        assert fsz.fsz_compress_async(xd.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(), out.data_ptr(),
                                      cap, r1.data_ptr(), _stream()) == fsz.FSZ_OK
        assert fsz.fsz_decompress_async(out.data_ptr(), cap, y.data_ptr(), n, r2.data_ptr(),
                                        _stream()) == fsz.FSZ_OK
        size, st, _ = fsz.read_result(r1)
        assert st == fsz.FSZ_OK
        assert fsz.read_result(r2)[1] == fsz.FSZ_OK
        ref = oracle.compress(x, oracle.REL, rel)
        got = out[:size].cpu().numpy().tobytes()
        assert got == ref, f"REL {rel}: {first_diff(got, ref)}"
        y_ref = oracle.decompress(ref, n)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), y_ref.view(np.uint32))


@pytest.mark.timeout(600)
def test_stream_beyond_4gib():
    """64-bit sizes and offsets: 2^31 + 4099 uniform values at REL 1e-6 give
    an input of 8 GiB and a stream of about 5.7 GB, so tile offsets, the
    lookback sums and the header's total pass 2^32 bytes.  Every byte
    against the oracle; the decode against the closed form fl(rint(fl(x *
    inv)) * E) computed with plain torch operations on the device."""
    n = (1 << 31) + 4099
    rng = np.random.default_rng(17)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    rel = 1e-6
    announce(f"stream beyond 4 GiB: uniform n={n} REL {rel:g}")
    xd = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    out = torch.zeros(cap, dtype=torch.uint8, device=_dev())
    r1 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_compress_async(xd.data_ptr(), n, fsz.FSZ_REL, rel, None, out.data_ptr(), cap, r1.data_ptr(),
                                  _stream()) == fsz.FSZ_OK
    size, st, _ = fsz.read_result(r1)
    assert st == fsz.FSZ_OK and size > (1 << 32)
    ref = oracle.compress(x, oracle.REL, rel)
    assert size == len(ref)
    got = out[:size].cpu().numpy()
    assert np.array_equal(got, np.frombuffer(ref, dtype=np.uint8))
    E = np.float32(fmt.parse_header(ref)["E"])
    del ref, got
    announce(f"stream beyond 4 GiB: decode of {size} bytes")
    y = torch.empty(n, dtype=torch.float32, device=_dev())
    r2 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_decompress_async(out.data_ptr(), size, y.data_ptr(), n, r2.data_ptr(), _stream()) == fsz.FSZ_OK
    assert fsz.read_result(r2)[1] == fsz.FSZ_OK
    del out
    inv = np.float32(1) / E
    # binary32 product, round half to even, then the integer q (|q| < 2^22:
    # exact), whose zero is +0 whatever the sign of the product
    q = torch.round(xd * float(inv)).to(torch.int32)
    del xd
    expect = q.to(torch.float32) * float(E)
    del q
    step = 1 << 28  # compared slice by slice, so a mismatch names its position
    for k in range(0, n, step):
        a = y[k:k + step].view(torch.int32)
        b = expect[k:k + step].view(torch.int32)
        bad = (a != b).nonzero()
        if bad.numel():
            i = k + int(bad[0])
            raise AssertionError(f"{bad.numel()} of the elements [{k}, {k + a.numel()}) differ; first at {i}: "
                                 f"decoded {float(y[i])} expected {float(expect[i])} (x = {float(x[i])})")


def test_stream_beyond_4gib_unaligned():
    """The kernels for pointers that are not 16-byte aligned at 64-bit sizes:
    2^31 + 4099 uniform values at REL 1e-6 read from an input one float past
    a 16-byte boundary give the same 5.7 GB stream as the aligned
    (pipelined) kernel, their first and last 4096 tiles (the last ones
    stored beyond 2^32 bytes) equal the oracle's streams of the same
    elements, and the decode into an output one float past a 16-byte
    boundary equals the closed form fl(rint(fl(x * inv)) * E)."""
    n = (1 << 31) + 4099
    rng = np.random.default_rng(37)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    rel = 1e-6
    cap = fsz.fsz_compressed_bound(n)
    xa = torch.from_numpy(x).to(_dev())
    xu = torch.empty(n + 4, dtype=torch.float32, device=_dev())
    xu[1:n + 1] = xa
    streams = []
    for name, xp in (("aligned", xa.data_ptr()), ("unaligned", xu.data_ptr() + 4)):
        announce(f"stream beyond 4 GiB, {name} input: uniform n={n} REL {rel:g}")
        out = torch.zeros(cap, dtype=torch.uint8, device=_dev())
        r = torch.zeros(4, dtype=torch.int32, device=_dev())
        assert fsz.fsz_compress_async(xp, n, fsz.FSZ_REL, rel, None, out.data_ptr(), cap, r.data_ptr(),
                                      _stream()) == fsz.FSZ_OK
        size, st, _ = fsz.read_result(r)
        assert st == fsz.FSZ_OK and size > (1 << 32)
        streams.append((out, size))
    del xu
    (oa, sa), (ou, size) = streams
    assert sa == size and torch.equal(oa[:size], ou[:size])
    del oa, streams
    d0 = fmt.data_start(n)
    head = ou[:d0].cpu().numpy().tobytes()
    hdr = fmt.parse_header(head)
    E = float(hdr["E"])
    sizes = fmt.tile_sizes_np(head, n)
    assert hdr["total"] == size == d0 + int(sizes.sum())
    m = 4096
    for first in (0, sizes.size - m):
        lo, hi = first * fmt.TILE, min(n, (first + m) * fmt.TILE)
        xs = x[lo:hi]
        # an ABS bound of E/2 + 4 ulp(max|xs|) resolves to the same step E
        u = float(np.spacing(np.float32(np.abs(xs).max())))
        ref = oracle.compress(xs, oracle.ABS, E / 2 + 4 * u)
        assert fmt.parse_header(ref)["E"] == hdr["E"]
        nb = fmt.ceil_div(hi - lo, fmt.BLOCK)
        r0 = fmt.HEADER + lo // fmt.BLOCK
        assert head[r0:r0 + nb] == ref[fmt.HEADER:fmt.HEADER + nb], f"rate bytes of tiles from {first}"
        at = d0 + int(sizes[:first].sum())
        body = int(sizes[first:first + m].sum())
        if first:
            assert at > (1 << 32)
        ds = fmt.data_start(hi - lo)
        assert len(ref) == ds + body
        got = ou[at:at + body].cpu().numpy().tobytes()
        assert got == ref[ds:], f"data of tiles from {first}: " + first_diff(got, ref[ds:])
    announce(f"stream beyond 4 GiB: decode of {size} bytes into an unaligned output")
    yb = torch.full((n + 8,), float("nan"), dtype=torch.float32, device=_dev())
    r2 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_decompress_async(ou.data_ptr(), size, yb.data_ptr() + 4, n, r2.data_ptr(),
                                    _stream()) == fsz.FSZ_OK
    assert fsz.read_result(r2)[1] == fsz.FSZ_OK
    del ou
    assert bool(torch.isnan(yb[0])) and bool(torch.isnan(yb[n + 1:]).all())
    y = yb[1:n + 1]
    inv = float(np.float32(1) / np.float32(E))
    q = torch.round(xa * inv).to(torch.int32)  # zero as +0 whatever the product's sign
    del xa
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


# ----------------------------------------------------------------- ragged / edge sizes


@pytest.mark.parametrize("n", [0, 1, 2, 3, 31, 32, 33, 255, 256, 257, 2047, 2048, 2049, 8191, 8192,
                               8193, 65537])
def test_edge_sizes(n):
    x = workloads.sinusoid_field(n, n + 7)
    check_round_trip("edge", x, fsz.FSZ_REL, 1e-3)
    check_round_trip("edge-abs", x, fsz.FSZ_ABS, 1e-4)


def test_compress_output_offsets():
    """Aligned input (the pipelined kernel) into outputs at every 4-byte
    phase of a 16-byte line: the staging area follows the destination's
    phase, so each phase must give the oracle's bytes."""
    x = workloads.grf_field((64, 64, 80), 11)
    for rel in (1e-2, 1e-4):
        ref = oracle.compress(x, oracle.REL, rel)
        for off in (1, 2, 3):
            announce(f"compress output offset {off} words, REL {rel:g}")
            st, got = gpu_compress(x, fsz.FSZ_REL, rel, out_offset=off)
            assert st == fsz.FSZ_OK
            assert got == ref, first_diff(got, ref)


def test_unaligned_pointers():
    x = workloads.sinusoid_field(100_001, 3)
    for off_in, off_out in ((1, 0), (2, 3), (3, 1)):
        check_round_trip("unaligned", x, fsz.FSZ_REL, 1e-3, in_offset=off_in, out_offset=off_out)


def _fuzz_field(rng, n):
    kind = int(rng.integers(0, 7))
    if kind == 0:
        return "sinusoid", workloads.sinusoid_field(n, int(rng.integers(1 << 30)))
    if kind == 1:
        return "uniform", rng.uniform(-1, 1, n).astype(np.float32)
    if kind == 2:
        return "offset-noise", (1000.0 + rng.normal(0, 0.01, n)).astype(np.float32)
    if kind == 3:
        q = np.cumsum(rng.integers(-3, 4, n))
        return "random-walk", (q * 0.125).astype(np.float32)
    if kind == 4:
        x = np.zeros(n, np.float32)
        x[rng.integers(0, n, max(1, n // 100))] = rng.uniform(-50, 50, max(1, n // 100))
        return "sparse-spikes", x
    if kind == 5:
        i = np.arange(n, dtype=np.float64)
        return "quadratic", (3.0 + 0.01 * i - 1e-6 * i * i).astype(np.float32)
    v = np.repeat(rng.uniform(-5, 5, n // 97 + 1), 97)[:n]
    return "piecewise-const", v.astype(np.float32)


def test_fuzz():
    rng = np.random.default_rng(1234)
    for case in range(40):
        n = int(rng.choice([int(rng.integers(1, 600)), int(rng.integers(1, 40_000)),
                            int(rng.integers(1, 1 << 20))]))
        name, x = _fuzz_field(rng, n)
        mode = int(rng.integers(0, 2))
        value = float(10.0 ** rng.uniform(-5, -1)) if mode == 1 else float(10.0 ** rng.uniform(-4, 0))
        check_round_trip(f"fuzz{case}-{name}", x, mode, value)


# ----------------------------------------------------------------- special fields and statuses


def test_special_fields():
    n = 256 * 33 + 5
    check_round_trip("zeros-abs", np.zeros(n, np.float32), fsz.FSZ_ABS, 1e-3)
    check_round_trip("zeros-rel", np.zeros(n, np.float32), fsz.FSZ_REL, 1e-3)
    check_round_trip("constant-rel", np.full(n, 1013.25, np.float32), fsz.FSZ_REL, 1e-3)
    check_round_trip("constant-neg-rel", np.full(n, -7.5, np.float32), fsz.FSZ_REL, 1e-2)
    check_round_trip("subnormal-constant", np.full(n, 1e-40, np.float32), fsz.FSZ_REL, 1e-3)
    big = np.full(300, 3.0e38, np.float32)
    big[::2] = 2.9e38
    check_round_trip("huge-values", big, fsz.FSZ_ABS, 1e35)
    too_large = np.full(10, 3.3e38, np.float32)
    too_large[0] = -1
    check_round_trip("eb-too-large", too_large, fsz.FSZ_ABS, 1e37)
    x = workloads.sinusoid_field(5000, 9)
    check_round_trip("eb-too-small", x, fsz.FSZ_ABS, 1e-9)
    bad = x.copy()
    bad[4321] = np.nan
    check_round_trip("nan", bad, fsz.FSZ_REL, 1e-3)
    bad[4321] = -np.inf
    check_round_trip("inf", bad, fsz.FSZ_ABS, 1e-3)


def test_capacity_too_small():
    x = workloads.sinusoid_field(50_000, 5)
    ref = oracle.compress(x, oracle.REL, 1e-3)
    announce("capacity")
    for cap in (fmt.data_start(x.size), len(ref) - 4):
        st, _ = gpu_compress(x, fsz.FSZ_REL, 1e-3, capacity=cap)
        assert st == fsz.FSZ_ERR_CAPACITY
    st, got = gpu_compress(x, fsz.FSZ_REL, 1e-3, capacity=len(ref))
    assert st == fsz.FSZ_OK and got == ref


def test_compress_ex_reuses_stats():
    x = workloads.grf_field((32, 64, 64), 4)
    announce("compress_ex")
    xd = torch.from_numpy(x).to(_dev())
    stats = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_field_stats(xd.data_ptr(), x.size, stats.data_ptr(), _stream()) == fsz.FSZ_OK
    st_cpu = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=np.float32)
    assert st_cpu[0] == x.min() and st_cpu[1] == x.max() and st_cpu[2] == np.abs(x).max()
    for rel in (1e-2, 1e-3, 1e-4):
        out = torch.zeros(fsz.fsz_compressed_bound(x.size), dtype=torch.uint8, device=_dev())
        st, size = fsz.fsz_compress_ex(xd.data_ptr(), x.size, fsz.FSZ_REL, rel, stats.data_ptr(),
                                       out.data_ptr(), out.numel(), _stream())
        assert st == fsz.FSZ_OK
        assert out[:size].cpu().numpy().tobytes() == oracle.compress(x, oracle.REL, rel)


# ----------------------------------------------------------------- decoder


def test_decoder_any_variant_and_mean():
    rng = np.random.default_rng(77)
    for n in (5, 256, 700, 5000, 20_001):
        announce(f"python-encoded n={n}")
        x = workloads.sinusoid_field(n, int(rng.integers(1000)))
        st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
        choices = [(int(rng.integers(2)), int(rng.integers(2)), int(rng.integers(-5000, 5000)))
                   for _ in range(fmt.ceil_div(n, 256))]
        s = fmt.encode_stream(x, E, inv, oracle.REL, 1e-3, 0, choices)
        st, y = gpu_decompress(s, n)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y, fmt.closed_form(x, E, inv))


def test_decoder_high_rates():
    """Rates up to 31 (the format's maximum; the compressor itself stays at
    or below 24): tiles centred on means far from their data give tile-start
    residuals near 2^31, so waves assemble all four byte groups of the
    magnitude planes next to waves of low rates."""
    rng = np.random.default_rng(78)
    for n in (256, 3000, 20_001):
        announce(f"python-encoded high rates n={n}")
        x = workloads.sinusoid_field(n, int(rng.integers(1000)))
        st, E, inv, _ = oracle.resolve(x, oracle.REL, 1e-3)
        lim = (1 << 31) - (1 << 23)
        choices = []
        for t in range(fmt.ceil_div(n, 256)):
            far = t == 0 or rng.random() < 0.5
            mu = int(rng.integers(-lim, lim)) if far else int(rng.integers(-5000, 5000))
            choices.append((int(rng.integers(2)), 1 if far else int(rng.integers(2)), mu))
        s = fmt.encode_stream(x, E, inv, oracle.REL, 1e-3, 0, choices)
        assert max(b & 31 for b in fmt.rate_bytes(s, n)) >= 25
        st, y = gpu_decompress(s, n)
        assert st == fsz.FSZ_OK
        assert np.array_equal(y.view(np.uint32), fmt.closed_form(x, E, inv).view(np.uint32))
        assert np.array_equal(y.view(np.uint32), oracle.decompress(s, n).view(np.uint32))


def test_corrupt_streams_match_oracle_status():
    from tests.test_oracle import _mutations
    n = 3000
    x = workloads.sinusoid_field(n, 2)
    s = oracle.compress(x, oracle.REL, 1e-4)
    for name, c, want in _mutations(s, n):
        announce(f"corrupt-{name}")
        st, _ = gpu_decompress(c, n)
        assert st == want == oracle.decompress_status(c, n)[0], name
    announce("corrupt-truncated")
    st, _ = gpu_decompress(s[:-4], n)
    assert st == fsz.FSZ_ERR_CORRUPT


def test_repeated_calls_are_deterministic():
    x = workloads.sinusoid_field(3_000_001, 11)
    ref = oracle.compress(x, oracle.REL, 1e-4)
    announce("determinism")
    xd = torch.from_numpy(x).to(_dev())
    out = torch.zeros(fsz.fsz_compressed_bound(x.size), dtype=torch.uint8, device=_dev())
    y = torch.zeros(x.size, dtype=torch.float32, device=_dev())
    y_ref = oracle.decompress(ref, x.size)
    for _ in range(20):
        st, size = fsz.fsz_compress(xd.data_ptr(), x.size, fsz.FSZ_REL, 1e-4, out.data_ptr(),
                                    out.numel(), _stream())
        assert st == fsz.FSZ_OK and out[:size].cpu().numpy().tobytes() == ref
        assert fsz.fsz_decompress(out.data_ptr(), size, y.data_ptr(), x.size, _stream()) == fsz.FSZ_OK
        assert np.array_equal(y.cpu().numpy(), y_ref)


def test_async_calls_chain_on_stream():
    """Async forms: no host read between calls; outcomes land in device fsz_result structs."""
    x = workloads.sinusoid_field(500_001, 8)
    announce("async chain")
    xd = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(x.size)
    out = torch.zeros(cap, dtype=torch.uint8, device=_dev())
    y = torch.zeros(x.size, dtype=torch.float32, device=_dev())
    stats = torch.zeros(4, dtype=torch.int32, device=_dev())
    r1 = torch.zeros(4, dtype=torch.int32, device=_dev())
    r2 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_field_stats(xd.data_ptr(), x.size, stats.data_ptr(), _stream()) == fsz.FSZ_OK
    assert fsz.fsz_compress_async(xd.data_ptr(), x.size, fsz.FSZ_REL, 1e-3, stats.data_ptr(),
                                  out.data_ptr(), cap, r1.data_ptr(), _stream()) == fsz.FSZ_OK
    # decompress straight from the capacity-sized buffer: the header carries the length
    assert fsz.fsz_decompress_async(out.data_ptr(), cap, y.data_ptr(), x.size, r2.data_ptr(),
                                    _stream()) == fsz.FSZ_OK
    ref = oracle.compress(x, oracle.REL, 1e-3)
    size, st, _ = fsz.read_result(r1)
    assert st == fsz.FSZ_OK and size == len(ref)
    assert out[:size].cpu().numpy().tobytes() == ref
    size2, st2, _ = fsz.read_result(r2)
    assert st2 == fsz.FSZ_OK and size2 == len(ref)
    assert np.array_equal(y.cpu().numpy(), oracle.decompress(ref, x.size))
    # the range pass runs inside the call when no stats are given; errors arrive on device
    bad = xd.clone()
    bad[1234] = float("nan")
    assert fsz.fsz_compress_async(bad.data_ptr(), x.size, fsz.FSZ_REL, 1e-3, None, out.data_ptr(),
                                  cap, r1.data_ptr(), _stream()) == fsz.FSZ_OK
    assert fsz.read_result(r1)[1] == fsz.FSZ_ERR_NONFINITE


def _check_bound_case(name, x, mode, value):
    """Status and header step E through fsz_compress equal the exact rational
    reading; accepted streams equal the oracle's byte for byte."""
    from tests.test_oracle_resolve import expected

    announce(f"{name} n={x.size} mode={mode} value={value!r}")
    est, eE, _, _ = expected(x, mode, value)
    st, got = gpu_compress(x, mode, value)
    assert st == est, (name, st, est)
    if st == fsz.FSZ_OK:
        assert np.float32(fmt.parse_header(got)["E"]) == eE, name
        assert got == oracle.compress(x, mode, value), name
    return st


def test_bound_threshold_at_eight_ulp():
    """eb = 8 ulp(max|x|) is accepted and the next binary64 below it rejected,
    through the device's bound resolution, for ABS and REL."""
    from fractions import Fraction

    from tests.test_oracle_resolve import ulp_above

    for M in (1.0, 0.75, 1000.0, 6.0e37, 2.0 ** -100):
        x = np.array([M, -M / 2, 0.0] * 100, dtype=np.float32)
        at = float(8 * ulp_above(np.float32(M)))
        assert _check_bound_case("abs at 8u", x, fsz.FSZ_ABS, at) == fsz.FSZ_OK
        below = float(np.nextafter(at, 0.0))
        assert _check_bound_case("abs below 8u", x, fsz.FSZ_ABS, below) == fsz.FSZ_ERR_EB_TOO_SMALL
    for M in (1.0, 0.5, 128.0, 2.0 ** -40):
        x = np.array([M, -M, M / 4] * 100, dtype=np.float32)
        value = float(4 * ulp_above(np.float32(M)) / Fraction(M))
        assert _check_bound_case("rel at 8u", x, fsz.FSZ_REL, value) == fsz.FSZ_OK
        below = float(np.nextafter(value, 0.0))
        assert _check_bound_case("rel below 8u", x, fsz.FSZ_REL, below) == fsz.FSZ_ERR_EB_TOO_SMALL


def test_bound_step_exact_cases():
    """Random (field, mode, value) pairs and the cases where a rounded binary64
    difference eb - 4u would give another step: device E = exact rational E."""
    from tests.test_oracle_resolve import _random_cases

    seen = set()
    for k, (x, mode, value) in enumerate(_random_cases(1, 300)):
        seen.add(_check_bound_case(f"random {k}", np.tile(x, 9), mode, value))
    assert fsz.FSZ_OK in seen and fsz.FSZ_ERR_EB_TOO_SMALL in seen
    for value in (0.5, 3.0, 1024.0):
        x = np.array([1e-12, -3e-13, 0.0] * 90, dtype=np.float32)
        assert _check_bound_case("huge eb over tiny data", x, fsz.FSZ_ABS, value) == fsz.FSZ_OK
    x = np.array([1e-40, -3e-41] * 200, dtype=np.float32)
    assert _check_bound_case("subnormal step", x, fsz.FSZ_ABS, 1e-39) == fsz.FSZ_ERR_EB_TOO_SMALL
    y = np.array([1.0, 2.0] * 200, dtype=np.float32)
    assert _check_bound_case("clamped step", y, fsz.FSZ_ABS, 1e38) == fsz.FSZ_OK
    big = np.array([3.3e38, -1.0] * 200, dtype=np.float32)
    assert _check_bound_case("step too large", big, fsz.FSZ_ABS, 1e37) == fsz.FSZ_ERR_EB_TOO_LARGE


@pytest.mark.timeout(600)
def test_decoder_regimes_and_corrupt_streams():
    """Whole-field decodes use the lookback decoder for small fields (8-wave
    chunks up to 2^21 elements, 16-wave ones above) and the offsets pre-pass
    (one chunk per workgroup, or the persistent grid) for larger ones: each
    regime decodes bit-exactly and reports corrupt streams (reserved bits,
    sizes that disagree with the total, padding, header fields, a mismatched
    n) with the oracle's status."""
    from tests.test_oracle import _mutations

    old = oracle.set_threads(8)
    try:
        for n in (1000, (3 << 20) + 5, (1 << 23) + 77, (1 << 26) + 5):
            x = workloads.sinusoid_field(n, 17)
            s = oracle.compress(x, oracle.REL, 1e-4)
            announce(f"decoder regime n={n}: clean stream")
            st, y = gpu_decompress(s, n)
            assert st == fsz.FSZ_OK
            assert np.array_equal(y.view(np.uint32), oracle.decompress(s, n).view(np.uint32))
            for name, c, want in _mutations(s, n):
                announce(f"decoder regime n={n}: {name}")
                st, _ = gpu_decompress(c, n)
                assert st == want == oracle.decompress_status(c, n)[0], (n, name, st, want)
            announce(f"decoder regime n={n}: stream cut short")
            st, _ = gpu_decompress(s[:-4], n)
            assert st == fsz.FSZ_ERR_CORRUPT
    finally:
        oracle.set_threads(old)
