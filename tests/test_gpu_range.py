"""GPU random-access decode: elements [begin, end) of a stream decoded alone
equal the same elements of the oracle's whole-field decode bit for bit
(ranges at the start, the end, across tile and chunk boundaries, empty,
unaligned outputs, streams with independent blocks), and corrupt rate bytes
before or inside the range are reported.  Every case prints its name before
touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests import fsz_format as fmt
from tests.test_gpu_parity import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    return torch.device("cuda:0")


def gpu_decompress_range(stream_bytes, n, begin, end, out_offset=0):
    buf = torch.from_numpy(np.frombuffer(stream_bytes, dtype=np.uint8).copy()).to(_dev())
    m = end - begin
    guard = 8
    out = torch.full((m + out_offset + 2 * guard,), float("nan"), dtype=torch.float32, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    st = fsz.fsz_decompress_range_async(buf.data_ptr(), len(stream_bytes), n, begin, end,
                                        out.data_ptr() + 4 * (guard + out_offset), res.data_ptr(), stream)
    if st != fsz.FSZ_OK:
        return st, None
    torch.cuda.synchronize()
    st = int(res.cpu()[1]) & 0xFFFFFFFF
    o = out.cpu().numpy()
    # nothing outside the requested range was written
    assert np.all(np.isnan(o[:guard + out_offset])) and np.all(np.isnan(o[guard + out_offset + m:]))
    return st, o[guard + out_offset:guard + out_offset + m]


def _ranges(n):
    chunk = 64 * 256
    cand = [(0, n), (0, 1), (n - 1, n), (255, 257), (256, 512), (1000, 70000), (n // 2, n),
            (chunk - 3, 3 * chunk + 5), (5, 5), (n, n), (n // 3, n // 3 + 100001)]
    return [(b, e) for b, e in cand if 0 <= b <= e <= n]


@pytest.mark.parametrize("features", [fsz.FSZ_FEATURES_ALL, 0])
def test_range_decode_matches_whole_field(features):
    for name, x in (("grf 64x64x80", workloads.grf_field((64, 64, 80), 3)),
                    ("pwq 5x301x181 (ragged)", workloads.piecewise_quadratic((5, 301, 181), 4))):
        n = x.size
        s = oracle.compress(x, oracle.REL, 1e-3, features=features)
        full = oracle.decompress(s, n)
        for begin, end in _ranges(n):
            for off in (0, 1):
                announce(f"range {name} features {features} [{begin}, {end}) output offset {off}")
                st, y = gpu_decompress_range(s, n, begin, end, out_offset=off)
                assert st == fsz.FSZ_OK
                assert np.array_equal(y.view(np.uint32), full[begin:end].view(np.uint32)), (begin, end)


def test_long_range_decode_matches_whole_field():
    """Ranges of more than 2^21 elements decode in 16-wave chunks: bit-exact
    against the oracle's whole-field decode, ragged ends and an odd output
    offset included."""
    n = (1 << 22) + 333
    x = workloads.sinusoid_field(n, 8)
    s = oracle.compress(x, oracle.REL, 1e-4)
    full = oracle.decompress(s, n)
    for begin, end in ((0, n), (1000, (3 << 20) + 17), (n - (5 << 19) - 9, n)):
        for off in (0, 1):
            announce(f"long range n={n} [{begin}, {end}) output offset {off}")
            st, y = gpu_decompress_range(s, n, begin, end, out_offset=off)
            assert st == fsz.FSZ_OK
            assert np.array_equal(y.view(np.uint32), full[begin:end].view(np.uint32)), (begin, end)


def test_range_decode_errors():
    x = workloads.sinusoid_field(100000, 5)
    n = x.size
    s = oracle.compress(x, oracle.REL, 1e-3)
    announce("range: begin > end, end > n")
    buf = torch.from_numpy(np.frombuffer(s, dtype=np.uint8).copy()).to(_dev())
    out = torch.zeros(16, dtype=torch.float32, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    assert fsz.fsz_decompress_range_async(buf.data_ptr(), len(s), n, 10, 5, out.data_ptr(), res.data_ptr(),
                                          stream) == fsz.FSZ_ERR_INVALID_ARG
    assert fsz.fsz_decompress_range_async(buf.data_ptr(), len(s), n, 0, n + 1, out.data_ptr(), res.data_ptr(),
                                          stream) == fsz.FSZ_ERR_INVALID_ARG
    # a reserved bit (bit 5 of a tile's first rate byte) in a block before the
    # range (tile 3; the range starts at tile 4), then in one inside it (tile 8)
    for blk, begin, end, name in ((24, 1024, 3000, "before the range"), (64, 0, 5000, "inside the range")):
        bad = bytearray(s)
        bad[32 + blk] |= 0x20
        announce(f"range: corrupt rate byte {name} (block {blk})")
        st, _ = gpu_decompress_range(bytes(bad), n, begin, end)
        assert st == fsz.FSZ_ERR_CORRUPT, name


def test_range_decode_beyond_4gib():
    """Random access in a stream of about 5.7 GB (2^31 + 4099 uniform values
    at REL 1e-6): a range across the tile whose data straddles byte 2^32,
    ranges whose data lies beyond it (several chunks, the field's end, its
    last element) and one across element 2^31 decode to the closed form
    fl(rint(fl(x * inv)) * E) bit for bit, with nothing written outside the
    range."""
    n = (1 << 31) + 4099
    rng = np.random.default_rng(29)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    announce(f"range beyond 4 GiB: compress uniform n={n} REL 1e-6")
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    xd = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    cmp = torch.zeros(cap, dtype=torch.uint8, device=_dev())
    r1 = torch.zeros(4, dtype=torch.int32, device=_dev())
    assert fsz.fsz_compress_async(xd.data_ptr(), n, fsz.FSZ_REL, 1e-6, None, cmp.data_ptr(), cap, r1.data_ptr(),
                                  stream) == fsz.FSZ_OK
    size, st, _ = fsz.read_result(r1)
    assert st == fsz.FSZ_OK and size > (1 << 32)
    head = cmp[:fmt.data_start(n)].cpu().numpy().tobytes()
    E = float(fmt.parse_header(head)["E"])
    ends = fmt.data_start(n) + np.cumsum(fmt.tile_sizes_np(head, n))
    assert int(ends[-1]) == size
    t = int(np.searchsorted(ends, 1 << 32, side="right"))  # the first tile whose data ends beyond 2^32
    assert int(ends[t - 1]) <= (1 << 32) < int(ends[t])
    inv = float(np.float32(1) / np.float32(E))
    ranges = [(fmt.TILE * t - 100, fmt.TILE * t + 300), (n - 70001, n - 3), (n - 1, n), (n - 1000003, n),
              ((1 << 31) - 5, (1 << 31) + 4000)]
    for begin, end in ranges:
        for off in (0, 1):
            announce(f"range beyond 4 GiB: [{begin}, {end}) output offset {off}")
            m = end - begin
            guard = 8
            out = torch.full((m + off + 2 * guard,), float("nan"), dtype=torch.float32, device=_dev())
            res = torch.zeros(2, dtype=torch.int64, device=_dev())
            assert fsz.fsz_decompress_range_async(cmp.data_ptr(), size, n, begin, end,
                                                  out.data_ptr() + 4 * (guard + off), res.data_ptr(),
                                                  stream) == fsz.FSZ_OK
            torch.cuda.synchronize()
            assert int(res.cpu()[1]) & 0xFFFFFFFF == fsz.FSZ_OK
            q = torch.round(xd[begin:end] * inv).to(torch.int32)  # zero as +0 whatever the product's sign
            expect = q.to(torch.float32) * E
            y = out[guard + off:guard + off + m]
            assert torch.equal(y.view(torch.int32), expect.view(torch.int32)), (begin, end)
            assert bool(torch.isnan(out[:guard + off]).all()) and bool(torch.isnan(out[guard + off + m:]).all())


def test_range_short_or_mismatched_stream_rejected():
    """A buffer shorter than the rate header of the caller's n fails on the
    host before any launch; a whole stream with another n fails in the decoder
    with a size mismatch (the range pass then reads only the stream's own
    rate bytes)."""
    x = workloads.sinusoid_field(50_000, 6)
    n = x.size
    s = oracle.compress(x, oracle.REL, 1e-3)
    rate_end = 32 + fmt.pad16(fmt.ceil_div(n, 32))
    for size in (32, 40, rate_end - 1):
        announce(f"range decode of a stream cut to {size} bytes")
        st, _ = gpu_decompress_range(s[:size], n, 20_000, 30_000)
        assert st == fsz.FSZ_ERR_CORRUPT, size
    # the caller's n larger than the stream's: its rate header would end past the buffer
    announce("range decode with n larger than the stream's rate header")
    big = n + 64 * len(s)
    st, _ = gpu_decompress_range(s, big, 20_000, 30_000)
    assert st == fsz.FSZ_ERR_CORRUPT
    # the caller's n a little larger: the buffer holds that many rate bytes, the header disagrees
    announce("range decode with a mismatched n")
    st, _ = gpu_decompress_range(s, n + 7, 20_000, 30_000)
    assert st == fsz.FSZ_ERR_SIZE_MISMATCH
