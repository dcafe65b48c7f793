"""GPU test of the allocation-free compression entry point: through the C ABI,
fsz_compress_noalloc_async writes the same stream and result as
fsz_compress_async (and as the oracle) on consecutive calls, the second on a
smaller input, so stale scratch contents of the first call must not leak into
the second.  Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    return torch.device("cuda:0")


def announce(name):
    print(f"\n[case] {name}", flush=True)


def _run(entry, xd, n, mode, value, stats_ptr, in_offset=0):
    """One call of `entry` (fsz_compress_async or fsz_compress_noalloc_async)
    on the current stream; returns (status, size, stream bytes or None)."""
    cap = fsz.fsz_compressed_bound(n)
    out = torch.full((cap + 64,), 0xA5, dtype=torch.uint8, device=_dev())
    res = torch.full((2,), -1, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    st = entry(xd.data_ptr() + 4 * in_offset, n, mode, value, stats_ptr, out.data_ptr(), cap, res.data_ptr(),
               stream)
    assert st == fsz.FSZ_OK, st
    torch.cuda.synchronize()
    r = res.cpu().numpy().view(np.uint64)
    size, status = int(r[0]), int(r[1] & 0xFFFFFFFF)
    if status != fsz.FSZ_OK:
        return status, size, None
    o = out.cpu().numpy()
    assert np.all(o[size:] == 0xA5), "bytes written past the stream"
    return status, size, o[:size].tobytes()


def _fields():
    yield "pwq 3,000,001", workloads.piecewise_quadratic((12, 500, 500), 2).reshape(-1)[:3_000_001]
    yield "sinusoid 100,003", workloads.sinusoid_field(100_003, 7)
    yield "grf 64x64x64 + 77", np.concatenate([workloads.grf_field((64, 64, 64), 5),
                                               workloads.sinusoid_field(77, 1)])
    yield "sinusoid 1,000", workloads.sinusoid_field(1_000, 3)
    yield "empty", np.zeros(0, dtype=np.float32)


@pytest.mark.parametrize("with_stats", [False, True])
@pytest.mark.parametrize("in_offset", [0, 1])
def test_noalloc_matches_async_on_consecutive_calls(with_stats, in_offset):
    for name, x in _fields():
        n = x.size
        for mode, value in ((fsz.FSZ_REL, 1e-3), (fsz.FSZ_ABS, 1e-2), (fsz.FSZ_REL, 1e-4)):
            announce(f"noalloc {name} mode={mode} value={value} stats={with_stats} in_offset={in_offset}")
            xd = torch.zeros(n + in_offset + 4, dtype=torch.float32, device=_dev())
            if n:
                xd[in_offset:in_offset + n] = torch.from_numpy(x).to(_dev())
            stats_ptr = None
            if with_stats:
                stats = torch.zeros(2, dtype=torch.float64, device=_dev())  # 16 bytes
                stream = torch.cuda.current_stream(_dev()).cuda_stream
                assert fsz.fsz_field_stats(xd.data_ptr() + 4 * in_offset, n, stats.data_ptr(), stream) == fsz.FSZ_OK
                stats_ptr = stats.data_ptr()
            ref = _run(fsz.fsz_compress_async, xd, n, mode, value, stats_ptr, in_offset)
            got = _run(fsz.fsz_compress_noalloc_async, xd, n, mode, value, stats_ptr, in_offset)
            assert got == ref, name
            st_o, want = oracle.compress_status(x, mode, value)
            assert got[0] == st_o, name
            if st_o == oracle.OK:
                assert got[2] == want, name


def test_noalloc_repeated_calls_shrinking():
    """Ten calls in a row on shrinking prefixes of one field: every stream
    equals the oracle's (flags and ticket start clear at each call)."""
    x = workloads.grf_field((96, 96, 96), 8).reshape(-1)
    xd = torch.from_numpy(x).to(_dev())
    for k in range(10):
        n = x.size >> k
        announce(f"noalloc shrinking prefix n={n}")
        st, size, got = _run(fsz.fsz_compress_noalloc_async, xd, n, fsz.FSZ_REL, 1e-3, None)
        assert st == fsz.FSZ_OK
        assert got == oracle.compress(x[:n], oracle.REL, 1e-3)


def test_noalloc_rejects_fields_beyond_its_scratch():
    announce("noalloc n = 2^30 + 1 rejected on the host")
    n = (1 << 30) + 1
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    # no device memory is touched: the size check comes before any launch
    st = fsz.fsz_compress_noalloc_async(16, n, fsz.FSZ_REL, 1e-3, None, 16, fsz.fsz_compressed_bound(n),
                                        res.data_ptr(), None)
    assert st == fsz.FSZ_ERR_TOO_LARGE
