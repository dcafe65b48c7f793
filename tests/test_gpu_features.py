"""GPU parity of the feature switches (the ablation of Sec. VI-B) and of the
five-read baseline (Sec. V-C, Fig. 6).  For every
subset of {cross-block state, centering, LZ2} the HIP streams equal the
oracle's byte for byte, through the aligned (pipelined) and the unaligned
(one chunk per workgroup) kernels, and every decoder path reconstructs them
bit-identically.  Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests import fsz_format as fmt
from tests.test_gpu_parity import announce, first_diff, gpu_decompress

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SETTINGS = list(range(8))  # bit 0 cross-block, bit 1 centering, bit 2 LZ2


def _dev():
    return torch.device("cuda:0")


def gpu_compress_features(x, mode, value, features, in_offset=0):
    """Compress numpy float32 x with a feature subset; returns (status, bytes or None)."""
    n = x.size
    xd = torch.zeros(n + in_offset + 4, dtype=torch.float32, device=_dev())
    if n:
        xd[in_offset:in_offset + n] = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    out = torch.zeros(max(cap, 1), dtype=torch.uint8, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    st = fsz.fsz_compress_features_async(xd.data_ptr() + 4 * in_offset, n, mode, value, None, features,
                                         out.data_ptr(), cap, res.data_ptr(), stream)
    if st != fsz.FSZ_OK:
        return st, None
    torch.cuda.synchronize()
    r = res.cpu()
    size, st = int(r[0]), int(r[1]) & 0xFFFFFFFF
    if st != fsz.FSZ_OK:
        return st, None
    return st, out[:size].cpu().numpy().tobytes()


def _fields():
    yield "sinusoid 1", workloads.sinusoid_field(1, 3)
    yield "sinusoid 1000", workloads.sinusoid_field(1000, 4)
    yield "pwq 8x40x200 (64000)", workloads.piecewise_quadratic((8, 40, 200), 5)
    yield "grf 64x64x80 (20 pipelined chunks)", workloads.grf_field((64, 64, 80), 6)
    yield "pwq 5x301x181 (ragged tail, 272405)", workloads.piecewise_quadratic((5, 301, 181), 7)


@pytest.mark.parametrize("features", SETTINGS)
def test_feature_streams_match_oracle(features):
    for name, x in _fields():
        for rel in (1e-2, 1e-4):
            for off in (0, 1):
                announce(f"features {features} {name} REL {rel:g} input offset {off}")
                exp = oracle.compress(x, oracle.REL, rel, features=features)
                st, got = gpu_compress_features(x, oracle.REL, rel, features, in_offset=off)
                assert st == fsz.FSZ_OK
                assert got == exp, first_diff(got, exp)
            st, y = gpu_decompress(exp, x.size)
            assert st == fsz.FSZ_OK
            assert np.array_equal(y.view(np.uint32), oracle.decompress(exp, x.size).view(np.uint32))


def test_full_setting_equals_plain_call():
    x = workloads.grf_field((64, 64, 64), 9)
    announce("features 7 vs fsz_compress on grf 64^3")
    st, got = gpu_compress_features(x, oracle.REL, 1e-3, fsz.FSZ_FEATURES_ALL)
    assert st == fsz.FSZ_OK
    assert got == oracle.compress(x, oracle.REL, 1e-3)


def test_feature_argument_errors():
    x = workloads.sinusoid_field(100, 1)
    announce("feature bits outside the mask")
    st, _ = gpu_compress_features(x, oracle.REL, 1e-3, 8)
    assert st == fsz.FSZ_ERR_INVALID_ARG


def test_ablation_sizes_on_a_grf_slice():
    """The ablation's four columns (Base, +Cross, +Cent, +LZ2) on a 2^21-element
    k^-3 field: sizes equal the oracle's and never grow as designs are added
    with the same block structure."""
    x = workloads.grf_field((128, 128, 128), 1)
    sizes = {}
    for features in (0, 1, 3, 7):
        announce(f"ablation column features {features} on grf 128^3")
        st, got = gpu_compress_features(x, oracle.REL, 1e-3, features)
        assert st == fsz.FSZ_OK
        exp = oracle.compress(x, oracle.REL, 1e-3, features=features)
        assert got == exp, first_diff(got, exp)
        sizes[features] = len(got)
    assert sizes[7] <= sizes[3] <= sizes[1]


def gpu_compress_five_read(x, mode, value, in_offset=0):
    n = x.size
    xd = torch.zeros(n + in_offset + 4, dtype=torch.float32, device=_dev())
    if n:
        xd[in_offset:in_offset + n] = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    out = torch.zeros(max(cap, 1), dtype=torch.uint8, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    st = fsz.fsz_compress_five_read_async(xd.data_ptr() + 4 * in_offset, n, mode, value, None,
                                          out.data_ptr(), cap, res.data_ptr(), stream)
    if st != fsz.FSZ_OK:
        return st, None
    torch.cuda.synchronize()
    r = res.cpu()
    size, st = int(r[0]), int(r[1]) & 0xFFFFFFFF
    if st != fsz.FSZ_OK:
        return st, None
    return st, out[:size].cpu().numpy().tobytes()


def test_five_read_baseline_matches_oracle():
    """Sec. V-C: the naive five-read evaluation produces the same stream as
    the single pass."""
    for name, x in list(_fields()) + [("empty", np.zeros(0, dtype=np.float32))]:
        for rel in (1e-2, 1e-4):
            for off in (0, 1):
                announce(f"five-read {name} REL {rel:g} input offset {off}")
                st, got = gpu_compress_five_read(x, oracle.REL, rel, in_offset=off)
                assert st == fsz.FSZ_OK
                exp = oracle.compress(x, oracle.REL, rel)
                assert got == exp, first_diff(got, exp)


def test_five_read_reports_errors():
    x = workloads.sinusoid_field(5000, 2)
    announce("five-read: bound too small, then a NaN")
    st, _ = gpu_compress_five_read(x, oracle.ABS, 1e-12)
    assert st == fsz.FSZ_ERR_EB_TOO_SMALL
    x[77] = np.nan
    st, _ = gpu_compress_five_read(x, oracle.REL, 1e-3)
    assert st == fsz.FSZ_ERR_NONFINITE


def test_base_features_stream_beyond_4gib():
    """64-bit offsets in the feature-switch kernel: 2^31 + 4099 uniform values
    at REL 1e-6 with every feature off (independent blocks, first order, no
    centering) give a stream beyond 2^32 bytes.  The rate header sums to its
    size, the first and the last 4096 tiles (the last ones stored beyond
    2^32 bytes) equal the oracle's streams of the same elements, and the
    plain decoder, which honours the independent-blocks flag, gives the
    closed form fl(rint(fl(x * inv)) * E) over the whole field."""
    n = (1 << 31) + 4099
    rng = np.random.default_rng(31)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    rel = 1e-6
    announce(f"features 0, stream beyond 4 GiB: uniform n={n} REL {rel:g}")
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    xd = torch.from_numpy(x).to(_dev())
    cap = fsz.fsz_compressed_bound(n)
    out = torch.zeros(cap, dtype=torch.uint8, device=_dev())
    res = torch.zeros(2, dtype=torch.int64, device=_dev())
    assert fsz.fsz_compress_features_async(xd.data_ptr(), n, fsz.FSZ_REL, rel, None, 0, out.data_ptr(), cap,
                                           res.data_ptr(), stream) == fsz.FSZ_OK
    torch.cuda.synchronize()
    r = res.cpu()
    size, st = int(r[0]), int(r[1]) & 0xFFFFFFFF
    assert st == fsz.FSZ_OK and size > (1 << 32)
    d0 = fmt.data_start(n)
    head = out[:d0].cpu().numpy().tobytes()
    hdr = fmt.parse_header(head)
    assert hdr["total"] == size and hdr["flags"] & 2
    E = float(hdr["E"])
    sizes = fmt.tile_sizes_np(head, n)
    assert d0 + int(sizes.sum()) == size
    m = 4096
    for first in (0, sizes.size - m):
        lo, hi = first * fmt.TILE, min(n, (first + m) * fmt.TILE)
        xs = x[lo:hi]
        # an ABS bound of E/2 + 4 ulp(max|xs|) resolves to the same step E
        u = float(np.spacing(np.float32(np.abs(xs).max())))
        ref = oracle.compress(xs, oracle.ABS, E / 2 + 4 * u, features=0)
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
        got = out[at:at + body].cpu().numpy().tobytes()
        assert got == ref[ds:], f"data of tiles from {first}: " + first_diff(got, ref[ds:])
    announce(f"features 0, stream beyond 4 GiB: decode of {size} bytes")
    y = torch.empty(n, dtype=torch.float32, device=_dev())
    r2 = torch.zeros(2, dtype=torch.int64, device=_dev())
    assert fsz.fsz_decompress_async(out.data_ptr(), size, y.data_ptr(), n, r2.data_ptr(), stream) == fsz.FSZ_OK
    torch.cuda.synchronize()
    assert int(r2.cpu()[1]) & 0xFFFFFFFF == fsz.FSZ_OK
    del out
    inv = float(np.float32(1) / np.float32(E))
    q = torch.round(xd * inv).to(torch.int32)  # zero as +0 whatever the product's sign
    del xd
    expect = q.to(torch.float32) * E
    del q
    step = 1 << 28
    for k in range(0, n, step):
        a = y[k:k + step].view(torch.int32)
        e = expect[k:k + step].view(torch.int32)
        bad = (a != e).nonzero()
        if bad.numel():
            i = k + int(bad[0])
            raise AssertionError(f"{bad.numel()} of the elements [{k}, {k + a.numel()}) differ; first at {i}: "
                                 f"decoded {float(y[i])} expected {float(expect[i])} (x = {float(x[i])})")
