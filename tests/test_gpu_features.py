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
