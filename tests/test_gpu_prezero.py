"""GPU pre-zeroed decompression (Sec. III-A): the output is cleared, then
groups of 8 all-zero tiles are skipped.  Reconstructions must equal the
oracle's decode and the plain decoder's bit for bit on sparse, all-zero,
partly zero and ordinary fields, ragged sizes and unaligned outputs (the
output is pre-filled with NaN so that an element the fill or the decoder
misses shows).  Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests.test_gpu_parity import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    return torch.device("cuda:0")


def gpu_decode(entry, data, n, out_offset=0):
    buf = torch.from_numpy(np.frombuffer(data, dtype=np.uint8).copy()).to(_dev())
    out = torch.full((n + out_offset + 8,), float("nan"), dtype=torch.float32, device=_dev())
    res = torch.full((2,), -1, dtype=torch.int64, device=_dev())
    stream = torch.cuda.current_stream(_dev()).cuda_stream
    st = entry(buf.data_ptr(), len(data), out.data_ptr() + 4 * out_offset, n, res.data_ptr(), stream)
    assert st == fsz.FSZ_OK, st
    torch.cuda.synchronize()
    status = int(res.cpu().numpy().view(np.uint64)[1] & 0xFFFFFFFF)
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[:out_offset])) and np.all(np.isnan(o[out_offset + n:])), "write outside the output"
    return status, o[out_offset:out_offset + n]


def _fields():
    yield "sparse 2^22 (1 spike per 20000)", workloads.sparse_field(1 << 22, 5), 1e-3
    yield "all zero 3,000,017", np.zeros(3_000_017, dtype=np.float32), 1e-3
    yield "sparse 1,048,583 (1 per 2000)", workloads.sparse_field(1_048_583, 6, spacing=2000), 1e-3
    yield "piecewise quadratic 20x100x500 (zero boxes)", workloads.piecewise_quadratic((20, 100, 500), 2), 1e-2
    yield "grf 64x64x80", workloads.grf_field((64, 64, 80), 3), 1e-3
    for n in (1, 255, 256, 257, 2047, 2049, 16385):
        x = np.zeros(n, dtype=np.float32)
        x[n // 2] = 3.5
        yield f"one spike n={n}", x, 1e-3


@pytest.mark.parametrize("out_offset", [0, 1, 3])
def test_prezero_decode_matches_oracle(out_offset):
    for name, x, rel in _fields():
        n = x.size
        announce(f"prezero {name} REL {rel} out_offset {out_offset}")
        s = oracle.compress(x, oracle.REL, rel)
        ref = oracle.decompress(s, n)
        st, y = gpu_decode(fsz.fsz_decompress_prezero_async, s, n, out_offset)
        assert st == fsz.FSZ_OK, name
        assert np.array_equal(y.view(np.uint32), ref.view(np.uint32)), f"{name}: differs from the oracle"
        st, y2 = gpu_decode(fsz.fsz_decompress_async, s, n, out_offset)
        assert st == fsz.FSZ_OK and np.array_equal(y2.view(np.uint32), y.view(np.uint32)), name


def test_prezero_decode_empty_and_corrupt():
    announce("prezero n = 0")
    s = oracle.compress(np.zeros(0, dtype=np.float32), oracle.REL, 1e-3)
    st, y = gpu_decode(fsz.fsz_decompress_prezero_async, s, 0)
    assert st == fsz.FSZ_OK and y.size == 0
    announce("prezero corrupt rate byte and mismatched n")
    x = workloads.sparse_field(300_001, 8, spacing=500)
    s = bytearray(oracle.compress(x, oracle.REL, 1e-3))
    s[40] |= 0x20 if (40 - 32) % 8 == 0 else 0x80
    st, _ = gpu_decode(fsz.fsz_decompress_prezero_async, bytes(s), x.size)
    assert st == oracle.decompress_status(bytes(s), x.size)[0] == fsz.FSZ_ERR_CORRUPT
    good = oracle.compress(x, oracle.REL, 1e-3)
    st, _ = gpu_decode(fsz.fsz_decompress_prezero_async, good, x.size + 1)
    assert st == fsz.FSZ_ERR_SIZE_MISMATCH
