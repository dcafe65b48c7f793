"""GPU parity of the batched form (one launch over many jobs) and its plans.

Every job of a batch must produce exactly the plain call's bytes, so the
streams are compared with the CPU oracle byte for byte and reconstructions
bit for bit, under every launch shape the autotuner may pick, in HIP-graph
replays, with per-job errors, and with jobs that are not 16-byte aligned.
"""
import numpy as np
import pytest

import oracle
from paper_2607_15413_amd import fsz, workloads
from tests import fsz_format as fmt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(2, 0), (4, 0), (8, 0), (4, 2), (4, 3), (2, 4)]


def _dev():
    return torch.device("cuda:0")


def _stream():
    return torch.cuda.current_stream(_dev()).cuda_stream


def announce(name):
    print(f"\n[case] {name}", flush=True)


class DeviceBatch:
    """Device buffers and fsz_job records for a list of job specs.

    spec ("c", x, mode, value[, capacity]) compresses numpy float32 x;
    spec ("d", stream_bytes, n) decompresses a stream into n floats.
    offset > 0 shifts every device pointer by that many 4-byte words;
    out_offset (default: offset) shifts the compress outputs alone.
    """

    def __init__(self, specs, offset=0, out_offset=None):
        oo = offset if out_offset is None else out_offset
        dev = _dev()
        self.specs = specs
        self.res = torch.zeros((max(len(specs), 1), 4), dtype=torch.int32, device=dev)
        self.src, self.dst, self.jobs = [], [], []
        for k, s in enumerate(specs):
            rp = self.res[k].data_ptr()
            if s[0] == "c":
                x, mode, value = s[1], s[2], s[3]
                n = x.size
                cap = s[4] if len(s) > 4 else fsz.fsz_compressed_bound(n)
                xs = torch.zeros(n + offset + 4, dtype=torch.float32, device=dev)
                if n:
                    xs[offset:offset + n] = torch.from_numpy(x).to(dev)
                out = torch.full((cap + 4 * oo + 16,), 0xA5, dtype=torch.uint8, device=dev)
                self.src.append(xs)
                self.dst.append(out)
                self.jobs.append(fsz.compress_job(xs.data_ptr() + 4 * offset, n, mode, value,
                                                  out.data_ptr() + 4 * oo, cap, rp))
            else:
                data, n = s[1], s[2]
                buf = torch.zeros(len(data) + 4 * offset + 16, dtype=torch.uint8, device=dev)
                if data:
                    buf[4 * offset:4 * offset + len(data)] = torch.from_numpy(
                        np.frombuffer(data, dtype=np.uint8).copy()).to(dev)
                out = torch.full((n + offset + 4,), float("nan"), dtype=torch.float32, device=dev)
                self.src.append(buf)
                self.dst.append(out)
                self.jobs.append(fsz.decompress_job(buf.data_ptr() + 4 * offset, len(data),
                                                    out.data_ptr() + 4 * offset, n, rp))
        self.offset = offset
        self.out_offset = oo

    def run(self, tuning=None):
        st = fsz.fsz_batch_async(self.jobs, tuning, _stream())
        assert st == fsz.FSZ_OK, fsz.fsz_status_string(st)
        torch.cuda.synchronize()

    def results(self):
        r = self.res.cpu().numpy()
        out = []
        for k in range(len(self.specs)):
            size = int(r[k, 0].astype(np.uint32)) | (int(r[k, 1].astype(np.uint32)) << 32)
            out.append((size, int(r[k, 2])))
        return out

    def output(self, k):
        s = self.specs[k]
        size, st = self.results()[k]
        if st != fsz.FSZ_OK:
            return st, None
        if s[0] == "c":
            o = 4 * self.out_offset
            return st, self.dst[k][o:o + size].cpu().numpy().tobytes()
        n = s[2]
        return st, self.dst[k][self.offset:self.offset + n].cpu().numpy()

    def clear_outputs(self):
        for k, s in enumerate(self.specs):
            self.dst[k].fill_(0x5A if s[0] == "c" else float("nan"))
        self.res.zero_()


def check_against_oracle(b, refs, label):
    """refs[k] = (status, bytes) for compress specs, (status, floats) for decompress specs."""
    for k, s in enumerate(b.specs):
        st, got = b.output(k)
        st_ref, ref = refs[k]
        assert st == st_ref, (label, k, s[0], st, st_ref)
        if st != fsz.FSZ_OK:
            continue
        if s[0] == "c":
            assert got == ref, f"{label}: job {k} stream differs from the oracle"
        else:
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), \
                f"{label}: job {k} reconstruction differs"


def oracle_refs(specs):
    refs = []
    for s in specs:
        if s[0] == "c":
            st, data = oracle.compress_status(s[1], s[2], s[3])
            if st == fsz.FSZ_OK and len(s) > 4 and len(data) > s[4]:
                st, data = fsz.FSZ_ERR_CAPACITY, None
            refs.append((st, data))
        else:
            st, y = oracle.decompress_status(s[1], s[2])
            refs.append((st, y))
    return refs


def small_fields(count, seed, hi=1 << 19):
    return workloads.batch_fields(count, seed, lo=1 << 10, hi=hi, grf_shape=(64, 64, 128))


# ----------------------------------------------------------------- cases


def test_batch_compress_matches_oracle():
    fields = small_fields(24, 3)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    announce(f"batch compress 24 fields, sizes {[f.data.size for f in fields]}")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    b.run((4, 0))
    check_against_oracle(b, refs, "batch compress")


@pytest.mark.parametrize("shape", SHAPES)
def test_batch_every_shape_identical(shape):
    fields = small_fields(12, 5)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    for f in fields[:4]:
        _, data = oracle.compress_status(f.data, fsz.FSZ_ABS, 1e-3)
        specs.append(("d", data, f.data.size))
    announce(f"batch shape {shape}: 12 compress + 4 decompress jobs")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    if not fsz.load_library().fsz_batch_async(None, 0, fsz._tuning_ptr(shape), None) == fsz.FSZ_OK:
        pytest.skip(f"shape {shape} not supported on this device")
    b.run(shape)
    check_against_oracle(b, refs, f"shape {shape}")


def test_batch_mixed_decompress_matches_oracle():
    rng = np.random.default_rng(11)
    specs = []
    for k in range(20):
        n = int(rng.integers(1, 300_000))
        x = workloads.sinusoid_field(n, 100 + k)
        if k % 2 == 0:
            specs.append(("c", x, fsz.FSZ_REL, [1e-2, 1e-3, 1e-4][k % 3]))
        else:
            _, data = oracle.compress_status(x, fsz.FSZ_REL, 1e-3)
            specs.append(("d", data, n))
    announce("batch mixed 10 compress + 10 decompress")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    b.run()
    check_against_oracle(b, refs, "mixed")


def test_batch_many_jobs_and_edge_sizes():
    # more than 64 jobs (several probes of the job search) and every ragged edge
    sizes = [0, 1, 2, 31, 32, 33, 255, 256, 257, 2047, 2048, 2049, 8191, 8192, 8193, 16383, 16385]
    specs = []
    for k in range(150):
        n = sizes[k % len(sizes)] + (k // len(sizes)) * 97
        x = workloads.sinusoid_field(n, 500 + k) * (1.0 + k)
        specs.append(("c", x.astype(np.float32), fsz.FSZ_REL if k % 3 else fsz.FSZ_ABS, 1e-3))
    announce("batch 150 jobs with edge sizes")
    refs = oracle_refs(specs)
    for shape in [(2, 0), (4, 0), (8, 0)]:
        b = DeviceBatch(specs)
        b.run(shape)
        check_against_oracle(b, refs, f"150 jobs shape {shape}")


def test_batch_unaligned_pointers():
    fields = small_fields(8, 7, hi=1 << 17)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    _, data = oracle.compress_status(fields[0].data, fsz.FSZ_REL, 1e-2)
    specs.append(("d", data, fields[0].data.size))
    announce("batch unaligned (offset 1 word)")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs, offset=1)
    b.run()
    check_against_oracle(b, refs, "unaligned")


def test_batch_per_job_errors_are_isolated():
    good = workloads.sinusoid_field(50_000, 21)
    nan = good.copy()
    nan[1234] = np.nan
    tiny = good.copy()
    _, stream = oracle.compress_status(good, fsz.FSZ_REL, 1e-3)
    corrupt = bytearray(stream)
    corrupt[32] |= 0x20  # reserved bit of block 0's rate byte
    header_cap = 32 + (-(-good.size // 32) + 15) // 16 * 16
    specs = [
        ("c", good, fsz.FSZ_REL, 1e-3),
        ("c", nan, fsz.FSZ_REL, 1e-3),
        ("c", tiny, fsz.FSZ_ABS, 1e-12),           # bound below 8 ulp(max|x|)
        ("c", good, fsz.FSZ_REL, 1e-4, header_cap),  # capacity: rate header only
        ("d", bytes(corrupt), good.size),
        ("d", stream, good.size + 1),              # element count mismatch
        ("c", np.zeros(0, np.float32), fsz.FSZ_REL, 1e-3),
        ("d", stream, good.size),
    ]
    announce("batch per-job errors")
    refs = oracle_refs(specs)
    assert [r[0] for r in refs] == [0, 2, 3, 4, 5, 6, 0, 0]
    b = DeviceBatch(specs)
    b.run()
    check_against_oracle(b, refs, "errors")


def test_batch_compress_only_pipeline_errors():
    """A batch whose every job compresses (16-byte aligned) runs the persistent
    pipeline across job boundaries: jobs whose bound does not resolve pass
    through it as empty items and report their status, jobs that run out of
    capacity report it, and every other job's stream equals the oracle's."""
    good = workloads.sinusoid_field(300_000, 31)
    nan = good.copy()
    nan[777] = np.nan
    header_cap = 32 + (-(-good.size // 32) + 15) // 16 * 16
    specs = [
        ("c", good, fsz.FSZ_REL, 1e-3),
        ("c", nan, fsz.FSZ_REL, 1e-3),
        ("c", workloads.sinusoid_field(70_001, 32), fsz.FSZ_REL, 1e-2),
        ("c", good, fsz.FSZ_ABS, 1e-12),             # bound below 8 ulp(max|x|)
        ("c", np.zeros(0, np.float32), fsz.FSZ_REL, 1e-3),
        ("c", good, fsz.FSZ_REL, 1e-4, header_cap),  # capacity: rate header only
        ("c", workloads.grf_field((64, 64, 80), 33), fsz.FSZ_REL, 1e-4),
        ("c", np.full(5000, 3.0, np.float32), fsz.FSZ_REL, 1e-3),
        ("c", nan[:20000], fsz.FSZ_ABS, 1e-3),
        ("c", good[:16385], fsz.FSZ_ABS, 1e-4),
    ]
    refs = oracle_refs(specs)
    assert [r[0] for r in refs] == [0, 2, 0, 3, 0, 4, 0, 0, 2, 0]
    for shape in [(2, 0), (4, 0), (8, 0), (8, 1), (4, 1)]:
        announce(f"compress-only batch with per-job errors, shape {shape}")
        b = DeviceBatch(specs)
        b.run(shape)
        check_against_oracle(b, refs, f"compress-only errors {shape}")


def test_batch_compress_only_output_offsets():
    """Compress-only batch with aligned inputs (the pipelined kernel) writing
    to outputs at every 4-byte phase of a 16-byte line."""
    fields = small_fields(12, 23)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    refs = oracle_refs(specs)
    for oo in (1, 2, 3):
        announce(f"compress-only batch, outputs shifted by {oo} words")
        b = DeviceBatch(specs, offset=0, out_offset=oo)
        b.run((8, 0))
        check_against_oracle(b, refs, f"output offset {oo}")


def test_batch_decompress_only_persistent():
    """A batch whose every job decompresses runs the persistent decoder (the
    next item's size pass ahead of this item's decode): good streams of many
    sizes interleaved with bad ones (corrupt rate byte, bad magic, element
    count mismatch, empty field), at every shape and with unaligned pointers."""
    rng = np.random.default_rng(12)
    specs = []
    for k in range(40):
        n = int(rng.choice([0, 1, 255, 257, 16384, 16385, 70_000, 300_001]))
        x = workloads.sinusoid_field(n, 700 + k)
        _, data = oracle.compress_status(x, fsz.FSZ_REL, [1e-2, 1e-3, 1e-4][k % 3])
        if k % 7 == 3 and n > 300:
            bad = bytearray(data)
            bad[32 + 8 * (n // 512)] |= 0x20  # reserved bit in a middle tile
            data = bytes(bad)
        elif k % 7 == 5:
            bad = bytearray(data)
            bad[0] = ord("G")  # magic
            data = bytes(bad)
        specs.append(("d", data, n + 1 if k % 11 == 6 else n))
    refs = oracle_refs(specs)
    assert {r[0] for r in refs} >= {fsz.FSZ_OK, fsz.FSZ_ERR_CORRUPT, fsz.FSZ_ERR_SIZE_MISMATCH}
    for shape in [None, (2, 0), (4, 0), (8, 0), (8, 1)]:
        for offset in (0, 1):
            announce(f"batch decompress-only 40 jobs shape {shape} offset {offset}")
            b = DeviceBatch(specs, offset=offset)
            b.run(shape)
            check_against_oracle(b, refs, f"decompress-only shape {shape} offset {offset}")


def test_plan_graph_replays():
    fields = small_fields(16, 9)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    _, data = oracle.compress_status(fields[1].data, fsz.FSZ_REL, 1e-4)
    specs.append(("d", data, fields[1].data.size))
    announce("plan: graph capture + 3 replays with eager work between")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    st, plan = fsz.fsz_plan_create(b.jobs, (4, 0))
    assert st == fsz.FSZ_OK, fsz.fsz_status_string(st)
    try:
        other = torch.from_numpy(workloads.sinusoid_field(100_000, 3)).to(_dev())
        for rep in range(3):
            b.clear_outputs()
            # eager work on the same stream between replays (plain path + torch)
            out = torch.empty(fsz.fsz_compressed_bound(other.numel()), dtype=torch.uint8, device=_dev())
            st_p, _ = fsz.fsz_compress(other.data_ptr(), other.numel(), fsz.FSZ_REL, 1e-3, out.data_ptr(),
                                       out.numel(), _stream())
            assert st_p == fsz.FSZ_OK
            assert fsz.fsz_plan_launch(plan, _stream()) == fsz.FSZ_OK
            torch.cuda.synchronize()
            check_against_oracle(b, refs, f"replay {rep}")
        st, t = fsz.fsz_plan_get_tuning(plan)
        assert st == fsz.FSZ_OK and t == (4, 0)
    finally:
        fsz.fsz_plan_destroy(plan)


def test_plan_graph_replays_compress_only():
    """A captured compress-only batch (the persistent pipeline) replays
    correctly, with eager work between the replays."""
    fields = small_fields(10, 19)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    announce("plan: compress-only batch, graph capture + 3 replays")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    st, plan = fsz.fsz_plan_create(b.jobs, (8, 0))
    assert st == fsz.FSZ_OK, fsz.fsz_status_string(st)
    try:
        other = torch.from_numpy(workloads.sinusoid_field(100_000, 4)).to(_dev())
        for rep in range(3):
            b.clear_outputs()
            out = torch.empty(fsz.fsz_compressed_bound(other.numel()), dtype=torch.uint8, device=_dev())
            st_p, _ = fsz.fsz_compress(other.data_ptr(), other.numel(), fsz.FSZ_REL, 1e-3, out.data_ptr(),
                                       out.numel(), _stream())
            assert st_p == fsz.FSZ_OK
            assert fsz.fsz_plan_launch(plan, _stream()) == fsz.FSZ_OK
            torch.cuda.synchronize()
            check_against_oracle(b, refs, f"compress-only replay {rep}")
    finally:
        fsz.fsz_plan_destroy(plan)


def test_autotune_then_batch_identical():
    fields = small_fields(16, 13)
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    announce("autotune over launch shapes")
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    st, best = fsz.fsz_autotune(b.jobs, 2, _stream())
    assert st == fsz.FSZ_OK, fsz.fsz_status_string(st)
    assert best[0] in (2, 4, 8)
    torch.cuda.synchronize()
    check_against_oracle(b, refs, "after autotune")
    b.clear_outputs()
    b.run(None)  # cached choice for this size class
    check_against_oracle(b, refs, f"cached shape {best}")


@pytest.mark.slow
def test_batch_64_fields_full_sizes():
    """The 64-field workload (16K-16M elements, ~620 MB) in one launch against the oracle."""
    fields = workloads.batch_fields(64, 3)
    sizes = [f.data.size for f in fields]
    announce(f"batch 64 fields, {sum(sizes)} elements")
    specs = [("c", f.data, fsz.FSZ_REL, f.rel) for f in fields]
    refs = oracle_refs(specs)
    b = DeviceBatch(specs)
    b.run()
    check_against_oracle(b, refs, "64 fields compress")
    dspecs = [("d", refs[k][1], sizes[k]) for k in range(len(fields))]
    drefs = oracle_refs(dspecs)
    db = DeviceBatch(dspecs)
    db.run()
    check_against_oracle(db, drefs, "64 fields decompress")


def test_batch_stream_beyond_4gib():
    """64-bit offsets in the batched kernels: a ragged small field, 2^31 +
    4099 uniform values at REL 1e-6 (a stream of about 5.7 GB) and another
    small field, compressed in one launch (the pipelined kernel) and
    decompressed in another (the persistent decoder).  The small jobs
    against the oracle; for the large job, the rate header sums to the
    stream's size, the first and the last 4096 tiles (the last ones stored
    beyond 2^32 bytes) equal the oracle's streams of the same elements, and
    the decode equals the closed form fl(rint(fl(x * inv)) * E)."""
    small = small_fields(2, 21)
    n = (1 << 31) + 4099
    rng = np.random.default_rng(23)
    x = rng.random(n, dtype=np.float32)
    x *= 2
    x -= 1
    rel = 1e-6
    specs = [("c", small[0].data, fsz.FSZ_REL, small[0].rel), ("c", x, fsz.FSZ_REL, rel),
             ("c", small[1].data, fsz.FSZ_REL, small[1].rel)]
    announce(f"batch with a stream beyond 4 GiB: jobs of {[s[1].size for s in specs]} elements, compress")
    b = DeviceBatch(specs)
    b.run()
    for k in (0, 2):
        st, got = b.output(k)
        assert st == fsz.FSZ_OK and got == oracle.compress(specs[k][1], specs[k][2], specs[k][3]), k
    st, s = b.output(1)
    assert st == fsz.FSZ_OK and len(s) > (1 << 32)
    hdr = fmt.parse_header(s)
    assert hdr["total"] == len(s)
    E = float(hdr["E"])
    sizes = fmt.tile_sizes_np(s, n)
    d0 = fmt.data_start(n)
    assert d0 + int(sizes.sum()) == len(s)
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
        assert s[r0:r0 + nb] == ref[fmt.HEADER:fmt.HEADER + nb], f"rate bytes of tiles from {first}"
        at = d0 + int(sizes[:first].sum())
        body = int(sizes[first:first + m].sum())
        if first:
            assert at > (1 << 32)
        ds = fmt.data_start(hi - lo)
        assert len(ref) == ds + body
        assert s[at:at + body] == ref[ds:], f"data of tiles from {first}"
    xd = b.src[1][:n]
    del b
    dspecs = [("d", oracle.compress(small[0].data, fsz.FSZ_REL, small[0].rel), small[0].data.size), ("d", s, n),
              ("d", oracle.compress(small[1].data, fsz.FSZ_REL, small[1].rel), small[1].data.size)]
    del s
    announce("batch with a stream beyond 4 GiB: decompress")
    db = DeviceBatch(dspecs)
    db.run()
    r = db.results()
    assert all(st == fsz.FSZ_OK for _, st in r), r
    for k in (0, 2):
        y_ref = oracle.decompress(dspecs[k][1], dspecs[k][2])
        assert np.array_equal(db.output(k)[1].view(np.uint32), y_ref.view(np.uint32)), k
    y = db.dst[1][:n]
    inv = np.float32(1) / np.float32(E)
    q = torch.round(xd * float(inv)).to(torch.int32)  # zero as +0 whatever the product's sign
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
