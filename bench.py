"""FSZ benchmark on one MI355X.

One step = the whole hot path over the 512^3 float32 k^-3 Gaussian random
field (512 MiB): the value-range pass once, then for each REL bound in
{1e-2, 1e-3, 1e-4} one compression and one decompression, all enqueued
asynchronously on one stream (inputs and outputs resident in HBM).

Printed JSON line (rank 0): value = original bytes compressed + decompressed
per second over the timed steps (GB/s, 1 GB = 1e9 B), with per-bound
compress / decompress GB/s (4n / kernel time), compression ratios and
max|x - x'|/eb, the roofline of the dominant kernel measured with HIP events
on the launch stream, a plain device copy as the practical ceiling, the CPU
oracle timed on the host as a baseline, the batched form against per-field
calls on 64 uneven fields, and the two smaller field configurations.
`--served` runs the served request loop instead (its own JSON line).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
RELS = (1e-2, 1e-3, 1e-4)
PROFILE = os.path.join(ROOT, "profiles", "compress_decompress_grf512.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2607_15413_amd", "csrc", "fsz_kernels.hip")


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        text = open(PROFILE).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("kernel_source_sha256:"):
            fields["sha"] = line.split(":", 1)[1].strip()
        elif line.startswith("traffic_bytes_per_launch:"):
            for kv in line.split(":", 1)[1].split():
                k, v = kv.split("=")
                fields[k] = int(v)
    if fields.get("sha") != sha:
        return None
    return fields.get(kernel)


def batched_comparison(torch, fsz, workloads, reps: int, verify_oracle: bool):
    """64 uneven fields (seed 3, 16K-16M elements, REL from {1e-2, 1e-3, 1e-4}):
    64 plain asynchronous calls (each with its own range pass) against one
    batched launch, one autotuned batched launch and one graph replay of a plan,
    for compression and for decompression.  GB/s = original bytes / time."""
    t0 = time.time()
    fields = workloads.batch_fields(64, 3)
    print(f"[bench] generated 64 batch fields in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    xs = [torch.from_numpy(f.data).to(dev) for f in fields]
    ns = [f.data.size for f in fields]
    caps = [fsz.fsz_compressed_bound(n) for n in ns]
    total_bytes = 4 * sum(ns)
    outs_p = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    outs_b = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    ys_p = [torch.empty(n, dtype=torch.float32, device=dev) for n in ns]
    ys_b = [torch.empty(n, dtype=torch.float32, device=dev) for n in ns]
    res = torch.zeros((4 * 64, 4), dtype=torch.int32, device=dev)

    def rptr(k):
        return res[k].data_ptr()

    def check(st, what):
        if st != fsz.FSZ_OK:
            raise RuntimeError(f"{what}: {fsz.fsz_status_string(st)}")

    def plain_compress():
        for k in range(64):
            check(fsz.fsz_compress_async(xs[k].data_ptr(), ns[k], fsz.FSZ_REL, fields[k].rel, None,
                                         outs_p[k].data_ptr(), caps[k], rptr(k), sh), "plain compress")

    cjobs = [fsz.compress_job(xs[k].data_ptr(), ns[k], fsz.FSZ_REL, fields[k].rel, outs_b[k].data_ptr(),
                              caps[k], rptr(64 + k)) for k in range(64)]

    def timed(fn, n_reps):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n_reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n_reps

    ms_pc = timed(plain_compress, reps)
    ms_bc_default = timed(lambda: check(fsz.fsz_batch_async(cjobs, (4, 0), sh), "batch"), reps)
    st, tuned = fsz.fsz_autotune(cjobs, 3, sh)
    check(st, "autotune")
    ms_bc = timed(lambda: check(fsz.fsz_batch_async(cjobs, tuned, sh), "batch"), reps)
    st, plan = fsz.fsz_plan_create(cjobs, tuned)
    check(st, "plan")
    ms_gc = timed(lambda: check(fsz.fsz_plan_launch(plan, sh), "plan launch"), reps)
    fsz.fsz_plan_destroy(plan)
    torch.cuda.synchronize()
    r = res.cpu().numpy().astype(np.uint32)
    sizes_p = [int(r[k, 0]) | (int(r[k, 1]) << 32) for k in range(64)]
    sizes_b = [int(r[64 + k, 0]) | (int(r[64 + k, 1]) << 32) for k in range(64)]
    if any(int(r[k, 2]) != 0 for k in range(128)):
        raise RuntimeError("a batched or plain compression failed")
    identical = sizes_p == sizes_b and all(
        torch.equal(outs_p[k][:sizes_p[k]], outs_b[k][:sizes_b[k]]) for k in range(64))

    def plain_decompress():
        for k in range(64):
            check(fsz.fsz_decompress_async(outs_p[k].data_ptr(), sizes_p[k], ys_p[k].data_ptr(), ns[k],
                                           rptr(128 + k), sh), "plain decompress")

    djobs = [fsz.decompress_job(outs_p[k].data_ptr(), sizes_p[k], ys_b[k].data_ptr(), ns[k], rptr(192 + k))
             for k in range(64)]
    ms_pd = timed(plain_decompress, reps)
    st, dtuned = fsz.fsz_autotune(djobs, 3, sh)
    check(st, "autotune")
    ms_bd = timed(lambda: check(fsz.fsz_batch_async(djobs, dtuned, sh), "batch"), reps)
    st, dplan = fsz.fsz_plan_create(djobs, dtuned)
    check(st, "plan")
    ms_gd = timed(lambda: check(fsz.fsz_plan_launch(dplan, sh), "plan launch"), reps)
    fsz.fsz_plan_destroy(dplan)
    torch.cuda.synchronize()
    r = res.cpu().numpy().astype(np.uint32)
    if any(int(r[k, 2]) != 0 for k in range(128, 256)):
        raise RuntimeError("a batched or plain decompression failed")
    identical = identical and all(torch.equal(ys_p[k].view(torch.int32), ys_b[k].view(torch.int32))
                                  for k in range(64))
    oracle_ok = None
    if verify_oracle:
        import oracle
        oracle_ok = all(outs_b[k][:sizes_b[k]].cpu().numpy().tobytes()
                        == oracle.compress(fields[k].data, oracle.REL, fields[k].rel) for k in range(64))
    stream_bytes = sum(sizes_p)

    def gbps(ms):
        return round(total_bytes / ms / 1e6, 1)

    return {
        "workload": "64 fields, seed 3, 16K-16M elements (log-uniform, ragged), sinusoid or k^-3 GRF slice, "
                    "REL from {1e-2,1e-3,1e-4}",
        "elements": int(sum(ns)),
        "stream_bytes": int(stream_bytes),
        "per_field_compress_GBps": gbps(ms_pc),
        "batch_compress_GBps_default_shape": gbps(ms_bc_default),
        "batch_compress_GBps": gbps(ms_bc),
        "plan_compress_GBps": gbps(ms_gc),
        "per_field_decompress_GBps": gbps(ms_pd),
        "batch_decompress_GBps": gbps(ms_bd),
        "plan_decompress_GBps": gbps(ms_gd),
        "compress_ms": {"per_field": round(ms_pc, 4), "batch": round(ms_bc, 4), "plan": round(ms_gc, 4)},
        "decompress_ms": {"per_field": round(ms_pd, 4), "batch": round(ms_bd, 4), "plan": round(ms_gd, 4)},
        "tuning_compress": list(tuned),
        "tuning_decompress": list(dtuned),
        "identical_to_per_field": bool(identical),
        "oracle_identical": oracle_ok,
    }


SERVED_WORKLOAD = ("Poisson requests, seed 4, 70% compress / 30% decompress, 1K-64M elements log-uniform "
                   "from the 269x500x500 piecewise-quadratic field (seed 2), REL {1e-3,1e-4}")


def served_run(torch, fsz, workloads, loads, counts, plain_requests=10000, budget_gb=64.0, rounds_in_flight=4,
               jobs_per_round=256, timeline=None, verify_sample=0):
    """Served form: open-loop Poisson requests (seed 4; 70% compress / 30%
    decompress of previously compressed streams; log-uniform 1K-64M elements
    sliced from the 269x500x500 piecewise-quadratic master field; REL from
    {1e-3, 1e-4}) against a server with an HBM admission budget, at offered
    loads given as fractions of the plain kernels' measured closed-loop
    throughput on the same requests.  Per load: p50/p99 latency (arrival to
    completion seen by the host) and sustained GB/s (original bytes / span
    from first arrival to last completion).

    verify_sample > 0: a seeded sample of that many compress requests (every
    one of at least 2^24 elements among the first requests included) and a
    third as many decompress requests is served once more, at offered load
    0.9, by a server that keeps its outputs; each output is compared on the
    device with the plain path's output for the same request, byte for byte
    (streams) and bit for bit (floats)."""
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    nmax = max(counts)
    t0 = time.time()
    shape = (269, 500, 500)
    master_np = workloads.piecewise_quadratic(shape, 2)
    master = torch.from_numpy(master_np).to(dev)
    reqs = workloads.request_stream(1.0, nmax, 4, master_n=master_np.size)
    del master_np
    print(f"[served] master {shape} + {nmax} requests generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    def check(st, what):
        if st != fsz.FSZ_OK:
            raise RuntimeError(f"{what}: {fsz.fsz_status_string(st)}")

    # streams that decompress requests read: compressed once by the plain
    # path, then kept in buffers of their exact size
    res = torch.zeros((nmax, 4), dtype=torch.int32, device=dev)
    streams = {}
    ssize = {}
    tmp = torch.empty(fsz.fsz_compressed_bound(max(r.n for r in reqs)), dtype=torch.uint8, device=dev)
    for k, r in enumerate(reqs):
        if r.op == "decompress":
            check(fsz.fsz_compress_async(master.data_ptr() + 4 * r.offset, r.n, fsz.FSZ_REL, r.rel, None,
                                         tmp.data_ptr(), tmp.numel(), res[k].data_ptr(), sh), "precompress")
            size, st, _ = fsz.read_result(res[k])
            check(st, "precompress")
            streams[k] = tmp[:size].clone()
            ssize[k] = int(size)
    del tmp
    torch.cuda.synchronize()
    print(f"[served] {len(streams)} decompress inputs ready", file=sys.stderr, flush=True)

    # plain closed loop over the same requests: every request one plain call,
    # back to back on one stream (calls on a stream are ordered, so one output
    # buffer per operation serves them all)
    nmax_n = max(r.n for r in reqs)
    out_c = torch.empty(fsz.fsz_compressed_bound(nmax_n), dtype=torch.uint8, device=dev)
    out_d = torch.empty(nmax_n, dtype=torch.float32, device=dev)

    def plain_call(k, dst):
        r = reqs[k]
        if r.op == "compress":
            check(fsz.fsz_compress_async(master.data_ptr() + 4 * r.offset, r.n, fsz.FSZ_REL, r.rel, None,
                                         dst.data_ptr(), dst.numel(), res[k].data_ptr(), sh), "plain compress")
        else:
            check(fsz.fsz_decompress_async(streams[k].data_ptr(), ssize[k], dst.data_ptr(), r.n,
                                           res[k].data_ptr(), sh), "plain decompress")

    def plain_pass(n_req):
        for k in range(n_req):
            plain_call(k, out_c if reqs[k].op == "compress" else out_d)

    n_plain = min(nmax, plain_requests)
    plain_pass(n_plain)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    plain_pass(n_plain)
    b.record(stream)
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b)
    plain_bytes = sum(4 * reqs[k].n for k in range(n_plain))
    plain_gbps = plain_bytes / plain_ms / 1e6
    rr = res.cpu().numpy().astype(np.uint32)
    if any(int(rr[k, 2]) != 0 for k in range(n_plain)):
        raise RuntimeError("a plain call failed")
    del out_c, out_d
    torch.cuda.empty_cache()
    print(f"[served] plain closed loop: {n_plain} requests, {plain_gbps:.1f} GB/s", file=sys.stderr, flush=True)

    budget = int(budget_gb * 1e9)
    table = fsz.request_table(nmax)
    for k, r in enumerate(reqs):
        if r.op == "compress":
            table[k] = (fsz.FSZ_OP_COMPRESS, master.data_ptr() + 4 * r.offset, 0, r.n, fsz.FSZ_REL, r.rel, k, 0)
        else:
            table[k] = (fsz.FSZ_OP_DECOMPRESS, streams[k].data_ptr(), ssize[k], r.n, 0, 0.0, k, 0)
    arrival_s = np.array([r.arrival_s for r in reqs])

    def serve(server, sub, rate, keep=None):
        """Submit the request table rows `sub` with arrivals scaled to `rate`
        requests per second; collect every completion.  keep(c): called for
        completions whose output the server holds (then released)."""
        count = len(sub)
        before = fsz.fsz_server_get_stats(server)
        start = fsz.fsz_server_now_ns() + 5_000_000
        sub["arrival_ns"] = start + ((arrival_s[:count] - arrival_s[0]) / rate * 1e9).astype(np.uint64)
        check(fsz.fsz_server_submit_table(server, sub), "submit")
        lead_ms = (start - fsz.fsz_server_now_ns()) / 1e6  # > 0: submitted before the first arrival
        done = {}
        last_print = time.time()
        while len(done) < count:
            for c in fsz.fsz_server_poll(server, 4096, 200):
                done[c.tag] = (c.status, c.arrival_ns, c.admit_ns, c.launch_ns, c.complete_ns, c.size)
                if c.d_out:
                    keep(c)
                    check(fsz.fsz_server_release(server, c.d_out), "release")
            if time.time() - last_print > 5:
                print(f"[served] {len(done)}/{count} done", file=sys.stderr, flush=True)
                last_print = time.time()
        after = fsz.fsz_server_get_stats(server)
        return done, int(after.rounds - before.rounds), after, lead_ms

    import gc
    results = []
    runs = []
    gc.disable()  # no collector pauses in the client while requests are in flight
    # one long-running server for every load point, warmed up by one short pass
    st, server = fsz.fsz_server_create(budget, jobs_per_round, rounds_in_flight, True, (4, 0))
    check(st, "server create")
    try:
        n_warm = min(200, nmax)
        serve(server, table[:n_warm].copy(),
              0.5 * plain_gbps * 1e9 / float(np.mean([4 * reqs[k].n for k in range(n_warm)])))
        for load, count in zip(loads, counts):
            mean_bytes = float(np.mean([4 * reqs[k].n for k in range(count)]))
            rate = load * plain_gbps * 1e9 / mean_bytes  # requests per second
            runs.append((load, count, rate) + serve(server, table[:count].copy(), rate))
    finally:
        fsz.fsz_server_destroy(server)
        gc.enable()
    if timeline:
        np.savez(timeline, **{
            f"load_{load}": np.array([[done[k][1], done[k][2], done[k][3], done[k][4], reqs[k].n,
                                       int(reqs[k].op == "compress")] for k in range(count)], dtype=np.int64)
            for load, count, rate, done, rounds, stats, lead in runs})
    for load, count, rate, done, rounds, stats, lead in runs:
        bad = [k for k, v in done.items() if v[0] != fsz.FSZ_OK]
        if bad:
            raise RuntimeError(f"served requests failed: {bad[:5]}")
        sizes_ok = True
        for k, v in done.items():  # stream sizes equal the plain path's
            if reqs[k].op == "decompress":
                sizes_ok = sizes_ok and v[5] == ssize[k]
            elif v[5] != int(rr[k, 0]) | (int(rr[k, 1]) << 32) and k < n_plain:
                sizes_ok = False
        if not sizes_ok:
            raise RuntimeError("a served size differs from the plain path's")
        keys = list(done.keys())
        lat = np.array([(done[k][4] - done[k][1]) / 1e6 for k in keys])
        queue = np.array([(done[k][3] - done[k][1]) / 1e6 for k in keys])
        service = np.array([(done[k][4] - done[k][3]) / 1e6 for k in keys])
        sizes_n = np.array([reqs[k].n for k in keys])
        by_size = {}
        for label, lo, hi in (("<1M", 0, 1 << 20), ("1M-16M", 1 << 20, 1 << 24), (">=16M", 1 << 24, 1 << 62)):
            m = (sizes_n >= lo) & (sizes_n < hi)
            if m.any():
                by_size[label] = {"requests": int(m.sum()), "p50_ms": round(float(np.percentile(lat[m], 50)), 4),
                                  "p99_ms": round(float(np.percentile(lat[m], 99)), 4)}
        t_first = min(v[1] for v in done.values())
        span_s = (max(v[4] for v in done.values()) - t_first) / 1e9
        comp = np.sort(np.array([v[4] for v in done.values()], dtype=np.int64))
        gaps = np.diff(comp)
        gap_at = int(np.argmax(gaps)) if gaps.size else 0
        total_bytes = sum(4 * reqs[k].n for k in range(count))
        entry = {
            "offered_load": load,
            "requests": count,
            "rate_per_s": round(rate, 1),
            "offered_GBps": round(load * plain_gbps, 1),
            "sustained_GBps": round(total_bytes / span_s / 1e9, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "mean_ms": round(float(lat.mean()), 4),
            "p50_wait_to_launch_ms": round(float(np.percentile(queue, 50)), 4),
            "p99_wait_to_launch_ms": round(float(np.percentile(queue, 99)), 4),
            "p50_service_ms": round(float(np.percentile(service, 50)), 4),
            "p99_service_ms": round(float(np.percentile(service, 99)), 4),
            "latency_by_size": by_size,
            "rounds": rounds,
            "mean_jobs_per_round": round(count / max(rounds, 1), 2),
            "max_rounds_overlapping": int(stats.max_rounds_overlapping),
            "submit_lead_ms": round(lead, 3),
            "max_completion_gap_ms": round(float(gaps[gap_at]) / 1e6, 3) if gaps.size else 0.0,
            "max_gap_at_ms": round(float(comp[gap_at] - t_first) / 1e6, 3) if gaps.size else 0.0,
        }
        results.append(entry)
        print(f"[served] {json.dumps(entry)}", file=sys.stderr, flush=True)

    verify = None
    if verify_sample > 0:
        verify = served_verify(torch, fsz, reqs, table, streams, ssize, master, serve, check, plain_gbps,
                               budget, jobs_per_round, rounds_in_flight, verify_sample, res)
        print(f"[served] verify {json.dumps(verify)}", file=sys.stderr, flush=True)
    del streams, master
    torch.cuda.empty_cache()
    return {
        "workload": SERVED_WORKLOAD,
        "hbm_budget_GB": budget_gb,
        "rounds_in_flight": rounds_in_flight,
        "max_jobs_per_round": jobs_per_round,
        "plain_closed_loop_GBps": round(plain_gbps, 1),
        "plain_closed_loop_requests": n_plain,
        "server_hbm_peak_GB": round(runs[-1][5].hbm_peak / 1e9, 3) if runs else None,
        "per_load": results,
        "verify": verify,
    }


def served_verify(torch, fsz, reqs, table, streams, ssize, master, serve, check, plain_gbps, budget,
                  jobs_per_round, rounds_in_flight, sample, res):
    """Serve a seeded sample of requests on a server that keeps outputs, and
    compare each output with the plain path's for the same request."""
    dev = master.device
    sh = torch.cuda.current_stream(dev).cuda_stream
    rng = np.random.default_rng(40)
    comp = [k for k, r in enumerate(reqs) if r.op == "compress"]
    deco = [k for k, r in enumerate(reqs) if r.op == "decompress"]
    large = [k for k in comp if reqs[k].n >= 1 << 24][:max(8, sample // 20)]
    rest = [k for k in comp if k not in set(large)]
    pick_c = large + [int(k) for k in rng.choice(rest, size=max(0, sample - len(large)), replace=False)]
    pick_d = [int(k) for k in rng.choice(deco, size=max(1, sample // 3), replace=False)]
    tags = sorted(pick_c + pick_d)
    sub = table[tags].copy()
    # arrivals: Poisson at offered load 0.9 of the plain closed loop
    mean_bytes = float(np.mean([4 * reqs[k].n for k in tags]))
    rate = 0.9 * plain_gbps * 1e9 / mean_bytes
    mismatched = []
    checked = {"compress": 0, "decompress": 0}

    def keep(c):
        k = int(c.tag)
        r = reqs[k]
        if r.op == "compress":
            ref = torch.empty(fsz.fsz_compressed_bound(r.n), dtype=torch.uint8, device=dev)
            check(fsz.fsz_compress_async(master.data_ptr() + 4 * r.offset, r.n, fsz.FSZ_REL, r.rel, None,
                                         ref.data_ptr(), ref.numel(), res[k].data_ptr(), sh), "reference compress")
            size, st, _ = fsz.read_result(res[k])
            check(st, "reference compress")
            got = fsz.device_view(c.d_out, c.size, torch.uint8)
            same = int(size) == int(c.size) and torch.equal(got, ref[:size])
        else:
            ref = torch.empty(r.n, dtype=torch.float32, device=dev)
            check(fsz.fsz_decompress_async(streams[k].data_ptr(), ssize[k], ref.data_ptr(), r.n,
                                           res[k].data_ptr(), sh), "reference decompress")
            got = fsz.device_view(c.d_out, 4 * r.n, torch.float32)
            same = torch.equal(got.view(torch.int32), ref.view(torch.int32))
        torch.cuda.synchronize()
        checked[r.op] += 1
        if not same:
            mismatched.append(k)

    st, server = fsz.fsz_server_create(budget, jobs_per_round, rounds_in_flight, False, (4, 0))
    check(st, "server create")
    try:
        gaps = rng.exponential(1.0 / rate, len(tags))
        gaps[0] = 0.0
        done = {}
        start = fsz.fsz_server_now_ns() + 5_000_000
        sub["arrival_ns"] = start + (np.cumsum(gaps) * 1e9).astype(np.uint64)
        check(fsz.fsz_server_submit_table(server, sub), "submit")
        while len(done) < len(tags):
            for c in fsz.fsz_server_poll(server, 4096, 200):
                if c.status != fsz.FSZ_OK:
                    raise RuntimeError(f"served request {c.tag} failed")
                done[c.tag] = c.size
                keep(c)
                check(fsz.fsz_server_release(server, c.d_out), "release")
        stats = fsz.fsz_server_get_stats(server)
    finally:
        fsz.fsz_server_destroy(server)
    return {
        "sample_compress": len(pick_c),
        "sample_decompress": len(pick_d),
        "compress_at_least_2^24": len(large),
        "largest_n": int(max(reqs[k].n for k in tags)),
        "checked": checked,
        "mismatched": mismatched[:10],
        "identical": not mismatched and sum(checked.values()) == len(tags),
        "mean_jobs_per_round": round(len(tags) / max(int(stats.rounds), 1), 2),
        "max_rounds_overlapping": int(stats.max_rounds_overlapping),
    }


def served_benchmark(args):
    """The served form alone (`--served`): every load point of --served-loads."""
    import torch

    from paper_2607_15413_amd import fsz, workloads

    loads = [float(v) for v in args.served_loads.split(",")]
    counts = [int(v) for v in args.served_requests.split(",")]
    if len(counts) == 1:
        counts = counts * len(loads)
    served = served_run(torch, fsz, workloads, loads, counts, args.served_plain_requests, args.served_budget_gb,
                        args.served_rounds, args.served_jobs_per_round, args.served_timeline,
                        verify_sample=args.served_verify)
    results = served["per_load"]
    top = max((e for e in results if e["offered_load"] <= 0.9), key=lambda e: e["offered_load"],
              default=results[-1])
    line = {
        "metric": "served: sustained GB/s and p50/p99 latency under open-loop Poisson load on 1 MI355X",
        "value": top["sustained_GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": len(results),
        "warmup": 1,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": SERVED_WORKLOAD + f"; HBM budget {args.served_budget_gb} GB, {args.served_rounds} rounds "
                        f"in flight, up to {args.served_jobs_per_round} jobs per round",
            "requests_per_load": counts,
        },
        "served": served,
    }
    print(json.dumps(line), flush=True)


ABLATION_COLUMNS = (("base", 0), ("+cross", 1), ("+cent", 3), ("+lz2 (full)", 7))  # feature masks


def _timed(torch, stream, fn, reps):
    fn()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record(stream)
    for _ in range(reps):
        fn()
    e[1].record(stream)
    torch.cuda.synchronize()
    return e[0].elapsed_time(e[1]) / reps


def ablation_columns(torch, fsz, x, stats, reps: int = 5, reference=None):
    """The ablation's four columns (Sec. VI-B, Table IV: Base = LZ1 on
    independent blocks, +Cross, +Cent, +LZ2 = the full method) on one field:
    CR and compress GB/s (4n / kernel time) per bound.  reference: the
    default path's streams per bound, which the full column must equal."""
    stream = torch.cuda.current_stream(x.device)
    sh = stream.cuda_stream
    n = x.numel()
    cap = fsz.fsz_compressed_bound(n)
    buf = torch.empty(cap, dtype=torch.uint8, device=x.device)
    res = torch.zeros(4, dtype=torch.int32, device=x.device)
    rows = []
    for k, rel in enumerate(RELS):
        row = {"rel": rel}
        for name, f in ABLATION_COLUMNS:
            def run():
                st = fsz.fsz_compress_features_async(x.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(), f,
                                                     buf.data_ptr(), cap, res.data_ptr(), sh)
                if st != fsz.FSZ_OK:
                    raise RuntimeError(fsz.fsz_status_string(st))
            ms = _timed(torch, stream, run, reps)
            size, st, _ = fsz.read_result(res)
            if st != fsz.FSZ_OK:
                raise RuntimeError(f"ablation {name} rel={rel}: {fsz.fsz_status_string(st)}")
            row[name] = {"cr": round(4 * n / size, 4), "compress_GBps": round(4 * n / ms / 1e6, 1)}
            if f == fsz.FSZ_FEATURES_ALL and reference is not None:
                ref = reference[k]
                row[name]["identical_to_default"] = bool(size == ref.numel() and torch.equal(buf[:size], ref))
        rows.append(row)
    del buf
    return rows


def five_read_comparison(torch, fsz, x, stats, outs, sizes, reps: int = 5):
    """The single pass against the naive five-read evaluation (Sec. V-C,
    Fig. 6) on the timed field; the streams must be byte-identical."""
    stream = torch.cuda.current_stream(x.device)
    sh = stream.cuda_stream
    n = x.numel()
    cap = fsz.fsz_compressed_bound(n)
    buf = torch.empty(cap, dtype=torch.uint8, device=x.device)
    res = torch.zeros(4, dtype=torch.int32, device=x.device)
    rows = []
    for k, rel in enumerate(RELS):
        def five():
            st = fsz.fsz_compress_five_read_async(x.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(),
                                                  buf.data_ptr(), cap, res.data_ptr(), sh)
            if st != fsz.FSZ_OK:
                raise RuntimeError(fsz.fsz_status_string(st))
        f_ms = _timed(torch, stream, five, reps)
        size, st, _ = fsz.read_result(res)
        if st != fsz.FSZ_OK:
            raise RuntimeError(f"five-read rel={rel}: {fsz.fsz_status_string(st)}")

        def single():
            st = fsz.fsz_compress_async(x.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(), outs[k].data_ptr(),
                                        cap, res.data_ptr(), sh)
            if st != fsz.FSZ_OK:
                raise RuntimeError(fsz.fsz_status_string(st))
        s_ms = _timed(torch, stream, single, reps)
        rows.append({"rel": rel, "single_pass_ms": round(s_ms, 4), "five_read_ms": round(f_ms, 4),
                     "speedup": round(f_ms / s_ms, 2),
                     "identical": bool(size == sizes[k] and torch.equal(buf[:size], outs[k][:size]))})
    del buf
    return rows


def random_access(torch, fsz, outs, sizes, n, full_ms, reps: int = 20):
    """Random-access decode (rate-header prefix + the range's tiles) of ranges
    in the middle of the REL 1e-3 stream, against the whole-field decode."""
    dev = outs[0].device
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    k = 1
    res = torch.zeros(4, dtype=torch.int32, device=dev)
    rows = []
    for m in (256, 1 << 18, n // 10):
        begin = n // 2 - m // 2
        y = torch.empty(m, dtype=torch.float32, device=dev)

        def run():
            st = fsz.fsz_decompress_range_async(outs[k].data_ptr(), sizes[k], n, begin, begin + m, y.data_ptr(),
                                                res.data_ptr(), sh)
            if st != fsz.FSZ_OK:
                raise RuntimeError(fsz.fsz_status_string(st))
        ms = _timed(torch, stream, run, reps)
        _, st, _ = fsz.read_result(res)
        if st != fsz.FSZ_OK:
            raise RuntimeError(f"range decode: {fsz.fsz_status_string(st)}")
        rows.append({"elements": m, "begin": begin, "ms": round(ms, 4), "whole_field_ms": round(full_ms, 4)})
        del y
    return {"rel": RELS[k], "ranges": rows}


def ablation_benchmark(torch, fsz, workloads, x, stats, outs, sizes):
    """Ablation columns on the timed k^-3 field and on the 100x500x500
    piecewise-quadratic field (offsets, zero boxes and quadratic trends), plus
    the five-read comparison on the timed field."""
    grf = ablation_columns(torch, fsz, x, stats, reference=[outs[k][:sizes[k]] for k in range(len(RELS))])
    t0 = time.time()
    p_np = workloads.piecewise_quadratic((100, 500, 500), 2)
    print(f"[bench] generated piecewise quadratic in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    p = torch.from_numpy(p_np).to(x.device)
    pstats = torch.zeros(4, dtype=torch.int32, device=x.device)
    st = fsz.fsz_field_stats(p.data_ptr(), p.numel(), pstats.data_ptr(), torch.cuda.current_stream(x.device).cuda_stream)
    if st != fsz.FSZ_OK:
        raise RuntimeError(fsz.fsz_status_string(st))
    pwq = ablation_columns(torch, fsz, p, pstats)
    five = five_read_comparison(torch, fsz, x, stats, outs, sizes)
    return {"grf 512^3": grf, "piecewise quadratic 100x500x500": pwq}, five


TILE_CONFIGS = ((32, 4), (32, 8), (32, 16), (64, 4), (64, 8), (64, 16))  # (B, T); the paper sweeps all but 64/16


def tile_sweep(torch, fsz, workloads, x, stats, outs, sizes, reps: int = 5):
    """The tile-configuration sweep (Sec. VI-C, Table V, Fig. 10): block size B
    and blocks per tile T.  On the timed field: CR and compress / decompress
    GB/s (4n / kernel time) of every configuration through the generic
    configuration kernels, the 32 / 8 stream checked against the default
    path's.  On a set of synthetic fields x 3 bounds: per configuration the
    tests won / tied / lost against 32 / 8 (win = CR more than 2% higher) and
    the mean CR ratio, as Table V counts them."""
    dev = x.device
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    n = x.numel()
    cap = max(fsz.fsz_compressed_bound_config(n, B, T) for B, T in TILE_CONFIGS)
    buf = torch.empty(cap, dtype=torch.uint8, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    res = torch.zeros(4, dtype=torch.int32, device=dev)

    def compress_cfg(xt, st_t, rel, B, T):
        st = fsz.fsz_compress_config_async(xt.data_ptr(), xt.numel(), fsz.FSZ_REL, rel, st_t.data_ptr(), B, T,
                                           buf.data_ptr(), cap, res.data_ptr(), sh)
        if st != fsz.FSZ_OK:
            raise RuntimeError(fsz.fsz_status_string(st))

    rows = []
    identical = True
    for k, rel in enumerate(RELS):
        for B, T in TILE_CONFIGS:
            c_ms = _timed(torch, stream, lambda: compress_cfg(x, stats, rel, B, T), reps)
            size, st, _ = fsz.read_result(res)
            if st != fsz.FSZ_OK:
                raise RuntimeError(f"tile sweep B={B} T={T} rel={rel}: {fsz.fsz_status_string(st)}")
            if (B, T) == (32, 8):
                identical = identical and size == sizes[k] and torch.equal(buf[:size], outs[k][:size])

            def dec():
                st = fsz.fsz_decompress_config_async(buf.data_ptr(), size, y.data_ptr(), n, B, T, res.data_ptr(), sh)
                if st != fsz.FSZ_OK:
                    raise RuntimeError(fsz.fsz_status_string(st))
            d_ms = _timed(torch, stream, dec, reps)
            _, st, _ = fsz.read_result(res)
            if st != fsz.FSZ_OK:
                raise RuntimeError(f"tile sweep decode B={B} T={T} rel={rel}: {fsz.fsz_status_string(st)}")
            rows.append({"B": B, "T": T, "rel": rel, "cr": round(4 * n / size, 4),
                         "compress_GBps": round(4 * n / c_ms / 1e6, 1),
                         "decompress_GBps": round(4 * n / d_ms / 1e6, 1)})
    del y

    # win / tie / loss against 32 / 8 over synthetic fields x bounds
    fields = [("grf k^-3 512^3 (timed field)", None),
              ("grf k^-2 256^3", lambda: workloads.grf_field((256, 256, 256), 11, slope=-2.0)),
              ("grf k^-4 256^3", lambda: workloads.grf_field((256, 256, 256), 12, slope=-4.0)),
              ("piecewise quadratic 100x500x500", lambda: workloads.piecewise_quadratic((100, 500, 500), 2)),
              ("sinusoid 2^24", lambda: workloads.sinusoid_field(1 << 24, 5)),
              ("sinusoid 2^22 noise-free", lambda: workloads.sinusoid_field(1 << 22, 6, noise_sigma=0.0))]
    crs = {}  # (field, rel) -> {(B, T): cr}
    for name, gen in fields:
        if gen is None:
            xt, st_t = x, stats
        else:
            xt = torch.from_numpy(gen()).to(dev)
            st_t = torch.zeros(4, dtype=torch.int32, device=dev)
            st = fsz.fsz_field_stats(xt.data_ptr(), xt.numel(), st_t.data_ptr(), sh)
            if st != fsz.FSZ_OK:
                raise RuntimeError(fsz.fsz_status_string(st))
        for rel in RELS:
            for B, T in TILE_CONFIGS:
                compress_cfg(xt, st_t, rel, B, T)
                size, st, _ = fsz.read_result(res)
                if st != fsz.FSZ_OK:
                    raise RuntimeError(f"tile sweep {name} B={B} T={T}: {fsz.fsz_status_string(st)}")
                crs.setdefault((name, rel), {})[(B, T)] = 4 * xt.numel() / size
        del xt
    table = []
    for B, T in TILE_CONFIGS:
        if (B, T) == (32, 8):
            continue
        ratios = [c[(B, T)] / c[(32, 8)] for c in crs.values()]
        table.append({"B": B, "T": T, "tile": B * T, "win": sum(r > 1.02 for r in ratios),
                      "tie": sum(0.98 <= r <= 1.02 for r in ratios), "loss": sum(r < 0.98 for r in ratios),
                      "cr_ratio": round(float(np.mean(ratios)), 4)})
    del buf
    return {"timed_field": rows, "default_identical": bool(identical), "vs_default": table,
            "tests": len(crs), "fields": [f for f, _ in fields]}


def small_configs(torch, fsz, workloads, verify: bool, reps: int = 20):
    """The 2^20 sinusoid field (REL 1e-3; warm and MALL-flushed) and the
    100x500x500 piecewise-quadratic field (REL 1e-2/1e-3/1e-4; flushed: a
    1 GiB buffer is read before every timed call, so the MALL holds clean
    lines of it and nothing of the field, since both fields fit in the
    256 MB MALL).  Median of `reps` calls per row, HIP events around each
    asynchronous call (range pass precomputed)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB, read (not written) to flush
    rows = []
    cases = [("sinusoid 2^20, seed 0", workloads.sinusoid_field(1 << 20, 0), [1e-3], [False, True]),
             ("piecewise quadratic 100x500x500, seed 2", workloads.piecewise_quadratic((100, 500, 500), 2),
              [1e-2, 1e-3, 1e-4], [True])]
    for name, x_np, rels, modes in cases:
        n = x_np.size
        x = torch.from_numpy(x_np).to(dev)
        cap = fsz.fsz_compressed_bound(n)
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
        y = torch.empty(n, dtype=torch.float32, device=dev)
        stats = fsz.field_stats(x)
        res = torch.zeros(4, dtype=torch.int32, device=dev)
        st_np = stats.cpu().numpy().view(np.float32)
        span = float(st_np[1]) - float(st_np[0])
        for rel in rels:
            for flushed in modes:
                def timed(fn):
                    ts = []
                    for it in range(reps + 3):
                        if flushed:
                            flush.sum()
                        a = torch.cuda.Event(enable_timing=True)
                        b = torch.cuda.Event(enable_timing=True)
                        a.record(stream)
                        fn()
                        b.record(stream)
                        torch.cuda.synchronize()
                        if it >= 3:
                            ts.append(a.elapsed_time(b))
                    return float(np.median(ts))
                c_ms = timed(lambda: fsz.fsz_compress_async(x.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(),
                                                            out.data_ptr(), cap, res.data_ptr(), sh))
                size, st, _ = fsz.read_result(res)
                if st != fsz.FSZ_OK:
                    raise RuntimeError(f"{name}: {fsz.fsz_status_string(st)}")
                d_ms = timed(lambda: fsz.fsz_decompress_async(out.data_ptr(), size, y.data_ptr(), n,
                                                              res.data_ptr(), sh))
                _, st, _ = fsz.read_result(res)
                if st != fsz.FSZ_OK:
                    raise RuntimeError(f"{name}: {fsz.fsz_status_string(st)}")
                eb = rel * span
                err = float((x.double() - y.double()).abs().max().item()) / eb
                identical = None
                if verify:
                    import oracle
                    identical = out[:size].cpu().numpy().tobytes() == oracle.compress(x_np, oracle.REL, rel)
                alg = 4 * n + size
                rows.append({
                    "config": name, "rel": rel, "flushed": flushed, "cr": round(4 * n / size, 4),
                    "compress_GBps": round(4 * n / c_ms / 1e6, 1), "decompress_GBps": round(4 * n / d_ms / 1e6, 1),
                    "compress_hbm_frac": round(alg / c_ms / 1e6 / HBM_PEAK_GBPS, 4),
                    "decompress_hbm_frac": round(alg / d_ms / 1e6 / HBM_PEAK_GBPS, 4),
                    "compress_ms": round(c_ms, 4), "decompress_ms": round(d_ms, 4),
                    "max_err_over_eb": round(err, 6), "oracle_identical": identical,
                })
        del x, out, y
    del flush
    return rows


def prezero_rows(torch, fsz, workloads, x, outs, sizes, reps: int = 10):
    """Pre-zeroed decompression (Sec. III-A) against the plain decoder: on a
    512^3 sparse field (one U[-50,50] spike per 20000 zeros, REL 1e-3, CR
    near the format's cap) and on the timed field's REL 1e-2 stream.  Each
    decode is timed alone after a 1 GiB read refilled the MALL; the outputs
    must agree bit for bit."""
    dev = x.device
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    n = x.numel()
    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    res = torch.zeros(4, dtype=torch.int32, device=dev)
    sp = torch.from_numpy(workloads.sparse_field(n, 5)).to(dev)
    cap = fsz.fsz_compressed_bound(n)
    sbuf = torch.empty(cap, dtype=torch.uint8, device=dev)
    st = fsz.fsz_compress_async(sp.data_ptr(), n, fsz.FSZ_REL, 1e-3, None, sbuf.data_ptr(), cap, res.data_ptr(), sh)
    if st != fsz.FSZ_OK:
        raise RuntimeError("sparse compress failed")
    ssize, st, _ = fsz.read_result(res)
    del sp
    ya = torch.empty(n, dtype=torch.float32, device=dev)
    yb = torch.empty(n, dtype=torch.float32, device=dev)
    rows = []
    for name, buf, size in (("sparse 512^3, 1 spike per 20000, REL 1e-3", sbuf, int(ssize)),
                            ("grf k^-3 512^3, REL 1e-2", outs[0], sizes[0])):
        times = {}
        for label, entry, dst in (("plain", fsz.fsz_decompress_async, ya),
                                  ("prezero", fsz.fsz_decompress_prezero_async, yb)):
            t = []
            for _ in range(reps):
                flush.sum()
                e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                e[0].record(stream)
                st = entry(buf.data_ptr(), size, dst.data_ptr(), n, res.data_ptr(), sh)
                e[1].record(stream)
                torch.cuda.synchronize()
                if st != fsz.FSZ_OK or fsz.read_result(res)[1] != fsz.FSZ_OK:
                    raise RuntimeError(f"{label} decode failed")
                t.append(e[0].elapsed_time(e[1]))
            times[label] = float(np.median(t))
        alg = 4 * n + size
        rows.append({
            "field": name, "cr": round(4 * n / size, 2),
            "plain_ms": round(times["plain"], 4), "prezero_ms": round(times["prezero"], 4),
            "plain_hbm_frac": round(alg / times["plain"] / 1e6 / HBM_PEAK_GBPS, 4),
            "prezero_hbm_frac": round(alg / times["prezero"] / 1e6 / HBM_PEAK_GBPS, 4),
            "identical": bool(torch.equal(ya.view(torch.int32), yb.view(torch.int32))),
        })
    del flush, sbuf, ya, yb
    torch.cuda.empty_cache()
    return rows


def host_threads() -> int:
    """Host threads for the oracle's parallel mode: the CPUs this process may
    run on, at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def host_description() -> str:
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible, {host_threads()} used"


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--shape", type=str, default="512,512,512",
                    help="GRF shape (default: the 512^3 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true", help="skip the byte comparison with the oracle")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-form comparison on the 64-field workload and the two small "
                         "configurations (2^20 sinusoid, 100x500x500 piecewise quadratic)")
    ap.add_argument("--batched-reps", type=int, default=10)
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the ablation columns and the five-read comparison")
    ap.add_argument("--served", action="store_true",
                    help="run the served request-loop workload instead of the default one")
    ap.add_argument("--served-loads", type=str, default="0.1,0.3,0.5,0.7,0.9,1.2,1.5")
    ap.add_argument("--served-requests", type=str, default="10000",
                    help="requests per load point (one value for all, or one per load)")
    ap.add_argument("--served-plain-requests", type=int, default=10000)
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    ap.add_argument("--served-rounds", type=int, default=4)
    ap.add_argument("--served-jobs-per-round", type=int, default=256)
    ap.add_argument("--served-timeline", type=str, default=None,
                    help="write per-request times (arrival, admit, launch, complete; ns) per load to this .npz")
    ap.add_argument("--served-verify", type=int, default=200,
                    help="compress requests of the served byte comparison against the plain path (0: none)")
    ap.add_argument("--no-served", action="store_true",
                    help="skip the served section of the default line (offered loads 0.1 / 0.5 / 0.9)")
    ap.add_argument("--only-small", action="store_true",
                    help="time only the small configurations (2^20 sinusoid, 100x500x500 piecewise "
                         "quadratic) and print their rows; for kernel traces of those calls")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run one plain device copy of the input (n floats) so that "
                         "profiler counters can be calibrated against a kernel of known traffic")
    return ap.parse_args()


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "sharding across GPUs is a design only, never launched.",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.served:
        served_benchmark(args)
        return
    if args.only_small:
        import torch

        from paper_2607_15413_amd import fsz, workloads
        torch.cuda.set_device(torch.device("cuda:0"))
        print(json.dumps({"other_configs": small_configs(torch, fsz, workloads, not args.no_verify)}), flush=True)
        return

    import torch

    from paper_2607_15413_amd import fsz, workloads

    shape = tuple(int(s) for s in args.shape.split(","))
    t0 = time.time()
    x_np = workloads.grf_field(shape, 1)
    n = x_np.size
    print(f"[bench] generated grf {shape} n={n} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    sh = stream.cuda_stream
    x = torch.from_numpy(x_np).to(dev)
    cap = fsz.fsz_compressed_bound(n)
    outs = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in RELS]
    y = torch.empty(n, dtype=torch.float32, device=dev)
    stats = torch.zeros(4, dtype=torch.int32, device=dev)
    cres = [torch.zeros(4, dtype=torch.int32, device=dev) for _ in RELS]
    dres = [torch.zeros(4, dtype=torch.int32, device=dev) for _ in RELS]

    def check(st, what):
        if st != fsz.FSZ_OK:
            raise RuntimeError(f"{what}: {fsz.fsz_status_string(st)}")

    def step(events=None, stats_events=None):
        if stats_events is not None:
            stats_events[0].record(stream)
        check(fsz.fsz_field_stats(x.data_ptr(), n, stats.data_ptr(), sh), "stats")
        if stats_events is not None:
            stats_events[1].record(stream)
        for k, rel in enumerate(RELS):
            if events is not None:
                events[k][0].record(stream)
            check(fsz.fsz_compress_async(x.data_ptr(), n, fsz.FSZ_REL, rel, stats.data_ptr(),
                                         outs[k].data_ptr(), cap, cres[k].data_ptr(), sh), "compress")
            if events is not None:
                events[k][1].record(stream)
                events[k][2].record(stream)
            check(fsz.fsz_decompress_async(outs[k].data_ptr(), cap, y.data_ptr(), n,
                                           dres[k].data_ptr(), sh), "decompress")
            if events is not None:
                events[k][3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in RELS]
          for _ in range(args.steps)]
    sev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for s in range(args.steps):
        step(ev[s], sev[s])
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    stats_ms = float(np.mean([sev[s][0].elapsed_time(sev[s][1]) for s in range(args.steps)]))
    if args.copy_probe:
        y.copy_(x)  # n floats read + n floats written: the counter calibration kernel
        torch.cuda.synchronize()
    # practical ceiling: a plain device-to-device copy of the field (4n read + 4n written)
    ca = torch.cuda.Event(enable_timing=True)
    cb = torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    ca.record(stream)
    for _ in range(10):
        y.copy_(x)
    cb.record(stream)
    torch.cuda.synchronize()
    copy_GBps = 10 * 8 * n / ca.elapsed_time(cb) / 1e6

    comp_ms = [np.mean([ev[s][k][0].elapsed_time(ev[s][k][1]) for s in range(args.steps)])
               for k in range(len(RELS))]
    dec_ms = [np.mean([ev[s][k][2].elapsed_time(ev[s][k][3]) for s in range(args.steps)])
              for k in range(len(RELS))]
    sizes = []
    for k in range(len(RELS)):
        size, st, _ = fsz.read_result(cres[k])
        check(st, f"compress result rel={RELS[k]}")
        _, st, _ = fsz.read_result(dres[k])
        check(st, f"decompress result rel={RELS[k]}")
        sizes.append(int(size))

    # cold decompress: the 256 MB MALL refilled by a read of a 1 GiB buffer
    # (clean lines, nothing to write back) before each timed call, so the
    # stream is read from HBM (in the step, decompression follows the
    # compression that wrote the stream, which may still be cached)
    flush = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dec_cold_ms = []
    for k in range(len(RELS)):
        t = []
        for _ in range(3):
            flush.sum()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record(stream)
            check(fsz.fsz_decompress_async(outs[k].data_ptr(), sizes[k], y.data_ptr(), n, dres[k].data_ptr(), sh),
                  "decompress")
            e[1].record(stream)
            torch.cuda.synchronize()
            t.append(e[0].elapsed_time(e[1]))
        dec_cold_ms.append(float(np.median(t)))
    del flush

    # pointwise error of every bound's reconstruction, relative to eb
    st_np = stats.cpu().numpy().view(np.float32)
    span = float(st_np[1]) - float(st_np[0])
    max_err = []
    for k, rel in enumerate(RELS):
        check(fsz.fsz_decompress(outs[k].data_ptr(), sizes[k], y.data_ptr(), n, sh), "decompress")
        max_err.append(float((x.double() - y.double()).abs().max().item()) / (rel * span))

    per_bound = []
    comp_bytes = dec_bytes = 0
    comp_time = dec_time = 0.0
    for k, rel in enumerate(RELS):
        alg = 4 * n + sizes[k]  # bytes read + written by either direction
        per_bound.append({
            "max_err_over_eb": round(max_err[k], 6),
            "rel": rel,
            "cr": round(4 * n / sizes[k], 4),
            "stream_bytes": sizes[k],
            "compress_GBps": round(4 * n / comp_ms[k] / 1e6, 1),
            "decompress_GBps": round(4 * n / dec_ms[k] / 1e6, 1),
            "compress_ms": round(comp_ms[k], 4),
            "decompress_ms": round(dec_ms[k], 4),
            "compress_hbm_frac": round(alg / comp_ms[k] / 1e6 / HBM_PEAK_GBPS, 4),
            "decompress_hbm_frac": round(alg / dec_ms[k] / 1e6 / HBM_PEAK_GBPS, 4),
            "decompress_cold_ms": round(dec_cold_ms[k], 4),
            "decompress_cold_GBps": round(4 * n / dec_cold_ms[k] / 1e6, 1),
        })
        comp_bytes += alg
        dec_bytes += alg
        comp_time += comp_ms[k]
        dec_time += dec_ms[k]

    dominant = "compress" if comp_time >= dec_time else "decompress"
    # kernel names as rocprofv3 reports them (torch allocations are 16-byte aligned)
    waves = os.environ.get("FSZ_PIPE_WAVES", "9")
    if os.environ.get("FSZ_PIPE", "1") == "0":
        comp_kernel = "compress_kernel"
    elif waves in ("7", "9"):
        comp_kernel = "compress_ctrl_kernel"
    else:
        comp_kernel = "compress_pipe2_kernel"
    dom_kernel = comp_kernel if dominant == "compress" else "decompress_kernel"
    dom_bytes, dom_time = (comp_bytes, comp_time) if dominant == "compress" else (dec_bytes, dec_time)
    achieved = dom_bytes / dom_time / 1e6  # GB/s
    roofline = {
        "bound": "hbm",
        "kernel": dom_kernel,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBPS, 4),
        "traffic": measured_traffic(dom_kernel),
        "avg_launch_ms": round(dom_time / len(RELS), 4),
        "bytes_per_launch": int(dom_bytes / len(RELS)),
    }

    value = 2 * len(RELS) * 4 * n / (ms_per_step / 1e3) / 1e9

    verified = None
    cpu = None
    if not args.no_cpu_baseline or not args.no_verify:
        import oracle

        threads = host_threads()

        def oracle_pass(nthreads, x_part):
            """One compress + one decompress of x_part per bound on nthreads host
            threads; returns (compress s, decompress s, streams)."""
            old = oracle.set_threads(nthreads)
            try:
                t_c = t_d = 0.0
                refs = []
                for rel in RELS:
                    t = time.perf_counter()
                    ref = oracle.compress(x_part, oracle.REL, rel)
                    t_c += time.perf_counter() - t
                    t = time.perf_counter()
                    oracle.decompress(ref, x_part.size)
                    t_d += time.perf_counter() - t
                    refs.append(ref)
                return t_c, t_d, refs
            finally:
                oracle.set_threads(old)

        # the whole field on every host thread: the parallel CPU baseline, and
        # the streams the GPU's are compared with (bytes do not depend on threads)
        t_c, t_d, refs = oracle_pass(threads, x_np)
        if not args.no_verify:
            verified = all(outs[k][:sizes[k]].cpu().numpy().tobytes() == refs[k] for k in range(len(RELS)))
        del refs
        if not args.no_cpu_baseline:
            # single thread on a bounded sample: the first 2^25 elements (a quarter of the field)
            part = x_np[:min(n, 1 << 25)]
            s_c, s_d, _ = oracle_pass(1, part)
            cpu = {
                "value": round(2 * len(RELS) * 4 * n / (t_c + t_d) / 1e9, 4),
                "unit": "GB/s",
                "cores": threads,
                "kind": "oracle",
                "sample": f"full {shape} field, REL 1e-2/1e-3/1e-4, one compress + one decompress each "
                          f"on {threads} host threads (tile loops in parallel, offset scan serial; "
                          f"{t_c:.1f}s + {t_d:.1f}s); single thread on its first {part.size} elements",
                "compress_GBps": round(len(RELS) * 4 * n / t_c / 1e9, 4),
                "decompress_GBps": round(len(RELS) * 4 * n / t_d / 1e9, 4),
                "single_thread_GBps": round(2 * len(RELS) * 4 * part.size / (s_c + s_d) / 1e9, 4),
                "single_thread_compress_GBps": round(len(RELS) * 4 * part.size / s_c / 1e9, 4),
                "single_thread_decompress_GBps": round(len(RELS) * 4 * part.size / s_d / 1e9, 4),
                "host": host_description(),
            }

    pre_zero = prezero_rows(torch, fsz, workloads, x, outs, sizes)

    ablation = five_read = ranges = sweep = None
    if not args.no_ablation:
        ablation, five_read = ablation_benchmark(torch, fsz, workloads, x, stats, outs, sizes)
        ranges = random_access(torch, fsz, outs, sizes, n, dec_ms[1])
        sweep = tile_sweep(torch, fsz, workloads, x, stats, outs, sizes)
    others = None
    if not args.no_batched:
        others = small_configs(torch, fsz, workloads, not args.no_verify)
    batched = None
    if not args.no_batched:
        del outs, y  # room for the 64-field workload
        torch.cuda.empty_cache()
        batched = batched_comparison(torch, fsz, workloads, args.batched_reps, not args.no_verify)
    served = None
    if not args.no_served:
        # the served workload (10,000 Poisson requests per load) at three offered loads
        x = outs = y = None
        torch.cuda.empty_cache()
        served = served_run(torch, fsz, workloads, [0.1, 0.5, 0.9], [10000] * 3, 10000, args.served_budget_gb,
                            args.served_rounds, args.served_jobs_per_round,
                            verify_sample=0 if args.no_verify else args.served_verify)

    line = {
        "metric": "compress/decompress GB/s on 1 MI355X (% of HBM peak) + compression ratio",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "grf-k^-3 512x512x512 float32 (512 MiB), seed 1, REL 1e-2/1e-3/1e-4; "
                        "per step: range pass + 3 x (compress + decompress)",
            "n": n,
            "shape": list(shape),
            "rel_bounds": list(RELS),
        },
        "compress_GBps": round(len(RELS) * 4 * n / comp_time / 1e6, 1),
        "decompress_GBps": round(len(RELS) * 4 * n / dec_time / 1e6, 1),
        "range_pass_ms": round(stats_ms, 4),
        "compress_end_to_end_GBps": round(len(RELS) * 4 * n / (comp_time + len(RELS) * stats_ms) / 1e6, 1),
        # the range pass reads the field once more: 8 n + stream bytes per call
        "compress_end_to_end_hbm_frac": round(sum(8 * n + sizes[k] for k in range(len(RELS))) /
                                              (comp_time + len(RELS) * stats_ms) / 1e6 / HBM_PEAK_GBPS, 4),
        "per_bound": per_bound,
        "copy_ceiling_GBps": round(copy_GBps, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "oracle_identical": verified,
        "ablation": ablation,
        "five_read": five_read,
        "pre_zero": pre_zero,
        "random_access": ranges,
        "tile_sweep": sweep,
        "batched": batched,
        "other_configs": others,
        "served": served,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
