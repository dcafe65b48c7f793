// C ABI of libfsz.so: argument validation, per-(device, stream) workspace,
// kernel launches and the single device->host status read per call.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <utility>

#include "fsz_internal.h"

using namespace fsz;

namespace fsz {
const Tuning &tuning()
{
    static const Tuning t = [] {
        Tuning v;
        if (const char *e = std::getenv("FSZ_STAGED")) {  // letters: c = compress, d = decompress
            v.staged_compress = std::strchr(e, 'c') != nullptr;
            v.staged_decompress = std::strchr(e, 'd') != nullptr;
            v.staged_compress_loads = std::strchr(e, 'l') != nullptr;
        }
        if (const char *e = std::getenv("FSZ_GRID_FACTOR")) {
            const int f = std::atoi(e);
            if (f >= 1 && f <= 64) v.grid_factor = f;
        }
        return v;
    }();
    return t;
}
}  // namespace fsz

namespace {

struct Workspace {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    unsigned long long *d_flags = nullptr;  // chunk flag words
    uint64_t flags_cap = 0;
    unsigned long long *d_ticket = nullptr;  // chunk ticket, reset by each launch's last taker
    uint32_t call = 0;                       // per-call epoch
    fsz_result *d_final = nullptr;           // outcome of blocking calls
    fsz_result *h_final = nullptr;           // pinned host copy
    fsz_stats *d_stats = nullptr;            // range pass output when the caller has none
    StatsPartial *d_partials = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;

bool ok(hipError_t e) { return e == hipSuccess; }


Workspace *get_workspace(hipStream_t s, fsz_status *st)
{
    int dev = 0;
    if (!ok(hipGetDevice(&dev))) {
        *st = FSZ_ERR_DEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> g(g_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) return it->second.get();
    auto ws = std::make_unique<Workspace>();
    ws->device = dev;
    ws->stream = s;
    bool good = ok(hipMalloc(&ws->d_ticket, sizeof(unsigned long long))) &&
                ok(hipMalloc(&ws->d_final, sizeof(fsz_result))) &&
                ok(hipHostMalloc(&ws->h_final, sizeof(fsz_result), hipHostMallocDefault)) &&
                ok(hipMalloc(&ws->d_stats, sizeof(fsz_stats))) &&
                ok(hipMalloc(&ws->d_partials, sizeof(StatsPartial) * kStatsMaxBlocks)) &&
                ok(hipMemset(ws->d_ticket, 0, sizeof(unsigned long long))) &&
                ok(hipMemset(ws->d_final, 0, sizeof(fsz_result))) &&
                ok(hipDeviceSynchronize());
    if (!good) {
        *st = FSZ_ERR_DEVICE;
        return nullptr;
    }
    Workspace *raw = ws.get();
    g_ws.emplace(key, std::move(ws));
    return raw;
}

// Make room for nchunks flag words.  Growing waits for the stream, since an
// earlier launch may still use the old array.
bool ensure_flags(Workspace *ws, uint64_t nchunks)
{
    if (nchunks <= ws->flags_cap) return true;
    uint64_t cap = ws->flags_cap ? ws->flags_cap : 1024;
    while (cap < nchunks) cap *= 2;
    if (ws->d_flags) {
        if (!ok(hipStreamSynchronize(ws->stream))) return false;
        if (!ok(hipFree(ws->d_flags))) return false;
        ws->d_flags = nullptr;
        ws->flags_cap = 0;
    }
    if (!ok(hipMalloc(&ws->d_flags, cap * sizeof(unsigned long long)))) return false;
    if (!ok(hipMemsetAsync(ws->d_flags, 0, cap * sizeof(unsigned long long), ws->stream))) return false;
    ws->flags_cap = cap;
    return true;
}

// Next call epoch; clears the flag array whenever the 18-bit flag epoch wraps.
bool next_epoch(Workspace *ws, uint32_t *epoch, uint32_t *flag_epoch)
{
    if (++ws->call == 0) ++ws->call;
    *epoch = ws->call;
    *flag_epoch = (ws->call - 1) % kEpochMask + 1;
    if (*flag_epoch == 1 && ws->call > 1 && ws->d_flags)
        return ok(hipMemsetAsync(ws->d_flags, 0, ws->flags_cap * sizeof(unsigned long long), ws->stream));
    return true;
}

// Blocking calls: copy the outcome back and wait for the stream.
fsz_status finish(Workspace *ws, uint32_t epoch, size_t *size_out)
{
    if (!ok(hipMemcpyAsync(ws->h_final, ws->d_final, sizeof(fsz_result), hipMemcpyDeviceToHost, ws->stream)))
        return FSZ_ERR_DEVICE;
    if (!ok(hipStreamSynchronize(ws->stream))) return FSZ_ERR_DEVICE;
    const fsz_result r = *ws->h_final;
    if (r.epoch != epoch) return FSZ_ERR_DEVICE;
    if (r.status == FSZ_OK && size_out) *size_out = (size_t)r.size;
    return (fsz_status)r.status;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

bool valid_bound(int mode, double value)
{
    return (mode == FSZ_ABS || mode == FSZ_REL) && std::isfinite(value) && value > 0.0;
}

fsz_status check_compress_args(const float *d_in, size_t n, int mode, double value, const void *d_out,
                               size_t cap)
{
    if (!valid_bound(mode, value) || !d_out || (n > 0 && !d_in) || !aligned(d_in, 4) || !aligned(d_out, 4))
        return FSZ_ERR_INVALID_ARG;
    if (cap < kHeaderBytes + pad16(ceil_div(n, kBlock))) return FSZ_ERR_CAPACITY;
    return FSZ_OK;
}

fsz_status check_decompress_args(const void *d_cmp, size_t cmp_size, const float *d_out, size_t n)
{
    if (!d_cmp || (n > 0 && !d_out) || !aligned(d_cmp, 4) || !aligned(d_out, 4)) return FSZ_ERR_INVALID_ARG;
    if (cmp_size < (size_t)kHeaderBytes) return FSZ_ERR_CORRUPT;
    return FSZ_OK;
}

// Enqueue (range pass if d_stats is NULL) + compression kernel.
fsz_status enqueue_compress(Workspace *ws, const float *d_in, uint64_t n, int mode, double value,
                            const fsz_stats *d_stats, void *d_out, uint64_t cap, fsz_result *d_final,
                            uint32_t *epoch_out)
{
    if (!d_stats) {
        StatsArgs sa{d_in, n, ws->d_stats, ws->d_partials};
        if (!ok(launch_stats(sa, ws->stream))) return FSZ_ERR_DEVICE;
        d_stats = ws->d_stats;
    }
    CompressArgs a{};
    a.x = d_in;
    a.n = n;
    a.ntiles = ceil_div(n, kTile);
    a.nblocks = ceil_div(n, kBlock);
    a.nchunks = a.ntiles ? ceil_div(a.ntiles, kTilesPerChunk) : 1;
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    a.out = static_cast<uint8_t *>(d_out);
    a.capacity = cap;
    a.stats = d_stats;
    a.value = value;
    a.mode = mode;
    if (!ensure_flags(ws, a.nchunks)) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    if (!ok(launch_compress(a, aligned(d_in, 16), tuning().staged_compress, ws->stream))) return FSZ_ERR_DEVICE;
    *epoch_out = a.epoch;
    return FSZ_OK;
}

fsz_status enqueue_decompress(Workspace *ws, const void *d_cmp, uint64_t cmp_size, float *d_out, uint64_t n,
                              fsz_result *d_final, uint32_t *epoch_out)
{
    DecompressArgs a{};
    a.cmp = static_cast<const uint8_t *>(d_cmp);
    a.cmp_size = cmp_size;
    a.out = d_out;
    a.n = n;
    a.ntiles = ceil_div(n, kTile);
    a.nblocks = ceil_div(n, kBlock);
    a.nchunks = a.ntiles ? ceil_div(a.ntiles, kTilesPerChunk) : 1;
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    if (!ensure_flags(ws, a.nchunks)) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    if (!ok(launch_decompress(a, aligned(d_out, 16), tuning().staged_decompress, ws->stream))) return FSZ_ERR_DEVICE;
    *epoch_out = a.epoch;
    return FSZ_OK;
}

}  // namespace

extern "C" {

size_t fsz_compressed_bound(size_t n)
{
    const uint64_t nblocks = ceil_div(n, kBlock);
    const uint64_t ntiles = ceil_div(n, kTile);
    return (size_t)(kHeaderBytes + pad16(nblocks) + 4 * ntiles + (4 + 4 * 31) * nblocks);
}

const char *fsz_status_string(int s)
{
    switch (s) {
    case FSZ_OK: return "ok";
    case FSZ_ERR_INVALID_ARG: return "invalid argument";
    case FSZ_ERR_NONFINITE: return "input holds NaN or Inf";
    case FSZ_ERR_EB_TOO_SMALL: return "error bound below 8 ulp of max|x|";
    case FSZ_ERR_CAPACITY: return "output capacity too small";
    case FSZ_ERR_CORRUPT: return "corrupt stream";
    case FSZ_ERR_SIZE_MISMATCH: return "element count differs from the stream";
    case FSZ_ERR_DEVICE: return "HIP runtime error";
    case FSZ_ERR_EB_TOO_LARGE: return "error bound too large for the field magnitude";
    default: return "unknown status";
    }
}

fsz_status fsz_field_stats(const float *d_in, size_t n, fsz_stats *d_stats, void *stream)
{
    if ((n > 0 && !d_in) || !d_stats || !aligned(d_in, 4)) return FSZ_ERR_INVALID_ARG;
    fsz_status st = FSZ_OK;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    StatsArgs a{d_in, n, d_stats, ws->d_partials};
    return ok(launch_stats(a, ws->stream)) ? FSZ_OK : FSZ_ERR_DEVICE;
}

fsz_status fsz_compress(const float *d_in, size_t n, fsz_eb_mode mode, double value, void *d_out,
                        size_t out_capacity, size_t *out_size, void *stream)
{
    return fsz_compress_ex(d_in, n, mode, value, nullptr, d_out, out_capacity, out_size, stream);
}

fsz_status fsz_compress_ex(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                           const fsz_stats *d_stats, void *d_out, size_t out_capacity, size_t *out_size,
                           void *stream)
{
    if (!out_size) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_compress_args(d_in, n, mode, value, d_out, out_capacity);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    st = enqueue_compress(ws, d_in, n, mode, value, d_stats, d_out, out_capacity, ws->d_final, &epoch);
    if (st != FSZ_OK) return st;
    return finish(ws, epoch, out_size);
}

fsz_status fsz_decompress(const void *d_cmp, size_t cmp_size, float *d_out, size_t n, void *stream)
{
    fsz_status st = check_decompress_args(d_cmp, cmp_size, d_out, n);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    st = enqueue_decompress(ws, d_cmp, cmp_size, d_out, n, ws->d_final, &epoch);
    if (st != FSZ_OK) return st;
    return finish(ws, epoch, nullptr);
}

fsz_status fsz_compress_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                              const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                              fsz_result *d_result, void *stream)
{
    if (!d_result) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_compress_args(d_in, n, mode, value, d_out, out_capacity);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    return enqueue_compress(ws, d_in, n, mode, value, d_stats, d_out, out_capacity, d_result, &epoch);
}

fsz_status fsz_decompress_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n,
                                fsz_result *d_result, void *stream)
{
    if (!d_result) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_decompress_args(d_cmp, cmp_size, d_out, n);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    return enqueue_decompress(ws, d_cmp, cmp_size, d_out, n, d_result, &epoch);
}

}  // extern "C"
