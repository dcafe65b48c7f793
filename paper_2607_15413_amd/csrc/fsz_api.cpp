// C ABI of libfsz.so: argument validation, per-(device, stream) workspace,
// kernel launches and the single device->host status read per call.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

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
        if (const char *e = std::getenv("FSZ_PIPE")) v.pipe_compress = std::atoi(e) != 0;
        if (const char *e = std::getenv("FSZ_PIPE_WAVES")) {
            const int k = std::atoi(e);
            if (k == 1 || k == 2 || k == 4 || k == 7 || k == 8 || k == 9) v.pipe_waves = k;  // 7, 9: + 1 control wave
        }
        if (const char *e = std::getenv("FSZ_DEC_WAVES")) {
            const int k = std::atoi(e);
            if (k == 4 || k == 8 || k == 16) v.dec_waves = k;
        }
        if (const char *e = std::getenv("FSZ_PREZERO_CR")) v.prezero_min_cr = std::atof(e);
        if (const char *e = std::getenv("FSZ_DEC_PRESCAN")) v.dec_prescan = std::atoi(e) != 0;
        if (const char *e = std::getenv("FSZ_DEC_WIDE_ABOVE")) v.dec_wide_above = std::strtoull(e, nullptr, 10);
        if (const char *e = std::getenv("FSZ_DEC_LOOKBACK_BELOW")) v.dec_lookback_below = std::strtoull(e, nullptr, 10);
        if (const char *e = std::getenv("FSZ_CFG_DEC_LOOKBACK_BELOW"))
            v.cfg_dec_lookback_below = std::strtoull(e, nullptr, 10);
        if (const char *e = std::getenv("FSZ_DEC_DIRECT_BELOW")) v.dec_direct_below = std::strtoull(e, nullptr, 10);
        if (const char *e = std::getenv("FSZ_GRID_FACTOR")) {
            const int f = std::atoi(e);
            if (f >= 1 && f <= 64) v.grid_factor = f;
        }
        return v;
    }();
    return t;
}
}  // namespace fsz

namespace fsz {

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

}  // namespace fsz

namespace {

// Pinned staging + device copy of one batch's job table.  A slot is reused
// only after the event recorded behind the batch that last used it.
struct DescSlot {
    void *h = nullptr;
    void *d = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};

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
    // batched form
    std::array<DescSlot, 4> ring;
    unsigned ring_next = 0;
    unsigned long long *b_flags = nullptr;
    uint64_t b_flags_cap = 0;
    StatsPartial *b_partials = nullptr;
    uint64_t b_partials_cap = 0;
    fsz_stats *b_stats = nullptr;
    uint64_t b_stats_cap = 0;
    unsigned long long *b_ticket = nullptr;
    // random-access decode: the range's base offset, then the reduction partials
    unsigned long long *d_range = nullptr;
    // five-read baseline: evaluation tables (53 bytes per tile)
    uint8_t *d_naive = nullptr;
    uint64_t naive_cap = 0;
    // whole-field decodes: chunk offsets of the pre-pass and its outcome word
    unsigned long long *d_offs = nullptr;
    uint64_t offs_cap = 0;
    uint32_t *d_go = nullptr;
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
                ok(hipMalloc(&ws->b_ticket, sizeof(unsigned long long))) &&
                ok(hipMalloc(&ws->d_go, sizeof(uint32_t))) &&
                ok(hipMemset(ws->d_ticket, 0, sizeof(unsigned long long))) &&
                ok(hipMemset(ws->b_ticket, 0, sizeof(unsigned long long))) &&
                ok(hipMemset(ws->d_final, 0, sizeof(fsz_result))) &&
                ok(hipDeviceSynchronize());
    for (auto &slot : ws->ring) good = good && ok(hipEventCreateWithFlags(&slot.ev, hipEventDisableTiming));
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
    if (!ok(hipMalloc(&ws->d_flags, cap * kFlagStride * sizeof(unsigned long long)))) return false;
    if (!ok(hipMemsetAsync(ws->d_flags, 0, cap * kFlagStride * sizeof(unsigned long long), ws->stream))) return false;
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
        return ok(hipMemsetAsync(ws->d_flags, 0, ws->flags_cap * kFlagStride * sizeof(unsigned long long), ws->stream));
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

// Enqueue (range pass if d_stats is NULL) + compression kernel.
fsz_status enqueue_compress(Workspace *ws, const float *d_in, uint64_t n, int mode, double value,
                            const fsz_stats *d_stats, void *d_out, uint64_t cap, fsz_result *d_final,
                            uint32_t *epoch_out, uint32_t features = kFeaturesAll)
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
    a.features = features;
    // the pipelined kernel may use chunks as small as one wave's 8 tiles
    if (!ensure_flags(ws, std::max<uint64_t>(a.nchunks, ceil_div(a.ntiles, kTilesPerWave)))) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    if (!ok(launch_compress(a, aligned(d_in, 16), tuning().staged_compress, ws->stream))) return FSZ_ERR_DEVICE;
    *epoch_out = a.epoch;
    return FSZ_OK;
}

template <typename T>
bool grow(T **p, uint64_t *cap, uint64_t want, hipStream_t s);

// The five-read baseline (Sec. V-C, Fig. 6): the same stream as
// enqueue_compress, from four evaluation passes and one encode pass.
fsz_status enqueue_compress_naive(Workspace *ws, const float *d_in, uint64_t n, int mode, double value,
                                  const fsz_stats *d_stats, void *d_out, uint64_t cap, fsz_result *d_final)
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
    a.features = kFeaturesAll;
    const uint64_t nt = std::max<uint64_t>(a.ntiles, 1);
    const uint64_t off_rates = 16 * nt, off_mu = off_rates + 32 * nt, off_ok = off_mu + 4 * nt;
    if (!grow(&ws->d_naive, &ws->naive_cap, off_ok + nt, ws->stream)) return FSZ_ERR_DEVICE;
    NaiveTables t;
    t.cost = reinterpret_cast<uint32_t *>(ws->d_naive);
    t.rates = ws->d_naive + off_rates;
    t.mu = reinterpret_cast<int32_t *>(ws->d_naive + off_mu);
    t.centre_ok = ws->d_naive + off_ok;
    if (!ensure_flags(ws, a.nchunks)) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    if (!ok(launch_compress_naive(a, t, aligned(d_in, 16), ws->stream))) return FSZ_ERR_DEVICE;
    return FSZ_OK;
}

fsz_status enqueue_decompress(Workspace *ws, const void *d_cmp, uint64_t cmp_size, float *d_out, uint64_t n,
                              fsz_result *d_final, uint32_t *epoch_out, bool prezero = false)
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
    a.tile_begin = 0;
    a.tile_end = a.ntiles;
    a.elem_begin = 0;
    a.elem_end = n;
    a.range_base = nullptr;
    if (!ensure_flags(ws, std::max<uint64_t>(a.nchunks, ceil_div(a.ntiles, kTilesPerWave)))) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    hipError_t e;
    if (prezero) {
        e = launch_decompress_prezero(a, aligned(d_out, 16), ws->stream);
    } else if (tuning().dec_prescan && tuning().staged_decompress && n >= tuning().dec_lookback_below) {
        // chunk offsets from the rate header first (chunks of 32 or 64 tiles)
        if (!grow(&ws->d_offs, &ws->offs_cap, std::max<uint64_t>(ceil_div(a.ntiles, 32), 1), ws->stream))
            return FSZ_ERR_DEVICE;
        e = launch_decompress_prescan(a, ws->d_offs, ws->d_go, aligned(d_out, 16), n < tuning().dec_direct_below,
                                      ws->stream);
    } else {
        e = launch_decompress(a, aligned(d_out, 16), tuning().staged_decompress, ws->stream);
    }
    if (!ok(e)) return FSZ_ERR_DEVICE;
    *epoch_out = a.epoch;
    return FSZ_OK;
}

// Whole-field decodes pick the pre-zeroed decoder for streams whose
// compression ratio, judged from the buffer size, exceeds the threshold.
bool auto_prezero(uint64_t n, uint64_t cmp_size)
{
    const double cr = tuning().prezero_min_cr;
    return cr > 0.0 && (double)(4 * n) > cr * (double)cmp_size;
}

// Tile configurations (Sec. VI-C, Table V): the generic lane-per-segment
// kernels, one chunk of kCfgChunkSegs 32-element segments per workgroup
// (decoder: 64 x kCfgDecWaves, or 64 x kCfgDecWideWaves in the lookback form
// of fields above dec_wide_above elements).
fsz_status enqueue_compress_config(Workspace *ws, const float *d_in, uint64_t n, int mode, double value,
                                   const fsz_stats *d_stats, int block, int tile_blocks, void *d_out, uint64_t cap,
                                   fsz_result *d_final)
{
    if (!d_stats) {
        StatsArgs sa{d_in, n, ws->d_stats, ws->d_partials};
        if (!ok(launch_stats(sa, ws->stream))) return FSZ_ERR_DEVICE;
        d_stats = ws->d_stats;
    }
    CompressArgs a{};
    a.x = d_in;
    a.n = n;
    a.ntiles = ceil_div(n, (uint64_t)block * tile_blocks);
    a.nblocks = ceil_div(n, (uint64_t)block);
    a.nchunks = n ? ceil_div(ceil_div(n, kBlock), kCfgChunkSegs) : 1;
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    a.out = static_cast<uint8_t *>(d_out);
    a.capacity = cap;
    a.stats = d_stats;
    a.value = value;
    a.mode = mode;
    a.features = kFeaturesAll;
    a.cfg_flags = cfg_flag_bits(block, tile_blocks);
    // flags for the generic kernel's chunks or the pipelined one's (smaller)
    if (!ensure_flags(ws, std::max<uint64_t>(a.nchunks, ceil_div(ceil_div(n, kBlock), kCfgPipeChunkSegs))))
        return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    if (!ok(launch_compress_cfg(a, block, tile_blocks, aligned(d_in, 16), ws->stream))) return FSZ_ERR_DEVICE;
    return FSZ_OK;
}

fsz_status enqueue_decompress_config(Workspace *ws, const void *d_cmp, uint64_t cmp_size, float *d_out, uint64_t n,
                                     int block, int tile_blocks, fsz_result *d_final)
{
    DecompressArgs a{};
    a.cmp = static_cast<const uint8_t *>(d_cmp);
    a.cmp_size = cmp_size;
    a.out = d_out;
    a.n = n;
    a.ntiles = ceil_div(n, (uint64_t)block * tile_blocks);
    a.nblocks = ceil_div(n, (uint64_t)block);
    const bool prescan = tuning().dec_prescan && n >= tuning().cfg_dec_lookback_below;
    const uint64_t chunk_segs = 64ull * (uint64_t)(prescan ? kCfgDecWaves : cfg_dec_lookback_waves(n));
    a.nchunks = n ? ceil_div(ceil_div(n, kBlock), chunk_segs) : 1;
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    a.tile_begin = 0;
    a.tile_end = a.ntiles;
    a.elem_begin = 0;
    a.elem_end = n;
    a.range_base = nullptr;
    a.cfg_flags = cfg_flag_bits(block, tile_blocks);
    if (!ensure_flags(ws, a.nchunks)) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    hipError_t e;
    if (prescan) {
        // chunk offsets from the rate header first, as for the default format
        if (!grow(&ws->d_offs, &ws->offs_cap, a.nchunks, ws->stream)) return FSZ_ERR_DEVICE;
        a.offsets = ws->d_offs;
        a.go = ws->d_go;
        e = launch_decompress_cfg_prescan(a, block, tile_blocks, aligned(d_out, 16), ws->stream);
    } else {
        e = launch_decompress_cfg(a, block, tile_blocks, aligned(d_out, 16), ws->stream);
    }
    if (!ok(e)) return FSZ_ERR_DEVICE;
    return FSZ_OK;
}

// Random-access decode of elements [begin, end): the tiles that hold them,
// at the offset the rate header gives for the first one.
fsz_status enqueue_decompress_range(Workspace *ws, const void *d_cmp, uint64_t cmp_size, uint64_t n,
                                    uint64_t begin, uint64_t end, float *d_out, fsz_result *d_final)
{
    DecompressArgs a{};
    a.cmp = static_cast<const uint8_t *>(d_cmp);
    a.cmp_size = cmp_size;
    a.out = d_out;
    a.n = n;
    a.ntiles = ceil_div(n, kTile);
    a.nblocks = ceil_div(n, kBlock);
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    a.tile_begin = begin / kTile;
    a.tile_end = end > begin ? ceil_div(end, kTile) : a.tile_begin;
    a.elem_begin = begin;
    a.elem_end = end;
    const uint64_t tiles = a.tile_end - a.tile_begin;
    a.nchunks = tiles ? ceil_div(tiles, kTilesPerChunk) : 1;
    if (!ws->d_range && !ok(hipMalloc(&ws->d_range, (1 + kStatsMaxBlocks) * sizeof(unsigned long long))))
        return FSZ_ERR_DEVICE;
    if (!ok(launch_range_base(a, ws->d_range, ws->d_range + 1, ws->stream))) return FSZ_ERR_DEVICE;
    a.range_base = ws->d_range;
    if (!ensure_flags(ws, std::max<uint64_t>(a.nchunks, ceil_div(tiles, kTilesPerWave)))) return FSZ_ERR_DEVICE;
    if (!next_epoch(ws, &a.epoch, &a.flag_epoch)) return FSZ_ERR_DEVICE;
    a.flags = ws->d_flags;
    a.ticket = ws->d_ticket;
    a.final = d_final;
    // 16-byte stores need the field's element 0 (d_out - begin) 16-byte aligned
    const bool al16 = ((reinterpret_cast<uintptr_t>(d_out) - 4 * (uintptr_t)begin) & 15u) == 0;
    if (!ok(launch_decompress(a, al16, tuning().staged_decompress, ws->stream))) return FSZ_ERR_DEVICE;
    return FSZ_OK;
}


// ------------------------------------------------------------------ batched form

// Device-side layout of a batch for one launch shape.
struct BatchLayout {
    std::vector<BatchJob> jobs;
    std::vector<uint64_t> chunk_end, seg_end;
    uint64_t total_chunks = 0, total_segs = 0, total_elems = 0;
    bool aligned16 = true, any_compress = false, any_decompress = false;
    size_t desc_bytes() const { return jobs.size() * (sizeof(BatchJob) + 2 * sizeof(uint64_t)); }
    void pack(void *dst) const
    {
        char *p = static_cast<char *>(dst);
        std::memcpy(p, jobs.data(), jobs.size() * sizeof(BatchJob));
        p += jobs.size() * sizeof(BatchJob);
        std::memcpy(p, chunk_end.data(), jobs.size() * sizeof(uint64_t));
        p += jobs.size() * sizeof(uint64_t);
        std::memcpy(p, seg_end.data(), jobs.size() * sizeof(uint64_t));
    }
};

// Validates every job (nothing is enqueued unless all pass) and lays out
// global chunk and range-pass segment ranges in job order.
fsz_status layout_batch(const fsz_job *jobs, size_t njobs, int waves, BatchLayout *L)
{
    if (njobs > 0 && !jobs) return FSZ_ERR_INVALID_ARG;
    if (njobs >= (1u << 31)) return FSZ_ERR_INVALID_ARG;
    const uint64_t tiles_per_chunk = (uint64_t)kTilesPerWave * (uint64_t)waves;
    L->jobs.resize(njobs);
    L->chunk_end.resize(njobs);
    L->seg_end.resize(njobs);
    for (size_t k = 0; k < njobs; k++) {
        const fsz_job &j = jobs[k];
        if (!j.d_result) return FSZ_ERR_INVALID_ARG;
        fsz_status st;
        if (j.op == FSZ_OP_COMPRESS)
            st = check_compress_args(static_cast<const float *>(j.d_src), j.n, j.mode, j.value, j.d_dst,
                                     j.dst_capacity);
        else if (j.op == FSZ_OP_DECOMPRESS)
            st = check_decompress_args(j.d_src, j.src_size, static_cast<const float *>(j.d_dst), j.n);
        else
            st = FSZ_ERR_INVALID_ARG;
        if (st != FSZ_OK) return st;
        BatchJob J{};
        J.op = (uint32_t)j.op;
        J.mode = j.mode;
        J.n = j.n;
        J.ntiles = ceil_div(j.n, kTile);
        J.nblocks = ceil_div(j.n, kBlock);
        J.nchunks = J.ntiles ? ceil_div(J.ntiles, tiles_per_chunk) : 1;
        J.data0 = kHeaderBytes + pad16(J.nblocks);
        J.src = j.d_src;
        J.src_size = j.op == FSZ_OP_DECOMPRESS ? j.src_size : 0;
        J.dst = j.d_dst;
        J.dst_capacity = j.op == FSZ_OP_COMPRESS ? j.dst_capacity : 0;
        J.value = j.value;
        J.final = j.d_result;
        J.chunk_base = L->total_chunks;
        L->total_chunks += J.nchunks;
        J.seg_base = L->total_segs;
        J.nsegs = j.op == FSZ_OP_COMPRESS ? ceil_div(j.n, kSegElems) : 0;
        L->total_segs += J.nsegs;
        L->total_elems += j.n;
        L->chunk_end[k] = L->total_chunks;
        L->seg_end[k] = L->total_segs;
        if (j.op == FSZ_OP_COMPRESS) {
            L->any_compress = true;
            L->aligned16 = L->aligned16 && aligned(j.d_src, 16);
        } else {
            L->any_decompress = true;
            L->aligned16 = L->aligned16 && aligned(j.d_dst, 16);
        }
        L->jobs[k] = J;
    }
    // one work item per workgroup: grid x times workgroup size must fit 32 bits
    if (L->total_chunks * (uint64_t)(waves * 64) >= (1ull << 32) || L->total_segs * kStatsThreads >= (1ull << 32))
        return FSZ_ERR_INVALID_ARG;
    return FSZ_OK;
}

template <typename T>
bool grow(T **p, uint64_t *cap, uint64_t want, hipStream_t s)
{
    if (want <= *cap) return true;
    uint64_t c = *cap ? *cap : 256;
    while (c < want) c *= 2;
    if (*p) {
        if (!ok(hipStreamSynchronize(s)) || !ok(hipFree(*p))) return false;
        *p = nullptr;
        *cap = 0;
    }
    if (!ok(hipMalloc(p, c * sizeof(T)))) return false;
    *cap = c;
    return true;
}

BatchShape to_shape(const fsz_tuning &t)
{
    BatchShape s;
    s.waves = t.waves_per_group;
    s.groups_per_cu = t.groups_per_cu;
    return s;
}

// ---- autotune cache: best shape per (architecture, batch size class)

std::mutex g_tune_mu;
std::map<std::string, fsz_tuning> g_tune;
bool g_tune_loaded = false;

// Architecture name of the current device (cached per device; the caller
// holds g_tune_mu).
std::string arch_name()
{
    static std::map<int, std::string> names;
    int dev = 0;
    if (!ok(hipGetDevice(&dev))) return "unknown";
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop{};
    if (!ok(hipGetDeviceProperties(&prop, dev))) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    a = colon == std::string::npos ? a : a.substr(0, colon);
    names[dev] = a;
    return a;
}

int ilog2(uint64_t v)
{
    int l = 0;
    while (v > 1) {
        v >>= 1;
        l++;
    }
    return l;
}

// Size class: log2 of the total element count, log2 of the job count and
// which operations occur.
std::string size_class(const fsz_job *jobs, size_t njobs)
{
    uint64_t elems = 0;
    bool c = false, d = false;
    for (size_t k = 0; k < njobs; k++) {
        elems += jobs[k].n;
        (jobs[k].op == FSZ_OP_COMPRESS ? c : d) = true;
    }
    char buf[96];
    std::snprintf(buf, sizeof buf, "%s/e%d/j%d/%s%s", arch_name().c_str(), ilog2(elems + 1), ilog2(njobs + 1),
                  c ? "c" : "", d ? "d" : "");
    return buf;
}

void load_tune_file_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("FSZ_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[128];
    int w = 0, g = 0;
    while (std::fscanf(f, "%127s %d %d", key, &w, &g) == 3) g_tune[key] = fsz_tuning{w, g};
    std::fclose(f);
}

bool cached_tuning(const fsz_job *jobs, size_t njobs, fsz_tuning *out)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find(size_class(jobs, njobs));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void store_tuning(const fsz_job *jobs, size_t njobs, const fsz_tuning &t)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    load_tune_file_locked();
    const std::string key = size_class(jobs, njobs);
    g_tune[key] = t;
    if (const char *path = std::getenv("FSZ_TUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d %d\n", key.c_str(), t.waves_per_group, t.groups_per_cu);
            std::fclose(f);
        }
    }
}

fsz_status resolve_tuning(const fsz_job *jobs, size_t njobs, const fsz_tuning *tuning, fsz_tuning *out)
{
    if (tuning) {
        if (!batch_shape_supported(to_shape(*tuning))) return FSZ_ERR_INVALID_ARG;
        *out = *tuning;
        return FSZ_OK;
    }
    if (!cached_tuning(jobs, njobs, out)) *out = fsz_tuning{4, 0};
    return FSZ_OK;
}

BatchArgs batch_args(const BatchLayout &L, void *d_desc, uint32_t epoch, unsigned long long *flags,
                     unsigned long long *ticket, fsz_stats *stats, StatsPartial *partials)
{
    BatchArgs b{};
    const size_t nj = L.jobs.size();
    char *p = static_cast<char *>(d_desc);
    b.jobs = reinterpret_cast<const BatchJob *>(p);
    b.chunk_end = reinterpret_cast<const uint64_t *>(p + nj * sizeof(BatchJob));
    b.seg_end = reinterpret_cast<const uint64_t *>(p + nj * (sizeof(BatchJob) + sizeof(uint64_t)));
    b.njobs = (uint32_t)nj;
    b.epoch = epoch;
    b.total_chunks = L.total_chunks;
    b.total_segs = L.total_segs;
    b.nflags = L.total_chunks * kFlagStride;  // words
    b.flags = flags;
    b.ticket = ticket;
    b.stats = stats;
    b.partials = partials;
    return b;
}

// Make a job-table slot hold `bytes` (the slot is idle).  Freeing device
// memory synchronizes the device, so long-running callers reserve up front
// (reserve_batch).
bool grow_slot(DescSlot &slot, size_t bytes)
{
    if (bytes <= slot.cap) return true;
    if (slot.h && !ok(hipHostFree(slot.h))) return false;
    if (slot.d && !ok(hipFree(slot.d))) return false;
    slot.h = slot.d = nullptr;
    slot.cap = 0;
    size_t c = 4096;
    while (c < bytes) c *= 2;
    if (!ok(hipHostMalloc(&slot.h, c, hipHostMallocDefault)) || !ok(hipMalloc(&slot.d, c))) return false;
    slot.cap = c;
    return true;
}

// Enqueue one batch on the workspace's stream (caller holds ws->mu).
fsz_status enqueue_batch(Workspace *ws, const fsz_job *jobs, size_t njobs, const BatchShape &shape)
{
    BatchLayout L;
    fsz_status st = layout_batch(jobs, njobs, shape.waves, &L);
    if (st != FSZ_OK || njobs == 0) return st;
    if (!grow(&ws->b_flags, &ws->b_flags_cap, L.total_chunks * kFlagStride, ws->stream) ||
        !grow(&ws->b_partials, &ws->b_partials_cap, std::max<uint64_t>(L.total_segs, 1), ws->stream) ||
        !grow(&ws->b_stats, &ws->b_stats_cap, njobs, ws->stream))
        return FSZ_ERR_DEVICE;
    DescSlot &slot = ws->ring[ws->ring_next++ % ws->ring.size()];
    if (slot.used && !ok(hipEventSynchronize(slot.ev))) return FSZ_ERR_DEVICE;
    const size_t bytes = L.desc_bytes();
    if (!grow_slot(slot, bytes)) return FSZ_ERR_DEVICE;
    L.pack(slot.h);
    if (!ok(hipMemcpyAsync(slot.d, slot.h, bytes, hipMemcpyHostToDevice, ws->stream))) return FSZ_ERR_DEVICE;
    if (++ws->call == 0) ++ws->call;
    const BatchArgs b = batch_args(L, slot.d, ws->call, ws->b_flags, ws->b_ticket, ws->b_stats, ws->b_partials);
    if (!ok(launch_batch(b, L.aligned16, L.any_compress, L.any_decompress, shape, ws->stream))) return FSZ_ERR_DEVICE;
    if (!ok(hipEventRecord(slot.ev, ws->stream))) return FSZ_ERR_DEVICE;
    slot.used = true;
    return FSZ_OK;
}

}  // namespace

namespace fsz {

bool reserve_batch(hipStream_t stream, uint64_t jobs, uint64_t chunks, uint64_t segs)
{
    fsz_status st = FSZ_OK;
    Workspace *ws = get_workspace(stream, &st);
    if (!ws) return false;
    std::lock_guard<std::mutex> g(ws->mu);
    if (!grow(&ws->b_flags, &ws->b_flags_cap, std::max<uint64_t>(chunks, 1) * kFlagStride, ws->stream) ||
        !grow(&ws->b_partials, &ws->b_partials_cap, std::max<uint64_t>(segs, 1), ws->stream) ||
        !grow(&ws->b_stats, &ws->b_stats_cap, std::max<uint64_t>(jobs, 1), ws->stream))
        return false;
    const size_t bytes = jobs * (sizeof(BatchJob) + 2 * sizeof(uint64_t));
    for (auto &slot : ws->ring) {
        if (slot.used && !ok(hipEventSynchronize(slot.ev))) return false;
        if (!grow_slot(slot, bytes)) return false;
    }
    return true;
}

}  // namespace fsz

// A captured batch (see fsz_plan_create).
struct fsz_plan {
    int device = 0;
    fsz_tuning tuning{4, 0};
    size_t njobs = 0;
    void *d_desc = nullptr;
    unsigned long long *d_flags = nullptr;
    unsigned long long *d_ticket = nullptr;
    StatsPartial *d_partials = nullptr;
    fsz_stats *d_stats = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void free_plan(fsz_plan *p)
{
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->d_desc);
    (void)hipFree(p->d_flags);
    (void)hipFree(p->d_ticket);
    (void)hipFree(p->d_partials);
    (void)hipFree(p->d_stats);
    delete p;
}

uint32_t g_plan_ids = 0x80000000u;
}  // namespace

extern "C" {

size_t fsz_compressed_bound(size_t n)
{
    const uint64_t nblocks = ceil_div(n, kBlock);
    const uint64_t ntiles = ceil_div(n, kTile);
    return (size_t)(kHeaderBytes + pad16(nblocks) + 4 * ntiles + (4 + 4 * 31) * nblocks);
}

size_t fsz_compressed_bound_config(size_t n, int block, int tile_blocks)
{
    if (!cfg_supported(block, tile_blocks)) return 0;
    const uint64_t nblocks = ceil_div(n, (uint64_t)block);
    const uint64_t ntiles = ceil_div(n, (uint64_t)block * tile_blocks);
    return (size_t)(kHeaderBytes + pad16(nblocks) + 4 * ntiles + (uint64_t)(block / 8) * 32 * nblocks);
}

const char *fsz_status_string(fsz_status s)
{
    switch (static_cast<int>(s)) {  // C callers may pass any int
    case FSZ_OK: return "ok";
    case FSZ_ERR_INVALID_ARG: return "invalid argument";
    case FSZ_ERR_NONFINITE: return "input holds NaN or Inf";
    case FSZ_ERR_EB_TOO_SMALL: return "error bound below 8 ulp of max|x|";
    case FSZ_ERR_CAPACITY: return "output capacity too small";
    case FSZ_ERR_CORRUPT: return "corrupt stream";
    case FSZ_ERR_SIZE_MISMATCH: return "element count differs from the stream";
    case FSZ_ERR_DEVICE: return "HIP runtime error";
    case FSZ_ERR_EB_TOO_LARGE: return "error bound too large for the field magnitude";
    case FSZ_ERR_TOO_LARGE: return "field larger than the allocation-free scratch (2^30 elements)";
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
    st = enqueue_decompress(ws, d_cmp, cmp_size, d_out, n, ws->d_final, &epoch, auto_prezero(n, cmp_size));
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

fsz_status fsz_compress_features_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                       const fsz_stats *d_stats, unsigned features, void *d_out,
                                       size_t out_capacity, fsz_result *d_result, void *stream)
{
    if (!d_result || (features & ~(unsigned)FSZ_FEATURES_ALL) != 0) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_compress_args(d_in, n, mode, value, d_out, out_capacity);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    return enqueue_compress(ws, d_in, n, mode, value, d_stats, d_out, out_capacity, d_result, &epoch, features);
}

fsz_status fsz_compress_five_read_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                        const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                                        fsz_result *d_result, void *stream)
{
    if (!d_result) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_compress_args(d_in, n, mode, value, d_out, out_capacity);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    return enqueue_compress_naive(ws, d_in, n, mode, value, d_stats, d_out, out_capacity, d_result);
}

fsz_status fsz_decompress_range_async(const void *d_cmp, size_t cmp_size, size_t n, size_t begin, size_t end,
                                      float *d_out, fsz_result *d_result, void *stream)
{
    if (!d_result || begin > end || end > n) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_decompress_args(d_cmp, cmp_size, d_out, end - begin);
    if (st != FSZ_OK) return st;
    // The range pass reads rate bytes before the decoder checks the header:
    // the buffer must hold every rate byte of an n-element stream.
    if (cmp_size < kHeaderBytes + pad16(ceil_div((uint64_t)n, kBlock))) return FSZ_ERR_CORRUPT;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    return enqueue_decompress_range(ws, d_cmp, cmp_size, n, begin, end, d_out, d_result);
}

fsz_status fsz_compress_config_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                     const fsz_stats *d_stats, int block, int tile_blocks, void *d_out,
                                     size_t out_capacity, fsz_result *d_result, void *stream)
{
    if (!d_result || !cfg_supported(block, tile_blocks) || !valid_bound(mode, value) || !d_out ||
        (n > 0 && !d_in) || !aligned(d_in, 4) || !aligned(d_out, 4))
        return FSZ_ERR_INVALID_ARG;
    if (out_capacity < kHeaderBytes + pad16(ceil_div(n, (uint64_t)block))) return FSZ_ERR_CAPACITY;
    fsz_status st = FSZ_OK;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    return enqueue_compress_config(ws, d_in, n, mode, value, d_stats, block, tile_blocks, d_out, out_capacity,
                                   d_result);
}

fsz_status fsz_decompress_config_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n, int block,
                                       int tile_blocks, fsz_result *d_result, void *stream)
{
    if (!d_result || !cfg_supported(block, tile_blocks)) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_decompress_args(d_cmp, cmp_size, d_out, n);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    return enqueue_decompress_config(ws, d_cmp, cmp_size, d_out, n, block, tile_blocks, d_result);
}

fsz_status fsz_compress_noalloc_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                      const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                                      fsz_result *d_result, void *stream)
{
    if (!d_result) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_compress_args(d_in, n, mode, value, d_out, out_capacity);
    if (st != FSZ_OK) return st;
    return compress_noalloc(d_in, n, mode, value, d_stats, d_out, out_capacity, d_result,
                            static_cast<hipStream_t>(stream));
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
    return enqueue_decompress(ws, d_cmp, cmp_size, d_out, n, d_result, &epoch, auto_prezero(n, cmp_size));
}

fsz_status fsz_decompress_prezero_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n,
                                        fsz_result *d_result, void *stream)
{
    if (!d_result) return FSZ_ERR_INVALID_ARG;
    fsz_status st = check_decompress_args(d_cmp, cmp_size, d_out, n);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    uint32_t epoch = 0;
    return enqueue_decompress(ws, d_cmp, cmp_size, d_out, n, d_result, &epoch, true);
}

fsz_status fsz_batch_async(const fsz_job *jobs, size_t njobs, const fsz_tuning *tuning, void *stream)
{
    if (njobs > 0 && !jobs) return FSZ_ERR_INVALID_ARG;
    fsz_tuning t{};
    fsz_status st = resolve_tuning(jobs, njobs, tuning, &t);
    if (st != FSZ_OK) return st;
    {
        BatchLayout L;  // host-side validation before any device work
        st = layout_batch(jobs, njobs, t.waves_per_group, &L);
        if (st != FSZ_OK || njobs == 0) return st;
    }
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    std::lock_guard<std::mutex> g(ws->mu);
    return enqueue_batch(ws, jobs, njobs, to_shape(t));
}

fsz_status fsz_autotune(const fsz_job *jobs, size_t njobs, int reps, void *stream, fsz_tuning *best)
{
    if (!best || reps < 1 || njobs == 0 || !jobs) return FSZ_ERR_INVALID_ARG;
    BatchLayout L;
    fsz_status st = layout_batch(jobs, njobs, 4, &L);
    if (st != FSZ_OK) return st;
    Workspace *ws = get_workspace(static_cast<hipStream_t>(stream), &st);
    if (!ws) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!ok(hipEventCreate(&e0)) || !ok(hipEventCreate(&e1))) return FSZ_ERR_DEVICE;
    float best_ms = 0.0f;
    bool found = false;
    st = FSZ_OK;
    const int waves[] = {2, 4, 8};
    const int groups[] = {0, 1, 2, 3, 4, 6};
    for (int w : waves) {
        for (int gcu : groups) {
            const fsz_tuning cand{w, gcu};
            if (!batch_shape_supported(to_shape(cand))) continue;
            std::lock_guard<std::mutex> g(ws->mu);
            st = enqueue_batch(ws, jobs, njobs, to_shape(cand));  // warm-up
            if (st != FSZ_OK) break;
            if (!ok(hipEventRecord(e0, ws->stream))) { st = FSZ_ERR_DEVICE; break; }
            for (int r = 0; r < reps && st == FSZ_OK; r++) st = enqueue_batch(ws, jobs, njobs, to_shape(cand));
            if (st != FSZ_OK) break;
            float ms = 0.0f;
            if (!ok(hipEventRecord(e1, ws->stream)) || !ok(hipEventSynchronize(e1)) ||
                !ok(hipEventElapsedTime(&ms, e0, e1))) {
                st = FSZ_ERR_DEVICE;
                break;
            }
            if (!found || ms < best_ms) {
                best_ms = ms;
                *best = cand;
                found = true;
            }
        }
        if (st != FSZ_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FSZ_OK) return st;
    if (!found) return FSZ_ERR_DEVICE;
    store_tuning(jobs, njobs, *best);
    return FSZ_OK;
}

fsz_status fsz_plan_create(const fsz_job *jobs, size_t njobs, const fsz_tuning *tuning, fsz_plan **plan)
{
    if (!plan || (njobs > 0 && !jobs)) return FSZ_ERR_INVALID_ARG;
    *plan = nullptr;
    fsz_tuning t{};
    fsz_status st = resolve_tuning(jobs, njobs, tuning, &t);
    if (st != FSZ_OK) return st;
    BatchLayout L;
    st = layout_batch(jobs, njobs, t.waves_per_group, &L);
    if (st != FSZ_OK) return st;
    auto *p = new fsz_plan();
    p->tuning = t;
    p->njobs = njobs;
    bool good = ok(hipGetDevice(&p->device));
    if (good && njobs > 0) {
        std::vector<char> host(L.desc_bytes());
        L.pack(host.data());
        hipStream_t cs = nullptr;
        good = ok(hipMalloc(&p->d_desc, host.size())) &&
               ok(hipMalloc(&p->d_flags, std::max<uint64_t>(L.total_chunks, 1) * kFlagStride * sizeof(unsigned long long))) &&
               ok(hipMalloc(&p->d_ticket, sizeof(unsigned long long))) &&
               ok(hipMalloc(&p->d_partials, std::max<uint64_t>(L.total_segs, 1) * sizeof(StatsPartial))) &&
               ok(hipMalloc(&p->d_stats, njobs * sizeof(fsz_stats))) &&
               ok(hipMemcpy(p->d_desc, host.data(), host.size(), hipMemcpyHostToDevice)) &&
               ok(hipMemset(p->d_ticket, 0, sizeof(unsigned long long))) && ok(hipDeviceSynchronize()) &&
               ok(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        if (good) {
            const BatchArgs b = batch_args(L, p->d_desc, g_plan_ids++, p->d_flags, p->d_ticket, p->d_stats,
                                           p->d_partials);
            good = ok(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            if (good) {
                const bool launched =
                    ok(launch_batch(b, L.aligned16, L.any_compress, L.any_decompress, to_shape(t), cs));
                const bool ended = ok(hipStreamEndCapture(cs, &p->graph));
                good = launched && ended && ok(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
            }
        }
        if (cs) (void)hipStreamDestroy(cs);
    }
    if (!good) {
        free_plan(p);
        return FSZ_ERR_DEVICE;
    }
    *plan = p;
    return FSZ_OK;
}

fsz_status fsz_plan_launch(fsz_plan *plan, void *stream)
{
    if (!plan) return FSZ_ERR_INVALID_ARG;
    if (plan->njobs == 0) return FSZ_OK;
    return ok(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream))) ? FSZ_OK : FSZ_ERR_DEVICE;
}

fsz_status fsz_plan_get_tuning(const fsz_plan *plan, fsz_tuning *out)
{
    if (!plan || !out) return FSZ_ERR_INVALID_ARG;
    *out = plan->tuning;
    return FSZ_OK;
}

void fsz_plan_destroy(fsz_plan *plan) { free_plan(plan); }

}  // extern "C"
