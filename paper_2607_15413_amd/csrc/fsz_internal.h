// Internal declarations shared by the kernel and host translation units of
// libfsz.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsz.h"

namespace fsz {

// Format constants: block of 32 elements, tile of 8 blocks (Sec. III-A).
constexpr int kBlock = 32;
constexpr int kBlocksPerTile = 8;
constexpr int kTile = kBlock * kBlocksPerTile;
constexpr int kHeaderBytes = 32;

// Launch geometry.  One lane owns one 32-element block, so a wave64 holds 8
// tiles; a workgroup of kWaves waves owns one chunk of 8*kWaves tiles.
constexpr int kWaves = 4;
constexpr int kThreads = kWaves * 64;
constexpr int kTilesPerWave = 8;
constexpr int kTilesPerChunk = kTilesPerWave * kWaves;
constexpr int kStatsThreads = 256;
constexpr int kStatsMaxBlocks = 1024;

// Per-lane LDS staging row: 32 floats + 4 dwords of padding (bank spread).
constexpr int kStageRowDwords = 36;
constexpr int kStageWaveDwords = 64 * kStageRowDwords;

// Chunk flag word for the decoupled lookback (Sec. IV-D): 2-bit state,
// 18-bit call epoch (stale words from earlier calls read as "not ready"),
// 1 error bit (OR-ed along the prefix), 43-bit byte count.
constexpr uint64_t kFlagAggregate = 1;
constexpr uint64_t kFlagInclusive = 2;
constexpr int kEpochBits = 18;
constexpr uint32_t kEpochMask = (1u << kEpochBits) - 1;
constexpr int kEpochShift = 44;
constexpr int kErrorBit = 43;
constexpr uint64_t kValueMask = (1ull << kErrorBit) - 1;
// Chunk c's flag word sits at index c * kFlagStride of a flag array (32 bytes
// apart, four per 128-byte line).  The words are read and written at agent
// scope from all XCDs; packed eight to a line they measurably slowed the
// compressor's data traffic, spread four to a line they did not.
constexpr uint64_t kFlagStride = 4;

// All prediction features on: cross-block state, centering, second order.
constexpr uint32_t kFeaturesAll = FSZ_FEATURES_ALL;

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t pad16(uint64_t a) { return (a + 15) / 16 * 16; }

struct StatsPartial {
    float xmin, xmax, maxabs;
    uint32_t flags;
};

struct StatsArgs {
    const float *x;
    uint64_t n;
    fsz_stats *out;
    StatsPartial *partials;
};

struct CompressArgs {
    const float *x;
    uint64_t n, ntiles, nblocks, nchunks, data0;
    uint8_t *out;
    uint64_t capacity;
    const fsz_stats *stats;
    double value;
    int mode;
    uint32_t features;    // FSZ_FEAT_* switches (kFeaturesAll = the full method)
    uint32_t cfg_flags;   // header flags bits 2-4: tile configuration (0 = B 32, T 8)
    uint32_t epoch;       // 32-bit call epoch (result words)
    uint32_t flag_epoch;  // 18-bit nonzero epoch (chunk flags)
    unsigned long long *flags;
    unsigned long long *ticket;  // zero between launches (self-resetting)
    fsz_result *final;           // written by the workgroup owning the last chunk
};

struct DecompressArgs {
    const uint8_t *cmp;
    uint64_t cmp_size;
    float *out;  // element elem_begin of the field
    uint64_t n, ntiles, nblocks, nchunks, data0;
    // Decoded range: tiles [tile_begin, tile_end) (chunks count from
    // tile_begin), elements [elem_begin, elem_end) written.  range_base: the
    // byte offset of tile_begin's data after data0 (device; null = 0 for a
    // whole-field decode, which also checks the stream's total and padding).
    uint64_t tile_begin, tile_end, elem_begin, elem_end;
    const unsigned long long *range_base;
    uint32_t cfg_flags;  // tile-configuration decoders: the header flags bits 2-4 required
    // Whole-field decodes with the offsets pre-pass: each chunk's byte offset
    // after data0 (written by the pre-pass), and its outcome (FSZ_OK: decode).
    const unsigned long long *offsets;
    const uint32_t *go;
    uint32_t epoch, flag_epoch;
    unsigned long long *flags;
    unsigned long long *ticket;  // zero between launches (self-resetting)
    fsz_result *final;           // written by the workgroup owning the last chunk
};

// ---- naive five-read baseline (Sec. V-C, Fig. 6): per-tile evaluation tables
// written by four evaluation passes (one per variant) and read by the encode
// pass.  Laid out [variant][tile] (cost), [variant][tile][block] (rates).
struct NaiveTables {
    uint32_t *cost;      // 4 * ntiles: tile cost C of LZ1, LZ2, LZ1c, LZ2c
    uint8_t *rates;      // 4 * ntiles * 8: block rates of each variant
    int32_t *mu;         // ntiles: quantized tile mean (written by the centred passes)
    uint8_t *centre_ok;  // ntiles: the mean is finite
};

// ---- batched form: one launch over many jobs (compress or decompress)

constexpr int kSegElems = 32768;  // elements per workgroup of the batched range pass

// One job of a batch, as the kernels read it (built by the host, uploaded to
// device memory once per batch).  Chunks of job j are global chunks
// [chunk_base, chunk_base + nchunks); its range-pass segments are
// [seg_base, seg_base + nsegs) (compress only).
struct BatchJob {
    uint32_t op;  // FSZ_OP_COMPRESS or FSZ_OP_DECOMPRESS
    int32_t mode;
    uint64_t n, ntiles, nblocks, nchunks, data0;
    const void *src;
    uint64_t src_size;
    void *dst;
    uint64_t dst_capacity;
    double value;
    fsz_result *final;
    uint64_t chunk_base, seg_base, nsegs;
    uint64_t pad;
};
static_assert(sizeof(BatchJob) == 128, "BatchJob layout");

struct BatchArgs {
    const BatchJob *jobs;
    const uint64_t *chunk_end;  // chunk_end[j] = chunk_base[j] + nchunks[j]
    const uint64_t *seg_end;    // seg_end[j] = seg_base[j] + nsegs[j]
    uint32_t njobs;
    uint32_t epoch;             // result tag
    uint64_t total_chunks, total_segs, nflags;  // nflags: flag words (kFlagStride per chunk)
    unsigned long long *flags;  // cleared by the batch's range pass
    unsigned long long *ticket; // zero between launches (self-resetting)
    fsz_stats *stats;           // one per job
    StatsPartial *partials;     // one per segment
};

// Launch shape of the batched kernel: waves per workgroup (a chunk is 8 tiles
// per wave) and a cap on resident workgroups per CU (0 = no cap).
struct BatchShape {
    int waves = 4;
    int groups_per_cu = 0;
};

// Kernel launchers (fsz_kernels.hip).
hipError_t launch_stats(const StatsArgs &a, hipStream_t s);
// staged = write outputs through an LDS staging buffer with coalesced stores
// instead of lane-per-block stores.
hipError_t launch_compress(const CompressArgs &a, bool in_aligned16, bool staged, hipStream_t s);
// The five-read baseline: four evaluation launches, then the encode launch
// (a.nchunks counts chunks of kTilesPerChunk tiles).
hipError_t launch_compress_naive(const CompressArgs &a, const NaiveTables &t, bool in_aligned16, hipStream_t s);
hipError_t launch_decompress(const DecompressArgs &a, bool out_aligned16, bool staged, hipStream_t s);
// Whole-field decompression with the chunk offsets computed first from the
// rate header (no lookback in the decoder): offsets has room for one word per
// chunk of 32 tiles, go for one status word.  direct: one chunk of 32 tiles
// per workgroup instead of the persistent grid over chunks of 64 tiles.
hipError_t launch_decompress_prescan(const DecompressArgs &a, unsigned long long *offsets, uint32_t *go,
                                     bool out_aligned16, bool direct, hipStream_t s);
// Pre-zeroed decompression (Sec. III-A): a fill of out[0, n) with +0.0, then
// the decoder that skips waves whose tiles are all zero.
hipError_t launch_decompress_prezero(const DecompressArgs &a, bool out_aligned16, hipStream_t s);
// Tile configurations (Sec. VI-C): one chunk of kCfgWaves x 64 32-element segments per
// workgroup (a.nchunks counts those; for the decoder kCfgDecWaves x 64), block in {32, 64},
// tile_blocks in {4, 8, 16}.  A
// 16-byte aligned input runs the pipelined compressor instead, whose chunks of
// kCfgPipeChunkSegs segments the launch counts itself (the flags must cover them).
hipError_t launch_compress_cfg(const CompressArgs &a, int block, int tile_blocks, bool in_aligned16, hipStream_t s);
hipError_t launch_decompress_cfg(const DecompressArgs &a, int block, int tile_blocks, bool out_aligned16,
                                 hipStream_t s);
// The same decode with chunk offsets from a pre-pass over the rate header
// (a.nchunks and a.offsets: one per chunk of kCfgDecChunkSegs segments; a.go:
// its outcome).
hipError_t launch_decompress_cfg_prescan(const DecompressArgs &a, int block, int tile_blocks, bool out_aligned16,
                                         hipStream_t s);
constexpr int kCfgWaves = 16;
constexpr int kCfgChunkSegs = kCfgWaves * 64;
constexpr int kCfgPipeChunkSegs = 8 * 64;  // the pipelined configuration compressor's chunk
// the configuration decoder: workgroups of 4 waves, one chunk of 4 x 64 segments each
// (the lookback form of fields above dec_wide_above elements: 16 waves)
constexpr int kCfgDecWaves = 4;
constexpr int kCfgDecChunkSegs = kCfgDecWaves * 64;
constexpr int kCfgDecWideWaves = 16;
// header flags bits 2-4 of a tile configuration (0 for B 32, T 8)
inline uint32_t cfg_flag_bits(int block, int tile_blocks)
{
    return (block == 64 ? 4u : 0u) | (tile_blocks == 4 ? 8u : tile_blocks == 16 ? 16u : 0u);
}
inline bool cfg_supported(int block, int tile_blocks)
{
    return (block == 32 || block == 64) && (tile_blocks == 4 || tile_blocks == 8 || tile_blocks == 16);
}
// Byte offset of tile_begin's data: a reduction of the block sizes before it
// over the rate header into *range_base (partials: kStatsMaxBlocks words).
hipError_t launch_range_base(const DecompressArgs &a, unsigned long long *range_base, unsigned long long *partials,
                             hipStream_t s);
// Range pass + flag clear, per-job stats, then the batched kernel.
// Compress-only batches with 16-byte aligned inputs run a persistent
// pipelined kernel, decompress-only batches a persistent decoder, mixed
// batches one work item per workgroup.
hipError_t launch_batch(const BatchArgs &b, bool aligned16, bool any_compress, bool any_decompress,
                        const BatchShape &shape, hipStream_t s);
bool batch_shape_supported(const BatchShape &shape);

// Allocation-free compression: fsz_compress_async's work with every scratch
// word in a fixed device array (fsz_kernels.hip); n above 2^30 elements
// returns FSZ_ERR_TOO_LARGE.  Arguments already checked by the caller.
fsz_status compress_noalloc(const float *d_in, uint64_t n, int mode, double value, const fsz_stats *d_stats,
                            void *d_out, uint64_t cap, fsz_result *d_result, hipStream_t s);

// Host-side argument checks shared by every entry point (fsz_api.cpp).
bool aligned(const void *p, uintptr_t a);
bool valid_bound(int mode, double value);
fsz_status check_compress_args(const float *d_in, size_t n, int mode, double value, const void *d_out,
                               size_t cap);
fsz_status check_decompress_args(const void *d_cmp, size_t cmp_size, const float *d_out, size_t n);

// Sizes the batch workspace of `stream` for rounds of up to `jobs` jobs,
// `chunks` work items and `segs` range-pass segments, so that later batches
// within those limits allocate (and synchronize the device) never again.
bool reserve_batch(hipStream_t stream, uint64_t jobs, uint64_t chunks, uint64_t segs);

// Launch tuning knobs, process-wide, read once from the environment:
// FSZ_STAGED (letters c / d / l: stage compress output / decompress output /
// compress input through LDS), FSZ_PIPE (0: no pipelined persistent
// compression for 16-byte aligned inputs), FSZ_PIPE_WAVES (its waves per
// workgroup: 1, 2, 4 or 8), FSZ_DEC_WAVES (waves per workgroup of the
// default format's whole-field lookback decoder: 4, 8 or 16, for every size),
// FSZ_DEC_WIDE_ABOVE (16-wave chunks above this many decoded elements, else 8,
// for that decoder without FSZ_DEC_WAVES and for random access; for the tile
// configurations' lookback form 16, else 4),
// FSZ_DEC_LOOKBACK_BELOW and FSZ_CFG_DEC_LOOKBACK_BELOW (whole-field decodes of
// the default format / the tile configurations below this many elements use
// the lookback decoder, larger ones the offsets pre-pass), FSZ_DEC_DIRECT_BELOW
// (pre-pass decodes below this size: one chunk per workgroup), FSZ_GRID_FACTOR
// (persistent workgroups per CU slot,
// default 1) and FSZ_PREZERO_CR (whole-field decodes of streams above this
// compression ratio, judged from the buffer size, use the pre-zeroed decoder)
// and FSZ_DEC_PRESCAN (0: whole-field decodes find chunk offsets by lookback
// instead of the offsets pre-pass).
struct Tuning {
    bool staged_compress = true;
    bool staged_decompress = true;
    bool staged_compress_loads = true;
    bool pipe_compress = true;  // persistent compression with asynchronous LDS prefetch
    int pipe_waves = 9;         // pipelined compression: data waves per workgroup (1, 2, 4, 8), or 9 / 7:
                                // 8 / 7 data waves and a control wave (compress_ctrl_kernel)
    int dec_waves = 0;          // waves per workgroup of the lookback decoder (4, 8, 16; 0: by size)
    uint64_t dec_wide_above = 1ull << 21;  // by size: 16 waves above this many decoded elements, else 8
                                           // (tile configurations: 16, else 4)
    int grid_factor = 1;
    double prezero_min_cr = 0.0;  // whole-field decodes pre-zero above this CR (0: never)
    bool dec_prescan = true;      // whole-field decodes take chunk offsets from a pre-pass (no lookback)
    uint64_t dec_lookback_below = 1ull << 23;      // ... except fields below this many elements (one launch)
    uint64_t cfg_dec_lookback_below = 1ull << 23;  // the same for the tile configurations
    uint64_t dec_direct_below = 1ull << 26;    // pre-pass decodes below this size: one chunk per workgroup
};
const Tuning &tuning();

// Waves per workgroup of the configuration decoder's lookback form for an
// n-element field (the pre-pass form always takes kCfgDecWaves).
inline int cfg_dec_lookback_waves(uint64_t n) { return n > tuning().dec_wide_above ? kCfgDecWideWaves : kCfgDecWaves; }

}  // namespace fsz
