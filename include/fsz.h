/*
 * fsz.h -- C ABI of the MI355X (gfx950) FSZ compressor library, libfsz.so.
 *
 * FSZ is an error-bounded lossy compressor for float32 fields (paper: "FSZ:
 * Breaking the Prediction-Throughput Trade-off in GPU Lossy Compression").
 * Every element x is reconstructed as x' with |x - x'| <= eb (Sec. V-A).
 * The stream is: a 32-byte header, one rate byte per 32-element block
 * (Sec. III-A, "Compressed format"), zero-padded to 16 bytes, then the
 * variable-length data of each 256-element tile (optional inline mean,
 * sign word + bit planes per nonzero-rate block, Sec. IV-C).
 *
 * Conventions for every entry point
 *   - Pointers named d_* are DEVICE pointers (hipMalloc, or a PyTorch CUDA
 *     tensor's data pointer) on the current HIP device.  The caller owns
 *     them; the library never frees or retains them after the call.
 *   - d_in / d_out float arrays need 4-byte alignment; 16-byte alignment
 *     selects vector loads.  Compressed buffers need 4-byte alignment.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *     return a size block the host until the stream has executed them.
 *     Calls on the same stream are ordered; the library keeps one
 *     workspace per (device, stream), so concurrent calls on different
 *     streams are safe, and concurrent calls on the SAME stream from
 *     several host threads are serialized by an internal lock.
 *   - The library allocates its workspace (chunk flags, tickets, result
 *     words, batch job tables) on first use per (device, stream) and grows
 *     it when a larger field or batch arrives; plans own their buffers; it
 *     never allocates on the device otherwise.
 *   - Errors are returned as fsz_status values; nothing is thrown across
 *     the ABI.  Device-detected errors (non-finite input, bound too small,
 *     capacity, corrupt stream) arrive through the final status read.
 */
#ifndef FSZ_H
#define FSZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error-bound modes (Sec. V-A): ABS = absolute bound eb = value; REL = bound
 * relative to the value range, eb = value * (max(x) - min(x)). */
typedef enum { FSZ_ABS = 0, FSZ_REL = 1 } fsz_eb_mode;

typedef enum {
    FSZ_OK = 0,
    FSZ_ERR_INVALID_ARG = 1,   /* bad pointer / mode / value / alignment */
    FSZ_ERR_NONFINITE = 2,     /* input holds NaN or Inf */
    FSZ_ERR_EB_TOO_SMALL = 3,  /* eb below 8 ulp(max|x|): no binary32 grid honours it */
    FSZ_ERR_CAPACITY = 4,      /* output buffer smaller than the stream */
    FSZ_ERR_CORRUPT = 5,       /* stream fails validation */
    FSZ_ERR_SIZE_MISMATCH = 6, /* n differs from the stream's element count */
    FSZ_ERR_DEVICE = 7,        /* a HIP runtime call failed */
    FSZ_ERR_EB_TOO_LARGE = 8,  /* step so large that max|x| + step overflows binary32 */
    FSZ_ERR_TOO_LARGE = 9      /* n beyond the fixed scratch of fsz_compress_noalloc_async */
} fsz_status;

/* Field statistics used to resolve the error bound (written by
 * fsz_field_stats, read by fsz_compress_ex).  flags bit 0 = a non-finite
 * value was seen (then xmin/xmax/maxabs are unspecified). */
typedef struct {
    float xmin;
    float xmax;
    float maxabs;
    uint32_t flags;
} fsz_stats;

/* Outcome of an asynchronous call, written to device memory by the call's
 * kernel when it completes: size = stream bytes written (compress) or read
 * (decompress), status = an fsz_status, epoch = library-internal call tag. */
typedef struct {
    uint64_t size;
    uint32_t status;
    uint32_t epoch;
} fsz_result;

/* Worst-case stream size in bytes for n elements (every block at the
 * format's maximum rate 31, every tile centred):
 * 32 + pad16(ceil(n/32)) + 4*ceil(n/256) + 128*ceil(n/32).  Pure host
 * arithmetic; never fails. */
size_t fsz_compressed_bound(size_t n);

/* Human-readable name of a status value (static string; "unknown status"
 * for values outside the enumeration). */
const char *fsz_status_string(fsz_status status);

/* Value-range pass (needed for REL, Sec. V-A, and for the step tightening
 * in both modes): min, max, max|x| and finiteness of d_in[0..n) into the
 * device struct *d_stats.  Asynchronous: returns after enqueueing on
 * stream.  Errors: FSZ_ERR_INVALID_ARG (NULL pointers with n > 0),
 * FSZ_ERR_DEVICE. */
fsz_status fsz_field_stats(const float *d_in, size_t n, fsz_stats *d_stats, void *stream);

/* Compress d_in[0..n) with bound (mode, value) into d_out[0..out_capacity).
 * Runs the value-range pass, then the single compression kernel (Sec. III-A
 * steps 1-5: quantize + cross-block prediction, four-way evaluation,
 * adaptive select, in-kernel decoupled-lookback offset scan, bit-shuffle
 * encode).  On FSZ_OK, *out_size holds the stream length.  Blocks until the
 * stream finished.  value must be finite and > 0.  out_capacity must be at
 * least 32 + pad16(ceil(n/32)); fsz_compressed_bound(n) always suffices,
 * otherwise FSZ_ERR_CAPACITY may be returned with d_out partly written. */
fsz_status fsz_compress(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                        void *d_out, size_t out_capacity, size_t *out_size, void *stream);

/* As fsz_compress but with field statistics already computed by
 * fsz_field_stats on the same stream (one HBM read of d_in instead of
 * two; lets several bounds reuse one range pass). */
fsz_status fsz_compress_ex(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                           const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                           size_t *out_size, void *stream);

/* Decompress a stream of cmp_size bytes into d_out[0..n) (Sec. III-A,
 * decompression steps 1-5, in one kernel).  n must equal the stream's
 * element count (else FSZ_ERR_SIZE_MISMATCH).  Corrupt streams return
 * FSZ_ERR_CORRUPT; d_out contents are then unspecified.  Blocks until the
 * stream finished. */
fsz_status fsz_decompress(const void *d_cmp, size_t cmp_size, float *d_out, size_t n,
                          void *stream);

/* Asynchronous forms: enqueue the work on `stream` and return at once with
 * the host-side validation status (FSZ_OK, FSZ_ERR_INVALID_ARG,
 * FSZ_ERR_CAPACITY for out_capacity below the rate header, FSZ_ERR_CORRUPT
 * for cmp_size < 32, FSZ_ERR_DEVICE).  The call's outcome appears in the
 * caller-owned device struct *d_result once the stream reaches it; nothing
 * is read back to the host, so these calls can be chained on a stream and
 * issued from a tight loop.  fsz_compress_async runs the value-range pass
 * first when d_stats is NULL, otherwise it reuses *d_stats.  Each call is
 * one kernel launch (two with the range pass). */
fsz_status fsz_compress_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                              const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                              fsz_result *d_result, void *stream);

fsz_status fsz_decompress_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n,
                                fsz_result *d_result, void *stream);

/* Pre-zeroed decompression (Sec. III-A: the decoder clears the output first
 * when the compression ratio is high, so that all-zero data need no
 * decoding): fills d_out[0, n) with +0.0, then decodes, skipping every group
 * of 8 tiles whose blocks all have rate 0 and whose tiles are all uncentred
 * (they decode to +0.0).  The values equal fsz_decompress_async's bit for
 * bit.  Arguments, ownership and errors as fsz_decompress_async; on an
 * error the output holds zeros or partial values.  fsz_decompress and
 * fsz_decompress_async choose this decoder by themselves when
 * 4n / cmp_size exceeds the threshold in the environment variable
 * FSZ_PREZERO_CR (read once; unset or 0: never). */
fsz_status fsz_decompress_prezero_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n,
                                        fsz_result *d_result, void *stream);

/* Allocation-free compression, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, work and stream bytes as
 * fsz_compress_async (d_stats NULL runs the range pass), but the library's
 * scratch words (chunk flags, ticket, range-pass partials and stats) live
 * in one fixed array of device memory, 16,793,856 bytes per device, held
 * from the first call on that device until the process ends; the call
 * itself allocates nothing and enqueues only kernels (no memset or copy
 * nodes), so it may be captured in a graph and replayed.
 * Limit: n <= 2^30 elements, else FSZ_ERR_TOO_LARGE before any device work.
 * Every call on one device shares that array and clears what it uses at
 * its start: calls that overlap on one device (several streams, several
 * host threads, or a graph replayed while another call runs) race and
 * corrupt each other's output; serialize them.  The caller owns d_in,
 * d_stats, d_out and d_result.  Errors: as fsz_compress_async, plus
 * FSZ_ERR_TOO_LARGE; FSZ_ERR_DEVICE if the array's address cannot be
 * found on the current device. */
fsz_status fsz_compress_noalloc_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                      const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                                      fsz_result *d_result, void *stream);

/* Random-access decode: elements [begin, end) of the n-element field that
 * d_cmp[0..cmp_size) holds, into d_out[0 .. end - begin).  Decompression
 * steps 1-5 of Sec. III-A restricted to the tiles that hold the range: the
 * byte offset of the first one is a reduction of the block sizes before it
 * over the rate header (no data bytes before the range are read), then the
 * offset scan and the decode run over the range's tiles only.  The values
 * equal the same elements of a whole-field decode bit for bit.  Checks the
 * header, the range's rate bytes and those before it; unlike a whole-field
 * decode it does not check that the stream's sizes add up to its total.
 * Errors: FSZ_ERR_INVALID_ARG for begin > end, end > n, a null or
 * misaligned pointer, d_result null; then as fsz_decompress_async
 * (result size = the stream's total bytes). */
fsz_status fsz_decompress_range_async(const void *d_cmp, size_t cmp_size, size_t n, size_t begin, size_t end,
                                      float *d_out, fsz_result *d_result, void *stream);

/* ------------------------------------------------------------------------
 * Feature switches (the ablation of Sec. VI-B, Table IV): compression with a
 * subset of the method's three prediction designs.  0 is the base the paper
 * starts from (first-order Lorenzo on independent 32-element blocks, no
 * centering); FSZ_FEATURES_ALL is the full method, i.e. what every other
 * entry point does.
 *   FSZ_FEAT_CROSS_BLOCK  prediction state carried across the 8 blocks of a
 *                         tile (Sec. IV-A, Eq. (2)); off: every block starts
 *                         from a zero state (Eq. (1)) and the stream header
 *                         sets flags bit 1, which every decoder here honours
 *   FSZ_FEAT_CENTERING    the tile-mean variants LZ1c / LZ2c (Sec. IV-B)
 *   FSZ_FEAT_LZ2          the second-order variants LZ2 / LZ2c (Sec. IV-B)
 * With independent blocks, centering subtracts the tile mean before every
 * block's prediction.  The reconstruction x' = q E is the
 * same under every setting; only the stream size differs.  Arguments,
 * ownership and errors as fsz_compress_async, plus FSZ_ERR_INVALID_ARG for
 * bits outside FSZ_FEATURES_ALL. */
typedef enum {
    FSZ_FEAT_CROSS_BLOCK = 1,
    FSZ_FEAT_CENTERING = 2,
    FSZ_FEAT_LZ2 = 4,
    FSZ_FEATURES_ALL = 7
} fsz_feature;

fsz_status fsz_compress_features_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                       const fsz_stats *d_stats, unsigned features, void *d_out,
                                       size_t out_capacity, fsz_result *d_result, void *stream);

/* The naive five-read baseline the paper measures its single-pass evaluation
 * against (Sec. V-C, Fig. 6): four evaluation passes, one per variant (LZ1,
 * LZ2, LZ1c, LZ2c), each reading the whole input and writing per-tile costs
 * and block rates to library-owned device tables (53 bytes per 256-element
 * tile, grown on demand), then an encode pass that reads the input a fifth
 * time, selects from the tables and encodes.  The stream is byte-identical
 * to fsz_compress_async's; it exists to measure what the single pass saves.
 * Five kernel launches (six with the range pass when d_stats is NULL).
 * Arguments, ownership and errors as fsz_compress_async. */
fsz_status fsz_compress_five_read_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                        const fsz_stats *d_stats, void *d_out, size_t out_capacity,
                                        fsz_result *d_result, void *stream);

/* ------------------------------------------------------------------------
 * Tile configurations (the sweep of Sec. VI-C, Table V): block size
 * `block` in {32, 64} elements and `tile_blocks` in {4, 8, 16} blocks per
 * tile (a tile of block * tile_blocks elements).  32 / 8 is the default, the
 * only configuration the other entry points use.  The full method (all three
 * features) with the tile geometry changed:
 *   - one rate byte per block; the cross-block prediction chain, the tile
 *     mean (pairwise binary32 sum of the block * tile_blocks slots times
 *     1 / (block * tile_blocks)) and the four-way selection span the tile;
 *   - a 64-element block stores its sign map and each bit plane as one
 *     64-bit word, element i at bit 63 - i, most-significant byte first
 *     (block cost 8 + 8r bytes for rate r > 0);
 *   - the stream header records the configuration in flags bits 2-4 (bit 2:
 *     block 64; bits 3-4: 0 for 8 blocks per tile, 1 for 4, 2 for 16), which
 *     are zero for 32 / 8, so the default configuration gives exactly the
 *     stream of fsz_compress_async.
 * The reconstruction x' = q E does not depend on the configuration.  These
 * calls run the same kernels for every configuration, 32 / 8 included: a
 * lane per 32 elements; compression of a 16-byte aligned input by the
 * pipelined persistent kernel of the default path (chunks of 16384
 * elements), other inputs one chunk of 32768 elements per workgroup;
 * decompression one chunk of 8192 elements per workgroup (32768 in the
 * lookback form of fields above 2^21 elements), its offset from a pre-pass
 * over the rate header for fields of 2^23 elements or more.
 *
 * fsz_compressed_bound_config: worst-case stream size (every block at rate
 *   31); 0 for an unsupported configuration.
 * fsz_compress_config_async: arguments, ownership and errors as
 *   fsz_compress_async, plus FSZ_ERR_INVALID_ARG for an unsupported
 *   configuration; FSZ_ERR_CAPACITY for out_capacity below the header and
 *   rate bytes (32 + ceil(n / block) rounded up to 16).
 * fsz_decompress_config_async: decodes a stream of that configuration;
 *   arguments and errors as fsz_decompress_async.  A stream whose header
 *   names another configuration is FSZ_ERR_CORRUPT, as is a configuration
 *   stream handed to fsz_decompress / fsz_decompress_async. */
size_t fsz_compressed_bound_config(size_t n, int block, int tile_blocks);

fsz_status fsz_compress_config_async(const float *d_in, size_t n, fsz_eb_mode mode, double value,
                                     const fsz_stats *d_stats, int block, int tile_blocks, void *d_out,
                                     size_t out_capacity, fsz_result *d_result, void *stream);

fsz_status fsz_decompress_config_async(const void *d_cmp, size_t cmp_size, float *d_out, size_t n, int block,
                                       int tile_blocks, fsz_result *d_result, void *stream);

/* ------------------------------------------------------------------------
 * Batched form: many fields of uneven sizes in one launch.
 *
 * Every job produces exactly the bytes (compress) or floats (decompress)
 * that the plain call with the same arguments produces; only the launch
 * differs.  A batch runs as three kernels on the stream: a segmented
 * value-range pass over all compress jobs, a per-job fold of that pass, and
 * one kernel that takes (job, chunk) work items from a single ticket counter
 * in job order, each chunk following Sec. III-A steps 1-5 (compress) or
 * decompression steps 1-5, with one decoupled-lookback chain (Sec. IV-D) per
 * job.  That kernel is a persistent pipeline (the single-field kernels'
 * prefetch and overlap, across job boundaries) when every job compresses
 * from a 16-byte aligned input or every job decompresses, and one work item
 * per workgroup otherwise.
 *
 * Jobs of one batch must not write memory that another job of the same batch
 * reads or writes.  Per-job errors (non-finite input, bound too small,
 * capacity, corrupt stream) arrive in that job's *d_result and do not affect
 * the other jobs.
 * ------------------------------------------------------------------------ */
typedef enum { FSZ_OP_COMPRESS = 0, FSZ_OP_DECOMPRESS = 1 } fsz_op;

typedef struct {
    int op;               /* fsz_op */
    const void *d_src;    /* compress: const float[n]; decompress: the stream */
    size_t src_size;      /* decompress: stream bytes (>= 32); compress: ignored */
    void *d_dst;          /* compress: stream buffer; decompress: float[n] */
    size_t dst_capacity;  /* compress: stream buffer bytes (as out_capacity of
                             fsz_compress); decompress: ignored */
    size_t n;             /* element count of the float field */
    int mode;             /* compress: fsz_eb_mode */
    double value;         /* compress: bound value (finite, > 0) */
    fsz_result *d_result; /* outcome of the job (device memory, caller-owned) */
} fsz_job;

/* Launch shape of the batched kernel.  waves_per_group in {2, 4, 8} (a
 * workgroup owns 8 tiles per wave); groups_per_cu caps resident workgroups
 * per CU through extra LDS (0 = no cap, else 1..8; a cap that the kernel's
 * own LDS or the device's per-workgroup LDS limit makes void or impossible
 * is rejected as FSZ_ERR_INVALID_ARG; the pipelined compress-only kernel,
 * whose own LDS already allows few workgroups per CU, treats such a cap as
 * no cap).  Neither changes any output byte. */
typedef struct {
    int waves_per_group;
    int groups_per_cu;
} fsz_tuning;

/* Enqueue one batch on `stream` and return.  tuning NULL = the shape the
 * autotuner cached for this batch's size class, else the default {4, 0}.
 * Host-side errors: FSZ_ERR_INVALID_ARG (NULL jobs with njobs > 0, an
 * invalid job or tuning), FSZ_ERR_CAPACITY (a compress job whose capacity is
 * below its rate header), FSZ_ERR_CORRUPT (a decompress job with src_size <
 * 32), FSZ_ERR_DEVICE; then nothing is enqueued.  The job table is copied,
 * so `jobs` may be reused when the call returns. */
fsz_status fsz_batch_async(const fsz_job *jobs, size_t njobs, const fsz_tuning *tuning, void *stream);

/* Autotuner: runs the batch under every supported shape (`reps` timed runs
 * each, HIP events on `stream`), stores the fastest in the process-wide
 * cache for the batch's size class (and in the file named by the
 * FSZ_TUNE_CACHE environment variable, if set), and returns it in *best.
 * The jobs' outputs are written (identically) by every run.  Blocks. */
fsz_status fsz_autotune(const fsz_job *jobs, size_t njobs, int reps, void *stream, fsz_tuning *best);

/* A plan is a fixed batch captured once in a HIP graph: its job table,
 * flags and range-pass scratch live in plan-owned device memory, and
 * fsz_plan_launch replays the graph (three kernel nodes, no host work per
 * replay).  Buffers named by the jobs must stay valid for the plan's life.
 * Launches of one plan are ordered only if they share a stream; a plan must
 * not run concurrently with itself.  tuning NULL = as fsz_batch_async. */
typedef struct fsz_plan fsz_plan;
fsz_status fsz_plan_create(const fsz_job *jobs, size_t njobs, const fsz_tuning *tuning, fsz_plan **plan);
fsz_status fsz_plan_launch(fsz_plan *plan, void *stream);
fsz_status fsz_plan_get_tuning(const fsz_plan *plan, fsz_tuning *out);
void fsz_plan_destroy(fsz_plan *plan);

/* ------------------------------------------------------------------------
 * Served form: a request loop with admission by memory and continuous
 * batching (one device, one process).
 *
 * A server owns a worker thread, a device arena of `hbm_budget` bytes for job
 * outputs, and `rounds_in_flight` HIP streams.  Requests may be submitted
 * ahead of time: each carries its arrival time on the fsz_server_now_ns
 * clock and counts as arrived once that time has passed.  Arrived requests
 * are admitted in arrival order as soon as their output reservation fits in
 * the arena: fsz_compressed_bound(n) bytes for a compression, 4n for a
 * decompression (a request larger than the whole budget completes at once
 * with FSZ_ERR_CAPACITY).  Admitted requests are folded into one batched
 * launch (as fsz_batch_async) on the next idle stream, so requests that
 * arrive while earlier rounds run are launched beside them and overlap on
 * the device.  Inputs stay where the caller put them (device memory that
 * must remain valid until the request completes); outputs live in the
 * arena until released.  Every result equals the plain call's.
 * ------------------------------------------------------------------------ */
typedef struct fsz_server fsz_server;

typedef struct {
    size_t hbm_budget;      /* bytes of device memory for outputs (> 0) */
    int max_jobs_per_round; /* jobs folded into one launch, 1..65536 */
    int rounds_in_flight;   /* launches in flight, one HIP stream each, 1..16 */
    int auto_release;       /* nonzero: free a job's output when it completes
                               (its bytes are then not kept; size and status
                               are still reported) */
    fsz_tuning tuning;      /* launch shape; {0, 0} = {4, 0} */
} fsz_server_config;

typedef struct {
    int op;               /* fsz_op */
    const void *d_src;    /* compress: const float[n]; decompress: the stream */
    size_t src_size;      /* decompress: stream bytes; compress: ignored */
    size_t n;             /* element count of the float field */
    int mode;             /* compress: fsz_eb_mode */
    double value;         /* compress: bound value */
    uint64_t tag;         /* caller's identifier, returned in the completion */
    uint64_t arrival_ns;  /* arrival time on the fsz_server_now_ns clock */
} fsz_request;

typedef struct {
    uint64_t tag;
    uint32_t status;      /* fsz_status of the job */
    uint32_t op;
    uint64_t size;        /* stream bytes written (compress) or read (decompress) */
    void *d_out;          /* server-owned output (stream or floats); NULL when
                             auto_release is set or the job failed */
    uint64_t arrival_ns;  /* as submitted */
    uint64_t admit_ns;    /* output reserved in the arena */
    uint64_t launch_ns;   /* its round was enqueued */
    uint64_t complete_ns; /* the worker saw its round finish */
} fsz_completion;

typedef struct {
    uint64_t submitted, completed, rounds;
    uint64_t max_jobs_in_round;
    uint64_t max_rounds_overlapping; /* most rounds in flight at once */
    size_t hbm_in_use, hbm_peak;     /* arena bytes reserved now / at most */
} fsz_server_stats;

/* Monotonic clock (nanoseconds) used for arrival and completion times. */
uint64_t fsz_server_now_ns(void);

/* Create a server on the current device.  Errors: FSZ_ERR_INVALID_ARG (bad
 * config), FSZ_ERR_DEVICE (allocation of the arena or streams failed). */
fsz_status fsz_server_create(const fsz_server_config *cfg, fsz_server **server);

/* Queue `count` requests (thread-safe; returns at once).  Every request is
 * validated first (as fsz_batch_async validates jobs); on an error nothing
 * is queued. */
fsz_status fsz_server_submit(fsz_server *server, const fsz_request *reqs, size_t count);

/* Move up to `max` completions into out[], waiting up to wait_ms
 * milliseconds for the first one (0 = do not wait).  Returns the count. */
size_t fsz_server_poll(fsz_server *server, fsz_completion *out, size_t max, int wait_ms);

/* Return a completion's output to the arena (d_out as reported). */
fsz_status fsz_server_release(fsz_server *server, void *d_out);

fsz_status fsz_server_get_stats(fsz_server *server, fsz_server_stats *out);

/* Wait for every submitted request to complete, then free the server and
 * every output it still holds. */
void fsz_server_destroy(fsz_server *server);

#ifdef __cplusplus
}
#endif
#endif /* FSZ_H */
