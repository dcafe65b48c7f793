// FSZ compression / decompression kernels for MI355X (gfx950, CDNA4, wave64).
//
// Data layout on the GPU (the format itself is fixed by Sec. III-A / IV-C):
//   - one lane owns one 32-element block; lanes 8t..8t+7 of a wave own the
//     8 blocks of one 256-element tile, so a wave64 holds 8 tiles;
//   - a workgroup of kWaves waves owns a chunk of 8*kWaves consecutive
//     tiles; chunk ids come from an atomic ticket so that the decoupled
//     lookback (Sec. IV-D) only ever waits on chunks already running;
//   - HBM is read once with coalesced 16-byte loads, transposed through LDS
//     into the lane-per-block layout, and kept in VGPRs across the lookback
//     (the paper's kernel re-reads its input for the encode pass instead);
//   - the cross-block prediction state (Sec. IV-A, Eq. (2)) moves between
//     the lanes of a tile with one DPP row shift per block;
//   - per-tile reductions (mean, costs) use DPP within 8-lane groups.
//
// Floating point: compiled with -ffp-contract=off; the quantizer is one
// binary32 multiply and a round-half-even (v_mul_f32, v_rndne_f32), the
// dequantizer one int->float conversion and one multiply.
#include "fsz_internal.h"

#include <float.h>

namespace fsz {
namespace {

// ------------------------------------------------------------------ lanes

constexpr int kQuadXor1 = 0xB1;       // quad_perm:[1,0,3,2]
constexpr int kQuadXor2 = 0x4E;       // quad_perm:[2,3,0,1]
constexpr int kRowShr1 = 0x111;
constexpr int kRowShr2 = 0x112;
constexpr int kRowShr4 = 0x114;
constexpr int kRowShr8 = 0x118;
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ float dppf(float v)
{
    return __int_as_float(dpp<CTRL>(__float_as_int(v)));
}

// value of lane 8*(lane/8) (block 0 of the lane's tile)
__device__ __forceinline__ int group_head(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, 0x0018);
}

// sum over the 8 lanes of a tile, result in all 8 lanes
__device__ __forceinline__ int group_sum(int v)
{
    v += dpp<kQuadXor1>(v);
    v += dpp<kQuadXor2>(v);
    v += dpp<kRowHalfMirror>(v);
    return v;
}

// exclusive prefix over the 8 lanes of a tile (j = lane & 7)
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t v, int j)
{
    uint32_t s = v;
    uint32_t t = (uint32_t)dpp<kRowShr1>((int)s);
    s += j >= 1 ? t : 0u;
    t = (uint32_t)dpp<kRowShr2>((int)s);
    s += j >= 2 ? t : 0u;
    t = (uint32_t)dpp<kRowShr4>((int)s);
    s += j >= 4 ? t : 0u;
    return s - v;
}

// inclusive prefix over the 64 lanes of the wave
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += dpp<kRowShr1>(v);
    v += dpp<kRowShr2>(v);
    v += dpp<kRowShr4>(v);
    v += dpp<kRowShr8>(v);
    v += dpp<kRowBcast15, 0xA>(v);
    v += dpp<kRowBcast31, 0xC>(v);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ uint32_t uabs(int v) { return v < 0 ? 0u - (uint32_t)v : (uint32_t)v; }

// number of significant bits = ceil(log2(v + 1)) (the rate of Sec. IV-A)
__device__ __forceinline__ uint32_t bitlen(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }

// Eq. (3): zero-rate blocks cost nothing, else a sign word and r planes
__device__ __forceinline__ uint32_t block_bytes(uint32_t r) { return r ? 4u + 4u * r : 0u; }

__device__ __forceinline__ uint32_t bswap32(uint32_t v) { return __builtin_bswap32(v); }

// ------------------------------------------------------------------ results

// The call's outcome, written once per launch by the workgroup that owns the
// last chunk (it sees the inclusive prefix, hence every chunk's error bit).
__device__ __forceinline__ void write_final(fsz_result *final, uint64_t size, uint32_t status, uint32_t epoch)
{
    final->size = status == FSZ_OK ? size : 0;
    final->status = status;
    final->epoch = epoch;
}

// ------------------------------------------------------------------ bound

struct Resolved {
    float E, inv;
    uint32_t flags;
    int status;
};

// binary32 spacing at magnitude m, from its exponent field
__device__ __forceinline__ double spacing32(float m)
{
    uint32_t e = (__float_as_uint(m) >> 23) & 0xFFu;
    int p = e == 0 ? -149 : (int)e - 150;
    return __longlong_as_double((long long)(p + 1023) << 52);
}

// d (> 0) to binary32, rounding toward zero
__device__ __forceinline__ float f32_toward_zero(double d)
{
    float f = (float)d;
    if ((double)f > d) f = __uint_as_float(__float_as_uint(f) - 1u);
    return f;
}

// Error-bound resolution (Sec. V-A) with the binary32 step tightening:
// eb_q = eb - 4 ulp(max|x|), E = 2 eb_q rounded toward zero, inv = 1/E.
__device__ Resolved resolve_bound(const fsz_stats *stp, int mode, double value, uint64_t n)
{
    Resolved r{1.0f, 1.0f, 0u, FSZ_OK};
    if (n == 0) return r;
    const fsz_stats s = *stp;
    if (s.flags & 1u) {
        r.status = FSZ_ERR_NONFINITE;
        return r;
    }
    float E;
    if (mode == FSZ_REL && s.xmax == s.xmin) {
        const float c = fabsf(s.xmin);
        if (c == 0.0f) {
            E = 1.0f;
        } else if (c < FLT_MIN) {
            r.status = FSZ_ERR_EB_TOO_SMALL;
            return r;
        } else {
            E = c;
        }
        r.flags = 1;
    } else {
        const double eb = mode == FSZ_REL ? value * ((double)s.xmax - (double)s.xmin) : value;
        const double u = spacing32(s.maxabs);
        if (!(eb >= 8.0 * u)) {
            r.status = FSZ_ERR_EB_TOO_SMALL;
            return r;
        }
        const double ebq = eb - 4.0 * u;
        E = f32_toward_zero(2.0 * ebq);
        if (E > 0x1p126f) E = 0x1p126f;
        if (E < FLT_MIN) {
            r.status = FSZ_ERR_EB_TOO_SMALL;
            return r;
        }
        if ((double)s.maxabs + (double)E > (double)FLT_MAX) {
            r.status = FSZ_ERR_EB_TOO_LARGE;
            return r;
        }
    }
    r.E = E;
    r.inv = 1.0f / E;
    return r;
}

// ------------------------------------------------------------------ lookback

constexpr uint32_t kLookbackSpinLimit = 1u << 22;

// Chunk id from the launch's ticket counter; the workgroup that takes the
// last ticket resets the counter for the next launch on the stream.
__device__ __forceinline__ unsigned long long take_ticket(unsigned long long *ticket, uint64_t nchunks)
{
    const unsigned long long t = atomicAdd(ticket, 1ull);
    if (t == nchunks - 1)
        __hip_atomic_store(ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return t;
}

__device__ __forceinline__ unsigned long long pack_flag(uint64_t state, uint32_t ep, bool err, uint64_t v)
{
    return (state << 62) | ((uint64_t)ep << kEpochShift) | ((uint64_t)err << kErrorBit) | (v & kValueMask);
}

// Decoupled lookback (Sec. IV-D, three-state flags) run by one whole wave:
// publishes this chunk's aggregate, sums predecessors' aggregates 64 at a
// time until an inclusive prefix is found, publishes the inclusive prefix
// and returns the exclusive one.  Each flag word also carries an error bit
// that is OR-ed along the prefix, so the last chunk learns whether any chunk
// failed.  Flags are plain relaxed agent-scope atomics (coherent across the
// 8 XCDs' L2s, no cache-flushing fences): the value travels inside the flag
// word, so no other memory needs ordering.  The spin is bounded so that every
// wave exits even if the protocol were broken (*err is then set).
struct Prefix {
    uint64_t excl;
    bool err;
};

__device__ Prefix lookback(unsigned long long *flags, uint64_t chunk, uint32_t ep, uint64_t total, bool err)
{
    const int lane = __lane_id();
    if (chunk == 0) {
        if (lane == 0)
            __hip_atomic_store(&flags[0], pack_flag(kFlagInclusive, ep, err, total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        return Prefix{0, err};
    }
    if (lane == 0)
        __hip_atomic_store(&flags[chunk], pack_flag(kFlagAggregate, ep, err, total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    bool perr = false;
    long long pos = (long long)chunk - 1;
    for (uint32_t spins = 0;; spins++) {
        if (spins >= kLookbackSpinLimit) {  // a predecessor never published: give up
            perr = true;
            break;
        }
        const long long idx = pos - lane;
        unsigned long long f;
        if (idx >= 0)
            f = __hip_atomic_load(&flags[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            f = pack_flag(kFlagInclusive, ep, false, 0);
        const bool current = (uint32_t)((f >> kEpochShift) & kEpochMask) == ep;
        const uint32_t state = current ? (uint32_t)(f >> 62) : 0u;
        const unsigned long long not_ready = __ballot(state == 0);
        const unsigned long long incl = __ballot(state == kFlagInclusive);
        const uint64_t v = f & kValueMask;
        const bool e = (f >> kErrorBit) & 1ull;
        if (incl != 0) {
            const int first = __builtin_ctzll(incl);
            const unsigned long long need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
            if ((not_ready & need) == 0) {
                excl += wave_sum_u64(lane <= first ? v : 0);
                perr = perr || (__ballot(lane <= first && e) != 0);
                break;
            }
        } else if (not_ready == 0) {
            excl += wave_sum_u64(v);
            perr = perr || (__ballot(e) != 0);
            pos -= 64;
            continue;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    err = err || perr;
    if (lane == 0)
        __hip_atomic_store(&flags[chunk], pack_flag(kFlagInclusive, ep, err, excl + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return Prefix{excl, err};
}

// ------------------------------------------------------------------ staging

// Loads the wave's 8 tiles (2048 floats starting at element e0) with
// coalesced loads and hands lane L the 32 floats of block L via LDS.
// Elements at or beyond n read as +0.
template <bool ALIGNED>
__device__ __forceinline__ void load_blocks(const float *__restrict__ x, uint64_t n, uint64_t e0,
                                            uint32_t *st, int lane, float (&v)[32])
{
    const bool full = e0 + 2048 <= n;
    if (ALIGNED) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int p = k * 64 + lane;  // 16-byte piece of the wave's 8 KiB
            const uint64_t e = e0 + 4ull * p;
            float4 f;
            if (full || e + 4 <= n) {
                f = *reinterpret_cast<const float4 *>(x + e);
            } else {
                f.x = e + 0 < n ? x[e + 0] : 0.0f;
                f.y = e + 1 < n ? x[e + 1] : 0.0f;
                f.z = e + 2 < n ? x[e + 2] : 0.0f;
                f.w = e + 3 < n ? x[e + 3] : 0.0f;
            }
            *reinterpret_cast<float4 *>(st + (p >> 3) * kStageRowDwords + (p & 7) * 4) = f;
        }
    } else {
#pragma unroll 8
        for (int k = 0; k < 32; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = e0 + p;
            const float f = (full || e < n) ? x[e] : 0.0f;
            st[(p >> 5) * kStageRowDwords + (p & 31)] = __float_as_uint(f);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const float4 f = *reinterpret_cast<const float4 *>(st + lane * kStageRowDwords + k * 4);
        v[4 * k + 0] = f.x;
        v[4 * k + 1] = f.y;
        v[4 * k + 2] = f.z;
        v[4 * k + 3] = f.w;
    }
}

// ------------------------------------------------------------------ stats

__device__ __forceinline__ void stats_combine(float &mn, float &mx, float &ma, uint32_t &nf, const StatsPartial &p)
{
    mn = fminf(mn, p.xmin);
    mx = fmaxf(mx, p.xmax);
    ma = fmaxf(ma, p.maxabs);
    nf |= p.flags;
}

// block-wide reduction of (min, max, max|x|, non-finite); result in thread 0
__device__ StatsPartial stats_block_reduce(float mn, float mx, float ma, uint32_t nf)
{
    for (int m = 32; m >= 1; m >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, m));
        mx = fmaxf(mx, __shfl_xor(mx, m));
        ma = fmaxf(ma, __shfl_xor(ma, m));
        nf |= __shfl_xor(nf, m);
    }
    __shared__ StatsPartial wsum[kStatsThreads / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = StatsPartial{mn, mx, ma, nf};
    __syncthreads();
    StatsPartial p = wsum[0];
    for (int k = 1; k < kStatsThreads / 64; k++) stats_combine(p.xmin, p.xmax, p.maxabs, p.flags, wsum[k]);
    return p;
}

// Value-range pass, part 1: one partial (min, max, max|x|, non-finite) per
// workgroup over a grid-stride slice of x.
template <bool ALIGNED>
__global__ __launch_bounds__(kStatsThreads) void stats_partial_kernel(StatsArgs a)
{
    float mn = INFINITY, mx = -INFINITY, ma = 0.0f;
    uint32_t nonfinite = 0;
    auto take = [&](float v) {
        if (__builtin_isfinite(v)) {
            mn = fminf(mn, v);
            mx = fmaxf(mx, v);
            ma = fmaxf(ma, fabsf(v));
        } else {
            nonfinite = 1;
        }
    };
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    if (ALIGNED) {
        const uint64_t nvec = a.n / 4;
        const float4 *x4 = reinterpret_cast<const float4 *>(a.x);
        for (uint64_t i = tid; i < nvec; i += nthreads) {
            const float4 f = x4[i];
            take(f.x);
            take(f.y);
            take(f.z);
            take(f.w);
        }
        for (uint64_t i = nvec * 4 + tid; i < a.n; i += nthreads) take(a.x[i]);
    } else {
        for (uint64_t i = tid; i < a.n; i += nthreads) take(a.x[i]);
    }
    const StatsPartial p = stats_block_reduce(mn, mx, ma, nonfinite);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = p;
}

// Value-range pass, part 2: one workgroup folds the partials into *out.
__global__ __launch_bounds__(kStatsThreads) void stats_final_kernel(StatsArgs a, unsigned nparts)
{
    float mn = INFINITY, mx = -INFINITY, ma = 0.0f;
    uint32_t nf = 0;
    for (unsigned i = threadIdx.x; i < nparts; i += blockDim.x) stats_combine(mn, mx, ma, nf, a.partials[i]);
    const StatsPartial p = stats_block_reduce(mn, mx, ma, nf);
    if (threadIdx.x == 0) *a.out = fsz_stats{p.xmin, p.xmax, p.maxabs, p.flags};
}

// ------------------------------------------------------------------ compress

// Compression kernel: Sec. III-A steps 1-5 in one launch.
//   1 quantize + cross-block LZ1/LZ2 residuals (Sec. IV-A, Eq. (2))
//   2 four-way evaluation (Sec. IV-B, Eq. (3)-(4)): blocks 1..7 have one rate
//     per order; block 0 is re-rated per variant from q0, q1 - 2 q0 and mu
//   3 adaptive select (strict minimum in the order LZ1, LZ2, LZ1c, LZ2c)
//     and the rate header
//   4 chunk offsets by decoupled lookback (Sec. IV-D)
//   5 fixed-length sign / bit-plane encoding (Sec. IV-C), staged in LDS and
//     written with coalesced stores
template <bool ALIGNED>
__global__ __launch_bounds__(kThreads) void compress_kernel(CompressArgs a)
{
    __shared__ __attribute__((aligned(16))) uint32_t stage[kWaves * kStageWaveDwords];
    __shared__ uint32_t s_wave_total[kWaves];
    __shared__ unsigned long long s_chunk, s_base;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;  // block within the tile

    if (tid == 0) s_chunk = take_ticket(a.ticket, a.nchunks);
    __syncthreads();
    const uint64_t chunk = s_chunk;
    if (chunk >= a.nchunks) return;  // inconsistent ticket counter: never index past the flags

    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {
        if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        return;
    }

    const uint64_t tile0 = chunk * kTilesPerChunk + (uint64_t)w * kTilesPerWave;
    const uint64_t tile = tile0 + (lane >> 3);
    const bool tile_ok = tile < a.ntiles;
    const uint64_t eblk = tile * kTile + (uint64_t)j * kBlock;
    const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
    uint32_t *st = stage + w * kStageWaveDwords;

    float x[32];
    if (tile0 < a.ntiles) {
        load_blocks<ALIGNED>(a.x, a.n, tile0 * kTile, st, lane, x);
    } else {
#pragma unroll
        for (int i = 0; i < 32; i++) x[i] = 0.0f;
    }

    // ---- tile mean: index-order pairwise binary32 tree over the 256 slots
    float s16[16];
#pragma unroll
    for (int i = 0; i < 16; i++) s16[i] = x[2 * i] + x[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 8; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 2; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
    float ts = s16[0] + s16[1];
    ts = ts + dppf<kQuadXor1>(ts);      // blocks (0,1) (2,3) ...
    ts = ts + dppf<kQuadXor2>(ts);      // (0-1, 2-3) ...
    ts = ts + dppf<kRowHalfMirror>(ts); // (0-3, 4-7)
    const float mean_q = (ts * 0x1p-8f) * R.inv;
    const bool centre_ok = __builtin_isfinite(mean_q);
    const int mu = centre_ok ? (int)__builtin_rintf(mean_q) : 0;

    // ---- quantize (Sec. IV-B): q = rint(x * inv)
    int q[32];
#pragma unroll
    for (int i = 0; i < 32; i++) q[i] = (int)__builtin_rintf(x[i] * R.inv);

    // ---- cross-block state: last q and last LZ1 residual of block j-1
    int t0 = dpp<kRowShr1>(q[31]);
    int t1 = dpp<kRowShr1>(q[31] - q[30]);
    const int carry_q = j ? t0 : 0;
    const int carry_l1 = j ? t1 : 0;

    // ---- residuals and their extrema (block 0 keeps its first residuals aside)
    int mx1 = INT_MIN, mn1 = INT_MAX, mx2 = INT_MIN, mn2 = INT_MAX;
    int l2_1 = 0;
    {
        int pq = carry_q, pl = carry_l1;
#pragma unroll
        for (int i = 0; i < 32; i++) {
            int l1 = q[i] - pq;
            int l2 = l1 - pl;
            pq = q[i];
            pl = l1;
            if (i >= cnt) {
                l1 = 0;
                l2 = 0;
            }
            if (i == 1) l2_1 = l2;
            const bool in1 = i >= 1 || j != 0;
            const bool in2 = i >= 2 || j != 0;
            if (in1) {
                mx1 = max(mx1, l1);
                mn1 = min(mn1, l1);
            }
            if (in2) {
                mx2 = max(mx2, l2);
                mn2 = min(mn2, l2);
            }
        }
    }
    const uint32_t a1 = max(uabs(mx1), uabs(mn1));
    const uint32_t a2 = max(uabs(mx2), uabs(mn2));
    const uint32_t r1 = bitlen(a1), r2 = bitlen(a2);
    const int T1 = group_sum(j ? (int)block_bytes(r1) : 0);
    const int T2 = group_sum(j ? (int)block_bytes(r2) : 0);

    // ---- four-way evaluation of block 0 and the selection (lane j == 0)
    int dec;
    {
        const int q0 = q[0];
        const int d1 = cnt >= 2 ? l2_1 : 0;  // q1 - 2 q0
        const int c0 = q0 - mu;
        const int c1 = cnt >= 2 ? l2_1 + mu : 0;
        const uint32_t ra = bitlen(max(uabs(q0), a1));
        const uint32_t rb = bitlen(max(max(uabs(q0), uabs(d1)), a2));
        const uint32_t rc = bitlen(max(uabs(c0), a1));
        const uint32_t rd = bitlen(max(max(uabs(c0), uabs(c1)), a2));
        int best = 0;
        uint32_t C = block_bytes(ra) + T1, r0 = ra;
        const uint32_t Cb = block_bytes(rb) + T2;
        if (Cb < C) {
            best = 1;
            C = Cb;
            r0 = rb;
        }
        if (centre_ok) {
            const uint32_t Cc = block_bytes(rc) + T1 + 4;
            const uint32_t Cd = block_bytes(rd) + T2 + 4;
            if (Cc < C) {
                best = 2;
                C = Cc;
                r0 = rc;
            }
            if (Cd < C) {
                best = 3;
                C = Cd;
                r0 = rd;
            }
        }
        dec = (int)((C << 8) | ((uint32_t)(best & 1) << 7) | ((uint32_t)(best >> 1) << 6) | r0);
        if (!tile_ok) dec = 0;
    }
    dec = group_head(dec);
    const int order2 = (dec >> 7) & 1;
    const int cent = (dec >> 6) & 1;
    const uint32_t Z = (uint32_t)dec >> 8;
    const uint32_t r = j == 0 ? (uint32_t)(dec & 31) : (order2 ? r2 : r1);
    if (cnt > 0) a.out[kHeaderBytes + tile * kBlocksPerTile + j] = (uint8_t)(j == 0 ? (dec & 0xFF) : r);
    const uint32_t S = block_bytes(r);

    // ---- offsets inside the wave / chunk
    const int zt = j == 0 ? (int)Z : 0;
    const int incl = wave_incl_scan(zt);
    const uint32_t tile_excl = (uint32_t)incl - Z;
    const uint32_t wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    const uint32_t blk_off = tile_excl + group_excl_scan(S, j) + 4u * cent;
    if (lane == 0) s_wave_total[w] = wave_total;
    __syncthreads();
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) {
        if (k < w) wave_base += s_wave_total[k];
        chunk_total += s_wave_total[k];
    }

    // ---- step 4: device-wide exclusive prefix by decoupled lookback
    if (w == 0) {
        const Prefix pre = lookback(a.flags, chunk, a.flag_epoch, chunk_total, false);
        if (lane == 0) {
            s_base = pre.excl;
            if (chunk == a.nchunks - 1) {
                const uint64_t total = a.data0 + pre.excl + chunk_total;
                uint32_t st = pre.err ? (uint32_t)FSZ_ERR_DEVICE : (uint32_t)FSZ_OK;
                if (st == FSZ_OK && total > a.capacity) st = FSZ_ERR_CAPACITY;
                if (st == FSZ_OK) {
                    uint32_t *h = reinterpret_cast<uint32_t *>(a.out);
                    h[0] = 0x315A5346u;  // "FSZ1"
                    h[1] = 1u | ((uint32_t)a.mode << 16) | (R.flags << 24);
                    h[2] = (uint32_t)a.n;
                    h[3] = (uint32_t)(a.n >> 32);
                    h[4] = __float_as_uint(R.E);
                    h[5] = __float_as_uint((float)a.value);
                    h[6] = (uint32_t)total;
                    h[7] = (uint32_t)(total >> 32);
                    for (uint64_t k = kHeaderBytes + a.nblocks; k < a.data0; k++) a.out[k] = 0;
                }
                write_final(a.final, total, st, a.epoch);
            }
        }
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (a.data0 + base + chunk_total > a.capacity || tile0 >= a.ntiles) return;

    // ---- step 5: encode the selected variant into the wave's LDS region
    if (cnt > 0 && j == 0 && cent) st[tile_excl >> 2] = (uint32_t)mu;
    uint32_t code[32];
    {
        int pq = carry_q, pl = carry_l1;
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const int l1 = q[i] - pq;
            int e = order2 ? l1 - pl : l1;
            pq = q[i];
            pl = l1;
            if (i == 0 && j == 0 && cent) e = q[0] - mu;
            if (i == 1 && j == 0 && cent && order2) e = e + mu;
            if (i >= cnt) e = 0;
            code[i] = (uabs(e) << 1) | ((uint32_t)e >> 31);
        }
    }
    const uint32_t nwords = r ? r + 1 : 0;  // sign word + r planes
    for (uint32_t b = 0; __ballot(b < nwords) != 0; b++) {
        uint32_t word = 0;
#pragma unroll
        for (int i = 0; i < 32; i++) word |= ((code[i] >> b) & 1u) << (31 - i);
        if (b < nwords) st[(blk_off >> 2) + b] = bswap32(word);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    uint32_t *dst = reinterpret_cast<uint32_t *>(a.out + a.data0 + base + wave_base);
    for (uint32_t k = lane; k < (wave_total >> 2); k += 64) dst[k] = st[k];
}

// ------------------------------------------------------------------ decompress

// Decompression kernel: Sec. III-A decompression steps 1-5 in one launch:
// rate bytes -> block and tile sizes -> lookback offsets -> bit-unshuffle
// -> inverse cross-block prediction (one inclusive scan for LZ1, two for
// LZ2, plus the tile mean) -> x' = (float)q * E.
template <bool ALIGNED>
__global__ __launch_bounds__(kThreads) void decompress_kernel(DecompressArgs a)
{
    __shared__ __attribute__((aligned(16))) uint32_t stage[kWaves * kStageWaveDwords];
    __shared__ uint32_t s_wave_total[kWaves];
    __shared__ unsigned long long s_chunk, s_base;
    __shared__ int s_bad;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;

    if (tid == 0) {
        s_chunk = take_ticket(a.ticket, a.nchunks);
        s_bad = 0;
    }
    __syncthreads();
    const uint64_t chunk = s_chunk;
    if (chunk >= a.nchunks) return;  // inconsistent ticket counter: never index past the flags

    // ---- header validation (same for every workgroup)
    const uint32_t *h = reinterpret_cast<const uint32_t *>(a.cmp);
    int hst = FSZ_OK;
    float E = 1.0f;
    uint64_t total = 0;
    {
        const uint32_t h1 = h[1];
        if (h[0] != 0x315A5346u || (h1 & 0xFFFFu) != 1u || ((h1 >> 16) & 0xFFu) > 1u ||
            ((h1 >> 24) & ~1u) != 0u) {
            hst = FSZ_ERR_CORRUPT;
        } else if (((uint64_t)h[3] << 32 | h[2]) != a.n) {
            hst = FSZ_ERR_SIZE_MISMATCH;
        } else {
            E = __uint_as_float(h[4]);
            total = (uint64_t)h[7] << 32 | h[6];
            if (!__builtin_isfinite(E) || !(E > 0.0f) || total > a.cmp_size || total < a.data0)
                hst = FSZ_ERR_CORRUPT;
        }
    }
    if (hst != FSZ_OK) {
        if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, hst, a.epoch);
        return;
    }

    const uint64_t tile0 = chunk * kTilesPerChunk + (uint64_t)w * kTilesPerWave;
    const uint64_t tile = tile0 + (lane >> 3);
    const bool tile_ok = tile < a.ntiles;
    const uint64_t gblock = tile * kBlocksPerTile + j;
    const bool blk_ok = gblock < a.nblocks;

    // ---- steps 1-2: rates, tile metadata, block and tile sizes
    const uint32_t rb = blk_ok ? a.cmp[kHeaderBytes + gblock] : 0u;
    const bool bad = blk_ok && (j == 0 ? (rb & 0x20u) : (rb & 0xE0u)) != 0;
    const uint32_t head = (uint32_t)group_head((int)rb);
    const int order2 = tile_ok ? (int)((head >> 7) & 1u) : 0;
    const int cent = tile_ok ? (int)((head >> 6) & 1u) : 0;
    const uint32_t r = rb & 31u;
    const uint32_t S = block_bytes(r);
    const uint32_t Z = (uint32_t)group_sum((int)S) + 4u * cent;
    const int incl = wave_incl_scan(j == 0 ? (int)Z : 0);
    const uint32_t tile_excl = (uint32_t)incl - Z;
    const uint32_t wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    const uint32_t blk_off = tile_excl + group_excl_scan(S, j) + 4u * cent;
    if (__ballot(bad) != 0 && lane == 0) s_bad = 1;
    if (lane == 0) s_wave_total[w] = wave_total;
    __syncthreads();
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < kWaves; k++) {
        if (k < w) wave_base += s_wave_total[k];
        chunk_total += s_wave_total[k];
    }

    // ---- step 3: offsets by decoupled lookback
    if (w == 0) {
        const Prefix pre = lookback(a.flags, chunk, a.flag_epoch, chunk_total, s_bad != 0);
        if (lane == 0) {
            s_base = pre.excl;
            if (chunk == a.nchunks - 1) {
                bool ok = !pre.err && a.data0 + pre.excl + chunk_total == total;
                for (uint64_t k = kHeaderBytes + a.nblocks; ok && k < a.data0; k++) ok = a.cmp[k] == 0;
                write_final(a.final, total, ok ? (uint32_t)FSZ_OK : (uint32_t)FSZ_ERR_CORRUPT, a.epoch);
            }
        }
    }
    __syncthreads();
    const uint64_t base = s_base;
    if (s_bad || a.data0 + base + chunk_total > total || tile0 >= a.ntiles) return;

    // ---- step 4: decode + bit-unshuffle
    const uint8_t *tile_data = a.cmp + a.data0 + base + wave_base;
    int mu = 0;
    if (cent) mu = (int)*reinterpret_cast<const uint32_t *>(tile_data + tile_excl);
    uint32_t code[32];
#pragma unroll
    for (int i = 0; i < 32; i++) code[i] = 0;
    const uint32_t nwords = (blk_ok && r) ? r + 1 : 0;
    const uint32_t *words = reinterpret_cast<const uint32_t *>(tile_data + blk_off);
    for (uint32_t b = 0; __ballot(b < nwords) != 0; b++) {
        if (b < nwords) {
            const uint32_t word = bswap32(words[b]);
#pragma unroll
            for (int i = 0; i < 32; i++) code[i] |= ((word >> (31 - i)) & 1u) << b;
        }
    }

    // ---- step 5: inverse cross-block prediction + dequantization
    uint32_t d[32];
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const uint32_t m = code[i] >> 1;
        const uint32_t e = (code[i] & 1u) ? 0u - m : m;
        acc += e;
        d[i] = acc;
    }
    const uint32_t start1 = group_excl_scan(acc, j);
#pragma unroll
    for (int i = 0; i < 32; i++) d[i] += start1;
    uint32_t acc2 = 0;
    uint32_t q2[32];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        acc2 += d[i];
        q2[i] = acc2;
    }
    const uint32_t start2 = group_excl_scan(acc2, j);
    float xo[32];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const uint32_t qh = order2 ? q2[i] + start2 : d[i];
        const int qi = (int)(qh + (uint32_t)mu);
        xo[i] = (float)qi * E;
    }

    // ---- write back through LDS with coalesced stores
    uint32_t *st = stage + w * kStageWaveDwords;
#pragma unroll
    for (int k = 0; k < 8; k++)
        *reinterpret_cast<float4 *>(st + lane * kStageRowDwords + 4 * k) =
            make_float4(xo[4 * k], xo[4 * k + 1], xo[4 * k + 2], xo[4 * k + 3]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const uint64_t e0 = tile0 * kTile;
    const bool full = e0 + 2048 <= a.n;
    if (ALIGNED) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = e0 + 4ull * p;
            const float4 f = *reinterpret_cast<const float4 *>(st + (p >> 3) * kStageRowDwords + (p & 7) * 4);
            if (full || e + 4 <= a.n) {
                *reinterpret_cast<float4 *>(a.out + e) = f;
            } else {
                if (e + 0 < a.n) a.out[e + 0] = f.x;
                if (e + 1 < a.n) a.out[e + 1] = f.y;
                if (e + 2 < a.n) a.out[e + 2] = f.z;
            }
        }
    } else {
#pragma unroll 8
        for (int k = 0; k < 32; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = e0 + p;
            if (full || e < a.n) a.out[e] = __uint_as_float(st[(p >> 5) * kStageRowDwords + (p & 31)]);
        }
    }
}

}  // namespace

hipError_t launch_stats(const StatsArgs &a, hipStream_t s)
{
    const uint64_t want = ceil_div(a.n, (uint64_t)kStatsThreads * 16);
    const unsigned grid = (unsigned)(want < 1 ? 1 : (want > kStatsMaxBlocks ? kStatsMaxBlocks : want));
    if ((reinterpret_cast<uintptr_t>(a.x) & 15u) == 0)
        hipLaunchKernelGGL(stats_partial_kernel<true>, dim3(grid), dim3(kStatsThreads), 0, s, a);
    else
        hipLaunchKernelGGL(stats_partial_kernel<false>, dim3(grid), dim3(kStatsThreads), 0, s, a);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(kStatsThreads), 0, s, a, grid);
    return hipGetLastError();
}

hipError_t launch_compress(const CompressArgs &a, bool in_aligned16, hipStream_t s)
{
    if (in_aligned16)
        hipLaunchKernelGGL(compress_kernel<true>, dim3((unsigned)a.nchunks), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(compress_kernel<false>, dim3((unsigned)a.nchunks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_decompress(const DecompressArgs &a, bool out_aligned16, hipStream_t s)
{
    if (out_aligned16)
        hipLaunchKernelGGL(decompress_kernel<true>, dim3((unsigned)a.nchunks), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL(decompress_kernel<false>, dim3((unsigned)a.nchunks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace fsz
