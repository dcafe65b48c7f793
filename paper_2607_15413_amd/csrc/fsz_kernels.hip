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

#include <mutex>

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

// value of lane 8*(lane/8) (block 0 of the lane's tile), in registers: each
// quad takes its first lane, then banks 1 and 3 of every row (lanes 4-7,
// 12-15) take the quad 4 lanes below
__device__ __forceinline__ int group_head(int v)
{
    v = dpp<0x00>(v);  // quad_perm:[0,0,0,0]
    return __builtin_amdgcn_update_dpp(v, v, kRowShr4, 0xF, 0xA, false);
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

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v)
{
    const uint32_t lo = (uint32_t)dpp<CTRL, ROW_MASK>((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)dpp<CTRL, ROW_MASK>((int)(uint32_t)(v >> 32));
    return (unsigned long long)hi << 32 | lo;
}

// sum over the 64 lanes of the wave (register-only prefix, total of lane
// 63); the result is wave-uniform.  Every lane must be active.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    v += dpp64<kRowShr1>(v);
    v += dpp64<kRowShr2>(v);
    v += dpp64<kRowShr4>(v);
    v += dpp64<kRowShr8>(v);
    v += dpp64<kRowBcast15, 0xA>(v);
    v += dpp64<kRowBcast31, 0xC>(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), 63);
    return (unsigned long long)hi << 32 | lo;
}

// Workgroup barrier that orders LDS only: the waves of a workgroup exchange
// data through LDS alone, so outstanding global loads and stores (such as
// the asynchronous copies of a prefetched chunk, which a release fence would
// wait for) stay in flight across it.  The wave's own LDS accesses complete
// before the barrier (lgkmcnt(0)); the memory clobber keeps the compiler
// from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Global-memory views of the hot loads and stores.  Pointers that come out of
// a job table (the batched forms) carry no address space, and the compiler
// accesses them with FLAT instructions, whose waits also cover LDS traffic;
// accesses through these types are plain global loads and stores.
typedef __attribute__((address_space(1))) uint8_t g_u8;
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) float g_f32;
typedef __attribute__((address_space(1))) u32x4 g_u32x4;

// Store of nw dwords from a wave's LDS staging area to global memory at a
// 4-byte aligned address g, by the whole wave: 4-byte stores up to the first
// 16-byte boundary of g and after the last one, 16-byte stores in between (a
// quarter of the store instructions of a dword-wide copy).
__device__ __forceinline__ void wave_store_staged(uint32_t *gp, const uint32_t *st, uint32_t nw, int lane)
{
    g_u32 *g = (g_u32 *)gp;
    const uint32_t head = min(nw, ((16u - ((uint32_t)(uintptr_t)gp & 15u)) & 15u) >> 2);
    if ((uint32_t)lane < head) g[lane] = st[lane];
    const uint32_t nq = (nw - head) >> 2;
    for (uint32_t q = lane; q < nq; q += 64) {
        const uint32_t o = head + 4 * q;
        const u32x4 v = {st[o], st[o + 1], st[o + 2], st[o + 3]};
        *reinterpret_cast<g_u32x4 *>(g + o) = v;
    }
    const uint32_t t0 = head + 4 * nq;
    if ((uint32_t)lane < nw - t0) g[t0 + lane] = st[t0 + lane];
}

// As wave_store_staged, for a staging area laid out at the same 16-byte
// phase as g (st + head is 16-byte aligned): the body is read with one
// 16-byte LDS read per lane (consecutive lanes, consecutive 16 bytes), free of
// bank conflicts.
__device__ __forceinline__ void wave_store_staged_phased(uint32_t *gp, const uint32_t *st, uint32_t nw, int lane)
{
    g_u32 *g = (g_u32 *)gp;
    const uint32_t head = min(nw, ((16u - ((uint32_t)(uintptr_t)gp & 15u)) & 15u) >> 2);
    if ((uint32_t)lane < head) g[lane] = st[lane];
    const uint32_t nq = (nw - head) >> 2;
    for (uint32_t q = lane; q < nq; q += 64) {
        const uint32_t o = head + 4 * q;
        *reinterpret_cast<g_u32x4 *>(g + o) = *reinterpret_cast<const u32x4 *>(st + o);
    }
    const uint32_t t0 = head + 4 * nq;
    if ((uint32_t)lane < nw - t0) g[t0 + lane] = st[t0 + lane];
}

__device__ __forceinline__ uint32_t uabs(int v) { return v < 0 ? 0u - (uint32_t)v : (uint32_t)v; }

// number of significant bits = ceil(log2(v + 1)) (the rate of Sec. IV-A)
__device__ __forceinline__ uint32_t bitlen(uint32_t v) { return v ? 32u - (uint32_t)__builtin_clz(v) : 0u; }

// Eq. (3): zero-rate blocks cost nothing, else a sign word and r planes
__device__ __forceinline__ uint32_t block_bytes(uint32_t r) { return r ? 4u + 4u * r : 0u; }

__device__ __forceinline__ uint32_t bswap32(uint32_t v) { return __builtin_bswap32(v); }

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f4 g_f4;  // global-memory view (see g_u32)

// ------------------------------------------------------------------ bit planes
//
// Bit-shuffle (Sec. IV-C) as an in-register transpose.  A block's residual
// codes c[i] = (|l_i| << 1) | sign_i hold the sign in bit 0 and magnitude bit
// p in bit p + 1, so the block's stored words are exactly the bit planes of
// the codes: word b = bit b of every code (word 0 = sign map, word b = plane
// b - 1).  Stored words are written most-significant byte first, so in the
// little-endian dword element i sits at bit i ^ 7.
//
// Eight planes at a time (byte g of the codes): registers R[rho] take byte g
// of codes 8k + 7 - rho in their byte k; three delta-swap stages exchange the
// register index with the bit-in-byte index, after which R[p] is the stored
// dword of plane word 8g + p.  The same stages invert the mapping on decode.

// byte g of a0..a3 packed into bytes 0..3
__device__ __forceinline__ uint32_t pack_byte_g(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t g)
{
    const uint32_t sel = g | ((4u + g) << 8) | 0x0C0C0000u;
    const uint32_t t01 = __builtin_amdgcn_perm(a1, a0, sel);
    const uint32_t t23 = __builtin_amdgcn_perm(a3, a2, sel);
    return __builtin_amdgcn_perm(t23, t01, 0x05040100u);
}

template <int D, uint32_t M>
__device__ __forceinline__ void delta_swap(uint32_t &lo, uint32_t &hi)
{
    const uint32_t nlo = (M & (hi << D)) | (~M & lo);
    const uint32_t nhi = (M & hi) | (~M & (lo >> D));
    lo = nlo;
    hi = nhi;
}

// swaps the register index (0..7) with the bit-in-byte index of every byte
__device__ __forceinline__ void transpose8(uint32_t (&R)[8])
{
    delta_swap<1, 0xAAAAAAAAu>(R[0], R[1]);
    delta_swap<1, 0xAAAAAAAAu>(R[2], R[3]);
    delta_swap<1, 0xAAAAAAAAu>(R[4], R[5]);
    delta_swap<1, 0xAAAAAAAAu>(R[6], R[7]);
    delta_swap<2, 0xCCCCCCCCu>(R[0], R[2]);
    delta_swap<2, 0xCCCCCCCCu>(R[1], R[3]);
    delta_swap<2, 0xCCCCCCCCu>(R[4], R[6]);
    delta_swap<2, 0xCCCCCCCCu>(R[5], R[7]);
    delta_swap<4, 0xF0F0F0F0u>(R[0], R[4]);
    delta_swap<4, 0xF0F0F0F0u>(R[1], R[5]);
    delta_swap<4, 0xF0F0F0F0u>(R[2], R[6]);
    delta_swap<4, 0xF0F0F0F0u>(R[3], R[7]);
}

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

// a - b (a > b > 0) rounded toward zero in binary64: the round-to-nearest
// difference plus its exact two-sum error term; a negative error means the
// rounding went up, so the result steps one unit down.  Truncated again to
// binary32 it gives the exact difference truncated to binary32.
__device__ __forceinline__ double sub_toward_zero(double a, double b)
{
    double s = a - b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (-b - bb);
    if (e < 0.0) s = __longlong_as_double(__double_as_longlong(s) - 1);
    return s;
}

// Error-bound resolution (Sec. V-A) with the binary32 step tightening:
// E = the largest binary32 <= 2 (eb - 4 ulp(max|x|)), inv = 1/E.
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
        const double ebq = sub_toward_zero(eb, 4.0 * u);
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

// Chunk ids come from the launch's ticket counter, so a chunk is only ever
// owned by a running workgroup and the lookback always makes progress.
// A grid of G workgroups takes `takes` tickets in total (G for one chunk per
// workgroup; nchunks + G for a persistent grid, whose workgroups take tickets
// until one is out of range); the last take resets the counter for the next
// launch on the stream.
__device__ __forceinline__ unsigned long long take_ticket(unsigned long long *ticket, uint64_t takes)
{
    const unsigned long long t = atomicAdd(ticket, 1ull);
    if (t == takes - 1) __hip_atomic_store(ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Publishes this chunk's aggregate (chunk 0 publishes its inclusive prefix).
__device__ __forceinline__ void publish_aggregate(unsigned long long *flags, uint64_t chunk, uint32_t ep,
                                                  uint64_t total, bool err)
{
    __hip_atomic_store(&flags[chunk * kFlagStride], pack_flag(chunk == 0 ? kFlagInclusive : kFlagAggregate, ep, err, total),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for the exclusive prefix of `chunk` (whose aggregate is published)
// and publishes its inclusive prefix.  Run by one whole wave.  A probe reads
// the 64 nearest unresolved predecessors; while one of them is not ready the
// wave re-reads only that single flag word (with a short sleep), so waiting
// chunks add little memory traffic, and then probes the window again.
//
// The caller may read the nearest kProbeWindows windows ahead of time
// (window m, lane l: the flag of chunk - 1 - 64 m - l); the lookback walks
// those values before it issues a load of its own.  A flag that was ready
// when it was read stays valid (an aggregate or an inclusive prefix of this
// launch never changes value); a window read ahead that still shows a word
// not ready is read again before the wave waits on that word.  One window:
// flag words are read across the XCDs' caches at agent scope, and on the
// 512^3 field one more window read ahead per step (walked or not) cost the
// compressor more time than the walks it saved.
constexpr int kProbeWindows = 1;
struct Probe {
    unsigned long long f[kProbeWindows];
};

__device__ __forceinline__ Probe lookback_probe(unsigned long long *flags, uint64_t chunk, uint32_t ep)
{
    Probe p;
#pragma unroll
    for (int m = 0; m < kProbeWindows; m++) {
        const long long idx = (long long)chunk - 1 - 64 * m - __lane_id();
        p.f[m] = idx >= 0 ? __hip_atomic_load(&flags[idx * kFlagStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : pack_flag(kFlagInclusive, ep, false, 0);
    }
    return p;
}

// Makes the probe's loads complete here on every path (an empty asm that
// reads the registers).
__device__ __forceinline__ void consume_probe(const Probe &p)
{
#pragma unroll
    for (int m = 0; m < kProbeWindows; m++) asm volatile("; probe %0" ::"v"(p.f[m]));
}

__device__ Prefix lookback_wait(unsigned long long *flags, uint64_t chunk, uint32_t ep, uint64_t total, bool err,
                                bool has_probe = false, Probe probe = Probe{})
{
    const int lane = __lane_id();
    if (chunk == 0) return Prefix{0, err};
    uint64_t excl = 0;
    bool perr = false;
    long long pos = (long long)chunk - 1;
    uint32_t spins = 0;
    auto state_of = [&](unsigned long long f) -> uint32_t {
        return (uint32_t)((f >> kEpochShift) & kEpochMask) == ep ? (uint32_t)(f >> 62) : 0u;
    };
    int window = has_probe ? 0 : kProbeWindows;  // windows walked so far (read-ahead ones first)
    bool reread = false;                          // read the current window now
    for (;;) {
        const long long idx = pos - lane;
        const bool ahead = window < kProbeWindows && !reread;
        unsigned long long f;
        if (ahead) {
            f = probe.f[0];
#pragma unroll
            for (int m = 1; m < kProbeWindows; m++) f = window == m ? probe.f[m] : f;
        } else {
            f = idx >= 0 ? __hip_atomic_load(&flags[idx * kFlagStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : pack_flag(kFlagInclusive, ep, false, 0);
        }
        const uint32_t state = state_of(f);
        const unsigned long long not_ready = __ballot(state == 0);
        const unsigned long long incl = __ballot(state == kFlagInclusive);
        const uint64_t v = f & kValueMask;
        const bool e = (f >> kErrorBit) & 1ull;
        const unsigned long long need =
            incl ? (__builtin_ctzll(incl) >= 63 ? ~0ull : ((2ull << __builtin_ctzll(incl)) - 1ull)) : ~0ull;
        if ((not_ready & need) == 0) {
            if (incl != 0) {
                const int first = __builtin_ctzll(incl);
                excl += wave_sum_u64(lane <= first ? v : 0);
                perr = perr || (__ballot(lane <= first && e) != 0);
                break;
            }
            excl += wave_sum_u64(v);
            perr = perr || (__ballot(e) != 0);
            pos -= 64;
            window = window < kProbeWindows ? window + 1 : kProbeWindows;
            reread = false;
            continue;
        }
        reread = true;
        if (ahead) continue;  // the read-ahead values are old: read the window first
        // wait on the nearest predecessor that is not ready yet, then read
        // this window again
        const long long widx = pos - __builtin_ctzll(not_ready & need);
        for (;;) {
            if (++spins >= kLookbackSpinLimit) break;
            __builtin_amdgcn_s_sleep(2);
            const unsigned long long g =
                __hip_atomic_load(&flags[widx * kFlagStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (state_of(g) != 0) break;
        }
        if (spins >= kLookbackSpinLimit) {  // a predecessor never published: give up
            perr = true;
            break;
        }
    }
    err = err || perr;
    if (lane == 0)
        __hip_atomic_store(&flags[chunk * kFlagStride], pack_flag(kFlagInclusive, ep, err, excl + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return Prefix{excl, err};
}

// ------------------------------------------------------------------ staging

// Lane-per-block loads straight from HBM: lane L reads its block's 128
// contiguous bytes (8 x 16 B); the wave's 8 loads cover 64 whole blocks.
// Elements at or beyond n read as +0.
template <bool ALIGNED>
__device__ __forceinline__ void load_block(const float *__restrict__ x, uint64_t eblk, int cnt, float (&v)[32])
{
    if (ALIGNED && cnt == 32) {
        const f4 *p = reinterpret_cast<const f4 *>(x + eblk);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const f4 f = __builtin_nontemporal_load(p + k);
            v[4 * k + 0] = f.x;
            v[4 * k + 1] = f.y;
            v[4 * k + 2] = f.z;
            v[4 * k + 3] = f.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 32; i++) v[i] = i < cnt ? x[eblk + i] : 0.0f;
    }
}

// Coalesced loads of the wave's 8 tiles (2048 floats from element e0, 16 B
// per lane per instruction), handed to the lane-per-block layout through LDS
// (rows padded to 36 dwords so that neither side has bank conflicts).
// Elements at or beyond n read as +0.
template <bool ALIGNED>
__device__ __forceinline__ void load_blocks_staged(const float *__restrict__ x, uint64_t n, uint64_t e0, uint32_t *st,
                                                   int lane, float (&v)[32])
{
    const bool full = e0 + 2048 <= n;
    if (ALIGNED) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int p = k * 64 + lane;  // 16-byte piece of the wave's 8 KiB
            const uint64_t e = e0 + 4ull * p;
            f4 f;
            if (full || e + 4 <= n) {
                f = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(x + e));
            } else {
                f.x = e + 0 < n ? x[e + 0] : 0.0f;
                f.y = e + 1 < n ? x[e + 1] : 0.0f;
                f.z = e + 2 < n ? x[e + 2] : 0.0f;
                f.w = e + 3 < n ? x[e + 3] : 0.0f;
            }
            *reinterpret_cast<f4 *>(st + (p >> 3) * kStageRowDwords + (p & 7) * 4) = f;
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
        const f4 f = *reinterpret_cast<const f4 *>(st + lane * kStageRowDwords + k * 4);
        v[4 * k + 0] = f.x;
        v[4 * k + 1] = f.y;
        v[4 * k + 2] = f.z;
        v[4 * k + 3] = f.w;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
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

// Running (min, max, max |x| bit pattern) of a thread.  The largest |x|
// pattern doubles as the finiteness test: it is >= 0x7F800000 exactly when
// an Inf or NaN was seen (min and max are then of no use).
struct RangeAcc {
    float mn = INFINITY, mx = -INFINITY;
    uint32_t ma = 0;
    __device__ __forceinline__ void take(float v)
    {
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
        ma = max(ma, __float_as_uint(v) & 0x7FFFFFFFu);
    }
    __device__ __forceinline__ void take4(const f4 &f)
    {
        mn = fminf(fminf(mn, f.x), fminf(fminf(f.y, f.z), f.w));
        mx = fmaxf(fmaxf(mx, f.x), fmaxf(fmaxf(f.y, f.z), f.w));
        const uint32_t m = 0x7FFFFFFFu;
        ma = max(max(ma, __float_as_uint(f.x) & m),
                 max(max(__float_as_uint(f.y) & m, __float_as_uint(f.z) & m), __float_as_uint(f.w) & m));
    }
    __device__ __forceinline__ StatsPartial reduce() const
    {
        const uint32_t nf = ma >= 0x7F800000u ? 1u : 0u;
        return stats_block_reduce(mn, mx, __uint_as_float(ma & 0x7FFFFFFFu), nf);
    }
};

// Value-range pass, part 1: one partial (min, max, max|x|, non-finite) per
// workgroup over a grid-stride slice of x (four 16-byte loads in flight per
// thread).
template <bool ALIGNED>
__global__ __launch_bounds__(kStatsThreads) void stats_partial_kernel(StatsArgs a)
{
    RangeAcc acc;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    if (ALIGNED) {
        const uint64_t nvec = a.n / 4;
        const f4 *x4 = reinterpret_cast<const f4 *>(a.x);
        uint64_t i = tid;
        for (; i + 3 * nthreads < nvec; i += 4 * nthreads) {
            const f4 f0 = __builtin_nontemporal_load(x4 + i);
            const f4 f1 = __builtin_nontemporal_load(x4 + i + nthreads);
            const f4 f2 = __builtin_nontemporal_load(x4 + i + 2 * nthreads);
            const f4 f3 = __builtin_nontemporal_load(x4 + i + 3 * nthreads);
            acc.take4(f0);
            acc.take4(f1);
            acc.take4(f2);
            acc.take4(f3);
        }
        for (; i < nvec; i += nthreads) acc.take4(x4[i]);
        for (uint64_t k = nvec * 4 + tid; k < a.n; k += nthreads) acc.take(a.x[k]);
    } else {
        for (uint64_t k = tid; k < a.n; k += nthreads) acc.take(a.x[k]);
    }
    const StatsPartial p = acc.reduce();
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

// The accumulator goes first: max(max(acc, a), b) selects to one v_max3 per
// two new values, where max(acc, max(a, b)) costs a v_max and a v_max3.
__device__ __forceinline__ int max3i(int acc, int a, int b) { return max(max(acc, a), b); }
__device__ __forceinline__ int min3i(int acc, int a, int b) { return min(min(acc, a), b); }

// Quantization (Sec. IV-B, q = round(x / (2 eb)) read as rint(fl(x * inv))):
// for |t| < 2^22 the binary32 sum t + 1.5 * 2^23 rounds t to the nearest
// integer with ties to even and holds it in the low mantissa bits, so
// bits(fl(fl(x * inv) + 1.5 * 2^23)) = kQBias + rint(fl(x * inv)) exactly.
// The bias cancels in every Lorenzo difference; |q| <= 2^21 + 1 follows from
// the step tightening of the error-bound resolution.
constexpr float kQMagic = 12582912.0f;  // 1.5 * 2^23
constexpr int kQBias = 0x4B400000;       // bits of kQMagic

// Extrema of the LZ1 / LZ2 residual magnitudes of one block (Sec. IV-A,
// Eq. (2); Sec. IV-B) from biased quantized values B, which are replaced by
// the block's LZ1 residuals d[i] = q[i] - q[i-1] (0 in slots past the end of
// the field); the LZ2 residual is d[i] - d[i-1].  The predictor state
// (carry_b = biased q of the previous block's last element, carry_l1 = its
// LZ1 residual) crosses the block boundary; at a tile start q[-1] = q[-2] = 0,
// so there d[0] = q[0].  Block 0 of a tile (j == 0) leaves its first one
// (LZ1) or two (LZ2) residuals out: they are re-rated per variant.  Slots
// whose bit in vm is clear lie past the end of the field and carry residual 0.
template <bool FULL>
__device__ __forceinline__ void block_extrema(int (&B)[32], int carry_b, int carry_l1, int j, uint32_t vm,
                                              uint32_t &a1, uint32_t &a2, int &l2_1)
{
    auto live = [&](int i, int v) { return FULL ? v : (v & ((int)(vm << (31 - i)) >> 31)); };
    const int d0 = B[0] - carry_b, d1 = B[1] - B[0], d2 = B[2] - B[1];
    const int l1_0 = live(0, d0), l2_0 = live(0, d0 - carry_l1);
    const int l1_1 = live(1, d1), l2_1v = live(1, d1 - d0);
    const int l1_2 = live(2, d2), l2_2 = live(2, d2 - d1);
    l2_1 = l2_1v;
    // neutral substitutes for the excluded leading residuals of block 0
    const int e10 = j ? l1_0 : l1_1;
    const int e20 = j ? l2_0 : l2_2;
    const int e21 = j ? l2_1v : l2_2;
    int mx1 = max3i(e10, l1_1, l1_2), mn1 = min3i(e10, l1_1, l1_2);
    int mx2 = max3i(e20, e21, l2_2), mn2 = min3i(e20, e21, l2_2);
    int pl = d2, pb = B[2];
    B[0] = l1_0;
    B[1] = l1_1;
    B[2] = l1_2;
#pragma unroll
    for (int i = 3; i < 31; i += 2) {
        const int ba = B[i], bb = B[i + 1];
        const int da = ba - pb;
        const int db = bb - ba;
        const int l1a = live(i, da), l2a = live(i, da - pl);
        const int l1b = live(i + 1, db), l2b = live(i + 1, db - da);
        pl = db;
        pb = bb;
        B[i] = l1a;
        B[i + 1] = l1b;
        mx1 = max3i(mx1, l1a, l1b);
        mn1 = min3i(mn1, l1a, l1b);
        mx2 = max3i(mx2, l2a, l2b);
        mn2 = min3i(mn2, l2a, l2b);
    }
    const int d31 = B[31] - pb;
    const int l1z = live(31, d31), l2z = live(31, d31 - pl);
    B[31] = l1z;
    mx1 = max(mx1, l1z);
    mn1 = min(mn1, l1z);
    mx2 = max(mx2, l2z);
    mn2 = min(mn2, l2z);
    // max(|mx|, |mn|) = max(mx, -mn) for mx >= mn
    a1 = (uint32_t)max(mx1, -mn1);
    a2 = (uint32_t)max(mx2, -mn2);
}

// Residual codes of the selected variant, in place, from the LZ1 residuals d
// that block_extrema left: e[i] = d[i] - order2 * d[i-1] with d[-1] =
// carry_l1, and at a centred tile start (j == 0, cent) d[0] = q[0] less the
// tile mean (the later residuals are differences, so mu cancels there).
// code = (|e| << 1) | sign.  |d| <= 2^22 + 2 fits the 24-bit multiplier.
// Codes of slots past the end of the field are garbage; the encoder clears
// them in the transposed plane words.
// a * b + c with a and b taken as signed 24-bit integers (one VALU
// instruction; the compiler splits __mul24(a, b) + c into two)
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ void block_codes(int (&D)[32], int carry_l1, int j, int order2, int cent, int mu)
{
    const int no2 = -order2;
    int pl = carry_l1;
    D[0] -= (j == 0 && cent) ? mu : 0;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const int d = D[i];
        const int e = mad_i24(pl, no2, d);
        pl = d;
        const uint32_t m = (uint32_t)max(e, -e);
        D[i] = (int)__builtin_amdgcn_alignbit(m, (uint32_t)e, 31);  // (|e| << 1) | (e >> 31)
    }
}

// Per-lane result of the rate pass of one chunk, kept until its encode.
struct ChunkState {
    uint64_t chunk;
    int first;  // the block restarts prediction (tile start; every block without cross-block state)
    int carry_l1, mu;  // LZ1 residual of the previous block (0 where prediction restarts), tile mean
    uint32_t vm, r, blk_off, tile_excl, wave_total;
    int order2, cent;
    uint32_t rbyte;  // the block's rate byte (Sec. III-A)
};

template <int W>
struct CompressShared {
    uint32_t wave_total[2][W];
    unsigned long long base;
    unsigned long long ticket[2];  // alternating broadcast slots
};

// Rate pass of one chunk (8 tiles per wave), Sec. III-A steps 1-3:
//   1 quantize + cross-block LZ1/LZ2 residuals
//   2 four-way evaluation (Eq. (3)-(4)): blocks 1..7 have one rate per order;
//     block 0 is re-rated per variant from q0, q1 - 2 q0 and mu
//   3 adaptive select (strict minimum in the order LZ1, LZ2, LZ1c, LZ2c),
//     rate header; the chunk's byte count is published for the lookback.
// On return x holds the blocks' LZ1 residuals (block_extrema).
// DEFER: leave the rate byte in cs.rbyte for the caller to store, and publish
// the aggregate from wave 1 (whose memory queue the lookback does not wait on).
// FEAT: honour a.features (the ablation's switches, Sec. VI-B): without the
// cross-block state every block restarts prediction and is re-rated per
// variant like block 0; switched-off variants are never selected.
template <int W, bool DEFER = false, bool FEAT = false>
__device__ __forceinline__ ChunkState compress_rates(const CompressArgs &a, const Resolved &R, uint64_t chunk,
                                                     int (&x)[32], int slot, CompressShared<W> &sh)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    const uint64_t tile0 = chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
    const uint64_t tile = tile0 + (lane >> 3);
    const bool tile_ok = tile < a.ntiles;
    const uint64_t eblk = tile * kTile + (uint64_t)j * kBlock;
    const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
    const bool full = (tile0 + kTilesPerWave) * kTile <= a.n;  // wave-uniform
    ChunkState cs;
    cs.chunk = chunk;
    cs.vm = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);  // valid slots of the block

    // ---- tile mean: index-order pairwise binary32 tree over the 256 slots
    float s16[16];
#pragma unroll
    for (int i = 0; i < 16; i++) s16[i] = __int_as_float(x[2 * i]) + __int_as_float(x[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 8; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 2; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
    float ts = s16[0] + s16[1];
    ts = ts + dppf<kQuadXor1>(ts);       // blocks (0,1) (2,3) ...
    ts = ts + dppf<kQuadXor2>(ts);       // (0-1, 2-3) ...
    ts = ts + dppf<kRowHalfMirror>(ts);  // (0-3, 4-7)
    const float mean_q = (ts * 0x1p-8f) * R.inv;
    const bool centre_ok = __builtin_isfinite(mean_q);
    const int mu = centre_ok ? (int)__builtin_rintf(mean_q) : 0;
    cs.mu = mu;

    // ---- quantize, biased: x[i] = kQBias + rint(x * inv)
#pragma unroll
    for (int i = 0; i < 32; i++) x[i] = __float_as_int(__int_as_float(x[i]) * R.inv + kQMagic);

    // ---- cross-block state from block j-1 of the same tile (none where the
    // prediction restarts)
    const int t0 = dpp<kRowShr1>(x[31]);
    const int t1 = dpp<kRowShr1>(x[31] - x[30]);
    const bool first = FEAT ? (j == 0 || !(a.features & FSZ_FEAT_CROSS_BLOCK)) : j == 0;
    const int jr = first ? 0 : 1;  // 0: the leading residuals are re-rated per variant
    cs.first = first;
    const int carry_b = first ? kQBias : t0;
    cs.carry_l1 = first ? 0 : t1;

    uint32_t a1, a2;
    int l2_1;
    if (full)
        block_extrema<true>(x, carry_b, cs.carry_l1, jr, cs.vm, a1, a2, l2_1);
    else
        block_extrema<false>(x, carry_b, cs.carry_l1, jr, cs.vm, a1, a2, l2_1);
    const uint32_t r1 = bitlen(a1), r2 = bitlen(a2);
    uint32_t Z;
    if (FEAT) {
        // every restarting block is rated per variant, the others have one
        // rate per order; tile costs by 8-lane sums (same in all 8 lanes)
        const int q0 = x[0];  // d[0] = q[0] at a tile start
        const int d1 = cnt >= 2 ? l2_1 : 0;  // q1 - 2 q0
        const int c0 = q0 - mu;
        const int c1 = cnt >= 2 ? l2_1 + mu : 0;
        uint32_t ra = r1, rb = r2, rc = r1, rd = r2;
        if (first) {
            ra = bitlen(max(uabs(q0), a1));
            rb = bitlen(max(max(uabs(q0), uabs(d1)), a2));
            rc = bitlen(max(uabs(c0), a1));
            rd = bitlen(max(max(uabs(c0), uabs(c1)), a2));
        }
        if (cnt == 0) ra = rb = rc = rd = 0;  // blocks past the end of the field do not exist
        const uint32_t Ca = (uint32_t)group_sum((int)block_bytes(ra));
        const uint32_t Cb = (uint32_t)group_sum((int)block_bytes(rb));
        const uint32_t Cc = (uint32_t)group_sum((int)block_bytes(rc)) + 4;
        const uint32_t Cd = (uint32_t)group_sum((int)block_bytes(rd)) + 4;
        const bool lz2 = (a.features & FSZ_FEAT_LZ2) != 0;
        const bool cen = centre_ok && (a.features & FSZ_FEAT_CENTERING) != 0;
        int best = 0;
        uint32_t C = Ca, r = ra;
        if (lz2 && Cb < C) {
            best = 1;
            C = Cb;
            r = rb;
        }
        if (cen && Cc < C) {
            best = 2;
            C = Cc;
            r = rc;
        }
        if (cen && lz2 && Cd < C) {
            best = 3;
            C = Cd;
            r = rd;
        }
        if (!tile_ok) {
            best = 0;
            C = 0;
            r = 0;
        }
        cs.order2 = best & 1;
        cs.cent = best >> 1;
        Z = C;
        cs.r = r;
        cs.rbyte = j == 0 ? (r | (uint32_t)cs.order2 << 7 | (uint32_t)cs.cent << 6) : r;
    } else {
    const int T1 = group_sum(j ? (int)block_bytes(r1) : 0);
    const int T2 = group_sum(j ? (int)block_bytes(r2) : 0);

    // ---- four-way evaluation of block 0 and the selection (valid in lane j == 0)
    int dec;
    {
        const int q0 = x[0];  // d[0] = q[0] at a tile start
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
    cs.order2 = (dec >> 7) & 1;
    cs.cent = (dec >> 6) & 1;
    Z = (uint32_t)dec >> 8;
    cs.r = j == 0 ? (uint32_t)(dec & 31) : (cs.order2 ? r2 : r1);
    cs.rbyte = j == 0 ? (uint32_t)(dec & 0xFF) : cs.r;
    }
    if (!DEFER && cnt > 0) ((g_u8 *)a.out)[kHeaderBytes + tile * kBlocksPerTile + j] = (uint8_t)cs.rbyte;
    const uint32_t S = block_bytes(cs.r);

    // ---- offsets inside the wave / chunk, aggregate for the lookback
    const int incl = wave_incl_scan(j == 0 ? (int)Z : 0);
    cs.tile_excl = (uint32_t)incl - Z;
    cs.wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    cs.blk_off = cs.tile_excl + group_excl_scan(S, j) + 4u * cs.cent;
    if (lane == 0) sh.wave_total[slot][w] = cs.wave_total;
    lds_barrier();
    if (tid == (DEFER && W > 1 ? 64 : 0)) {
        uint32_t chunk_total = 0;
#pragma unroll
        for (int k = 0; k < W; k++) chunk_total += sh.wave_total[slot][k];
        publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, false);
    }
    return cs;
}

// Run by the thread that learns the last chunk's prefix: the stream header,
// the rate header's zero padding and the call's result.
__device__ __forceinline__ void finish_stream(const CompressArgs &a, const Resolved &R, const Prefix &pre,
                                              uint32_t chunk_total)
{
    const uint64_t total = a.data0 + pre.excl + chunk_total;
    uint32_t status = pre.err ? (uint32_t)FSZ_ERR_DEVICE : (uint32_t)FSZ_OK;
    if (status == FSZ_OK && total > a.capacity) status = FSZ_ERR_CAPACITY;
    if (status == FSZ_OK) {
        uint32_t *h = reinterpret_cast<uint32_t *>(a.out);
        h[0] = 0x315A5346u;  // "FSZ1"
        // bit 1: independent blocks; bits 2-4: tile configuration (0 = B 32, T 8)
        const uint32_t hflags = R.flags | ((a.features & FSZ_FEAT_CROSS_BLOCK) ? 0u : 2u) | a.cfg_flags;
        h[1] = 1u | ((uint32_t)a.mode << 16) | (hflags << 24);
        h[2] = (uint32_t)a.n;
        h[3] = (uint32_t)(a.n >> 32);
        h[4] = __float_as_uint(R.E);
        h[5] = __float_as_uint((float)a.value);
        h[6] = (uint32_t)total;
        h[7] = (uint32_t)(total >> 32);
        for (uint64_t k = kHeaderBytes + a.nblocks; k < a.data0; k++) a.out[k] = 0;
    }
    write_final(a.final, total, status, a.epoch);
}

// Steps 4-5 of one chunk whose rate pass is done: wait for the chunk's output
// offset (decoupled lookback, Sec. IV-D), then the sign / bit-plane encoding
// (Sec. IV-C) straight to the output.  B holds the LZ1 residuals.
template <bool STAGED, int W, bool FEAT = false>
__device__ __forceinline__ void compress_encode(const CompressArgs &a, const Resolved &R, const ChunkState &cs,
                                                int (&B)[32], int slot, CompressShared<W> &sh, uint32_t *st)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        if (k < w) wave_base += sh.wave_total[slot][k];
        chunk_total += sh.wave_total[slot][k];
    }
    if (w == 0) {
        const Prefix pre = lookback_wait(a.flags, cs.chunk, a.flag_epoch, chunk_total, false);
        if (lane == 0) {
            sh.base = pre.excl;
            if (cs.chunk == a.nchunks - 1) finish_stream(a, R, pre, chunk_total);
        }
    }
    lds_barrier();
    const uint64_t base = sh.base;
    const uint64_t tile0 = cs.chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
    if (a.data0 + base + chunk_total > a.capacity || tile0 >= a.ntiles) return;

    uint8_t *wave_out = a.out + a.data0 + base + wave_base;
    if (cs.vm != 0 && j == 0 && cs.cent) {
        if (STAGED)
            st[cs.tile_excl >> 2] = (uint32_t)cs.mu;
        else
            *reinterpret_cast<uint32_t *>(wave_out + cs.tile_excl) = (uint32_t)cs.mu;
    }
    block_codes(B, cs.carry_l1, FEAT ? (cs.first ? 0 : 1) : j, cs.order2, cs.cent, cs.mu);
    // valid slots in stored bit order (element i at bit i ^ 7)
    const uint32_t keep = __builtin_bswap32(__builtin_bitreverse32(cs.vm));
    const uint32_t nwords = cs.r ? cs.r + 1 : 0;  // sign word + r planes
    uint32_t *words = STAGED ? st + (cs.blk_off >> 2) : reinterpret_cast<uint32_t *>(wave_out + cs.blk_off);
    for (uint32_t g = 0; __ballot(8 * g < nwords) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int rho = 0; rho < 8; rho++)
            Rg[rho] = pack_byte_g((uint32_t)B[7 - rho], (uint32_t)B[15 - rho], (uint32_t)B[23 - rho],
                                  (uint32_t)B[31 - rho], g);
        transpose8(Rg);
#pragma unroll
        for (int p = 0; p < 8; p++)
            if (8 * g + p < nwords) words[8 * g + p] = Rg[p] & keep;
    }
    if (STAGED) {  // coalesced copy of the wave's contiguous output
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        wave_store_staged(reinterpret_cast<uint32_t *>(wave_out), st, cs.wave_total >> 2, lane);
    }
}

// Thread 0 takes the next ticket and broadcasts it.  Consecutive calls use
// alternating slots, so a slot is rewritten only after a barrier that every
// reader of its previous value has passed.
template <typename Shared>
__device__ __forceinline__ uint64_t next_ticket(unsigned long long *ticket, uint64_t takes, Shared &sh, int &slot)
{
    if (threadIdx.x == 0) sh.ticket[slot] = take_ticket(ticket, takes);
    lds_barrier();
    const uint64_t t = sh.ticket[slot];
    slot ^= 1;
    return t;
}

// One chunk of a compression (Sec. III-A steps 1-5) by a workgroup of W
// waves: bound resolution, coalesced load, rate pass, lookback, encode.
template <bool ALIGNED, bool LOAD_STAGED, bool STORE_STAGED, int W, bool FEAT = false>
__device__ __forceinline__ void compress_chunk(const CompressArgs &a, uint64_t chunk, CompressShared<W> &sh,
                                               uint32_t *st)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {
        if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        return;
    }
    const uint64_t tile0 = chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
    int x[32];
    {
        float f[32];
        if (LOAD_STAGED) {
            if (tile0 < a.ntiles) {
                load_blocks_staged<ALIGNED>(a.x, a.n, tile0 * kTile, st, lane, f);
            } else {
#pragma unroll
                for (int i = 0; i < 32; i++) f[i] = 0.0f;
            }
        } else {
            const uint64_t eblk = (tile0 + (lane >> 3)) * kTile + (uint64_t)(lane & 7) * kBlock;
            const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
            load_block<ALIGNED>(a.x, eblk, cnt, f);
        }
#pragma unroll
        for (int i = 0; i < 32; i++) x[i] = __float_as_int(f[i]);
    }
    const ChunkState cs = compress_rates<W, false, FEAT>(a, R, chunk, x, 0, sh);
    compress_encode<STORE_STAGED, W, FEAT>(a, R, cs, x, 0, sh, st);
}

// Compression kernel: one chunk per workgroup, chunk ids from the ticket
// counter, so the lookback only waits on chunks that are already running.
// The kernel is kept small in registers so that many chunks are in flight per
// CU: chunks waiting in the lookback leave the CU to the others.
template <bool ALIGNED, bool LOAD_STAGED, bool STORE_STAGED, bool FEAT = false>
__global__ __launch_bounds__(kThreads) void compress_kernel(CompressArgs a)
{
    __shared__ CompressShared<kWaves> sh;
    __shared__ __attribute__((aligned(16))) uint32_t
        stage[(LOAD_STAGED || STORE_STAGED) ? kWaves * kStageWaveDwords : 4];
    const int w = threadIdx.x >> 6;
    uint32_t *st = stage + ((LOAD_STAGED || STORE_STAGED) ? w * kStageWaveDwords : 0);
    int tslot = 0;
    const uint64_t chunk = next_ticket(a.ticket, a.nchunks, sh, tslot);
    if (chunk >= a.nchunks) return;  // inconsistent ticket counter: never index past the flags
    compress_chunk<ALIGNED, LOAD_STAGED, STORE_STAGED, kWaves, FEAT>(a, chunk, sh, st);
}

// ------------------------------------------------------------------ naive five-read baseline

// The comparison point of Sec. V-C (Fig. 6): the four variants evaluated in
// four separate passes over the input, each writing per-tile costs and block
// rates, then an encode pass that reads the input a fifth time.  It produces
// the same stream as the single-pass kernels; only the reads differ.

// Evaluation pass of variant v (bit 0: second order, bit 1: centred) over a
// chunk of kTilesPerChunk tiles per workgroup.
template <bool ALIGNED>
__global__ __launch_bounds__(kThreads) void naive_eval_kernel(CompressArgs a, NaiveTables t, int v)
{
    __shared__ __attribute__((aligned(16))) uint32_t stage[kWaves * kStageWaveDwords];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) return;  // the encode pass reports the status
    const uint64_t tile0 = (uint64_t)blockIdx.x * kTilesPerChunk + (uint64_t)w * kTilesPerWave;
    if (tile0 >= a.ntiles) return;  // wave-uniform; the kernel has no workgroup barrier
    float f[32];
    load_blocks_staged<ALIGNED>(a.x, a.n, tile0 * kTile, stage + w * kStageWaveDwords, lane, f);
    const uint64_t tile = tile0 + (lane >> 3);
    const bool tile_ok = tile < a.ntiles;
    const uint64_t eblk = tile * kTile + (uint64_t)j * kBlock;
    const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
    const uint32_t vm = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);
    const bool full = (tile0 + kTilesPerWave) * kTile <= a.n;
    const int order2 = v & 1, cen = v >> 1;

    int mu = 0;
    bool centre_ok = true;
    if (cen) {  // tile mean, as in the single pass
        float s16[16];
#pragma unroll
        for (int i = 0; i < 16; i++) s16[i] = f[2 * i] + f[2 * i + 1];
#pragma unroll
        for (int i = 0; i < 8; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
        for (int i = 0; i < 4; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
        for (int i = 0; i < 2; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
        float ts = s16[0] + s16[1];
        ts = ts + dppf<kQuadXor1>(ts);
        ts = ts + dppf<kQuadXor2>(ts);
        ts = ts + dppf<kRowHalfMirror>(ts);
        const float mean_q = (ts * 0x1p-8f) * R.inv;
        centre_ok = __builtin_isfinite(mean_q);
        mu = centre_ok ? (int)__builtin_rintf(mean_q) : 0;
    }
    int x[32];
#pragma unroll
    for (int i = 0; i < 32; i++) x[i] = __float_as_int(f[i] * R.inv + kQMagic);
    const int t0 = dpp<kRowShr1>(x[31]);
    const int t1 = dpp<kRowShr1>(x[31] - x[30]);
    const int carry_b = j ? t0 : kQBias;
    const int carry_l1 = j ? t1 : 0;
    uint32_t a1, a2;
    int l2_1;
    if (full)
        block_extrema<true>(x, carry_b, carry_l1, j, vm, a1, a2, l2_1);
    else
        block_extrema<false>(x, carry_b, carry_l1, j, vm, a1, a2, l2_1);
    uint32_t r = bitlen(order2 ? a2 : a1);
    if (j == 0) {  // block 0: the variant's own first residuals
        const int q0 = x[0];  // d[0] = q[0] at a tile start
        const int f0 = cen ? q0 - mu : q0;
        const int d1 = cnt >= 2 ? l2_1 : 0;
        const int f1 = cnt >= 2 ? (cen ? l2_1 + mu : d1) : 0;
        r = order2 ? bitlen(max(max(uabs(f0), uabs(f1)), a2)) : bitlen(max(uabs(f0), a1));
    }
    const uint32_t C = (uint32_t)group_sum((int)block_bytes(r)) + (cen ? 4u : 0u);
    if (tile_ok) {
        t.rates[((uint64_t)v * a.ntiles + tile) * kBlocksPerTile + j] = (uint8_t)r;
        if (j == 0) {
            t.cost[(uint64_t)v * a.ntiles + tile] = C;
            if (cen) {
                t.mu[tile] = mu;
                t.centre_ok[tile] = centre_ok ? 1 : 0;
            }
        }
    }
}

// Selection and bookkeeping of the encode pass: the rate pass of the single
// pass with the evaluation replaced by reads of the tables (same choice,
// same tie order).  On return x holds the blocks' LZ1 residuals.
__device__ __forceinline__ ChunkState naive_select(const CompressArgs &a, const Resolved &R, const NaiveTables &t,
                                                   uint64_t chunk, int (&x)[32], CompressShared<kWaves> &sh)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    const uint64_t tile0 = chunk * kTilesPerChunk + (uint64_t)w * kTilesPerWave;
    const uint64_t tile = tile0 + (lane >> 3);
    const bool tile_ok = tile < a.ntiles;
    const uint64_t eblk = tile * kTile + (uint64_t)j * kBlock;
    const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
    ChunkState cs;
    cs.chunk = chunk;
    cs.vm = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);
#pragma unroll
    for (int i = 0; i < 32; i++) x[i] = __float_as_int(__int_as_float(x[i]) * R.inv + kQMagic);
    const int t0 = dpp<kRowShr1>(x[31]);
    const int t1 = dpp<kRowShr1>(x[31] - x[30]);
    cs.first = j == 0;
    cs.carry_l1 = j ? t1 : 0;
    {  // LZ1 residuals in place, as the encoder takes them
        int pb = j ? t0 : kQBias;
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const int b = x[i];
            x[i] = b - pb;
            pb = b;
        }
    }

    int best = 0;
    uint32_t Z = 0, r = 0;
    cs.mu = 0;
    if (tile_ok) {
        const uint32_t Ca = t.cost[tile], Cb = t.cost[a.ntiles + tile];
        const uint32_t Cc = t.cost[2 * a.ntiles + tile], Cd = t.cost[3 * a.ntiles + tile];
        const bool centre_ok = t.centre_ok[tile] != 0;
        uint32_t C = Ca;
        if (Cb < C) {
            best = 1;
            C = Cb;
        }
        if (centre_ok) {
            if (Cc < C) {
                best = 2;
                C = Cc;
            }
            if (Cd < C) {
                best = 3;
                C = Cd;
            }
        }
        Z = C;
        r = t.rates[((uint64_t)best * a.ntiles + tile) * kBlocksPerTile + j];
        if (best >> 1) cs.mu = t.mu[tile];
    }
    cs.order2 = best & 1;
    cs.cent = best >> 1;
    cs.r = r;
    cs.rbyte = j == 0 ? (r | (uint32_t)cs.order2 << 7 | (uint32_t)cs.cent << 6) : r;
    if (cnt > 0) ((g_u8 *)a.out)[kHeaderBytes + tile * kBlocksPerTile + j] = (uint8_t)cs.rbyte;
    const uint32_t S = block_bytes(cs.r);
    const int incl = wave_incl_scan(j == 0 ? (int)Z : 0);
    cs.tile_excl = (uint32_t)incl - Z;
    cs.wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    cs.blk_off = cs.tile_excl + group_excl_scan(S, j) + 4u * cs.cent;
    if (lane == 0) sh.wave_total[0][w] = cs.wave_total;
    lds_barrier();
    if (tid == 0) {
        uint32_t chunk_total = 0;
#pragma unroll
        for (int k = 0; k < kWaves; k++) chunk_total += sh.wave_total[0][k];
        publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, false);
    }
    return cs;
}

// Encode pass: one chunk per workgroup from the ticket counter (the fifth
// read of the input), the tables' choice, lookback, the single pass's encoder.
template <bool ALIGNED>
__global__ __launch_bounds__(kThreads) void naive_encode_kernel(CompressArgs a, NaiveTables t)
{
    __shared__ CompressShared<kWaves> sh;
    __shared__ __attribute__((aligned(16))) uint32_t stage[kWaves * kStageWaveDwords];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    uint32_t *st = stage + w * kStageWaveDwords;
    int tslot = 0;
    const uint64_t chunk = next_ticket(a.ticket, a.nchunks, sh, tslot);
    if (chunk >= a.nchunks) return;
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {
        if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        return;
    }
    const uint64_t tile0 = chunk * kTilesPerChunk + (uint64_t)w * kTilesPerWave;
    int x[32];
    {
        float f[32];
        if (tile0 < a.ntiles) {
            load_blocks_staged<ALIGNED>(a.x, a.n, tile0 * kTile, st, lane, f);
        } else {
#pragma unroll
            for (int i = 0; i < 32; i++) f[i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 32; i++) x[i] = __float_as_int(f[i]);
    }
    const ChunkState cs = naive_select(a, R, t, chunk, x, sh);
    compress_encode<true, kWaves>(a, R, cs, x, 0, sh, st);
}

// ------------------------------------------------------------------ pipelined compress
//
// Persistent form of the compression kernel for 16-byte aligned inputs: each
// workgroup keeps the next chunk's input in flight while it works on the
// current ones, through asynchronous global->LDS copies that hold no
// registers.  The LDS image of a wave's 8 tiles is unpadded and rotated:
// piece m (16 B) of block b sits at 16-byte slot 8b + ((m + b) & 7), so that
// both the copies (each instruction covers 1 KiB of contiguous input) and the
// lane-per-block reads (lane b reads piece m at step m) are free of bank
// conflicts.

constexpr int kCachePolicyNT = 2;  // cache-policy operand of the LDS copies: nontemporal
constexpr int kPipeWaveDwords = 2060;  // 8 tiles of input, or the wave's output (<= 8 x 1028 B) at a 16-byte phase
typedef __attribute__((address_space(3))) void lds_void;

// Input of the wave's 8 tiles (element e0 onward, all in bounds) -> LDS.
// The copies carry the nontemporal hint: the input is read once, and without
// the hint it displaces cached data, among it the stream just written.
__device__ __forceinline__ void chunk_copy_async(const float *__restrict__ x, uint64_t e0, uint32_t *wbuf, int lane)
{
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int b = 8 * k + (lane >> 3);
        const int m = ((lane & 7) - b) & 7;
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const void *>(x + e0 + 32 * b + 4 * m),
                                         (lds_void *)(wbuf + 256 * k), 16, 0, kCachePolicyNT);
    }
}

// Same image, loaded synchronously; elements at or beyond n read as +0.
__device__ __forceinline__ void chunk_copy_sync(const float *__restrict__ x, uint64_t n, uint64_t e0, uint32_t *wbuf,
                                                int lane)
{
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int b = 8 * k + (lane >> 3);
        const int m = ((lane & 7) - b) & 7;
        const uint64_t e = e0 + 32 * b + 4 * m;
        f4 f;
        f.x = e + 0 < n ? x[e + 0] : 0.0f;
        f.y = e + 1 < n ? x[e + 1] : 0.0f;
        f.z = e + 2 < n ? x[e + 2] : 0.0f;
        f.w = e + 3 < n ? x[e + 3] : 0.0f;
        *reinterpret_cast<f4 *>(wbuf + 4 * (64 * k + lane)) = f;
    }
}

// Starts bringing the wave's part of `chunk` (W waves per chunk) into wbuf.
template <int W>
__device__ __forceinline__ void chunk_fetch(const CompressArgs &a, uint64_t chunk, uint32_t *wbuf, int w, int lane)
{
    const uint64_t e0 = (chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave) * kTile;
    if (e0 + kTilesPerWave * kTile <= a.n)
        chunk_copy_async(a.x, e0, wbuf, lane);
    else
        chunk_copy_sync(a.x, a.n, e0, wbuf, lane);
}

// Lane-per-block read of the wave's image (block = lane).
__device__ __forceinline__ void chunk_read(const uint32_t *wbuf, int lane, int (&v)[32])
{
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's copies have landed
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int t = 0; t < 8; t++) {
        const int slot = 8 * lane + ((t + lane) & 7);
        const f4 f = *reinterpret_cast<const f4 *>(wbuf + 4 * slot);
        v[4 * t + 0] = __float_as_int(f.x);
        v[4 * t + 1] = __float_as_int(f.y);
        v[4 * t + 2] = __float_as_int(f.z);
        v[4 * t + 3] = __float_as_int(f.w);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// The pipeline keeps every wait away from memory operations issued just
// before it: the vector memory operations of a wave complete in issue order,
// so a wait also waits for everything issued earlier.  Per step, wave 0 takes
// the next ticket and reads the lookback's first window before the rate
// pass and uses both after it; wave 1 publishes the aggregates; rate bytes go
// out with the chunk's data; the next chunk is read from LDS after staging
// but before the stores.  One LDS buffer per wave always receives the copy in
// flight, the other stages output.

// Lookback of cs.chunk by wave 0 (W0) from the pre-read window `probe`; the
// last chunk finishes the stream.  Wave 0 also resolves the ticket `traw` it
// took at the start of the step (resetting the counter if it was the last
// take) and broadcasts it.  Returns the chunk's exclusive prefix in every
// thread and the broadcast ticket in *next.
template <bool W0, int W>
__device__ __forceinline__ uint64_t pipe2_lookback(const CompressArgs &a, const Resolved &R, const ChunkState &cs,
                                                   int slot, CompressShared<W> &sh, const Probe &probe,
                                                   bool took, unsigned long long traw, uint64_t takes,
                                                   uint64_t *next)
{
    const int lane = threadIdx.x & 63;
    if (W0) {
        uint32_t chunk_total = 0;
#pragma unroll
        for (int k = 0; k < W; k++) chunk_total += sh.wave_total[slot][k];
        // the probe is consumed on every path (also for chunk 0), so the
        // next step's reads into its registers do not wait on stale loads
        consume_probe(probe);
        const Prefix pre = lookback_wait(a.flags, cs.chunk, a.flag_epoch, chunk_total, false, true, probe);
        const unsigned long long tk =
            took ? ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(traw >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)traw)
                 : a.nchunks;
        if (lane == 0) {
            if (took && tk == takes - 1)
                __hip_atomic_store(a.ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh.base = pre.excl;
            sh.ticket[0] = tk;
            if (cs.chunk == a.nchunks - 1) finish_stream(a, R, pre, chunk_total);
        }
    }
    lds_barrier();
    *next = sh.ticket[0];
    return sh.base;
}

// Residual codes and bit planes of one wave's blocks into its staging area
// (offsets relative to the wave's first byte).
template <bool FEAT>
__device__ __forceinline__ void pipe2_stage(const ChunkState &cs, int (&B)[32], uint32_t *st)
{
    const int j = __lane_id() & 7;
    if (cs.vm != 0 && j == 0 && cs.cent) st[cs.tile_excl >> 2] = (uint32_t)cs.mu;
    block_codes(B, cs.carry_l1, FEAT ? (cs.first ? 0 : 1) : j, cs.order2, cs.cent, cs.mu);
    const uint32_t keep = __builtin_bswap32(__builtin_bitreverse32(cs.vm));
    const uint32_t nwords = cs.r ? cs.r + 1 : 0;
    uint32_t *words = st + (cs.blk_off >> 2);
    for (uint32_t g = 0; __ballot(8 * g < nwords) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int rho = 0; rho < 8; rho++)
            Rg[rho] = pack_byte_g((uint32_t)B[7 - rho], (uint32_t)B[15 - rho], (uint32_t)B[23 - rho],
                                  (uint32_t)B[31 - rho], g);
        transpose8(Rg);
#pragma unroll
        for (int p = 0; p < 8; p++)
            if (8 * g + p < nwords) words[8 * g + p] = Rg[p] & keep;
    }
}

// The tile geometry a compression pipeline runs: its rate pass (one
// workgroup barrier), its staging of the codes, whether a wave's first tile
// exists, and where a lane's rate byte goes.  TileB32T8 is the default format
// (blocks of 32 elements, tiles of 8 blocks); the tile-configuration sweep
// has its own.
struct TileB32T8 {
    template <int W, bool FEAT>
    static __device__ __forceinline__ ChunkState rates(const CompressArgs &a, const Resolved &R, uint64_t chunk,
                                                       int (&x)[32], int slot, CompressShared<W> &sh)
    {
        return compress_rates<W, true, FEAT>(a, R, chunk, x, slot, sh);
    }
    template <bool FEAT>
    static __device__ __forceinline__ void stage(const ChunkState &cs, int (&B)[32], uint32_t *st)
    {
        pipe2_stage<FEAT>(cs, B, st);
    }
    template <int W>
    static __device__ __forceinline__ bool wave_live(const CompressArgs &a, uint64_t chunk, int w)
    {
        return chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave < a.ntiles;
    }
    template <int W>
    static __device__ __forceinline__ void store_rate(const CompressArgs &a, const ChunkState &cs, int w, int lane)
    {
        const uint64_t tile0 = cs.chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
        if (cs.vm != 0)
            ((g_u8 *)a.out)[kHeaderBytes + (tile0 + (lane >> 3)) * kBlocksPerTile + (lane & 7)] = (uint8_t)cs.rbyte;
    }
};

// One step with chunk A rate-passed (registers xa, wave totals in slot sa),
// chunk B read (registers yb) and chunk C being copied into qb: rate pass of
// B, lookback + staging of A, read C into xa, start the copy of the ticket
// taken in this step, store A.  Returns that ticket (nchunks if none).
// W0: the calling wave is wave 0, which takes the ticket and reads the
// lookback window at the start and uses both after the rate pass.
template <bool W0, int W, bool FEAT, class M = TileB32T8>
__device__ __forceinline__ uint64_t pipe2_step(const CompressArgs &a, const Resolved &R, uint64_t takes,
                                               const ChunkState &ca, int (&xa)[32], int sa, uint64_t B,
                                               int (&yb)[32], ChunkState &cb, uint64_t C, uint32_t *qb,
                                               uint32_t *pb, CompressShared<W> &sh, int w)
{
    const int lane = threadIdx.x & 63;
    const bool take = C < a.nchunks;
    unsigned long long traw = 0;
    Probe probe{};
    if (W0) {
        if (take && lane == 0) traw = atomicAdd(a.ticket, 1ull);
        probe = lookback_probe(a.flags, ca.chunk, a.flag_epoch);
    }
    if (B < a.nchunks) cb = M::template rates<W, FEAT>(a, R, B, yb, sa ^ 1, sh);
    uint64_t D;
    const uint64_t base = pipe2_lookback<W0, W>(a, R, ca, sa, sh, probe, take, traw, takes, &D);

    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        if (k < w) wave_base += sh.wave_total[sa][k];
        chunk_total += sh.wave_total[sa][k];
    }
    const bool ok = a.data0 + base + chunk_total <= a.capacity && M::template wave_live<W>(a, ca.chunk, w);
    uint32_t *wave_out = reinterpret_cast<uint32_t *>(a.out + a.data0 + base + wave_base);
    uint32_t *ps = pb + (((uint32_t)(uintptr_t)wave_out >> 2) & 3u);  // staging at the output's 16-byte phase
    if (ok) M::template stage<FEAT>(ca, xa, ps);
    if (C < a.nchunks) chunk_read(qb, lane, xa);
    if (D < a.nchunks) {
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the read of qb is done before it is overwritten
        chunk_fetch<W>(a, D, qb, w, lane);
    }
    M::template store_rate<W>(a, ca, w, lane);
    if (ok) {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        wave_store_staged_phased(wave_out, ps, ca.wave_total >> 2, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    return D;
}

// The whole pipeline of one wave (W0: wave 0's role), from the first ticket on.
template <bool W0, int W, bool FEAT, class M = TileB32T8>
__device__ __forceinline__ void pipe2_run(const CompressArgs &a, const Resolved &R, CompressShared<W> &sh,
                                          uint32_t *qb, uint32_t *pb, int w)
{
    const int lane = threadIdx.x & 63;
    const uint64_t N = a.nchunks;
    const uint64_t takes = N + gridDim.x;
    int tslot = 0;
    const uint64_t A = next_ticket(a.ticket, takes, sh, tslot);
    if (A >= N) return;
    chunk_fetch<W>(a, A, qb, w, lane);
    uint64_t B = next_ticket(a.ticket, takes, sh, tslot);
    int x[32], y[32];
    chunk_read(qb, lane, x);
    if (B < N) {
        __builtin_amdgcn_s_waitcnt(0xC07F);
        chunk_fetch<W>(a, B, qb, w, lane);
    }
    ChunkState ca = M::template rates<W, FEAT>(a, R, A, x, 0, sh);
    ChunkState cb = ca;
    uint64_t C = N;
    if (B < N) {
        C = next_ticket(a.ticket, takes, sh, tslot);
        chunk_read(qb, lane, y);
        if (C < N) {
            __builtin_amdgcn_s_waitcnt(0xC07F);
            chunk_fetch<W>(a, C, qb, w, lane);
        }
    }
    // loop invariant: A rate-passed in x (slot 0), B read into y, C in flight
    for (;;) {
        const uint64_t D = pipe2_step<W0, W, FEAT, M>(a, R, takes, ca, x, 0, B, y, cb, C, qb, pb, sh, w);
        if (B >= N) return;
        const uint64_t E = pipe2_step<W0, W, FEAT, M>(a, R, takes, cb, y, 1, C, x, ca, D, qb, pb, sh, w);
        if (C >= N) return;
        B = D;
        C = E;
    }
}

// The control wave of compress_ctrl_kernel: wave 0's part of the pipeline
// without its data.  Per step it takes the ticket and walks the lookback of
// the chunk rate-passed in the previous step while the data waves run the
// next rate pass, so the offset is usually known when they reach the second
// barrier; its own memory queue holds only flag reads, so they are not
// queued behind copies and stores.  It passes every barrier the data waves
// pass (pipe2_run<false, WD>): the ticket broadcasts, the rate pass's, and
// the step's second one.
template <int WD>
__device__ __forceinline__ uint64_t ctrl_step(const CompressArgs &a, const Resolved &R, uint64_t takes,
                                              uint64_t A, int sa, uint64_t B, uint64_t C, CompressShared<WD> &sh)
{
    const uint64_t N = a.nchunks;
    const int lane = __lane_id();
    const bool take = C < N;
    unsigned long long traw = 0;
    if (take && lane == 0) traw = atomicAdd(a.ticket, 1ull);
    uint32_t chunk_total = 0;
#pragma unroll
    for (int k = 0; k < WD; k++) chunk_total += sh.wave_total[sa][k];  // A's, from the previous step
    const Prefix pre = lookback_wait(a.flags, A, a.flag_epoch, chunk_total, false);
    if (B < N) lds_barrier();  // the data waves' rate pass of B
    const unsigned long long tk =
        take ? ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(traw >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)traw)
             : N;
    if (lane == 0) {
        if (take && tk == takes - 1) __hip_atomic_store(a.ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sh.base = pre.excl;
        sh.ticket[0] = tk;
        if (A == N - 1) finish_stream(a, R, pre, chunk_total);
    }
    lds_barrier();  // the offset and the ticket go out
    return tk;
}

template <int WD>
__device__ __forceinline__ void ctrl_run(const CompressArgs &a, const Resolved &R, CompressShared<WD> &sh)
{
    const uint64_t N = a.nchunks;
    const uint64_t takes = N + gridDim.x;
    // first pick of its SIMD's issue slots: the wave shares a SIMD with two
    // data waves in their rate pass, and its short lookback bursts gate the
    // step's second barrier
    __builtin_amdgcn_s_setprio(3);
    int tslot = 0;
    uint64_t A = next_ticket(a.ticket, takes, sh, tslot);
    if (A >= N) return;
    uint64_t B = next_ticket(a.ticket, takes, sh, tslot);
    lds_barrier();  // the rate pass of A
    uint64_t C = N;
    if (B < N) C = next_ticket(a.ticket, takes, sh, tslot);
    for (int sa = 0;; sa ^= 1) {
        const uint64_t D = ctrl_step<WD>(a, R, takes, A, sa, B, C, sh);
        if (B >= N) return;
        A = B;
        B = C;
        C = D;
    }
}

// The pipelined compressor with WD data waves (8 tiles each per chunk) and
// one control wave (ctrl_run).  a.nchunks must count chunks of 8 WD tiles.
template <int WD>
__global__ __launch_bounds__((WD + 1) * 64) void compress_ctrl_kernel(CompressArgs a)
{
    __shared__ CompressShared<WD> sh;
    __shared__ __attribute__((aligned(16))) uint32_t inbuf[WD * kPipeWaveDwords];
    __shared__ __attribute__((aligned(16))) uint32_t stbuf[WD * kPipeWaveDwords];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {  // no data work: hand out the tickets, the last chunk reports
        const uint64_t takes = a.nchunks + gridDim.x;
        int tslot = 0;
        for (;;) {
            const uint64_t t = next_ticket(a.ticket, takes, sh, tslot);
            if (t >= a.nchunks) return;
            if (threadIdx.x == 0 && t == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        }
    }
    if (w < WD)
        pipe2_run<false, WD, false>(a, R, sh, inbuf + w * kPipeWaveDwords, stbuf + w * kPipeWaveDwords, w);
    else
        ctrl_run<WD>(a, R, sh);
}

// W waves per workgroup; a chunk is 8 tiles per wave.  a.nchunks must count
// chunks of that size.  FEAT: honour the feature switches in a.features.
template <int W, bool FEAT = false>
__global__ __launch_bounds__(W * 64) void compress_pipe2_kernel(CompressArgs a)
{
    __shared__ CompressShared<W> sh;
    __shared__ __attribute__((aligned(16))) uint32_t inbuf[W * kPipeWaveDwords];
    __shared__ __attribute__((aligned(16))) uint32_t stbuf[W * kPipeWaveDwords];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    uint32_t *qb = inbuf + w * kPipeWaveDwords;
    uint32_t *pb = stbuf + w * kPipeWaveDwords;

    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {  // no data work: hand out the tickets, the last chunk reports
        const uint64_t takes = a.nchunks + gridDim.x;
        int tslot = 0;
        for (;;) {
            const uint64_t t = next_ticket(a.ticket, takes, sh, tslot);
            if (t >= a.nchunks) return;
            if (threadIdx.x == 0 && t == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        }
    }
    if (w == 0)
        pipe2_run<true, W, FEAT>(a, R, sh, qb, pb, w);
    else if (W > 1)
        pipe2_run<false, W, FEAT>(a, R, sh, qb, pb, w);
}

// ------------------------------------------------------------------ decompress

// Per-lane state of one chunk between the size pass and the decode pass.
struct DecChunk {
    uint64_t chunk;
    uint64_t base;  // the chunk's data offset after data0 (decodes with the offsets pre-pass)
    uint32_t r, blk_off, tile_excl, wave_total;
    int order2, cent;
};

template <int W>
struct DecompressShared {
    uint32_t wave_total[2][W];
    int bad[2];
    unsigned long long base;
    unsigned long long ticket[2];  // alternating broadcast slots
};

// Decompression steps 1-2 (Sec. III-A): rate bytes and tile metadata ->
// block and tile sizes -> this chunk's aggregate, published at once so that
// successors' lookbacks rarely wait.
// RANGE: decode the tiles [a.tile_begin, a.tile_end) only (random access);
// otherwise the whole field (the range fields are not read).
// The lane's rate byte of `chunk` (0 past the end or outside a range).
template <int W, bool RANGE = false>
__device__ __forceinline__ uint32_t dec_rate_byte(const DecompressArgs &a, uint64_t chunk)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const uint64_t tile =
        (RANGE ? a.tile_begin : 0) + chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave + (lane >> 3);
    const bool tile_ok = tile < (RANGE ? a.tile_end : a.ntiles);
    const uint64_t gblock = tile * kBlocksPerTile + (lane & 7);
    const bool blk_ok = (RANGE ? tile_ok : true) && gblock < a.nblocks;
    return blk_ok ? ((const g_u8 *)a.cmp)[kHeaderBytes + gblock] : 0u;
}

// rb: the lane's rate byte from dec_rate_byte (loaded ahead by the caller).
// PRESCAN: the offsets pre-pass has checked the rate bytes and placed every
// chunk; the chunk's offset is read instead of publishing its aggregate.
template <int W, bool RANGE = false, bool PRESCAN = false>
__device__ __forceinline__ DecChunk dec_sizes(const DecompressArgs &a, uint64_t chunk, uint32_t rb, int slot,
                                              DecompressShared<W> &sh)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    const uint64_t tile =
        (RANGE ? a.tile_begin : 0) + chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave + (lane >> 3);
    const bool tile_ok = tile < (RANGE ? a.tile_end : a.ntiles);
    const uint64_t gblock = tile * kBlocksPerTile + j;
    const bool blk_ok = (RANGE ? tile_ok : true) && gblock < a.nblocks;
    const bool bad = blk_ok && (j == 0 ? (rb & 0x20u) : (rb & 0xE0u)) != 0;
    const uint32_t head = (uint32_t)group_head((int)rb);
    DecChunk d;
    d.chunk = chunk;
    d.order2 = tile_ok ? (int)((head >> 7) & 1u) : 0;
    d.cent = tile_ok ? (int)((head >> 6) & 1u) : 0;
    d.r = rb & 31u;
    const uint32_t S = block_bytes(d.r);
    const uint32_t Z = (uint32_t)group_sum((int)S) + 4u * d.cent;
    const int incl = wave_incl_scan(j == 0 ? (int)Z : 0);
    d.tile_excl = (uint32_t)incl - Z;
    d.wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    d.blk_off = d.tile_excl + group_excl_scan(S, j) + 4u * d.cent;
    d.base = 0;
    if (PRESCAN) {
        d.base = a.offsets[__builtin_amdgcn_readfirstlane((uint32_t)chunk)];
        if (lane == 0) sh.wave_total[slot][w] = d.wave_total;
        lds_barrier();
        return d;
    }
    const bool wave_bad = __ballot(bad) != 0;
    if (lane == 0) {
        sh.wave_total[slot][w] = d.wave_total;
        if (w == 0) sh.bad[slot] = 0;
    }
    lds_barrier();
    if (lane == 0 && wave_bad) sh.bad[slot] = 1;
    lds_barrier();
    uint32_t chunk_total = 0;
#pragma unroll
    for (int k = 0; k < W; k++) chunk_total += sh.wave_total[slot][k];
    if (tid == 0) publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, sh.bad[slot] != 0);
    return d;
}

// Decompression step 3 (Sec. III-A): the chunk's byte offset from the
// lookback (wave 0; the workgroup waits at one barrier), then where the
// wave's share of the chunk's data starts.  The workgroup owning the last
// chunk reports the outcome.  live: the wave has blocks to decode.
// PREZERO: the output was cleared to +0.0 before the launch (Sec. III-A, for
// highly compressible streams); a wave whose blocks all have rate 0 and whose
// tiles are all uncentred decodes to q = 0, i.e. +0.0 everywhere, and is not
// live.
struct DecPlace {
    const uint8_t *wave_data;
    uint64_t tile0;
    bool live;
};

template <int W, bool RANGE = false, bool PREZERO = false, bool PRESCAN = false>
__device__ __forceinline__ DecPlace dec_place(const DecompressArgs &a, const DecChunk &d, int slot, uint64_t total,
                                              DecompressShared<W> &sh)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int j = lane & 7;
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        if (k < w) wave_base += sh.wave_total[slot][k];
        chunk_total += sh.wave_total[slot][k];
    }
    if (PRESCAN) {  // placed and checked by the pre-pass
        DecPlace p;
        p.tile0 = d.chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
        p.wave_data = a.cmp + a.data0 + d.base + wave_base;
        p.live = p.tile0 < a.ntiles;
        if (PREZERO && p.live) {
            const uint64_t gblock = (p.tile0 + (lane >> 3)) * kBlocksPerTile + j;
            p.live = __ballot(gblock < a.nblocks && (d.r != 0 || d.cent != 0)) != 0;
        }
        return p;
    }
    const bool bad = sh.bad[slot] != 0;
    const uint64_t base0 = RANGE ? *a.range_base : 0;  // data of tiles before the range
    if (w == 0) {
        const Prefix pre = lookback_wait(a.flags, d.chunk, a.flag_epoch, chunk_total, bad);
        if (lane == 0) {
            sh.base = base0 + pre.excl;
            if (d.chunk == a.nchunks - 1) {
                bool ok;
                if (RANGE) {  // a range: its data lies inside the stream
                    ok = !pre.err && a.data0 + base0 + pre.excl + chunk_total <= total;
                } else {  // the whole field: the sizes add up to the stream's total, padding is zero
                    ok = !pre.err && a.data0 + pre.excl + chunk_total == total;
                    for (uint64_t k = kHeaderBytes + a.nblocks; ok && k < a.data0; k++) ok = a.cmp[k] == 0;
                }
                write_final(a.final, total, ok ? (uint32_t)FSZ_OK : (uint32_t)FSZ_ERR_CORRUPT, a.epoch);
            }
        }
    }
    lds_barrier();
    const uint64_t base = sh.base;
    DecPlace p;
    p.tile0 = (RANGE ? a.tile_begin : 0) + d.chunk * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
    p.wave_data = a.cmp + a.data0 + base + wave_base;
    p.live = !(bad || a.data0 + base + chunk_total > total || p.tile0 >= (RANGE ? a.tile_end : a.ntiles));
    if (PREZERO && p.live) {
        const uint64_t gblock = (p.tile0 + (lane >> 3)) * kBlocksPerTile + j;
        p.live = __ballot(gblock < a.nblocks && (d.r != 0 || d.cent != 0)) != 0;
    }
    return p;
}

// Decompression steps 4-5 of a live wave: bit-unshuffle, inverse cross-block
// prediction (one inclusive scan for LZ1, two for LZ2, plus the tile mean),
// x' = (float)q * E.
template <bool ALIGNED, bool STAGED, int W, bool RANGE = false>
__device__ __forceinline__ void dec_decode(const DecompressArgs &a, const DecChunk &d, const DecPlace &p, float E,
                                           bool indep, uint32_t *st)
{
    const int lane = threadIdx.x & 63;
    const int j = lane & 7;
    const uint64_t tile0 = p.tile0;
    const uint64_t gblock = (tile0 + (lane >> 3)) * kBlocksPerTile + j;
    const bool blk_ok = gblock < a.nblocks;
    const uint8_t *wave_data = p.wave_data;
    int mu = 0;
    if (d.cent) mu = (int)*(const g_u32 *)(wave_data + d.tile_excl);

    // ---- bit-unshuffle: stored words -> residuals.  With ns = -sign, a
    // residual is (m ^ ns) + sign for its magnitude m, and the bit planes of
    // m ^ ns are the stored magnitude planes xor the sign map (word 0); the
    // planes at or above the block's rate are zero, so there it is the sign
    // map itself.  G groups of 8 planes give x = (m ^ ns) mod 2^(8 G), so the
    // residual is x + sign (1 - 2^(8 G)) (mod 2^32).
    uint32_t code[32];
#pragma unroll
    for (int i = 0; i < 32; i++) code[i] = 0;
    const uint32_t r = blk_ok ? d.r : 0;  // magnitude planes
    const g_u32 *words = (const g_u32 *)(wave_data + d.blk_off);
    const uint32_t sw = r ? words[0] : 0u;  // sign map: element i at bit i ^ 7
    uint32_t G = 0;                         // groups assembled (wave-uniform)
    for (uint32_t g = 0; __ballot(8 * g < r) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int k = 0; k < 8; k++) Rg[k] = (8 * g + k < r ? words[1 + 8 * g + k] : 0u) ^ sw;
        transpose8(Rg);
        // Rg[rho] byte k = byte g of x of element 8k + 7 - rho
#pragma unroll
        for (int rho = 0; rho < 8; rho++) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t sel = (0x03020100u & ~(0xFFu << (8 * g))) | ((4u + k) << (8 * g));
                code[8 * k + 7 - rho] = __builtin_amdgcn_perm(Rg[rho], code[8 * k + 7 - rho], sel);
            }
        }
        G = g + 1;
    }

    // ---- inverse cross-block prediction + dequantization
    const uint32_t M = G < 4 ? 1u - (1u << (8 * G)) : 1u;  // 1 - 2^(8 G) mod 2^32
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const uint32_t ns = (uint32_t)((int)(sw << (31 - (i ^ 7))) >> 31);  // -sign
        acc += code[i] + (ns & M);
        code[i] = acc;  // first running sum (LZ1 reconstruction / LZ2 first differences)
    }
    // carries from the blocks before in the tile (none when every block
    // restarts prediction)
    const uint32_t start1 = indep ? 0u : group_excl_scan(acc, j);
    const bool any2 = __ballot(d.order2) != 0;  // wave-uniform: some tile of the wave is LZ2
    uint32_t acc2 = 0;
    if (any2) {
#pragma unroll
        for (int i = 0; i < 32; i++) {
            acc2 += code[i] + start1;
        }
    }
    const uint32_t start2 = indep ? 0u : group_excl_scan(acc2, j);
    float xo[32];
    // the tile mean enters the start of the running sum that is the lane's
    // result: the first (LZ1) or the second (LZ2)
    const uint32_t s1 = start1 + (d.order2 ? 0u : (uint32_t)mu);
    if (!any2) {
#pragma unroll
        for (int i = 0; i < 32; i++) xo[i] = (float)(int)(code[i] + s1) * E;
    } else {
        uint32_t run = start2 + (d.order2 ? (uint32_t)mu : 0u);
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const uint32_t d1 = code[i] + s1;  // first running sum with the carry
            run += d1;                         // second running sum
            xo[i] = (float)(int)(d.order2 ? run : d1) * E;
        }
    }

    const uint64_t eblk = gblock * kBlock;
    const int cnt = eblk >= a.n ? 0 : (a.n - eblk >= kBlock ? kBlock : (int)(a.n - eblk));
    // element e of the field goes to out[e - eb], for eb <= e < ee
    g_f32 *out = (g_f32 *)a.out;
    const uint64_t eb = RANGE ? a.elem_begin : 0, ee = RANGE ? a.elem_end : a.n;
    if (!STAGED) {  // lane-per-block stores, 8 x 16 B per lane
        if (ALIGNED && cnt == 32 && eblk >= eb && eblk + 32 <= ee) {
            g_u32x4 *p = (g_u32x4 *)(out + (eblk - eb));
#pragma unroll
            for (int k = 0; k < 8; k++)
                p[k] = u32x4{__float_as_uint(xo[4 * k]), __float_as_uint(xo[4 * k + 1]), __float_as_uint(xo[4 * k + 2]),
                             __float_as_uint(xo[4 * k + 3])};
        } else {
#pragma unroll
            for (int i = 0; i < 32; i++)
                if (i < cnt && eblk + i >= eb && eblk + i < ee) out[eblk + i - eb] = xo[i];
        }
        return;
    }
    // ---- write back through LDS with coalesced stores
#pragma unroll
    for (int k = 0; k < 8; k++)
        *reinterpret_cast<float4 *>(st + lane * kStageRowDwords + 4 * k) =
            make_float4(xo[4 * k], xo[4 * k + 1], xo[4 * k + 2], xo[4 * k + 3]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const uint64_t e0 = tile0 * kTile;
    const bool fullw = e0 >= eb && e0 + 2048 <= ee;  // the wave's 8 tiles lie inside the range
    if (ALIGNED) {  // 16-byte aligned: a.out - eb (the field's element 0) is
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = e0 + 4ull * p;
            const u32x4 f = *reinterpret_cast<const u32x4 *>(st + (p >> 3) * kStageRowDwords + (p & 7) * 4);
            if (fullw || (e >= eb && e + 4 <= ee)) {
                __builtin_nontemporal_store(f, (g_u32x4 *)(out + (e - eb)));
            } else {
                if (e + 0 >= eb && e + 0 < ee) out[e + 0 - eb] = __uint_as_float(f.x);
                if (e + 1 >= eb && e + 1 < ee) out[e + 1 - eb] = __uint_as_float(f.y);
                if (e + 2 >= eb && e + 2 < ee) out[e + 2 - eb] = __uint_as_float(f.z);
                if (e + 3 >= eb && e + 3 < ee) out[e + 3 - eb] = __uint_as_float(f.w);
            }
        }
    } else {
#pragma unroll 8
        for (int k = 0; k < 32; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = e0 + p;
            if (fullw || (e >= eb && e < ee))
                out[e - eb] = __uint_as_float(st[(p >> 5) * kStageRowDwords + (p & 31)]);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// Stream header validation (identical in every workgroup): status, step E
// and the stream's total size.
__device__ __forceinline__ int dec_header(const DecompressArgs &a, float &E, uint64_t &total, bool &indep)
{
    const uint32_t *h = reinterpret_cast<const uint32_t *>(a.cmp);
    E = 1.0f;
    total = 0;
    const uint32_t h1 = h[1];
    indep = false;
    // flags: bits 0-1 free, bits 2-4 the tile configuration (a.cfg_flags: 0 for
    // the default format), the rest zero
    if (h[0] != 0x315A5346u || (h1 & 0xFFFFu) != 1u || ((h1 >> 16) & 0xFFu) > 1u || ((h1 >> 24) & ~0x1Fu) != 0u ||
        ((h1 >> 24) & 0x1Cu) != a.cfg_flags)
        return FSZ_ERR_CORRUPT;
    indep = ((h1 >> 25) & 1u) != 0;  // flags bit 1: prediction restarts at every block
    if (((uint64_t)h[3] << 32 | h[2]) != a.n) return FSZ_ERR_SIZE_MISMATCH;
    E = __uint_as_float(h[4]);
    total = (uint64_t)h[7] << 32 | h[6];
    if (!__builtin_isfinite(E) || !(E > 0.0f) || total > a.cmp_size || total < a.data0) return FSZ_ERR_CORRUPT;
    return FSZ_OK;
}

// Persistent decompression kernel: the size pass of the next chunk (which
// publishes its aggregate) runs before the decode of the current one.
// W waves per workgroup; a chunk is 8 tiles per wave (a.nchunks counts chunks
// of that size).
template <bool ALIGNED, bool STAGED, int W, bool RANGE = false, bool PREZERO = false, bool PRESCAN = false>
__global__ __launch_bounds__(W * 64) void decompress_kernel(DecompressArgs a)
{
    __shared__ __attribute__((aligned(16))) uint32_t stage[STAGED ? W * kStageWaveDwords : 4];
    __shared__ DecompressShared<W> sh;
    const int tid = threadIdx.x;
    uint32_t *st = stage + (STAGED ? (tid >> 6) * kStageWaveDwords : 0);

    float E;
    uint64_t total;
    bool indep;
    const int hst = dec_header(a, E, total, indep);
    if (PRESCAN) {  // the pre-pass checked the stream and reported its outcome
        if (*a.go != FSZ_OK) return;
    } else if (hst != FSZ_OK) {
        if (tid == 0 && blockIdx.x == 0) write_final(a.final, 0, hst, a.epoch);
        return;
    }

    // Chunks come from the ticket counter, in increasing order over the
    // running workgroups, so that lookbacks only wait on running chunks.  With
    // offsets from the pre-pass no workgroup waits on another, and a static
    // schedule (chunk = workgroup + k * grid) saves the ticket's round trip.
    int tslot = 0;
    const uint64_t takes = a.nchunks + gridDim.x;
    uint64_t cur = PRESCAN ? (uint64_t)blockIdx.x : next_ticket(a.ticket, takes, sh, tslot);
    if (cur >= a.nchunks) return;
    int slot = 0;
    DecChunk dc = dec_sizes<W, RANGE, PRESCAN>(a, cur, dec_rate_byte<W, RANGE>(a, cur), slot, sh);
    for (;;) {
        const uint64_t nxt = PRESCAN ? cur + gridDim.x : next_ticket(a.ticket, takes, sh, tslot);
        DecChunk dn;
        if (nxt < a.nchunks)
            dn = dec_sizes<W, RANGE, PRESCAN>(a, nxt, dec_rate_byte<W, RANGE>(a, nxt), slot ^ 1, sh);
        const DecPlace pl = dec_place<W, RANGE, PREZERO, PRESCAN>(a, dc, slot, total, sh);
        if (pl.live) dec_decode<ALIGNED, STAGED, W, RANGE>(a, dc, pl, E, indep, st);
        if (nxt >= a.nchunks) break;
        dc = dn;
        cur = nxt;
        slot ^= 1;
    }
}

// ------------------------------------------------------------------ whole-field decode: offsets pre-pass
//
// A whole-field decode's chunk offsets depend on the rate header alone
// (decompression steps 1-2, Sec. III-A), so one small launch computes them
// before the decoder starts, and the decoder reads its chunk's offset instead
// of waiting on a lookback.

// The offsets pre-pass, in one pass: workgroups of 1024 threads, each thread
// 4 consecutive tiles, taken in ticket order.  A workgroup adds up its tiles'
// sizes, publishes its total in the flag words and takes its exclusive prefix
// by the decoupled lookback, then writes the offsets of its chunks (TPC tiles
// each, so no chunk straddles two threads or workgroups).  Reserved rate-byte
// bits ride on the flags' error bit; the workgroup holding the last tiles
// checks the header's total and the padding and reports the outcome.
constexpr int kScanThreads = 1024;
constexpr int kScanTilesPerThread = 4;
constexpr int kScanTiles = kScanThreads * kScanTilesPerThread;

// TPC tiles per decoder chunk; T blocks per tile of HB 32-element segments
// each (the default format: 8 and 1; the tile configurations: the stream's).
template <int TPC, int T = kBlocksPerTile, int HB = 1>
__global__ __launch_bounds__(kScanThreads) void dec_offsets_single_kernel(DecompressArgs a, unsigned long long *offs,
                                                                          uint32_t *go, uint64_t ngroups)
{
    static_assert(T == 4 || T == 8 || T == 16, "a tile's rate bytes are 1, 2 or 4 words");
    static_assert(TPC % kScanTilesPerThread == 0, "a chunk starts at a thread's first tile");
    __shared__ uint32_t wsum[kScanThreads / 64];
    __shared__ unsigned long long gbase;
    __shared__ unsigned long long tk;
    __shared__ int gbad;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    if (tid == 0) {
        tk = take_ticket(a.ticket, ngroups);
        gbad = 0;
    }
    __syncthreads();
    const uint64_t g = tk;
    float E;
    uint64_t total;
    bool indep;
    const int hst = dec_header(a, E, total, indep);
    if (hst != FSZ_OK) {
        if (tid == 0 && g == 0) {
            *go = (uint32_t)hst;
            write_final(a.final, 0, hst, a.epoch);
        }
        return;
    }
    // the rate bytes of a tile lie inside the (zero-padded) rate header, which
    // the header check placed inside the buffer
    const uint64_t tile0 = (g * kScanThreads + tid) * kScanTilesPerThread;
    uint32_t z = 0, bad = 0;
#pragma unroll
    for (int i = 0; i < kScanTilesPerThread; i++) {
        const uint64_t tile = tile0 + i;
        if (tile < a.ntiles) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(a.cmp + kHeaderBytes + tile * T);
            uint32_t rw[T / 4];
#pragma unroll
            for (int q = 0; q < T / 4; q++) rw[q] = p[q];
            const uint64_t nb64 = a.nblocks - tile * T;
            const uint32_t nb = nb64 < (uint64_t)T ? (uint32_t)nb64 : (uint32_t)T;
#pragma unroll
            for (uint32_t b = 0; b < (uint32_t)T; b++) {
                const uint32_t rb = (rw[b >> 2] >> (8 * (b & 3))) & 0xFFu;
                if (b < nb) {
                    bad |= b == 0 ? (rb & 0x20u) : (rb & 0xE0u);
                    z += HB * block_bytes(rb & 31u) + ((b == 0 && (rb & 0x40u)) ? 4u : 0u);
                }
            }
        }
    }
    const uint32_t incl = (uint32_t)wave_incl_scan((int)z);
    if (lane == 63) wsum[w] = incl;
    if (__ballot(bad != 0) != 0 && lane == 0) gbad = 1;
    __syncthreads();
    uint32_t wave_base = 0, gtotal = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; k++) {
        if (k < w) wave_base += wsum[k];
        gtotal += wsum[k];
    }
    if (w == 0) {
        bool padbad = false;
        if (g == ngroups - 1) {  // the rate header's zero padding: at most 15 bytes, one lane each
            const uint64_t k = kHeaderBytes + a.nblocks + (uint64_t)lane;
            padbad = __ballot(lane < 16 && k < a.data0 && a.cmp[k] != 0) != 0;
        }
        if (lane == 0) publish_aggregate(a.flags, g, a.flag_epoch, gtotal, gbad != 0);
        const Prefix pre = lookback_wait(a.flags, g, a.flag_epoch, gtotal, gbad != 0);
        if (lane == 0) {
            gbase = pre.excl;
            if (g == ngroups - 1) {  // pre.err: a reserved bit in any group (or a lookback that gave up)
                const bool ok = !pre.err && !padbad && a.data0 + pre.excl + gtotal == total;
                const uint32_t st = ok ? (uint32_t)FSZ_OK : (uint32_t)FSZ_ERR_CORRUPT;
                *go = st;
                write_final(a.final, total, st, a.epoch);
            }
        }
    }
    __syncthreads();
    if (tile0 < a.ntiles && (tile0 % TPC) == 0) offs[tile0 / TPC] = gbase + wave_base + incl - z;
    if (a.ntiles == 0 && tid == 0) offs[0] = 0;
}

// Whole-field decoder for the offsets pre-pass, one chunk of 8*W tiles per
// workgroup and no ticket: with every chunk's offset known there is no order
// to keep, and the hardware dispatcher keeps the CUs busy.  Used for fields
// too small to give a persistent grid several chunks per workgroup.
template <bool ALIGNED, int W>
__global__ __launch_bounds__(W * 64) void decompress_direct_kernel(DecompressArgs a)
{
    __shared__ __attribute__((aligned(16))) uint32_t stage[W * kStageWaveDwords];
    __shared__ DecompressShared<W> sh;
    if (*a.go != FSZ_OK) return;  // the pre-pass checked the stream and reported its outcome
    float E;
    uint64_t total;
    bool indep;
    dec_header(a, E, total, indep);
    const uint64_t chunk = blockIdx.x;
    uint32_t *st = stage + (threadIdx.x >> 6) * kStageWaveDwords;
    const DecChunk dc = dec_sizes<W, false, true>(a, chunk, dec_rate_byte<W>(a, chunk), 0, sh);
    const DecPlace pl = dec_place<W, false, false, true>(a, dc, 0, total, sh);
    if (pl.live) dec_decode<ALIGNED, true, W>(a, dc, pl, E, indep, st);
}

// ------------------------------------------------------------------ random-access decode

// Byte offset of a range's first tile, from the rate header alone (the block
// sizes of decompression step 2, Sec. III-A): each workgroup sums the sizes of
// a grid-stride share of the blocks before tile_begin; a reserved rate-byte
// bit sets bit 63 of the partial.
__global__ __launch_bounds__(kStatsThreads) void range_partial_kernel(DecompressArgs a, unsigned long long *partials)
{
    const uint64_t nb = a.tile_begin * kBlocksPerTile;  // every tile before the last is whole
    unsigned long long sum = 0;
    uint32_t bad = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
        if (kHeaderBytes + b >= a.cmp_size) {  // a stream shorter than its rate header
            bad = 1;
            break;
        }
        const uint32_t rb = a.cmp[kHeaderBytes + b];
        const bool head = (b & (kBlocksPerTile - 1)) == 0;
        bad |= head ? (rb & 0x20u) : (rb & 0xE0u);
        sum += block_bytes(rb & 31u) + ((head && (rb & 0x40u)) ? 4u : 0u);
    }
    sum = wave_sum_u64(sum);
    const bool wbad = __ballot(bad != 0) != 0;
    __shared__ unsigned long long wsum[kStatsThreads / 64];
    __shared__ uint32_t wflag[kStatsThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6] = sum;
        wflag[threadIdx.x >> 6] = wbad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        uint32_t f = 0;
        for (int k = 0; k < kStatsThreads / 64; k++) {
            t += wsum[k];
            f |= wflag[k];
        }
        partials[blockIdx.x] = t | ((unsigned long long)f << 63);
    }
}

// Folds the partials into *out; a reserved bit anywhere makes the offset
// 2^62, past any stream, so the decode reports a corrupt stream.
__global__ __launch_bounds__(64) void range_final_kernel(const unsigned long long *partials, unsigned nparts,
                                                         unsigned long long *out)
{
    unsigned long long t = 0;
    bool bad = false;
    for (unsigned i = threadIdx.x; i < nparts; i += 64) {
        t += partials[i] & ~(1ull << 63);
        bad = bad || (partials[i] >> 63) != 0;
    }
    t = wave_sum_u64(t);
    bad = __ballot(bad) != 0;
    if (threadIdx.x == 0) *out = bad ? (1ull << 62) : t;
}

// ------------------------------------------------------------------ batched form

// Index of the job owning global item t, given the non-decreasing array
// end[j] = first item after job j: the number of jobs with end[j] <= t.
// Run by a whole wave (64 jobs per probe); the result is wave-uniform.
__device__ __forceinline__ uint32_t find_job(const uint64_t *end, uint32_t njobs, uint64_t t)
{
    const int lane = __lane_id();
    for (uint32_t base = 0; base < njobs; base += 64) {
        const uint32_t idx = base + lane;
        const unsigned long long m = __ballot(idx < njobs && end[idx] <= t);
        if (m != ~0ull) return base + (uint32_t)__builtin_popcountll(m);
    }
    return njobs;
}

// Batched range pass: workgroup s reduces segment s (kSegElems elements of
// one compress job) into partials[s]; every workgroup also clears a slice of
// the batch's chunk flags for the kernel that follows.
template <bool ALIGNED>
__global__ __launch_bounds__(kStatsThreads) void batch_stats_kernel(BatchArgs b)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kStatsThreads + threadIdx.x; i < b.nflags;
         i += (uint64_t)gridDim.x * kStatsThreads)
        b.flags[i] = 0;
    // workgroups loop over segments (one partial each), so the job search and
    // the workgroup start are paid once per several segments
    for (uint64_t seg = blockIdx.x; seg < b.total_segs; seg += gridDim.x) {
        const uint32_t job = __builtin_amdgcn_readfirstlane(find_job(b.seg_end, b.njobs, seg));
        if (job >= b.njobs) return;
        const BatchJob &J = b.jobs[job];
        const g_f32 *x = (const g_f32 *)J.src;
        const uint64_t e0 = (seg - J.seg_base) * kSegElems;
        const uint64_t e1 = J.n - e0 < (uint64_t)kSegElems ? J.n : e0 + kSegElems;
        RangeAcc acc;
        const int tid = threadIdx.x;
        if (ALIGNED) {  // 16-byte loads, four in flight per thread; a ragged segment's last 0-3 elements singly
            const g_f4 *x4 = (const g_f4 *)(x + e0);
            const uint32_t nv = (uint32_t)((e1 - e0) / 4);
            if (nv == kSegElems / 4) {
#pragma unroll 2
                for (int k = 0; k < kSegElems / (4 * kStatsThreads); k += 4) {
                    const f4 f0 = __builtin_nontemporal_load(x4 + (k + 0) * kStatsThreads + tid);
                    const f4 f1 = __builtin_nontemporal_load(x4 + (k + 1) * kStatsThreads + tid);
                    const f4 f2 = __builtin_nontemporal_load(x4 + (k + 2) * kStatsThreads + tid);
                    const f4 f3 = __builtin_nontemporal_load(x4 + (k + 3) * kStatsThreads + tid);
                    acc.take4(f0);
                    acc.take4(f1);
                    acc.take4(f2);
                    acc.take4(f3);
                }
            } else {
                uint32_t k = tid;
                for (; k + 3 * kStatsThreads < nv; k += 4 * kStatsThreads) {
                    const f4 f0 = __builtin_nontemporal_load(x4 + k);
                    const f4 f1 = __builtin_nontemporal_load(x4 + k + kStatsThreads);
                    const f4 f2 = __builtin_nontemporal_load(x4 + k + 2 * kStatsThreads);
                    const f4 f3 = __builtin_nontemporal_load(x4 + k + 3 * kStatsThreads);
                    acc.take4(f0);
                    acc.take4(f1);
                    acc.take4(f2);
                    acc.take4(f3);
                }
                for (; k < nv; k += kStatsThreads) acc.take4(f4(x4[k]));
                const uint64_t t = e0 + 4ull * nv + tid;
                if (t < e1) acc.take(x[t]);
            }
        } else {
            for (uint64_t i = e0 + tid; i < e1; i += kStatsThreads) acc.take(x[i]);
        }
        const StatsPartial p = acc.reduce();
        if (tid == 0) b.partials[seg] = p;
        __syncthreads();  // the reduction's shared slots are reused by the next segment
    }
}

// Per-job fold of the batched range pass (one workgroup per job).
__global__ __launch_bounds__(kStatsThreads) void batch_stats_final_kernel(BatchArgs b)
{
    const BatchJob &J = b.jobs[blockIdx.x];
    if (J.op != FSZ_OP_COMPRESS) return;
    float mn = INFINITY, mx = -INFINITY, ma = 0.0f;
    uint32_t nf = 0;
    for (uint64_t i = threadIdx.x; i < J.nsegs; i += kStatsThreads)
        stats_combine(mn, mx, ma, nf, b.partials[J.seg_base + i]);
    const StatsPartial p = stats_block_reduce(mn, mx, ma, nf);
    if (threadIdx.x == 0) b.stats[blockIdx.x] = fsz_stats{p.xmin, p.xmax, p.maxabs, p.flags};
}

// The arguments of job J's chunks, as the whole-field kernels take them.
__device__ __forceinline__ CompressArgs batch_compress_args(const BatchArgs &b, uint32_t job, const BatchJob &J)
{
    CompressArgs a;
    a.x = static_cast<const float *>(J.src);
    a.n = J.n;
    a.ntiles = J.ntiles;
    a.nblocks = J.nblocks;
    a.nchunks = J.nchunks;
    a.data0 = J.data0;
    a.out = static_cast<uint8_t *>(J.dst);
    a.capacity = J.dst_capacity;
    a.stats = b.stats + job;
    a.value = J.value;
    a.mode = J.mode;
    a.features = kFeaturesAll;
    a.cfg_flags = 0;
    a.epoch = b.epoch;
    a.flag_epoch = 1;
    a.flags = b.flags + J.chunk_base * kFlagStride;
    a.ticket = nullptr;
    a.final = J.final;
    return a;
}

__device__ __forceinline__ DecompressArgs batch_decompress_args(const BatchArgs &b, const BatchJob &J)
{
    DecompressArgs a;
    a.cmp = static_cast<const uint8_t *>(J.src);
    a.cmp_size = J.src_size;
    a.out = static_cast<float *>(J.dst);
    a.n = J.n;
    a.ntiles = J.ntiles;
    a.nblocks = J.nblocks;
    a.nchunks = J.nchunks;
    a.data0 = J.data0;
    a.tile_begin = 0;
    a.tile_end = J.ntiles;
    a.elem_begin = 0;
    a.elem_end = J.n;
    a.range_base = nullptr;
    a.cfg_flags = 0;
    a.epoch = b.epoch;
    a.flag_epoch = 1;
    a.flags = b.flags + J.chunk_base * kFlagStride;
    a.ticket = nullptr;
    a.final = J.final;
    return a;
}

// Batched kernel: one (job, chunk) item per workgroup, items from one ticket
// counter in job order, so every lookback waits only on items already
// running, and lookback chains stay per job (each job has its own flag
// range).  The item runs the whole-field per-chunk code, so every job's bytes
// equal a plain call's.
template <bool ALIGNED, int W>
__global__ __launch_bounds__(W * 64) void batch_kernel(BatchArgs b)
{
    __shared__ union {
        CompressShared<W> c;
        DecompressShared<W> d;
    } sh;
    __shared__ __attribute__((aligned(16))) uint32_t stage[W * kStageWaveDwords];
    __shared__ unsigned long long tk;
    const int tid = threadIdx.x;
    uint32_t *st = stage + (tid >> 6) * kStageWaveDwords;
    if (tid == 0) tk = take_ticket(b.ticket, b.total_chunks);
    lds_barrier();
    const uint64_t t = tk;
    if (t >= b.total_chunks) return;
    const uint32_t job = __builtin_amdgcn_readfirstlane(find_job(b.chunk_end, b.njobs, t));
    if (job >= b.njobs) return;
    const BatchJob &J = b.jobs[job];
    const uint64_t chunk = t - J.chunk_base;
    if (J.op == FSZ_OP_COMPRESS) {
        compress_chunk<ALIGNED, true, true, W>(batch_compress_args(b, job, J), chunk, sh.c, st);
    } else {
        const DecompressArgs a = batch_decompress_args(b, J);
        float E;
        uint64_t total;
        bool indep;
        const int hst = dec_header(a, E, total, indep);
        if (hst != FSZ_OK) {
            if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, hst, a.epoch);
            return;
        }
        const DecChunk dc = dec_sizes<W>(a, chunk, dec_rate_byte<W>(a, chunk), 0, sh.d);
        const DecPlace pl = dec_place<W>(a, dc, 0, total, sh.d);
        if (pl.live) dec_decode<ALIGNED, true, W>(a, dc, pl, E, indep, st);
    }
}

// Batched decompression when every job decompresses: a persistent grid whose
// workgroups take items from the ticket counter until one is past the end.
// The size pass of the next item runs before this item's decode, so its
// aggregate is out before any lookback waits on it (as in the whole-field
// decoder); every item publishes its aggregate before its own lookback and
// tickets are taken in increasing order, so the waits always drain.  Held to
// 128 VGPRs (4 waves per SIMD), as the whole-field decoder.
template <bool ALIGNED, int W>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4))) void batch_dec_kernel(BatchArgs b)
{
    __shared__ DecompressShared<W> sh;
    __shared__ __attribute__((aligned(16))) uint32_t stage[W * kStageWaveDwords];
    const int tid = threadIdx.x;
    uint32_t *st = stage + (tid >> 6) * kStageWaveDwords;
    const uint64_t takes = b.total_chunks + gridDim.x;
    int tslot = 0;
    uint64_t t = next_ticket(b.ticket, takes, sh, tslot);
    bool have = false;  // dc holds the size pass of item t (slot `slot`)
    DecChunk dc;
    int slot = 0;
    while (t < b.total_chunks) {
        const uint32_t job = __builtin_amdgcn_readfirstlane(find_job(b.chunk_end, b.njobs, t));
        const DecompressArgs a = batch_decompress_args(b, b.jobs[job]);
        const uint64_t chunk = t - b.jobs[job].chunk_base;
        const uint64_t nxt = next_ticket(b.ticket, takes, sh, tslot);
        float E;
        uint64_t total;
        bool indep;
        const int hst = dec_header(a, E, total, indep);
        if (hst != FSZ_OK) {
            if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, hst, a.epoch);
            have = false;
        } else {
            if (!have) dc = dec_sizes<W>(a, chunk, dec_rate_byte<W>(a, chunk), slot, sh);
            bool next_have = false;
            DecChunk dn;
            if (nxt < b.total_chunks) {
                const uint32_t job2 = __builtin_amdgcn_readfirstlane(find_job(b.chunk_end, b.njobs, nxt));
                const DecompressArgs a2 = batch_decompress_args(b, b.jobs[job2]);
                const uint64_t chunk2 = nxt - b.jobs[job2].chunk_base;
                float E2;
                uint64_t total2;
                bool indep2;
                if (dec_header(a2, E2, total2, indep2) == FSZ_OK) {
                    dn = dec_sizes<W>(a2, chunk2, dec_rate_byte<W>(a2, chunk2), slot ^ 1, sh);
                    next_have = true;
                }
            }
            const DecPlace pl = dec_place<W>(a, dc, slot, total, sh);
            if (pl.live) dec_decode<ALIGNED, true, W>(a, dc, pl, E, indep, st);
            if (next_have) {
                dc = dn;
                slot ^= 1;
            }
            have = next_have;
        }
        t = nxt;
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

// ------------------------------------------------------------------ batched pipelined compression
//
// Compress-only batches with 16-byte aligned inputs: the pipeline of
// compress_pipe2_kernel over the batch's work items.  Tickets are global item
// ids in job order; every item in flight carries its job, whose arguments
// (input, output, flag range, bound) come from the job table where they are
// needed, so one pipeline runs across job boundaries.  Items of a job whose
// bound does not resolve stay in the pipeline as empty items (no flags, no
// stores); the job's last item reports its status.  Each job's bytes equal a
// plain call's.

struct BItem {
    uint64_t t;    // global item id (>= total_chunks: none)
    uint32_t job;  // job index (njobs: none)
    uint64_t c;    // chunk index inside the job
};

// Up to kPipeLdsJobs job records and their resolved bounds are copied to LDS
// when the kernel starts, so that no step waits on global memory for its
// items' arguments; larger batches read the job table and resolve per use.
constexpr uint32_t kPipeLdsJobs = 96;

struct JobView {
    const BatchJob *jobs;       // LDS copy or the global table
    const Resolved *bound;      // LDS (null: resolve from the job's stats)
    const uint64_t *chunk_end;  // LDS copy or the global table
};

__device__ __forceinline__ Resolved job_bound(const BatchArgs &b, const JobView &v, uint32_t job, const BatchJob &J)
{
    if (v.bound) return v.bound[job];
    return resolve_bound(b.stats + job, J.mode, J.value, J.n);
}

__device__ __forceinline__ BItem batch_item(const BatchArgs &b, const JobView &v, uint64_t t, uint32_t job)
{
    BItem it;
    it.t = t;
    it.job = t < b.total_chunks && job < b.njobs ? job : b.njobs;
    it.c = it.job < b.njobs ? t - v.jobs[it.job].chunk_base : 0;
    return it;
}

__device__ __forceinline__ BItem batch_item_of(const BatchArgs &b, const JobView &v, uint64_t t)
{
    const uint32_t job = t < b.total_chunks ? __builtin_amdgcn_readfirstlane(find_job(v.chunk_end, b.njobs, t))
                                            : b.njobs;
    return batch_item(b, v, t, job);
}

template <int W>
__device__ __forceinline__ void batch_fetch(const BatchArgs &b, const JobView &v, const BItem &it, uint32_t *qb,
                                            int w, int lane)
{
    const BatchJob &J = v.jobs[it.job];
    chunk_fetch<W>(batch_compress_args(b, it.job, J), it.c, qb, w, lane);
}

// Rate pass of item B (as compress_rates with DEFER), or an empty state and
// the same barrier for an item whose job has no valid bound.
template <int W>
__device__ __forceinline__ ChunkState batch_rates(const BatchArgs &b, const JobView &v, const BItem &it,
                                                  int (&x)[32], int slot, CompressShared<W> &sh)
{
    const BatchJob &J = v.jobs[it.job];
    const CompressArgs a = batch_compress_args(b, it.job, J);
    const Resolved R = job_bound(b, v, it.job, J);
    if (R.status == FSZ_OK) {
        ChunkState cs = compress_rates<W, true>(a, R, it.c, x, slot, sh);
        cs.chunk = it.c;
        return cs;
    }
    ChunkState cs{};
    cs.chunk = it.c;
    if ((threadIdx.x & 63) == 0) sh.wave_total[slot][threadIdx.x >> 6] = 0;
    lds_barrier();
    return cs;
}

// One step of the batched pipeline: as pipe2_step, with A, B, C and the new
// item each in its own job.
template <bool W0, int W>
__device__ __forceinline__ BItem batch_pipe_step(const BatchArgs &b, const JobView &v, uint64_t takes,
                                                 const BItem &iA, const ChunkState &ca, int (&xa)[32], int sa,
                                                 const BItem &iB, int (&yb)[32], ChunkState &cb, const BItem &iC,
                                                 uint32_t *qb, uint32_t *pb, CompressShared<W> &sh,
                                                 uint32_t &s_job, int w)
{
    const uint64_t N = b.total_chunks;
    const int lane = threadIdx.x & 63;
    const int j = lane & 7;
    const bool take = iC.t < N;
    const BatchJob &JA = v.jobs[iA.job];
    const CompressArgs aA = batch_compress_args(b, iA.job, JA);
    const Resolved RA = job_bound(b, v, iA.job, JA);
    const bool liveA = RA.status == FSZ_OK;
    unsigned long long traw = 0;
    Probe probe{};
    if (W0) {
        if (take && lane == 0) traw = atomicAdd(b.ticket, 1ull);
        if (liveA) probe = lookback_probe(aA.flags, iA.c, aA.flag_epoch);
    }
    if (iB.t < N) cb = batch_rates<W>(b, v, iB, yb, sa ^ 1, sh);

    // ---- lookback of A (wave 0), the new ticket and its job
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        if (k < w) wave_base += sh.wave_total[sa][k];
        chunk_total += sh.wave_total[sa][k];
    }
    if (W0) {
        // lookback first (as in the single-field pipeline), then the new
        // ticket and its job, found in the LDS copy of the job ends
        Prefix pre{0, false};
        consume_probe(probe);
        if (liveA) pre = lookback_wait(aA.flags, iA.c, aA.flag_epoch, chunk_total, false, true, probe);
        const unsigned long long tk =
            take ? ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(traw >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)traw)
                 : N;
        const uint32_t jobD = tk < N ? find_job(v.chunk_end, b.njobs, tk) : b.njobs;
        if (lane == 0) {
            if (take && tk == takes - 1)
                __hip_atomic_store(b.ticket, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh.base = pre.excl;
            sh.ticket[0] = tk;
            s_job = jobD;
            if (iA.c == aA.nchunks - 1) {
                if (liveA)
                    finish_stream(aA, RA, pre, chunk_total);
                else
                    write_final(aA.final, 0, (uint32_t)RA.status, aA.epoch);
            }
        }
    }
    lds_barrier();
    const uint64_t base = sh.base;
    const BItem iD = batch_item(b, v, sh.ticket[0], s_job);

    const uint64_t tile0 = iA.c * (kTilesPerWave * W) + (uint64_t)w * kTilesPerWave;
    const bool ok = liveA && aA.data0 + base + chunk_total <= aA.capacity && tile0 < aA.ntiles;
    uint32_t *wave_out = reinterpret_cast<uint32_t *>(aA.out + aA.data0 + base + wave_base);
    uint32_t *ps = pb + (((uint32_t)(uintptr_t)wave_out >> 2) & 3u);  // staging at the output's 16-byte phase
    if (ok) pipe2_stage<false>(ca, xa, ps);
    if (iC.t < N) chunk_read(qb, lane, xa);
    if (iD.t < N) {
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the read of qb is done before it is overwritten
        batch_fetch<W>(b, v, iD, qb, w, lane);
    }
    if (liveA && ca.vm != 0)
        ((g_u8 *)aA.out)[kHeaderBytes + (tile0 + (lane >> 3)) * kBlocksPerTile + j] = (uint8_t)ca.rbyte;
    if (ok) {
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        wave_store_staged_phased(wave_out, ps, ca.wave_total >> 2, lane);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    return iD;
}

template <bool W0, int W>
__device__ __forceinline__ void batch_pipe_run(const BatchArgs &b, const JobView &v, CompressShared<W> &sh,
                                               uint32_t &s_job, uint32_t *qb, uint32_t *pb, int w)
{
    const int lane = threadIdx.x & 63;
    const uint64_t N = b.total_chunks;
    const uint64_t takes = N + gridDim.x;
    int tslot = 0;
    BItem iA = batch_item_of(b, v, next_ticket(b.ticket, takes, sh, tslot));
    if (iA.t >= N) return;
    batch_fetch<W>(b, v, iA, qb, w, lane);
    BItem iB = batch_item_of(b, v, next_ticket(b.ticket, takes, sh, tslot));
    int x[32], y[32];
    chunk_read(qb, lane, x);
    if (iB.t < N) {
        __builtin_amdgcn_s_waitcnt(0xC07F);
        batch_fetch<W>(b, v, iB, qb, w, lane);
    }
    ChunkState ca = batch_rates<W>(b, v, iA, x, 0, sh);
    ChunkState cb = ca;
    BItem iC = batch_item(b, v, N, b.njobs);
    if (iB.t < N) {
        iC = batch_item_of(b, v, next_ticket(b.ticket, takes, sh, tslot));
        chunk_read(qb, lane, y);
        if (iC.t < N) {
            __builtin_amdgcn_s_waitcnt(0xC07F);
            batch_fetch<W>(b, v, iC, qb, w, lane);
        }
    }
    // loop invariant: A rate-passed in x (slot 0), B read into y, C in flight
    for (;;) {
        const BItem iD = batch_pipe_step<W0, W>(b, v, takes, iA, ca, x, 0, iB, y, cb, iC, qb, pb, sh, s_job, w);
        if (iB.t >= N) return;
        const BItem iE = batch_pipe_step<W0, W>(b, v, takes, iB, cb, y, 1, iC, x, ca, iD, qb, pb, sh, s_job, w);
        if (iC.t >= N) return;
        iA = iC;
        iB = iD;
        iC = iE;
    }
}

// LDSJOBS (njobs <= kPipeLdsJobs): the job records, their resolved bounds
// and chunk ends are copied to LDS at the start; the view's address space is
// then fixed at compile time, so job fields are read with LDS instructions.
template <int W, bool LDSJOBS>
__global__ __launch_bounds__(W * 64) void batch_pipe_kernel(BatchArgs b)
{
    __shared__ CompressShared<W> sh;
    __shared__ uint32_t s_job;
    __shared__ __attribute__((aligned(16))) uint32_t inbuf[W * kPipeWaveDwords];
    __shared__ __attribute__((aligned(16))) uint32_t stbuf[W * kPipeWaveDwords];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    uint32_t *qb = inbuf + w * kPipeWaveDwords;
    uint32_t *pb = stbuf + w * kPipeWaveDwords;
    if (LDSJOBS) {
        __shared__ __attribute__((aligned(16))) BatchJob ljobs[kPipeLdsJobs];
        __shared__ Resolved lbound[kPipeLdsJobs];
        __shared__ uint64_t lend[kPipeLdsJobs];
        for (uint32_t k = threadIdx.x; k < b.njobs * (uint32_t)(sizeof(BatchJob) / 16); k += blockDim.x)
            reinterpret_cast<u32x4 *>(ljobs)[k] = reinterpret_cast<const u32x4 *>(b.jobs)[k];
        for (uint32_t k = threadIdx.x; k < b.njobs; k += blockDim.x) {
            const BatchJob &J = b.jobs[k];
            lbound[k] = J.op == FSZ_OP_COMPRESS ? resolve_bound(b.stats + k, J.mode, J.value, J.n)
                                                : Resolved{1.0f, 1.0f, 0u, FSZ_ERR_INVALID_ARG};
            lend[k] = b.chunk_end[k];
        }
        lds_barrier();
        const JobView v{ljobs, lbound, lend};
        if (w == 0)
            batch_pipe_run<true, W>(b, v, sh, s_job, qb, pb, w);
        else if (W > 1)
            batch_pipe_run<false, W>(b, v, sh, s_job, qb, pb, w);
    } else {
        const JobView v{b.jobs, nullptr, b.chunk_end};
        if (w == 0)
            batch_pipe_run<true, W>(b, v, sh, s_job, qb, pb, w);
        else if (W > 1)
            batch_pipe_run<false, W>(b, v, sh, s_job, qb, pb, w);
    }
}

// ------------------------------------------------------------------ tile configurations
//
// The tile-configuration sweep of Sec. VI-C (Table V): blocks of B = 32 HB
// elements (HB = 1 or 2) and tiles of T blocks, recorded in header flags bits
// 2-4.  As in the default kernels a lane holds one 32-element segment; a block
// spans HB lanes and a tile L = HB T lanes (4 to 32), so the cross-block chain
// runs over L lanes.  A 64-element block's words (sign map, planes) are 64
// bits with element i at bit 63 - i, written most-significant byte first:
// the stored words of its two halves side by side, so the lane of half h
// writes its word k at byte 8k + 4h of the block.  One chunk of kCfgWaves
// waves (decoder: kCfgDecWaves) per workgroup, chunk ids from the ticket
// counter (as compress_kernel).

// a wave's staging area: the padded input rows (64 x 36 dwords), reused for
// its output (at most 64 x 128 B + 16 tile means = 2064 dwords)
constexpr int kCfgStageDwords = 64 * kStageRowDwords;

// Sum over aligned groups of L lanes, in every lane of the group.  For binary32
// values the butterfly adds the groups' halves in index order at each level,
// so it reproduces the pairwise tree bit for bit (addition is commutative).
template <int L, typename V>
__device__ __forceinline__ V lane_group_sum(V v)
{
#pragma unroll
    for (int k = 1; k < L; k <<= 1) v = v + __shfl_xor(v, k);
    return v;
}

// Inclusive prefix sum over aligned runs of `run` lanes (a power of two, at
// most L); pos = the lane's index inside its group of L lanes.
template <int L>
__device__ __forceinline__ uint32_t lane_run_incl_scan(uint32_t v, int pos, int run)
{
#pragma unroll
    for (int k = 1; k < L; k <<= 1) {
        const uint32_t t = __shfl_up(v, k);
        if (k < run && (pos & (run - 1)) >= k) v += t;
    }
    return v;
}

// Rate pass of one chunk of W waves in a tile configuration (the pipelined
// counterpart of compress_cfg_kernel's first half, for TileCfg): tile mean,
// quantization, cross-block extrema, four-way evaluation and selection, and
// the offsets of the lane's words inside its wave (blk_off, with the lane's
// half h of a 64-element block at byte 4 h).  One workgroup barrier; wave 1
// publishes the chunk's aggregate.  On return x holds the LZ1 residuals.
template <int HB, int L, int W>
__device__ __forceinline__ ChunkState cfg_rates(const CompressArgs &a, const Resolved &R, uint64_t chunk,
                                                int (&x)[32], int slot, CompressShared<W> &sh)
{
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int tl = lane % L;  // lane inside the tile
    const int h = tl % HB;    // half of a 64-element block
    const uint64_t seg0 = (chunk * W + (uint64_t)w) * 64;  // the wave's first segment
    const uint64_t seg = seg0 + lane;
    const uint64_t e0 = seg * 32;
    const int cnt = e0 >= a.n ? 0 : (a.n - e0 >= 32 ? 32 : (int)(a.n - e0));
    const bool tile_ok = seg / L < a.ntiles;
    const bool full = (seg0 + 64) * 32 <= a.n;  // wave-uniform
    ChunkState cs;
    cs.chunk = chunk;
    cs.vm = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);

    // ---- tile mean: pairwise binary32 tree over the B T slots, times 1/(B T)
    float s16[16];
#pragma unroll
    for (int i = 0; i < 16; i++) s16[i] = __int_as_float(x[2 * i]) + __int_as_float(x[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 8; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 2; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
    const float ts = lane_group_sum<L>(s16[0] + s16[1]);
    const float mean_q = (ts * (1.0f / (float)(32 * L))) * R.inv;
    const bool centre_ok = __builtin_isfinite(mean_q);
    const int mu = centre_ok ? (int)__builtin_rintf(mean_q) : 0;
    cs.mu = mu;

    // ---- quantize (biased), cross-block state from the previous lane of the tile
#pragma unroll
    for (int i = 0; i < 32; i++) x[i] = __float_as_int(__int_as_float(x[i]) * R.inv + kQMagic);
    const int p31 = __shfl_up(x[31], 1);
    const int p30 = __shfl_up(x[30], 1);
    const bool first = tl == 0;  // the tile start: the prediction restarts
    cs.first = first;
    const int carry_b = first ? kQBias : p31;
    cs.carry_l1 = first ? 0 : p31 - p30;
    uint32_t a1, a2;
    int l2_1;
    if (full)
        block_extrema<true>(x, carry_b, cs.carry_l1, first ? 0 : 1, cs.vm, a1, a2, l2_1);
    else
        block_extrema<false>(x, carry_b, cs.carry_l1, first ? 0 : 1, cs.vm, a1, a2, l2_1);

    // ---- four-way evaluation (Eq. (3)-(4)) and selection
    uint32_t m0 = a1, m1 = a2, m2 = a1, m3 = a2;
    if (first) {
        const int q0 = x[0];  // d[0] = q[0] at a tile start
        const int d1 = cnt >= 2 ? l2_1 : 0;  // q1 - 2 q0
        const int c0 = q0 - mu;
        const int c1 = cnt >= 2 ? l2_1 + mu : 0;
        m0 = max(uabs(q0), a1);
        m1 = max(max(uabs(q0), uabs(d1)), a2);
        m2 = max(uabs(c0), a1);
        m3 = max(max(uabs(c0), uabs(c1)), a2);
    }
    if (cnt == 0) m0 = m1 = m2 = m3 = 0;  // segments past the end of the field
    if (HB == 2) {
        m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 1));
        m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 1));
        m2 = max(m2, (uint32_t)__shfl_xor((int)m2, 1));
        m3 = max(m3, (uint32_t)__shfl_xor((int)m3, 1));
    }
    const uint32_t r0 = bitlen(m0), r1 = bitlen(m1), r2 = bitlen(m2), r3 = bitlen(m3);
    const uint32_t Ca = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r0) : 0u);
    const uint32_t Cb = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r1) : 0u);
    const uint32_t Cc = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r2) : 0u) + 4u;
    const uint32_t Cd = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r3) : 0u) + 4u;
    int best = 0;
    uint32_t C = Ca, r = r0;
    if (Cb < C) {
        best = 1;
        C = Cb;
        r = r1;
    }
    if (centre_ok) {
        if (Cc < C) {
            best = 2;
            C = Cc;
            r = r2;
        }
        if (Cd < C) {
            best = 3;
            C = Cd;
            r = r3;
        }
    }
    if (!tile_ok) {
        best = 0;
        C = 0;
        r = 0;
    }
    cs.order2 = best & 1;
    cs.cent = best >> 1;
    cs.r = r;
    cs.rbyte = first ? (r | (uint32_t)cs.order2 << 7 | (uint32_t)cs.cent << 6) : r;

    // ---- offsets: the lane's block inside the tile, the tile inside the wave
    const uint32_t S = block_bytes(r);  // this lane's words: 4 (1 + r) bytes
    const uint32_t pre = lane_run_incl_scan<L>(S, tl, L) - S;
    const int incl = wave_incl_scan(first ? (int)C : 0);
    cs.tile_excl = (uint32_t)incl - C;
    cs.wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    cs.blk_off = cs.tile_excl + 4u * (uint32_t)cs.cent + pre - (uint32_t)h * S + 4u * (uint32_t)h;
    if (lane == 0) sh.wave_total[slot][w] = cs.wave_total;
    lds_barrier();
    if (tid == (W > 1 ? 64 : 0)) {
        uint32_t chunk_total = 0;
#pragma unroll
        for (int k = 0; k < W; k++) chunk_total += sh.wave_total[slot][k];
        publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, false);
    }
    return cs;
}

// Residual codes and bit planes of one wave's segments into its staging area
// (word k of the lane's half h of a block at dword blk_off / 4 + HB k).
template <int HB>
__device__ __forceinline__ void cfg_stage(const ChunkState &cs, int (&B)[32], uint32_t *st)
{
    if (cs.vm != 0 && cs.first && cs.cent) st[cs.tile_excl >> 2] = (uint32_t)cs.mu;
    block_codes(B, cs.carry_l1, cs.first ? 0 : 1, cs.order2, cs.cent, cs.mu);
    const uint32_t keep = __builtin_bswap32(__builtin_bitreverse32(cs.vm));
    const uint32_t nwords = cs.r ? cs.r + 1 : 0;
    uint32_t *words = st + (cs.blk_off >> 2);
    for (uint32_t g = 0; __ballot(8 * g < nwords) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int rho = 0; rho < 8; rho++)
            Rg[rho] = pack_byte_g((uint32_t)B[7 - rho], (uint32_t)B[15 - rho], (uint32_t)B[23 - rho],
                                  (uint32_t)B[31 - rho], g);
        transpose8(Rg);
#pragma unroll
        for (int p = 0; p < 8; p++)
            if (8 * g + p < nwords) words[HB * (8 * g + p)] = Rg[p] & keep;
    }
}

// Tile geometry of a configuration for the compression pipeline: HB lanes
// per block, L lanes per tile (a wave's 64 segments hold 64 / L tiles).
template <int HB, int L>
struct TileCfg {
    template <int W, bool FEAT>
    static __device__ __forceinline__ ChunkState rates(const CompressArgs &a, const Resolved &R, uint64_t chunk,
                                                       int (&x)[32], int slot, CompressShared<W> &sh)
    {
        static_assert(!FEAT, "the configuration kernels run the full method");
        return cfg_rates<HB, L, W>(a, R, chunk, x, slot, sh);
    }
    template <bool FEAT>
    static __device__ __forceinline__ void stage(const ChunkState &cs, int (&B)[32], uint32_t *st)
    {
        cfg_stage<HB>(cs, B, st);
    }
    template <int W>
    static __device__ __forceinline__ bool wave_live(const CompressArgs &a, uint64_t chunk, int w)
    {
        return (chunk * W + (uint64_t)w) * 64 / L < a.ntiles;
    }
    template <int W>
    static __device__ __forceinline__ void store_rate(const CompressArgs &a, const ChunkState &cs, int w, int lane)
    {
        if (cs.vm != 0 && lane % HB == 0)
            ((g_u8 *)a.out)[kHeaderBytes + ((cs.chunk * W + (uint64_t)w) * 64 + lane) / HB] = (uint8_t)cs.rbyte;
    }
};

// Pipelined compressor of a tile configuration: compress_ctrl_kernel's
// pipeline (8 data waves, one control wave, persistent workgroups, chunks of
// 8 x 64 segments from the ticket counter) over the configuration's tiles.
// The input must be 16-byte aligned; a.nchunks counts chunks of
// kCfgPipeChunkSegs segments.  A wave's output (rates <= 24: at most 64 x 100
// B of words and 16 tile means) fits its staging area.
template <int HB, int L>
__global__ __launch_bounds__(9 * 64) void compress_cfg_pipe_kernel(CompressArgs a)
{
    __shared__ CompressShared<8> sh;
    __shared__ __attribute__((aligned(16))) uint32_t inbuf[8 * kPipeWaveDwords];
    __shared__ __attribute__((aligned(16))) uint32_t stbuf[8 * kPipeWaveDwords];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {  // no data work: hand out the tickets, the last chunk reports
        const uint64_t takes = a.nchunks + gridDim.x;
        int tslot = 0;
        for (;;) {
            const uint64_t t = next_ticket(a.ticket, takes, sh, tslot);
            if (t >= a.nchunks) return;
            if (threadIdx.x == 0 && t == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        }
    }
    if (w < 8)
        pipe2_run<false, 8, false, TileCfg<HB, L>>(a, R, sh, inbuf + w * kPipeWaveDwords,
                                                    stbuf + w * kPipeWaveDwords, w);
    else
        ctrl_run<8>(a, R, sh);
}

template <bool ALIGNED, int HB, int L>
__global__ __launch_bounds__(kCfgWaves * 64) void compress_cfg_kernel(CompressArgs a)
{
    __shared__ CompressShared<kCfgWaves> sh;
    __shared__ __attribute__((aligned(16))) uint32_t stage[kCfgWaves * kCfgStageDwords];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int tl = lane % L;  // lane inside the tile
    const int h = tl % HB;    // half of a 64-element block
    uint32_t *st = stage + w * kCfgStageDwords;
    int tslot = 0;
    const uint64_t chunk = next_ticket(a.ticket, a.nchunks, sh, tslot);
    if (chunk >= a.nchunks) return;  // inconsistent ticket counter: never index past the flags
    const Resolved R = resolve_bound(a.stats, a.mode, a.value, a.n);
    if (R.status != FSZ_OK) {
        if (tid == 0 && chunk == a.nchunks - 1) write_final(a.final, 0, R.status, a.epoch);
        return;
    }
    const uint64_t seg0 = (chunk * kCfgWaves + w) * 64;  // the wave's first segment
    const uint64_t seg = seg0 + lane;
    const uint64_t e0 = seg * 32;
    const int cnt = e0 >= a.n ? 0 : (a.n - e0 >= 32 ? 32 : (int)(a.n - e0));
    const bool tile_ok = seg / L < a.ntiles;
    const bool full = (seg0 + 64) * 32 <= a.n;  // wave-uniform
    const uint32_t vm = cnt >= 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);
    int x[32];
    {
        float f[32];
        if (seg0 * 32 < a.n) {  // coalesced loads of the wave's 2048 elements through LDS
            load_blocks_staged<ALIGNED>(a.x, a.n, seg0 * 32, st, lane, f);
        } else {
#pragma unroll
            for (int i = 0; i < 32; i++) f[i] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 32; i++) x[i] = __float_as_int(f[i]);
    }

    // ---- tile mean: pairwise binary32 tree over the B T slots, times 1/(B T)
    float s16[16];
#pragma unroll
    for (int i = 0; i < 16; i++) s16[i] = __int_as_float(x[2 * i]) + __int_as_float(x[2 * i + 1]);
#pragma unroll
    for (int i = 0; i < 8; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 4; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
#pragma unroll
    for (int i = 0; i < 2; i++) s16[i] = s16[2 * i] + s16[2 * i + 1];
    const float ts = lane_group_sum<L>(s16[0] + s16[1]);
    const float mean_q = (ts * (1.0f / (float)(32 * L))) * R.inv;
    const bool centre_ok = __builtin_isfinite(mean_q);
    const int mu = centre_ok ? (int)__builtin_rintf(mean_q) : 0;

    // ---- quantize (biased), cross-block state from the previous lane of the tile
#pragma unroll
    for (int i = 0; i < 32; i++) x[i] = __float_as_int(__int_as_float(x[i]) * R.inv + kQMagic);
    const int p31 = __shfl_up(x[31], 1);
    const int p30 = __shfl_up(x[30], 1);
    const bool first = tl == 0;  // the tile start: the prediction restarts
    const int carry_b = first ? kQBias : p31;
    const int carry_l1 = first ? 0 : p31 - p30;
    uint32_t a1, a2;
    int l2_1;
    if (full)
        block_extrema<true>(x, carry_b, carry_l1, first ? 0 : 1, vm, a1, a2, l2_1);
    else
        block_extrema<false>(x, carry_b, carry_l1, first ? 0 : 1, vm, a1, a2, l2_1);

    // ---- four-way evaluation (Eq. (3)-(4)): block magnitude maxima per
    // variant, the tile start re-rated per variant
    uint32_t m0 = a1, m1 = a2, m2 = a1, m3 = a2;
    if (first) {
        const int q0 = x[0];  // d[0] = q[0] at a tile start
        const int d1 = cnt >= 2 ? l2_1 : 0;  // q1 - 2 q0
        const int c0 = q0 - mu;
        const int c1 = cnt >= 2 ? l2_1 + mu : 0;
        m0 = max(uabs(q0), a1);
        m1 = max(max(uabs(q0), uabs(d1)), a2);
        m2 = max(uabs(c0), a1);
        m3 = max(max(uabs(c0), uabs(c1)), a2);
    }
    if (cnt == 0) m0 = m1 = m2 = m3 = 0;  // segments past the end of the field
    if (HB == 2) {
        m0 = max(m0, (uint32_t)__shfl_xor((int)m0, 1));
        m1 = max(m1, (uint32_t)__shfl_xor((int)m1, 1));
        m2 = max(m2, (uint32_t)__shfl_xor((int)m2, 1));
        m3 = max(m3, (uint32_t)__shfl_xor((int)m3, 1));
    }
    const uint32_t r0 = bitlen(m0), r1 = bitlen(m1), r2 = bitlen(m2), r3 = bitlen(m3);
    // block costs (B/8 bytes per word, sign map + r planes), counted once per block
    const uint32_t Ca = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r0) : 0u);
    const uint32_t Cb = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r1) : 0u);
    const uint32_t Cc = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r2) : 0u) + 4u;
    const uint32_t Cd = lane_group_sum<L>(h == 0 ? (uint32_t)HB * block_bytes(r3) : 0u) + 4u;
    int best = 0;
    uint32_t C = Ca, r = r0;
    if (Cb < C) {
        best = 1;
        C = Cb;
        r = r1;
    }
    if (centre_ok) {
        if (Cc < C) {
            best = 2;
            C = Cc;
            r = r2;
        }
        if (Cd < C) {
            best = 3;
            C = Cd;
            r = r3;
        }
    }
    if (!tile_ok) {
        best = 0;
        C = 0;
        r = 0;
    }
    const int order2 = best & 1, cent = best >> 1;
    if (h == 0 && cnt > 0)  // the block's rate byte (Sec. III-A)
        ((g_u8 *)a.out)[kHeaderBytes + seg / HB] = (uint8_t)(first ? (r | (uint32_t)order2 << 7 | (uint32_t)cent << 6) : r);

    // ---- offsets: the lane's block inside the tile, the tile inside the wave
    const uint32_t S = block_bytes(r);  // this lane's words: 4 (1 + r) bytes
    const uint32_t pre = lane_run_incl_scan<L>(S, tl, L) - S;
    const uint32_t blk_rel = 4u * (uint32_t)cent + pre - (uint32_t)h * S;
    const int incl = wave_incl_scan(first ? (int)C : 0);
    const uint32_t tile_excl = (uint32_t)incl - C;
    const uint32_t wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    if (lane == 0) sh.wave_total[0][w] = wave_total;
    lds_barrier();
    uint32_t chunk_total = 0, wave_base = 0;
#pragma unroll
    for (int k = 0; k < kCfgWaves; k++) {
        if (k < w) wave_base += sh.wave_total[0][k];
        chunk_total += sh.wave_total[0][k];
    }
    if (tid == 0) publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, false);
    if (w == 0) {  // decoupled lookback (Sec. IV-D)
        const Prefix pre_c = lookback_wait(a.flags, chunk, a.flag_epoch, chunk_total, false);
        if (lane == 0) {
            sh.base = pre_c.excl;
            if (chunk == a.nchunks - 1) finish_stream(a, R, pre_c, chunk_total);
        }
    }
    lds_barrier();
    const uint64_t base = sh.base;
    if (a.data0 + base + chunk_total > a.capacity || seg0 / L >= a.ntiles) return;

    // ---- encode (Sec. IV-C) into the wave's staging area, then one copy
    if (first && cent && tile_ok) st[tile_excl >> 2] = (uint32_t)mu;
    block_codes(x, carry_l1, first ? 0 : 1, order2, cent, mu);
    const uint32_t keep = __builtin_bswap32(__builtin_bitreverse32(vm));
    const uint32_t nwords = r ? r + 1 : 0;
    uint32_t *words = st + ((tile_excl + blk_rel) >> 2) + h;
    for (uint32_t g = 0; __ballot(8 * g < nwords) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int rho = 0; rho < 8; rho++)
            Rg[rho] = pack_byte_g((uint32_t)x[7 - rho], (uint32_t)x[15 - rho], (uint32_t)x[23 - rho],
                                  (uint32_t)x[31 - rho], g);
        transpose8(Rg);
#pragma unroll
        for (int p = 0; p < 8; p++)
            if (8 * g + p < nwords) words[HB * (8 * g + p)] = Rg[p] & keep;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    wave_store_staged(reinterpret_cast<uint32_t *>(a.out + a.data0 + base + wave_base), st, wave_total >> 2, lane);
}

// WV waves per workgroup, chunks of 64 WV segments (4 waves: a wider grid,
// which small fields need, and several workgroups per CU to hide the lookback
// and the tile loads; 16 in the lookback form of fields above 2^21 elements,
// whose chain the larger chunks halve twice).  PRESCAN: the chunk offsets come from
// dec_offsets_single_kernel<64 WV / L, L / HB, HB> (which also checked the
// stream and reported its outcome): chunk = workgroup, no lookback.
template <bool ALIGNED, int HB, int L, bool PRESCAN = false, int WV = kCfgDecWaves>
__global__ __launch_bounds__(WV * 64) void decompress_cfg_kernel(DecompressArgs a)
{
    __shared__ DecompressShared<WV> sh;
    __shared__ __attribute__((aligned(16))) uint32_t stage[WV * kCfgStageDwords];
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int lane = tid & 63;
    const int tl = lane % L;
    const int h = tl % HB;

    // ---- header: as dec_header, with the configuration bits of this kernel
    const uint32_t *hw = reinterpret_cast<const uint32_t *>(a.cmp);
    const uint32_t h1 = hw[1];
    int hst = FSZ_OK;
    if (hw[0] != 0x315A5346u || (h1 & 0xFFFFu) != 1u || ((h1 >> 16) & 0xFFu) > 1u || ((h1 >> 24) & ~0x1Fu) != 0u ||
        ((h1 >> 24) & 0x1Cu) != a.cfg_flags)
        hst = FSZ_ERR_CORRUPT;
    else if (((uint64_t)hw[3] << 32 | hw[2]) != a.n)
        hst = FSZ_ERR_SIZE_MISMATCH;
    const bool indep = ((h1 >> 25) & 1u) != 0;  // flags bit 1: prediction restarts at every block
    const float E = __uint_as_float(hw[4]);
    const uint64_t total = (uint64_t)hw[7] << 32 | hw[6];
    if (hst == FSZ_OK && (!__builtin_isfinite(E) || !(E > 0.0f) || total > a.cmp_size || total < a.data0))
        hst = FSZ_ERR_CORRUPT;
    if (PRESCAN) {
        if (*a.go != FSZ_OK) return;
    } else if (hst != FSZ_OK) {
        if (tid == 0 && blockIdx.x == 0) write_final(a.final, 0, hst, a.epoch);
        return;
    }
    int tslot = 0;
    const uint64_t chunk = PRESCAN ? (uint64_t)blockIdx.x : next_ticket(a.ticket, a.nchunks, sh, tslot);
    if (chunk >= a.nchunks) return;

    // ---- steps 1-2: rate bytes -> block, tile and wave sizes
    const uint64_t seg0 = (chunk * WV + w) * 64;
    const uint64_t seg = seg0 + lane;
    const bool tile_ok = seg / L < a.ntiles;
    const uint64_t blk = seg / HB;
    const bool blk_ok = tile_ok && blk < a.nblocks;
    const bool first = tl == 0;
    const uint32_t rb = blk_ok ? a.cmp[kHeaderBytes + blk] : 0u;
    const bool bad = blk_ok && h == 0 && (first ? (rb & 0x20u) : (rb & 0xE0u)) != 0;
    const uint32_t head = (uint32_t)__shfl((int)rb, lane - tl);  // the tile's first rate byte
    const int order2 = tile_ok ? (int)((head >> 7) & 1u) : 0;
    const int cent = tile_ok ? (int)((head >> 6) & 1u) : 0;
    const uint32_t r = rb & 31u;
    const uint32_t S = block_bytes(r);  // this lane's words
    const uint32_t Z = lane_group_sum<L>(S) + 4u * (uint32_t)cent;
    const uint32_t pre = lane_run_incl_scan<L>(S, tl, L) - S;
    const uint32_t blk_rel = 4u * (uint32_t)cent + pre - (uint32_t)h * S;
    const int incl = wave_incl_scan(first ? (int)Z : 0);
    const uint32_t tile_excl = (uint32_t)incl - Z;
    const uint32_t wave_total = (uint32_t)__builtin_amdgcn_readlane(incl, 63);
    const bool wave_bad = __ballot(bad) != 0;
    if (lane == 0) {
        sh.wave_total[0][w] = wave_total;
        sh.wave_total[1][w] = wave_bad ? 1u : 0u;
    }
    lds_barrier();
    uint32_t chunk_total = 0, wave_base = 0;
    bool any_bad = false;
#pragma unroll
    for (int k = 0; k < WV; k++) {
        if (k < w) wave_base += sh.wave_total[0][k];
        chunk_total += sh.wave_total[0][k];
        any_bad = any_bad || sh.wave_total[1][k] != 0;
    }
    uint64_t base;
    if (PRESCAN) {
        base = a.offsets[chunk];
    } else {
        if (tid == 0) publish_aggregate(a.flags, chunk, a.flag_epoch, chunk_total, any_bad);
        if (w == 0) {
            const Prefix pre_c = lookback_wait(a.flags, chunk, a.flag_epoch, chunk_total, any_bad);
            if (lane == 0) {
                sh.base = pre_c.excl;
                if (chunk == a.nchunks - 1) {  // the sizes add up to the stream's total, padding is zero
                    bool good = !pre_c.err && a.data0 + pre_c.excl + chunk_total == total;
                    for (uint64_t k = kHeaderBytes + a.nblocks; good && k < a.data0; k++) good = a.cmp[k] == 0;
                    write_final(a.final, total, good ? (uint32_t)FSZ_OK : (uint32_t)FSZ_ERR_CORRUPT, a.epoch);
                }
            }
        }
        lds_barrier();
        base = sh.base;
    }
    if (any_bad || a.data0 + base + chunk_total > total || seg0 / L >= a.ntiles) return;

    // ---- steps 3-5: bit-unshuffle, inverse prediction, x' = (float)q * E
    const uint8_t *wave_data = a.cmp + a.data0 + base + wave_base;
    int mu = 0;
    if (cent) mu = (int)*reinterpret_cast<const uint32_t *>(wave_data + tile_excl);
    // the sign map folded into the magnitude planes, as in dec_decode: a
    // residual is x + sign (1 - 2^(8 G)) (mod 2^32)
    uint32_t code[32];
#pragma unroll
    for (int i = 0; i < 32; i++) code[i] = 0;
    const uint32_t rp = blk_ok ? r : 0;  // magnitude planes
    const uint32_t *words = reinterpret_cast<const uint32_t *>(wave_data + tile_excl + blk_rel) + h;
    const uint32_t sw = rp ? words[0] : 0u;  // the lane's half of the sign map
    uint32_t G = 0;
    for (uint32_t g = 0; __ballot(8 * g < rp) != 0; g++) {
        uint32_t Rg[8];
#pragma unroll
        for (int p = 0; p < 8; p++) Rg[p] = (8 * g + p < rp ? words[HB * (1 + 8 * g + p)] : 0u) ^ sw;
        transpose8(Rg);
        // Rg[rho] byte k = byte g of x of element 8k + 7 - rho
#pragma unroll
        for (int rho = 0; rho < 8; rho++) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t sel = (0x03020100u & ~(0xFFu << (8 * g))) | ((4u + k) << (8 * g));
                code[8 * k + 7 - rho] = __builtin_amdgcn_perm(Rg[rho], code[8 * k + 7 - rho], sel);
            }
        }
        G = g + 1;
    }
    const uint32_t M = G < 4 ? 1u - (1u << (8 * G)) : 1u;  // 1 - 2^(8 G) mod 2^32
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const uint32_t ns = (uint32_t)((int)(sw << (31 - (i ^ 7))) >> 31);  // -sign
        acc += code[i] + (ns & M);
        code[i] = acc;  // first running sum inside the segment
    }
    // carries from the earlier lanes of the prediction run (the tile, or the
    // block when every block restarts)
    const int run = indep ? HB : L;
    const uint32_t start1 = lane_run_incl_scan<L>(acc, tl, run) - acc;
    uint32_t acc2 = 0;
#pragma unroll
    for (int i = 0; i < 32; i++) acc2 += code[i] + start1;
    const uint32_t start2 = lane_run_incl_scan<L>(acc2, tl, run) - acc2;
    float xo[32];
    {
        // the tile mean enters the start of the running sum that is the result
        const uint32_t s1 = start1 + (order2 ? 0u : (uint32_t)mu);
        uint32_t run2 = start2 + (order2 ? (uint32_t)mu : 0u);
#pragma unroll
        for (int i = 0; i < 32; i++) {
            const uint32_t d1 = code[i] + s1;  // first running sum with the carry
            run2 += d1;                        // second running sum
            xo[i] = (float)(int)(order2 ? run2 : d1) * E;
        }
    }
    // ---- write back through LDS with coalesced stores (the wave's 2048 elements)
    uint32_t *st = stage + w * kCfgStageDwords;
#pragma unroll
    for (int k = 0; k < 8; k++)
        *reinterpret_cast<float4 *>(st + lane * kStageRowDwords + 4 * k) =
            make_float4(xo[4 * k], xo[4 * k + 1], xo[4 * k + 2], xo[4 * k + 3]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const uint64_t w0 = seg0 * 32;
    const bool fullw = w0 + 2048 <= a.n;
    if (ALIGNED) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = w0 + 4ull * p;
            const f4 f = *reinterpret_cast<const f4 *>(st + (p >> 3) * kStageRowDwords + (p & 7) * 4);
            if (fullw || e + 4 <= a.n) {
                __builtin_nontemporal_store(f, reinterpret_cast<f4 *>(a.out + e));
            } else {
                if (e + 0 < a.n) a.out[e + 0] = f.x;
                if (e + 1 < a.n) a.out[e + 1] = f.y;
                if (e + 2 < a.n) a.out[e + 2] = f.z;
                if (e + 3 < a.n) a.out[e + 3] = f.w;
            }
        }
    } else {
#pragma unroll 8
        for (int k = 0; k < 32; k++) {
            const int p = k * 64 + lane;
            const uint64_t e = w0 + p;
            if (fullw || e < a.n) a.out[e] = __uint_as_float(st[(p >> 5) * kStageRowDwords + (p & 31)]);
        }
    }
}

// Workgroups of a persistent grid: enough to fill every CU at the kernel's
// occupancy, never more than there are chunks.
template <typename K>
static unsigned persistent_grid(K kernel, uint64_t nchunks, int threads = kThreads)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || cus <= 0 ||
        per_cu <= 0) {
        cus = 256;
        per_cu = 2;
    }
    const uint64_t g = (uint64_t)cus * (uint64_t)per_cu * (uint64_t)tuning().grid_factor;
    return (unsigned)(nchunks < g ? nchunks : g);
}

template <bool ALIGNED, bool LS, bool SS>
static hipError_t launch_compress_t(const CompressArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((compress_kernel<ALIGNED, LS, SS>), dim3((unsigned)a.nchunks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <bool ALIGNED, bool STAGED, int W, bool RANGE = false, bool PREZERO = false, bool PRESCAN = false>
static hipError_t launch_decompress_w(const DecompressArgs &a, hipStream_t s)
{
    // the arguments count chunks of kTilesPerChunk tiles
    DecompressArgs p = a;
    const uint64_t tiles = p.tile_end - p.tile_begin;
    p.nchunks = tiles ? ceil_div(tiles, (uint64_t)kTilesPerWave * W) : 1;
    static const unsigned cap =
        persistent_grid(decompress_kernel<ALIGNED, STAGED, W, RANGE, PREZERO, PRESCAN>, ~0ull, W * 64);
    const unsigned grid = (unsigned)(p.nchunks < cap ? p.nchunks : cap);
    hipLaunchKernelGGL((decompress_kernel<ALIGNED, STAGED, W, RANGE, PREZERO, PRESCAN>), dim3(grid), dim3(W * 64), 0,
                       s, p);
    return hipGetLastError();
}

hipError_t launch_decompress_prescan(const DecompressArgs &a, unsigned long long *offsets, uint32_t *go,
                                     bool out_aligned16, bool direct, hipStream_t s)
{
    // chunks of 8 tiles per wave: 8 waves (persistent grid) or 4 (one chunk per workgroup)
    const int W = direct ? 4 : 8;
    DecompressArgs p = a;
    p.offsets = offsets;
    p.go = go;
    const uint64_t nchunks = a.ntiles ? ceil_div(a.ntiles, (uint64_t)kTilesPerWave * W) : 1;
    const uint64_t ngroups = a.ntiles ? ceil_div(a.ntiles, (uint64_t)kScanTiles) : 1;
    if (direct)
        hipLaunchKernelGGL(dec_offsets_single_kernel<kTilesPerWave * 4>, dim3((unsigned)ngroups), dim3(kScanThreads), 0,
                           s, p, offsets, go, ngroups);
    else
        hipLaunchKernelGGL(dec_offsets_single_kernel<kTilesPerWave * 8>, dim3((unsigned)ngroups), dim3(kScanThreads), 0,
                           s, p, offsets, go, ngroups);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (direct) {
        p.nchunks = nchunks;
        if (out_aligned16)
            hipLaunchKernelGGL((decompress_direct_kernel<true, 4>), dim3((unsigned)nchunks), dim3(256), 0, s, p);
        else
            hipLaunchKernelGGL((decompress_direct_kernel<false, 4>), dim3((unsigned)nchunks), dim3(256), 0, s, p);
        return hipGetLastError();
    }
    return out_aligned16 ? launch_decompress_w<true, true, 8, false, false, true>(p, s)
                         : launch_decompress_w<false, true, 8, false, false, true>(p, s);
}

// +0.0 into out[0, n): 16-byte nontemporal stores from the first 16-byte
// boundary, 4-byte stores for the ragged ends.
__global__ __launch_bounds__(256) void fill_zero_kernel(float *out, uint64_t n)
{
    const uint64_t head = ((16u - (reinterpret_cast<uintptr_t>(out) & 15u)) & 15u) / 4u;
    const uint64_t h = head < n ? head : n;
    const uint64_t nv = (n - h) / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    f4 *v = reinterpret_cast<f4 *>(out + h);
    for (uint64_t i = t; i < nv; i += stride) __builtin_nontemporal_store(f4{0.0f, 0.0f, 0.0f, 0.0f}, v + i);
    if (t < h) out[t] = 0.0f;
    const uint64_t tail = h + 4 * nv;
    if (t < n - tail) out[tail + t] = 0.0f;
}

hipError_t launch_decompress_prezero(const DecompressArgs &a, bool out_aligned16, hipStream_t s)
{
    if (a.n) {
        const uint64_t want = ceil_div(a.n, 4ull * 256);
        const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
        hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, a.out, a.n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return out_aligned16 ? launch_decompress_w<true, true, 8, false, true>(a, s)
                         : launch_decompress_w<false, true, 8, false, true>(a, s);
}

// Waves per workgroup: FSZ_DEC_WAVES if set, else by the elements to decode:
// 8 (64-tile chunks) for up to dec_wide_above, 16 above it, where the shorter
// lookback chain of the larger chunks pays for their coarser spread.
template <bool ALIGNED, bool STAGED>
static hipError_t launch_decompress_t(const DecompressArgs &a, hipStream_t s)
{
    const uint64_t elems = (a.tile_end - a.tile_begin) * kTile;
    const int w = tuning().dec_waves ? tuning().dec_waves : (elems > tuning().dec_wide_above ? 16 : 8);
    switch (w) {
    case 16: return launch_decompress_w<ALIGNED, STAGED, 16>(a, s);
    case 8: return launch_decompress_w<ALIGNED, STAGED, 8>(a, s);
    default: return launch_decompress_w<ALIGNED, STAGED, 4>(a, s);
    }
}

hipError_t launch_compress(const CompressArgs &a, bool in_aligned16, bool staged, hipStream_t s)
{
    if (a.features != kFeaturesAll) {  // the ablation's feature subsets: 8-wave pipeline or the plain kernel
        if (in_aligned16) {
            CompressArgs p = a;
            p.nchunks = p.ntiles ? ceil_div(p.ntiles, (uint64_t)kTilesPerWave * 8) : 1;
            static const unsigned cap = persistent_grid(compress_pipe2_kernel<8, true>, ~0ull, 512);
            hipLaunchKernelGGL((compress_pipe2_kernel<8, true>), dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(512), 0, s, p);
        } else {
            hipLaunchKernelGGL((compress_kernel<false, true, true, true>), dim3((unsigned)a.nchunks), dim3(kThreads), 0,
                               s, a);
        }
        return hipGetLastError();
    }
    if (in_aligned16 && tuning().pipe_compress) {
        // the arguments count chunks of kTilesPerChunk tiles; the pipeline's
        // chunks are 8 tiles per wave
        CompressArgs p = a;
        const int W = tuning().pipe_waves;
        p.nchunks = p.ntiles ? ceil_div(p.ntiles, (uint64_t)kTilesPerWave * W) : 1;
        if (W == 7) p.nchunks = p.ntiles ? ceil_div(p.ntiles, (uint64_t)kTilesPerWave * 7) : 1;
        if (W == 9) p.nchunks = p.ntiles ? ceil_div(p.ntiles, (uint64_t)kTilesPerWave * 8) : 1;
        switch (W) {
        case 7: {  // 7 data waves + 1 control wave
            static const unsigned cap = persistent_grid(compress_ctrl_kernel<7>, ~0ull, 512);
            hipLaunchKernelGGL(compress_ctrl_kernel<7>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(512), 0, s, p);
            break;
        }
        case 9: {  // 8 data waves + 1 control wave
            static const unsigned cap = persistent_grid(compress_ctrl_kernel<8>, ~0ull, 576);
            hipLaunchKernelGGL(compress_ctrl_kernel<8>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(576), 0, s, p);
            break;
        }
        case 1: {
            static const unsigned cap = persistent_grid(compress_pipe2_kernel<1>, ~0ull, 64);
            hipLaunchKernelGGL(compress_pipe2_kernel<1>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(64), 0, s, p);
            break;
        }
        case 2: {
            static const unsigned cap = persistent_grid(compress_pipe2_kernel<2>, ~0ull, 128);
            hipLaunchKernelGGL(compress_pipe2_kernel<2>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(128), 0, s, p);
            break;
        }
        case 8: {
            static const unsigned cap = persistent_grid(compress_pipe2_kernel<8>, ~0ull, 512);
            hipLaunchKernelGGL(compress_pipe2_kernel<8>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(512), 0, s, p);
            break;
        }
        default: {
            static const unsigned cap = persistent_grid(compress_pipe2_kernel<4>, ~0ull, 256);
            hipLaunchKernelGGL(compress_pipe2_kernel<4>, dim3((unsigned)(p.nchunks < cap ? p.nchunks : cap)),
                               dim3(256), 0, s, p);
            break;
        }
        }
        return hipGetLastError();
    }
    const bool ls = tuning().staged_compress_loads;
    if (in_aligned16) {
        if (ls) return staged ? launch_compress_t<true, true, true>(a, s) : launch_compress_t<true, true, false>(a, s);
        return staged ? launch_compress_t<true, false, true>(a, s) : launch_compress_t<true, false, false>(a, s);
    }
    if (ls) return staged ? launch_compress_t<false, true, true>(a, s) : launch_compress_t<false, true, false>(a, s);
    return staged ? launch_compress_t<false, false, true>(a, s) : launch_compress_t<false, false, false>(a, s);
}

hipError_t launch_compress_naive(const CompressArgs &a, const NaiveTables &t, bool in_aligned16, hipStream_t s)
{
    const unsigned grid = (unsigned)a.nchunks;
    for (int v = 0; v < 4; v++) {
        if (in_aligned16)
            hipLaunchKernelGGL(naive_eval_kernel<true>, dim3(grid), dim3(kThreads), 0, s, a, t, v);
        else
            hipLaunchKernelGGL(naive_eval_kernel<false>, dim3(grid), dim3(kThreads), 0, s, a, t, v);
    }
    if (in_aligned16)
        hipLaunchKernelGGL(naive_encode_kernel<true>, dim3(grid), dim3(kThreads), 0, s, a, t);
    else
        hipLaunchKernelGGL(naive_encode_kernel<false>, dim3(grid), dim3(kThreads), 0, s, a, t);
    return hipGetLastError();
}

hipError_t launch_range_base(const DecompressArgs &a, unsigned long long *range_base, unsigned long long *partials,
                             hipStream_t s)
{
    const uint64_t nb = a.tile_begin * kBlocksPerTile;
    const uint64_t want = ceil_div(nb, (uint64_t)kStatsThreads * 16);
    const unsigned grid = (unsigned)(want < 1 ? 1 : (want > kStatsMaxBlocks ? kStatsMaxBlocks : want));
    hipLaunchKernelGGL(range_partial_kernel, dim3(grid), dim3(kStatsThreads), 0, s, a, partials);
    hipLaunchKernelGGL(range_final_kernel, dim3(1), dim3(64), 0, s, partials, grid, range_base);
    return hipGetLastError();
}

hipError_t launch_decompress(const DecompressArgs &a, bool out_aligned16, bool staged, hipStream_t s)
{
    if (a.range_base) {  // random access: the staged decoder with range bookkeeping, 16 waves for long ranges
        if ((a.tile_end - a.tile_begin) * kTile > tuning().dec_wide_above)
            return out_aligned16 ? launch_decompress_w<true, true, 16, true>(a, s)
                                 : launch_decompress_w<false, true, 16, true>(a, s);
        return out_aligned16 ? launch_decompress_w<true, true, 8, true>(a, s)
                             : launch_decompress_w<false, true, 8, true>(a, s);
    }
    if (out_aligned16)
        return staged ? launch_decompress_t<true, true>(a, s) : launch_decompress_t<true, false>(a, s);
    return staged ? launch_decompress_t<false, true>(a, s) : launch_decompress_t<false, false>(a, s);
}

// Tile configurations (Sec. VI-C): (B, T) -> (HB, L) = (B / 32, T B / 32).
template <bool ALIGNED>
static hipError_t launch_compress_cfg_t(const CompressArgs &a, int block, int tile_blocks, hipStream_t s)
{
    const dim3 grid((unsigned)a.nchunks), threads(kCfgWaves * 64);
    const int key = block * 100 + tile_blocks;
    switch (key) {
    case 3204: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 1, 4>), grid, threads, 0, s, a); break;
    case 3208: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 1, 8>), grid, threads, 0, s, a); break;
    case 3216: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 1, 16>), grid, threads, 0, s, a); break;
    case 6404: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 2, 8>), grid, threads, 0, s, a); break;
    case 6408: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 2, 16>), grid, threads, 0, s, a); break;
    case 6416: hipLaunchKernelGGL((compress_cfg_kernel<ALIGNED, 2, 32>), grid, threads, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool ALIGNED, int WV>
static hipError_t launch_decompress_cfg_w(const DecompressArgs &a, int block, int tile_blocks, hipStream_t s)
{
    const dim3 grid((unsigned)a.nchunks), threads(WV * 64);
    const int key = block * 100 + tile_blocks;
    switch (key) {
    case 3204: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 1, 4, false, WV>), grid, threads, 0, s, a); break;
    case 3208: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 1, 8, false, WV>), grid, threads, 0, s, a); break;
    case 3216: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 1, 16, false, WV>), grid, threads, 0, s, a); break;
    case 6404: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 2, 8, false, WV>), grid, threads, 0, s, a); break;
    case 6408: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 2, 16, false, WV>), grid, threads, 0, s, a); break;
    case 6416: hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, 2, 32, false, WV>), grid, threads, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Lookback form: a.nchunks counts chunks of 64 cfg_dec_lookback_waves(n) segments.
template <bool ALIGNED>
static hipError_t launch_decompress_cfg_t(const DecompressArgs &a, int block, int tile_blocks, hipStream_t s)
{
    return cfg_dec_lookback_waves(a.n) == kCfgDecWideWaves
               ? launch_decompress_cfg_w<ALIGNED, kCfgDecWideWaves>(a, block, tile_blocks, s)
               : launch_decompress_cfg_w<ALIGNED, kCfgDecWaves>(a, block, tile_blocks, s);
}

// Pipelined form (16-byte aligned input): persistent workgroups of 8 data
// waves and a control wave, chunks of kCfgPipeChunkSegs segments.
template <int HB, int L>
static hipError_t launch_compress_cfg_pipe_t(const CompressArgs &a, hipStream_t s)
{
    static const unsigned cap = persistent_grid(compress_cfg_pipe_kernel<HB, L>, ~0ull, 9 * 64);
    hipLaunchKernelGGL((compress_cfg_pipe_kernel<HB, L>), dim3((unsigned)(a.nchunks < cap ? a.nchunks : cap)),
                       dim3(9 * 64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_compress_cfg(const CompressArgs &a, int block, int tile_blocks, bool in_aligned16, hipStream_t s)
{
    if (in_aligned16) {
        CompressArgs p = a;
        p.nchunks = a.n ? ceil_div(ceil_div(a.n, (uint64_t)kBlock), (uint64_t)kCfgPipeChunkSegs) : 1;
        switch (block * 100 + tile_blocks) {
        case 3204: return launch_compress_cfg_pipe_t<1, 4>(p, s);
        case 3208: return launch_compress_cfg_pipe_t<1, 8>(p, s);
        case 3216: return launch_compress_cfg_pipe_t<1, 16>(p, s);
        case 6404: return launch_compress_cfg_pipe_t<2, 8>(p, s);
        case 6408: return launch_compress_cfg_pipe_t<2, 16>(p, s);
        case 6416: return launch_compress_cfg_pipe_t<2, 32>(p, s);
        default: return hipErrorInvalidValue;
        }
    }
    return launch_compress_cfg_t<false>(a, block, tile_blocks, s);
}

hipError_t launch_decompress_cfg(const DecompressArgs &a, int block, int tile_blocks, bool out_aligned16,
                                 hipStream_t s)
{
    return out_aligned16 ? launch_decompress_cfg_t<true>(a, block, tile_blocks, s)
                         : launch_decompress_cfg_t<false>(a, block, tile_blocks, s);
}

// Offsets pre-pass (chunks of kCfgDecChunkSegs segments = kCfgDecChunkSegs / L
// tiles), then one chunk per workgroup without lookback.
template <bool ALIGNED, int HB, int L>
static hipError_t launch_decompress_cfg_prescan_t(const DecompressArgs &a, hipStream_t s)
{
    const uint64_t ngroups = a.ntiles ? ceil_div(a.ntiles, (uint64_t)kScanTiles) : 1;
    hipLaunchKernelGGL((dec_offsets_single_kernel<kCfgDecChunkSegs / L, L / HB, HB>), dim3((unsigned)ngroups),
                       dim3(kScanThreads), 0, s, a, const_cast<unsigned long long *>(a.offsets),
                       const_cast<uint32_t *>(a.go), ngroups);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((decompress_cfg_kernel<ALIGNED, HB, L, true>), dim3((unsigned)a.nchunks),
                       dim3(kCfgDecWaves * 64), 0, s, a);
    return hipGetLastError();
}

template <bool ALIGNED>
static hipError_t launch_decompress_cfg_prescan_a(const DecompressArgs &a, int block, int tile_blocks,
                                                  hipStream_t s)
{
    switch (block * 100 + tile_blocks) {
    case 3204: return launch_decompress_cfg_prescan_t<ALIGNED, 1, 4>(a, s);
    case 3208: return launch_decompress_cfg_prescan_t<ALIGNED, 1, 8>(a, s);
    case 3216: return launch_decompress_cfg_prescan_t<ALIGNED, 1, 16>(a, s);
    case 6404: return launch_decompress_cfg_prescan_t<ALIGNED, 2, 8>(a, s);
    case 6408: return launch_decompress_cfg_prescan_t<ALIGNED, 2, 16>(a, s);
    case 6416: return launch_decompress_cfg_prescan_t<ALIGNED, 2, 32>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_decompress_cfg_prescan(const DecompressArgs &a, int block, int tile_blocks, bool out_aligned16,
                                         hipStream_t s)
{
    return out_aligned16 ? launch_decompress_cfg_prescan_a<true>(a, block, tile_blocks, s)
                         : launch_decompress_cfg_prescan_a<false>(a, block, tile_blocks, s);
}

constexpr size_t kLdsPerCu = 160 * 1024;

// Dynamic LDS that caps resident workgroups per CU at `groups` (0 = none);
// returns false when the cap needs more LDS per workgroup than allowed or
// would change nothing.
template <typename K>
static bool batch_lds_pad(K kernel, int groups, size_t *pad)
{
    *pad = 0;
    if (groups <= 0) return true;
    hipFuncAttributes attr{};
    int dev = 0, max_lds = 0;
    if (hipFuncGetAttributes(&attr, reinterpret_cast<const void *>(kernel)) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    const size_t per = kLdsPerCu / (size_t)groups;
    const size_t want = per > attr.sharedSizeBytes ? (per - attr.sharedSizeBytes) / 256 * 256 : 0;
    if (want == 0) return false;  // the kernel's own LDS already allows no more than `groups`
    if (attr.sharedSizeBytes + want > (size_t)max_lds) return false;
    // the pad must make the next workgroup not fit
    if ((size_t)(groups + 1) * (attr.sharedSizeBytes + want) <= kLdsPerCu) return false;
    *pad = want;
    return true;
}

template <int W, bool LDSJOBS>
static hipError_t launch_batch_pipe(const BatchArgs &b, int groups, hipStream_t s)
{
    size_t pad = 0;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_pipe_kernel<W, LDSJOBS>, W * 64, 0) !=
            hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        cus = 256;
        per_cu = 1;
    }
    if (groups > 0 && groups < per_cu) {  // the cap is a hint: dropped where no pad can set it
        if (batch_lds_pad(batch_pipe_kernel<W, LDSJOBS>, groups, &pad))
            per_cu = groups;
        else
            pad = 0;
    }
    const uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
    const unsigned grid = (unsigned)(b.total_chunks < g ? b.total_chunks : g);
    hipLaunchKernelGGL((batch_pipe_kernel<W, LDSJOBS>), dim3(grid), dim3(W * 64), pad, s, b);
    return hipGetLastError();
}

template <bool ALIGNED, int W>
static hipError_t launch_batch_t(const BatchArgs &b, bool any_compress, bool any_decompress, int groups,
                                 hipStream_t s)
{
    size_t pad = 0;
    if (ALIGNED && any_compress && !any_decompress) {
        // compression only, 16-byte aligned inputs: the persistent pipeline,
        // one workgroup per CU at most (its LDS); a cap of 1 needs no pad
        return b.njobs <= kPipeLdsJobs ? launch_batch_pipe<W, true>(b, groups, s)
                                       : launch_batch_pipe<W, false>(b, groups, s);
    }
    if (any_compress) {
        if (!batch_lds_pad(batch_kernel<ALIGNED, W>, groups, &pad)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((batch_kernel<ALIGNED, W>), dim3((unsigned)b.total_chunks), dim3(W * 64), pad, s, b);
        return hipGetLastError();
    }
    // decompression only: persistent, as many workgroups as fit at this shape
    if (!batch_lds_pad(batch_dec_kernel<ALIGNED, W>, groups, &pad)) return hipErrorInvalidValue;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_dec_kernel<ALIGNED, W>, W * 64, pad) !=
            hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        cus = 256;
        per_cu = 1;
    }
    const uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
    const unsigned grid = (unsigned)(b.total_chunks < g ? b.total_chunks : g);
    hipLaunchKernelGGL((batch_dec_kernel<ALIGNED, W>), dim3(grid), dim3(W * 64), pad, s, b);
    return hipGetLastError();
}

bool batch_shape_supported(const BatchShape &shape)
{
    if (shape.groups_per_cu < 0 || shape.groups_per_cu > 8) return false;
    size_t pad = 0;
    switch (shape.waves) {
    case 2: return batch_lds_pad(batch_kernel<true, 2>, shape.groups_per_cu, &pad);
    case 4: return batch_lds_pad(batch_kernel<true, 4>, shape.groups_per_cu, &pad);
    case 8: return batch_lds_pad(batch_kernel<true, 8>, shape.groups_per_cu, &pad);
    default: return false;
    }
}

hipError_t launch_batch(const BatchArgs &b, bool aligned16, bool any_compress, bool any_decompress,
                        const BatchShape &shape, hipStream_t s)
{
    // workgroups loop over segments; enough of them to clear the flags
    uint64_t grid = b.total_segs < 2048 ? b.total_segs : 2048;
    const uint64_t clear = ceil_div(b.nflags, kStatsThreads);
    if (grid < clear) grid = clear < kStatsMaxBlocks ? clear : kStatsMaxBlocks;
    if (grid < 1) grid = 1;
    if (aligned16)
        hipLaunchKernelGGL(batch_stats_kernel<true>, dim3((unsigned)grid), dim3(kStatsThreads), 0, s, b);
    else
        hipLaunchKernelGGL(batch_stats_kernel<false>, dim3((unsigned)grid), dim3(kStatsThreads), 0, s, b);
    if (any_compress)
        hipLaunchKernelGGL(batch_stats_final_kernel, dim3(b.njobs), dim3(kStatsThreads), 0, s, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.total_chunks == 0) return hipSuccess;
    switch (shape.waves) {
    case 2: return aligned16 ? launch_batch_t<true, 2>(b, any_compress, any_decompress, shape.groups_per_cu, s)
                             : launch_batch_t<false, 2>(b, any_compress, any_decompress, shape.groups_per_cu, s);
    case 4: return aligned16 ? launch_batch_t<true, 4>(b, any_compress, any_decompress, shape.groups_per_cu, s)
                             : launch_batch_t<false, 4>(b, any_compress, any_decompress, shape.groups_per_cu, s);
    case 8: return aligned16 ? launch_batch_t<true, 8>(b, any_compress, any_decompress, shape.groups_per_cu, s)
                             : launch_batch_t<false, 8>(b, any_compress, any_decompress, shape.groups_per_cu, s);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ allocation-free compression
//
// fsz_compress_noalloc_async keeps its chunk flags, ticket and range-pass
// partials in one fixed device array instead of the per-stream workspace.
// Layout: [0, 16 KiB) range-pass partials, then the field stats (16 bytes)
// and the ticket (8 bytes, 128 bytes further), then from byte 16640 the flag
// words (kFlagStride words per chunk) of the smallest chunk any compress
// kernel uses (8 tiles, 2048 elements), enough for n <= kNoAllocMaxElements.
// Each call clears the flag words it uses and the ticket with a fill kernel
// (no memset node, so the call may be captured in a graph and replayed).
constexpr uint64_t kNoAllocMaxElements = 1ull << 30;
constexpr size_t kNoAllocStatsOff = sizeof(StatsPartial) * kStatsMaxBlocks;
constexpr size_t kNoAllocTicketOff = kNoAllocStatsOff + 128;
constexpr size_t kNoAllocFlagsOff = kNoAllocStatsOff + 256;
constexpr uint64_t kNoAllocMaxFlags = kNoAllocMaxElements / ((uint64_t)kTile * kTilesPerWave);
constexpr size_t kNoAllocScratchBytes = kNoAllocFlagsOff + kNoAllocMaxFlags * kFlagStride * sizeof(unsigned long long);
static_assert(kNoAllocScratchBytes == 16640 + 32 * 524288, "scratch layout");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).  Host code passes
// this address, never the array's name, to kernels.
static unsigned char *scratch_address(int dev)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        addr[dev] = static_cast<unsigned char *>(ptr);
    }
    return addr[dev];
}

__global__ __launch_bounds__(256) void zero_words_kernel(unsigned long long *p, uint64_t count,
                                                         unsigned long long *one)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) *one = 0;
}

fsz_status compress_noalloc(const float *d_in, uint64_t n, int mode, double value, const fsz_stats *d_stats,
                            void *d_out, uint64_t cap, fsz_result *d_result, hipStream_t s)
{
    if (n > kNoAllocMaxElements) return FSZ_ERR_TOO_LARGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FSZ_ERR_DEVICE;
    unsigned char *base = scratch_address(dev);
    if (!base) return FSZ_ERR_DEVICE;
    StatsPartial *partials = reinterpret_cast<StatsPartial *>(base);
    fsz_stats *stats = reinterpret_cast<fsz_stats *>(base + kNoAllocStatsOff);
    unsigned long long *ticket = reinterpret_cast<unsigned long long *>(base + kNoAllocTicketOff);
    unsigned long long *flags = reinterpret_cast<unsigned long long *>(base + kNoAllocFlagsOff);

    CompressArgs a{};
    a.x = d_in;
    a.n = n;
    a.ntiles = ceil_div(n, kTile);
    a.nblocks = ceil_div(n, kBlock);
    a.nchunks = a.ntiles ? ceil_div(a.ntiles, kTilesPerChunk) : 1;
    a.data0 = kHeaderBytes + pad16(a.nblocks);
    a.out = static_cast<uint8_t *>(d_out);
    a.capacity = cap;
    a.value = value;
    a.mode = mode;
    a.features = kFeaturesAll;
    a.epoch = 1;       // flags start cleared at every call, so one epoch serves
    a.flag_epoch = 1;  // every call
    a.flags = flags;
    a.ticket = ticket;
    a.final = d_result;
    const uint64_t nflags = (a.ntiles ? ceil_div(a.ntiles, kTilesPerWave) : 1) * kFlagStride;  // words
    const uint64_t want = ceil_div(nflags, 256);
    const unsigned grid = (unsigned)(want < 1024 ? want : 1024);
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(256), 0, s, flags, nflags, ticket);
    if (hipGetLastError() != hipSuccess) return FSZ_ERR_DEVICE;
    if (!d_stats) {
        const StatsArgs sa{d_in, n, stats, partials};
        if (launch_stats(sa, s) != hipSuccess) return FSZ_ERR_DEVICE;
        d_stats = stats;
    }
    a.stats = d_stats;
    const bool al16 = (reinterpret_cast<uintptr_t>(d_in) & 15u) == 0;
    if (launch_compress(a, al16, tuning().staged_compress, s) != hipSuccess) return FSZ_ERR_DEVICE;
    return FSZ_OK;
}

}  // namespace fsz
