/*
 * FSZ oracle -- plain, serial, obviously-correct CPU implementation of the
 * FSZ compressor and decompressor (stream format v1, block B = 32 elements,
 * tile = T = 8 blocks = 256 elements).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the HIP library.
 *
 * Build with -O2 -ffp-contract=off and without fast-math: every floating
 * point operation below is a single IEEE-754 binary32 (or binary64 where
 * stated) operation in the written order.
 *
 * Paper references (FSZ, "Breaking the Prediction-Throughput Trade-off in
 * GPU Lossy Compression"):
 *   Sec. III-A   tile = 8 blocks x 32 elements; compressed format (rate
 *                header byte per block, block-0 bit 7 = LZ order, bit 6 =
 *                centering, bits 4-0 = rate; 4-byte sign map + 4*rate bytes
 *                per block; zero-rate blocks store nothing; inline tile mean)
 *   Sec. IV-A    cross-block prediction state, Eq. (1)-(2)
 *   Sec. IV-B    four variants LZ1/LZ2 x centering, quantizer
 *                q = round(d / (2 eb)), rate r = ceil(log2(max|l| + 1)),
 *                block cost Eq. (3), cancellation property Eq. (4)
 *   Sec. IV-C    fixed-length encoding, sign map, bit-shuffle (element i's
 *                bit at position 31 - i of a 4-byte word)
 *   Sec. IV-D    exclusive prefix sum of compressed sizes
 *   Sec. V-A     REL bound: eb = REL * (max - min); pointwise |d - d'| <= eb
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - quantizer: multiply by inv = fl32(1/E) then round-half-even; the step
 *     E is the largest binary32 not above 2 (eb - 4 ulp(max|x|)), computed
 *     exactly, so that the pointwise bound holds in binary32 arithmetic;
 *     bounds below 8 ulp(max|x|) are rejected;
 *   - four-way evaluation: each variant's residuals are formed in full and
 *     rated block by block (the plain definition; the one-read shortcut that
 *     Eq. (4) licenses is what the GPU kernels do, and the tests check the
 *     two agree);
 *   - zero predictor state at each tile start: q[-1] = q[-2] = 0;
 *   - tile mean: index-order pairwise binary32 sum of the 256 slots (missing
 *     slots of a ragged last tile count as +0), times 2^-8, quantized like
 *     any element; centering is disabled if that value is not finite;
 *   - selection ties: strict '<' in the order LZ1, LZ2, LZ1c, LZ2c;
 *   - centered tile: the mean is stored as a little-endian int32 in the first
 *     4 bytes of the tile's data;
 *   - sign bit 1 = negative; sign word first, then planes 0..r-1; each
 *     32-bit word is written most-significant byte first;
 *   - a 32-byte stream header precedes the rate bytes, which are zero-padded
 *     to a multiple of 16 bytes.
 *
 * Feature switches (the ablation of Sec. VI-B, Table IV; the base is the
 * cuSZp-equivalent compressor: LZ1 only, independent blocks, no centering):
 *   - cross-block state off: the zero predictor state is restored at every
 *     block start instead of only at the tile start (header flags bit 1, so
 *     the decoder restarts its running sums there too);
 *   - centering off / second order off: those variants are never selected.
 * Centering with independent blocks subtracts the tile mean from every
 * value, which changes the first residual of every block (and the second
 * one under LZ2).
 *
 * Tile configurations (Sec. VI-C, Table V): the block size B (32 or 64
 * elements) and the blocks per tile T (4, 8 or 16) are stream parameters,
 * recorded in header flags bits 2-4 (bit 2: B = 64; bits 3-4: 0 for T = 8,
 * 1 for T = 4, 2 for T = 16), so the default B = 32, T = 8 keeps those bits
 * zero.  A block of 64 elements encodes each bit plane (and the sign map) as
 * one 64-bit word, element i at bit 63 - i, written most-significant byte
 * first; its cost is 8 + 8r bytes for rate r > 0.  The tile mean is the
 * pairwise sum of the B*T slots times 1/(B*T), and the prediction state
 * restarts at every tile start as before.
 */
#include "fsz_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAX_BLOCK 64
#define MAX_BLOCKS_PER_TILE 16
#define MAX_TILE (MAX_BLOCK * MAX_BLOCKS_PER_TILE)
#define HEADER_BYTES 32

/* the default tile configuration */
#define BLOCK 32
#define BLOCKS_PER_TILE 8

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static uint64_t pad16(uint64_t a) { return (a + 15) / 16 * 16; }

/* rate r = ceil(log2(v + 1)) = number of significant bits of v (Sec. IV-A) */
static uint32_t rate_of(uint32_t v)
{
    uint32_t r = 0;
    while (v != 0) {
        r++;
        v >>= 1;
    }
    return r;
}

/* block cost, Eq. (3): nothing for a zero-rate block, else sign map + r
 * planes of B bits each */
static uint32_t block_cost(uint32_t r, int B) { return r == 0 ? 0 : (uint32_t)(B / 8) * (1 + r); }

/* whether (B, T) is a supported tile configuration */
static int config_ok(int B, int T) { return (B == 32 || B == 64) && (T == 4 || T == 8 || T == 16); }

/* header flags bits 2-4 of a configuration, and back (-1: reserved code) */
static uint32_t config_flags(int B, int T) { return (B == 64 ? 4u : 0u) | (T == 4 ? 8u : T == 16 ? 16u : 0u); }
static int config_from_flags(uint32_t flags, int *B, int *T)
{
    uint32_t tc = (flags >> 3) & 3u;
    if (tc == 3) return -1;
    *B = (flags & 4u) ? 64 : 32;
    *T = tc == 0 ? 8 : tc == 1 ? 4 : 16;
    return 0;
}

static uint32_t magnitude(int32_t v) { return v < 0 ? (uint32_t)0 - (uint32_t)v : (uint32_t)v; }

static void put_u16(uint8_t *p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t *p, uint32_t v)
{
    for (int k = 0; k < 4; k++) p[k] = (uint8_t)(v >> (8 * k));
}
static void put_u64(uint8_t *p, uint64_t v)
{
    for (int k = 0; k < 8; k++) p[k] = (uint8_t)(v >> (8 * k));
}
static uint32_t get_u32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint64_t get_u64(const uint8_t *p)
{
    uint64_t v = 0;
    for (int k = 7; k >= 0; k--) v = (v << 8) | p[k];
    return v;
}
/* bit-shuffled words of B = 32 or 64 bits are stored most-significant byte first */
static void put_bits_msb_first(uint8_t *p, uint64_t w, int B)
{
    for (int k = 0; k < B / 8; k++) p[k] = (uint8_t)(w >> (B - 8 - 8 * k));
}
static uint64_t get_bits_msb_first(const uint8_t *p, int B)
{
    uint64_t w = 0;
    for (int k = 0; k < B / 8; k++) w = (w << 8) | p[k];
    return w;
}
static float bits_to_float(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}
static uint32_t float_to_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

uint64_t fszo_bound_config(uint64_t n, int B, int T)
{
    if (!config_ok(B, T)) return 0;
    uint64_t nblocks = ceil_div(n, (uint64_t)B);
    uint64_t ntiles = ceil_div(n, (uint64_t)B * T);
    return HEADER_BYTES + pad16(nblocks) + 4 * ntiles + block_cost(31, B) * nblocks;
}

uint64_t fszo_bound(uint64_t n) { return fszo_bound_config(n, BLOCK, BLOCKS_PER_TILE); }

/* ------------------------------------------------------------------ */
/* error-bound resolution (Sec. V-A and the binary32 reading above)    */
/* ------------------------------------------------------------------ */

/* spacing of binary32 numbers at magnitude m (m finite, >= 0) */
static double ulp32(float m)
{
    if (m < FLT_MIN) return ldexp(1.0, -149);
    int e;
    frexpf(m, &e); /* m = f * 2^e, 0.5 <= f < 1 */
    return ldexp(1.0, e - 24);
}

/* binary32 value of d (> 0) rounded toward zero */
static float to_f32_toward_zero(double d)
{
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, 0.0f);
    return f;
}

/* a - b (a > b > 0) rounded toward zero in binary64.  The round-to-nearest
 * difference s carries an exact error term e (Knuth's two-sum: a - b = s + e
 * exactly); when e < 0 the rounding went up, so step s one unit down.  Taken
 * toward zero again into binary32, the result is then the binary32 value of
 * the exact difference rounded toward zero (the binary32 numbers are binary64
 * numbers, so the two truncations compose). */
static double sub_toward_zero(double a, double b)
{
    double s = a - b;
    double bb = s - a;
    double e = (a - (s - bb)) + (-b - bb);
    if (e < 0.0) s = nextafter(s, 0.0);
    return s;
}

int fszo_resolve(const float *x, uint64_t n, int mode, double value,
                 float *E_out, float *inv_out, uint32_t *flags_out)
{
    if (mode != 0 && mode != 1) return FSZO_ERR_INVALID_ARG;
    if (!isfinite(value) || !(value > 0.0)) return FSZO_ERR_INVALID_ARG;

    float xmin = INFINITY, xmax = -INFINITY, M = 0.0f;
    for (uint64_t i = 0; i < n; i++) {
        float v = x[i];
        if (!isfinite(v)) return FSZO_ERR_NONFINITE;
        if (v < xmin) xmin = v;
        if (v > xmax) xmax = v;
        if (fabsf(v) > M) M = fabsf(v);
    }

    float E;
    uint32_t flags = 0;
    if (n == 0) {
        E = 1.0f;
    } else if (mode == 1 && xmax == xmin) {
        /* zero value range: the field is one constant c, reproduced exactly
         * with step |c| (q in {-1, 0, 1}) */
        float c = fabsf(xmin);
        if (c == 0.0f) E = 1.0f;
        else if (c < FLT_MIN) return FSZO_ERR_EB_TOO_SMALL;
        else E = c;
        flags = 1;
    } else {
        double eb = mode == 1 ? value * ((double)xmax - (double)xmin) : value;
        double u = ulp32(M);
        if (!(eb >= 8.0 * u)) return FSZO_ERR_EB_TOO_SMALL;
        /* E = the largest binary32 <= 2 (eb - 4u), computed exactly */
        double eb_q = sub_toward_zero(eb, 4.0 * u);
        E = to_f32_toward_zero(2.0 * eb_q);
        if (E > 0x1p126f) E = 0x1p126f;
        if (E < FLT_MIN) return FSZO_ERR_EB_TOO_SMALL;
        if ((double)M + (double)E > (double)FLT_MAX) return FSZO_ERR_EB_TOO_LARGE;
    }
    *E_out = E;
    *inv_out = 1.0f / E;
    *flags_out = flags;
    return FSZO_OK;
}

/* ------------------------------------------------------------------ */
/* per-tile analysis: single pass + four-way evaluation (Sec. IV-B)    */
/* ------------------------------------------------------------------ */

typedef struct {
    int B, T;                       /* block size, blocks per tile */
    int indep;                      /* prediction restarts at every block */
    int m;                          /* valid elements in the tile */
    int nb;                         /* blocks in the tile */
    int32_t q[MAX_TILE];            /* quantized values */
    int32_t res[4][MAX_TILE];       /* residuals of LZ1, LZ2, LZ1c, LZ2c */
    int32_t mu;                     /* quantized tile mean */
    int centre_ok;                  /* mean finite -> centered variants allowed */
    uint32_t cost[4];               /* C of LZ1, LZ2, LZ1c, LZ2c */
    uint32_t vrate[4][MAX_BLOCKS_PER_TILE]; /* per-block rates of each variant */
    int order2, centred;            /* selected variant */
    uint32_t rate[MAX_BLOCKS_PER_TILE]; /* selected per-block rates */
    uint32_t bytes;                 /* selected tile cost C */
} tile_t;

/* whether a variant may be selected under the feature switches */
static int variant_allowed(int v, uint32_t features, int centre_ok)
{
    if ((v & 1) && !(features & FSZO_FEAT_LZ2)) return 0;
    if ((v >> 1) && (!(features & FSZO_FEAT_CENTERING) || !centre_ok)) return 0;
    return 1;
}

/* Prequantization (Sec. IV-B item 1): q = round(x / (2 eb)), here one
 * binary32 multiply by inv = fl32(1/E) and round-half-even.  Missing slots
 * of a ragged last tile are 0. */
static void quantize_tile(const float *x, int m, int tile, float inv, int32_t *q)
{
    for (int i = 0; i < tile; i++) q[i] = i < m ? (int32_t)rintf(x[i] * inv) : 0;
}

/* Residuals of one variant (Sec. IV-A Eq. (1)-(2), Sec. IV-B): the
 * predicted sequence is p = q - c (c = the tile mean for a centered
 * variant, else 0); the residual is its first (LZ1) or second (LZ2)
 * difference, with zero prediction state before the tile start (before
 * every block start when blocks are independent).  Missing slots of a
 * ragged last tile carry residual 0. */
static void variant_residuals(const int32_t *q, int m, int B, int tile, int indep, int order2, int32_t c,
                              int32_t *res)
{
    int32_t pm1 = 0, pm2 = 0;
    for (int i = 0; i < tile; i++) {
        if (indep && i % B == 0) pm1 = pm2 = 0;
        if (i >= m) {
            res[i] = 0;
            continue;
        }
        int32_t p = q[i] - c;
        res[i] = order2 ? p - 2 * pm1 + pm2 : p - pm1;
        pm2 = pm1;
        pm1 = p;
    }
}

/* Tile mean (Sec. IV-B item 3): index-order pairwise binary32 sum of the
 * B*T slots (missing slots of a ragged last tile count as +0), divided by
 * B*T (a power of two, so the division is exact), then quantized like any
 * element.  Returns 0 when that value is not finite (centering disabled). */
static int tile_mean(const float *x, int m, int tile, float inv, int32_t *mu)
{
    float s[MAX_TILE];
    for (int i = 0; i < tile; i++) s[i] = i < m ? x[i] : 0.0f;
    for (int w = 1; w < tile; w *= 2)
        for (int i = 0; i < tile; i += 2 * w) s[i] = s[i] + s[i + w];
    float mean_q = (s[0] * (1.0f / (float)tile)) * inv;
    if (!isfinite(mean_q)) {
        *mu = 0;
        return 0;
    }
    *mu = (int32_t)rintf(mean_q);
    return 1;
}

/* Four-way evaluation and selection of one tile (Sec. IV-B, Eq. (3)): each
 * variant's residuals are formed in full, each block's rate is the bit
 * length of its largest residual magnitude, the cost C sums the block costs
 * plus 4 bytes for a stored mean; the minimum wins. */
static void analyse_tile(const float *x, int m, float inv, uint32_t features, int B, int T, tile_t *t)
{
    const int TILE = B * T;
    t->B = B;
    t->T = T;
    t->indep = (features & FSZO_FEAT_CROSS_BLOCK) ? 0 : 1;
    t->m = m;
    t->nb = (m + B - 1) / B;

    quantize_tile(x, m, TILE, inv, t->q);
    t->centre_ok = tile_mean(x, m, TILE, inv, &t->mu);

    for (int v = 0; v < 4; v++) {
        int ord2 = v & 1, cen = v >> 1;
        variant_residuals(t->q, m, B, TILE, t->indep, ord2, cen ? t->mu : 0, t->res[v]);
        t->cost[v] = cen ? 4 : 0;
        for (int b = 0; b < T; b++) {
            uint32_t a = 0;
            if (b < t->nb)
                for (int i = b * B; i < b * B + B; i++) {
                    uint32_t mg = magnitude(t->res[v][i]);
                    if (mg > a) a = mg;
                }
            t->vrate[v][b] = rate_of(a);
            t->cost[v] += block_cost(t->vrate[v][b], B);
        }
    }

    /* Adaptive select: minimum C; ties keep the earlier of LZ1, LZ2, LZ1c,
     * LZ2c; centered variants only with a finite mean; variants switched
     * off are never selected (LZ1 always may be). */
    int best = 0;
    for (int v = 1; v < 4; v++)
        if (variant_allowed(v, features, t->centre_ok) && t->cost[v] < t->cost[best]) best = v;
    t->order2 = best & 1;
    t->centred = best >> 1;
    t->bytes = t->cost[best];
    for (int b = 0; b < T; b++) t->rate[b] = t->vrate[best][b];
}

int fszo_tile_eval_config(const float *x, int m, float inv, uint32_t features, int B, int T, int32_t *mu,
                          int *centre_ok, uint32_t *cost4, uint32_t *rates, int *best)
{
    if (!config_ok(B, T) || m < 1 || m > B * T || (features & ~(uint32_t)FSZO_FEATURES_ALL))
        return FSZO_ERR_INVALID_ARG;
    tile_t *t = (tile_t *)malloc(sizeof(tile_t));
    if (!t) return FSZO_ERR_INVALID_ARG;
    analyse_tile(x, m, inv, features, B, T, t);
    *best = t->order2 | (t->centred << 1);
    *mu = t->mu;
    *centre_ok = t->centre_ok;
    for (int v = 0; v < 4; v++) {
        cost4[v] = t->cost[v];
        for (int b = 0; b < T; b++) rates[v * T + b] = t->vrate[v][b];
    }
    free(t);
    return FSZO_OK;
}

int fszo_tile_eval_features(const float *x, int m, float inv, uint32_t features, int32_t *mu,
                            int *centre_ok, uint32_t *cost4, uint32_t *rates4x8, int *best)
{
    return fszo_tile_eval_config(x, m, inv, features, BLOCK, BLOCKS_PER_TILE, mu, centre_ok, cost4, rates4x8,
                                 best);
}

int fszo_tile_eval(const float *x, int m, float inv, int32_t *mu, int *centre_ok,
                   uint32_t *cost4, uint32_t *rates4x8)
{
    int best;
    return fszo_tile_eval_features(x, m, inv, FSZO_FEATURES_ALL, mu, centre_ok, cost4, rates4x8, &best);
}

/* Fixed-length encoding + bit-shuffle of one block of B residuals at rate r
 * (Sec. IV-C): the sign map, then planes 0..r-1, each one B-bit word with
 * element j at bit B - 1 - j. */
static uint8_t *encode_block(const int32_t *res, uint32_t r, int B, uint8_t *p)
{
    if (r == 0) return p;
    uint32_t mag[MAX_BLOCK];
    uint64_t sign = 0;
    for (int j = 0; j < B; j++) {
        mag[j] = magnitude(res[j]);
        if (res[j] < 0) sign |= 1ull << (B - 1 - j);
    }
    put_bits_msb_first(p, sign, B);
    p += B / 8;
    for (uint32_t plane = 0; plane < r; plane++) {
        uint64_t w = 0;
        for (int j = 0; j < B; j++) w |= (uint64_t)((mag[j] >> plane) & 1u) << (B - 1 - j);
        put_bits_msb_first(p, w, B);
        p += B / 8;
    }
    return p;
}

/* Host threads for the tile loops (the CPU baseline's parallel mode).
 * Tiles are independent, so pass 1 (analysis) and pass 3 (encode) run over
 * tiles in parallel; the prefix sum between them stays serial.  The bytes
 * do not depend on the thread count. */
static int g_threads = 1;

int fszo_set_threads(int n)
{
    int old = g_threads;
    if (n >= 1) g_threads = n;
    return old;
}

int fszo_compress_config(const float *x, uint64_t n, int mode, double value, uint32_t features, int B, int T,
                         uint8_t *out, uint64_t cap, uint64_t *out_size)
{
    if ((features & ~(uint32_t)FSZO_FEATURES_ALL) || !config_ok(B, T)) return FSZO_ERR_INVALID_ARG;
    float E, inv;
    uint32_t flags;
    int st = fszo_resolve(x, n, mode, value, &E, &inv, &flags);
    if (st != FSZO_OK) return st;

    const uint64_t TILE = (uint64_t)B * T;
    const int indep = (features & FSZO_FEAT_CROSS_BLOCK) ? 0 : 1;
    uint64_t nblocks = ceil_div(n, (uint64_t)B);
    uint64_t ntiles = ceil_div(n, TILE);
    uint64_t data0 = HEADER_BYTES + pad16(nblocks);

    uint8_t *rates = (uint8_t *)malloc(nblocks ? nblocks : 1);
    uint64_t *offset = (uint64_t *)malloc(sizeof(uint64_t) * (ntiles + 1));
    int32_t *mus = (int32_t *)malloc(sizeof(int32_t) * (ntiles ? ntiles : 1));
    if (!rates || !offset || !mus) {
        free(rates);
        free(offset);
        free(mus);
        return FSZO_ERR_INVALID_ARG;
    }
    int failed = 0;

    /* Pass 1: per-tile analysis -> rate bytes, tile sizes, tile means. */
#pragma omp parallel num_threads(g_threads)
    {
        tile_t *tl = (tile_t *)malloc(sizeof(tile_t));
        if (!tl) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (uint64_t t = 0; t < ntiles; t++) {
            if (!tl) continue;
            uint64_t start = t * TILE;
            int m = (int)(n - start < TILE ? n - start : TILE);
            analyse_tile(x + start, m, inv, features, B, T, tl);
            for (int b = 0; b < tl->nb; b++) {
                uint8_t byte = (uint8_t)tl->rate[b];
                if (b == 0) byte |= (uint8_t)((tl->order2 << 7) | (tl->centred << 6)); /* Sec. III-A */
                rates[t * (uint64_t)T + b] = byte;
            }
            offset[t + 1] = tl->bytes;
            mus[t] = tl->mu;
        }
        free(tl);
    }
    if (failed) {
        free(rates);
        free(offset);
        free(mus);
        return FSZO_ERR_INVALID_ARG;
    }

    /* Pass 2: exclusive prefix sum of tile sizes (Sec. IV-D). */
    offset[0] = 0;
    for (uint64_t t = 0; t < ntiles; t++) offset[t + 1] += offset[t];
    uint64_t total = data0 + offset[ntiles];
    if (total > cap) {
        free(rates);
        free(offset);
        free(mus);
        return FSZO_ERR_CAPACITY;
    }

    /* Header (32 bytes), then the rate header: one byte per block. */
    memset(out, 0, data0);
    out[0] = 'F';
    out[1] = 'S';
    out[2] = 'Z';
    out[3] = '1';
    put_u16(out + 4, 1);
    out[6] = (uint8_t)mode;
    out[7] = (uint8_t)(flags | (indep ? 2u : 0u) | config_flags(B, T));
    put_u64(out + 8, n);
    put_u32(out + 16, float_to_bits(E));
    put_u32(out + 20, float_to_bits((float)value));
    put_u64(out + 24, total);
    memcpy(out + HEADER_BYTES, rates, nblocks);

    /* Pass 3: encode every tile at its offset with the variant recorded in
     * its rate bytes: the residuals of that variant are formed again from
     * the input (the paper's encoder re-reads its input too). */
#pragma omp parallel num_threads(g_threads)
    {
        int32_t q[MAX_TILE], res[MAX_TILE];
#pragma omp for schedule(static)
        for (uint64_t t = 0; t < ntiles; t++) {
            uint64_t start = t * TILE;
            int m = (int)(n - start < TILE ? n - start : TILE);
            int nb = (m + B - 1) / B;
            const uint8_t *rb = rates + t * (uint64_t)T;
            int order2 = (rb[0] >> 7) & 1, centred = (rb[0] >> 6) & 1;
            quantize_tile(x + start, m, (int)TILE, inv, q);
            variant_residuals(q, m, B, (int)TILE, indep, order2, centred ? mus[t] : 0, res);
            uint8_t *p = out + data0 + offset[t];
            if (centred) {
                put_u32(p, (uint32_t)mus[t]);
                p += 4;
            }
            for (int b = 0; b < nb; b++) p = encode_block(res + b * B, rb[b] & 0x1Fu, B, p);
        }
    }

    free(rates);
    free(offset);
    free(mus);
    *out_size = total;
    return FSZO_OK;
}

int fszo_compress_features(const float *x, uint64_t n, int mode, double value, uint32_t features,
                           uint8_t *out, uint64_t cap, uint64_t *out_size)
{
    return fszo_compress_config(x, n, mode, value, features, BLOCK, BLOCKS_PER_TILE, out, cap, out_size);
}

int fszo_compress(const float *x, uint64_t n, int mode, double value,
                  uint8_t *out, uint64_t cap, uint64_t *out_size)
{
    return fszo_compress_features(x, n, mode, value, FSZO_FEATURES_ALL, out, cap, out_size);
}

/* ------------------------------------------------------------------ */
/* decompression (Sec. III-A, decompression steps 1-5)                 */
/* ------------------------------------------------------------------ */

int fszo_decompress(const uint8_t *cmp, uint64_t cmp_size, float *out, uint64_t n)
{
    if (cmp_size < HEADER_BYTES) return FSZO_ERR_CORRUPT;
    if (cmp[0] != 'F' || cmp[1] != 'S' || cmp[2] != 'Z' || cmp[3] != '1') return FSZO_ERR_CORRUPT;
    if ((cmp[4] | (cmp[5] << 8)) != 1) return FSZO_ERR_CORRUPT;
    if (cmp[6] > 1 || (cmp[7] & ~0x1Fu) != 0) return FSZO_ERR_CORRUPT;
    int indep = (cmp[7] >> 1) & 1; /* independent blocks: sums restart per block */
    int B, T;
    if (config_from_flags(cmp[7], &B, &T) != 0) return FSZO_ERR_CORRUPT;
    const uint64_t TILE = (uint64_t)B * T;
    uint64_t hn = get_u64(cmp + 8);
    if (hn != n) return FSZO_ERR_SIZE_MISMATCH;
    float E = bits_to_float(get_u32(cmp + 16));
    if (!isfinite(E) || !(E > 0.0f)) return FSZO_ERR_CORRUPT;
    uint64_t total = get_u64(cmp + 24);

    uint64_t nblocks = ceil_div(n, (uint64_t)B);
    uint64_t ntiles = ceil_div(n, TILE);
    uint64_t data0 = HEADER_BYTES + pad16(nblocks);
    if (total > cmp_size || total < data0) return FSZO_ERR_CORRUPT;
    const uint8_t *rates = cmp + HEADER_BYTES;
    for (uint64_t k = nblocks; k < pad16(nblocks); k++)
        if (rates[k] != 0) return FSZO_ERR_CORRUPT;

    /* 1-3: rates and tile metadata -> block sizes -> exclusive prefix sum */
    uint64_t *offset = (uint64_t *)malloc(sizeof(uint64_t) * (ntiles + 1));
    if (!offset) return FSZO_ERR_INVALID_ARG;
    offset[0] = 0;
    for (uint64_t t = 0; t < ntiles; t++) {
        uint64_t nb = nblocks - t * T;
        if (nb > (uint64_t)T) nb = T;
        uint64_t bytes = 0;
        for (uint64_t b = 0; b < nb; b++) {
            uint8_t byte = rates[t * T + b];
            if (b == 0 ? (byte & 0x20) != 0 : (byte & 0xE0) != 0) {
                free(offset);
                return FSZO_ERR_CORRUPT;
            }
            bytes += block_cost(byte & 0x1F, B);
            if (b == 0 && (byte & 0x40)) bytes += 4;
        }
        offset[t + 1] = offset[t] + bytes;
    }
    if (data0 + offset[ntiles] != total) {
        free(offset);
        return FSZO_ERR_CORRUPT;
    }

    /* 4-5: decode + bit-unshuffle, inverse prediction, dequantize (tiles
     * are independent once their offsets are known) */
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (uint64_t t = 0; t < ntiles; t++) {
        uint64_t start = t * TILE;
        int m = (int)(n - start < TILE ? n - start : TILE);
        int nb = (m + B - 1) / B;
        uint8_t head = rates[t * T];
        int order2 = (head >> 7) & 1, centred = (head >> 6) & 1;
        const uint8_t *p = cmp + data0 + offset[t];
        int32_t mu = 0;
        if (centred) {
            mu = (int32_t)get_u32(p);
            p += 4;
        }
        uint32_t e[MAX_TILE];
        for (int b = 0; b < nb; b++) {
            uint32_t r = rates[t * T + b] & 0x1F;
            for (int j = 0; j < B; j++) e[b * B + j] = 0;
            if (r == 0) continue;
            uint64_t sign = get_bits_msb_first(p, B);
            p += B / 8;
            for (uint32_t plane = 0; plane < r; plane++) {
                uint64_t w = get_bits_msb_first(p, B);
                p += B / 8;
                for (int j = 0; j < B; j++) e[b * B + j] |= (uint32_t)((w >> (B - 1 - j)) & 1u) << plane;
            }
            for (int j = 0; j < B; j++)
                if ((sign >> (B - 1 - j)) & 1u) e[b * B + j] = (uint32_t)0 - e[b * B + j];
        }
        /* inverse Lorenzo: one running sum for LZ1, two for LZ2 (wrapping
         * 32-bit arithmetic, so corrupt streams cannot overflow) */
        uint32_t acc1 = 0, acc2 = 0;
        for (int i = 0; i < m; i++) {
            if (indep && i % B == 0) acc1 = acc2 = 0;
            acc1 += e[i];
            uint32_t qhat;
            if (order2) {
                acc2 += acc1;
                qhat = acc2;
            } else {
                qhat = acc1;
            }
            int32_t q = (int32_t)(qhat + (uint32_t)mu);
            out[start + i] = (float)q * E;
        }
    }
    free(offset);
    return FSZO_OK;
}
