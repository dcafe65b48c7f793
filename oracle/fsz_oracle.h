/*
 * FSZ oracle: a plain, serial CPU implementation of the FSZ stream format.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) shares no code, header, table or helper with it.
 *
 * Status values mirror the public library's numbering so that tests can
 * compare them, but are declared here independently.
 */
#ifndef FSZ_ORACLE_H
#define FSZ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FSZO_OK = 0,
    FSZO_ERR_INVALID_ARG = 1,
    FSZO_ERR_NONFINITE = 2,
    FSZO_ERR_EB_TOO_SMALL = 3,
    FSZO_ERR_CAPACITY = 4,
    FSZO_ERR_CORRUPT = 5,
    FSZO_ERR_SIZE_MISMATCH = 6,
    FSZO_ERR_EB_TOO_LARGE = 8
};

/* Feature switches of the ablation (Sec. VI-B): cross-block prediction
 * state, adaptive centering, second-order Lorenzo.  0 = the cuSZp-equivalent
 * base (LZ1 on independent blocks), all three = the full method. */
enum {
    FSZO_FEAT_CROSS_BLOCK = 1,
    FSZO_FEAT_CENTERING = 2,
    FSZO_FEAT_LZ2 = 4,
    FSZO_FEATURES_ALL = 7
};

/* Worst-case stream size for n floats. */
uint64_t fszo_bound(uint64_t n);

/* Error-bound resolution (absolute bound from ABS/REL, quantizer step E and
 * its reciprocal).  flags bit 0 = constant-field special case. */
int fszo_resolve(const float *x, uint64_t n, int mode, double value,
                 float *E, float *inv, uint32_t *flags);

/* Full compression.  Writes at most cap bytes to out. */
int fszo_compress(const float *x, uint64_t n, int mode, double value,
                  uint8_t *out, uint64_t cap, uint64_t *out_size);

/* Compression with a subset of the features (header flags bit 1 marks
 * independent blocks). */
int fszo_compress_features(const float *x, uint64_t n, int mode, double value, uint32_t features,
                           uint8_t *out, uint64_t cap, uint64_t *out_size);

/* Four-way evaluation of one tile of m (1..256) floats with reciprocal step
 * inv: quantized mean, whether centering is allowed, the cost C of LZ1, LZ2,
 * LZ1c, LZ2c and their per-block rates (4 x 8, row per variant). */
int fszo_tile_eval(const float *x, int m, float inv, int32_t *mu, int *centre_ok,
                   uint32_t *cost4, uint32_t *rates4x8);

/* The same evaluation under a feature subset; *best = the selected variant
 * (order2 | centred << 1).  cost4/rates4x8 cover all four variants. */
int fszo_tile_eval_features(const float *x, int m, float inv, uint32_t features, int32_t *mu,
                            int *centre_ok, uint32_t *cost4, uint32_t *rates4x8, int *best);

/* Tile configurations (Sec. VI-C, Table V): block size B in {32, 64}
 * elements, T in {4, 8, 16} blocks per tile; B = 32, T = 8 is the default
 * and the only one the calls above produce.  The stream records B and T in
 * header flags bits 2-4.  Invalid (B, T): FSZO_ERR_INVALID_ARG (bound: 0). */
uint64_t fszo_bound_config(uint64_t n, int B, int T);
int fszo_compress_config(const float *x, uint64_t n, int mode, double value, uint32_t features, int B, int T,
                         uint8_t *out, uint64_t cap, uint64_t *out_size);
/* Four-way evaluation of one tile of m (1..B*T) floats; rates holds 4 x T
 * per-block rates (row per variant). */
int fszo_tile_eval_config(const float *x, int m, float inv, uint32_t features, int B, int T, int32_t *mu,
                          int *centre_ok, uint32_t *cost4, uint32_t *rates, int *best);

/* Host threads for the tile loops of compression and decompression
 * (default 1).  The bytes written do not depend on it.  Returns the previous
 * value; n < 1 leaves it unchanged. */
int fszo_set_threads(int n);

/* Full decompression of a stream of cmp_size bytes into n floats (any tile
 * configuration, read from the header). */
int fszo_decompress(const uint8_t *cmp, uint64_t cmp_size, float *out, uint64_t n);

#ifdef __cplusplus
}
#endif
#endif
