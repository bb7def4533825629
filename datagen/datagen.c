/*
 * Seeded synthetic inputs: 100-byte records with a 10-byte key (bytes 0..9)
 * and a 90-byte payload (bytes 10..99), the record format of the paper's
 * evaluation workloads (Section 4.1).  These generators stand in for the
 * sortbenchmark.org record tool, which is not used or reproduced here.
 *
 * This module holds no sorting arithmetic.  It is shared, as the only common
 * code, by the CPU oracle side and the GPU side of the test suite.
 *
 * Random words come from a counter-based generator: the splitmix64 output
 * function (Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) evaluated at stream position (16*i + k) of a
 * stream keyed by the seed.  Word k of record i is therefore a pure function
 * of (seed, i, k), so generation is independent of thread count and any
 * record range can be produced on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Stream key of a seed: the first splitmix64 output of that seed. */
static inline uint64_t seed_key(uint64_t seed) { return sm64_out(seed + GOLDEN); }

/* Word k (0..15) of record i in the stream keyed by `key`. */
static inline uint64_t word_at(uint64_t key, uint64_t i, uint64_t k) {
    return sm64_out(key + (i * 16u + k + 1u) * GOLDEN);
}

static inline double unit53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

uint64_t dg_word(uint64_t seed, uint64_t i, uint64_t k) { return word_at(seed_key(seed), i, k); }

/* Uniform records: all 100 bytes are the little-endian bytes of words 0..12. */
static void fill_uniform_one(uint8_t *dst, uint64_t key, uint64_t i) {
    uint64_t w[13];
    for (int k = 0; k < 13; k++) w[k] = word_at(key, i, (uint64_t)k);
    memcpy(dst, w, 100);
}

void dg_records_uniform(uint8_t *out, uint64_t count, uint64_t seed, uint64_t first) {
    const uint64_t key = seed_key(seed);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)count; j++) fill_uniform_one(out + (uint64_t)j * 100u, key, first + (uint64_t)j);
}

/* Records whose payload bytes 10..17 hold the record's own global index
 * (little-endian u64); the key and the remaining payload are as in the
 * uniform generator.  Lets a test read the permutation off the output. */
void dg_records_indexed(uint8_t *out, uint64_t count, uint64_t seed, uint64_t first) {
    const uint64_t key = seed_key(seed);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)count; j++) {
        uint8_t *dst = out + (uint64_t)j * 100u;
        uint64_t gi = first + (uint64_t)j;
        fill_uniform_one(dst, key, gi);
        memcpy(dst + 10, &gi, 8);
    }
}

/* ---- skewed keys: Zipf(s) prefix over `nvals` values + duplicates ---------- */

/* murmur3 fmix32: an invertible map on 32-bit words, so distinct ranks give
 * distinct, scattered 4-byte prefixes. */
static inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85EBCA6BU;
    h ^= h >> 13; h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

typedef struct {
    double *cdf;      /* cdf[r-1] = P(rank <= r), r = 1..nvals */
    uint32_t nvals;
} zipf_table;

static int zipf_build(zipf_table *t, uint32_t nvals, double s) {
    t->nvals = nvals;
    t->cdf = (double *)malloc(sizeof(double) * nvals);
    if (!t->cdf) return -1;
    double acc = 0.0;
    for (uint32_t r = 1; r <= nvals; r++) { acc += pow((double)r, -s); t->cdf[r - 1] = acc; }
    for (uint32_t r = 0; r < nvals; r++) t->cdf[r] /= acc;
    t->cdf[nvals - 1] = 1.0;
    return 0;
}

/* Smallest rank r with u < cdf[r-1]. */
static inline uint32_t zipf_rank(const zipf_table *t, double u) {
    uint32_t lo = 0, hi = t->nvals - 1;
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (u < t->cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo + 1;
}

/* Key of record j before duplication: bytes 0..3 = big-endian fmix32(rank ^ seed),
 * bytes 4..9 = six uniform bytes. */
static inline void base_key(uint8_t *k10, const zipf_table *t, uint64_t key, uint32_t s32, uint64_t j) {
    uint32_t r = zipf_rank(t, unit53(word_at(key, j, 13)));
    uint32_t v = fmix32(r ^ s32);
    k10[0] = (uint8_t)(v >> 24); k10[1] = (uint8_t)(v >> 16); k10[2] = (uint8_t)(v >> 8); k10[3] = (uint8_t)v;
    uint64_t w = word_at(key, j, 14);
    for (int b = 0; b < 6; b++) k10[4 + b] = (uint8_t)(w >> (8 * b));
}

/* Skewed records.  Record i: payload as in the uniform generator; with
 * probability dup_frac (and i >= 1) its key is an exact copy of base_key(j)
 * for j uniform in [0, i), otherwise base_key(i).  Returns 0, or -1 on
 * allocation failure. */
int dg_records_skewed(uint8_t *out, uint64_t count, uint64_t seed, uint64_t first,
                      uint32_t nvals, double s, double dup_frac) {
    zipf_table t;
    if (nvals == 0 || zipf_build(&t, nvals, s) != 0) return -1;
    const uint64_t key = seed_key(seed);
    const uint32_t s32 = (uint32_t)(key >> 32);
#pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < (int64_t)count; jj++) {
        uint64_t i = first + (uint64_t)jj;
        uint8_t *dst = out + (uint64_t)jj * 100u;
        fill_uniform_one(dst, key, i);
        uint64_t src = i;
        if (i >= 1 && unit53(word_at(key, i, 15)) < dup_frac) {
            src = (uint64_t)(unit53(sm64_out(word_at(key, i, 15) ^ GOLDEN)) * (double)i);
            if (src >= i) src = i - 1;
        }
        base_key(dst, &t, key, s32, src);
    }
    free(t.cdf);
    return 0;
}

/* Probability mass of rank r (1-based) under the same Zipf table, for tests. */
double dg_zipf_pmf(uint32_t nvals, double s, uint32_t r) {
    double acc = 0.0;
    for (uint32_t k = 1; k <= nvals; k++) acc += pow((double)k, -s);
    return pow((double)r, -s) / acc;
}

/* The 4-byte prefix value assigned to Zipf rank r for a seed (for tests). */
uint32_t dg_zipf_value(uint64_t seed, uint32_t r) {
    const uint64_t key = seed_key(seed);
    return fmix32(r ^ (uint32_t)(key >> 32));
}

/* ---- printable (ASCII) keys ------------------------------------------------- */

/* Printable-key records: the payload as in the uniform generator, the key ten
 * bytes each uniform over the 95 printable ASCII values 0x20..0x7E (the
 * key format of the paper's 20 GB dataset, Section 4.1).  Byte b of the key is
 * 0x20 + floor(95 * c / 65536) for the 16-bit chunk c = bits 16*(b%4)..+15 of
 * word 13 + b/4. */
void dg_records_ascii(uint8_t *out, uint64_t count, uint64_t seed, uint64_t first) {
    const uint64_t key = seed_key(seed);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < (int64_t)count; j++) {
        uint8_t *dst = out + (uint64_t)j * 100u;
        const uint64_t i = first + (uint64_t)j;
        fill_uniform_one(dst, key, i);
        uint64_t w[3] = {word_at(key, i, 13), word_at(key, i, 14), word_at(key, i, 15)};
        for (int b = 0; b < 10; b++) {
            const uint32_t c = (uint32_t)(w[b / 4] >> (16 * (b % 4))) & 0xFFFFu;
            dst[b] = (uint8_t)(0x20u + ((95u * c) >> 16));
        }
    }
}
