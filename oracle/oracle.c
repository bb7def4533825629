/*
 * CPU oracle for the record sort -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library never links, calls or
 * includes anything from here, and this file includes nothing from it.
 *
 * What the sort computes (a plain definition, which every schedule of the
 * paper's method reaches exactly):
 *   Records are 100 bytes; the key is bytes [0,10) and the value bytes
 *   [10,100) (Section 4.1).  Keys are ordered as unsigned byte strings, most
 *   significant byte first: the 256-way digit buckets of Algorithm 1 are taken
 *   over the key bytes from radix 0 upward, and the worked example of
 *   Section 2.2 orders "abc" < "bcd" < "cde" < "cfe" < "dfg" byte by byte.
 *   That is memcmp order on the 10 key bytes.  The paper does not say how
 *   records with equal keys are ordered; this oracle keeps them in input
 *   order (a stable sort), which makes the sorted output unique.
 *
 * Functions:
 *   oracle_sort           stable sort by memcmp on the key, then gather records
 *   oracle_output_rank    output position of chosen input records, one by one
 *   oracle_count_less     keys below given probe keys (sorted position of a
 *                         probe whose key is unique)
 *   oracle_equal_neighbours  adjacent equal keys in an output
 *   oracle_first_unsorted first adjacent pair out of key order
 *   oracle_multiset_hash  order-independent hash of a record multiset
 *   oracle_ties_in_order  equal-key runs of an output hold their records in
 *                         input order (with the two checks above, this
 *                         pins a large output without a full oracle sort)
 *   oracle_sort_par       oracle_sort on several host threads (slices sorted
 *                         by the same comparison, then merged); the same result
 *   oracle_sort_key       the same stable sort with a key of the first K
 *                         bytes, 1 <= K <= 100: the flexible key sizes that
 *                         Section 5 names as the method's next step (same
 *                         order definition: memcmp on the K key bytes, equal
 *                         keys in input order)
 */
#define _GNU_SOURCE
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REC 100
#define KEY 10

/* ---- oracle_sort ---------------------------------------------------------- */

typedef struct {
    uint8_t key[KEY];
    uint8_t pad[2];
    uint32_t idx;
} key_idx;

/* memcmp order on the key, then input order for equal keys. */
static int cmp_key_idx(const void *pa, const void *pb) {
    const key_idx *a = (const key_idx *)pa, *b = (const key_idx *)pb;
    int c = memcmp(a->key, b->key, KEY);
    if (c != 0) return c;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Stable sort of n records by key; writes the sorted records to out and, if
 * perm is not NULL, perm[j] = input index of output record j.  n must be
 * below 2^32.  Returns 0, or -1 if memory could not be allocated. */
int oracle_sort(const uint8_t *rec, uint64_t n, uint8_t *out, uint32_t *perm) {
    if (n == 0) return 0;
    if (n >= 0xFFFFFFFFull) return -1;
    key_idx *t = (key_idx *)malloc(sizeof(key_idx) * n);
    if (!t) return -1;
    for (uint64_t i = 0; i < n; i++) {
        memcpy(t[i].key, rec + i * REC, KEY);
        t[i].pad[0] = t[i].pad[1] = 0;
        t[i].idx = (uint32_t)i;
    }
    qsort(t, n, sizeof(key_idx), cmp_key_idx);
    for (uint64_t j = 0; j < n; j++) {
        memcpy(out + j * REC, rec + (uint64_t)t[j].idx * REC, REC);
        if (perm) perm[j] = t[j].idx;
    }
    free(t);
    return 0;
}

/* ---- oracle_sort_par ---------------------------------------------------------- */

/* Host threads the parallel oracle uses when asked for 0 (all of them). */
int oracle_threads(void) { return omp_get_max_threads(); }

/* Number of elements the first r outputs of merging the sorted arrays a (na
 * elements) and b (nb) take from a.  The (key, index) order is total -- no
 * two pairs compare equal -- so the split is unique: the largest i with
 * a[i-1] < b[r-i], found by binary search. */
static uint64_t merge_split(const key_idx *a, uint64_t na, const key_idx *b, uint64_t nb, uint64_t r) {
    uint64_t lo = r > nb ? r - nb : 0, hi = r < na ? r : na;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (cmp_key_idx(&a[mid], &b[r - mid - 1]) < 0) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* The same stable sort as oracle_sort, on `threads` host threads (0: all).
 * The (key, index) pairs are cut into one slice per thread; each slice is
 * sorted by qsort under the comparison oracle_sort uses; neighbouring sorted
 * slices are then merged pairwise until one remains, each merge cut into
 * per-thread pieces at exact output ranks (merge_split), and the records are
 * gathered.  Since no two pairs compare equal, the merged order is the one
 * qsort gives over the whole array.  Returns the thread count used, or -1 if
 * memory could not be allocated. */
int oracle_sort_par(const uint8_t *rec, uint64_t n, uint8_t *out, uint32_t *perm, int threads) {
    if (threads <= 0) threads = omp_get_max_threads();
    if (n == 0) return threads;
    if (n >= 0xFFFFFFFFull) return -1;
    key_idx *a = (key_idx *)malloc(sizeof(key_idx) * n);
    key_idx *b = (key_idx *)malloc(sizeof(key_idx) * n);
    uint64_t *bnd = (uint64_t *)malloc(sizeof(uint64_t) * ((uint64_t)threads + 1));
    if (!a || !b || !bnd) { free(a); free(b); free(bnd); return -1; }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t i = 0; i < (int64_t)n; i++) {
        memcpy(a[i].key, rec + (uint64_t)i * REC, KEY);
        a[i].pad[0] = a[i].pad[1] = 0;
        a[i].idx = (uint32_t)i;
    }
    uint64_t ns = (uint64_t)threads;  /* slices: bnd[k] .. bnd[k + 1] */
    for (uint64_t k = 0; k <= ns; k++) bnd[k] = n * k / ns;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (int64_t k = 0; k < (int64_t)ns; k++)
        qsort(a + bnd[k], bnd[k + 1] - bnd[k], sizeof(key_idx), cmp_key_idx);
    while (ns > 1) {
        /* merge slices (2m, 2m + 1) into b; an odd last slice is copied */
        const uint64_t pairs = (ns + 1) / 2;
        const uint64_t pieces = (uint64_t)threads;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1) collapse(2)
        for (int64_t m = 0; m < (int64_t)pairs; m++) {
            for (int64_t p = 0; p < (int64_t)pieces; p++) {
                const uint64_t lo = bnd[2 * m], mid = 2 * m + 1 <= ns ? bnd[2 * m + 1] : bnd[ns];
                const uint64_t hi = 2 * m + 2 <= ns ? bnd[2 * m + 2] : bnd[ns];
                const uint64_t na = mid - lo, nb = hi - mid, tot = hi - lo;
                const uint64_t r0 = tot * (uint64_t)p / pieces, r1 = tot * (uint64_t)(p + 1) / pieces;
                uint64_t i = merge_split(a + lo, na, a + mid, nb, r0);
                uint64_t j = r0 - i;
                const uint64_t i1 = merge_split(a + lo, na, a + mid, nb, r1), j1 = r1 - i1;
                for (uint64_t o = lo + r0; o < lo + r1; o++) {
                    if (j >= j1 || (i < i1 && cmp_key_idx(&a[lo + i], &a[mid + j]) < 0)) b[o] = a[lo + i++];
                    else b[o] = a[mid + j++];
                }
            }
        }
        for (uint64_t m = 0; m < pairs; m++) bnd[m] = bnd[2 * m];
        bnd[pairs] = n;
        ns = pairs;
        key_idx *t = a; a = b; b = t;
    }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t j = 0; j < (int64_t)n; j++) {
        memcpy(out + (uint64_t)j * REC, rec + (uint64_t)a[j].idx * REC, REC);
        if (perm) perm[j] = a[j].idx;
    }
    free(a);
    free(b);
    free(bnd);
    return threads;
}

/* ---- oracle_sort_key ---------------------------------------------------------- */

typedef struct {
    const uint8_t *rec;
    uint32_t key_bytes;
} key_ctx;

/* memcmp order on the first key_bytes bytes of two records, then input order. */
static int cmp_prefix_idx(const void *pa, const void *pb, void *pc) {
    const key_ctx *c = (const key_ctx *)pc;
    const uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    int r = memcmp(c->rec + (uint64_t)a * REC, c->rec + (uint64_t)b * REC, c->key_bytes);
    if (r != 0) return r;
    return (a > b) - (a < b);
}

/* Stable sort of n records by their first key_bytes bytes (1..100); out and
 * perm as in oracle_sort.  Returns 0, -1 if memory could not be allocated,
 * -2 for a key size outside 1..100. */
int oracle_sort_key(const uint8_t *rec, uint64_t n, uint32_t key_bytes, uint8_t *out, uint32_t *perm) {
    if (key_bytes < 1 || key_bytes > REC) return -2;
    if (n == 0) return 0;
    if (n >= 0xFFFFFFFFull) return -1;
    uint32_t *ix = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!ix) return -1;
    for (uint64_t i = 0; i < n; i++) ix[i] = (uint32_t)i;
    key_ctx c = {rec, key_bytes};
    qsort_r(ix, n, sizeof(uint32_t), cmp_prefix_idx, &c);
    for (uint64_t j = 0; j < n; j++) {
        memcpy(out + j * REC, rec + (uint64_t)ix[j] * REC, REC);
        if (perm) perm[j] = ix[j];
    }
    free(ix);
    return 0;
}

/* ---- oracle_output_rank ----------------------------------------------------- */

/* For each sample s (an input index), its position in the stable sorted output:
 *   rank(s) = #{ j : key_j < key_s } + #{ j < s : key_j == key_s }.
 * One pass over the input for all samples; the pass is split over threads,
 * each with its own counters, and the counters are summed at the end. */
void oracle_output_rank(const uint8_t *rec, uint64_t n, const uint64_t *samples, uint64_t m,
                        uint64_t *ranks) {
    for (uint64_t s = 0; s < m; s++) ranks[s] = 0;
#pragma omp parallel
    {
        uint64_t *local = (uint64_t *)calloc(m ? m : 1, sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t jj = 0; jj < (int64_t)n; jj++) {
            uint64_t j = (uint64_t)jj;
            const uint8_t *kj = rec + j * REC;
            for (uint64_t s = 0; s < m; s++) {
                int c = memcmp(kj, rec + samples[s] * REC, KEY);
                if (c < 0 || (c == 0 && j < samples[s])) local[s]++;
            }
        }
#pragma omp critical
        for (uint64_t s = 0; s < m; s++) ranks[s] += local[s];
        free(local);
    }
}

/* ---- oracle_count_less ------------------------------------------------------ */

/* counts[s] = #{ j : key_j < key of probe s } over n records, for m probe
 * records (given as records of their own, so the array may be any permutation
 * of the input).  When the probe's key occurs once, this is its position in
 * the sorted output. */
void oracle_count_less(const uint8_t *rec, uint64_t n, const uint8_t *probes, uint64_t m, uint64_t *counts) {
    for (uint64_t s = 0; s < m; s++) counts[s] = 0;
#pragma omp parallel
    {
        uint64_t *local = (uint64_t *)calloc(m ? m : 1, sizeof(uint64_t));
#pragma omp for schedule(static)
        for (int64_t jj = 0; jj < (int64_t)n; jj++) {
            const uint8_t *kj = rec + (uint64_t)jj * REC;
            for (uint64_t s = 0; s < m; s++)
                if (memcmp(kj, probes + s * REC, KEY) < 0) local[s]++;
        }
#pragma omp critical
        for (uint64_t s = 0; s < m; s++) counts[s] += local[s];
        free(local);
    }
}

/* Number of adjacent output pairs with equal keys. */
uint64_t oracle_equal_neighbours(const uint8_t *out, uint64_t n) {
    uint64_t c = 0;
    if (n < 2) return 0;
#pragma omp parallel for schedule(static) reduction(+ : c)
    for (int64_t j = 0; j < (int64_t)n - 1; j++)
        if (memcmp(out + (uint64_t)j * REC, out + (uint64_t)(j + 1) * REC, KEY) == 0) c++;
    return c;
}

/* ---- oracle_first_unsorted -------------------------------------------------- */

/* Smallest j with key(out[j]) > key(out[j+1]), or -1 if keys never decrease. */
int64_t oracle_first_unsorted(const uint8_t *out, uint64_t n) {
    int64_t best = INT64_MAX;
    if (n < 2) return -1;
#pragma omp parallel for schedule(static) reduction(min : best)
    for (int64_t j = 0; j < (int64_t)n - 1; j++) {
        if (memcmp(out + (uint64_t)j * REC, out + (uint64_t)(j + 1) * REC, KEY) > 0 && j < best) best = j;
    }
    return best == INT64_MAX ? -1 : best;
}

/* ---- oracle_multiset_hash --------------------------------------------------- */

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* A keyed hash of one 100-byte record, taken over its 25 little-endian words. */
static inline uint64_t record_hash(const uint8_t *r, uint64_t key) {
    uint64_t h = key;
    for (int k = 0; k < 25; k++) {
        uint32_t w;
        memcpy(&w, r + 4 * k, 4);
        h = mix64(h ^ ((uint64_t)w + 0x9E3779B97F4A7C15ULL * (uint64_t)(k + 1)));
    }
    return h;
}

/* Sums, modulo 2^64, of two independently keyed record hashes.  The sums do
 * not depend on record order, so equal multisets give equal pairs. */
void oracle_multiset_hash(const uint8_t *rec, uint64_t n, uint64_t *h2) {
    uint64_t a = 0, b = 0;
#pragma omp parallel for schedule(static) reduction(+ : a, b)
    for (int64_t j = 0; j < (int64_t)n; j++) {
        a += record_hash(rec + (uint64_t)j * REC, 0x243F6A8885A308D3ULL);
        b += record_hash(rec + (uint64_t)j * REC, 0x13198A2E03707344ULL);
    }
    h2[0] = a;
    h2[1] = b;
}

/* ---- oracle_ties_in_order --------------------------------------------------- */

/* Checks that every run of equal keys in `out` (length >= 2) holds exactly the
 * input records with that key, in input order.  Walks the input once in index
 * order; each input record whose key owns a run must equal the next unread
 * record of that run.
 * Returns 0 if so, 1 if a run is out of input order or incomplete, -1 if
 * memory could not be allocated. */
typedef struct {
    uint64_t start, len, cursor;
} run_t;

static inline uint64_t key_hash(const uint8_t *k) {
    uint64_t a, b = 0;
    memcpy(&a, k, 8);
    memcpy(&b, k + 8, 2);
    return mix64(a ^ mix64(b + 0x9E3779B97F4A7C15ULL));
}

int oracle_ties_in_order(const uint8_t *in, const uint8_t *out, uint64_t n) {
    /* 1. runs of equal keys in the output */
    uint64_t nruns = 0;
    for (uint64_t j = 0; j + 1 < n;) {
        uint64_t e = j + 1;
        while (e < n && memcmp(out + j * REC, out + e * REC, KEY) == 0) e++;
        if (e - j >= 2) nruns++;
        j = e;
    }
    if (nruns == 0) return 0;
    run_t *runs = (run_t *)malloc(sizeof(run_t) * nruns);
    uint64_t cap = 1;
    while (cap < 2 * nruns) cap <<= 1;
    int64_t *table = (int64_t *)malloc(sizeof(int64_t) * cap);
    if (!runs || !table) { free(runs); free(table); return -1; }
    for (uint64_t t = 0; t < cap; t++) table[t] = -1;
    uint64_t r = 0;
    for (uint64_t j = 0; j + 1 < n;) {
        uint64_t e = j + 1;
        while (e < n && memcmp(out + j * REC, out + e * REC, KEY) == 0) e++;
        if (e - j >= 2) {
            runs[r].start = j; runs[r].len = e - j; runs[r].cursor = j;
            uint64_t h = key_hash(out + j * REC) & (cap - 1);
            while (table[h] != -1) h = (h + 1) & (cap - 1);
            table[h] = (int64_t)r;
            r++;
        }
        j = e;
    }
    /* 2. walk the input in index order */
    int bad = 0;
    for (uint64_t i = 0; i < n && !bad; i++) {
        const uint8_t *k = in + i * REC;
        uint64_t h = key_hash(k) & (cap - 1);
        while (table[h] != -1) {
            run_t *ru = &runs[table[h]];
            if (memcmp(out + ru->start * REC, k, KEY) == 0) {
                if (ru->cursor >= ru->start + ru->len || memcmp(out + ru->cursor * REC, k, REC) != 0) bad = 1;
                ru->cursor++;
                break;
            }
            h = (h + 1) & (cap - 1);
        }
    }
    for (uint64_t t = 0; t < nruns && !bad; t++)
        if (runs[t].cursor != runs[t].start + runs[t].len) bad = 1;
    free(runs);
    free(table);
    return bad;
}
