/*
 * leyenda.h -- C ABI of an MI355X (gfx950) record sorter.
 *
 * Sorts 100-byte records by their 10-byte key: the record format of the
 * paper's workloads (Section 4.1: a 10-byte key followed by a 90-byte value).
 * Keys compare as unsigned byte strings, most significant byte first -- the
 * order in which the 256-way digit buckets of Algorithm 1 (Adaptive Parallel
 * MSD Radix Sort, Section 3.1) split the key from radix 0 upward, and the order
 * of the worked bucket example of Section 2.2.  Records with equal keys keep
 * their input order (a stable sort; the paper leaves ties open), so the output
 * is unique and every entry point below returns exactly the same bytes for the
 * same input, whatever its tuning.
 *
 * Conventions for every entry point:
 *   - Return value: LEYENDA_OK (0) or a negative leyenda_status.  No exception
 *     or signal crosses this boundary.  leyenda_last_error() gives a text for
 *     the last failure on the calling thread.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  GPU
 *     work is enqueued on it and the call returns before that work finishes
 *     unless stated otherwise; results are valid after the stream is
 *     synchronized.  Concurrent calls on different streams are allowed; two
 *     calls on the same stream run in order.
 *   - Record buffers are arrays of n * 100 bytes, 4-byte aligned.  The caller
 *     owns every buffer passed in; the library owns only its scratch memory,
 *     drawn from a per-device, per-stream pool that it keeps between calls
 *     (released by leyenda_release_workspaces()).  The external calls
 *     (leyenda_sort_runs, leyenda_merge, leyenda_sort_external,
 *     leyenda_sort_external_keys) likewise keep one device arena per device,
 *     at most the last call's budget, and one set of pinned bounce buffers
 *     (512 MB) with its host copy threads; a call reuses them when they fit
 *     its budget, and makes its own when another call holds them.
 *   - On error, output buffers hold unspecified bytes, but nothing is written
 *     outside them.
 */
#ifndef LEYENDA_H
#define LEYENDA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LEYENDA_RECORD_BYTES 100
#define LEYENDA_KEY_BYTES 10
/* Largest record count of one sort, run or batch segment: record indices are
 * carried in 32 bits inside the (key, index) tuples (AlphaSort-style key +
 * pointer pairs, Sections 2.1 and 3.2). */
#define LEYENDA_MAX_RECORDS 0xFFFFFFFEull

typedef enum {
    LEYENDA_OK = 0,
    LEYENDA_EINVAL = -1,  /* bad argument: NULL with n > 0, misaligned, overlapping, bad params */
    LEYENDA_ENOMEM = -2,  /* device or pinned-host allocation failed */
    LEYENDA_EBUDGET = -3, /* the work cannot be planned within the given device budget */
    LEYENDA_EHIP = -4,    /* a HIP runtime call failed (see leyenda_last_error) */
    LEYENDA_ETOOBIG = -5, /* more than LEYENDA_MAX_RECORDS records in one sort/run/segment */
    LEYENDA_EINTERNAL = -6 /* a device-side capacity guard fired (a bug; see leyenda_sort_stats) */
} leyenda_status;

/* ---------------------------------------------------------------------------
 * Internal (device-resident) sort -- Algorithm 1 of Section 3.1 plus the
 * key-pointer extraction and record scatter of Section 3.2.
 *
 * records_dev: device pointer, n records (read only).
 * out_dev:     device pointer, n records; receives the records in key order.
 *              Must not overlap records_dev.
 * n:           0 is a no-op returning LEYENDA_OK.
 * Steps run on the GPU: extraction of (key, index) tuples with the first-digit
 * histogram, device-wide MSD digit partitions of buckets larger than the big
 * bucket threshold, per-bucket sorts in LDS (radix partition, then a
 * comparison sort of tiny buckets) and the record gather.
 * ------------------------------------------------------------------------- */
int leyenda_sort(const void *records_dev, uint64_t n, void *out_dev, void *stream);

/* The same sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no hipMalloc, hipFree or other allocating call.  Its scratch is a fixed
 * 64 MiB device array inside the library, one copy per GPU, held until the
 * process ends; its address is looked up once per device on the first call.
 * Arguments, layout, ownership and output are those of leyenda_sort; the
 * caller still allocates records_dev and out_dev.  n is limited by the array:
 * leyenda_noalloc_max_records() gives the largest n for the current
 * parameters (about 1.67 million records with the defaults); a larger n
 * returns LEYENDA_EBUDGET and touches nothing.  Every call on one GPU shares
 * that GPU's array: calls that overlap on the device (different streams, or
 * host threads) race and must be serialized by the caller.  Phase timing
 * (leyenda_profile_*) and leyenda_sort_stats do not cover these calls.
 * Asynchronous on `stream`. */
int leyenda_sort_noalloc(const void *records_dev, uint64_t n, void *out_dev, void *stream);
uint64_t leyenda_noalloc_max_records(void);

/* Flexible key sizes (Section 5 names keys of any size as the method's next
 * step: a prefix sort combined with comparisons of the full keys where the
 * prefixes tie).  Stable sort of n device-resident records by a key of their
 * first key_bytes bytes, 1 <= key_bytes <= 100, in memcmp order; equal keys
 * keep input order.  key_bytes == 10 is leyenda_sort.  key_bytes < 10: the
 * prefix sort with the prefix bytes past the key ignored.  key_bytes > 10: the
 * prefix sort, then rounds over the runs of output records whose leading bytes
 * tie, each round ordering every run by its next six key bytes with one
 * sort of (run number + next bytes, entry number) key-pointer tuples and
 * permuting the runs' record indices to match; rounds end when no tie is left
 * or the key is used up, and the tied positions then take their records from
 * records_dev (which must stay unchanged until the call returns).  Buffers and
 * errors as leyenda_sort, plus LEYENDA_EINVAL for key_bytes outside 1..100 and
 * LEYENDA_ENOMEM when the rounds' scratch (about 92 bytes per record inside a
 * tie run, plus one byte per record and about 6 bytes per 1,024 records, kept
 * per stream between calls) cannot be allocated.  With key_bytes > 10 the call
 * returns after the stream has drained (it reads each round's tie count on the
 * host). */
int leyenda_sort_keyed(const void *records_dev, uint64_t n, uint32_t key_bytes, void *out_dev, void *stream);

/* Device bytes of scratch memory leyenda_sort uses for n records under the
 * current parameters (tuple buffers, index array, bucket tables). */
uint64_t leyenda_workspace_bytes(uint64_t n);

/* First pass (0, 1 or 2: see leyenda_params.first_pass) a leyenda_sort of n
 * records takes under the current parameters: the parameter's value for
 * sorts of at least 8 Mi records whose partition tile holds a fused tile
 * (tile_items 32 for 1, 16 or 32 for 2), else 0. */
uint32_t leyenda_first_pass(uint64_t n);

/* Output parts a leyenda_sort of n records runs in: 1 below 8 Mi records,
 * else 4 (holding 1/16, 1/16, 1/8 and 3/4 of the records in output order).
 * With several parts the local sorts are launched once per part, in
 * output order, and each part's record gather runs on the library's side
 * stream (one per device, shared by every caller stream) as soon as that part
 * is sorted, overlapping the local sorts of the later parts; the sort's stream
 * waits for every gather before it continues, so callers see one ordered
 * operation.  Pure function. */
uint32_t leyenda_sort_parts(uint64_t n);

/* ---------------------------------------------------------------------------
 * Limited-memory (external) sort -- Section 3.2, "Overlapping Computation with
 * I/O": a sort stage that sorts chunks into sorted intermediate runs, then a
 * merge stage that merges the runs with a K-way merge, partition by
 * partition.  host_records and host_runs must be pinned (hipHostMalloc,
 * leyenda_host_alloc, or torch pin_memory()): the copy engines read them and
 * the merge's co-rank kernel reads run keys from them directly.  host_out may
 * be pinned (written by the copy engine) or pageable (written through
 * pinned bounce buffers by host threads).  Both calls are synchronous: they
 * return when the host output is complete.
 *
 * leyenda_sort_runs:
 *   host_records: n records in pinned host memory (read only unless aliased).
 *   device_budget_bytes: cap on the device memory the call allocates.
 *   host_runs: n records of pinned host memory; run r is written, sorted,
 *              over the input range it came from, so host_runs may equal
 *              host_records (in-place run formation).
 *   run_bounds: array of k_max + 1 entries; on success run r covers records
 *              [run_bounds[r], run_bounds[r+1]) and run_bounds[0] = 0,
 *              run_bounds[k] = n (the runs leyenda_plan_runs describes).
 *   k_out: number of runs written.
 *   Returns LEYENDA_EBUDGET if the budget cannot hold the smallest run plan or
 *   more than k_max runs would be needed.
 *
 * leyenda_merge:
 *   host_runs, run_bounds, k: k sorted runs (as produced above; ties between
 *              runs are ordered by run, which is input order).
 *   host_out: n = run_bounds[k] records of host memory (pinned or pageable);
 *              receives the merged output.  Must not overlap host_runs.
 * ------------------------------------------------------------------------- */
int leyenda_sort_runs(const void *host_records, uint64_t n, uint64_t device_budget_bytes,
                      void *host_runs, uint64_t *run_bounds, uint64_t k_max, uint64_t *k_out,
                      void *stream);
int leyenda_merge(const void *host_runs, const uint64_t *run_bounds, uint64_t k, void *host_out,
                  uint64_t device_budget_bytes, void *stream);

/* Runs + merge in one call (Section 3.2, "Overlapping Computation with I/O"):
 * leyenda_sort_runs then leyenda_merge, except that the last two runs stay
 * in device memory after their sorts (the run stage ends with both in its
 * output buffers) instead of being written to host_runs and read back for the
 * merge; their slices reach the merge by device copies.  The merge plans its
 * chunks within the run stage's device memory less the kept runs (else within
 * device_budget_bytes less them), so the whole call stays within the budget.
 * When that is too little for a merge of the runs
 * (many tiny runs under a budget near one run's footprint), only the last run
 * is kept, and when even that is too little, every run is written to
 * host_runs and the merge plans within the whole budget, as leyenda_merge
 * does.
 *   host_records: n records in pinned host memory (read only unless aliased).
 *   host_runs:    n records of pinned host memory for the runs (may equal
 *                 host_records; the ranges of the kept runs are left
 *                 unwritten).
 *   host_out:     n records of host memory, pinned or pageable, overlapping
 *                 neither of the above.
 * Output: the stable sort of the records by their 10-byte key, the same bytes
 * as leyenda_sort.  Synchronous.  LEYENDA_EINVAL (NULL, misaligned,
 * overlapping, unpinned input or runs), LEYENDA_EBUDGET (the budget holds no
 * run, or more runs than the merge takes), LEYENDA_ENOMEM, LEYENDA_EHIP,
 * LEYENDA_EINTERNAL (a device-side guard fired). */
int leyenda_sort_external(const void *host_records, uint64_t n, uint64_t device_budget_bytes, void *host_runs,
                          void *host_out, void *stream);

/* Keys-only external sort (Section 3.2: key-pointer tuples extracted while
 * the input is read, sorted, then the records scattered by the sorted
 * tuples).  The input streams host -> device in chunks and every record's
 * 16-byte (key, index) tuple is kept on the device; all n tuples are then
 * sorted in one device-resident pass (Algorithm 1).  A pinned host_out: the
 * input streams up a second time, in order, and every record is written by
 * the device straight to its place in host_out (random 100-byte PCIe writes).
 * A pageable host_out: the records are gathered in sorted order by device
 * loads straight from the pinned input (random 100-byte PCIe reads) and
 * streamed out through pinned bounce buffers.  No runs, no
 * merge: it needs the tuples and sort tables of all n records on the device
 * (leyenda_workspace_bytes(n) + 256 bytes, about 43 bytes per record), and
 * returns LEYENDA_EBUDGET, touching nothing, when device_budget_bytes is
 * below that (leyenda_sort_runs + leyenda_merge then fit).
 *   host_records: n records in pinned host memory (read only; read by the
 *                 copy engine, and by the pageable-output gather through its
 *                 device mapping).
 *   host_out:     n records of host memory, pinned (written by the device
 *                 through its mapping) or pageable (through pinned bounce
 *                 buffers and host copies); must not overlap host_records.
 * Output: the stable sort of the records by their 10-byte key, the same bytes
 * as leyenda_sort.  Synchronous: returns when host_out is complete.
 * LEYENDA_EINVAL (NULL, misaligned, overlapping, unpinned input),
 * LEYENDA_ETOOBIG (n > LEYENDA_MAX_RECORDS), LEYENDA_ENOMEM, LEYENDA_EHIP,
 * LEYENDA_EINTERNAL (a device-side guard of the sort or the scatter fired). */
int leyenda_sort_external_keys(const void *host_records, uint64_t n, uint64_t device_budget_bytes,
                               void *host_out, void *stream);

/* Pinned host memory for the external path (hipHostMalloc; exactly `bytes`,
 * no rounding).  leyenda_host_free(NULL) is a no-op. */
int leyenda_host_alloc(uint64_t bytes, void **out);
int leyenda_host_free(void *p);

/* Run plan of leyenda_sort_runs for n records under a budget: records per run
 * and number of runs (equal runs, the last possibly shorter; host-only
 * arithmetic, no GPU work).  LEYENDA_EBUDGET if the budget is too small. */
int leyenda_plan_runs(uint64_t n, uint64_t device_budget_bytes, uint64_t *run_records,
                      uint64_t *num_runs);

/* Plan of leyenda_sort_external for n records under a budget (host-only
 * arithmetic, no GPU work): records per run, number of runs, and how many of
 * the last runs stay on the device between the two stages (2, 1, or 0 when
 * the merge needs the whole budget; 1 for a single run, which is the output).
 * LEYENDA_EINVAL (NULL), LEYENDA_EBUDGET (no run fits, or more runs than the
 * merge takes). */
int leyenda_plan_external(uint64_t n, uint64_t device_budget_bytes, uint64_t *run_records,
                          uint64_t *num_runs, uint64_t *kept_runs);

/* ---------------------------------------------------------------------------
 * Batched sort: many independent sort requests in one launch sequence (the
 * analogue of Algorithm 1's shared small-bucket task queue, applied across
 * requests).  Each segment is sorted on its own, exactly as leyenda_sort would
 * sort it; segments never interact.  Segment buffers are device pointers.
 * The launch sequence is captured once per stream into a HIP graph and
 * replayed; per-batch arguments travel in a device descriptor table.
 * ------------------------------------------------------------------------- */
typedef struct {
    const void *in; /* device, n records */
    void *out;      /* device, n records, not overlapping in */
    uint64_t n;
} leyenda_segment;

int leyenda_sort_batch(const leyenda_segment *segs, uint64_t count, void *stream);

/* ---------------------------------------------------------------------------
 * Serving engine (continuous batching).  Sort requests arrive over time; a
 * dispatcher thread admits them in arrival order while their output buffers
 * fit the device budget, groups the admitted ones into batches (at most
 * max_batch requests and max_batch_records records per batch) and runs each
 * batch as one batched sort on one of `slots` streams, so batches overlap on
 * the GPU and requests arriving meanwhile join the next free slot.  Output
 * buffers are owned by the engine and stay resident until released.
 * With batched == 0 the engine runs one plain leyenda_sort per request, in
 * arrival order, on one stream (the comparison baseline).
 *
 * budget_bytes covers every device byte the engine allocates: one sort
 * workspace per slot plus the arena holding admitted requests' outputs
 * (100 bytes per record).  LEYENDA_EBUDGET if it cannot hold the workspaces
 * and one full batch.
 * ------------------------------------------------------------------------- */
typedef struct leyenda_server leyenda_server;

typedef struct {
    uint64_t budget_bytes;
    uint32_t slots;
    uint32_t max_batch;
    uint64_t max_batch_records;  /* also the largest request accepted */
    int32_t batched;
} leyenda_server_config;

typedef struct {
    uint64_t tag;
    void *out_dev;     /* the sorted records, valid until leyenda_server_release(tag) */
    uint64_t n;
    double submit_s;   /* steady-clock seconds: submitted, launched, seen complete */
    double start_s;
    double done_s;
    int32_t status;
} leyenda_done;

int leyenda_server_create(const leyenda_server_config *cfg, leyenda_server **out);
/* Queues a request: n records at in_dev (device memory the caller keeps
 * unchanged until the request completes); tag must be unused. */
int leyenda_server_submit(leyenda_server *s, const void *in_dev, uint64_t n, uint64_t tag);
/* Completed requests (up to cap), waiting up to timeout_s seconds for one. */
int leyenda_server_poll(leyenda_server *s, leyenda_done *out, uint64_t cap, uint64_t *count, double timeout_s);
/* Frees a completed request's output buffer. */
int leyenda_server_release(leyenda_server *s, uint64_t tag);
int leyenda_server_destroy(leyenda_server *s);

/* Replays an arrival stream against a fresh engine: request i (n[i] records
 * at in_dev[i]) is submitted arrival_s[i] seconds after the start (arrivals
 * non-decreasing); latency_s[i] = completion - arrival, including queueing;
 * makespan_s = last completion - start.  Outputs are released on completion. */
int leyenda_serve_replay(const leyenda_server_config *cfg, uint64_t count, const void *const *in_dev,
                         const uint64_t *n, const double *arrival_s, double *latency_s, double *makespan_s);

/* ---------------------------------------------------------------------------
 * Tuning parameters.  They change speed only, never the output bytes.
 * Defaults: digit_bits 8, tile_items 32, big_threshold 2048, tiny_threshold 128,
 * local_capacity 2048, scatter_threads 1024, local_threads 512 (the fastest of
 * the autotuner's sweep on the 10 GB uniform and 20 GB skewed workloads; the
 * tiny threshold from a later sweep of 64..256 on those and on printable keys,
 * whose local-sort tasks pack sub-buckets of about a hundred keys and gain
 * from it, while the binary workloads do not change), first_pass 1 (the
 * fused pass: 10.34 against 10.95 ms for the 10 GB sort, 25.8 against 27.0 ms
 * for the 20 GB skewed one; the record copy of 2 costs more in its pass than
 * it saves in the gather, 13.4 ms).
 * digit_bits     radix digit width in bits, 4..8 (8: 256 buckets per pass, the
 *                byte digit of Algorithm 1; a narrower digit splits each big
 *                bucket 2^digit_bits ways and needs up to ceil(80 / digit_bits)
 *                partition levels).
 * tile_items     keys per thread in a device-wide partition tile (8, 16 or 32;
 *                a tile is 256 * tile_items keys).
 * big_threshold  buckets with more keys than this get another device-wide
 *                partition pass (Algorithm 1's bigBucketThreshold);
 *                1 <= big_threshold <= local_capacity.
 * tiny_threshold buckets of at most this many keys inside a local sort are
 *                ordered by comparisons instead of another radix partition
 *                (Algorithm 1's tinyBucketThreshold); 1..256.
 * local_capacity keys one workgroup sorts in LDS (2048).
 * scatter_threads threads per device-wide partition workgroup (256, 512 or
 *                1024; the tile stays 256 * tile_items keys).
 * local_threads  threads per local-sort workgroup (256 or 512).
 * first_pass     how a single sort of at least 8 Mi records makes its
 *                first-digit buckets (Algorithm 1's first partition round on
 *                the key-pointer tuples of Section 3.2):
 *                0  an extraction pass writes the tuples in input order with
 *                   the first-digit histogram, then a partition pass moves
 *                   them into their buckets;
 *                1  one pass extracts the tuples and writes them straight
 *                   into their buckets, each bucket a chain of fixed-size
 *                   chunks (its size is unknown while the pass runs; a tile's
 *                   offset inside a bucket comes from a look-back over the
 *                   tiles before it);
 *                2  as 1, and the pass also copies every record into its
 *                   bucket's chunks, so the final gather reads one bucket's
 *                   region at a time (Section 3.1, cache-aware scattering)
 *                   instead of the whole input.
 *                Smaller sorts, batches and the external calls always use 0.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint32_t digit_bits;
    uint32_t tile_items;
    uint32_t big_threshold;
    uint32_t tiny_threshold;
    uint32_t local_capacity;
    uint32_t scatter_threads;
    uint32_t local_threads;
    uint32_t first_pass;
} leyenda_params;

int leyenda_get_params(leyenda_params *out);
int leyenda_set_params(const leyenda_params *p); /* LEYENDA_EINVAL if out of range */
/* Loads a flat JSON object with any of the field names above (the file the
 * autotuner writes).  Unknown keys are ignored. */
int leyenda_load_params(const char *json_path);

/* ---------------------------------------------------------------------------
 * Diagnostics.
 * ------------------------------------------------------------------------- */
#define LEYENDA_MAX_LEVELS 20 /* partition levels of the narrowest digit (4 bits over 80 key bits) */
typedef struct {
    uint32_t levels;          /* device-wide partition levels that moved data */
    uint32_t segments[LEYENDA_MAX_LEVELS]; /* big buckets planned at each level */
    uint64_t moved[LEYENDA_MAX_LEVELS];    /* keys moved by the device-wide partition at each level */
    uint64_t tasks;           /* local-sort tasks */
    uint32_t guard;           /* nonzero if a device-side capacity guard fired */
} leyenda_stats;

/* Synchronizes `stream` and reports the plan of the last leyenda_sort on it. */
int leyenda_sort_stats(void *stream, leyenda_stats *out);

/* Phase timing with HIP events recorded on each sort's own stream.  While
 * enabled, every leyenda_sort records events between its phases; phase_ms
 * receives the summed milliseconds since the last enable of
 *   [0] tuple extraction (+ first-digit histograms),
 *   [1] device-wide partition levels (histograms, planning, scatter passes),
 *   [2] local sorts in LDS,
 *   [3] record gather,
 * and calls the number of sorts timed.  A sort of 8 Mi records or more runs
 * its local sorts and gathers per output part, the gather of a part on a side
 * stream while later parts are sorted; there [2] ends with the last part's
 * local sorts and [3] is the sum of the gather kernels' own durations, so the
 * phases overlap.  leyenda_profile_read synchronizes the events it reads. */
int leyenda_profile_enable(int on);
int leyenda_profile_read(double *phase_ms, uint64_t *calls);

const char *leyenda_status_string(int status);
const char *leyenda_last_error(void);
/* Frees every cached workspace, external arena and bounce buffer not in use
 * by a running call (synchronizes the device first). */
int leyenda_release_workspaces(void);

/* ---------------------------------------------------------------------------
 * Step-level entry points used by the parity tests.
 *
 * leyenda_debug_extract: the first stage of leyenda_sort alone -- the request
 *   table, the level-0 bucket and the sort's own extraction kernel, launched
 *   exactly as the sort launches it (same tiles, key masks and histogram
 *   replicas) on the workspace of `stream` -- for the key-pointer tuples of
 *   Section 3.2 and the first-digit histogram of Algorithm 1.  For record i:
 *   hi[i] = big-endian key bytes 0..7 and lo[i] = (big-endian key bytes 8..9)
 *   << 32 | i, with the bytes at and past key_bytes (1..10) cleared (the
 *   masked prefix of leyenda_sort_keyed); hist[d] = number of records whose
 *   leading digit_bits (leyenda_params) key bits equal d, 256 counters (those
 *   at and above 2^digit_bits stay zero).  All device pointers: records 4-byte
 *   aligned, hi and lo 8-byte aligned (n entries each), hist 256 u32.
 *   Asynchronous on `stream`.  LEYENDA_EINVAL for NULL or misaligned buffers
 *   or key_bytes outside 1..10, LEYENDA_ETOOBIG for n > LEYENDA_MAX_RECORDS,
 *   LEYENDA_ENOMEM if the workspace cannot be allocated.
 * leyenda_debug_gather: out[j] = records[idx[j]] for j < n with the sort's
 *   record gather kernel (device pointers; idx holds n indices below
 *   n_records).
 * ------------------------------------------------------------------------- */
int leyenda_debug_extract(const void *records_dev, uint64_t n, uint32_t key_bytes, uint64_t *hi_dev,
                          uint64_t *lo_dev, uint32_t *hist_dev, void *stream);
int leyenda_debug_gather(const void *records_dev, uint64_t n_records, const uint32_t *idx_dev,
                         uint64_t n, void *out_dev, void *stream);

/* leyenda_debug_first_pass: the fused first pass of leyenda_sort alone
 * (first_pass 1 or 2, see leyenda_params), launched as the sort launches it
 * (for any n >= 1; the sort itself takes it from 8 Mi records on): one pass
 * that extracts the key-pointer tuples (Section 3.2) and partitions them by
 * the leading digit (Algorithm 1's first round) into per-bucket chains of
 * chunks, then the level-1 bucket table.  The buckets are copied out in
 * bucket order: bucket d's tuples at hi/lo[base_d + p] for its positions p =
 * 0..count[d]-1, base_d being the sum of count[d'] over d' < d; position p is
 * the p-th record of bucket d in input order (hi as leyenda_debug_extract;
 * lo's low 32 bits are the record index for first_pass 1 and p for 2).  With
 * first_pass 2 rec_out (n x 100 bytes) receives the copied records in the
 * same order.  count: 256 u32.  Key bytes past key_bytes (1..10) are cleared.
 * Runs on the workspace of `stream`, asynchronously.  LEYENDA_EINVAL for
 * NULL or misaligned buffers, first_pass or key_bytes out of range, or
 * parameters whose partition tile cannot hold a fused tile; LEYENDA_ETOOBIG
 * for n > LEYENDA_MAX_RECORDS; LEYENDA_ENOMEM if the workspace cannot be
 * allocated. */
int leyenda_debug_first_pass(const void *records_dev, uint64_t n, uint32_t first_pass, uint32_t key_bytes,
                             uint64_t *hi_dev, uint64_t *lo_dev, uint32_t *count_dev, void *rec_out_dev,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LEYENDA_H */
