// Internal definitions shared by the device kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ley {

constexpr int kRec = 100;          // record bytes (Section 4.1)
constexpr int kKeyBits = 80;       // 10-byte key
constexpr uint32_t kKeyBytes = 10;
constexpr int kRB = 8;             // widest digit: 256-way buckets per pass (Algorithm 1's byte digit)
constexpr int kRadix = 1 << kRB;   // counters per histogram (a narrower digit leaves the top ones at zero)
constexpr int kMinRB = 4;          // narrowest digit width the partition levels take
constexpr int kWG = 256;           // threads per workgroup, all kernels (4 wave64)
constexpr int kWaves = kWG / 64;
constexpr int kMaxRep = 64;        // histogram replicas per bucket (spreads the tiles' atomics)
constexpr int kRepWords = kRadix + 8;  // replica: 256 counts + OR / OR-of-complement masks (4 x u64)
constexpr int kMaxLev = (kKeyBits + kMinRB - 1) / kMinRB;  // device-wide partition levels at most (narrowest digit)
// Partition levels a digit width of `bits` needs to cover the key.
__host__ __device__ constexpr int levels_for(int bits) { return (kKeyBits + bits - 1) / bits; }
constexpr int kLocalCap = 2048;    // keys per local (LDS) sort task
constexpr uint16_t kNoScatter = 0xFFFF;

constexpr uint64_t kFlagAgg = 1ull << 62;  // look-back status: chunk aggregate published
constexpr uint64_t kFlagInc = 2ull << 62;  // look-back status: inclusive prefix published
constexpr int kChunkTiles = 64;            // tiles per chunk of the tile-offset scan
constexpr uint64_t kCountMask = (1ull << 62) - 1;

constexpr uint8_t kTaskSorted = 1;  // task range is already in final order
// Output parts of a large single sort: the local sorts of part k run as one
// launch, and the gather of part k overlaps the local sorts of later parts.
constexpr int kParts = 4;

// A bucket that gets a device-wide partition pass at some level.
struct Seg {
    uint64_t start;       // first key in the tuple arrays
    uint32_t count;
    uint32_t first_tile;  // its tiles at this level are [first_tile, first_tile + ntiles)
    uint32_t ntiles;
    uint32_t rep_first;   // its histogram replicas are [rep_first, rep_first + nrep)
    uint16_t pos;         // key bit where the histogram digit starts
    uint16_t spos;        // key bit of the partition digit, or kNoScatter
    uint8_t buf;          // tuple buffer holding the segment
    uint8_t nrep;
    uint16_t req;         // batch request the segment belongs to
};
static_assert(sizeof(Seg) == 32, "Seg layout");

// A local-sort task: a contiguous range of whole buckets, each small enough
// for LDS, or a range that is already in order.
struct Task {
    uint64_t start;
    uint32_t count;
    uint8_t buf;
    uint8_t flags;
    uint16_t req;         // batch request the range belongs to
};
static_assert(sizeof(Task) == 16, "Task layout");

// Per-sort control block (device memory).
struct Ctl {
    uint32_t nseg[kMaxLev + 2];
    uint32_t ntiles[kMaxLev + 2];
    uint32_t tile_ctr[kMaxLev + 2];
    uint32_t rep_ctr[kMaxLev + 2];
    uint32_t chunk_ctr[kMaxLev + 2];
    uint32_t ntask[kParts];     // local-sort tasks per output part
    uint32_t task_ctr[kParts];  // next task of each part
    uint32_t guard;
    uint32_t pad;
    unsigned long long moved[kMaxLev + 2];
    uint32_t ftile_ctr;         // next tile of the fused first pass
    uint32_t pool_ctr;          // next free chunk of the first-pass tuple pool
};

// Batch request (level-0 segment) descriptor.
struct Req {
    const uint8_t *in;
    uint8_t *out;
    uint64_t start;       // first key of the request in the batch's tuple space
    uint64_t n;
    uint32_t first_tile;  // its level-0 tiles
    uint32_t ntiles;
    uint32_t rep_first;   // its level-0 histogram replicas
    uint32_t nrep;
};

// Batch header: sizes the kernels read from device memory, so a captured
// launch sequence can be replayed for another batch.
struct Hdr {
    uint64_t n_total;     // keys over all requests
    uint32_t nreq;
    uint32_t tiles0;      // level-0 tiles over all requests
};

// Runtime tuning values the kernels read.
struct Tune {
    uint32_t digit;        // partition digit width in bits (kMinRB..kRB)
    uint32_t tile_items;   // 8, 16 or 32
    uint32_t tile;         // kWG * tile_items
    uint32_t big;          // big-bucket threshold
    uint32_t tiny;         // comparison-sort threshold inside the local sort
    uint32_t scatter_wg;   // threads per partition workgroup (256, 512 or 1024; same tile)
    uint32_t local_wg;     // threads per local-sort workgroup (256 or 512)
    uint32_t first_pass;   // kFirstSplit, kFirstFused or kFirstRecords (large single sorts)
};

// How a large single sort makes its level-0 buckets.
//   kFirstSplit    extraction pass (tuples in input order + first-digit
//                  histogram), then a partition pass over the tuples
//   kFirstFused    one pass: tuples extracted and written straight into their
//                  first-digit buckets, held as chains of chunks (the bucket
//                  sizes are not known while the pass runs); a tile's offset
//                  inside each bucket comes from a look-back over the tiles
//                  before it
//   kFirstRecords  the same pass also copies each record into its bucket's
//                  chunks, so the final gather reads records from a region of
//                  one bucket at a time instead of from the whole input
constexpr uint32_t kFirstSplit = 0, kFirstFused = 1, kFirstRecords = 2;
// Fused first pass: 1,024 threads a tile, 8 keys each (4 with the record
// copy, whose staging needs LDS too).  A tile must not exceed the partition
// tile (the chunk), so a tile's run of one digit spans at most two chunks.
constexpr int kFuseWG = 1024;
__host__ __device__ constexpr int fuse_items(uint32_t first_pass) { return first_pass == kFirstRecords ? 4 : 8; }
__host__ __device__ constexpr uint32_t fuse_tile(uint32_t first_pass) { return kFuseWG * fuse_items(first_pass); }

// Device workspace views for one sort.
struct Work {
    uint64_t *H[3];      // big-endian key bytes 0..7 (buffers 0 and 1; 2: the first-pass chunk pool)
    uint64_t *L[3];      // (key bytes 8..9) << 32 | record index
    uint32_t *idx;       // sorted record index per output position
    Ctl *ctl;
    Seg *segs[2];        // by level parity
    uint32_t *rep[2];    // histogram replicas [rep][kRepWords], by level parity
    uint32_t *tile_seg[2];
    unsigned long long *status;  // [tile][kRadix]: digit count, then offset among the bucket's tiles
    unsigned long long *cstat;   // [chunk][kRadix]: look-back words of the tile-offset scan
    Task *tasks;         // [kParts][max_tasks]
    Req *reqs;
    Hdr *hdr;
    uint64_t n;          // keys in the tuple space
    uint64_t part_end[kParts];  // output part k ends before tuple position part_end[k]; a task
                                // joins the part of its start (entries past nparts unused)
    uint32_t nparts;            // output parts in use (1..kParts)
    uint32_t max_seg, max_tiles, max_tasks, max_reqs, max_reps;
    // key bytes that take part in the order: extraction ANDs the tuple's key
    // words with these (all ones for the 10-byte key; a shorter key clears
    // the bytes past it, so records equal on it tie and keep index order)
    uint64_t kmask_h;
    uint32_t kmask_l;
    // fused first pass (null/zero otherwise): bucket d's chunk j is pool chunk
    // ctab[d * ctab_stride + j] - 1 (0: not yet allocated); a chunk holds
    // `tile` keys, so level-1 tile k of a bucket is its chunk k, and
    // tsrc[tile] names that chunk for the level-1 tile map
    uint32_t *ctab;
    uint32_t ctab_stride;
    uint32_t max_chunks;
    uint32_t *tsrc;
    uint8_t *rpool;      // kFirstRecords: records in pool order (max_chunks * tile records)
};

// Buffer a partition pass writes the children of a bucket held in buffer b to.
__host__ __device__ constexpr uint8_t next_buf(uint8_t b) { return b == 2 ? 1 : b ^ 1; }

// Workspace sizing for a tuple space of n keys and up to `reqs` requests.
struct Layout {
    uint64_t n;
    uint32_t max_seg, max_tiles, max_tasks, max_reqs, max_reps;
    size_t off_H0, off_H1, off_L0, off_L1, off_idx, off_ctl, off_seg0, off_seg1, off_rep0,
        off_rep1, off_ts0, off_ts1, off_status, off_cstat, off_tasks, off_reqs, off_hdr, total;
    // fused first pass (first_pass != kFirstSplit; all zero otherwise)
    uint32_t first_pass, max_chunks, ctab_stride;
    size_t off_PH, off_PL, off_ctab, off_tsrc, off_rpool;
};
// first_pass: the first pass the layout has room for (kFirstSplit: none of
// the pool regions).
Layout plan_layout(uint64_t n, uint32_t reqs, const Tune &t, uint32_t first_pass = kFirstSplit);
Work bind_layout(const Layout &L, void *base);

// Launch wrappers (sort_kernels.hip).  All return hipError_t of the launches.
// ev (optional): three events recorded after extraction, after the
// partition levels and after the local sorts.  nreq = tiles0 = 0 launches
// fixed grids that read every size from the device (for graph capture).
// Part of the launch sequence.  A sort may run in two parts: the first with
// the levels [0, gate) and a tail that stands down when level `gate` still has
// big buckets (reported through `flag`), the second with the remaining levels
// and the tail.
struct Stage {
    int lev_begin = 0, lev_end = kMaxLev;  // partition levels launched
    bool head = true;                      // k_init + k_extract first
    bool tuples_in = false;                // head: the tuples are already in buffer 0 (level-0
                                           // histogram pass instead of the extraction)
    uint32_t first = kFirstSplit;          // head: how level 0 is made (kFirstFused/kFirstRecords:
                                           // one fused pass, the levels start at 1)
    bool tail = true;                      // the local sorts after
    int gate = kMaxLev;                    // the tail exits if level `gate` has big buckets
    uint32_t *flag = nullptr;              // host-visible word: 1 if level `gate` has big buckets
};
hipError_t launch_sort_core(const Work &w, const Tune &t, uint32_t nreq, uint32_t tiles0,
                            hipStream_t s, int cus, hipEvent_t *ev = nullptr, const Stage &st = Stage{});
// The local sorts of the tasks of output part `part` alone (for a sort run
// with Stage::tail false and w.nparts > 1, one launch per part in order).
hipError_t launch_local_part(const Work &w, const Tune &t, hipStream_t s, int cus, int part);
hipError_t launch_gather_single(const uint8_t *rec, uint64_t n_rec, const uint32_t *idx, uint8_t *out,
                                uint64_t n, hipStream_t s, uint8_t *ties = nullptr, bool has_prev = false);
// The batch gather (sizes from the device header); exits like the tail of a
// Stage when level `gate` has big buckets.
hipError_t launch_gather_batch(const Work &w, hipStream_t s, int gate = kMaxLev);

}  // namespace ley
