// Flexible key sizes.  The method sorts records by a fixed-size key; Section 5
// names keys of any size as its next step, through a prefix sort combined with
// comparisons of the full keys where prefixes tie.  Here the key is the first
// K bytes of each 100-byte record, 1 <= K <= 100, in the same order as the
// 10-byte key (unsigned bytes, most significant first; equal keys keep input
// order).
//
// K <= 10: the prefix sort itself, with the tuple bytes past the key cleared
// at extraction, so records equal on the key tie and keep index order.
//
// K > 10: the prefix sort on bytes [0, 10), then rounds that resolve the runs
// of adjacent output records whose bytes [0, P) tie (P = 10, 16, 22, ...).  A
// round marks which neighbours tie, counts and numbers the runs (a scan of
// per-block counts), then writes for every record inside a run an entry: a
// key-pointer tuple whose 10-byte key is the run number (big-endian 32 bits)
// followed by key bytes [P, P + 6) of the record (bytes at or past K read as
// zero) and whose index is the entry's own number (entries are numbered in
// output-position order), written straight into the tuple buffers of a sort
// workspace.  One sort of the tuples (the in-HBM sort's partition and
// local-sort stages, no record gather) orders every run by its next six key
// bytes at once: the run number keeps runs apart and in place, and equal keys
// keep entry order, which is position order and so input order.  The rounds
// move record indices, not records: the q-th entry in sorted order takes the
// q-th position of the round, and each position's input record index is
// carried to the next round; after the last round one gather copies every
// tied position's record from the input.  A tie on [0, P + 6) implies a tie
// on [0, P), so a round looks only at the previous round's entries: in sorted
// order they describe the records now at consecutive positions of each run,
// and two neighbours tie exactly when their entries' keys agree.  The first
// round's ties come from the prefix sort itself: its record gather marks every
// output record whose key bytes 0..9 equal those of the record before it, so
// no round reads the records to find ties.  Rounds stop when no run is left
// or P reaches K.  The host reads the entry count of each round (one stream
// synchronisation per round).
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace ley {
namespace {

constexpr int kTB = 256;                // threads per block
constexpr int kTPer = 16;               // consecutive positions per thread (one 16-byte load of tie marks)
constexpr int kTSpan = kTB * kTPer;     // positions per block
constexpr int kRecWords = kRec / 4;     // dwords per record
constexpr uint32_t kWindow = 6;         // key bytes resolved per round

constexpr int kTWaves = kTB / 64;

// Exclusive sums of two per-thread counts over the block's threads in thread
// order (wave scans by lane shuffles, then the waves' totals through LDS);
// *ta, *tb get the block totals.  Whole block.
__device__ __forceinline__ void block_scan2(uint32_t a, uint32_t b, uint32_t *ea, uint32_t *eb, uint32_t *ta,
                                            uint32_t *tb) {
    __shared__ uint32_t wa[kTWaves], wb[kTWaves];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t ia = a, ib = b;  // inclusive within the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= (uint32_t)d) { ia += xa; ib += xb; }
    }
    if (lane == 63) { wa[w] = ia; wb[w] = ib; }
    __syncthreads();
    uint32_t pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
    for (int k = 0; k < kTWaves; k++) {
        pa += k < (int)w ? wa[k] : 0u;
        pb += k < (int)w ? wb[k] : 0u;
        sa += wa[k];
        sb += wb[k];
    }
    __syncthreads();
    *ea = pa + ia - a;
    *eb = pb + ib - b;
    *ta = sa;
    *tb = sb;
}

// Candidates c = 0..nc-1 of a round, in output-position order; P[c] = 1 if
// candidate c holds the record right after candidate c - 1's and ties with it
// on the key bytes sorted so far.  First round: candidate c is output position
// c and the prefix sort's record gather writes P.  Later rounds (this kernel):
// the candidates are the previous round's entries in sorted order, whose
// records now sit at consecutive positions within each run; c ties with c - 1
// when their entry keys (run number and window bytes: SKh, SKl in sorted
// order) agree.
__global__ __launch_bounds__(kTB) void k_tie_eq(const uint64_t *SKh, const uint32_t *SKl, uint64_t nc, uint8_t *P) {
    const uint64_t base = (uint64_t)blockIdx.x * kTSpan;
    for (int u = 0; u < kTPer; u++) {
        const uint64_t c = base + (uint64_t)u * kTB + threadIdx.x;
        if (c >= nc) continue;
        const bool eq = c > 0 && SKh[c] == SKh[c - 1] && SKl[c] == SKl[c - 1];
        P[c] = eq ? 1 : 0;
    }
}

// The tie flags of the thread's kTPer candidates c0 + k (c0 = block base +
// kTPer * thread): bit k of *in_run when candidate c0 + k lies inside a run of
// at least two (it ties with a neighbour), of *starts when such a run starts
// there.  One 16-byte load of the marks (P is 16-byte aligned) and one byte
// for the next thread's first mark.
__device__ __forceinline__ void tie_bits(const uint8_t *P, uint64_t nc, uint64_t c0, uint32_t *in_run,
                                         uint32_t *starts) {
    uint32_t eq = 0;  // bit k: candidate c0 + k ties with the candidate before it
    if (c0 + kTPer <= nc) {
        const uint4 v = *reinterpret_cast<const uint4 *>(P + c0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < kTPer; k++) eq |= (((w[k >> 2] >> (8 * (k & 3))) & 0xFFu) != 0u ? 1u : 0u) << k;
    } else {
        for (int k = 0; k < kTPer; k++)
            if (c0 + k < nc && P[c0 + k] != 0) eq |= 1u << k;
    }
    if (c0 == 0) eq &= ~1u;  // the first candidate has no predecessor
    const uint32_t next = (c0 + kTPer < nc && P[c0 + kTPer] != 0) ? 1u : 0u;
    const uint32_t eq_next = (eq >> 1) | (next << (kTPer - 1));  // bit k: c0 + k ties with c0 + k + 1
    const uint32_t valid = c0 >= nc ? 0u : (nc - c0 >= (uint64_t)kTPer ? 0xFFFFu : ((1u << (nc - c0)) - 1u));
    *in_run = (eq | eq_next) & valid;
    *starts = eq_next & ~eq & valid;
}

// Per block of kTSpan candidates: candidates inside runs and run starts.
__global__ __launch_bounds__(kTB) void k_tie_count(const uint8_t *P, uint64_t nc, uint32_t *cnt_in,
                                                   uint32_t *cnt_start) {
    const uint64_t c0 = (uint64_t)blockIdx.x * kTSpan + (uint64_t)threadIdx.x * kTPer;
    uint32_t r, st;
    tie_bits(P, nc, c0, &r, &st);
    uint32_t ei, es, ti, ts;
    block_scan2((uint32_t)__popc(r), (uint32_t)__popc(st), &ei, &es, &ti, &ts);
    if (threadIdx.x == 0) {
        cnt_in[blockIdx.x] = ti;
        cnt_start[blockIdx.x] = ts;
    }
}

// Exclusive scans of both per-block counts, in three launches: per group of
// kSG counts its sums (up), the groups' offsets (top, one block), then every
// count's offset (down); totals[0] = positions inside runs, totals[1] = runs.
constexpr int kSB = 1024;            // threads per scan block
constexpr int kSPer = 4;             // counts per thread
constexpr int kSG = kSB * kSPer;     // counts per group

__device__ __forceinline__ void load_counts(const uint32_t *ci, const uint32_t *cs, uint64_t nb, uint64_t b0,
                                            uint32_t *vi, uint32_t *vs) {
#pragma unroll
    for (int k = 0; k < kSPer; k++) {
        vi[k] = b0 + k < nb ? ci[b0 + k] : 0u;
        vs[k] = b0 + k < nb ? cs[b0 + k] : 0u;
    }
}

// Exclusive scan of a uint32 pair over the kSB threads of a block (wave
// shuffles, then the wave totals through LDS).  Whole block.
__device__ __forceinline__ void scan_block_pair(uint32_t a, uint32_t b, uint32_t *ea, uint32_t *eb, uint32_t *ta,
                                                uint32_t *tb) {
    constexpr int W = kSB / 64;
    __shared__ uint32_t wa[W], wb[W];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t ia = a, ib = b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t xa = __shfl_up(ia, d), xb = __shfl_up(ib, d);
        if (lane >= (uint32_t)d) { ia += xa; ib += xb; }
    }
    if (lane == 63) { wa[w] = ia; wb[w] = ib; }
    __syncthreads();
    uint32_t pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
    for (int k = 0; k < W; k++) {
        pa += k < (int)w ? wa[k] : 0u;
        pb += k < (int)w ? wb[k] : 0u;
        sa += wa[k];
        sb += wb[k];
    }
    __syncthreads();
    *ea = pa + ia - a;
    *eb = pb + ib - b;
    *ta = sa;
    *tb = sb;
}

__global__ __launch_bounds__(kSB) void k_tie_scan_up(const uint32_t *cnt_in, const uint32_t *cnt_start, uint64_t nb,
                                                     uint64_t *grp_in, uint64_t *grp_start) {
    uint32_t vi[kSPer], vs[kSPer];
    load_counts(cnt_in, cnt_start, nb, (uint64_t)blockIdx.x * kSG + (uint64_t)threadIdx.x * kSPer, vi, vs);
    uint32_t si = 0, ss = 0;
#pragma unroll
    for (int k = 0; k < kSPer; k++) { si += vi[k]; ss += vs[k]; }
    uint32_t ei, es, ti, ts;
    scan_block_pair(si, ss, &ei, &es, &ti, &ts);
    if (threadIdx.x == 0) {
        grp_in[blockIdx.x] = ti;
        grp_start[blockIdx.x] = ts;
    }
}

// One block: exclusive scan of the ng <= kSB group sums in place, and the totals.
__global__ __launch_bounds__(kSB) void k_tie_scan_top(uint64_t *grp_in, uint64_t *grp_start, uint64_t ng,
                                                      uint64_t *totals) {
    __shared__ uint64_t si[kSB], ss[kSB];
    const uint32_t t = threadIdx.x;
    const uint64_t vi = t < ng ? grp_in[t] : 0ull, vs = t < ng ? grp_start[t] : 0ull;
    si[t] = vi;
    ss[t] = vs;
    __syncthreads();
    for (uint32_t off = 1; off < (uint32_t)kSB; off <<= 1) {
        const uint64_t ai = t >= off ? si[t - off] : 0ull, as = t >= off ? ss[t - off] : 0ull;
        __syncthreads();
        si[t] += ai;
        ss[t] += as;
        __syncthreads();
    }
    if (t < ng) {
        grp_in[t] = si[t] - vi;
        grp_start[t] = ss[t] - vs;
    }
    if (t == kSB - 1) {
        totals[0] = si[t];
        totals[1] = ss[t];
    }
}

__global__ __launch_bounds__(kSB) void k_tie_scan_down(const uint32_t *cnt_in, const uint32_t *cnt_start, uint64_t nb,
                                                       const uint64_t *grp_in, const uint64_t *grp_start,
                                                       uint64_t *off_in, uint64_t *off_start) {
    const uint64_t b0 = (uint64_t)blockIdx.x * kSG + (uint64_t)threadIdx.x * kSPer;
    uint32_t vi[kSPer], vs[kSPer];
    load_counts(cnt_in, cnt_start, nb, b0, vi, vs);
    uint32_t si = 0, ss = 0;
#pragma unroll
    for (int k = 0; k < kSPer; k++) { si += vi[k]; ss += vs[k]; }
    uint32_t ei, es, ti, ts;
    scan_block_pair(si, ss, &ei, &es, &ti, &ts);
    uint64_t ci = grp_in[blockIdx.x] + ei, cs = grp_start[blockIdx.x] + es;
#pragma unroll
    for (int k = 0; k < kSPer; k++) {
        if (b0 + k < nb) {
            off_in[b0 + k] = ci;
            off_start[b0 + k] = cs;
        }
        ci += vi[k];
        cs += vs[k];
    }
}

// Entries of the round: for candidate c inside a run, entry t (its rank among
// such candidates) gets the tuple key = run number (big-endian) + key bytes
// [p, p + 6) of its record, masked to the key, with index t (TH[t], TL[t]: the
// sort's tuple words), the same key in Kh[t], Kl[t] (kept for the next round's
// tie marks), its record's input index srcx[t] and its first-round entry
// number e0x[t].  First round (src_prev null): candidate c is output position
// c, holding input record pidx[c] (the prefix sort's order), whose bytes are
// read from the sorted output A; e0x[t] = t and slot0[t] = c.  Later rounds:
// candidate c is the previous round's sorted entry c, holding input record
// src_prev[c] (its bytes read from the input) at the position of first-round
// entry e0_prev[c].  An index out of range, which only a failed sort could
// leave, is not read: it sets *err.
__global__ __launch_bounds__(kTB) void k_tie_emit(const uint8_t *A, const uint8_t *in, uint64_t n,
                                                  const uint8_t *P, uint64_t nc, const uint32_t *pidx,
                                                  const uint32_t *src_prev, const uint32_t *e0_prev, uint32_t p,
                                                  uint32_t key_bytes, const uint64_t *off_in,
                                                  const uint64_t *off_start, uint64_t *TH, uint64_t *TL,
                                                  uint64_t *Kh, uint32_t *Kl, uint32_t *srcx, uint32_t *e0x,
                                                  uint64_t *slot0, uint32_t *err) {
    // the block's entries are the contiguous range [off_in[block], + total):
    // their candidates are listed in LDS first, then each thread takes every
    // kTB-th entry, so the entry stores are contiguous across the block
    __shared__ uint16_t s_c[kTSpan];    // candidate offset in the block
    __shared__ uint16_t s_run[kTSpan];  // runs started in the block up to it (0: a run from an earlier block)
    const uint64_t cb = (uint64_t)blockIdx.x * kTSpan;
    const uint32_t c_off = threadIdx.x * kTPer;
    uint32_t r, st;
    tie_bits(P, nc, cb + c_off, &r, &st);
    uint32_t ei, es, ti, ts;
    block_scan2((uint32_t)__popc(r), (uint32_t)__popc(st), &ei, &es, &ti, &ts);
    for (uint32_t j = ei; r; j++) {
        const int k = __builtin_ctz(r);
        r &= r - 1;
        s_c[j] = (uint16_t)(c_off + (uint32_t)k);
        s_run[j] = (uint16_t)(es + (uint32_t)__popc(st & ((2u << k) - 1u)));
    }
    __syncthreads();
    const uint64_t t0 = off_in[blockIdx.x], runs0 = off_start[blockIdx.x];
    // key bytes past the key read as zero: byte mask of the six window bytes
    uint32_t keep = 0;
    for (uint32_t k = 0; k < kWindow; k++)
        if (p + k < key_bytes) keep |= 1u << k;
    for (uint32_t j = threadIdx.x; j < ti; j += kTB) {
        const uint64_t c = cb + s_c[j];
        const uint64_t t = t0 + j;
        // the run holding c began at the latest start at or before c
        const uint32_t run = (uint32_t)(runs0 + s_run[j] - 1u);
        const uint32_t src = src_prev ? src_prev[c] : pidx[c];
        const uint32_t e0 = src_prev ? e0_prev[c] : (uint32_t)t;
        const bool ok = src < n;
        if (!ok) atomicOr(err, 1u << 17);
        // the window's six bytes from two aligned dwords (the record offset and
        // p are even; the two dwords end inside the record for every p < 100)
        uint32_t b6[kWindow] = {0, 0, 0, 0, 0, 0};
        if (ok) {
            const uint64_t o = (src_prev ? (uint64_t)src : c) * kRec + p;
            const uint32_t *w = reinterpret_cast<const uint32_t *>(src_prev ? in : A) + (o >> 2);
            const uint64_t v = ((uint64_t)w[1] << 32) | w[0];
            const uint32_t sh = (uint32_t)(o & 3u) * 8u;
#pragma unroll
            for (uint32_t q = 0; q < kWindow; q++) b6[q] = (keep >> q & 1u) ? (uint32_t)(v >> (sh + 8u * q)) & 0xFFu : 0u;
        }
        const uint64_t h = ((uint64_t)run << 32) | (b6[0] << 24) | (b6[1] << 16) | (b6[2] << 8) | b6[3];
        const uint32_t wl = (b6[4] << 8) | b6[5];
        TH[t] = h;
        TL[t] = ((uint64_t)wl << 32) | (uint32_t)t;
        Kh[t] = h;
        Kl[t] = wl;
        srcx[t] = src;
        e0x[t] = e0;
        if (!src_prev) slot0[t] = c;
    }
}

// After the entry sort (idx[q] = the entry number t in sorted position q):
// the entry's key in SKh[q], SKl[q] (sorted order, for the next round's tie
// marks) and its record's input index in src_s[q]; the q-th sorted entry takes
// the position of entry q, which belongs to first-round entry e0x[q], so
// final_src[e0x[q]] = that input index.  An entry number or first-round entry
// out of range, which only a failed entry sort could leave, sets *err.
__global__ __launch_bounds__(kTB) void k_tie_perm(const uint32_t *idx, uint64_t m, const uint64_t *Kh,
                                                  const uint32_t *Kl, const uint32_t *srcx, const uint32_t *e0x,
                                                  uint64_t m0, uint64_t *SKh, uint32_t *SKl, uint32_t *src_s,
                                                  uint32_t *final_src, uint32_t *err) {
    const uint64_t q = (uint64_t)blockIdx.x * kTB + threadIdx.x;
    if (q >= m) return;
    const uint32_t t = idx[q];
    if (t >= m) { atomicOr(err, 1u << 16); return; }
    const uint32_t src = srcx[t];
    SKh[q] = Kh[t];
    SKl[q] = Kl[t];
    src_s[q] = src;
    const uint32_t e = e0x[q];
    if (e < m0) final_src[e] = src;
    else atomicOr(err, 1u << 16);
}

// The tied positions' records, once after the last round: A[slot0[t]] =
// in[final_src[t]] for the first-round entries t of a block of kTB (positions
// through LDS, then a dword per thread, every load in flight before the
// stores).  A position or index out of range sets *err and is skipped.
__global__ __launch_bounds__(kTB) void k_tie_final(const uint32_t *in, uint64_t n, const uint64_t *slot0,
                                                   const uint32_t *final_src, uint64_t m0, uint32_t *A,
                                                   uint32_t *err) {
    __shared__ uint64_t sd[kTB];
    __shared__ uint32_t ss[kTB];
    const uint64_t t0 = (uint64_t)blockIdx.x * kTB;
    const uint32_t nr = (uint32_t)min<uint64_t>(kTB, m0 - t0);
    if (threadIdx.x < nr) {
        const uint64_t d = slot0[t0 + threadIdx.x];
        const uint32_t sidx = final_src[t0 + threadIdx.x];
        const bool ok = d < n && sidx < n;
        if (!ok) atomicOr(err, 1u << 18);
        sd[threadIdx.x] = ok ? d : ~0ull;
        ss[threadIdx.x] = sidx;
    }
    __syncthreads();
    uint32_t v[kRecWords];
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u, r = g / kRecWords, d = g - r * kRecWords;
        v[u] = 0;
        if (r < nr && sd[r] != ~0ull) v[u] = in[(uint64_t)ss[r] * kRecWords + d];
    }
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u, r = g / kRecWords, d = g - r * kRecWords;
        if (r < nr && sd[r] != ~0ull) A[sd[r] * kRecWords + d] = v[u];
    }
}

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// Scratch of the tie rounds, from the stream's pooled slot 0 (kept between
// calls): the tie marks (n bytes), the per-block counts and offsets of the
// run numbering, and the totals + error word.
struct RoundTables {
    uint8_t *P;
    uint32_t *cnt_in, *cnt_start;
    uint64_t *off_in, *off_start, *grp, *totals;
};

size_t tables_bytes(uint64_t n) {
    const uint64_t nb = (n + kTSpan - 1) / kTSpan;
    return a256(n) + 2 * a256(nb * 4) + 2 * a256(nb * 8) + a256(2 * kSB * 8) + 256;
}

RoundTables bind_tables(void *base, uint64_t n) {
    const uint64_t nb = (n + kTSpan - 1) / kTSpan;
    char *b = static_cast<char *>(base);
    RoundTables r;
    r.P = reinterpret_cast<uint8_t *>(b); b += a256(n);
    r.cnt_in = reinterpret_cast<uint32_t *>(b); b += a256(nb * 4);
    r.cnt_start = reinterpret_cast<uint32_t *>(b); b += a256(nb * 4);
    r.off_in = reinterpret_cast<uint64_t *>(b); b += a256(nb * 8);
    r.off_start = reinterpret_cast<uint64_t *>(b); b += a256(nb * 8);
    r.grp = reinterpret_cast<uint64_t *>(b); b += a256(2 * kSB * 8);  // group sums of the count scan
    r.totals = reinterpret_cast<uint64_t *>(b);  // tie count, run count, error word
    return r;
}

// Rounds over the tie runs of the prefix-sorted records in A (n records,
// sorted from the input `in` on stream s, whose pooled workspace still holds
// that sort's order); tb.P (n bytes) holds the first round's tie marks and is
// reused by later rounds.  The entries live in the stream's pooled slot 1.
int resolve_ties(const uint32_t *in, uint32_t *A, uint64_t n, uint32_t key_bytes, hipStream_t s, const Tune &t,
                 const RoundTables &tb) {
    int rc;
    uint8_t *P = tb.P;
    uint32_t *cnt_in = tb.cnt_in, *cnt_start = tb.cnt_start;
    uint64_t *off_in = tb.off_in, *off_start = tb.off_start;
    uint64_t *grp = tb.grp, *totals = tb.totals;
    // error word next to the totals: the sorts' device-side guard words
    // (capacity guards, bounded waits) and the rounds' index checks
    uint32_t *err = reinterpret_cast<uint32_t *>(totals + 2);
    hipError_t e0 = hipMemsetAsync(err, 0, 4, s);
    if (e0 != hipSuccess) return hip_fail(e0, "leyenda_sort_keyed: error word");
    if ((rc = guard_or_pooled(s, err))) return rc;  // the prefix sort
    const uint32_t *pidx = pooled_sort_idx(s, n);   // its input index per output position
    if (!pidx) return fail(LEYENDA_EINTERNAL, "leyenda_sort_keyed: the prefix sort's order is not in its workspace");
    // scratch of the rounds, sized by the first round's count (the largest):
    // the entry sort's workspace; the entries' keys (Kh, Kl) and in sorted
    // order (SKh, SKl); their records' input indices (srcx) and in sorted order
    // (src_s); their first-round entry numbers by round parity (e0x); per
    // first-round entry its position (slot0) and final input index (final_src)
    char *ws = nullptr;
    uint64_t *Kh = nullptr, *SKh = nullptr, *slot0 = nullptr;
    uint32_t *Kl = nullptr, *SKl = nullptr, *srcx = nullptr, *src_s = nullptr, *final_src = nullptr;
    uint32_t *e0x[2] = {nullptr, nullptr};
    uint64_t cap = 0, nc = n;
    int r = 0;
    for (uint32_t p = kKeyBytes; p < key_bytes; p += kWindow, r++) {
        const uint64_t nb = (nc + kTSpan - 1) / kTSpan;
        if (r) k_tie_eq<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(SKh, SKl, nc, P);
        const uint64_t ng = (nb + kSG - 1) / kSG;
        k_tie_count<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(P, nc, cnt_in, cnt_start);
        k_tie_scan_up<<<dim3((uint32_t)ng), dim3(kSB), 0, s>>>(cnt_in, cnt_start, nb, grp, grp + kSB);
        k_tie_scan_top<<<dim3(1), dim3(kSB), 0, s>>>(grp, grp + kSB, ng, totals);
        k_tie_scan_down<<<dim3((uint32_t)ng), dim3(kSB), 0, s>>>(cnt_in, cnt_start, nb, grp, grp + kSB, off_in,
                                                                  off_start);
        uint64_t h[3] = {0, 0, 0};  // tie count, run count, error word
        hipError_t e = hipMemcpyAsync(h, totals, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: tie count");
        if ((uint32_t)h[2]) return fail(LEYENDA_EINTERNAL, "leyenda_sort_keyed: device-side guard 0x%x", (uint32_t)h[2]);
        const uint64_t m = h[0];
        if (m == 0) break;
        if (m > nc || h[1] > m / 2) return fail(LEYENDA_EHIP, "leyenda_sort_keyed: inconsistent tie count");
        if (!ws) {  // the first round has the most entries: later rounds reuse its room
            cap = m;
            const size_t wsb = a256(plan_layout(cap, 1, t).total);
            void *base = nullptr;
            if ((rc = get_aux(s, 1, wsb + 3 * a256(cap * 8) + 7 * a256(cap * 4), &base))) return rc;
            char *b = static_cast<char *>(base);
            ws = b; b += wsb;
            Kh = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            SKh = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            slot0 = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            Kl = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            SKl = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            srcx = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            src_s = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            final_src = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            e0x[0] = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            e0x[1] = reinterpret_cast<uint32_t *>(b);
        }
        // the entries go straight into the tuple buffers of a workspace laid out for m tuples
        const Layout Lm = plan_layout(m, 1, t);
        uint64_t *TH = reinterpret_cast<uint64_t *>(ws + Lm.off_H0);
        uint64_t *TL = reinterpret_cast<uint64_t *>(ws + Lm.off_L0);
        const uint32_t *idx = reinterpret_cast<const uint32_t *>(ws + Lm.off_idx);
        k_tie_emit<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(
            reinterpret_cast<const uint8_t *>(A), reinterpret_cast<const uint8_t *>(in), n, P, nc, pidx,
            r ? src_s : nullptr, r ? e0x[(r - 1) & 1] : nullptr, p, key_bytes, off_in, off_start, TH, TL, Kh, Kl,
            srcx, e0x[r & 1], slot0, err);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: entries");
        if ((rc = sort_tuples_ws(m, s, t, ws))) return rc;
        if ((e = launch_guard_or(ws, m, t, err, s)) != hipSuccess) return hip_fail(e, "guard kernel");
        const uint64_t blocks = (m + kTB - 1) / kTB;
        k_tie_perm<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(idx, m, Kh, Kl, srcx, e0x[r & 1], cap, SKh, SKl,
                                                                 src_s, final_src, err);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: order");
        nc = m;  // the next round looks only inside these runs
    }
    if (cap) {  // the tied positions' records, from the input
        const uint64_t blocks = (cap + kTB - 1) / kTB;
        k_tie_final<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(in, n, slot0, final_src, cap, A, err);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: records");
    }
    uint32_t eh = 0;
    hipError_t e = hipMemcpyAsync(&eh, err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_keyed");
    if (eh) return fail(LEYENDA_EINTERNAL, "leyenda_sort_keyed: device-side guard 0x%x", eh);
    return LEYENDA_OK;
}

}  // namespace
}  // namespace ley

using namespace ley;

extern "C" int leyenda_sort_keyed(const void *records_dev, uint64_t n, uint32_t key_bytes, void *out_dev,
                                  void *stream) {
    if (key_bytes < 1 || key_bytes > (uint32_t)kRec)
        return fail(LEYENDA_EINVAL, "leyenda_sort_keyed: key_bytes %u outside 1..100", key_bytes);
    if (n == 0) return LEYENDA_OK;
    int rc = check_records(records_dev, out_dev, n, "leyenda_sort_keyed");
    if (rc) return rc;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const Tune t = tune_of(current_params());
    if (key_bytes <= kKeyBytes || n < 2)
        return sort_device(records_dev, n, out_dev, s, t, key_bytes < kKeyBytes ? key_bytes : kKeyBytes);
    void *tab = nullptr;  // tie marks of the prefix sort's gather, then the rounds' tables
    if ((rc = get_aux(s, 0, tables_bytes(n), &tab))) return rc;
    const RoundTables tb = bind_tables(tab, n);
    if ((rc = sort_device(records_dev, n, out_dev, s, t, kKeyBytes, tb.P))) return rc;
    return resolve_ties(static_cast<const uint32_t *>(records_dev), static_cast<uint32_t *>(out_dev), n, key_bytes, s,
                        t, tb);
}
