// Device kernels of the in-HBM record sort (gfx950, wave64).
//
// The schedule follows Algorithm 1 (Adaptive Parallel MSD Radix Sort,
// Section 3.1) on the key-pointer tuples of Section 3.2:
//
//   k_init      request table -> level-0 buckets and tile map
//   k_extract   (key, index) tuple per record + first-digit histogram and key
//               masks (AlphaSort-style key-pointer extraction, Section 3.2)
//   k_hist      per level >= 1: digit histograms and key masks of big buckets
//   k_plan      per level: bucket policy of Algorithm 1 for every big bucket,
//               then each tile's per-digit offset among its bucket's tiles
//               (from the tile counts of the histogram pass)
//   k_scatter   per level: stable device-wide partition of big buckets by one
//               digit (ParallelRadixSort, "cache aware scattering": tiles are
//               ranked and staged in LDS, then written as runs)
//   k_local     per small bucket, in one workgroup's LDS: radix partition of
//               its (key, index) tuples on the first varying tuple digit
//               (SingleThreadRadixSort), recursion on sub-buckets above the
//               tiny threshold, and a comparison sort of tiny sub-buckets
//               (ComparisonSort)
//   k_gather    record scatter by the sorted tuples (Section 3.2):
//               out[j] = in[idx[j]]
//
// A large single sort files its local-sort tasks under output parts (by the
// task's start) and launches the local sorts once per part, so each part's
// gather can start on another stream while later parts are sorted.
//
// Tuples are kept as two arrays (struct of arrays): H = key bytes 0..7 as a
// big-endian u64, L = key bytes 8..9 (big-endian) << 32 | record index.
// (H, L) compared as an unsigned 128-bit number is the key order with ties
// broken by record index, i.e. exactly the stable order.
#include "common.h"

namespace ley {

// ---------------------------------------------------------------------------
// small helpers

// Bits [pos, pos + bits) of the 80-bit key (most significant bit first); bits
// past the key read as zero.  pos < 80, kMinRB <= bits <= kRB.
__device__ __forceinline__ uint32_t digit_at(uint64_t h, uint64_t l, uint32_t pos, uint32_t bits) {
    const uint64_t k2 = (l >> 32) << 48;
    uint64_t w;
    if (pos == 0) w = h;
    else if (pos < 64) w = (h << pos) | (k2 >> (64 - pos));
    else w = k2 << (pos - 64);
    return (uint32_t)(w >> (64 - bits));
}

__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_agent32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stable rank of digit d among the earlier lanes of this wave and the earlier
// items of this wave (counted in cnt[]), over lanes with valid == true.  It is
// split in two so that the counter updates of all of a thread's items issue
// back to back instead of one LDS round trip per item:
// rank_issue leaves in `old` (in one lane per digit) the wave counter's value
// before this item's keys were added, and packs the digit, the lane holding
// `old` and the count of lower lanes with the same digit into `pk`;
// rank_finish turns the pair into the rank.  LDS executes one wave's
// operations in order, so items issued in key order rank in key order.
// The lanes that share the digit come from one ballot per digit bit: a lane
// accumulates, per 32-lane half, the lanes whose bit differs from its own
// (n |= ballot ^ own-bit-mask, one three-input bit operation per half).
__device__ __forceinline__ void rank_issue(uint32_t d, bool valid, uint32_t *cnt, uint32_t &old, uint32_t &pk) {
    const uint64_t vb = __ballot(valid);
    uint32_t nlo = ~(uint32_t)vb, nhi = ~(uint32_t)(vb >> 32);  // lanes that differ (or are idle)
#pragma unroll
    for (int b = 0; b < kRB; b++) {
        const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);  // 0 or all ones
        const uint64_t bal = __ballot(m != 0u);
        nlo = __builtin_amdgcn_bitop3_b32(nlo, (uint32_t)bal, m, 0xF6);  // nlo | (bal ^ m)
        nhi = __builtin_amdgcn_bitop3_b32(nhi, (uint32_t)(bal >> 32), m, 0xF6);
    }
    const uint32_t plo = ~nlo, phi = ~nhi;  // peers: valid lanes with the same digit
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
    // an idle lane has no peers; it reads lane 0
    const uint32_t leader = (uint32_t)__builtin_ctzll(((uint64_t)phi << 32) | plo | (uint64_t)!valid);
    old = 0;
    if (valid && below == 0) old = atomicAdd(&cnt[d], (uint32_t)(__popc(plo) + __popc(phi)));
    pk = d | (leader << 8) | (below << 16);
}
__device__ __forceinline__ uint32_t rank_finish(uint32_t old, uint32_t pk) {
    return (uint32_t)__shfl((int)old, (int)((pk >> 8) & 63u)) + (pk >> 16);
}

// Wave-wide OR / AND (the device library's cross-lane reductions, per half).
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    return ((uint64_t)__ockl_wfred_or_u32((uint32_t)(v >> 32)) << 32) | __ockl_wfred_or_u32((uint32_t)v);
}
__device__ __forceinline__ uint64_t wave_and64(uint64_t v) {
    return ((uint64_t)__ockl_wfred_and_u32((uint32_t)(v >> 32)) << 32) | __ockl_wfred_and_u32((uint32_t)v);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts: a
// Hillis-Steele scan inside each row of 16 lanes, then the last lane of row 0
// is added to row 1 (and of row 2 to row 3), then lane 31 to rows 2 and 3.
// Lanes a shift would read from outside the row add zero.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowShr + 1, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowShr + 2, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowShr + 4, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowShr + 8, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowBcast15, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kRowBcast31, 0xc, 0xf, false);
    return x;
}

// Raw buffer loads: lanes whose offset lies past the end of the resource read
// zero, so loads are issued without branches (the wait counts stay exact and
// no lane can touch memory outside the range).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

// A value every lane holds alike, moved to scalar registers (buffer resources
// must be uniform; the compiler cannot always prove it).
__device__ __forceinline__ uint32_t ufirst(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Dwords in device (global) memory, for pointers read from device tables,
// whose address space the compiler cannot infer (it would emit flat accesses).
typedef const __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint32_t gu32w;

// Exclusive prefix sum over the workgroup's threads (one value each; NW waves).
template <int NW = kWaves>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tmp /*[NW]*/) {
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t x = wave_incl_scan(v);
    if (lane == 63) tmp[w] = x;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int k = 0; k < NW; k++) pre += (k < (int)w) ? tmp[k] : 0u;
    __syncthreads();
    return pre + x - v;
}

constexpr uint32_t kSpinLimit = 1u << 24;

// A segment read back from a device table is inside the tuple space and owns
// the tile that points at it (defence against a fired capacity guard).
__device__ __forceinline__ bool seg_ok(const Work &w, const Seg &sg, uint32_t tile) {
    return sg.count > 0 && sg.start + sg.count <= w.n && tile >= sg.first_tile &&
           tile - sg.first_tile < sg.ntiles && sg.buf <= 2 && sg.nrep >= 1 && sg.nrep <= kMaxRep &&
           (uint64_t)sg.rep_first + sg.nrep <= w.max_reps;
}

// First tuple of tile `tile` of bucket sg (tile k of the bucket starts at key
// k * tile): in buffer 0 or 1 the bucket is contiguous; in the first-pass pool
// (buffer 2) tile k is the bucket's chunk k, named by the tile map tsrc.
// ok false (nothing may be read) if the chunk lies outside the pool.
__device__ __forceinline__ uint64_t tile_src(const Work &w, const Seg &sg, uint32_t tile, uint32_t tsize, bool &ok) {
    ok = true;
    if (sg.buf != 2) return sg.start + (uint64_t)(tile - sg.first_tile) * tsize;
    const uint32_t c = w.tsrc[tile];
    ok = w.tsrc != nullptr && c < w.max_chunks;
    return (uint64_t)c * tsize;
}

// ---------------------------------------------------------------------------
// planning of one big bucket (Algorithm 1: big buckets recurse on the next
// digit, small ones go to the task queue, tiny ones are sorted by comparison
// inside the local sort).  Called by all threads of a workgroup.

// Output part of a task starting at tuple position `start`.
__device__ __forceinline__ uint32_t part_of(const Work &w, uint64_t start) {
    uint32_t p = 0;
    while (p + 1 < w.nparts && start >= w.part_end[p]) p++;
    return p;
}

__device__ void emit_task(const Work &w, uint64_t start, uint32_t count, uint8_t buf, uint8_t flags,
                          uint16_t req) {
    const uint32_t p = part_of(w, start);
    const uint32_t j = atomicAdd(&w.ctl->ntask[p], 1u);
    if (j >= w.max_tasks) { atomicOr(&w.ctl->guard, 1u); return; }
    Task t;
    t.start = start; t.count = count; t.buf = buf; t.flags = flags; t.req = req;
    w.tasks[(size_t)p * w.max_tasks + j] = t;
}

// A range whose keys are all equal is already in final (index) order; it is
// cut into local-capacity chunks so each task stays bounded.  Consecutive
// chunks of one output part take their slots with one atomic.
__device__ void emit_sorted(const Work &w, uint64_t start, uint64_t count, uint8_t buf, uint16_t req) {
    const uint64_t nch = (count + kLocalCap - 1) / kLocalCap;
    for (uint64_t k0 = 0; k0 < nch;) {
        const uint32_t p = part_of(w, start + k0 * kLocalCap);
        // first chunk that starts in a later part
        const uint64_t k1 = p + 1 >= w.nparts
                                ? nch
                                : min(nch, (w.part_end[p] - start + kLocalCap - 1) / kLocalCap);
        const uint32_t j0 = atomicAdd(&w.ctl->ntask[p], (uint32_t)(k1 - k0));
        if ((uint64_t)j0 + (k1 - k0) > w.max_tasks) { atomicOr(&w.ctl->guard, 2u); return; }
        for (uint64_t k = k0; k < k1; k++) {
            Task t;
            t.start = start + k * kLocalCap;
            t.count = (uint32_t)min<uint64_t>(kLocalCap, count - k * kLocalCap);
            t.buf = buf; t.flags = kTaskSorted; t.req = req;
            w.tasks[(size_t)p * w.max_tasks + j0 + (k - k0)] = t;
        }
        k0 = k1;
    }
}

__device__ void new_segment(const Work &w, const Tune &tu, int lev, uint64_t start, uint32_t count,
                            uint32_t pos, uint8_t buf, uint16_t req) {
    const uint32_t s = atomicAdd(&w.ctl->nseg[lev], 1u);
    const uint32_t nt = (count + tu.tile - 1) / tu.tile;
    const uint32_t nr = min(nt, (uint32_t)kMaxRep);
    const uint32_t ft = atomicAdd(&w.ctl->ntiles[lev], nt);
    const uint32_t rf = atomicAdd(&w.ctl->rep_ctr[lev], nr);
    if (s >= w.max_seg || (uint64_t)ft + nt > w.max_tiles || (uint64_t)rf + nr > w.max_reps) {
        atomicOr(&w.ctl->guard, 4u);
        if (s < w.max_seg) {  // leave a harmless entry: no tiles, nothing to zero
            Seg g{};
            g.spos = kNoScatter;
            w.segs[lev & 1][s] = g;
        }
        return;
    }
    Seg g;
    g.start = start; g.count = count; g.first_tile = ft; g.ntiles = nt; g.rep_first = rf; g.nrep = (uint8_t)nr;
    g.pos = (uint16_t)pos; g.spos = kNoScatter; g.buf = buf; g.req = req;
    w.segs[lev & 1][s] = g;
}

// new_segment for every thread of the workgroup with `need` set, with one
// atomic per counter for the whole workgroup (the counters of a level are
// shared by all buckets, so per-child atomics would serialize).  Whole
// workgroup.
__device__ void new_segments_block(const Work &w, const Tune &tu, int lev, bool need, uint64_t start,
                                   uint32_t count, uint32_t pos, uint8_t buf, uint16_t req) {
    __shared__ uint32_t ns_tmp[kWaves];
    __shared__ uint32_t ns_tot[3], ns_base[3];
    const uint32_t nt = need ? (count + tu.tile - 1) / tu.tile : 0u;
    const uint32_t nr = min(nt, (uint32_t)kMaxRep);
    const uint32_t es = block_excl_scan(need ? 1u : 0u, ns_tmp);
    const uint32_t et = block_excl_scan(nt, ns_tmp);
    const uint32_t er = block_excl_scan(nr, ns_tmp);
    if (threadIdx.x == kWG - 1) {
        ns_tot[0] = es + (need ? 1u : 0u);
        ns_tot[1] = et + nt;
        ns_tot[2] = er + nr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ns_base[0] = ns_tot[0] ? atomicAdd(&w.ctl->nseg[lev], ns_tot[0]) : 0u;
        ns_base[1] = ns_tot[1] ? atomicAdd(&w.ctl->ntiles[lev], ns_tot[1]) : 0u;
        ns_base[2] = ns_tot[2] ? atomicAdd(&w.ctl->rep_ctr[lev], ns_tot[2]) : 0u;
    }
    __syncthreads();
    if (need) {
        const uint32_t s = ns_base[0] + es, ft = ns_base[1] + et, rf = ns_base[2] + er;
        if (s >= w.max_seg || (uint64_t)ft + nt > w.max_tiles || (uint64_t)rf + nr > w.max_reps) {
            atomicOr(&w.ctl->guard, 4u);
            if (s < w.max_seg) {  // leave a harmless entry: no tiles, nothing to zero
                Seg g{};
                g.spos = kNoScatter;
                w.segs[lev & 1][s] = g;
            }
        } else {
            Seg g;
            g.start = start; g.count = count; g.first_tile = ft; g.ntiles = nt; g.rep_first = rf;
            g.nrep = (uint8_t)nr; g.pos = (uint16_t)pos; g.spos = kNoScatter; g.buf = buf; g.req = req;
            w.segs[lev & 1][s] = g;
        }
    }
}

// Sums the nrep histogram replicas of a bucket for digit lane d (and ORs the
// key masks for d < 4), eight loads in flight per thread.
__device__ __forceinline__ uint32_t reduce_replicas(const uint32_t *rp, uint32_t nrep, uint32_t d,
                                                    unsigned long long *mask_out) {
    uint32_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool dm = d < 4;
    uint32_t r = 0;
    for (; r + 8 <= nrep; r += 8) {
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const uint32_t *q = rp + (size_t)(r + k) * kRepWords;
            acc[k] += q[d];
            if (dm) m[k] |= reinterpret_cast<const unsigned long long *>(q + kRadix)[d];
        }
    }
    for (; r < nrep; r++) {
        const uint32_t *q = rp + (size_t)r * kRepWords;
        acc[0] += q[d];
        if (dm) m[0] |= reinterpret_cast<const unsigned long long *>(q + kRadix)[d];
    }
    if (dm) *mask_out = m[0] | m[1] | m[2] | m[3] | m[4] | m[5] | m[6] | m[7];
    return acc[0] + acc[1] + acc[2] + acc[3] + acc[4] + acc[5] + acc[6] + acc[7];
}

// First key bit that differs between keys of a bucket, from its OR and
// OR-of-complement masks; kKeyBits if every key is equal.
__device__ __forceinline__ uint32_t first_varying(uint64_t orh, uint64_t ornh, uint64_t orl, uint64_t ornl) {
    const uint64_t vh = orh & ornh, vl = orl & ornl & 0xFFFFu;
    if (vh) return (uint32_t)__clzll(vh);
    if (vl) return 64u + ((uint32_t)__clz((uint32_t)vl) - 16u);
    return kKeyBits;
}

// Planning of one big bucket (Algorithm 1): if its digit at `pos` splits it,
// it gets a partition pass and its sub-buckets become either big buckets of
// the next level, or local-sort tasks (consecutive small sub-buckets packed
// together up to the local capacity); if the digit is constant, the bucket
// moves to the next level unmoved, starting at its first varying key bit;
// if no key bit varies, it is already in order.  Whole workgroup.
__device__ void plan_segment(const Work &w, const Tune &tu, int lev, uint32_t s) {
    __shared__ uint32_t p_cnt[kRadix];
    __shared__ uint32_t p_base[kRadix];
    __shared__ uint32_t p_tmp[kWaves];
    __shared__ unsigned long long p_mask[4];
    __shared__ uint32_t p_tstart[kRadix];
    __shared__ uint32_t p_tcnt[kRadix];
    __shared__ uint32_t p_ntask;
    __shared__ uint32_t p_pcnt[kParts], p_pfirst[kParts], p_pslot[kParts];
    const uint32_t d = threadIdx.x;
    Seg *sp = &w.segs[lev & 1][s];
    const Seg sg = *sp;
    if (sg.count == 0 || sg.nrep == 0) return;  // placeholder left by a fired guard
    // a bucket held as chunks of the first-pass pool always gets its partition
    // pass, which also makes it contiguous (tasks read contiguous ranges)
    const bool chunked = sg.buf == 2;
    if (sg.count <= tu.big && !chunked) {  // small bucket: one local-sort task as it is
        if (d == 0) {
            sp->spos = kNoScatter;
            emit_task(w, sg.start, sg.count, sg.buf, 0, sg.req);
        }
        return;
    }
    uint32_t *rp = w.rep[lev & 1] + (size_t)sg.rep_first * kRepWords;
    unsigned long long m = 0;
    const uint32_t cnt = reduce_replicas(rp, sg.nrep, d, &m);
    if (d < 4) p_mask[d] = m;
    const int isconst = __syncthreads_or(cnt == sg.count);
    if (isconst && !chunked) {  // digit at pos is constant over the bucket: skip ahead without moving data
        if (d == 0) {
            sp->spos = kNoScatter;
            const uint32_t f = first_varying(p_mask[0], p_mask[1], p_mask[2], p_mask[3]);
            if (f >= kKeyBits) emit_sorted(w, sg.start, sg.count, sg.buf, sg.req);
            else new_segment(w, tu, lev + 1, sg.start, sg.count, max(f, (uint32_t)sg.pos + tu.digit), sg.buf, sg.req);
        }
        return;
    }
    const uint32_t p = sg.pos;
    const uint32_t base = block_excl_scan(cnt, p_tmp);
    rp[d] = base;  // replica 0 now holds the bucket offsets used by k_scatter
    p_cnt[d] = cnt;
    p_base[d] = base;
    if (d == 0) {
        sp->spos = (uint16_t)p;
        atomicAdd(&w.ctl->moved[lev], (unsigned long long)sg.count);
    }
    const uint8_t cbuf = next_buf(sg.buf);
    const uint32_t cpos = p + tu.digit;
    if (cnt > tu.big && cpos >= kKeyBits) emit_sorted(w, sg.start + base, cnt, cbuf, sg.req);  // equal keys
    new_segments_block(w, tu, lev + 1, cnt > tu.big && cpos < kKeyBits, sg.start + base, cnt, cpos, cbuf, sg.req);
    __syncthreads();
    if (d < 64) {
        // pack consecutive small buckets into tasks of at most kLocalCap keys
        // (greedy, in digit order): wave 0 holds the counts and offsets in
        // registers (lane l: digits 4l..4l+3) and walks them with lane reads,
        // so the sequential walk costs no memory round trips
        uint32_t c4[4], b4[4];
        bool big4 = false;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            c4[k] = p_cnt[4 * d + k];
            b4[k] = p_base[4 * d + k];
            big4 = big4 || c4[k] > tu.big;
        }
        uint32_t nt = 0, cur_start = 0, cur = 0;
        if (__ballot(big4) == 0 && sg.count <= 16u * kLocalCap) {
            // no big sub-bucket and few tasks: the same greedy cuts a task at a
            // time.  A task starting at offset `base` ends at the last digit
            // whose inclusive prefix count stays within base + capacity; those
            // digits form a prefix of the 256, counted with four ballots.
            uint32_t s4[4];
#pragma unroll
            for (int k = 0; k < 4; k++) s4[k] = b4[k] + c4[k];
            uint32_t base = 0;
            while (base < sg.count) {
                const uint32_t lim = base + (uint32_t)kLocalCap;
                uint32_t nle = 0;
#pragma unroll
                for (int k = 0; k < 4; k++) nle += (uint32_t)__popcll(__ballot(s4[k] <= lim));
                const uint32_t e = nle - 1u;  // >= the next non-empty digit: it fits alone
                const uint32_t v0 = __builtin_amdgcn_readlane(s4[0], e >> 2), v1 = __builtin_amdgcn_readlane(s4[1], e >> 2),
                               v2 = __builtin_amdgcn_readlane(s4[2], e >> 2), v3 = __builtin_amdgcn_readlane(s4[3], e >> 2);
                const uint32_t se = (e & 3u) == 0 ? v0 : (e & 3u) == 1 ? v1 : (e & 3u) == 2 ? v2 : v3;
                if (d == 0) { p_tstart[nt] = base; p_tcnt[nt] = se - base; }
                nt++;
                base = se;
            }
        } else
        for (int e4 = 0; e4 < kRadix / 4; e4++) {
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const uint32_t ce = __builtin_amdgcn_readlane(c4[k], e4);
                if (ce == 0) continue;
                if (ce > tu.big) {
                    if (cur) {
                        if (d == 0) { p_tstart[nt] = cur_start; p_tcnt[nt] = cur; }
                        nt++;
                        cur = 0;
                    }
                    continue;
                }
                if (cur && cur + ce > (uint32_t)kLocalCap) {
                    if (d == 0) { p_tstart[nt] = cur_start; p_tcnt[nt] = cur; }
                    nt++;
                    cur = 0;
                }
                if (cur == 0) cur_start = __builtin_amdgcn_readlane(b4[k], e4);
                cur += ce;
            }
        }
        if (cur) {
            if (d == 0) { p_tstart[nt] = cur_start; p_tcnt[nt] = cur; }
            nt++;
        }
        if (d == 0) p_ntask = nt;
    }
    if (d < kParts) { p_pcnt[d] = 0; p_pfirst[d] = 0xFFFFFFFFu; }
    __syncthreads();
    // the tasks' output parts: their starts increase with t, so each part is a
    // run of consecutive tasks; one slot allocation per run
    const uint32_t ntk = p_ntask;
    for (uint32_t t = d; t < ntk; t += kWG) {
        const uint32_t pt = part_of(w, sg.start + p_tstart[t]);
        atomicAdd(&p_pcnt[pt], 1u);
        atomicMin(&p_pfirst[pt], t);
    }
    __syncthreads();
    if (d < kParts && p_pcnt[d]) {
        const uint32_t slot = atomicAdd(&w.ctl->ntask[d], p_pcnt[d]);
        if ((uint64_t)slot + p_pcnt[d] > w.max_tasks) {
            atomicOr(&w.ctl->guard, 1u);
            p_pslot[d] = 0xFFFFFFFFu;
        } else {
            p_pslot[d] = slot;
        }
    }
    __syncthreads();
    for (uint32_t t = d; t < ntk; t += kWG) {
        const uint32_t pt = part_of(w, sg.start + p_tstart[t]);
        if (p_pslot[pt] == 0xFFFFFFFFu) continue;
        Task tk;
        tk.start = sg.start + p_tstart[t]; tk.count = p_tcnt[t]; tk.buf = cbuf; tk.flags = 0; tk.req = sg.req;
        w.tasks[(size_t)pt * w.max_tasks + p_pslot[pt] + (t - p_pfirst[pt])] = tk;
    }
    __syncthreads();
}

// Adds digit d of the valid lanes into the LDS histogram sh; called by the
// whole wave, the valid lanes being a prefix of it.  Lanes that share the
// first lane's digit add once, through the lowest of them: with skewed keys
// whole waves fall on one digit, and per-lane atomics on one counter serialize.
__device__ __forceinline__ void hist_add(uint32_t *sh, uint32_t d, bool valid) {
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t same = __ballot(valid && d == d0);
    if (valid && d != d0) atomicAdd(&sh[d], 1u);
    if (same && __lane_id() == (uint32_t)__builtin_ctzll(same)) atomicAdd(&sh[d0], (uint32_t)__popcll(same));
}

// Adds a tile's LDS histogram and key masks into one replica of its bucket,
// and stores the tile's digit counts.
__device__ __forceinline__ void flush_tile_hist(uint32_t *rep, const uint32_t *sh, const unsigned long long *smask,
                                                unsigned long long *tile_count) {
    const uint32_t v = sh[threadIdx.x];
    tile_count[threadIdx.x] = v;  // this tile's digit counts, for the tile-offset scan
    if (v) atomicAdd(&rep[threadIdx.x], v);
    if (threadIdx.x < 4) {
        const unsigned long long m = smask[threadIdx.x];
        if (m) atomicOr(reinterpret_cast<unsigned long long *>(rep + kRadix) + threadIdx.x, m);
    }
}

// Reduces per-thread key masks (OR of h, OR of ~h, OR of k16, OR of ~k16) over the workgroup.
__device__ __forceinline__ void block_masks(uint64_t oh, uint64_t onh, uint64_t ol, uint64_t onl,
                                            unsigned long long *smask) {
    oh = wave_or64(oh);
    onh = wave_or64(onh);
    ol = wave_or64(ol);
    onl = wave_or64(onl);
    if ((threadIdx.x & 63) == 0) {
        atomicOr(&smask[0], (unsigned long long)oh);
        atomicOr(&smask[1], (unsigned long long)onh);
        atomicOr(&smask[2], (unsigned long long)ol);
        atomicOr(&smask[3], (unsigned long long)onl);
    }
}

// ---------------------------------------------------------------------------
// k_init: level-0 buckets (one per request), their tile map and replicas

__global__ __launch_bounds__(kWG) void k_init(Work w) {
    const Hdr hd = *w.hdr;
    if (blockIdx.x == 0) {
        uint32_t *c = reinterpret_cast<uint32_t *>(w.ctl);
        for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += kWG) c[i] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            w.ctl->nseg[0] = hd.nreq;
            w.ctl->ntiles[0] = hd.tiles0;
        }
    }
    for (uint32_t r = blockIdx.x; r < hd.nreq; r += gridDim.x) {
        const Req rq = w.reqs[r];
        const bool ok = (uint64_t)rq.first_tile + rq.ntiles <= w.max_tiles &&
                        (uint64_t)rq.rep_first + rq.nrep <= w.max_reps && rq.nrep <= kMaxRep;
        if (threadIdx.x == 0) {
            Seg g;
            g.start = rq.start; g.count = ok ? (uint32_t)rq.n : 0; g.first_tile = rq.first_tile;
            g.ntiles = rq.ntiles; g.rep_first = rq.rep_first; g.nrep = (uint8_t)rq.nrep; g.pos = 0;
            g.spos = kNoScatter; g.buf = 0; g.req = (uint16_t)r;
            w.segs[0][r] = g;
            if (!ok) atomicOr(&w.ctl->guard, 256u);
        }
        if (!ok) continue;
        for (uint32_t k = threadIdx.x; k < rq.ntiles; k += kWG) w.tile_seg[0][rq.first_tile + k] = r;
        uint32_t *rp = w.rep[0] + (size_t)rq.rep_first * kRepWords;
        for (uint32_t i = threadIdx.x; i < rq.nrep * kRepWords; i += kWG) rp[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// k_extract: tuples + first-digit histogram and key masks of every record

template <int ITEMS>
__global__ __launch_bounds__(kWG) void k_extract(Work w, Tune tu) {
    constexpr int RI = ITEMS > 8 ? 8 : ITEMS;
    __shared__ uint32_t sh[kRadix];
    __shared__ unsigned long long smask[4];
    const uint32_t ntiles = min(w.ctl->ntiles[0], w.max_tiles);
    const uint32_t nreq = w.hdr->nreq;
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        sh[threadIdx.x] = 0;
        if (threadIdx.x < 4) smask[threadIdx.x] = 0;
        w.status[(size_t)tile * kRadix + threadIdx.x] = 0;
        if (tile % kChunkTiles == 0) w.cstat[(size_t)(tile / kChunkTiles) * kRadix + threadIdx.x] = 0;
        const uint32_t s = w.tile_seg[0][tile];
        if (s >= nreq || s >= w.max_seg) { if (threadIdx.x == 0) atomicOr(&w.ctl->guard, 8u); __syncthreads(); continue; }
        const Seg sg = w.segs[0][s];
        if (!seg_ok(w, sg, tile)) { if (threadIdx.x == 0) atomicOr(&w.ctl->guard, 8u); __syncthreads(); continue; }
        const Req rq = w.reqs[sg.req];
        const uint64_t local0 = (uint64_t)(tile - sg.first_tile) * tu.tile;
        const uint32_t nvalid = (uint32_t)min<uint64_t>(tu.tile, sg.count - local0);
        __syncthreads();
        uint64_t *H = w.H[0] + sg.start + local0;
        uint64_t *L = w.L[0] + sg.start + local0;
        uint64_t oh = 0, onh = 0, ol = 0, onl = 0;
#pragma unroll 1
        for (int r0 = 0; r0 < ITEMS; r0 += RI) {  // RI keys per thread in flight
            uint32_t a[RI], b[RI], c[RI];
#pragma unroll
            for (int u = 0; u < RI; u++) {
                const uint32_t q = (r0 + u) * kWG + threadIdx.x;
                // lanes past the tile's last record load that record again: no
                // branch around the loads, so all RI of them are in flight
                // together (a load inside a branch is waited for at its end)
                const uint32_t qc = q < nvalid ? q : nvalid - 1;
                // the caller's records are device memory: global (not flat)
                // loads, marked non-temporal (each line is read once here)
                const gu32 *p = (const gu32 *)(rq.in + (local0 + qc) * kRec);
                a[u] = __builtin_nontemporal_load(p);
                b[u] = __builtin_nontemporal_load(p + 1);
                c[u] = __builtin_nontemporal_load(p + 2);
            }
#pragma unroll
            for (int u = 0; u < RI; u++) {
                const uint32_t q = (r0 + u) * kWG + threadIdx.x;
                const bool valid = q < nvalid;
                const uint64_t h = __builtin_bswap64(((uint64_t)b[u] << 32) | a[u]) & w.kmask_h;
                if (valid) {
                    const uint64_t k16 = __builtin_bswap16((uint16_t)(c[u] & 0xFFFFu)) & w.kmask_l;
                    // tuples: written once, read by the next pass (far beyond the caches)
                    __builtin_nontemporal_store(h, H + q);
                    __builtin_nontemporal_store((k16 << 32) | (uint32_t)(local0 + q), L + q);
                    oh |= h; onh |= ~h; ol |= k16; onl |= (~k16) & 0xFFFFu;
                }
                hist_add(sh, (uint32_t)(h >> (64 - tu.digit)), valid);
            }
        }
        block_masks(oh, onh, ol, onl, smask);
        __syncthreads();
        flush_tile_hist(w.rep[0] + ((size_t)sg.rep_first + (tile - sg.first_tile) % sg.nrep) * kRepWords, sh, smask,
                        w.status + (size_t)tile * kRadix);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Fused first pass (one request): extraction and the level-0 partition in one
// pass over the records.
//
// A bucket's size is known only once every tile has been read, so the pass
// cannot place a bucket at its final offset.  Each bucket is instead a chain
// of chunks of `tile` keys taken from a pool as the bucket grows: a tile's run
// of digit d occupies positions [v, v + c) of bucket d's own position space,
// v being the count of digit d in the tiles before it (a decoupled look-back
// over per-tile status words, tiles taken in order from a counter), and
// position p of bucket d lives in slot p % tile of chunk ctab[d][p / tile].
// The tile whose run covers a chunk's first position takes that chunk from
// the pool counter and publishes it; a tile whose run starts inside a chunk
// waits for it (the owner is an earlier tile that has finished its
// look-back, so the wait ends).  Runs are at most one tile long, so a run
// touches at most two chunks.  Positions follow input order within a bucket
// (tiles in order, keys ranked stably inside a tile), so the buckets hold
// their keys in stable order, as the separate passes would.
//
// RECORDS: the pass also copies each record to pool slot (chunk * tile +
// slot) of a record pool, and a tuple carries its position inside its bucket
// instead of the record index (positions order the bucket's keys like the
// input does, so ties still break by input order); the local sorts turn
// positions into pool slots for the gather.

// Clears the first pass's look-back words and chunk table.
__global__ __launch_bounds__(kWG) void k_fzero(unsigned long long *status, uint64_t nstatus, uint32_t *ctab,
                                               uint64_t nctab) {
    const uint64_t stride = (uint64_t)gridDim.x * kWG;
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < nstatus; i += stride) status[i] = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < nctab; i += stride) ctab[i] = 0;
}

// A free chunk of the pool (0xFFFFFFFF and a guard bit if none is left).
__device__ __forceinline__ uint32_t fuse_chunk_take(const Work &w) {
    const uint32_t c = atomicAdd(&w.ctl->pool_ctr, 1u);
    if (c >= w.max_chunks) { atomicOr(&w.ctl->guard, 512u); return 0xFFFFFFFFu; }
    return c;
}

// 12 bytes at a 4-byte aligned address (a record's first three dwords in one load)
typedef uint32_t u32x3a __attribute__((ext_vector_type(3), aligned(4)));
typedef const __attribute__((address_space(1))) u32x3a gu32x3;

template <int FWG, int FI, bool RECORDS>
__global__ __launch_bounds__(FWG, 1) void k_fuse0(Work w, Tune tu) {
    constexpr int FT = FWG * FI;
    constexpr int NW = FWG / 64;
    __shared__ uint64_t sH[FT];
    __shared__ uint64_t sL[FT];
    __shared__ uint32_t cnt[NW][kRadix];
    __shared__ uint32_t lbase[kRadix];
    __shared__ uint32_t vbase[kRadix];      // first position of the tile's run in its bucket
    __shared__ uint32_t cph[2][kRadix];     // pool chunks of the run's first and second part
    __shared__ uint32_t tmp[NW];
    __shared__ uint32_t s_tile;
    __shared__ uint16_t sQ[RECORDS ? FT : 1];  // staged slot -> key within the tile
    __shared__ uint32_t sP[RECORDS ? FT : 1];  // staged slot -> pool slot (~0: none)

    const Req rq = w.reqs[0];
    const uint64_t n = rq.n;
    const uint32_t nft = (uint32_t)((n + FT - 1) / FT);
    const uint32_t C = tu.tile;
    const uint32_t cshift = 31u - (uint32_t)__builtin_clz(C);
    const uint32_t ndig = 1u << tu.digit;
    const uint32_t shift = 64u - tu.digit;
    const uint64_t pool_keys = (uint64_t)w.max_chunks * C;
    for (;;) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const uint32_t wv = tid >> 6, lane = tid & 63;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&w.ctl->ftile_ctr, 1u);
        for (uint32_t i = tid; i < NW * kRadix; i += FWG) (&cnt[0][0])[i] = 0;
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= nft) break;
        const uint64_t local0 = (uint64_t)tile * FT;
        const uint32_t nvalid = (uint32_t)min<uint64_t>(FT, n - local0);
        // keys of the tile: wave wv holds keys [wv * FI * 64, (wv + 1) * FI * 64)
        // of the tile, item u of lane l being key wv * FI * 64 + u * 64 + l
        uint64_t h[FI], l[FI];
        {
            uint32_t a[FI], b[FI], c[FI];
#pragma unroll
            for (int u = 0; u < FI; u++) {
                const uint32_t q = wv * (FI * 64) + u * 64 + lane;
                const uint32_t qc = q < nvalid ? q : nvalid - 1;  // loads stay branch-free
                const gu32 *p = (const gu32 *)(rq.in + (local0 + qc) * kRec);
                if (RECORDS) {  // the record is copied below: keep its lines in the caches
                    a[u] = p[0]; b[u] = p[1]; c[u] = p[2];
                } else {  // each line is read once here: non-temporal
                    const u32x3a v = __builtin_nontemporal_load((gu32x3 *)p);
                    a[u] = v.x; b[u] = v.y; c[u] = v.z;
                }
            }
#pragma unroll
            for (int u = 0; u < FI; u++) {
                const uint32_t q = wv * (FI * 64) + u * 64 + lane;
                h[u] = __builtin_bswap64(((uint64_t)b[u] << 32) | a[u]) & w.kmask_h;
                const uint64_t k16 = __builtin_bswap16((uint16_t)(c[u] & 0xFFFFu)) & w.kmask_l;
                l[u] = (k16 << 32) | (uint32_t)(local0 + q);
            }
        }
        // stable ranks by the leading digit (eight items at a time)
        uint32_t pk[FI];
        constexpr int RCH = FI < 8 ? FI : 8;
#pragma unroll
        for (int c0 = 0; c0 < FI; c0 += RCH) {
            uint32_t old[RCH];
#pragma unroll
            for (int u = c0; u < c0 + RCH; u++) {
                const uint32_t q = wv * (FI * 64) + u * 64 + lane;
                const bool valid = q < nvalid;
                rank_issue(valid ? (uint32_t)(h[u] >> shift) : 0u, valid, cnt[wv], old[u - c0], pk[u]);
            }
#pragma unroll
            for (int u = c0; u < c0 + RCH; u++) pk[u] = (pk[u] & 0xFFu) | (rank_finish(old[u - c0], pk[u]) << 8);
        }
        __syncthreads();
        const bool dl = tid < ndig;  // digit lanes
        uint32_t tot = 0;
        if (dl) {
#pragma unroll
            for (int j = 0; j < NW; j++) {
                const uint32_t cj = cnt[j][tid];
                cnt[j][tid] = tot;
                tot += cj;
            }
        }
        const uint32_t lb = block_excl_scan<NW>(tot, tmp);
        unsigned long long *const st = w.status + (size_t)tile * kRadix + tid;
        if (dl) {
            lbase[tid] = lb;
            // the tile's count, published before the staging so later tiles
            // can sum past this one while it stages
            st_agent(st, (tile == 0 ? kFlagInc : kFlagAgg) | tot);
        }
        __syncthreads();
        // keys to their slots in the tile (digit-major)
#pragma unroll
        for (int u = 0; u < FI; u++) {
            const uint32_t q = wv * (FI * 64) + u * 64 + lane;
            if (q < nvalid) {
                const uint32_t d = pk[u] & 0xFFu;
                const uint32_t pos = lbase[d] + cnt[wv][d] + (pk[u] >> 8);
                sH[pos] = h[u];
                sL[pos] = l[u];
                if (RECORDS) sQ[pos] = (uint16_t)q;
            }
        }
        if (dl) {
            // look back over the tiles before this one for the counts of digit tid
            uint64_t excl = 0;
            if (tile > 0) {
                constexpr int LW = 8;
                uint32_t spins = 0;
                bool done = false;
                for (uint32_t t0 = tile - 1; !done; t0 -= LW) {
                    unsigned long long v[LW];
#pragma unroll
                    for (int k = 0; k < LW; k++)
                        v[k] = t0 >= (uint32_t)k ? ld_agent(w.status + (size_t)(t0 - k) * kRadix + tid) : 0ull;
#pragma unroll
                    for (int k = 0; k < LW; k++) {
                        if (done) break;
                        const uint32_t tt = t0 - k;
                        while ((v[k] >> 62) == 0 && spins < kSpinLimit) {
                            __builtin_amdgcn_s_sleep(1);
                            spins++;
                            v[k] = ld_agent(w.status + (size_t)tt * kRadix + tid);
                        }
                        if (spins >= kSpinLimit) { atomicOr(&w.ctl->guard, 16u); done = true; break; }
                        excl += v[k] & kCountMask;
                        if ((v[k] & kFlagInc) || tt == 0) done = true;
                    }
                }
                st_agent(st, kFlagInc | (excl + tot));
            }
            vbase[tid] = (uint32_t)excl;
            // the run's chunks: take those whose first position lies in the
            // run, then wait for the one it starts inside (if any)
            uint32_t c0 = 0xFFFFFFFFu, c1 = 0xFFFFFFFFu;
            if (tot) {
                uint32_t *ct = w.ctab + (size_t)tid * w.ctab_stride;
                const uint64_t j0 = excl >> cshift, j1 = (excl + tot - 1) >> cshift;
                const bool own0 = (excl & (C - 1)) == 0;
                if (j1 >= w.ctab_stride) {
                    atomicOr(&w.ctl->guard, 512u);
                } else {
                    if (own0) {
                        c0 = fuse_chunk_take(w);
                        __hip_atomic_store(ct + j0, c0 + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (j1 != j0) {
                        c1 = fuse_chunk_take(w);
                        __hip_atomic_store(ct + j1, c1 + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (!own0) {
                        uint32_t x = ld_agent32(ct + j0);
                        uint32_t spins = 0;
                        while (x == 0 && spins < kSpinLimit) {
                            __builtin_amdgcn_s_sleep(1);
                            spins++;
                            x = ld_agent32(ct + j0);
                        }
                        if (x == 0) atomicOr(&w.ctl->guard, 16u);
                        c0 = x - 1u;  // 0xFFFFFFFF if never published
                    }
                }
            }
            cph[0][tid] = c0;
            cph[1][tid] = c1;
        }
        __syncthreads();
        // runs to their chunks
        uint64_t *PH = w.H[2], *PL = w.L[2];
#pragma unroll
        for (int u = 0; u < FI; u++) {
            const uint32_t q = u * FWG + tid;
            if (q < nvalid) {
                const uint64_t hh = sH[q];
                const uint32_t d = (uint32_t)(hh >> shift);
                const uint32_t v = vbase[d] + (q - lbase[d]);
                const uint32_t ch = ((v >> cshift) == (vbase[d] >> cshift)) ? cph[0][d] : cph[1][d];
                const uint64_t slot = (uint64_t)ch * C + (v & (C - 1));
                uint64_t ll = sL[q];
                if (RECORDS) ll = (ll & ~0xFFFFFFFFull) | v;
                if (ch < w.max_chunks && slot < pool_keys) {
                    // the pool is read by the next level's passes, far beyond the caches
                    __builtin_nontemporal_store(hh, PH + slot);
                    __builtin_nontemporal_store(ll, PL + slot);
                    if (RECORDS) sP[q] = (uint32_t)slot;
                } else {
                    atomicOr(&w.ctl->guard, 512u);
                    if (RECORDS) sP[q] = 0xFFFFFFFFu;
                }
            }
        }
        if (RECORDS) {
            __syncthreads();
            // records to their pool slots, 25 dwords each, staged order (the
            // reads hit lines the key loads brought in; the writes are runs)
            const gu32 *src = (const gu32 *)(rq.in + local0 * kRec);
            gu32w *dst = (gu32w *)w.rpool;
            constexpr int PER = (FT * 25 + FWG - 1) / FWG;
            constexpr int B = 25;  // loads in flight per thread
#pragma unroll 1
            for (int u0 = 0; u0 < PER; u0 += B) {
                uint32_t val[B], dsl[B];
#pragma unroll
                for (int u = 0; u < B; u++) {
                    const uint32_t g = (uint32_t)(u0 + u) * FWG + tid;
                    const uint32_t sidx = g / 25u, k = g - 25u * sidx;
                    dsl[u] = 0xFFFFFFFFu;
                    val[u] = 0;
                    if (u0 + u < PER && sidx < nvalid) {
                        dsl[u] = sP[sidx];
                        if (dsl[u] != 0xFFFFFFFFu) val[u] = src[(uint32_t)sQ[sidx] * 25u + k];
                    }
                }
#pragma unroll
                for (int u = 0; u < B; u++) {
                    const uint32_t g = (uint32_t)(u0 + u) * FWG + tid;
                    const uint32_t k = g - 25u * (g / 25u);
                    if (dsl[u] != 0xFFFFFFFFu) __builtin_nontemporal_store(val[u], dst + (uint64_t)dsl[u] * 25u + k);
                }
            }
        }
    }
}

// Level-1 buckets of the fused first pass: the bucket counts are the last
// tile's inclusive look-back words; bucket d (when not empty) becomes level-1
// bucket number (non-empty digits before d), starting at the sum of the
// counts before it, with one level-1 tile per chunk.  Every block computes the
// same scans; block 0 writes the buckets and counters, and all blocks fill the
// level-1 tile map and chunk names and clear the level-1 replicas.
__global__ __launch_bounds__(kWG) void k_plan0(Work w, Tune tu, uint32_t ftile) {
    __shared__ uint32_t tmp[kWaves];
    __shared__ uint32_t s_ft[kRadix + 1];
    __shared__ uint32_t s_seg[kRadix];
    __shared__ uint32_t s_tot[3];
    const uint32_t d = threadIdx.x;
    const uint64_t n = w.reqs[0].n;
    const uint32_t nft = (uint32_t)((n + ftile - 1) / ftile);
    const uint32_t C = tu.tile;
    uint32_t c = 0;
    if (nft > 0 && d < (1u << tu.digit)) {
        const unsigned long long v = ld_agent(w.status + (size_t)(nft - 1) * kRadix + d);
        if (!(v & kFlagInc)) { if (blockIdx.x == 0) atomicOr(&w.ctl->guard, 16u); }
        else c = (uint32_t)(v & kCountMask);
    }
    const bool need = c > 0;
    const uint32_t nt = need ? (c + C - 1) / C : 0u;
    const uint32_t nr = min(nt, (uint32_t)kMaxRep);
    const uint32_t es = block_excl_scan(need ? 1u : 0u, tmp);
    const uint32_t et = block_excl_scan(nt, tmp);
    const uint32_t er = block_excl_scan(nr, tmp);
    const uint32_t base = block_excl_scan(c, tmp);
    s_ft[d] = et;
    s_seg[d] = es;
    if (d == kWG - 1) {
        s_ft[kRadix] = et + nt;
        s_tot[0] = es + (need ? 1u : 0u);
        s_tot[1] = et + nt;
        s_tot[2] = er + nr;
    }
    __syncthreads();
    const bool fits = s_tot[0] <= w.max_seg && s_tot[1] <= w.max_tiles && s_tot[2] <= w.max_reps &&
                      (uint64_t)base + c <= w.n;
    const int all_fit = __syncthreads_and(fits);
    if (!all_fit) {
        if (blockIdx.x == 0 && d == 0) { atomicOr(&w.ctl->guard, 4u); w.ctl->nseg[1] = 0; w.ctl->ntiles[1] = 0; }
        return;
    }
    if (blockIdx.x == 0) {
        if (need) {
            Seg g;
            g.start = base; g.count = c; g.first_tile = et; g.ntiles = nt; g.rep_first = er; g.nrep = (uint8_t)nr;
            g.pos = (uint16_t)tu.digit; g.spos = kNoScatter; g.buf = 2; g.req = 0;
            w.segs[1][es] = g;
        }
        if (d == 0) {
            w.ctl->nseg[1] = s_tot[0];
            w.ctl->ntiles[1] = s_tot[1];
            w.ctl->rep_ctr[1] = s_tot[2];
            w.ctl->moved[0] = n;
        }
    }
    // tile map and chunk names of the level-1 tiles
    const uint32_t ntl = s_tot[1];
    for (uint32_t t = blockIdx.x * kWG + d; t < ntl; t += gridDim.x * kWG) {
        uint32_t lo = 0, hi = kRadix - 1;  // last digit whose first tile is <= t
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (s_ft[mid] <= t) lo = mid; else hi = mid - 1;
        }
        w.tile_seg[1][t] = s_seg[lo];
        const uint32_t cv = w.ctab[(size_t)lo * w.ctab_stride + (t - s_ft[lo])];
        w.tsrc[t] = cv - 1u;  // 0xFFFFFFFF (outside the pool) if never taken
    }
    const uint64_t nw = (uint64_t)s_tot[2] * kRepWords;
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + d; i < nw; i += (uint64_t)gridDim.x * kWG) w.rep[1][i] = 0;
}

// ---------------------------------------------------------------------------
// k_hist: digit histogram and key masks of the big buckets of level lev >= 1

template <int ITEMS>
__global__ __launch_bounds__(kWG) void k_hist(Work w, Tune tu, int lev) {
    constexpr int RI = ITEMS > 16 ? 16 : ITEMS;
    __shared__ uint32_t sh[kRadix];
    __shared__ unsigned long long smask[4];
    const uint32_t ntiles = min(w.ctl->ntiles[lev], w.max_tiles);
    const uint32_t nseg = min(w.ctl->nseg[lev], w.max_seg);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        sh[threadIdx.x] = 0;
        if (threadIdx.x < 4) smask[threadIdx.x] = 0;
        w.status[(size_t)tile * kRadix + threadIdx.x] = 0;
        if (tile % kChunkTiles == 0) w.cstat[(size_t)(tile / kChunkTiles) * kRadix + threadIdx.x] = 0;
        const uint32_t s = w.tile_seg[lev & 1][tile];
        if (s >= nseg) { if (threadIdx.x == 0) atomicOr(&w.ctl->guard, 8u); __syncthreads(); continue; }
        const Seg sg = w.segs[lev & 1][s];
        if (!seg_ok(w, sg, tile) || sg.pos >= kKeyBits) {
            if (threadIdx.x == 0) atomicOr(&w.ctl->guard, 8u);
            __syncthreads();
            continue;
        }
        const uint64_t local0 = (uint64_t)(tile - sg.first_tile) * tu.tile;
        bool src_ok;
        const uint64_t src = tile_src(w, sg, tile, tu.tile, src_ok);
        if (!src_ok) { if (threadIdx.x == 0) atomicOr(&w.ctl->guard, 8u); __syncthreads(); continue; }
        const uint32_t nvalid = (uint32_t)min<uint64_t>(tu.tile, sg.count - local0);
        const uint64_t *H = w.H[sg.buf] + src;
        const uint64_t *L = w.L[sg.buf] + src;
        // key bytes 8..9 are read only when the digit reaches them; otherwise
        // their mask reads "varying", so a bucket constant through byte 7
        // moves on to bit 64 and the next level reads them
        const bool needL = sg.pos + tu.digit > 64;
        __syncthreads();
        uint64_t oh = 0, onh = 0, ol = needL ? 0 : 0xFFFFu, onl = needL ? 0 : 0xFFFFu;
#pragma unroll 1
        for (int r0 = 0; r0 < ITEMS; r0 += RI) {  // RI keys per thread in flight
            uint64_t h[RI], l[RI];
#pragma unroll
            for (int u = 0; u < RI; u++) {
                const uint32_t q = (r0 + u) * kWG + threadIdx.x;
                h[u] = 0; l[u] = 0;
                if (q < nvalid) {
                    // non-temporal: the bucket is far larger than the caches
                    h[u] = __builtin_nontemporal_load(H + q);
                    if (needL) l[u] = __builtin_nontemporal_load(L + q);
                }
            }
#pragma unroll
            for (int u = 0; u < RI; u++) {
                const uint32_t q = (r0 + u) * kWG + threadIdx.x;
                hist_add(sh, digit_at(h[u], l[u], sg.pos, tu.digit), q < nvalid);
                if (q < nvalid) {
                    oh |= h[u]; onh |= ~h[u];
                    if (needL) {
                        const uint64_t k16 = (l[u] >> 32) & 0xFFFFu;
                        ol |= k16; onl |= (~k16) & 0xFFFFu;
                    }
                }
            }
        }
        block_masks(oh, onh, ol, onl, smask);
        __syncthreads();
        flush_tile_hist(w.rep[lev & 1] + ((size_t)sg.rep_first + (tile - sg.first_tile) % sg.nrep) * kRepWords, sh,
                        smask, w.status + (size_t)tile * kRadix);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_plan: plans every big bucket of level lev (after its histogram pass)

// ---------------------------------------------------------------------------
// tile-offset scan: every tile's offset, per digit, among the tiles of its bucket
//
// status[tile][d] holds the tile's count of digit d (from the histogram pass);
// this replaces it with the sum over the earlier tiles of the same bucket, so
// the partition pass needs no cross-tile wait.  Chunks of kChunkTiles tiles
// are scanned by one workgroup each (digit d by thread d); a bucket that runs
// over a chunk boundary takes its carry from a decoupled look-back over the
// earlier chunks, which publish their totals as soon as they have them (a
// chunk whose last bucket starts inside it publishes an inclusive value at
// once).

__device__ void tscan_chunks(const Work &w, int lev) {
    __shared__ uint32_t s_chunk;
    const uint32_t ntiles = min(w.ctl->ntiles[lev], w.max_tiles);
    const uint32_t nseg = min(w.ctl->nseg[lev], w.max_seg);
    const uint32_t nchunks = (ntiles + kChunkTiles - 1) / kChunkTiles;
    // at most one workgroup per chunk takes part (the others would only add
    // contention on the chunk counter): the last ones of the grid, which have
    // the fewest buckets to plan first
    if (gridDim.x - 1 - blockIdx.x >= nchunks) return;
    const uint32_t *tmap = w.tile_seg[lev & 1];
    const Seg *segs = w.segs[lev & 1];
    const uint32_t d = threadIdx.x;
    for (;;) {
        __syncthreads();
        if (d == 0) s_chunk = atomicAdd(&w.ctl->chunk_ctr[lev], 1u);
        __syncthreads();
        const uint32_t c = ufirst(s_chunk);
        if (c >= nchunks) break;
        const uint32_t t0 = c * kChunkTiles, t1 = min(t0 + kChunkTiles, ntiles);
        // the first bucket part continues from earlier chunks unless it starts here
        const uint32_t s0 = ufirst(tmap[t0]);
        const bool cont = s0 < nseg && segs[s0].first_tile < t0;
        uint32_t cur = s0, first_end = t1;
        unsigned long long run = 0;
        constexpr int B = 16;  // tiles whose loads are in flight together
        for (uint32_t tb = t0; tb < t1; tb += B) {
            uint32_t sv[B];
            unsigned long long cv[B];
#pragma unroll
            for (int i = 0; i < B; i++) {
                const uint32_t t = tb + i;
                sv[i] = t < t1 ? tmap[t] : cur;
                cv[i] = t < t1 ? w.status[(size_t)t * kRadix + d] : 0ull;
            }
            for (int i = 0; i < B; i++) {
                const uint32_t t = tb + i;
                if (t >= t1) break;
                const uint32_t st = ufirst(sv[i]);
                if (st != cur) {  // a new bucket starts at t
                    if (first_end == t1) first_end = t;
                    cur = st;
                    run = 0;
                }
                w.status[(size_t)t * kRadix + d] = run;
                run += cv[i];
            }
        }
        unsigned long long *cs = w.cstat + (size_t)c * kRadix + d;
        if (!cont || first_end < t1) st_agent(cs, kFlagInc | run);  // the last part starts in this chunk
        else st_agent(cs, kFlagAgg | run);
        if (!cont) continue;
        // carry of the first part: look back over earlier chunks, eight at a
        // time (their words load together; a walk over aggregates costs one
        // round trip per eight chunks)
        constexpr int LW = 8;
        unsigned long long carry = 0;
        uint32_t spins = 0;
        bool done = false;
        for (uint32_t c0 = c - 1; !done; c0 -= LW) {
            unsigned long long v[LW];
#pragma unroll
            for (int k = 0; k < LW; k++)
                v[k] = c0 >= (uint32_t)k ? ld_agent(w.cstat + (size_t)(c0 - k) * kRadix + d) : 0ull;
#pragma unroll
            for (int k = 0; k < LW; k++) {
                if (done) break;
                const uint32_t cc = c0 - k;
                while ((v[k] >> 62) == 0 && spins < kSpinLimit) {
                    __builtin_amdgcn_s_sleep(1);
                    spins++;
                    v[k] = ld_agent(w.cstat + (size_t)cc * kRadix + d);
                }
                if (spins >= kSpinLimit) { atomicOr(&w.ctl->guard, 16u); done = true; break; }
                carry += v[k] & kCountMask;
                if ((v[k] & kFlagInc) || cc == 0) done = true;
            }
        }
        if (first_end == t1) st_agent(cs, kFlagInc | (carry + run));
        for (uint32_t t = t0; t < first_end; t++) w.status[(size_t)t * kRadix + d] += carry;
    }
}

// k_plan: the bucket policy for every big bucket of the level (blocks take
// buckets in a fixed stride), then the tile-offset scan (blocks take chunks
// from a counter, so a chunk only waits on chunks already taken).  One launch
// per level for both keeps the fixed cost of levels without big buckets low.
__global__ __launch_bounds__(kWG) void k_plan(Work w, Tune tu, int lev) {
    const uint32_t nseg = min(w.ctl->nseg[lev], w.max_seg);
    for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        plan_segment(w, tu, lev, s);
        __syncthreads();
    }
    tscan_chunks(w, lev);
}

// ---------------------------------------------------------------------------
// k_scatter: one device-wide stable partition pass of the big buckets of level lev

// WG threads, ITEMS keys each (a tile is WG * ITEMS keys); the 256 digit
// lanes of the histogram and offsets are threads 0..255.  A tile's global
// offsets are the bucket's digit offsets plus the tile's offsets among the
// bucket's tiles (from k_plan), so tiles never wait on each other.
// waves per SIMD the scatter's registers are sized for: one workgroup per CU
// when the tile's LDS staging exceeds half the LDS, else at least two
template <int ITEMS, int WG>
constexpr int scatter_waves() {
    return (WG * ITEMS * 16 > 80 * 1024) ? WG / 256 : (WG >= 512 ? 4 : 2);
}

template <int ITEMS, int WG>
__global__ __launch_bounds__(WG, (scatter_waves<ITEMS, WG>())) void k_scatter(Work w, Tune tu, int lev) {
    constexpr int TILE = WG * ITEMS;
    constexpr int NW = WG / 64;
    __shared__ uint64_t sH[TILE];
    __shared__ uint64_t sL[TILE];
    __shared__ uint32_t cnt[NW][kRadix];
    __shared__ uint32_t lbase[kRadix];
    __shared__ unsigned long long gbase[kRadix];
    __shared__ uint32_t tmp[NW];
    __shared__ uint32_t s_tile;

    const uint32_t ntiles = min(w.ctl->ntiles[lev], w.max_tiles);
    const uint32_t nseg = min(w.ctl->nseg[lev], w.max_seg);
    // at most one workgroup per tile takes tiles (the others go straight to
    // the set-up of the next level)
    for (bool more = blockIdx.x < ntiles; more;) {
        // thread coordinates re-derived per tile: keeps the compiler from
        // hoisting every per-item index out of the loop (and spilling them)
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const uint32_t wv = tid >> 6, lane = tid & 63;
        __syncthreads();
        if (tid == 0) s_tile = atomicAdd(&w.ctl->tile_ctr[lev], 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= ntiles) { more = false; continue; }
        const uint32_t s = w.tile_seg[lev & 1][tile];
        if (s >= nseg) continue;
        const Seg sg = w.segs[lev & 1][s];
        if (sg.spos == kNoScatter || !seg_ok(w, sg, tile) || sg.spos >= kKeyBits) continue;
        const uint64_t seg_end = sg.start + sg.count;
        const uint64_t local0 = (uint64_t)(tile - sg.first_tile) * TILE;
        bool src_ok;
        const uint64_t src = tile_src(w, sg, tile, TILE, src_ok);
        if (!src_ok) { if (tid == 0) atomicOr(&w.ctl->guard, 8u); continue; }
        const uint32_t nvalid = (uint32_t)min<uint64_t>(TILE, sg.count - local0);
        const uint64_t *Hs = w.H[sg.buf] + src;
        const uint64_t *Ls = w.L[sg.buf] + src;
        const bool dl = tid < (uint32_t)kRadix;  // digit lanes
        // digit lane: the digit's bucket offset and this tile's offset among the
        // bucket's tiles (both known before the pass; used after the ranking)
        uint64_t toff = 0;
        if (dl) toff = (uint64_t)w.rep[lev & 1][(size_t)sg.rep_first * kRepWords + tid] +
                       w.status[(size_t)tile * kRadix + tid];
        for (uint32_t i = tid; i < NW * kRadix; i += WG) (&cnt[0][0])[i] = 0;
        uint64_t h[ITEMS], l[ITEMS];
        uint32_t pk[ITEMS];  // digit | rank in the wave's digit << 8
#pragma unroll
        for (int u = 0; u < ITEMS; u++) {
            const uint32_t q = wv * (ITEMS * 64) + u * 64 + lane;
            h[u] = 0; l[u] = 0;
            if (q < nvalid) { h[u] = Hs[q]; l[u] = Ls[q]; }
        }
        __syncthreads();
        // ranks, eight items at a time (bounds the registers of the old values)
        constexpr int RCH = ITEMS < 8 ? ITEMS : 8;
#pragma unroll
        for (int c0 = 0; c0 < ITEMS; c0 += RCH) {
            uint32_t old[RCH];
#pragma unroll
            for (int u = c0; u < c0 + RCH; u++) {
                const uint32_t q = wv * (ITEMS * 64) + u * 64 + lane;
                const bool valid = q < nvalid;
                rank_issue(valid ? digit_at(h[u], l[u], sg.spos, tu.digit) : 0u, valid, cnt[wv], old[u - c0], pk[u]);
            }
#pragma unroll
            for (int u = c0; u < c0 + RCH; u++) pk[u] = (pk[u] & 0xFFu) | (rank_finish(old[u - c0], pk[u]) << 8);
        }
        __syncthreads();
        // per-digit wave prefixes and the tile total (digit lanes)
        uint32_t tot = 0;
        if (dl) {
#pragma unroll
            for (int j = 0; j < NW; j++) {
                const uint32_t cj = cnt[j][tid];
                cnt[j][tid] = tot;
                tot += cj;
            }
        }
        const uint32_t lb = block_excl_scan<NW>(tot, tmp);
        if (dl) lbase[tid] = lb;
        __syncthreads();
        // keys to their slots in the tile (digit-major), freeing their registers
#pragma unroll
        for (int u = 0; u < ITEMS; u++) {
            const uint32_t q = wv * (ITEMS * 64) + u * 64 + lane;
            if (q < nvalid) {
                const uint32_t d = pk[u] & 0xFFu;
                const uint32_t pos = lbase[d] + cnt[wv][d] + (pk[u] >> 8);
                sH[pos] = h[u];
                sL[pos] = l[u];
            }
        }
        if (dl) gbase[tid] = sg.start + toff - lb;
        __syncthreads();
        uint64_t *Hd = w.H[next_buf(sg.buf)];
        uint64_t *Ld = w.L[next_buf(sg.buf)];
#pragma unroll
        for (int u = 0; u < ITEMS; u++) {
            const uint32_t q = u * WG + tid;
            if (q < nvalid) {
                const uint64_t hh = sH[q], ll = sL[q];
                const uint64_t dst = gbase[digit_at(hh, ll, sg.spos, tu.digit)] + q;
                if (dst >= sg.start && dst < seg_end) {
                    Hd[dst] = hh;
                    Ld[dst] = ll;
                } else {
                    atomicOr(&w.ctl->guard, 32u);
                }
            }
        }
    }
    // set up level lev + 1: tile map and zeroed histogram replicas of its buckets
    const uint32_t tid = threadIdx.x;
    const uint32_t nn = min(w.ctl->nseg[lev + 1], w.max_seg);
    for (uint32_t s2 = blockIdx.x; s2 < nn; s2 += gridDim.x) {
        const Seg g = w.segs[(lev + 1) & 1][s2];
        if (g.count == 0 || (uint64_t)g.first_tile + g.ntiles > w.max_tiles ||
            (uint64_t)g.rep_first + g.nrep > w.max_reps)
            continue;
        for (uint32_t t = tid; t < g.ntiles; t += WG) w.tile_seg[(lev + 1) & 1][g.first_tile + t] = s2;
        uint32_t *rp = w.rep[(lev + 1) & 1] + (size_t)g.rep_first * kRepWords;
        for (uint32_t i = tid; i < g.nrep * kRepWords; i += WG) rp[i] = 0;
    }
}

// ---------------------------------------------------------------------------
// k_local: small buckets sorted inside one workgroup's LDS



constexpr int kStack = kLocalCap / 2;



// A task descriptor made uniform across the workgroup; ok false (and count 0)
// when it lies outside the tuple space (defence against a fired capacity guard).
struct LTask {
    uint64_t start;
    uint32_t count;
    uint32_t buf, flags, req;
    bool ok;
};

// dw: lane k of every wave holds dword k (k < 4) of the raw descriptor
__device__ __forceinline__ LTask task_of(const Work &w, uint32_t dw) {
    LTask t;
    t.start = ((uint64_t)__builtin_amdgcn_readlane(dw, 1) << 32) | __builtin_amdgcn_readlane(dw, 0);
    t.count = __builtin_amdgcn_readlane(dw, 2);
    const uint32_t x = __builtin_amdgcn_readlane(dw, 3);
    t.buf = x & 0xFFu;
    t.flags = (x >> 8) & 0xFFu;
    t.req = x >> 16;
    t.ok = t.start + t.count <= w.n && t.buf <= 1 && t.count <= (uint32_t)kLocalCap;
    if (!t.ok) t.count = 0;
    return t;
}

// Small buckets, each sorted in one workgroup's LDS; the sorted order (record
// index per output position) goes to idx for the gather.  Three tasks are in
// flight per workgroup: the current one sorts in LDS while the next one's keys
// and the one after's descriptor load, and the id after that comes from the
// task counter.  Every global load is a branch-free buffer load issued after
// the counter's atomic, so no wait inside the sort stalls on them.
// Bits [pos, pos + 8) of the 112-bit tuple (the 80 key bits, then the 32-bit
// record index), most significant bit first; pos < 112.  Tuples are unique, so
// an order on them needs no stable partition.
__device__ __forceinline__ uint32_t tuple_digit(uint64_t h, uint64_t l, uint32_t pos) {
    const uint64_t l2 = l << 16;
    uint64_t v;
    if (pos == 0) v = h;
    else if (pos < 64) v = (h << pos) | (l2 >> (64 - pos));
    else v = l2 << (pos - 64);
    return (uint32_t)(v >> 56);
}

constexpr uint64_t kLowMask48 = 0xFFFFFFFFFFFFull;

// LWG threads, kLocalCap / LWG keys each; the 256 digit lanes of a partition
// step are threads 0..255.  Keys are ordered as whole (key, index) tuples:
// radix partitions on the tuple's first varying bit (placement inside a digit
// is by LDS atomics, not stable) down to tiny sub-buckets, whose members are
// placed by counting smaller tuples.
template <int LWG, int MINB>
__global__ __launch_bounds__(LWG, MINB) void k_local(Work w, Tune tu, int gate, int part) {
    constexpr int NW = LWG / 64;
    constexpr int LI = kLocalCap / LWG;
    __shared__ ulonglong2 sK[kLocalCap];  // (H, L) of each tuple, one 16-byte LDS access
    __shared__ uint32_t segb[kLocalCap];   // sub-bucket [lo, hi) per position (lo | hi << 16); then the order
    __shared__ uint32_t cnt[kRadix];
    __shared__ uint32_t lbase[kRadix];
    __shared__ uint32_t ltot[kRadix];
    __shared__ uint32_t stk[kStack];
    __shared__ uint64_t orh[NW], andh[NW], orl[NW], andl[NW];
    __shared__ int stk_n;
    __shared__ uint32_t s_next;
    __shared__ uint32_t s_d0;  // record pool: the task's leading digit (one first-pass bucket)

    // a first part of a two-part sort stands down when deeper levels remain
    if (gate < kMaxLev && w.ctl->nseg[gate] > 0) return;
    const uint32_t ntask = min(w.ctl->ntask[part], w.max_tasks);
    uint32_t *const task_ctr = &w.ctl->task_ctr[part];
    const uint32_t nreq = w.hdr->nreq;
    const uint32_t tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const __amdgpu_buffer_rsrc_t r_tasks =
        rsrc_of(w.tasks + (size_t)part * w.max_tasks, ntask * (uint32_t)sizeof(Task));
    const __amdgpu_buffer_rsrc_t r_reqs = rsrc_of(w.reqs, nreq * (uint32_t)sizeof(Req));

    uint64_t ph[LI], pl[LI];  // keys of the task after the current one
    uint32_t nd;              // raw descriptor of the task after that (dword lane & 3)
    uint32_t rq;              // (start, n) of the request of the keys in flight (dword lane & 3)
    auto issue_keys = [&](const LTask &t) {
        const __amdgpu_buffer_rsrc_t rh = rsrc_of(w.H[t.buf & 1] + t.start, t.count * 8u);
        const __amdgpu_buffer_rsrc_t rl = rsrc_of(w.L[t.buf & 1] + t.start, t.count * 8u);
#pragma unroll
        for (int u = 0; u < LI; u++) {
            const uint32_t q = u * LWG + tid;
            const auto vh = __builtin_amdgcn_raw_buffer_load_b64(rh, q * 8u, 0, 0);
            const auto vl = __builtin_amdgcn_raw_buffer_load_b64(rl, q * 8u, 0, 0);
            ph[u] = ((uint64_t)vh[1] << 32) | vh[0];
            pl[u] = ((uint64_t)vl[1] << 32) | vl[0];
        }
        rq = __builtin_amdgcn_raw_buffer_load_b32(r_reqs, t.req * (uint32_t)sizeof(Req) + 16u + (lane & 3u) * 4u, 0, 0);
    };
    auto issue_desc = [&](uint32_t id) {
        nd = __builtin_amdgcn_raw_buffer_load_b32(r_tasks, id * (uint32_t)sizeof(Task) + (lane & 3u) * 4u, 0, 0);
    };

    // at most one workgroup per task takes part (the others would only add
    // contention on the task counter)
    if (blockIdx.x >= ntask) return;
    // prologue: the first task's descriptor and keys, the second's descriptor,
    // the third's id; the partition counters start (and stay) at zero
    for (uint32_t i = tid; i < kRadix; i += LWG) cnt[i] = 0;
    if (tid == 0) s_next = atomicAdd(task_ctr, 1u);
    __syncthreads();
    uint32_t j = ufirst(s_next);
    if (j >= ntask) return;
    issue_desc(j);
    LTask cur = task_of(w, nd);
    issue_keys(cur);
    __syncthreads();
    if (tid == 0) s_next = atomicAdd(task_ctr, 1u);
    __syncthreads();
    uint32_t jn = ufirst(s_next);
    issue_desc(jn);
    __syncthreads();
    if (tid == 0) s_next = atomicAdd(task_ctr, 1u);
    __syncthreads();
    LTask nxt = task_of(w, nd);

    while (j < ntask) {
        // the current task: inside its request (the request bounds came with its keys)
        const uint64_t rs = ((uint64_t)__builtin_amdgcn_readlane(rq, 1) << 32) | __builtin_amdgcn_readlane(rq, 0);
        const uint64_t rn = ((uint64_t)__builtin_amdgcn_readlane(rq, 3) << 32) | __builtin_amdgcn_readlane(rq, 2);
        const bool cur_ok = cur.ok && cur.req < nreq && cur.start >= rs && cur.start + cur.count <= rs + rn;
        if (!cur_ok && tid == 0) atomicOr(&w.ctl->guard, 64u);
        const uint32_t m = cur_ok ? cur.count : 0u;
        const bool sorted = (cur.flags & kTaskSorted) || m <= 1;
        // the task's keys into LDS, with the key masks of the whole task
        uint64_t th = 0, tah = ~0ull, tl = 0, tal = ~0ull;
#pragma unroll
        for (int u = 0; u < LI; u++) {
            const uint32_t q = u * LWG + tid;
            if (q == 0 && m > 0) s_d0 = (uint32_t)(ph[u] >> (64 - tu.digit));
            if (q < m) {
                if (sorted) {
                    segb[q] = (uint32_t)pl[u];
                } else {
                    sK[q] = make_ulonglong2(ph[u], pl[u]);
                    segb[q] = q | ((q + 1) << 16);
                    const uint64_t kk = pl[u] & kLowMask48;
                    th |= ph[u]; tah &= ph[u]; tl |= kk; tal &= kk;
                }
            }
        }
        th = wave_or64(th); tah = wave_and64(tah);
        tl = wave_or64(tl); tal = wave_and64(tal);
        if (lane == 0) { orh[wv] = th; andh[wv] = tah; orl[wv] = tl; andl[wv] = tal; }
        if (tid == 0) stk_n = 0;
        // the id three tasks ahead (consumed after the sort), then the next
        // task's keys, then the descriptor of the one after
        uint32_t ahead = 0;
        if (tid == 0) ahead = atomicAdd(task_ctr, 1u);
        issue_keys(nxt);
        __syncthreads();
        const uint32_t jnn = ufirst(s_next);
        issue_desc(jnn);
        // stable-free partition of [a, a + len) by the tuple digit at bit f:
        // LDS-atomic ranks, one wave scans the 256 counts (and pushes the big
        // sub-buckets), then every key moves to its sub-bucket.  cnt is zero
        // on entry; it is zero again on exit.
        auto partition = [&](uint32_t a, uint32_t len, uint32_t f) {
            uint64_t h[LI], l[LI];
            uint32_t dg[LI], rk[LI];
#pragma unroll
            for (int u = 0; u < LI; u++) {
                const uint32_t i = u * LWG + tid;
                const bool valid = i < len;
                const ulonglong2 t = valid ? sK[a + i] : make_ulonglong2(0ull, 0ull);
                h[u] = t.x;
                l[u] = t.y;
                dg[u] = tuple_digit(h[u], l[u], f);
                rk[u] = valid ? atomicAdd(&cnt[dg[u]], 1u) : 0u;
            }
            __syncthreads();
            if (wv == 0) {
                // lane l: digits 4l..4l+3
                uint32_t c4[4], sum = 0;
#pragma unroll
                for (int k2 = 0; k2 < 4; k2++) { c4[k2] = cnt[4 * lane + k2]; sum += c4[k2]; }
                uint32_t base = wave_incl_scan(sum) - sum;
#pragma unroll
                for (int k2 = 0; k2 < 4; k2++) {
                    const uint32_t dd = 4 * lane + k2, c = c4[k2];
                    lbase[dd] = base;
                    ltot[dd] = c;
                    cnt[dd] = 0;
                    if (c > tu.tiny) {
                        const int slot = atomicAdd(&stk_n, 1);
                        if (slot < kStack) stk[slot] = (a + base) | (c << 16);
                        else atomicOr(&w.ctl->guard, 128u);
                    }
                    base += c;
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < LI; u++) {
                const uint32_t i = u * LWG + tid;
                if (i < len) {
                    const uint32_t d = dg[u];
                    const uint32_t np = a + lbase[d] + rk[u];
                    sK[np] = make_ulonglong2(h[u], l[u]);
                    const uint32_t c = ltot[d];
                    const uint32_t lo = a + lbase[d];
                    segb[np] = (c > tu.tiny) ? (np | ((np + 1) << 16)) : (lo | ((lo + c) << 16));
                }
            }
            __syncthreads();
        };
        // first varying tuple bit from the masks in LDS; kKeyBits + 32 if none
        auto varying_bit = [&]() -> uint32_t {
            uint64_t OH = 0, AH = ~0ull, OL = 0, AL = ~0ull;
#pragma unroll
            for (int k2 = 0; k2 < NW; k2++) { OH |= orh[k2]; AH &= andh[k2]; OL |= orl[k2]; AL &= andl[k2]; }
            const uint64_t vh = OH ^ AH, vl = (OL ^ AL) & kLowMask48;
            if (vh) return (uint32_t)__clzll(vh);
            if (vl) return 64u + ((uint32_t)__clzll(vl) - 16u);
            return kKeyBits + 32u;
        };
        if (!sorted) {
            // the whole task, with the masks from the load
            const uint32_t f = varying_bit();
            if (f < kKeyBits + 32u) partition(0u, m, f);
            // sub-buckets above the tiny threshold, depth first
            for (;;) {
                const int nst = min(stk_n, kStack);
                if (nst <= 0) break;
                const uint32_t e = stk[nst - 1];
                __syncthreads();
                if (tid == 0) stk_n = nst - 1;
                const uint32_t a = e & 0xFFFFu, len = e >> 16;
                uint64_t oh = 0, ah = ~0ull, ol = 0, al = ~0ull;
                for (uint32_t q = a + tid; q < a + len; q += LWG) {
                    const ulonglong2 t = sK[q];
                    const uint64_t hh = t.x, kk = t.y & kLowMask48;
                    oh |= hh; ah &= hh; ol |= kk; al &= kk;
                }
                oh = wave_or64(oh); ah = wave_and64(ah);
                ol = wave_or64(ol); al = wave_and64(al);
                if (lane == 0) { orh[wv] = oh; andh[wv] = ah; orl[wv] = ol; andl[wv] = al; }
                __syncthreads();
                const uint32_t f2 = varying_bit();
                if (f2 < kKeyBits + 32u) partition(a, len, f2);
            }
        }
        if (!sorted) {
            // tiny sub-buckets: position = sub-bucket start + number of smaller tuples
            uint32_t fv[LI], iv[LI];
#pragma unroll
            for (int u = 0; u < LI; u++) {
                const uint32_t q = u * LWG + tid;
                fv[u] = q; iv[u] = 0;
                if (q < m) {
                    const uint32_t sb = segb[q], lo = sb & 0xFFFFu, hi = min(sb >> 16, m);
                    const ulonglong2 me = sK[q];
                    const uint64_t kh = me.x, kl = me.y;
                    iv[u] = (uint32_t)kl;
                    if (hi > lo + 1) {
                        // four members per step: their LDS reads overlap
                        uint32_t r = 0, jj = lo;
                        for (; jj + 4 <= hi; jj += 4) {
                            const ulonglong2 o0 = sK[jj], o1 = sK[jj + 1], o2 = sK[jj + 2], o3 = sK[jj + 3];
                            r += (o0.x < kh) || (o0.x == kh && o0.y < kl);
                            r += (o1.x < kh) || (o1.x == kh && o1.y < kl);
                            r += (o2.x < kh) || (o2.x == kh && o2.y < kl);
                            r += (o3.x < kh) || (o3.x == kh && o3.y < kl);
                        }
                        for (; jj < hi; jj++) {
                            const ulonglong2 o = sK[jj];
                            r += (o.x < kh) || (o.x == kh && o.y < kl);
                        }
                        fv[u] = lo + r;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < LI; u++) {
                const uint32_t q = u * LWG + tid;
                if (q < m) segb[fv[u]] = iv[u];
            }
        }
        __syncthreads();
        // the descriptor and id loads of this round have landed (issued before
        // the sort); take them before the stores so no later wait counts stores
        const LTask after = task_of(w, nd);
        if (tid == 0) s_next = ahead;  // every thread read s_next before the sort's first barrier
        {
            // a fixed number of stores per thread; lanes past m are dropped
            const __amdgpu_buffer_rsrc_t ro = rsrc_of(w.idx + cur.start, m * 4u);
            if (w.rpool) {
                // record pool: a tuple's index is its position in its
                // first-pass bucket; the gather wants the pool slot
                const uint32_t C = tu.tile, cshift = 31u - (uint32_t)__builtin_clz(C);
                const uint32_t *ct = w.ctab + (size_t)ufirst(s_d0) * w.ctab_stride;
#pragma unroll
                for (int u = 0; u < LI; u++) {
                    const uint32_t q = u * LWG + tid;
                    uint32_t v = 0;
                    if (q < m) {
                        const uint32_t p = segb[q], j = p >> cshift;
                        const uint32_t c = j < w.ctab_stride ? ct[j] : 0u;
                        v = (c != 0u && c - 1u < w.max_chunks) ? (c - 1u) * C + (p & (C - 1u)) : 0xFFFFFFFFu;
                    }
                    __builtin_amdgcn_raw_buffer_store_b32(v, ro, q * 4u, 0, 0);
                }
            } else {
#pragma unroll
                for (int u = 0; u < LI; u++) {
                    const uint32_t q = u * LWG + tid;
                    __builtin_amdgcn_raw_buffer_store_b32(segb[q], ro, q * 4u, 0, 0);
                }
            }
        }
        __syncthreads();  // segb, s_next and the mask slots are reused by the next task
        cur = nxt;
        nxt = after;
        j = jn;
        jn = jnn;
    }
}

// ---------------------------------------------------------------------------
// k_gather: records in sorted order, out[j] = in[idx[j]] per request.  A
// block copies 256 records with one dword per lane per step, so stores are
// contiguous and each source record is read as whole 100-byte spans.

__device__ __forceinline__ uint32_t find_req(const Req *reqs, uint32_t nreq, uint64_t g) {
    uint32_t lo = 0, hi = nreq - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (reqs[mid].start <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kWG) void k_gather(const Req *reqs, const Hdr *hdr, const uint32_t *idx,
                                                const Ctl *ctl, int gate) {
    __shared__ uint32_t sidx[kWG];
    __shared__ uint32_t s_r0, s_r1;
    if (gate < kMaxLev && ctl->nseg[gate] > 0) return;  // the second part gathers
    const uint64_t n = hdr->n_total;
    const uint32_t nreq = hdr->nreq;
    const uint64_t g0 = (uint64_t)blockIdx.x * kWG;
    if (g0 >= n) return;
    const uint32_t nr = (uint32_t)min<uint64_t>(kWG, n - g0);
    if (threadIdx.x == 0) s_r0 = find_req(reqs, nreq, g0);
    if (threadIdx.x == 64) s_r1 = find_req(reqs, nreq, g0 + nr - 1);
    __syncthreads();
    const uint32_t r0 = __builtin_amdgcn_readfirstlane(s_r0), r1 = __builtin_amdgcn_readfirstlane(s_r1);
    if (r0 == r1) {  // the whole block belongs to one request (the common case)
        const uint8_t *in = reqs[r0].in;
        uint8_t *out = reqs[r0].out;
        const uint64_t rn = reqs[r0].n, rs = reqs[r0].start;
        if (threadIdx.x < nr) {
            const uint32_t ix = idx[g0 + threadIdx.x];
            sidx[threadIdx.x] = ix < rn ? ix : (uint32_t)(g0 + threadIdx.x - rs);
        }
        __syncthreads();
        // request buffers are device memory: global (not flat) accesses, so
        // the waits on the LDS index reads do not also wait on record loads
        const gu32 *src = (const gu32 *)in;
        gu32w *dst = (gu32w *)out + (g0 - rs) * 25;
        uint32_t v[25];
#pragma unroll
        for (int u = 0; u < 25; u++) {
            const uint32_t q = threadIdx.x + kWG * u, r = q / 25u, kk = q - 25u * r;
            if (r < nr) v[u] = src[(uint64_t)sidx[r] * 25 + kk];
        }
        // output lines are written once and not read back here: non-temporal
#pragma unroll
        for (int u = 0; u < 25; u++) {
            const uint32_t q = threadIdx.x + kWG * u, r = q / 25u;
            if (r < nr) __builtin_nontemporal_store(v[u], dst + q);
        }
        return;
    }
    // a block across a request boundary: one record per thread
    if (threadIdx.x < nr) {
        const uint64_t g = g0 + threadIdx.x;
        const uint32_t r = find_req(reqs, nreq, g);
        const Req rq = reqs[r];
        const uint32_t ix = idx[g];
        // a sorted index is always inside its request; fall back to the
        // record itself if a guard fired upstream
        const uint64_t si = ix < rq.n ? ix : (g - rq.start);
        const gu32 *s1 = (const gu32 *)(rq.in + si * kRec);
        gu32w *d1 = (gu32w *)(rq.out + (g - rq.start) * kRec);
        for (int kk = 0; kk < 25; kk++) d1[kk] = s1[kk];
    }
}

// Plain gather for the step-level test entry point.
// TIES: also ties[g] = 1 if output record g has the same key bytes 0..9 as
// output record g - 1 (0 for the first record of the sort); record -1 of a
// launch is idx[-1] when has_prev is set (a later output part).
template <bool TIES>
__device__ __forceinline__ void gather_body(const uint8_t *rec, uint64_t n_rec, const uint32_t *idx, uint8_t *out,
                                            uint64_t n, uint8_t *ties, int has_prev) {
    __shared__ uint32_t sidx[kWG];
    __shared__ uint32_t skey[TIES ? 3 * (kWG / 64) : 1];  // key words of each wave's last record
    const uint64_t g0 = (uint64_t)blockIdx.x * kWG;
    const uint32_t nr = (uint32_t)min<uint64_t>(kWG, n - g0);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(rec);
    // TIES: thread r loads key bytes 0..9 of output record g0 + r (dwords 0, 1
    // and half of 2) apart from the copy below, so the copy keeps the plain
    // gather's registers; the loads hit the lines the copy fetches
    uint32_t k0 = 0, k1 = 0, k2 = 0;
    bool have = false;
    if (threadIdx.x < nr) {
        const uint32_t j = idx[g0 + threadIdx.x];
        sidx[threadIdx.x] = j;
        if (TIES && j < n_rec) {
            k0 = src[(uint64_t)j * 25];
            k1 = src[(uint64_t)j * 25 + 1];
            k2 = src[(uint64_t)j * 25 + 2] & 0xFFFFu;
            have = true;
        }
    }
    __syncthreads();
    uint32_t *dst = reinterpret_cast<uint32_t *>(out) + g0 * 25;
    uint32_t v[25];
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u, r = q / 25u, kk = q - 25u * r;
        v[u] = 0;
        if (r < nr && sidx[r] < n_rec) v[u] = src[(uint64_t)sidx[r] * 25 + kk];
    }
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u, r = q / 25u;
        if (r < nr) __builtin_nontemporal_store(v[u], dst + q);
    }
    if (TIES) {
        // the previous record's key: lane l - 1 of the wave, the last lane of
        // the previous wave through LDS, or (first record of the block) read
        // through the index array (idx[-1]: the last record of the part before)
        const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        uint32_t p0 = __shfl_up(k0, 1), p1 = __shfl_up(k1, 1), p2 = __shfl_up(k2, 1);
        bool phave = __shfl_up(have ? 1 : 0, 1) != 0;
        if (lane == 63) { skey[3 * wv] = have ? k0 : ~0u; skey[3 * wv + 1] = k1; skey[3 * wv + 2] = have ? k2 : ~0u; }
        __syncthreads();
        const uint32_t r = threadIdx.x;
        if (r < nr) {
            const uint64_t g = g0 + r;
            if (lane == 0 && wv > 0) {
                p0 = skey[3 * wv - 3]; p1 = skey[3 * wv - 2]; p2 = skey[3 * wv - 1];
                phave = p2 != ~0u;  // a key's third word has its upper half clear
            } else if (r == 0) {
                phave = false;
                if (g > 0 || has_prev) {
                    const uint32_t j = idx[(int64_t)g - 1];
                    if (j < n_rec) {
                        p0 = src[(uint64_t)j * 25]; p1 = src[(uint64_t)j * 25 + 1]; p2 = src[(uint64_t)j * 25 + 2] & 0xFFFFu;
                        phave = true;
                    }
                }
            }
            ties[g] = (have && phave && p0 == k0 && p1 == k1 && p2 == k2) ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(kWG) void k_gather_plain(const uint8_t *rec, uint64_t n_rec, const uint32_t *idx,
                                                      uint8_t *out, uint64_t n) {
    gather_body<false>(rec, n_rec, idx, out, n, nullptr, 0);
}

// The same gather marking ties with the previous output record (the keyed
// sort's first tie round reads these flags instead of the records).
__global__ __launch_bounds__(kWG) void k_gather_ties(const uint8_t *rec, uint64_t n_rec, const uint32_t *idx,
                                                     uint8_t *out, uint64_t n, uint8_t *ties, int has_prev) {
    gather_body<true>(rec, n_rec, idx, out, n, ties, has_prev);
}

// ---------------------------------------------------------------------------
// launch wrappers

static int occupancy(const void *fn, int cus, int wg = kWG) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, wg, 0) != hipSuccess || per < 1) per = 1;
    return per * cus;
}

// Reports to the host whether level `gate` has big buckets (a second part of
// the sort is needed).  System-scope store: the host reads it after an event.
__global__ void k_flag(Work w, int gate, uint32_t *flag) {
    const uint32_t deep = (gate < kMaxLev && w.ctl->nseg[gate] > 0) ? 1u : 0u;
    __hip_atomic_store(flag, deep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int ITEMS, int SWG, int LWG>
static hipError_t launch_levels(const Work &w, const Tune &t, uint32_t nreq, uint32_t tiles0,
                                hipStream_t s, int cus, hipEvent_t *ev, const Stage &st) {
    constexpr int SITEMS = ITEMS * kWG / SWG;  // same tile, SWG threads
    // grid sizes from the occupancy of each kernel (static locals: initialised
    // once, safely under concurrent first calls)
    static const int g_sc = occupancy(reinterpret_cast<const void *>(&k_scatter<SITEMS, SWG>), cus, SWG);
    static const int g_hist = occupancy(reinterpret_cast<const void *>(&k_hist<ITEMS>), cus);
    static const int g_loc = occupancy(reinterpret_cast<const void *>(&k_local<LWG, LWG == 512 ? 2 : 3>), cus, LWG);
    const bool fused = st.head && st.first != kFirstSplit;
    if (fused) {
        // one request of w.n records; the workspace was laid out for this first pass
        const uint32_t ft = fuse_tile(st.first);
        const uint64_t nft = (w.n + ft - 1) / ft;
        k_init<<<dim3(1), dim3(kWG), 0, s>>>(w);
        k_fzero<<<dim3(cus * 4), dim3(kWG), 0, s>>>(w.status, nft * kRadix, w.ctab,
                                                    (uint64_t)kRadix * w.ctab_stride);
        // one workgroup per CU (the staging takes most of the LDS); tiles from a counter
        if (st.first == kFirstRecords)
            k_fuse0<kFuseWG, fuse_items(kFirstRecords), true><<<dim3(cus), dim3(kFuseWG), 0, s>>>(w, t);
        else
            k_fuse0<kFuseWG, fuse_items(kFirstFused), false><<<dim3(cus), dim3(kFuseWG), 0, s>>>(w, t);
        k_plan0<<<dim3(cus * 2), dim3(kWG), 0, s>>>(w, t, ft);
    } else if (st.head) {
        // nreq / tiles0 == 0: sizes known only on the device (captured sequences)
        k_init<<<dim3(nreq ? max(1u, min(nreq, 1024u)) : 1024u), dim3(kWG), 0, s>>>(w);
        if (st.tuples_in) {  // tuples already in buffer 0: level 0 starts with its histogram pass
            k_hist<ITEMS><<<dim3(g_hist), dim3(kWG), 0, s>>>(w, t, 0);
        } else {
            const int g_ext = tiles0 ? (int)max(1u, min(tiles0, (uint32_t)(cus * 16))) : cus * 16;
            k_extract<ITEMS><<<dim3(g_ext), dim3(kWG), 0, s>>>(w, t);
        }
    }
    if (ev) (void)hipEventRecord(ev[0], s);
    const int g_plan = cus * 4;
    const int lev_end = min(st.lev_end, levels_for((int)t.digit));
    for (int lev = fused ? max(st.lev_begin, 1) : st.lev_begin; lev < lev_end; lev++) {
        if (lev > 0) k_hist<ITEMS><<<dim3(g_hist), dim3(kWG), 0, s>>>(w, t, lev);
        k_plan<<<dim3(g_plan), dim3(kWG), 0, s>>>(w, t, lev);
        k_scatter<SITEMS, SWG><<<dim3(g_sc), dim3(SWG), 0, s>>>(w, t, lev);
    }
    if (st.flag) k_flag<<<dim3(1), dim3(1), 0, s>>>(w, st.gate, st.flag);
    if (ev) (void)hipEventRecord(ev[1], s);
    if (st.tail) k_local<LWG, LWG == 512 ? 2 : 3><<<dim3(g_loc), dim3(LWG), 0, s>>>(w, t, st.gate, 0);
    if (ev) (void)hipEventRecord(ev[2], s);
    return hipGetLastError();
}

template <int ITEMS, int SWG>
static hipError_t by_local(const Work &w, const Tune &t, uint32_t nreq, uint32_t tiles0, hipStream_t s, int cus,
                           hipEvent_t *ev, const Stage &st) {
    return t.local_wg == 512 ? launch_levels<ITEMS, SWG, 512>(w, t, nreq, tiles0, s, cus, ev, st)
                             : launch_levels<ITEMS, SWG, 256>(w, t, nreq, tiles0, s, cus, ev, st);
}

template <int ITEMS>
static hipError_t by_scatter(const Work &w, const Tune &t, uint32_t nreq, uint32_t tiles0, hipStream_t s, int cus,
                             hipEvent_t *ev, const Stage &st) {
    switch (t.scatter_wg) {
    case 256: return by_local<ITEMS, 256>(w, t, nreq, tiles0, s, cus, ev, st);
    case 512: return by_local<ITEMS, 512>(w, t, nreq, tiles0, s, cus, ev, st);
    default: return by_local<ITEMS, 1024>(w, t, nreq, tiles0, s, cus, ev, st);
    }
}

hipError_t launch_sort_core(const Work &w, const Tune &t, uint32_t nreq, uint32_t tiles0, hipStream_t s,
                            int cus, hipEvent_t *ev, const Stage &st) {
    switch (t.tile_items) {
    case 8: return by_scatter<8>(w, t, nreq, tiles0, s, cus, ev, st);
    case 16: return by_scatter<16>(w, t, nreq, tiles0, s, cus, ev, st);
    default: return by_scatter<32>(w, t, nreq, tiles0, s, cus, ev, st);
    }
}

hipError_t launch_gather_batch(const Work &w, hipStream_t s, int gate) {
    // one block per 256 records of the workspace capacity; blocks past the
    // batch's record count exit at once
    const uint64_t blocks = (w.n + kWG - 1) / kWG;
    k_gather<<<dim3((uint32_t)(blocks < 1 ? 1 : blocks)), dim3(kWG), 0, s>>>(w.reqs, w.hdr, w.idx, w.ctl, gate);
    return hipGetLastError();
}

template <int LWG>
static hipError_t local_part(const Work &w, const Tune &t, hipStream_t s, int cus, int part) {
    constexpr int MINB = LWG == 512 ? 2 : 3;
    static const int g_loc = occupancy(reinterpret_cast<const void *>(&k_local<LWG, MINB>), cus, LWG);
    k_local<LWG, MINB><<<dim3(g_loc), dim3(LWG), 0, s>>>(w, t, kMaxLev, part);
    return hipGetLastError();
}

hipError_t launch_local_part(const Work &w, const Tune &t, hipStream_t s, int cus, int part) {
    if (part < 0 || part >= (int)w.nparts) return hipErrorInvalidValue;
    return t.local_wg == 512 ? local_part<512>(w, t, s, cus, part) : local_part<256>(w, t, s, cus, part);
}

hipError_t launch_gather_single(const uint8_t *rec, uint64_t n_rec, const uint32_t *idx, uint8_t *out,
                                uint64_t n, hipStream_t s, uint8_t *ties, bool has_prev) {
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + kWG - 1) / kWG;
    if (ties)
        k_gather_ties<<<dim3((uint32_t)blocks), dim3(kWG), 0, s>>>(rec, n_rec, idx, out, n, ties, has_prev ? 1 : 0);
    else
        k_gather_plain<<<dim3((uint32_t)blocks), dim3(kWG), 0, s>>>(rec, n_rec, idx, out, n);
    return hipGetLastError();
}

}  // namespace ley
