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
// workspace, plus the record's position.  One sort of the tuples (the in-HBM
// sort's partition and local-sort stages, no record gather) orders every run
// by its next six key bytes at once: the run number keeps runs apart and in
// place, and equal keys keep entry order, which is position order and so
// input order.  The records of the runs are then gathered in the sorted order
// and written back over their runs.  A tie on [0, P + 6) implies a tie on
// [0, P), so a round looks only at the previous round's entries: in sorted
// order they describe the records now at consecutive positions of each run,
// and two neighbours tie exactly when their entries' keys agree.  The first round's ties come
// from the prefix sort itself: its record gather marks every output record
// whose key bytes 0..9 equal those of the record before it, so no round reads
// the records to find ties.  Rounds stop when no run is left or P reaches K.  The
// host reads the entry count of each round (one stream synchronisation per
// round).
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace ley {
namespace {

constexpr int kTB = 256;                // threads per block
constexpr int kTPer = 4;                // positions per thread
constexpr int kTSpan = kTB * kTPer;     // positions per block
constexpr int kRecWords = kRec / 4;     // dwords per record
constexpr uint32_t kWindow = 6;         // key bytes resolved per round

constexpr int kTWaves = kTB / 64;

// Exclusive counts of two flags over the block's threads in thread order (a
// ballot and a bit count per wave, then the waves' totals through LDS);
// *ta, *tb get the block totals.  Whole block.
__device__ __forceinline__ void block_count2(bool fa, bool fb, uint32_t *ea, uint32_t *eb, uint32_t *ta,
                                             uint32_t *tb) {
    __shared__ uint32_t wa[kTWaves], wb[kTWaves];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t ba = __ballot(fa), bb = __ballot(fb);
    const uint32_t below_a = __builtin_amdgcn_mbcnt_hi((uint32_t)(ba >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ba, 0u));
    const uint32_t below_b = __builtin_amdgcn_mbcnt_hi((uint32_t)(bb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bb, 0u));
    if (lane == 0) {
        wa[w] = (uint32_t)__popcll(ba);
        wb[w] = (uint32_t)__popcll(bb);
    }
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
    *ea = pa + below_a;
    *eb = pb + below_b;
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

// Candidate c is inside a run of at least two (it ties with a neighbour) and
// whether such a run starts there.
__device__ __forceinline__ void run_flags(const uint8_t *P, uint64_t nc, uint64_t c, bool *in_run, bool *starts) {
    const bool eq_prev = c > 0 && P[c] != 0;
    const bool eq_next = c + 1 < nc && P[c + 1] != 0;
    *in_run = eq_prev || eq_next;
    *starts = eq_next && !eq_prev;
}

// Per block of kTSpan candidates: candidates inside runs and run starts.
__global__ __launch_bounds__(kTB) void k_tie_count(const uint8_t *P, uint64_t nc, uint32_t *cnt_in,
                                                   uint32_t *cnt_start) {
    const uint64_t base = (uint64_t)blockIdx.x * kTSpan;
    uint32_t ci = 0, cs = 0;
    for (int u = 0; u < kTPer; u++) {
        const uint64_t c = base + (uint64_t)u * kTB + threadIdx.x;
        if (c < nc) {
            bool r, s;
            run_flags(P, nc, c, &r, &s);
            ci += r;
            cs += s;
        }
    }
    __shared__ uint32_t s_i, s_s;
    if (threadIdx.x == 0) { s_i = 0; s_s = 0; }
    __syncthreads();
    ci = __ockl_wfred_add_u32(ci);
    cs = __ockl_wfred_add_u32(cs);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_i, ci);
        atomicAdd(&s_s, cs);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt_in[blockIdx.x] = s_i;
        cnt_start[blockIdx.x] = s_s;
    }
}

// One block: exclusive scans of both per-block counts (each thread sums a
// contiguous range of blocks, the range totals are scanned in LDS, then each
// thread writes its range's offsets); totals[0] = positions inside runs,
// totals[1] = runs.
constexpr int kSB = 1024;
__global__ __launch_bounds__(kSB) void k_tie_scan(const uint32_t *cnt_in, const uint32_t *cnt_start, uint64_t nb,
                                                  uint64_t *off_in, uint64_t *off_start, uint64_t *totals) {
    __shared__ uint64_t si[kSB], ss[kSB];
    const uint32_t t = threadIdx.x;
    const uint64_t per = (nb + kSB - 1) / kSB;
    const uint64_t b0 = min(nb, (uint64_t)t * per), b1 = min(nb, b0 + per);
    constexpr int kG = 16;  // loads in flight per thread
    uint64_t ti = 0, ts = 0;
    for (uint64_t b = b0; b < b1; b += kG) {
        uint32_t vi[kG], vs[kG];
#pragma unroll
        for (int k = 0; k < kG; k++) {
            vi[k] = b + k < b1 ? cnt_in[b + k] : 0u;
            vs[k] = b + k < b1 ? cnt_start[b + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kG; k++) { ti += vi[k]; ts += vs[k]; }
    }
    si[t] = ti;
    ss[t] = ts;
    __syncthreads();
    for (uint32_t off = 1; off < (uint32_t)kSB; off <<= 1) {
        const uint64_t ai = t >= off ? si[t - off] : 0ull, as = t >= off ? ss[t - off] : 0ull;
        __syncthreads();
        si[t] += ai;
        ss[t] += as;
        __syncthreads();
    }
    uint64_t ci = si[t] - ti, cs = ss[t] - ts;
    for (uint64_t b = b0; b < b1; b += kG) {
        uint32_t vi[kG], vs[kG];
#pragma unroll
        for (int k = 0; k < kG; k++) {
            vi[k] = b + k < b1 ? cnt_in[b + k] : 0u;
            vs[k] = b + k < b1 ? cnt_start[b + k] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kG; k++) {
            if (b + k < b1) {
                off_in[b + k] = ci;
                off_start[b + k] = cs;
            }
            ci += vi[k];
            cs += vs[k];
        }
    }
    if (t == kSB - 1) {
        totals[0] = si[t];
        totals[1] = ss[t];
    }
}

// Entries of the round: for candidate c inside a run, entry t (its rank among
// such candidates) gets the tuple key = run number (big-endian) + key bytes
// [p, p + 6) of the record at its position j, masked to the key, with index t
// (TH[t], TL[t]: the sort's tuple words), the same key in Kh[t], Kl[t] (kept
// for the next round's tie marks), and dest[t] = j.  j = c in the first round,
// else the previous round's dest[c].
__global__ __launch_bounds__(kTB) void k_tie_emit(const uint32_t *A, const uint8_t *P, uint64_t nc,
                                                  const uint64_t *cand, uint32_t p, uint32_t key_bytes,
                                                  const uint64_t *off_in, const uint64_t *off_start, uint64_t *TH,
                                                  uint64_t *TL, uint64_t *Kh, uint32_t *Kl, uint64_t *dest) {
    const uint64_t base = (uint64_t)blockIdx.x * kTSpan;
    uint64_t ci = off_in[blockIdx.x], cs = off_start[blockIdx.x];
    const uint8_t *Ab = reinterpret_cast<const uint8_t *>(A);
    for (int u = 0; u < kTPer; u++) {
        const uint64_t c = base + (uint64_t)u * kTB + threadIdx.x;
        bool r = false, s = false;
        if (c < nc) run_flags(P, nc, c, &r, &s);
        uint32_t ei, es, ti, ts;
        block_count2(r, s, &ei, &es, &ti, &ts);
        if (r) {
            const uint64_t t = ci + ei;
            const uint64_t j = cand ? cand[c] : c;
            // the run holding c began at the latest start at or before c
            const uint32_t run = (uint32_t)(cs + es + (s ? 1u : 0u) - 1u);
            uint8_t kb[kWindow];
            for (uint32_t k = 0; k < kWindow; k++) {
                const uint32_t b = p + k;
                kb[k] = b < key_bytes ? Ab[j * kRec + b] : (uint8_t)0;
            }
            const uint64_t h = ((uint64_t)run << 32) | ((uint32_t)kb[0] << 24) | ((uint32_t)kb[1] << 16) |
                               ((uint32_t)kb[2] << 8) | (uint32_t)kb[3];
            const uint32_t w = ((uint32_t)kb[4] << 8) | (uint32_t)kb[5];
            TH[t] = h;
            TL[t] = ((uint64_t)w << 32) | (uint32_t)t;
            Kh[t] = h;
            Kl[t] = w;
            dest[t] = j;
        }
        ci += ti;
        cs += ts;
    }
}

// Sorted entries q of a block of kTB (idx[q] = the entry number t): out[q] =
// A[dest[t]] and the entry's key in SKh[q], SKl[q] (sorted order, for the next
// round's tie marks).  Each thread looks up one entry's position into LDS,
// then the block copies its records a dword per thread (contiguous stores).
// An entry number or position out of range, which only a failed entry sort
// could leave, is not read: it sets *err, and the call reports
// LEYENDA_EINTERNAL.
__global__ __launch_bounds__(kTB) void k_tie_gather(const uint32_t *A, uint64_t n, const uint32_t *idx,
                                                    const uint64_t *dest, const uint64_t *Kh, const uint32_t *Kl,
                                                    uint64_t m, uint32_t *out, uint64_t *SKh, uint32_t *SKl,
                                                    uint32_t *err) {
    __shared__ uint64_t sj[kTB];
    const uint64_t q0 = (uint64_t)blockIdx.x * kTB;
    const uint32_t nr = (uint32_t)min<uint64_t>(kTB, m - q0);
    if (threadIdx.x < nr) {
        const uint64_t q = q0 + threadIdx.x;
        const uint32_t t = idx[q];
        uint64_t j = ~0ull;
        if (t < m) {
            j = dest[t];
            SKh[q] = Kh[t];
            SKl[q] = Kl[t];
        }
        if (j >= n) { atomicOr(err, 1u << 16); j = ~0ull; }
        sj[threadIdx.x] = j;
    }
    __syncthreads();
    uint32_t *o = out + q0 * kRecWords;
    uint32_t v[kRecWords];  // every load of the thread in flight before the stores
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u, r = g / kRecWords, d = g - r * kRecWords;
        v[u] = 0;
        if (r < nr && sj[r] != ~0ull) v[u] = A[sj[r] * kRecWords + d];
    }
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u, r = g / kRecWords;
        if (r < nr && sj[r] != ~0ull) o[g] = v[u];
    }
}

// A[dest[t]] = R[t] for the entries t of a block of kTB (positions through LDS).
__global__ __launch_bounds__(kTB) void k_tie_scatter(const uint32_t *R, const uint64_t *dest, uint64_t m,
                                                     uint64_t n, uint32_t *A) {
    __shared__ uint64_t sj[kTB];
    const uint64_t t0 = (uint64_t)blockIdx.x * kTB;
    const uint32_t nr = (uint32_t)min<uint64_t>(kTB, m - t0);
    if (threadIdx.x < nr) sj[threadIdx.x] = dest[t0 + threadIdx.x];
    __syncthreads();
    const uint32_t *rr = R + t0 * kRecWords;
    uint32_t v[kRecWords];
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u;
        v[u] = g < nr * (uint32_t)kRecWords ? rr[g] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kRecWords; u++) {
        const uint32_t g = threadIdx.x + kTB * u, r = g / kRecWords, d = g - r * kRecWords;
        if (r < nr && sj[r] < n) A[sj[r] * kRecWords + d] = v[u];
    }
}

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// Scratch of the tie rounds, from the stream's pooled slot 0 (kept between
// calls): the tie marks (n bytes), the per-block counts and offsets of the
// run numbering, and the totals + error word.
struct RoundTables {
    uint8_t *P;
    uint32_t *cnt_in, *cnt_start;
    uint64_t *off_in, *off_start, *totals;
};

size_t tables_bytes(uint64_t n) {
    const uint64_t nb = (n + kTSpan - 1) / kTSpan;
    return a256(n) + 2 * a256(nb * 4) + 2 * a256(nb * 8) + 256;
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
    r.totals = reinterpret_cast<uint64_t *>(b);  // tie count, run count, error word
    return r;
}

// Rounds over the tie runs of the prefix-sorted records in A (n records);
// tb.P (n bytes) holds the first round's tie marks and is reused by later
// rounds.  The entries live in the stream's pooled slot 1.
int resolve_ties(uint32_t *A, uint64_t n, uint32_t key_bytes, hipStream_t s, const Tune &t, const RoundTables &tb) {
    int rc;
    uint8_t *P = tb.P;
    uint32_t *cnt_in = tb.cnt_in, *cnt_start = tb.cnt_start;
    uint64_t *off_in = tb.off_in, *off_start = tb.off_start;
    uint64_t *totals = tb.totals;
    // error word next to the totals: the sorts' device-side guard words
    // (capacity guards, bounded waits) and the entry gather's bound check
    uint32_t *err = reinterpret_cast<uint32_t *>(totals + 2);
    hipError_t e0 = hipMemsetAsync(err, 0, 4, s);
    if (e0 != hipSuccess) return hip_fail(e0, "leyenda_sort_keyed: error word");
    if ((rc = guard_or_pooled(s, err))) return rc;  // the prefix sort
    // scratch of the rounds (room for the first round's count, which is the largest):
    // the entry sort's workspace, the entries' keys (Kh, Kl) and in sorted order
    // (SKh, SKl), the records of the runs in sorted order (R), the entries' positions
    char *ws = nullptr;
    uint64_t *Kh = nullptr, *SKh = nullptr;
    uint32_t *Kl = nullptr, *SKl = nullptr, *R = nullptr;
    uint64_t *dest[2] = {nullptr, nullptr};  // positions of the entries, by round parity
    uint64_t cap = 0, nc = n;
    int r = 0;
    for (uint32_t p = kKeyBytes; p < key_bytes; p += kWindow, r++) {
        const uint64_t nb = (nc + kTSpan - 1) / kTSpan;
        if (r) k_tie_eq<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(SKh, SKl, nc, P);
        k_tie_count<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(P, nc, cnt_in, cnt_start);
        k_tie_scan<<<dim3(1), dim3(kSB), 0, s>>>(cnt_in, cnt_start, nb, off_in, off_start, totals);
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
            if ((rc = get_aux(s, 1, wsb + 2 * a256(cap * 8) + 2 * a256(cap * 4) + a256(cap * kRec) + 2 * a256(cap * 8),
                              &base)))
                return rc;
            char *b = static_cast<char *>(base);
            ws = b; b += wsb;
            Kh = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            SKh = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            Kl = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            SKl = reinterpret_cast<uint32_t *>(b); b += a256(cap * 4);
            R = reinterpret_cast<uint32_t *>(b); b += a256(cap * kRec);
            dest[0] = reinterpret_cast<uint64_t *>(b); b += a256(cap * 8);
            dest[1] = reinterpret_cast<uint64_t *>(b);
        }
        // the entries go straight into the tuple buffers of a workspace laid out for m tuples
        const Layout Lm = plan_layout(m, 1, t);
        uint64_t *TH = reinterpret_cast<uint64_t *>(ws + Lm.off_H0);
        uint64_t *TL = reinterpret_cast<uint64_t *>(ws + Lm.off_L0);
        const uint32_t *idx = reinterpret_cast<const uint32_t *>(ws + Lm.off_idx);
        k_tie_emit<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(A, P, nc, r ? dest[(r - 1) & 1] : nullptr, p, key_bytes,
                                                             off_in, off_start, TH, TL, Kh, Kl, dest[r & 1]);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: entries");
        if ((rc = sort_tuples_ws(m, s, t, ws))) return rc;
        if ((e = launch_guard_or(ws, m, t, err, s)) != hipSuccess) return hip_fail(e, "guard kernel");
        const uint64_t blocks = (m + kTB - 1) / kTB;
        k_tie_gather<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(A, n, idx, dest[r & 1], Kh, Kl, m, R, SKh, SKl, err);
        k_tie_scatter<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(R, dest[r & 1], m, n, A);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: permute");
        nc = m;  // the next round looks only inside these runs
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
    return resolve_ties(static_cast<uint32_t *>(out_dev), n, key_bytes, s, t, tb);
}
