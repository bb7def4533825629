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
// per-block counts), then writes for every record inside a run a 100-byte
// entry whose 10-byte key is the run number (big-endian 32 bits) followed by
// key bytes [P, P + 6) of the record (bytes at or past K read as zero), with
// the record's output position in entry bytes 12..19 (the rest of the entry is
// left unwritten).  One stable sort of the
// entries (the in-HBM sort) orders every run by its next six key bytes at
// once: the run number keeps runs apart and in place, and equal entries keep
// position order, which is input order.  The records of the runs are then
// gathered in the entries' order and written back over their runs.  A tie on
// [0, P + 6) implies a tie on [0, P), so a round looks only at the previous
// round's entries: in sorted order they describe the records now at
// consecutive positions of each run, and two neighbours tie exactly when their
// entries agree on run number and window bytes.  The first round's ties come
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

// Exclusive scan over the block's threads (one value each); *total gets the sum.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *total) {
    __shared__ uint32_t s[kTB];
    const uint32_t t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (uint32_t off = 1; off < (uint32_t)kTB; off <<= 1) {
        const uint32_t add = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    const uint32_t incl = s[t];
    *total = s[kTB - 1];
    __syncthreads();
    return incl - v;
}

// Candidates c = 0..nc-1 of a round, in output-position order; P[c] = 1 if
// candidate c holds the record right after candidate c - 1's and ties with it
// on the key bytes sorted so far.  First round: candidate c is output position
// c and the prefix sort's record gather writes P.  Later rounds (this kernel):
// the candidates are the previous round's entries in sorted order (E2), whose
// records now sit at consecutive positions within each run; c ties with c - 1
// when their entries agree on run number and window bytes (entry bytes 0..9).
__global__ __launch_bounds__(kTB) void k_tie_eq(const uint32_t *E2, uint64_t nc, uint8_t *P) {
    const uint64_t base = (uint64_t)blockIdx.x * kTSpan;
    for (int u = 0; u < kTPer; u++) {
        const uint64_t c = base + (uint64_t)u * kTB + threadIdx.x;
        if (c >= nc) continue;
        bool eq = false;
        if (c > 0) {
            const uint32_t *b = E2 + c * kRecWords, *a = b - kRecWords;
            eq = ((a[0] ^ b[0]) | (a[1] ^ b[1]) | ((a[2] ^ b[2]) & 0xFFFFu)) == 0;
        }
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
    uint32_t ti, ts;
    (void)block_scan_excl(ci, &ti);
    (void)block_scan_excl(cs, &ts);
    if (threadIdx.x == 0) {
        cnt_in[blockIdx.x] = ti;
        cnt_start[blockIdx.x] = ts;
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
    uint64_t ti = 0, ts = 0;
    for (uint64_t b = b0; b < b1; b++) {
        ti += cnt_in[b];
        ts += cnt_start[b];
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
    for (uint64_t b = b0; b < b1; b++) {
        off_in[b] = ci;
        off_start[b] = cs;
        ci += cnt_in[b];
        cs += cnt_start[b];
    }
    if (t == kSB - 1) {
        totals[0] = si[t];
        totals[1] = ss[t];
    }
}

// Entries of the round: for candidate c inside a run, entry t (its rank among
// such candidates) gets key = run number (big-endian) + key bytes [p, p + 6)
// of the record at its position j, masked to the key, and j in bytes 12..19;
// dest[t] = j.  j = c in the first round, else the previous round's dest[c].
__global__ __launch_bounds__(kTB) void k_tie_emit(const uint32_t *A, const uint8_t *P, uint64_t nc,
                                                  const uint64_t *cand, uint32_t p, uint32_t key_bytes,
                                                  const uint64_t *off_in, const uint64_t *off_start, uint32_t *E,
                                                  uint64_t *dest) {
    const uint64_t base = (uint64_t)blockIdx.x * kTSpan;
    uint64_t ci = off_in[blockIdx.x], cs = off_start[blockIdx.x];
    const uint8_t *Ab = reinterpret_cast<const uint8_t *>(A);
    for (int u = 0; u < kTPer; u++) {
        const uint64_t c = base + (uint64_t)u * kTB + threadIdx.x;
        bool r = false, s = false;
        if (c < nc) run_flags(P, nc, c, &r, &s);
        uint32_t ti, ts;
        const uint32_t ei = block_scan_excl(r ? 1u : 0u, &ti);
        const uint32_t es = block_scan_excl(s ? 1u : 0u, &ts);
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
            uint32_t *e = E + t * kRecWords;
            e[0] = __builtin_bswap32(run);
            e[1] = (uint32_t)kb[0] | ((uint32_t)kb[1] << 8) | ((uint32_t)kb[2] << 16) | ((uint32_t)kb[3] << 24);
            e[2] = (uint32_t)kb[4] | ((uint32_t)kb[5] << 8);
            e[3] = (uint32_t)j;
            e[4] = (uint32_t)(j >> 32);
            dest[t] = j;  // entry bytes 20..99 are not written: the sort carries them, nothing reads them
        }
        ci += ti;
        cs += ts;
    }
}

// out[t] = A[position held by sorted entry t], one dword per thread.  A
// position outside the n records, which only a failed entry sort could leave,
// is not read: it sets *err, and the call reports LEYENDA_EINTERNAL.
__global__ __launch_bounds__(kTB) void k_tie_gather(const uint32_t *A, uint64_t n, const uint32_t *E2, uint64_t m,
                                                    uint32_t *out, uint32_t *err) {
    const uint64_t g = (uint64_t)blockIdx.x * kTB + threadIdx.x;
    if (g >= m * kRecWords) return;
    const uint64_t t = g / kRecWords, d = g - t * kRecWords;
    const uint64_t j = (uint64_t)E2[t * kRecWords + 3] | ((uint64_t)E2[t * kRecWords + 4] << 32);
    if (j < n) out[g] = A[j * kRecWords + d];
    else atomicOr(err, 1u << 16);
}

// A[dest[t]] = R[t], one dword per thread.
__global__ __launch_bounds__(kTB) void k_tie_scatter(const uint32_t *R, const uint64_t *dest, uint64_t m,
                                                     uint32_t *A) {
    const uint64_t g = (uint64_t)blockIdx.x * kTB + threadIdx.x;
    if (g >= m * kRecWords) return;
    const uint64_t t = g / kRecWords, d = g - t * kRecWords;
    A[dest[t] * kRecWords + d] = R[g];
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
    uint32_t *E = nullptr, *E2 = nullptr;  // entries, then sorted entries (room for the first round's count)
    uint64_t *dest[2] = {nullptr, nullptr};  // positions of the entries, by round parity
    uint64_t cap = 0, nc = n;
    int r = 0;
    for (uint32_t p = kKeyBytes; p < key_bytes; p += kWindow, r++) {
        const uint64_t nb = (nc + kTSpan - 1) / kTSpan;
        if (r) k_tie_eq<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(E2, nc, P);
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
        if (!E) {  // the first round has the most entries: later rounds reuse its room
            cap = m;
            void *ent = nullptr;
            if ((rc = get_aux(s, 1, cap * kRec * 2 + cap * 16, &ent))) return rc;
            E = static_cast<uint32_t *>(ent);
            E2 = E + cap * kRecWords;
            dest[0] = reinterpret_cast<uint64_t *>(E2 + cap * kRecWords);
            dest[1] = dest[0] + cap;
        }
        k_tie_emit<<<dim3((uint32_t)nb), dim3(kTB), 0, s>>>(A, P, nc, r ? dest[(r - 1) & 1] : nullptr, p, key_bytes,
                                                             off_in, off_start, E, dest[r & 1]);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "leyenda_sort_keyed: entries");
        if ((rc = sort_device(E, m, E2, s, t))) return rc;
        if ((rc = guard_or_pooled(s, err))) return rc;  // the entry sort
        const uint64_t blocks = (m * kRecWords + kTB - 1) / kTB;
        k_tie_gather<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(A, n, E2, m, E, err);  // E is free again
        k_tie_scatter<<<dim3((uint32_t)blocks), dim3(kTB), 0, s>>>(E, dest[r & 1], m, A);
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
