// Limited-memory (external) sort: sorted runs, then a k-way merge of the runs,
// streamed between pinned host memory and a capped amount of device memory
// (Section 3.2, "Overlapping Computation with I/O": a sort stage writes sorted
// intermediate runs while reading and sorting the next chunk; a merge stage
// merges the runs one output partition at a time with a K-way merge, with
// reading, merging and writing overlapped).
//
// Run formation (leyenda_sort_runs): runs of R records go host -> device on
// one copy stream, are sorted on a compute stream by the in-HBM sort, and go
// back device -> host on a second copy stream, double-buffered so the three
// overlap.
//
// Merge (leyenda_merge): the output is cut into chunks of C records at exact
// ranks (merge-path partitioning): a co-rank kernel finds, for every chunk
// boundary, how many records of each run precede it, reading keys straight
// from the pinned runs.  Each chunk's k run slices then go host -> device, are
// merged on the GPU by rounds of pairwise merge-path merges of (key, index)
// tuples, gathered into output order and sent back, again double-buffered.
// Ties between runs resolve to the lower run, which is input order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "host_copy.h"
#include "runtime.h"

namespace ley {

constexpr int kMaxRuns = 256;       // merge fan-in: one co-rank thread per run
constexpr uint32_t kMergeTile = 2048;

// ---------------------------------------------------------------------------
// device helpers

struct Key80 {
    uint64_t h;
    uint32_t l;  // key bytes 8..9, big-endian
};

__device__ __forceinline__ Key80 load_key(const uint8_t *rec) {
    const uint32_t *p = reinterpret_cast<const uint32_t *>(rec);
    const uint32_t a = p[0], b = p[1], c = p[2];
    Key80 k;
    k.h = __builtin_bswap64(((uint64_t)b << 32) | a);
    k.l = __builtin_bswap16((uint16_t)(c & 0xFFFFu));
    return k;
}

// (key_a, run_a, pos_a) < (key_b, run_b, pos_b) in (key, run, position) order.
__device__ __forceinline__ bool tuple_less(const Key80 &a, uint32_t ra, uint64_t pa, const Key80 &b, uint32_t rb,
                                           uint64_t pb) {
    if (a.h != b.h) return a.h < b.h;
    if (a.l != b.l) return a.l < b.l;
    if (ra != rb) return ra < rb;
    return pa < pb;
}

// ---------------------------------------------------------------------------
// k_corank: for output rank b (one workgroup per boundary), the number s_i of
// records of each run i among the b first records of the merged output.
// Multisequence selection: keep lo_i <= s_i <= hi_i; take the middle record v
// of the widest interval, count the records below v in every run by binary
// search, and move lo (v below the boundary) or hi (v above it).  Every step
// halves one interval, so it ends after at most sum(log2 len_i) + k steps.

// Runs held in device memory instead of the pinned runs: runs first .. k - 1
// (at most two, the last ones) at p[i - first]; first == k when none is.
struct Resident {
    const uint8_t *p[2];
    uint32_t first;
};

// Record m of run i: in the pinned runs, or in device memory for a resident run.
__device__ __forceinline__ const uint8_t *run_rec(const uint8_t *runs, const uint64_t *run_off, const Resident &res,
                                                  uint32_t i, uint64_t m) {
    return i >= res.first ? res.p[i - res.first] + m * kRec : runs + (run_off[i] + m) * kRec;
}

__global__ __launch_bounds__(kWG) void k_corank(const uint8_t *runs, const uint64_t *run_off, uint32_t k,
                                                Resident res, const uint64_t *targets, uint64_t *splits,
                                                uint32_t *err) {
    __shared__ uint64_t lo[kMaxRuns], hi[kMaxRuns];
    __shared__ unsigned long long red_w[kWaves];
    __shared__ uint32_t red_i[kWaves];
    __shared__ unsigned long long sum_w[kWaves];
    __shared__ Key80 s_v;
    const uint32_t i = threadIdx.x, lane = i & 63, wv = i >> 6;
    const uint64_t b = targets[blockIdx.x];
    const uint64_t len_i = i < k ? run_off[i + 1] - run_off[i] : 0;
    lo[i] = 0;
    hi[i] = len_i;
    const uint32_t max_steps = 64u * kMaxRuns + 64u;
    uint32_t step = 0;
    for (;; step++) {
        __syncthreads();
        // widest interval (ties to the lowest run)
        unsigned long long wdt = hi[i] - lo[i];
        uint32_t who = i;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const unsigned long long w2 = __shfl_xor(wdt, o);
            const uint32_t i2 = __shfl_xor(who, o);
            if (w2 > wdt || (w2 == wdt && i2 < who)) { wdt = w2; who = i2; }
        }
        if (lane == 0) { red_w[wv] = wdt; red_i[wv] = who; }
        __syncthreads();
        unsigned long long bw = red_w[0];
        uint32_t j = red_i[0];
#pragma unroll
        for (int q = 1; q < kWaves; q++)
            if (red_w[q] > bw || (red_w[q] == bw && red_i[q] < j)) { bw = red_w[q]; j = red_i[q]; }
        if (bw == 0 || step >= max_steps) break;
        const uint64_t mid = (lo[j] + hi[j]) >> 1;
        if (i == 0) s_v = load_key(run_rec(runs, run_off, res, j, mid));
        __syncthreads();
        const Key80 v = s_v;
        // records of run i below v, over the whole run
        uint64_t r = 0;
        if (i < k) {
            if (i == j) {
                r = mid;
            } else {
                uint64_t a = 0, c = len_i;
                while (a < c) {
                    const uint64_t m = (a + c) >> 1;
                    const Key80 e = load_key(run_rec(runs, run_off, res, i, m));
                    if (tuple_less(e, i, m, v, j, mid)) a = m + 1; else c = m;
                }
                r = a;
            }
        }
        unsigned long long sum = r;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
        if (lane == 0) sum_w[wv] = sum;
        __syncthreads();
        unsigned long long R = 0;
#pragma unroll
        for (int q = 0; q < kWaves; q++) R += sum_w[q];
        if (i < k) {
            if (R < b) {  // v is among the first b records
                if (i == j) lo[i] = mid + 1;
                else if (r > lo[i]) lo[i] = r;
            } else {      // v and everything above it come after the boundary
                if (r < hi[i]) hi[i] = r;
            }
        }
    }
    __syncthreads();
    if (step >= max_steps && i == 0) atomicOr(err, 1u);
    if (i < k) splits[(size_t)blockIdx.x * k + i] = lo[i];
}

// ---------------------------------------------------------------------------
// merge of one chunk: tuples of the staged records, pairwise merge-path
// rounds, gather

__global__ __launch_bounds__(kWG) void k_merge_extract(const uint8_t *stage, uint64_t n, uint64_t *H, uint64_t *L) {
    const uint64_t q = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (q >= n) return;
    const Key80 k = load_key(stage + q * kRec);
    H[q] = k.h;
    L[q] = ((uint64_t)k.l << 32) | (uint32_t)q;
}

// Key-pointer tuples of m staged records whose input indices start at base
// (Section 3.2: the tuples are extracted while the input is read).
__global__ __launch_bounds__(kWG) void k_extract_chunk(const uint8_t *stage, uint64_t m, uint64_t base, uint64_t *H,
                                                       uint64_t *L) {
    const uint64_t q = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (q >= m) return;
    const Key80 k = load_key(stage + q * kRec);
    H[base + q] = k.h;
    L[base + q] = ((uint64_t)k.l << 32) | (uint32_t)(base + q);
}

struct MergePair {
    uint32_t a_off, a_len, b_len, first_tile;  // sequence B starts at a_off + a_len; output covers the same range
};

__device__ __forceinline__ bool tl(uint64_t h1, uint64_t l1, uint64_t h2, uint64_t l2) {
    return h1 < h2 || (h1 == h2 && l1 < l2);
}

// Elements of A taken among the first `diag` merged outputs (merge path).
__device__ __forceinline__ uint32_t merge_path(const uint64_t *AH, const uint64_t *AL, uint32_t alen,
                                               const uint64_t *BH, const uint64_t *BL, uint32_t blen,
                                               uint32_t diag) {
    uint32_t a = diag > blen ? diag - blen : 0u, c = min(diag, alen);
    while (a < c) {
        const uint32_t m = (a + c) >> 1;
        const uint32_t bi = diag - m - 1;
        if (tl(AH[m], AL[m], BH[bi], BL[bi])) a = m + 1; else c = m;
    }
    return a;
}

__global__ __launch_bounds__(kWG) void k_merge_pairs(const MergePair *pairs, uint32_t npairs, uint32_t ntiles,
                                                     const uint64_t *SH, const uint64_t *SL, uint64_t *DH,
                                                     uint64_t *DL) {
    __shared__ uint64_t th[kMergeTile], tlo[kMergeTile];
    __shared__ uint32_t s_i0, s_i1;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t p = 0;
        while (p + 1 < npairs && pairs[p + 1].first_tile <= t) p++;
        const MergePair mp = pairs[p];
        const uint32_t total = mp.a_len + mp.b_len;
        const uint32_t d0 = (t - mp.first_tile) * kMergeTile, d1 = min(d0 + kMergeTile, total);
        const uint64_t *AH = SH + mp.a_off, *AL = SL + mp.a_off;
        const uint64_t *BH = AH + mp.a_len, *BL = AL + mp.a_len;
        __syncthreads();
        if (threadIdx.x == 0) s_i0 = merge_path(AH, AL, mp.a_len, BH, BL, mp.b_len, d0);
        if (threadIdx.x == 64) s_i1 = merge_path(AH, AL, mp.a_len, BH, BL, mp.b_len, d1);
        __syncthreads();
        const uint32_t i0 = s_i0, i1 = s_i1, j0 = d0 - i0, j1 = d1 - i1;
        const uint32_t na = i1 - i0, nb = j1 - j0;
        for (uint32_t x = threadIdx.x; x < na; x += kWG) { th[x] = AH[i0 + x]; tlo[x] = AL[i0 + x]; }
        for (uint32_t y = threadIdx.x; y < nb; y += kWG) { th[na + y] = BH[j0 + y]; tlo[na + y] = BL[j0 + y]; }
        __syncthreads();
        uint64_t *OH = DH + mp.a_off + d0, *OL = DL + mp.a_off + d0;
        for (uint32_t x = threadIdx.x; x < na + nb; x += kWG) {
            const uint64_t h = th[x], l = tlo[x];
            // rank in the other list: elements below (h, l)
            uint32_t a, c;
            const uint32_t ob = x < na ? na : 0u, oe = x < na ? na + nb : na;
            a = ob; c = oe;
            while (a < c) {
                const uint32_t m = (a + c) >> 1;
                if (tl(th[m], tlo[m], h, l)) a = m + 1; else c = m;
            }
            const uint32_t pos = (x < na ? x : x - na) + (a - ob);
            OH[pos] = h;
            OL[pos] = l;
        }
    }
}

// out[j] = stage[index in L[j]]; an index outside the chunk (only a broken
// merge could leave one) is not read: it sets *err and leaves zeros.
__global__ __launch_bounds__(kWG) void k_gather_lo(const uint8_t *stage, const uint64_t *L, uint8_t *out, uint64_t n,
                                                   uint32_t *err) {
    __shared__ uint32_t sidx[kWG];
    const uint64_t g0 = (uint64_t)blockIdx.x * kWG;
    const uint32_t nr = (uint32_t)min<uint64_t>(kWG, n - g0);
    if (threadIdx.x < nr) {
        sidx[threadIdx.x] = (uint32_t)L[g0 + threadIdx.x];
        if (sidx[threadIdx.x] >= n) atomicOr(err, 2u);
    }
    __syncthreads();
    const uint32_t *src = reinterpret_cast<const uint32_t *>(stage);
    uint32_t *dst = reinterpret_cast<uint32_t *>(out) + g0 * 25;
    uint32_t v[25];
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u, r = q / 25u, kk = q - 25u * r;
        v[u] = 0;
        if (r < nr && sidx[r] < n) v[u] = src[(uint64_t)sidx[r] * 25 + kk];
    }
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u, r = q / 25u;
        if (r < nr) dst[q] = v[u];
    }
}

// Place of every input record in the output, the inverse of the sorted
// order: dest[idx[p]] = p.  An index outside the input sets *err (bit 4).
__global__ __launch_bounds__(kWG) void k_invert(const uint32_t *idx, uint64_t n, uint32_t *dest, uint32_t *err) {
    const uint64_t p = (uint64_t)blockIdx.x * kWG + threadIdx.x;
    if (p >= n) return;
    const uint32_t i = idx[p];
    if (i < n) dest[i] = (uint32_t)p;
    else atomicOr(err, 4u);
}

// Records of one staged input chunk written to their places in the output
// (Section 3.2: a pass over the input in order puts every record where its
// sorted tuple says).  A workgroup takes kWG records; thread t handles dwords
// t, t + kWG, ... of their dword stream, so that neighbouring lanes write
// neighbouring bytes of one record.  dest holds the places of the chunk's
// records; a place outside the output (no sorted tuple named that record) is
// not written and sets *err (bit 8).
__global__ __launch_bounds__(kWG) void k_scatter_chunk(const uint8_t *stage, uint64_t m, const uint32_t *dest,
                                                       uint64_t n, uint8_t *out, uint32_t *err) {
    __shared__ uint32_t sdst[kWG];
    const uint64_t g0 = (uint64_t)blockIdx.x * kWG;
    const uint32_t nr = (uint32_t)min<uint64_t>(kWG, m - g0);
    if (threadIdx.x < nr) {
        sdst[threadIdx.x] = dest[g0 + threadIdx.x];
        if (sdst[threadIdx.x] >= n) atomicOr(err, 8u);
    }
    __syncthreads();
    const uint32_t *src = reinterpret_cast<const uint32_t *>(stage) + g0 * 25;
    uint32_t *dst = reinterpret_cast<uint32_t *>(out);
    uint32_t v[25];
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u;
        v[u] = q < nr * 25u ? src[q] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 25; u++) {
        const uint32_t q = threadIdx.x + kWG * u, r = q / 25u, kk = q - 25u * r;
        if (r < nr && sdst[r] < n) dst[(uint64_t)sdst[r] * 25 + kk] = v[u];
    }
}

// ---------------------------------------------------------------------------
// host side

namespace {

// Device address of pinned host memory, or nullptr if p is not pinned host memory.
void *pinned_device_ptr(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
    if (a.hostPointer) return static_cast<char *>(a.devicePointer) + (static_cast<const char *>(p) -
                                                                      static_cast<const char *>(a.hostPointer));
    return a.devicePointer;
}

// Buffers a streaming loop cycles through (the merge uses three so the upload of
// chunk c + 1 never waits for the download of chunk c - 1; the others two).
constexpr int kPipeBufs = 3;

// Device memory of the external calls, kept between calls, one arena per
// device: allocating and freeing tens of GB in every call cost 0.1-0.4 s of
// a 60 GB sort's stages.  A call takes the kept arena when it holds at least
// what the call needs and no more than the call's budget (the call stays
// within its budget); otherwise the arena is replaced.  A call that finds the
// arena in use (another external call on the device) allocates its own and
// frees it when it returns.  leyenda_release_workspaces frees the arenas.
struct ExtArena {
    void *p = nullptr;
    size_t bytes = 0;
    bool busy = false;
};
std::mutex g_ext_mu;
ExtArena g_ext[64];

int current_device(int *dev) {
    const hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (*dev < 0 || *dev >= 64) return fail(LEYENDA_EINVAL, "device %d out of range", *dev);
    return LEYENDA_OK;
}

int ext_arena_take(size_t bytes, size_t budget, void **out, bool *pooled) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    *out = nullptr;
    *pooled = false;
    {
        std::lock_guard<std::mutex> lk(g_ext_mu);
        ExtArena &a = g_ext[dev];
        if (!a.busy) {
            if (a.p && a.bytes >= bytes && a.bytes <= budget) {
                a.busy = true;
                *out = a.p;
                *pooled = true;
                return LEYENDA_OK;
            }
            if (a.p) {  // too small or above this call's budget: replaced
                (void)hipFree(a.p);
                a.p = nullptr;
                a.bytes = 0;
            }
            hipError_t e = hipMalloc(&a.p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                a.p = nullptr;
                return fail(LEYENDA_ENOMEM, "hipMalloc(%zu) for the external sort failed", bytes);
            }
            a.bytes = bytes;
            a.busy = true;
            *out = a.p;
            *pooled = true;
            return LEYENDA_OK;
        }
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(LEYENDA_ENOMEM, "hipMalloc(%zu) for the external sort failed", bytes);
    }
    return LEYENDA_OK;
}

// Returns an arena from ext_arena_take; the caller's work on it has finished.
void ext_arena_give(void *p, bool pooled) {
    if (!p) return;
    if (!pooled) {
        (void)hipFree(p);
        return;
    }
    std::lock_guard<std::mutex> lk(g_ext_mu);
    for (ExtArena &a : g_ext)
        if (a.p == p) a.busy = false;
}

// The streams of an external call: its kernels run on the caller's stream
// (cs), its uploads and downloads on two streams of its own, so the process
// holds few streams (streams beyond the device's hardware queues share queues
// and serialise, and the copy streams must not share one).
struct Pipe {
    hipStream_t cs = nullptr, h2d = nullptr, d2h = nullptr;
    hipEvent_t ev[3][kPipeBufs] = {};  // [h2d_done, compute_done, d2h_done][buffer]
    void *arena = nullptr;
    bool pooled = false;
    int init(hipStream_t caller) {
        hipError_t e;
        cs = caller;
        if ((e = hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
        if ((e = hipStreamCreateWithFlags(&d2h, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
        for (auto &row : ev)
            for (auto &x : row)
                if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
        // the copies start after the caller's earlier work on its stream
        hipEvent_t start;
        if ((e = hipEventCreateWithFlags(&start, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
        (void)hipEventRecord(start, caller);
        (void)hipStreamWaitEvent(h2d, start, 0);
        (void)hipStreamWaitEvent(d2h, start, 0);
        (void)hipEventDestroy(start);
        return LEYENDA_OK;
    }
    // device memory for the call: `bytes` of a call limited to `budget`
    int alloc(size_t bytes, size_t budget) { return ext_arena_take(bytes, budget, &arena, &pooled); }
    // gives the arena back (every stream of the pipe has drained)
    void release_arena() {
        ext_arena_give(arena, pooled);
        arena = nullptr;
        pooled = false;
    }
    int finish() {
        hipError_t e1 = cs ? hipStreamSynchronize(cs) : hipSuccess;
        hipError_t e2 = h2d ? hipStreamSynchronize(h2d) : hipSuccess;
        hipError_t e3 = d2h ? hipStreamSynchronize(d2h) : hipSuccess;
        if (e1 != hipSuccess) return hip_fail(e1, "compute stream");
        if (e2 != hipSuccess) return hip_fail(e2, "copy stream");
        if (e3 != hipSuccess) return hip_fail(e3, "copy stream");
        return LEYENDA_OK;
    }
    ~Pipe() {
        if (cs) (void)hipStreamSynchronize(cs);
        if (h2d) (void)hipStreamSynchronize(h2d);
        if (d2h) (void)hipStreamSynchronize(d2h);
        release_arena();
        for (auto &row : ev)
            for (auto &x : row)
                if (x) (void)hipEventDestroy(x);
        if (h2d) (void)hipStreamDestroy(h2d);
        if (d2h) (void)hipStreamDestroy(d2h);
    }
};

size_t a256(size_t v) { return (v + 255) / 256 * 256; }

// Device -> pageable host through pinned bounce buffers: the copy engine
// fills them in turn while the host team empties the oldest one.
struct Bounce {
    static constexpr int kBufs = 4;
    static constexpr size_t kPiece = 128u << 20;
    uint8_t *buf[kBufs] = {};
    hipEvent_t ev[kBufs] = {};
    CopyTeam team;
    int init() {
        for (int i = 0; i < kBufs; i++) {
            hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&buf[i]), kPiece, hipHostMallocDefault);
            if (e != hipSuccess) { (void)hipGetLastError(); buf[i] = nullptr; return fail(LEYENDA_ENOMEM, "bounce buffer"); }
            if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
        }
        return LEYENDA_OK;
    }
    // Copies `bytes` of device memory at src_dev to dst once `ready` has
    // fired on the device; returns when dst is complete.
    int drain(const uint8_t *src_dev, uint8_t *dst, uint64_t bytes, hipEvent_t ready, hipStream_t s) {
        hipError_t e = hipStreamWaitEvent(s, ready, 0);
        if (e != hipSuccess) return hip_fail(e, "bounce wait");
        uint8_t *pend_dst[kBufs] = {};
        size_t pend_len[kBufs] = {};
        uint64_t issued = 0;
        // keep every buffer's download in flight; empty them oldest first
        for (uint64_t piece = 0;; piece++) {
            const int p = (int)(piece % kBufs);
            if (pend_len[p]) {
                if ((e = hipEventSynchronize(ev[p])) != hipSuccess) return hip_fail(e, "bounce copy");
                team.copy(pend_dst[p], buf[p], pend_len[p]);
                pend_len[p] = 0;
            }
            if (issued < bytes) {
                const size_t len = (size_t)std::min<uint64_t>(kPiece, bytes - issued);
                e = hipMemcpyAsync(buf[p], src_dev + issued, len, hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipEventRecord(ev[p], s);
                if (e != hipSuccess) return hip_fail(e, "bounce copy");
                pend_dst[p] = dst + issued;
                pend_len[p] = len;
                issued += len;
            } else {
                bool any = false;
                for (int q = 0; q < kBufs; q++) any = any || pend_len[q];
                if (!any) break;
            }
        }
        return LEYENDA_OK;
    }
    // waits for every copy into the buffers (before they serve another call)
    void quiesce() {
        for (int i = 0; i < kBufs; i++)
            if (ev[i]) (void)hipEventSynchronize(ev[i]);
    }
    ~Bounce() {
        for (int i = 0; i < kBufs; i++) {
            if (ev[i]) { (void)hipEventSynchronize(ev[i]); (void)hipEventDestroy(ev[i]); }
            if (buf[i]) (void)hipHostFree(buf[i]);
        }
    }
};

// The bounce buffers and copy threads of pageable outputs, kept between calls
// like the arena (one set per device; pinning them and starting the threads
// is work every pageable output would otherwise repeat).  A call that finds
// them in use makes its own set for the call.
std::unique_ptr<Bounce> g_bounce[64];
bool g_bounce_busy[64] = {};

struct BounceLease {
    Bounce *b = nullptr;
    bool pooled = false;
    int dev = 0;
    int take() {
        int rc = current_device(&dev);
        if (rc) return rc;
        {
            std::lock_guard<std::mutex> lk(g_ext_mu);
            if (!g_bounce_busy[dev]) {
                if (!g_bounce[dev]) {
                    std::unique_ptr<Bounce> nb(new Bounce());
                    if ((rc = nb->init())) return rc;
                    g_bounce[dev] = std::move(nb);
                }
                g_bounce_busy[dev] = true;
                b = g_bounce[dev].get();
                pooled = true;
                return LEYENDA_OK;
            }
        }
        b = new Bounce();
        return b->init();
    }
    ~BounceLease() {
        if (!b) return;
        if (pooled) {
            b->quiesce();  // an early error return may leave a download in flight
            std::lock_guard<std::mutex> lk(g_ext_mu);
            g_bounce_busy[dev] = false;
        } else {
            delete b;
        }
    }
};

// Device bytes one run of r records needs: two input and two output buffers
// (so upload, sort and download overlap) plus the sort's workspace.
uint64_t run_bytes(uint64_t r, const Tune &t) { return 4 * a256(r * kRec) + plan_layout(r, 1, t).total + 4096; }

// Boundaries of n records cut into equal pieces of at most `cap`.  (First and
// last pieces of an eighth, to shorten the one-way head and tail of the
// streaming loops, measured slower on the 60 GB workload: merge 2.03 against
// 1.5-1.7 s, runs no faster.)
std::vector<uint64_t> equal_bounds(uint64_t n, uint64_t cap) {
    std::vector<uint64_t> b{0};
    if (n == 0) return b;
    const uint64_t k = (n + cap - 1) / cap, r = (n + k - 1) / k;
    for (uint64_t o = r; o < n; o += r) b.push_back(o);
    b.push_back(n);
    return b;
}

int plan_runs_t(uint64_t n, uint64_t budget, const Tune &t, uint64_t *R, uint64_t *K,
                std::vector<uint64_t> *bounds = nullptr) {
    if (n == 0) { *R = 0; *K = 0; if (bounds) *bounds = {0}; return LEYENDA_OK; }
    uint64_t lo = 1, hi = std::min<uint64_t>(n, LEYENDA_MAX_RECORDS);
    if (run_bytes(1, t) > budget) return fail(LEYENDA_EBUDGET, "budget of %llu bytes is below one run's footprint",
                                              (unsigned long long)budget);
    while (lo < hi) {
        const uint64_t m = lo + (hi - lo + 1) / 2;
        if (run_bytes(m, t) <= budget) lo = m; else hi = m - 1;
    }
    const std::vector<uint64_t> b = equal_bounds(n, lo);
    uint64_t longest = 0;
    for (size_t i = 0; i + 1 < b.size(); i++) longest = std::max(longest, b[i + 1] - b[i]);
    *K = b.size() - 1;
    *R = longest;
    if (bounds) *bounds = b;
    return LEYENDA_OK;
}

}  // namespace

}  // namespace ley

using namespace ley;

extern "C" int leyenda_host_alloc(uint64_t bytes, void **out) {
    if (!out) return fail(LEYENDA_EINVAL, "leyenda_host_alloc: NULL");
    *out = nullptr;
    if (bytes == 0) return LEYENDA_OK;
    hipError_t e = hipHostMalloc(out, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(LEYENDA_ENOMEM, "hipHostMalloc(%llu): %s", (unsigned long long)bytes, hipGetErrorString(e));
    }
    return LEYENDA_OK;
}

extern "C" int leyenda_host_free(void *p) {
    if (!p) return LEYENDA_OK;
    hipError_t e = hipHostFree(p);
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "hipHostFree");
}

extern "C" int leyenda_plan_runs(uint64_t n, uint64_t device_budget_bytes, uint64_t *run_records, uint64_t *num_runs) {
    if (!run_records || !num_runs) return fail(LEYENDA_EINVAL, "leyenda_plan_runs: NULL");
    return plan_runs_t(n, device_budget_bytes, tune_of(current_params()), run_records, num_runs);
}

extern "C" int leyenda_sort_runs(const void *host_records, uint64_t n, uint64_t device_budget_bytes, void *host_runs,
                                 uint64_t *run_bounds, uint64_t k_max, uint64_t *k_out, void *stream) {
    if (!run_bounds || !k_out) return fail(LEYENDA_EINVAL, "leyenda_sort_runs: NULL run_bounds or k_out");
    *k_out = 0;
    if (n == 0) { run_bounds[0] = 0; return LEYENDA_OK; }
    if (!host_records || !host_runs) return fail(LEYENDA_EINVAL, "leyenda_sort_runs: NULL buffer");
    if ((reinterpret_cast<uintptr_t>(host_records) | reinterpret_cast<uintptr_t>(host_runs)) & 3u)
        return fail(LEYENDA_EINVAL, "leyenda_sort_runs: buffers must be 4-byte aligned");
    if (host_records != host_runs && overlaps(host_records, n * kRec, host_runs, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_sort_runs: host_runs partly overlaps host_records");
    if (!pinned_device_ptr(host_records) || !pinned_device_ptr(host_runs))
        return fail(LEYENDA_EINVAL, "leyenda_sort_runs: host buffers must be pinned (hipHostMalloc / pin_memory)");
    const Tune t = tune_of(current_params());
    uint64_t R = 0, K = 0;
    std::vector<uint64_t> run_off;
    int rc = plan_runs_t(n, device_budget_bytes, t, &R, &K, &run_off);
    if (rc) return rc;
    if (K > k_max) return fail(LEYENDA_EBUDGET, "leyenda_sort_runs: %llu runs needed, k_max is %llu",
                               (unsigned long long)K, (unsigned long long)k_max);
    Pipe P;
    if ((rc = P.init(static_cast<hipStream_t>(stream)))) return rc;
    const size_t rb = a256(R * kRec);
    const size_t ws_bytes = plan_layout(R, 1, t).total;
    if ((rc = P.alloc(4 * rb + ws_bytes + 256, device_budget_bytes))) return rc;
    char *base = static_cast<char *>(P.arena);
    uint8_t *in[2] = {reinterpret_cast<uint8_t *>(base), reinterpret_cast<uint8_t *>(base + rb)};
    uint8_t *out[2] = {reinterpret_cast<uint8_t *>(base + 2 * rb), reinterpret_cast<uint8_t *>(base + 3 * rb)};
    void *ws = base + 4 * rb;
    uint32_t *guard = reinterpret_cast<uint32_t *>(base + 4 * rb + a256(ws_bytes));  // OR of the runs' guard words
    const uint8_t *src = static_cast<const uint8_t *>(host_records);
    uint8_t *dst = static_cast<uint8_t *>(host_runs);
    hipError_t e = hipMemsetAsync(guard, 0, 4, P.cs);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_runs: guard word");
    for (uint64_t r = 0; r < K; r++) {
        const int b = (int)(r & 1);
        const uint64_t off = run_off[r], len = run_off[r + 1] - run_off[r];
        run_bounds[r] = off;
        // upload after the sort that last read in[b]
        if (r >= 2) e = hipStreamWaitEvent(P.h2d, P.ev[1][b], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(in[b], src + off * kRec, len * kRec, hipMemcpyHostToDevice, P.h2d);
        if (e == hipSuccess) e = hipEventRecord(P.ev[0][b], P.h2d);
        // sort after the upload, and after the download that last read out[b]
        if (e == hipSuccess) e = hipStreamWaitEvent(P.cs, P.ev[0][b], 0);
        if (e == hipSuccess && r >= 2) e = hipStreamWaitEvent(P.cs, P.ev[2][b], 0);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_runs: enqueue");
        if ((rc = sort_device_ws(in[b], len, out[b], P.cs, t, ws))) return rc;
        e = launch_guard_or(ws, len, t, guard, P.cs);
        if (e == hipSuccess) e = hipEventRecord(P.ev[1][b], P.cs);
        // download the sorted run over its own input range
        if (e == hipSuccess) e = hipStreamWaitEvent(P.d2h, P.ev[1][b], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(dst + off * kRec, out[b], len * kRec, hipMemcpyDeviceToHost, P.d2h);
        if (e == hipSuccess) e = hipEventRecord(P.ev[2][b], P.d2h);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_runs: enqueue");
    }
    run_bounds[K] = n;
    if ((rc = P.finish())) return rc;
    uint32_t g = 0;
    e = hipMemcpy(&g, guard, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_runs: guard word");
    if (g) return fail(LEYENDA_EINTERNAL, "leyenda_sort_runs: a device-side guard fired in a run's sort (0x%x)", g);
    *k_out = K;
    return LEYENDA_OK;
}

namespace ley {
namespace {

// Rounds of the in-chunk pairwise merge of k runs: ceil(log2 k).
uint32_t merge_rounds(uint64_t k) {
    uint32_t r = 0;
    while ((1ull << r) < k) r++;
    return r;
}

// Device tables of a merge of k runs in `chunks` output chunks: run offsets,
// chunk targets, co-rank splits, merge pair lists, the error word.
uint64_t merge_tables_bytes(uint64_t k, uint64_t chunks) {
    const uint32_t rounds = merge_rounds(k);
    return a256((k + 1) * 8) + a256(chunks * 8) + a256((chunks + 1) * k * 8) +
           a256(chunks * (rounds + 1) * ((k + 1) / 2 + 1) * sizeof(MergePair)) + 256;
}

// The merge's output chunks under a device budget: the largest chunk whose
// buffers (three staging and three output buffers of records, two tuple
// buffer pairs) fit next to the tables its chunk count needs.  Returns the
// chunk bounds (empty when the budget is too small) and the device bytes the
// merge then uses in *bytes.
std::vector<uint64_t> merge_plan(uint64_t n, uint64_t k, uint64_t device_budget_bytes, uint64_t *bytes) {
    auto buf_bytes = [&](uint64_t m) -> uint64_t { return 2 * kPipeBufs * a256(m * kRec) + 4 * a256(m * 8); };
    uint64_t lo = 0, tab = merge_tables_bytes(k, 1);
    for (int it = 0; it < 64; it++) {
        if (tab + buf_bytes(1) > device_budget_bytes) break;
        uint64_t a = 1, c = std::min<uint64_t>(n, LEYENDA_MAX_RECORDS);
        while (a < c) {
            const uint64_t m = a + (c - a + 1) / 2;
            if (buf_bytes(m) + tab <= device_budget_bytes) a = m; else c = m - 1;
        }
        const uint64_t t2 = merge_tables_bytes(k, (n + a - 1) / a);
        if (t2 <= tab) { lo = a; break; }
        tab = t2;
    }
    *bytes = 0;
    if (lo == 0) return {};
    std::vector<uint64_t> cb = equal_bounds(n, lo);
    uint64_t C = 0;  // longest chunk (buffer size)
    for (size_t c = 0; c + 1 < cb.size(); c++) C = std::max(C, cb[c + 1] - cb[c]);
    *bytes = buf_bytes(C) + merge_tables_bytes(k, cb.size() - 1);
    return cb;
}

// The merge of k sorted runs (validated by the caller) into host_out, on the
// streams of P.  runs_dev is the device view of the pinned runs.  The chunks
// come from merge_plan under device_budget_bytes; arena: device memory of at
// least the plan's bytes (null: allocate them).  res: the runs that live in
// device memory (their records are not read from the pinned runs).
int merge_impl(Pipe &P, const uint8_t *runs_dev, const uint8_t *runs_h, const uint64_t *run_bounds, uint64_t k,
               uint8_t *out_h, bool direct_out, uint64_t device_budget_bytes, char *arena, Resident res) {
    const uint64_t n = run_bounds[k];
    int rc = LEYENDA_OK;
    const uint32_t rounds = merge_rounds(k);
    uint64_t need = 0;
    const std::vector<uint64_t> cb = merge_plan(n, k, device_budget_bytes, &need);  // output chunks
    if (cb.empty()) return fail(LEYENDA_EBUDGET, "leyenda_merge: budget too small");
    const uint64_t nch = cb.size() - 1;
    uint64_t C = 0;  // longest chunk (buffer size)
    for (uint64_t c = 0; c < nch; c++) C = std::max(C, cb[c + 1] - cb[c]);

    const size_t sb = a256(C * kRec), tb = a256(C * 8);
    const size_t n_tab = (size_t)(nch + 1) * k;
    const size_t pair_cap = (size_t)nch * (rounds + 1) * ((k + 1) / 2 + 1);
    if (!arena) {
        if ((rc = P.alloc(need, device_budget_bytes))) return rc;
        arena = static_cast<char *>(P.arena);
    }
    char *base = arena;
    uint8_t *stage[kPipeBufs], *outb[kPipeBufs];
    for (int i = 0; i < kPipeBufs; i++) {
        stage[i] = reinterpret_cast<uint8_t *>(base + i * sb);
        outb[i] = reinterpret_cast<uint8_t *>(base + (kPipeBufs + i) * sb);
    }
    char *const tbase = base + 2 * kPipeBufs * sb;
    uint64_t *TH[2] = {reinterpret_cast<uint64_t *>(tbase), reinterpret_cast<uint64_t *>(tbase + tb)};
    uint64_t *TL[2] = {reinterpret_cast<uint64_t *>(tbase + 2 * tb), reinterpret_cast<uint64_t *>(tbase + 3 * tb)};
    char *tp = tbase + 4 * tb;
    uint64_t *d_off = reinterpret_cast<uint64_t *>(tp); tp += a256((k + 1) * 8);
    uint64_t *d_tgt = reinterpret_cast<uint64_t *>(tp); tp += a256(nch * 8);
    uint64_t *d_split = reinterpret_cast<uint64_t *>(tp); tp += a256(n_tab * 8);
    MergePair *d_pairs = reinterpret_cast<MergePair *>(tp); tp += a256(pair_cap * sizeof(MergePair));
    uint32_t *d_err = reinterpret_cast<uint32_t *>(tp);

    // 1. exact chunk boundaries (co-rank of ranks C, 2C, ...)
    std::vector<uint64_t> split((nch + 1) * k, 0);
    for (uint64_t i = 0; i < k; i++) split[nch * k + i] = run_bounds[i + 1] - run_bounds[i];
    hipError_t e = hipMemsetAsync(d_err, 0, 4, P.cs);  // error word of the co-rank and gather kernels
    if (e != hipSuccess) return hip_fail(e, "leyenda_merge: error word");
    if (nch > 1) {
        std::vector<uint64_t> tgt(nch - 1);
        for (uint64_t c = 1; c < nch; c++) tgt[c - 1] = cb[c];
        e = hipMemcpyAsync(d_off, run_bounds, (k + 1) * 8, hipMemcpyHostToDevice, P.cs);
        if (e == hipSuccess) e = hipMemcpyAsync(d_tgt, tgt.data(), (nch - 1) * 8, hipMemcpyHostToDevice, P.cs);
        if (e != hipSuccess) return hip_fail(e, "leyenda_merge: tables");
        k_corank<<<dim3((uint32_t)(nch - 1)), dim3(kWG), 0, P.cs>>>(runs_dev, d_off, (uint32_t)k, res, d_tgt,
                                                                   d_split, d_err);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "co-rank kernel");
        uint32_t err = 0;
        e = hipMemcpyAsync(split.data() + k, d_split, (nch - 1) * k * 8, hipMemcpyDeviceToHost, P.cs);
        if (e == hipSuccess) e = hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, P.cs);
        if (e == hipSuccess) e = hipStreamSynchronize(P.cs);
        if (e != hipSuccess) return hip_fail(e, "leyenda_merge: co-rank");
        if (err) return fail(LEYENDA_EINTERNAL, "leyenda_merge: co-rank did not converge");
        for (uint64_t c = 1; c < nch; c++) {
            uint64_t s = 0;
            for (uint64_t i = 0; i < k; i++) {
                const uint64_t a = split[c * k + i], b0 = split[(c - 1) * k + i];
                if (a < b0 || a > run_bounds[i + 1] - run_bounds[i])
                    return fail(LEYENDA_EINTERNAL, "leyenda_merge: co-rank out of order");
                s += a;
            }
            if (s != cb[c]) return fail(LEYENDA_EINTERNAL, "leyenda_merge: co-rank sums to the wrong rank");
        }
    }

    // 2. per chunk: slices, pairwise merge rounds
    struct Round {
        uint32_t pair_first, npairs, ntiles, in_buf;
    };
    std::vector<MergePair> pairs;
    std::vector<std::vector<Round>> plan(nch);
    std::vector<std::vector<uint64_t>> slice_off(nch), slice_len(nch);
    std::vector<uint32_t> final_buf(nch, 0);
    for (uint64_t c = 0; c < nch; c++) {
        std::vector<uint64_t> seq_off, seq_len;
        uint64_t o = 0;
        for (uint64_t i = 0; i < k; i++) {
            const uint64_t len = split[(c + 1) * k + i] - split[c * k + i];
            slice_off[c].push_back(o);
            slice_len[c].push_back(len);
            if (len) { seq_off.push_back(o); seq_len.push_back(len); }
            o += len;
        }
        uint32_t buf = 0;
        while (seq_off.size() > 1) {
            Round rd{(uint32_t)pairs.size(), 0, 0, buf};
            std::vector<uint64_t> no, nl;
            for (size_t s = 0; s < seq_off.size(); s += 2) {
                MergePair mp;
                mp.a_off = (uint32_t)seq_off[s];
                mp.a_len = (uint32_t)seq_len[s];
                mp.b_len = s + 1 < seq_off.size() ? (uint32_t)seq_len[s + 1] : 0u;
                mp.first_tile = rd.ntiles;
                rd.ntiles += (mp.a_len + mp.b_len + kMergeTile - 1) / kMergeTile;
                pairs.push_back(mp);
                rd.npairs++;
                no.push_back(seq_off[s]);
                nl.push_back(seq_len[s] + (s + 1 < seq_off.size() ? seq_len[s + 1] : 0));
            }
            plan[c].push_back(rd);
            seq_off.swap(no);
            seq_len.swap(nl);
            buf ^= 1;
        }
        final_buf[c] = buf;
    }
    if (pairs.size() > pair_cap) return fail(LEYENDA_EINTERNAL, "leyenda_merge: pair table overflow");
    if (!pairs.empty()) {
        e = hipMemcpyAsync(d_pairs, pairs.data(), pairs.size() * sizeof(MergePair), hipMemcpyHostToDevice, P.cs);
        if (e == hipSuccess) e = hipStreamSynchronize(P.cs);
        if (e != hipSuccess) return hip_fail(e, "leyenda_merge: pair table");
    }

    // 3. stream the chunks: upload slices | merge + gather | download, over
    //    three buffers.  A pageable output drains through the host (blocking
    //    this thread) two chunks behind: while chunk c - 2 drains, the uploads
    //    of chunks c - 1 and c are already queued, so the host-to-device copies
    //    never wait for a drain to return, and chunk c's buffers were freed by
    //    the drain of chunk c - 3 one step earlier.
    const int cus = device_cus();
    constexpr uint64_t kLag = kPipeBufs - 1;
    BounceLease bounce;
    if (!direct_out && (rc = bounce.take())) return rc;
    std::vector<uint64_t> chunk_len(nch, 0);
    for (uint64_t c = 0; c < nch; c++)
        for (uint64_t i = 0; i < k; i++) chunk_len[c] += slice_len[c][i];
    for (uint64_t c = 0; c < nch + (direct_out ? 0 : kLag); c++) {
        if (c < nch) {
            const int b = (int)(c % kPipeBufs);
            const uint64_t out_first = cb[c], clen = chunk_len[c];
            // the staging buffer's last reader was the merge of chunk c - 3
            if (c >= (uint64_t)kPipeBufs) e = hipStreamWaitEvent(P.h2d, P.ev[1][b], 0);
            for (uint64_t i = 0; i < k && e == hipSuccess; i++) {
                const uint64_t len = slice_len[c][i];
                if (!len) continue;
                if (i >= res.first)  // a run held in device memory
                    e = hipMemcpyAsync(stage[b] + slice_off[c][i] * kRec, res.p[i - res.first] + split[c * k + i] * kRec,
                                       len * kRec, hipMemcpyDeviceToDevice, P.h2d);
                else
                    e = hipMemcpyAsync(stage[b] + slice_off[c][i] * kRec,
                                       runs_h + (run_bounds[i] + split[c * k + i]) * kRec, len * kRec,
                                       hipMemcpyHostToDevice, P.h2d);
            }
            if (e == hipSuccess) e = hipEventRecord(P.ev[0][b], P.h2d);
            if (e == hipSuccess) e = hipStreamWaitEvent(P.cs, P.ev[0][b], 0);
            // the output buffer's last reader: the download of chunk c - 3 (a
            // pageable output's drain of it returned before this step)
            if (e == hipSuccess && c >= (uint64_t)kPipeBufs && direct_out) e = hipStreamWaitEvent(P.cs, P.ev[2][b], 0);
            if (e != hipSuccess) return hip_fail(e, "leyenda_merge: enqueue");
            k_merge_extract<<<dim3((uint32_t)((clen + kWG - 1) / kWG)), dim3(kWG), 0, P.cs>>>(stage[b], clen, TH[0],
                                                                                             TL[0]);
            for (const Round &rd : plan[c]) {
                const uint32_t g = std::max<uint32_t>(1, std::min<uint32_t>(rd.ntiles, (uint32_t)cus * 8));
                k_merge_pairs<<<dim3(g), dim3(kWG), 0, P.cs>>>(d_pairs + rd.pair_first, rd.npairs, rd.ntiles,
                                                                TH[rd.in_buf], TL[rd.in_buf], TH[rd.in_buf ^ 1],
                                                                TL[rd.in_buf ^ 1]);
            }
            k_gather_lo<<<dim3((uint32_t)((clen + kWG - 1) / kWG)), dim3(kWG), 0, P.cs>>>(stage[b], TL[final_buf[c]],
                                                                                       outb[b], clen, d_err);
            if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "merge kernels");
            e = hipEventRecord(P.ev[1][b], P.cs);
            if (e != hipSuccess) return hip_fail(e, "leyenda_merge: enqueue");
            if (direct_out) {
                e = hipStreamWaitEvent(P.d2h, P.ev[1][b], 0);
                if (e == hipSuccess) e = hipMemcpyAsync(out_h + out_first * kRec, outb[b], clen * kRec,
                                                        hipMemcpyDeviceToHost, P.d2h);
                if (e == hipSuccess) e = hipEventRecord(P.ev[2][b], P.d2h);
                if (e != hipSuccess) return hip_fail(e, "leyenda_merge: enqueue");
            }
        }
        if (!direct_out && c >= kLag) {
            const uint64_t d = c - kLag;
            const int bd = (int)(d % kPipeBufs);
            if ((rc = bounce.b->drain(outb[bd], out_h + cb[d] * kRec, chunk_len[d] * kRec, P.ev[1][bd], P.d2h)))
                return rc;
        }
    }
    if ((rc = P.finish())) return rc;
    uint32_t err = 0;
    e = hipMemcpy(&err, d_err, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "leyenda_merge: error word");
    if (err) return fail(LEYENDA_EINTERNAL, "leyenda_merge: a merged index fell outside its chunk (0x%x)", err);
    return LEYENDA_OK;
}

}  // namespace
}  // namespace ley

extern "C" int leyenda_merge(const void *host_runs, const uint64_t *run_bounds, uint64_t k, void *host_out,
                             uint64_t device_budget_bytes, void *stream) {
    if (!run_bounds) return fail(LEYENDA_EINVAL, "leyenda_merge: NULL run_bounds");
    if (k == 0) return LEYENDA_OK;
    if (k > (uint64_t)kMaxRuns) return fail(LEYENDA_EINVAL, "leyenda_merge: at most %d runs", kMaxRuns);
    if (run_bounds[0] != 0) return fail(LEYENDA_EINVAL, "leyenda_merge: run_bounds[0] must be 0");
    for (uint64_t i = 0; i < k; i++)
        if (run_bounds[i + 1] < run_bounds[i]) return fail(LEYENDA_EINVAL, "leyenda_merge: run_bounds decrease");
    const uint64_t n = run_bounds[k];
    if (n == 0) return LEYENDA_OK;
    if (!host_runs || !host_out) return fail(LEYENDA_EINVAL, "leyenda_merge: NULL buffer");
    if ((reinterpret_cast<uintptr_t>(host_runs) | reinterpret_cast<uintptr_t>(host_out)) & 3u)
        return fail(LEYENDA_EINVAL, "leyenda_merge: buffers must be 4-byte aligned");
    if (overlaps(host_runs, n * kRec, host_out, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_merge: host_out overlaps host_runs");
    const uint8_t *runs_dev = static_cast<const uint8_t *>(pinned_device_ptr(host_runs));
    if (!runs_dev) return fail(LEYENDA_EINVAL, "leyenda_merge: host_runs must be pinned (hipHostMalloc / pin_memory)");
    // pinned output: chunks go straight device -> host_out; pageable output:
    // through two pinned bounce buffers drained by host copies
    const bool direct_out = pinned_device_ptr(host_out) != nullptr;
    for (uint64_t i = 0; i < k; i++)
        if (run_bounds[i + 1] - run_bounds[i] > LEYENDA_MAX_RECORDS)
            return fail(LEYENDA_ETOOBIG, "leyenda_merge: run %llu too long", (unsigned long long)i);
    Pipe P;
    int rc = P.init(static_cast<hipStream_t>(stream));
    if (rc) return rc;
    return merge_impl(P, runs_dev, static_cast<const uint8_t *>(host_runs), run_bounds, k,
                      static_cast<uint8_t *>(host_out), direct_out, device_budget_bytes, nullptr,
                      Resident{{nullptr, nullptr}, (uint32_t)k});
}

// ---------------------------------------------------------------------------
// Runs + merge in one call: the same two stages, except that the last two
// runs stay in device memory after their sorts (in the two output buffers of
// the run stage) instead of going to host_runs and coming back for the merge;
// their slices reach the merge by device copies.  The merge plans its chunks
// within the run stage's footprint less the kept runs (else within the whole
// budget less them).  When that is too little for a merge
// of the runs (many tiny runs under a budget near one run's footprint), only
// the last run is kept (it is the one whose download would have nothing to
// overlap with), and when even that leaves too little, every run goes to
// host_runs and the merge runs as leyenda_merge would with the whole budget.

namespace {

// The plan of a one-call external sort: R records per run, K runs, and the
// number of last runs kept on the device with the merge's budget.  Two runs
// are kept if the merge's chunks and tables fit beside them, else one, else
// none (many tiny runs).  The merge is planned within the run stage's own
// footprint first, so that the call asks for no more device memory than its
// run stage does (a device arena kept from an earlier external call is then
// reused, not replaced), and within the whole budget only when that is too
// little.
struct ExternalPlan {
    uint64_t R = 0, K = 0, kept = 0;
    uint64_t rb = 0, ws_bytes = 0, total = 0;  // run buffer, sort workspace, run stage footprint
    uint64_t merge_budget = 0, merge_bytes = 0;
};

int plan_external(uint64_t n, uint64_t device_budget_bytes, const Tune &t, ExternalPlan *x) {
    int rc = plan_runs_t(n, device_budget_bytes, t, &x->R, &x->K);
    if (rc || n == 0) return rc;
    x->rb = a256(x->R * kRec);
    x->ws_bytes = plan_layout(x->R, 1, t).total;
    x->total = 4 * x->rb + x->ws_bytes + 256;  // <= the budget (plan_runs_t)
    if (x->K == 1) {
        x->kept = 1;
        return LEYENDA_OK;
    }
    for (const uint64_t lim : {x->total, device_budget_bytes}) {
        for (uint64_t kk = 2; kk >= 1; kk--)
            if (!merge_plan(n, x->K, lim - kk * x->rb, &x->merge_bytes).empty()) {
                x->kept = kk;
                x->merge_budget = lim - kk * x->rb;
                return LEYENDA_OK;
            }
    }
    x->merge_bytes = 0;  // nothing kept: the merge plans as leyenda_merge does
    return LEYENDA_OK;
}

}  // namespace

extern "C" int leyenda_plan_external(uint64_t n, uint64_t device_budget_bytes, uint64_t *run_records,
                                     uint64_t *num_runs, uint64_t *kept_runs) {
    if (!run_records || !num_runs || !kept_runs) return fail(LEYENDA_EINVAL, "leyenda_plan_external: NULL");
    ExternalPlan x;
    const int rc = plan_external(n, device_budget_bytes, tune_of(current_params()), &x);
    if (rc) return rc;
    if (x.K > (uint64_t)kMaxRuns)
        return fail(LEYENDA_EBUDGET, "leyenda_plan_external: %llu runs needed, the merge takes at most %d",
                    (unsigned long long)x.K, kMaxRuns);
    *run_records = x.R;
    *num_runs = x.K;
    *kept_runs = x.kept;
    return LEYENDA_OK;
}

extern "C" int leyenda_sort_external(const void *host_records, uint64_t n, uint64_t device_budget_bytes,
                                     void *host_runs, void *host_out, void *stream) {
    if (n == 0) return LEYENDA_OK;
    if (!host_records || !host_runs || !host_out) return fail(LEYENDA_EINVAL, "leyenda_sort_external: NULL buffer");
    if ((reinterpret_cast<uintptr_t>(host_records) | reinterpret_cast<uintptr_t>(host_runs) |
         reinterpret_cast<uintptr_t>(host_out)) & 3u)
        return fail(LEYENDA_EINVAL, "leyenda_sort_external: buffers must be 4-byte aligned");
    if (host_records != host_runs && overlaps(host_records, n * kRec, host_runs, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_sort_external: host_runs partly overlaps host_records");
    if (overlaps(host_out, n * kRec, host_runs, n * kRec) || overlaps(host_out, n * kRec, host_records, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_sort_external: host_out overlaps the input or the runs");
    const uint8_t *runs_dev = static_cast<const uint8_t *>(pinned_device_ptr(host_runs));
    if (!pinned_device_ptr(host_records) || !runs_dev)
        return fail(LEYENDA_EINVAL, "leyenda_sort_external: host_records and host_runs must be pinned");
    const bool direct_out = pinned_device_ptr(host_out) != nullptr;
    const Tune t = tune_of(current_params());
    ExternalPlan x;
    int rc = plan_external(n, device_budget_bytes, t, &x);
    if (rc) return rc;
    const uint64_t R = x.R, K = x.K, kept = x.kept;
    if (K > (uint64_t)kMaxRuns)
        return fail(LEYENDA_EBUDGET, "leyenda_sort_external: %llu runs needed, the merge takes at most %d",
                    (unsigned long long)K, kMaxRuns);
    Pipe P;
    if ((rc = P.init(static_cast<hipStream_t>(stream)))) return rc;
    const size_t rb = x.rb, ws_bytes = x.ws_bytes, total = x.total;
    if ((rc = P.alloc(kept ? std::max<uint64_t>(total, kept * rb + x.merge_bytes) : total, device_budget_bytes)))
        return rc;
    char *base = static_cast<char *>(P.arena);
    // the output buffers come first (the last run sorts into out[0], the one
    // before it into out[1]), so the memory after the kept runs is one block
    // for the merge
    uint8_t *const keep = reinterpret_cast<uint8_t *>(base);
    uint8_t *in[2] = {reinterpret_cast<uint8_t *>(base + 2 * rb), reinterpret_cast<uint8_t *>(base + 3 * rb)};
    uint8_t *out[2] = {keep, reinterpret_cast<uint8_t *>(base + rb)};
    void *ws = base + 4 * rb;
    uint32_t *guard = reinterpret_cast<uint32_t *>(base + 4 * rb + a256(ws_bytes));
    const uint8_t *src = static_cast<const uint8_t *>(host_records);
    uint8_t *dst = static_cast<uint8_t *>(host_runs);
    std::vector<uint64_t> bounds(K + 1, n);
    hipError_t e = hipMemsetAsync(guard, 0, 4, P.cs);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external: guard word");
    for (uint64_t r = 0; r < K; r++) {
        const int b = (int)((K - 1 - r) & 1);  // the last run sorts into out[0]
        const uint64_t off = r * R, len = std::min<uint64_t>(R, n - off);
        bounds[r] = off;
        if (r >= 2) e = hipStreamWaitEvent(P.h2d, P.ev[1][b], 0);
        if (e == hipSuccess) e = hipMemcpyAsync(in[b], src + off * kRec, len * kRec, hipMemcpyHostToDevice, P.h2d);
        if (e == hipSuccess) e = hipEventRecord(P.ev[0][b], P.h2d);
        if (e == hipSuccess) e = hipStreamWaitEvent(P.cs, P.ev[0][b], 0);
        if (e == hipSuccess && r >= 2) e = hipStreamWaitEvent(P.cs, P.ev[2][b], 0);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external: enqueue");
        if ((rc = sort_device_ws(in[b], len, out[b], P.cs, t, ws))) return rc;
        e = launch_guard_or(ws, len, t, guard, P.cs);
        if (e == hipSuccess) e = hipEventRecord(P.ev[1][b], P.cs);
        if (e == hipSuccess && r + kept < K) {  // not a kept run: to host_runs
            e = hipStreamWaitEvent(P.d2h, P.ev[1][b], 0);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dst + off * kRec, out[b], len * kRec, hipMemcpyDeviceToHost, P.d2h);
            if (e == hipSuccess) e = hipEventRecord(P.ev[2][b], P.d2h);
        }
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external: enqueue");
    }
    if ((rc = P.finish())) return rc;
    uint32_t g = 0;
    e = hipMemcpy(&g, guard, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external: guard word");
    if (g) return fail(LEYENDA_EINTERNAL, "leyenda_sort_external: a device-side guard fired in a run's sort (0x%x)", g);
    uint8_t *out_h = static_cast<uint8_t *>(host_out);
    if (K == 1) {  // one run: it is the output
        if (direct_out) {
            e = hipMemcpyAsync(out_h, keep, n * kRec, hipMemcpyDeviceToHost, P.d2h);
            if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external: download");
            return P.finish();
        }
        BounceLease bounce;
        if ((rc = bounce.take())) return rc;
        if ((rc = bounce.b->drain(keep, out_h, n * kRec, P.ev[1][0], P.d2h))) return rc;
        return P.finish();
    }
    if (!kept) {  // every run is in host_runs: the merge as leyenda_merge runs it
        P.release_arena();
        return merge_impl(P, runs_dev, dst, bounds.data(), K, out_h, direct_out, device_budget_bytes, nullptr,
                          Resident{{nullptr, nullptr}, (uint32_t)K});
    }
    const Resident res = kept == 2 ? Resident{{out[1], out[0]}, (uint32_t)(K - 2)}
                                   : Resident{{out[0], nullptr}, (uint32_t)(K - 1)};
    return merge_impl(P, runs_dev, dst, bounds.data(), K, out_h, direct_out, x.merge_budget, base + kept * rb, res);
}

// ---------------------------------------------------------------------------
// Keys-only external sort: every record's (key, index) tuple is extracted as
// the input streams in, and all tuples are sorted on the device at once (the
// tuples of the whole input fit the device budget, so there are no runs to
// merge).  Then, as Section 3.2 does with key-pointer tuples extracted while
// reading, the records are scattered by the sorted tuples: into a pinned
// output, by a second in-order pass over the input that writes every record
// to its place; into a pageable output, which the device cannot write, by a
// gather in sorted order from the pinned input into pinned bounce buffers
// that the host copies out.

extern "C" int leyenda_sort_external_keys(const void *host_records, uint64_t n, uint64_t device_budget_bytes,
                                          void *host_out, void *stream) {
    if (n == 0) return LEYENDA_OK;
    if (n > LEYENDA_MAX_RECORDS)
        return fail(LEYENDA_ETOOBIG, "leyenda_sort_external_keys: %llu records exceed the per-sort limit",
                    (unsigned long long)n);
    if (!host_records || !host_out) return fail(LEYENDA_EINVAL, "leyenda_sort_external_keys: NULL buffer");
    if ((reinterpret_cast<uintptr_t>(host_records) | reinterpret_cast<uintptr_t>(host_out)) & 3u)
        return fail(LEYENDA_EINVAL, "leyenda_sort_external_keys: buffers must be 4-byte aligned");
    if (overlaps(host_records, n * kRec, host_out, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_sort_external_keys: host_out overlaps host_records");
    const uint8_t *rec_dev = static_cast<const uint8_t *>(pinned_device_ptr(host_records));
    if (!rec_dev)
        return fail(LEYENDA_EINVAL, "leyenda_sort_external_keys: host_records must be pinned (hipHostMalloc / pin_memory)");
    const bool direct_out = pinned_device_ptr(host_out) != nullptr;
    const Tune t = tune_of(current_params());
    const Layout L = plan_layout(n, 1, t);
    const uint64_t need = L.total + 256;
    if (need > device_budget_bytes)
        return fail(LEYENDA_EBUDGET,
                    "leyenda_sort_external_keys: the tuples and sort tables of %llu records need %llu device bytes, "
                    "above the budget of %llu (runs + merge fit smaller budgets)",
                    (unsigned long long)n, (unsigned long long)need, (unsigned long long)device_budget_bytes);
    Pipe P;
    int rc = P.init(static_cast<hipStream_t>(stream));
    if (rc) return rc;
    if ((rc = P.alloc(need, device_budget_bytes))) return rc;
    char *base = static_cast<char *>(P.arena);
    uint64_t *H0 = reinterpret_cast<uint64_t *>(base + L.off_H0);
    uint64_t *L0 = reinterpret_cast<uint64_t *>(base + L.off_L0);
    const uint32_t *idx = reinterpret_cast<const uint32_t *>(base + L.off_idx);
    uint32_t *guard = reinterpret_cast<uint32_t *>(base + L.total);
    hipError_t e = hipMemsetAsync(guard, 0, 4, P.cs);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: guard word");

    // 1. read: the input streams through two staging areas that are the
    //    second tuple buffers (H1, L1; the sort first writes them in its
    //    first partition pass), each chunk's tuples extracted on arrival
    uint8_t *stage_in[2] = {reinterpret_cast<uint8_t *>(base + L.off_H1), reinterpret_cast<uint8_t *>(base + L.off_L1)};
    const uint64_t cap_in = std::min<uint64_t>(L.off_L0 - L.off_H1, L.off_idx - L.off_L1) / kRec;
    const uint64_t C1 = std::max<uint64_t>(1, std::min<uint64_t>(cap_in, 16ull << 20));
    const uint8_t *src = static_cast<const uint8_t *>(host_records);
    for (uint64_t c0 = 0, c = 0; c0 < n; c0 += C1, c++) {
        const int b = (int)(c & 1);
        const uint64_t len = std::min<uint64_t>(C1, n - c0);
        if (c >= 2) e = hipStreamWaitEvent(P.h2d, P.ev[1][b], 0);  // extraction of chunk c - 2 done
        if (e == hipSuccess) e = hipMemcpyAsync(stage_in[b], src + c0 * kRec, len * kRec, hipMemcpyHostToDevice, P.h2d);
        if (e == hipSuccess) e = hipEventRecord(P.ev[0][b], P.h2d);
        if (e == hipSuccess) e = hipStreamWaitEvent(P.cs, P.ev[0][b], 0);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: read");
        k_extract_chunk<<<dim3((uint32_t)((len + kWG - 1) / kWG)), dim3(kWG), 0, P.cs>>>(stage_in[b], len, c0, H0, L0);
        if ((e = hipGetLastError()) == hipSuccess) e = hipEventRecord(P.ev[1][b], P.cs);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: extraction");
    }

    // 2. sort all tuples (Algorithm 1 on the device, one pass)
    if ((rc = sort_tuples_ws(n, P.cs, t, base))) return rc;
    if ((e = launch_guard_or(base, n, t, guard, P.cs)) != hipSuccess) return hip_fail(e, "guard kernel");

    if (direct_out) {
        // 3. scatter (pinned output): the place of every input record in the
        //    output (in H0, free after the sort), then the input streams up a
        //    second time, in order, through the same staging areas as the
        //    first read, and every record is written straight to its place in
        //    host_out.  Random writes into pinned host memory run about 1.5x
        //    as fast as random reads of it, and they share the link with the
        //    in-order upload running the other way.
        uint32_t *dest = reinterpret_cast<uint32_t *>(base + L.off_H0);
        uint8_t *out_dev = static_cast<uint8_t *>(pinned_device_ptr(host_out));
        e = hipMemsetAsync(dest, 0xFF, n * 4, P.cs);  // a place no tuple sets stays out of range
        if (e == hipSuccess) {
            k_invert<<<dim3((uint32_t)((n + kWG - 1) / kWG)), dim3(kWG), 0, P.cs>>>(idx, n, dest, guard);
            e = hipGetLastError();
        }
        // the staging areas are sort buffers: the first upload waits for the sort
        if (e == hipSuccess) e = hipEventRecord(P.ev[1][0], P.cs);
        if (e == hipSuccess) e = hipEventRecord(P.ev[1][1], P.cs);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: output places");
        for (uint64_t c0 = 0, c = 0; c0 < n; c0 += C1, c++) {
            const int b = (int)(c & 1);
            const uint64_t len = std::min<uint64_t>(C1, n - c0);
            e = hipStreamWaitEvent(P.h2d, P.ev[1][b], 0);  // the sort, or the scatter of chunk c - 2, done
            if (e == hipSuccess) e = hipMemcpyAsync(stage_in[b], src + c0 * kRec, len * kRec, hipMemcpyHostToDevice, P.h2d);
            if (e == hipSuccess) e = hipEventRecord(P.ev[0][b], P.h2d);
            if (e == hipSuccess) e = hipStreamWaitEvent(P.cs, P.ev[0][b], 0);
            if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: second read");
            k_scatter_chunk<<<dim3((uint32_t)((len + kWG - 1) / kWG)), dim3(kWG), 0, P.cs>>>(stage_in[b], len,
                                                                                          dest + c0, n, out_dev, guard);
            if ((e = hipGetLastError()) == hipSuccess) e = hipEventRecord(P.ev[1][b], P.cs);
            if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: scatter");
        }
        if ((rc = P.finish())) return rc;
        uint32_t g = 0;
        e = hipMemcpy(&g, guard, 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: guard word");
        if (g) return fail(LEYENDA_EINTERNAL, "leyenda_sort_external_keys: a device-side guard fired (0x%x)", g);
        return LEYENDA_OK;
    }

    // 3. gather (pageable output): records gathered in sorted order from the
    //    pinned input straight into the pinned bounce buffers (device stores
    //    through their mapping), a piece at a time; the host copies each piece
    //    into host_out while the next pieces fill.  (Gathered into device
    //    staging and then copied into the bounce buffers, the copies shared
    //    the CUs with the next gather and ran at 16 GB/s, below the gather.)
    uint8_t *out_h = static_cast<uint8_t *>(host_out);
    BounceLease bounce;
    if ((rc = bounce.take())) return rc;
    Bounce &B = *bounce.b;
    constexpr int kB = Bounce::kBufs;
    uint8_t *pdev[kB];
    for (int i = 0; i < kB; i++)
        if (!(pdev[i] = static_cast<uint8_t *>(pinned_device_ptr(B.buf[i]))))
            return fail(LEYENDA_EHIP, "leyenda_sort_external_keys: a bounce buffer has no device mapping");
    const uint64_t per = Bounce::kPiece / kRec;
    uint64_t pend_first[kB] = {}, pend_len[kB] = {};
    for (uint64_t piece = 0, issued = 0;; piece++) {
        const int p = (int)(piece % kB);
        if (pend_len[p]) {  // the oldest piece: copied out while the others gather
            if ((e = hipEventSynchronize(B.ev[p])) != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: gather");
            B.team.copy(out_h + pend_first[p] * kRec, B.buf[p], pend_len[p] * kRec);
            pend_len[p] = 0;
        }
        if (issued < n) {
            const uint64_t len = std::min<uint64_t>(per, n - issued);
            e = launch_gather_single(rec_dev, n, idx + issued, pdev[p], len, P.cs);
            if (e == hipSuccess) e = hipEventRecord(B.ev[p], P.cs);
            if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: gather");
            pend_first[p] = issued;
            pend_len[p] = len;
            issued += len;
        } else {
            bool any = false;
            for (int q = 0; q < kB; q++) any = any || pend_len[q];
            if (!any) break;
        }
    }
    if ((rc = P.finish())) return rc;
    uint32_t g = 0;
    e = hipMemcpy(&g, guard, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "leyenda_sort_external_keys: guard word");
    if (g) return fail(LEYENDA_EINTERNAL, "leyenda_sort_external_keys: a device-side guard fired in the sort (0x%x)", g);
    return LEYENDA_OK;
}

namespace ley {

bool external_holds_any() {
    std::lock_guard<std::mutex> lk(g_ext_mu);
    for (int d = 0; d < 64; d++)
        if (g_ext[d].p || g_bounce[d]) return true;
    return false;
}

// Frees the kept arenas and bounce sets that no call is using (the device has
// been synchronised by the caller).
void external_release_all() {
    std::lock_guard<std::mutex> lk(g_ext_mu);
    for (int d = 0; d < 64; d++) {
        if (g_ext[d].p && !g_ext[d].busy) {
            (void)hipFree(g_ext[d].p);
            g_ext[d].p = nullptr;
            g_ext[d].bytes = 0;
        }
        if (g_bounce[d] && !g_bounce_busy[d]) g_bounce[d].reset();
    }
}

}  // namespace ley
