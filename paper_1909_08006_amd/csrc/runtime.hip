// Host runtime of the record sorter: parameters, workspace pool, argument
// checks and the leyenda_sort entry point (C ABI declared in leyenda.h).
#include <hip/hip_runtime.h>

#include <atomic>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/leyenda.h"
#include "common.h"
#include "runtime.h"

namespace ley {

// ---------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LEYENDA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// parameters

static std::mutex g_param_mu;
static leyenda_params g_params = {8, 32, 2048, 128, 2048, 1024, 512, kFirstFused};

leyenda_params current_params() {
    std::lock_guard<std::mutex> lk(g_param_mu);
    return g_params;
}

Tune tune_of(const leyenda_params &p) {
    Tune t;
    t.digit = p.digit_bits;
    t.tile_items = p.tile_items;
    t.tile = kWG * p.tile_items;
    t.big = p.big_threshold;
    t.tiny = p.tiny_threshold;
    t.scatter_wg = p.scatter_threads;
    t.local_wg = p.local_threads;
    t.first_pass = p.first_pass;
    return t;
}

static bool params_ok(const leyenda_params &p) {
    return p.digit_bits >= (uint32_t)kMinRB && p.digit_bits <= (uint32_t)kRB &&
           (p.tile_items == 8 || p.tile_items == 16 || p.tile_items == 32) && p.local_capacity == kLocalCap &&
           p.big_threshold >= 1 && p.big_threshold <= p.local_capacity && p.tiny_threshold >= 1 &&
           p.tiny_threshold <= 256 && (p.scatter_threads == 256 || p.scatter_threads == 512 || p.scatter_threads == 1024) &&
           (p.local_threads == 256 || p.local_threads == 512) && p.first_pass <= kFirstRecords;
}

// ---------------------------------------------------------------------------
// device facts

int device_cus() {
    static std::atomic<int> cus[64];  // zero-initialised; 0: not yet read
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int v = cus[dev].load(std::memory_order_relaxed);
    if (!v) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
        cus[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// ---------------------------------------------------------------------------
// workspace layout and pool

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Layout plan_layout(uint64_t n, uint32_t reqs, const Tune &t, uint32_t first_pass) {
    Layout L{};
    L.n = n;
    // a bucket gets a device-wide pass only above the big threshold, except the
    // level-1 buckets of a fused first pass, which all do (up to 256, each with
    // a partly filled last tile)
    const uint64_t fused_extra = first_pass != kFirstSplit ? (uint64_t)kRadix : 0;
    const uint64_t segs = std::max<uint64_t>(reqs, n / ((uint64_t)t.big + 1)) + 1 + fused_extra;
    const uint64_t tiles = (n + t.tile - 1) / t.tile + segs + reqs + fused_extra;
    const uint64_t tasks = 3 * (n / kLocalCap) + 4ull * (levels_for((int)t.digit) + 1) * segs + reqs + 64;
    L.max_seg = (uint32_t)std::min<uint64_t>(segs, 0xFFFFFFFFull);
    L.max_tiles = (uint32_t)std::min<uint64_t>(tiles, 0xFFFFFFFFull);
    L.max_tasks = (uint32_t)std::min<uint64_t>(tasks, 0xFFFFFFFFull);
    L.max_reqs = std::max<uint32_t>(reqs, 1);
    L.max_reps = L.max_tiles;  // a bucket has at most one replica per tile
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    const size_t nn = std::max<uint64_t>(n, 1);
    L.off_H0 = take(nn * 8);
    L.off_H1 = take(nn * 8);
    L.off_L0 = take(nn * 8);
    L.off_L1 = take(nn * 8);
    L.off_idx = take(nn * 4);
    L.off_ctl = take(sizeof(Ctl));
    L.off_seg0 = take((size_t)L.max_seg * sizeof(Seg));
    L.off_seg1 = take((size_t)L.max_seg * sizeof(Seg));
    L.off_rep0 = take((size_t)L.max_reps * kRepWords * 4);
    L.off_rep1 = take((size_t)L.max_reps * kRepWords * 4);
    L.off_ts0 = take((size_t)L.max_tiles * 4);
    L.off_ts1 = take((size_t)L.max_tiles * 4);
    L.off_status = take((size_t)L.max_tiles * kRadix * 8);
    L.off_cstat = take(((size_t)L.max_tiles / kChunkTiles + 1) * kRadix * 8);
    L.off_tasks = take((size_t)kParts * L.max_tasks * sizeof(Task));
    L.off_reqs = take((size_t)L.max_reqs * sizeof(Req));
    L.off_hdr = take(sizeof(Hdr));
    if (first_pass != kFirstSplit) {
        // chunk pool of the fused first pass: every bucket's last chunk may be
        // partly empty, so 256 chunks beyond the keys' own
        const uint64_t C = t.tile;
        L.first_pass = first_pass;
        L.max_chunks = (uint32_t)(n / C + kRadix + 1);
        L.ctab_stride = (uint32_t)(n / C + 2);
        L.off_PH = take((size_t)L.max_chunks * C * 8);
        L.off_PL = take((size_t)L.max_chunks * C * 8);
        L.off_ctab = take((size_t)kRadix * L.ctab_stride * 4);
        L.off_tsrc = take((size_t)L.max_tiles * 4);
        if (first_pass == kFirstRecords) L.off_rpool = take((size_t)L.max_chunks * C * kRec);
    }
    L.total = o;
    return L;
}

Work bind_layout(const Layout &L, void *base) {
    char *b = static_cast<char *>(base);
    Work w{};
    w.H[0] = reinterpret_cast<uint64_t *>(b + L.off_H0);
    w.H[1] = reinterpret_cast<uint64_t *>(b + L.off_H1);
    w.L[0] = reinterpret_cast<uint64_t *>(b + L.off_L0);
    w.L[1] = reinterpret_cast<uint64_t *>(b + L.off_L1);
    w.idx = reinterpret_cast<uint32_t *>(b + L.off_idx);
    w.ctl = reinterpret_cast<Ctl *>(b + L.off_ctl);
    w.segs[0] = reinterpret_cast<Seg *>(b + L.off_seg0);
    w.segs[1] = reinterpret_cast<Seg *>(b + L.off_seg1);
    w.rep[0] = reinterpret_cast<uint32_t *>(b + L.off_rep0);
    w.rep[1] = reinterpret_cast<uint32_t *>(b + L.off_rep1);
    w.tile_seg[0] = reinterpret_cast<uint32_t *>(b + L.off_ts0);
    w.tile_seg[1] = reinterpret_cast<uint32_t *>(b + L.off_ts1);
    w.status = reinterpret_cast<unsigned long long *>(b + L.off_status);
    w.cstat = reinterpret_cast<unsigned long long *>(b + L.off_cstat);
    w.tasks = reinterpret_cast<Task *>(b + L.off_tasks);
    w.reqs = reinterpret_cast<Req *>(b + L.off_reqs);
    w.hdr = reinterpret_cast<Hdr *>(b + L.off_hdr);
    w.n = L.n;
    for (uint64_t &e : w.part_end) e = ~0ull;  // one output part unless the caller splits the sort
    w.nparts = 1;
    w.max_seg = L.max_seg;
    w.max_tiles = L.max_tiles;
    w.max_tasks = L.max_tasks;
    w.max_reqs = L.max_reqs;
    w.max_reps = L.max_reps;
    w.kmask_h = ~0ull;
    w.kmask_l = 0xFFFFu;
    if (L.first_pass != kFirstSplit) {
        w.H[2] = reinterpret_cast<uint64_t *>(b + L.off_PH);
        w.L[2] = reinterpret_cast<uint64_t *>(b + L.off_PL);
        w.ctab = reinterpret_cast<uint32_t *>(b + L.off_ctab);
        w.ctab_stride = L.ctab_stride;
        w.max_chunks = L.max_chunks;
        w.tsrc = reinterpret_cast<uint32_t *>(b + L.off_tsrc);
        if (L.first_pass == kFirstRecords) w.rpool = reinterpret_cast<uint8_t *>(b + L.off_rpool);
    }
    return w;
}

// Side stream of a workspace: the gathers of the output parts run there,
// each after the local sorts of its part (events), so they overlap the local
// sorts of the later parts.
struct Side {
    hipStream_t s = nullptr;
    hipEvent_t ready[kParts] = {};
    hipEvent_t done = nullptr;
};

struct PoolEntry {
    void *ptr = nullptr;
    size_t bytes = 0;
    Layout layout{};
    Side side;
    void *aux[2] = {nullptr, nullptr};  // scratch of the keyed sort's tie rounds
    size_t aux_bytes[2] = {0, 0};
};

static void aux_free(PoolEntry &pe) {
    for (int k = 0; k < 2; k++) {
        if (pe.aux[k]) (void)hipFree(pe.aux[k]);
        pe.aux[k] = nullptr;
        pe.aux_bytes[k] = 0;
    }
}

// Destroys a workspace's side events (the side stream itself is shared).
static void side_destroy(Side &sd) {
    for (hipEvent_t &e : sd.ready)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    if (sd.done) (void)hipEventDestroy(sd.done), sd.done = nullptr;
    sd.s = nullptr;
}

static std::mutex g_pool_mu;
static std::map<std::pair<int, hipStream_t>, PoolEntry> g_pool;
// One side stream per device, shared by the workspaces of every caller stream
// (each keeps its own events).  Streams beyond the device's hardware queues
// share queues and serialise; a side stream per caller stream, kept after a
// large sort, made a later external sort's copy streams share queues with it
// (its stages took 2.1-2.2 s instead of 1.3-1.4 s).
static hipStream_t g_side_stream[64];

// Workspace of at least `bytes` for work on `stream` (one per device and
// stream, so concurrent sorts on different streams never share scratch).
int get_workspace(hipStream_t stream, size_t bytes, void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PoolEntry &pe = g_pool[{dev, stream}];
    if (pe.ptr && pe.bytes >= bytes) { *out = pe.ptr; return LEYENDA_OK; }
    if (pe.ptr) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipFree(pe.ptr);
        pe.ptr = nullptr;
        pe.bytes = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    void *p = nullptr;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LEYENDA_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    pe.ptr = p;
    pe.bytes = bytes;
    *out = p;
    return LEYENDA_OK;
}

int get_aux(hipStream_t stream, int which, size_t bytes, void **out) {
    if (which < 0 || which > 1) return fail(LEYENDA_EINVAL, "get_aux: slot %d", which);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    PoolEntry &pe = g_pool[{dev, stream}];
    if (pe.aux[which] && pe.aux_bytes[which] >= bytes) { *out = pe.aux[which]; return LEYENDA_OK; }
    if (pe.aux[which]) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        e = hipFree(pe.aux[which]);
        pe.aux[which] = nullptr;
        pe.aux_bytes[which] = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    // grow by a quarter beyond the request, so slowly growing calls do not
    // reallocate every time
    const size_t want = bytes + bytes / 4 + 256;
    void *p = nullptr;
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LEYENDA_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    pe.aux[which] = p;
    pe.aux_bytes[which] = want;
    *out = p;
    return LEYENDA_OK;
}

int remember_layout(hipStream_t stream, const Layout &L) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LEYENDA_EHIP;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool[{dev, stream}].layout = L;
    return LEYENDA_OK;
}

// The side stream and events of the workspace of `stream` (created on first use).
static int get_side(hipStream_t stream, Side **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (dev < 0 || dev >= 64) return fail(LEYENDA_EINVAL, "device %d out of range", dev);
    Side &sd = g_pool[{dev, stream}].side;
    if (!sd.s) {
        if (!g_side_stream[dev]) e = hipStreamCreateWithFlags(&g_side_stream[dev], hipStreamNonBlocking);
        for (int k = 0; k < kParts && e == hipSuccess; k++)
            e = hipEventCreateWithFlags(&sd.ready[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            side_destroy(sd);
            return hip_fail(e, "side stream");
        }
        sd.s = g_side_stream[dev];
    }
    *out = &sd;
    return LEYENDA_OK;
}

static int find_workspace(hipStream_t stream, void **ptr, Layout *L) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LEYENDA_EHIP;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.find({dev, stream});
    if (it == g_pool.end() || !it->second.ptr) return fail(LEYENDA_EINVAL, "no sort has run on this stream");
    *ptr = it->second.ptr;
    *L = it->second.layout;
    return LEYENDA_OK;
}

void pool_forget(hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_pool.find({dev, stream});
    if (it == g_pool.end()) return;
    (void)hipStreamSynchronize(stream);
    if (it->second.side.s) (void)hipStreamSynchronize(it->second.side.s);
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    aux_free(it->second);
    side_destroy(it->second.side);
    g_pool.erase(it);
}

int release_all() {
    // nothing held: leave the HIP runtime alone (this also runs at interpreter
    // exit, where the process may never have used a GPU)
    bool any = batch_holds_any() || external_holds_any();
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        any = any || !g_pool.empty();
        for (hipStream_t st : g_side_stream) any = any || st != nullptr;
    }
    if (!any) return LEYENDA_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
    batch_release_all();
    external_release_all();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &kv : g_pool) {
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
        aux_free(kv.second);
        side_destroy(kv.second.side);
    }
    g_pool.clear();
    for (hipStream_t &st : g_side_stream)
        if (st) (void)hipStreamDestroy(st), st = nullptr;
    return LEYENDA_OK;
}

// ---------------------------------------------------------------------------
// argument checks

bool overlaps(const void *a, uint64_t abytes, const void *b, uint64_t bbytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

int check_records(const void *in, const void *out, uint64_t n, const char *who) {
    if (n > LEYENDA_MAX_RECORDS) return fail(LEYENDA_ETOOBIG, "%s: %llu records exceed the per-sort limit", who,
                                             (unsigned long long)n);
    if (!in || !out) return fail(LEYENDA_EINVAL, "%s: NULL buffer", who);
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 3u)
        return fail(LEYENDA_EINVAL, "%s: buffers must be 4-byte aligned", who);
    if (overlaps(in, n * kRec, out, n * kRec)) return fail(LEYENDA_EINVAL, "%s: input and output overlap", who);
    return LEYENDA_OK;
}

// ---------------------------------------------------------------------------
// the single-request sort

__global__ void k_setup_single(Req *reqs, Hdr *hdr, const uint8_t *in, uint8_t *out, uint64_t n,
                               uint32_t tiles) {
    Req r;
    r.in = in; r.out = out; r.start = 0; r.n = n; r.first_tile = 0; r.ntiles = tiles;
    r.rep_first = 0; r.nrep = tiles < (uint32_t)kMaxRep ? tiles : (uint32_t)kMaxRep;
    reqs[0] = r;
    Hdr h;
    h.n_total = n; h.nreq = 1; h.tiles0 = tiles;
    *hdr = h;
}

// ---------------------------------------------------------------------------
// phase timing with HIP events on the sort's own stream

// e: sort start, after extraction, after the levels, after the local sorts,
// end.  When the gather runs per output part on the side stream, g holds an
// event pair around each part's gather and the gather phase is their sum.
struct ProfCall {
    hipEvent_t e[5];
    hipEvent_t g[2 * kParts];
    int ng = 0;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfCall> g_prof_pending;
static double g_prof_ms[4] = {0, 0, 0, 0};
static uint64_t g_prof_calls = 0;

static bool prof_start(ProfCall *pc, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on || g_prof_pending.size() >= 4096) return false;
    }
    for (int i = 0; i < 5; i++) {
        if (hipEventCreate(&pc->e[i]) != hipSuccess) {
            for (int k = 0; k < i; k++) (void)hipEventDestroy(pc->e[k]);
            return false;
        }
    }
    (void)hipEventRecord(pc->e[0], s);
    return true;
}

static void prof_finish(const ProfCall &pc, hipStream_t s) {
    (void)hipEventRecord(pc.e[4], s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(pc);
}

static int prof_drain() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &pc : g_prof_pending) {
        hipError_t e = hipEventSynchronize(pc.e[4]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        for (int i = 0; i < (pc.ng ? 3 : 4); i++) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, pc.e[i], pc.e[i + 1]) == hipSuccess) g_prof_ms[i] += ms;
        }
        for (int k = 0; k < pc.ng; k++) {
            float ms = 0;
            if (hipEventSynchronize(pc.g[2 * k + 1]) == hipSuccess &&
                hipEventElapsedTime(&ms, pc.g[2 * k], pc.g[2 * k + 1]) == hipSuccess)
                g_prof_ms[3] += ms;
        }
        g_prof_calls++;
        for (int i = 0; i < 5; i++) (void)hipEventDestroy(pc.e[i]);
        for (int i = 0; i < 2 * pc.ng; i++) (void)hipEventDestroy(pc.g[i]);
    }
    g_prof_pending.clear();
    return LEYENDA_OK;
}

// Output parts of a single sort of n records: one below 8 Mi records (the
// overlap would not pay for the extra launches), else kParts.
static uint32_t parts_for(uint64_t n) { return n < (8ull << 20) ? 1u : (uint32_t)kParts; }

// Ends of the K output parts: the first parts small, so the first gather
// starts early, the last one large (a gather takes several times longer per
// record than the local sort, so the later local sorts finish under the
// earlier gathers).  Fractions of n: 1/16, 1/16, 1/8, 3/4 (measured against
// equal quarters and three other splits on the 10 GB sort: 10.97 against
// 11.01-11.09 ms).
static void part_bounds(uint64_t n, uint32_t K, uint64_t *end) {
    static const uint32_t kEnd16[kParts] = {1, 2, 4, 16};  // in sixteenths of n
    for (uint32_t k = 0; k < K; k++) end[k] = k + 1 == K ? n : n * kEnd16[k] / 16;
}

// The first pass a single sort of n records takes with parameters t: the
// fused ones only for sorts split into output parts (at least 8 Mi records),
// with a partition tile that holds a fused tile, and look-back words for every
// fused tile; the record copy not when the gather also marks ties, nor when a
// pool slot would not fit the 32-bit index.
uint32_t first_pass_for(uint64_t n, const Tune &t, bool ties) {
    uint32_t fp = t.first_pass;
    if (fp == kFirstSplit || parts_for(n) < 2) return kFirstSplit;
    if (fp == kFirstRecords && ties) fp = kFirstFused;
    if (fuse_tile(fp) > t.tile) return kFirstSplit;
    const Layout L = plan_layout(n, 1, t, fp);
    if ((n + fuse_tile(fp) - 1) / fuse_tile(fp) > L.max_tiles) return kFirstSplit;
    if (fp == kFirstRecords && (uint64_t)L.max_chunks * t.tile >= 0xFFFFFFFFull) fp = kFirstFused;
    return fp;
}

int sort_device(const void *records_dev, uint64_t n, void *out_dev, hipStream_t stream, const Tune &t,
                uint32_t key_bytes, uint8_t *ties) {
    const uint32_t fp = first_pass_for(n, t, ties != nullptr);
    const Layout L = plan_layout(n, 1, t, fp);
    void *ws = nullptr;
    int rc = get_workspace(stream, L.total, &ws);
    if (rc) return rc;
    remember_layout(stream, L);
    return sort_device_ws(records_dev, n, out_dev, stream, t, ws, key_bytes, ties, false, fp);
}

void apply_key_mask(Work &w, uint32_t key_bytes) {
    if (key_bytes < kKeyBytes) {  // bytes key_bytes..9 of the prefix do not take part
        w.kmask_h = key_bytes >= 8 ? ~0ull : ~0ull << (64 - 8 * key_bytes);
        w.kmask_l = key_bytes == 9 ? 0xFF00u : 0u;
    }
}

// Device-side guards: a capacity guard or a bounded wait that gave up leaves
// a bit in the sort's control block instead of touching memory out of bounds.
__global__ void k_guard_or(const Ctl *ctl, uint32_t *acc) {
    const uint32_t g = ctl->guard;
    if (g) atomicOr(acc, g);
}

hipError_t launch_guard_or(const void *ws, uint64_t n, const Tune &t, uint32_t *acc, hipStream_t s) {
    const Layout L = plan_layout(n, 1, t);
    k_guard_or<<<1, 1, 0, s>>>(reinterpret_cast<const Ctl *>(static_cast<const char *>(ws) + L.off_ctl), acc);
    return hipGetLastError();
}

int guard_or_pooled(hipStream_t stream, uint32_t *acc) {
    void *ws = nullptr;
    Layout L{};
    if (find_workspace(stream, &ws, &L) != LEYENDA_OK) return LEYENDA_OK;  // no sort ran on this stream
    k_guard_or<<<1, 1, 0, stream>>>(reinterpret_cast<const Ctl *>(static_cast<const char *>(ws) + L.off_ctl), acc);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "guard kernel");
}

const uint32_t *pooled_sort_idx(hipStream_t stream, uint64_t n) {
    void *ws = nullptr;
    Layout L{};
    if (find_workspace(stream, &ws, &L) != LEYENDA_OK || L.n != n || L.first_pass == kFirstRecords) return nullptr;
    return reinterpret_cast<const uint32_t *>(static_cast<const char *>(ws) + L.off_idx);
}

int sort_tuples_ws(uint64_t n, hipStream_t s, const Tune &t, void *ws) {
    if (n == 0) return LEYENDA_OK;
    const Layout L = plan_layout(n, 1, t);
    const Work w = bind_layout(L, ws);
    const uint32_t tiles0 = (uint32_t)((n + t.tile - 1) / t.tile);
    k_setup_single<<<1, 1, 0, s>>>(w.reqs, w.hdr, nullptr, nullptr, n, tiles0);
    Stage st;
    st.tuples_in = true;
    if (n <= t.big) st.lev_end = 1;  // one bucket, one local-sort task
    const hipError_t e = launch_sort_core(w, t, 1, tiles0, s, device_cus(), nullptr, st);
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "tuple sort kernels");
}

int sort_device_ws(const void *records_dev, uint64_t n, void *out_dev, hipStream_t stream, const Tune &t, void *ws,
                   uint32_t key_bytes, uint8_t *ties, bool bare, uint32_t first_pass) {
    const Layout L = plan_layout(n, 1, t, first_pass);
    Work w = bind_layout(L, ws);
    apply_key_mask(w, key_bytes);
    const uint32_t tiles0 = (uint32_t)((n + t.tile - 1) / t.tile);
    const uint32_t K = parts_for(n);
    if (bare && K > 1) return fail(LEYENDA_EINTERNAL, "a bare sort runs one output part only");
    if (first_pass != kFirstSplit && K < 2) return fail(LEYENDA_EINTERNAL, "a fused first pass needs output parts");
    Side *sd = nullptr;  // K output parts: the gathers run on the side stream
    if (K > 1) {
        const int rc = get_side(stream, &sd);
        if (rc) return rc;
    }
    ProfCall pc;
    const bool prof = !bare && prof_start(&pc, stream);
    k_setup_single<<<1, 1, 0, stream>>>(w.reqs, w.hdr, static_cast<const uint8_t *>(records_dev),
                                        static_cast<uint8_t *>(out_dev), n, tiles0);
    if (K == 1) {
        // at most big_threshold records: the one level-0 bucket becomes a local
        // task as it is, so no deeper level can hold a bucket; launch level 0 only
        Stage st;
        if (n <= t.big) st.lev_end = 1;
        hipError_t e = launch_sort_core(w, t, 1, tiles0, stream, device_cus(), prof ? pc.e + 1 : nullptr, st);
        if (e != hipSuccess) return hip_fail(e, "sort kernels");
        e = launch_gather_single(static_cast<const uint8_t *>(records_dev), n, w.idx,
                                 static_cast<uint8_t *>(out_dev), n, stream, ties);
        if (prof) prof_finish(pc, stream);
        if (e != hipSuccess) return hip_fail(e, "gather kernel");
        return LEYENDA_OK;
    }
    // K output parts: the local sorts of part k, then (side stream) its gather
    Work wp = w;
    wp.nparts = K;
    part_bounds(n, K, wp.part_end);
    bool pg = false;  // per-part gather events (else the gather phase is what follows the local sorts)
    if (prof) {
        int made = 0;
        while (made < (int)(2 * K) && hipEventCreate(&pc.g[made]) == hipSuccess) made++;
        if (made == (int)(2 * K)) {
            pc.ng = (int)K;
            pg = true;
        } else {
            for (int i = 0; i < made; i++) (void)hipEventDestroy(pc.g[i]);
        }
    }
    Stage st;
    st.tail = false;
    st.first = first_pass;
    hipError_t e = launch_sort_core(wp, t, 1, tiles0, stream, device_cus(), prof ? pc.e + 1 : nullptr, st);
    // the gather reads the caller's records, or the record pool of the first pass
    const uint8_t *rec = static_cast<const uint8_t *>(records_dev);
    uint64_t n_rec = n;
    if (first_pass == kFirstRecords) {
        rec = w.rpool;
        n_rec = (uint64_t)L.max_chunks * t.tile;
    }
    uint8_t *out = static_cast<uint8_t *>(out_dev);
    for (uint32_t k = 0; k < K && e == hipSuccess; k++) {
        const uint64_t c0 = k ? wp.part_end[k - 1] : 0, c1 = wp.part_end[k];
        e = launch_local_part(wp, t, stream, device_cus(), (int)k);
        if (e == hipSuccess) e = hipEventRecord(sd->ready[k], stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(sd->s, sd->ready[k], 0);
        if (e == hipSuccess && pg) e = hipEventRecord(pc.g[2 * k], sd->s);
        if (e == hipSuccess && c1 > c0)
            e = launch_gather_single(rec, n_rec, w.idx + c0, out + c0 * kRec, c1 - c0, sd->s,
                                     ties ? ties + c0 : nullptr, c0 > 0);
        if (e == hipSuccess && pg) e = hipEventRecord(pc.g[2 * k + 1], sd->s);
    }
    if (e == hipSuccess && prof) e = hipEventRecord(pc.e[3], stream);
    if (e == hipSuccess) e = hipEventRecord(sd->done, sd->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, sd->done, 0);
    if (prof) prof_finish(pc, stream);
    if (e != hipSuccess) return hip_fail(e, "sort kernels");
    return LEYENDA_OK;
}

}  // namespace ley

using namespace ley;

// ---------------------------------------------------------------------------
// C ABI

extern "C" int leyenda_sort(const void *records_dev, uint64_t n, void *out_dev, void *stream) {
    if (n == 0) return LEYENDA_OK;
    int rc = check_records(records_dev, out_dev, n, "leyenda_sort");
    if (rc) return rc;
    return sort_device(records_dev, n, out_dev, static_cast<hipStream_t>(stream), tune_of(current_params()));
}

// ---------------------------------------------------------------------------
// leyenda_sort_noalloc: the same sort with its scratch in a fixed device array

namespace ley {

// The no-alloc sort's workspace: one copy per GPU, held until the process
// ends.  In host code the array's name is not a device address; the address
// comes from hipGetSymbolAddress once per device.
constexpr size_t kNoAllocBytes = 64ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device, with the device current).
static int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(LEYENDA_EINVAL, "leyenda_sort_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LEYENDA_OK;
}

// Largest record count whose workspace fits the array with parameters t
// (plan_layout grows with n, so a binary search finds it).
static uint64_t noalloc_max_records(const Tune &t) {
    uint64_t lo = 0, hi = kNoAllocBytes / 32;  // the tuples alone take 32 B per record
    while (lo < hi) {
        const uint64_t m = lo + (hi - lo + 1) / 2;
        if (plan_layout(m, 1, t).total <= kNoAllocBytes) lo = m; else hi = m - 1;
    }
    return lo;
}

}  // namespace ley

extern "C" uint64_t leyenda_noalloc_max_records(void) { return noalloc_max_records(tune_of(current_params())); }

extern "C" int leyenda_sort_noalloc(const void *records_dev, uint64_t n, void *out_dev, void *stream) {
    if (n == 0) return LEYENDA_OK;
    int rc = check_records(records_dev, out_dev, n, "leyenda_sort_noalloc");
    if (rc) return rc;
    const Tune t = tune_of(current_params());
    const Layout L = plan_layout(n, 1, t);
    if (L.total > kNoAllocBytes)
        return fail(LEYENDA_EBUDGET,
                    "leyenda_sort_noalloc: %llu records need %zu bytes of scratch, above the fixed %zu "
                    "(at most %llu records with the current parameters)",
                    (unsigned long long)n, L.total, kNoAllocBytes,
                    (unsigned long long)noalloc_max_records(t));
    void *ws = nullptr;
    if ((rc = scratch_ptr(&ws))) return rc;
    // the kernels clear what they read before writing it (control block,
    // replicas, look-back words), so the array's old contents do not matter
    return sort_device_ws(records_dev, n, out_dev, static_cast<hipStream_t>(stream), t, ws, kKeyBytes, nullptr,
                          true);
}

extern "C" uint32_t leyenda_sort_parts(uint64_t n) { return parts_for(n); }

extern "C" uint32_t leyenda_first_pass(uint64_t n) { return first_pass_for(n, tune_of(current_params()), false); }

extern "C" uint64_t leyenda_workspace_bytes(uint64_t n) {
    const Tune t = tune_of(current_params());
    return plan_layout(n, 1, t, first_pass_for(n, t, false)).total;
}

extern "C" int leyenda_get_params(leyenda_params *out) {
    if (!out) return fail(LEYENDA_EINVAL, "leyenda_get_params: NULL");
    *out = current_params();
    return LEYENDA_OK;
}

extern "C" int leyenda_set_params(const leyenda_params *p) {
    if (!p || !params_ok(*p)) return fail(LEYENDA_EINVAL, "leyenda_set_params: parameter out of range");
    std::lock_guard<std::mutex> lk(g_param_mu);
    g_params = *p;
    return LEYENDA_OK;
}

static bool json_field(const std::string &s, const char *name, uint32_t *v) {
    const std::string key = std::string("\"") + name + "\"";
    size_t p = s.find(key);
    if (p == std::string::npos) return false;
    p = s.find(':', p + key.size());
    if (p == std::string::npos) return false;
    *v = (uint32_t)strtoul(s.c_str() + p + 1, nullptr, 10);
    return true;
}

extern "C" int leyenda_load_params(const char *json_path) {
    if (!json_path) return fail(LEYENDA_EINVAL, "leyenda_load_params: NULL path");
    FILE *f = fopen(json_path, "rb");
    if (!f) return fail(LEYENDA_EINVAL, "leyenda_load_params: cannot open %s", json_path);
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, k);
    fclose(f);
    leyenda_params p = current_params();
    json_field(s, "digit_bits", &p.digit_bits);
    json_field(s, "tile_items", &p.tile_items);
    json_field(s, "big_threshold", &p.big_threshold);
    json_field(s, "tiny_threshold", &p.tiny_threshold);
    json_field(s, "local_capacity", &p.local_capacity);
    json_field(s, "scatter_threads", &p.scatter_threads);
    json_field(s, "local_threads", &p.local_threads);
    json_field(s, "first_pass", &p.first_pass);
    return leyenda_set_params(&p);
}

extern "C" int leyenda_sort_stats(void *stream, leyenda_stats *out) {
    if (!out) return fail(LEYENDA_EINVAL, "leyenda_sort_stats: NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    Layout L{};
    int rc = find_workspace(s, &ws, &L);
    if (rc) return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    Ctl c;
    e = hipMemcpy(&c, static_cast<char *>(ws) + L.off_ctl, sizeof(Ctl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    memset(out, 0, sizeof(*out));
    for (int l = 0; l < kMaxLev && l < LEYENDA_MAX_LEVELS; l++) {
        out->segments[l] = c.nseg[l];
        out->moved[l] = c.moved[l];
        if (c.moved[l]) out->levels = l + 1;
    }
    out->tasks = 0;
    for (int p = 0; p < kParts; p++) out->tasks += c.ntask[p];
    out->guard = c.guard;
    return LEYENDA_OK;
}

extern "C" const char *leyenda_status_string(int status) {
    switch (status) {
        case LEYENDA_OK: return "ok";
        case LEYENDA_EINVAL: return "invalid argument";
        case LEYENDA_ENOMEM: return "out of memory";
        case LEYENDA_EBUDGET: return "does not fit the device budget";
        case LEYENDA_EHIP: return "HIP runtime error";
        case LEYENDA_ETOOBIG: return "too many records";
        case LEYENDA_EINTERNAL: return "internal capacity guard";
        default: return "unknown status";
    }
}

extern "C" const char *leyenda_last_error(void) { return g_last_error.c_str(); }

extern "C" int leyenda_release_workspaces(void) { return release_all(); }

extern "C" int leyenda_profile_enable(int on) {
    int rc = prof_drain();
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    for (double &v : g_prof_ms) v = 0;
    g_prof_calls = 0;
    return LEYENDA_OK;
}

extern "C" int leyenda_profile_read(double *phase_ms, uint64_t *calls) {
    if (!phase_ms || !calls) return fail(LEYENDA_EINVAL, "leyenda_profile_read: NULL");
    int rc = prof_drain();
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < 4; i++) phase_ms[i] = g_prof_ms[i];
    *calls = g_prof_calls;
    return LEYENDA_OK;
}

// Sum of a bucket's histogram replicas (one thread per digit).
__global__ void k_rep_sum(const uint32_t *rep, uint32_t nrep, uint32_t *hist) {
    const uint32_t d = threadIdx.x;
    uint32_t v = 0;
    for (uint32_t r = 0; r < nrep; r++) v += rep[(size_t)r * kRepWords + d];
    hist[d] = v;
}

extern "C" int leyenda_debug_extract(const void *records_dev, uint64_t n, uint32_t key_bytes, uint64_t *hi_dev,
                                     uint64_t *lo_dev, uint32_t *hist_dev, void *stream) {
    if (n == 0) return LEYENDA_OK;
    if (n > LEYENDA_MAX_RECORDS) return fail(LEYENDA_ETOOBIG, "leyenda_debug_extract: too many records");
    if (key_bytes < 1 || key_bytes > kKeyBytes)
        return fail(LEYENDA_EINVAL, "leyenda_debug_extract: key_bytes %u outside 1..10", key_bytes);
    if (!records_dev || !hi_dev || !lo_dev || !hist_dev) return fail(LEYENDA_EINVAL, "leyenda_debug_extract: NULL");
    if ((reinterpret_cast<uintptr_t>(records_dev) & 3u) || (reinterpret_cast<uintptr_t>(hi_dev) & 7u) ||
        (reinterpret_cast<uintptr_t>(lo_dev) & 7u) || (reinterpret_cast<uintptr_t>(hist_dev) & 3u))
        return fail(LEYENDA_EINVAL, "leyenda_debug_extract: misaligned buffer");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the sort's own first stage: request table, level-0 bucket, then the
    // extraction kernel the sort launches (same masks, tiles and replicas)
    const Tune t = tune_of(current_params());
    const Layout L = plan_layout(n, 1, t);
    void *ws = nullptr;
    int rc = get_workspace(s, L.total, &ws);
    if (rc) return rc;
    remember_layout(s, L);
    Work w = bind_layout(L, ws);
    apply_key_mask(w, key_bytes);
    const uint32_t tiles0 = (uint32_t)((n + t.tile - 1) / t.tile);
    k_setup_single<<<1, 1, 0, s>>>(w.reqs, w.hdr, static_cast<const uint8_t *>(records_dev), nullptr, n, tiles0);
    Stage st;
    st.lev_end = 0;  // extraction only
    st.tail = false;
    hipError_t e = launch_sort_core(w, t, 1, tiles0, s, device_cus(), nullptr, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hi_dev, w.H[0], n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lo_dev, w.L[0], n * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) {
        k_rep_sum<<<1, kRadix, 0, s>>>(w.rep[0], tiles0 < (uint32_t)kMaxRep ? tiles0 : (uint32_t)kMaxRep, hist_dev);
        e = hipGetLastError();
    }
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "extract kernel");
}

namespace ley {

// The level-0 buckets a fused first pass left in its chunk pool, copied out in
// bucket order (bucket d at the sum of the counts before it, positions in
// order), with each bucket's count and, for the record copy, its records.
__global__ __launch_bounds__(kWG) void k_flatten0(Work w, Tune tu, uint64_t *hi, uint64_t *lo, uint32_t *count,
                                                  uint8_t *rec_out) {
    const uint32_t ntl = min(w.ctl->ntiles[1], w.max_tiles);
    const uint32_t nseg = min(w.ctl->nseg[1], w.max_seg);
    const uint32_t C = tu.tile;
    for (uint32_t t = blockIdx.x; t < ntl; t += gridDim.x) {
        const uint32_t s = w.tile_seg[1][t];
        if (s >= nseg) continue;
        const Seg sg = w.segs[1][s];
        const uint32_t k = t - sg.first_tile, c = w.tsrc[t];
        if (sg.buf != 2 || k >= sg.ntiles || c >= w.max_chunks || sg.start + sg.count > w.n) continue;
        const uint32_t nvalid = min(C, sg.count - k * C);
        const uint64_t src = (uint64_t)c * C, dst = sg.start + (uint64_t)k * C;
        if (k == 0 && threadIdx.x == 0) count[(uint32_t)(w.H[2][src] >> (64 - tu.digit))] = sg.count;
        for (uint32_t q = threadIdx.x; q < nvalid; q += kWG) {
            hi[dst + q] = w.H[2][src + q];
            lo[dst + q] = w.L[2][src + q];
        }
        if (rec_out && w.rpool)
            for (uint64_t b = threadIdx.x; b < (uint64_t)nvalid * kRec; b += kWG)
                rec_out[dst * kRec + b] = w.rpool[src * kRec + b];
    }
}

}  // namespace ley

extern "C" int leyenda_debug_first_pass(const void *records_dev, uint64_t n, uint32_t first_pass, uint32_t key_bytes,
                                        uint64_t *hi_dev, uint64_t *lo_dev, uint32_t *count_dev, void *rec_out_dev,
                                        void *stream) {
    if (n == 0) return LEYENDA_OK;
    if (n > LEYENDA_MAX_RECORDS) return fail(LEYENDA_ETOOBIG, "leyenda_debug_first_pass: too many records");
    if (first_pass != kFirstFused && first_pass != kFirstRecords)
        return fail(LEYENDA_EINVAL, "leyenda_debug_first_pass: first_pass %u is not 1 or 2", first_pass);
    if (key_bytes < 1 || key_bytes > kKeyBytes)
        return fail(LEYENDA_EINVAL, "leyenda_debug_first_pass: key_bytes %u outside 1..10", key_bytes);
    if (!records_dev || !hi_dev || !lo_dev || !count_dev || (first_pass == kFirstRecords && !rec_out_dev))
        return fail(LEYENDA_EINVAL, "leyenda_debug_first_pass: NULL");
    if ((reinterpret_cast<uintptr_t>(records_dev) & 3u) || (reinterpret_cast<uintptr_t>(hi_dev) & 7u) ||
        (reinterpret_cast<uintptr_t>(lo_dev) & 7u) || (reinterpret_cast<uintptr_t>(count_dev) & 3u))
        return fail(LEYENDA_EINVAL, "leyenda_debug_first_pass: misaligned buffer");
    const Tune t = tune_of(current_params());
    const Layout L = plan_layout(n, 1, t, first_pass);
    if (fuse_tile(first_pass) > t.tile || (n + fuse_tile(first_pass) - 1) / fuse_tile(first_pass) > L.max_tiles ||
        (first_pass == kFirstRecords && (uint64_t)L.max_chunks * t.tile >= 0xFFFFFFFFull))
        return fail(LEYENDA_EINVAL, "leyenda_debug_first_pass: the parameters do not allow first pass %u", first_pass);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    int rc = get_workspace(s, L.total, &ws);
    if (rc) return rc;
    remember_layout(s, L);
    Work w = bind_layout(L, ws);
    apply_key_mask(w, key_bytes);
    const uint32_t tiles0 = (uint32_t)((n + t.tile - 1) / t.tile);
    k_setup_single<<<1, 1, 0, s>>>(w.reqs, w.hdr, static_cast<const uint8_t *>(records_dev), nullptr, n, tiles0);
    // the sort's own first pass, launched as the sort launches it, and nothing after
    Stage st;
    st.first = first_pass;
    st.lev_end = 1;
    st.tail = false;
    hipError_t e = launch_sort_core(w, t, 1, tiles0, s, device_cus(), nullptr, st);
    if (e == hipSuccess) e = hipMemsetAsync(count_dev, 0, kRadix * 4, s);
    if (e == hipSuccess) {
        k_flatten0<<<dim3(device_cus() * 4), dim3(kWG), 0, s>>>(w, t, hi_dev, lo_dev, count_dev,
                                                               static_cast<uint8_t *>(rec_out_dev));
        e = hipGetLastError();
    }
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "first pass kernels");
}

extern "C" int leyenda_debug_gather(const void *records_dev, uint64_t n_records, const uint32_t *idx_dev,
                                    uint64_t n, void *out_dev, void *stream) {
    if (n == 0) return LEYENDA_OK;
    if (n > LEYENDA_MAX_RECORDS || n_records > LEYENDA_MAX_RECORDS)
        return fail(LEYENDA_ETOOBIG, "leyenda_debug_gather: too many records");
    if (!records_dev || !idx_dev || !out_dev) return fail(LEYENDA_EINVAL, "leyenda_debug_gather: NULL");
    if (overlaps(records_dev, n_records * kRec, out_dev, n * kRec))
        return fail(LEYENDA_EINVAL, "leyenda_debug_gather: input and output overlap");
    hipError_t e = launch_gather_single(static_cast<const uint8_t *>(records_dev), n_records, idx_dev,
                                        static_cast<uint8_t *>(out_dev), n, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? LEYENDA_OK : hip_fail(e, "gather kernel");
}
