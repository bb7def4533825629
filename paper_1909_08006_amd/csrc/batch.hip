// Batched sort: many independent requests sorted by one launch sequence.
//
// Each request becomes a level-0 bucket of the same device-driven MSD schedule
// the single sort uses (Algorithm 1 applied across requests: big buckets of
// every request share the partition passes, small buckets of every request
// share one local-sort task queue), so requests never mix and each one comes
// out exactly as leyenda_sort would sort it.  Kernel grids are fixed and every
// size is read from device tables, so the whole sequence is captured once per
// stream into a HIP graph and replayed for every batch that fits the captured
// capacity; the per-batch request table travels host -> device before each
// replay.
//
// An engine built for the serving loop ("split") captures two graphs: the
// first runs the levels [0, kSplitLevels) and then the local sorts and the
// gather, which stand down if deeper levels still hold big buckets; a word in
// pinned host memory tells the loop, which then replays the second graph (the
// remaining levels, local sorts, gather).  Inputs of uniform keys need no
// second graph up to 2048 * 256^2 records, so a batch pays the launches of
// kSplitLevels levels instead of all of them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "runtime.h"

namespace ley {

namespace {

constexpr int kSplitLevels = 3;

struct BatchEngine {
    hipStream_t cap = nullptr;
    void *ws = nullptr;
    Layout L{};
    uint64_t n_cap = 0;
    uint32_t r_cap = 0;
    Tune tune{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool split = false;
    hipGraph_t graph2 = nullptr;   // split: the remaining levels, local sorts, gather
    hipGraphExec_t exec2 = nullptr;
    char *stage = nullptr;  // pinned: request table + header (+ the split flag word)
    hipEvent_t staged = nullptr;
    bool staged_pending = false;

    uint32_t *flag() const {  // split: 1 when the second graph is needed
        return reinterpret_cast<uint32_t *>(stage + (size_t)r_cap * sizeof(Req) + sizeof(Hdr));
    }

    void release() {
        if (cap) (void)hipStreamSynchronize(cap);
        if (staged) (void)hipEventSynchronize(staged);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (exec2) (void)hipGraphExecDestroy(exec2);
        if (graph2) (void)hipGraphDestroy(graph2);
        if (ws) (void)hipFree(ws);
        if (stage) (void)hipHostFree(stage);
        if (staged) (void)hipEventDestroy(staged);
        if (cap) (void)hipStreamDestroy(cap);
        const bool keep_split = split;
        *this = BatchEngine{};
        split = keep_split;
    }
};

std::mutex g_batch_mu;
std::map<std::pair<int, hipStream_t>, BatchEngine> g_batch;

bool same_tune(const Tune &a, const Tune &b) {
    return a.digit == b.digit && a.tile_items == b.tile_items && a.tile == b.tile && a.big == b.big && a.tiny == b.tiny &&
           a.scatter_wg == b.scatter_wg && a.local_wg == b.local_wg;
}

// (Re)builds the engine for at least n records and r requests: workspace,
// pinned staging and the captured launch sequence.
int engine_build(BatchEngine &E, hipStream_t user, uint64_t n, uint32_t r, const Tune &t) {
    const bool split = E.split;
    hipError_t e;
    if (user) (void)hipStreamSynchronize(user);
    E.release();
    E.n_cap = std::max<uint64_t>(n, 1 << 12);
    E.r_cap = std::max<uint32_t>(r, 16);
    E.tune = t;
    E.L = plan_layout(E.n_cap, E.r_cap, t);
    if ((e = hipMalloc(&E.ws, E.L.total)) != hipSuccess) {
        (void)hipGetLastError();
        E.ws = nullptr;
        return fail(LEYENDA_ENOMEM, "batch workspace of %zu bytes", E.L.total);
    }
    E.split = split;
    if ((e = hipHostMalloc(reinterpret_cast<void **>(&E.stage), (size_t)E.r_cap * sizeof(Req) + sizeof(Hdr) + 256,
                           hipHostMallocDefault)) != hipSuccess)
        return fail(LEYENDA_ENOMEM, "batch staging: %s", hipGetErrorString(e));
    *E.flag() = 0;
    if ((e = hipEventCreateWithFlags(&E.staged, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    if ((e = hipStreamCreateWithFlags(&E.cap, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    const Work w = bind_layout(E.L, E.ws);
    if ((e = hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    Stage first;
    if (split) {
        first.lev_end = kSplitLevels;
        first.gate = kSplitLevels;
        first.flag = E.flag();
    }
    hipError_t le = launch_sort_core(w, t, 0, 0, E.cap, device_cus(), nullptr, first);
    if (le == hipSuccess) le = launch_gather_batch(w, E.cap, first.gate);
    e = hipStreamEndCapture(E.cap, &E.graph);
    if (le != hipSuccess) return hip_fail(le, "batch capture launches");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "hipGraphInstantiate");
    if (!split) return LEYENDA_OK;
    Stage second;
    second.lev_begin = kSplitLevels;
    second.head = false;
    if ((e = hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    le = launch_sort_core(w, t, 0, 0, E.cap, device_cus(), nullptr, second);
    if (le == hipSuccess) le = launch_gather_batch(w, E.cap);
    e = hipStreamEndCapture(E.cap, &E.graph2);
    if (le != hipSuccess) return hip_fail(le, "batch capture launches (second part)");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&E.exec2, E.graph2, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "hipGraphInstantiate");
    return LEYENDA_OK;
}

int batch_group(const leyenda_segment *segs, uint64_t count, hipStream_t s, const Tune &t) {
    // request table (non-empty segments only), in input order
    std::vector<Req> reqs;
    reqs.reserve(count);
    uint64_t start = 0;
    uint32_t ft = 0, rf = 0;
    for (uint64_t i = 0; i < count; i++) {
        const leyenda_segment &g = segs[i];
        if (g.n == 0) continue;
        Req q;
        q.in = static_cast<const uint8_t *>(g.in);
        q.out = static_cast<uint8_t *>(g.out);
        q.start = start;
        q.n = g.n;
        q.ntiles = (uint32_t)((g.n + t.tile - 1) / t.tile);
        q.first_tile = ft;
        q.nrep = std::min<uint32_t>(q.ntiles, kMaxRep);
        q.rep_first = rf;
        start += g.n;
        ft += q.ntiles;
        rf += q.nrep;
        reqs.push_back(q);
    }
    if (reqs.empty()) return LEYENDA_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchEngine &E = g_batch[{dev, s}];
    const uint32_t nreq = (uint32_t)reqs.size();
    if (!E.exec || start > E.n_cap || nreq > E.r_cap || !same_tune(E.tune, t)) {
        const uint64_t ncap = std::max<uint64_t>(start, E.n_cap + E.n_cap / 2);
        const uint32_t rcap = std::max<uint32_t>(nreq, E.r_cap + E.r_cap / 2);
        int rc = engine_build(E, s, std::min<uint64_t>(ncap, std::max<uint64_t>(start, (uint64_t)1 << 33)),
                              std::min<uint32_t>(rcap, 65535u), t);
        if (rc) { E.release(); return rc; }
    }
    if (E.staged_pending && (e = hipEventSynchronize(E.staged)) != hipSuccess) return hip_fail(e, "staging event");
    Req *sr = reinterpret_cast<Req *>(E.stage);
    Hdr *sh = reinterpret_cast<Hdr *>(E.stage + (size_t)E.r_cap * sizeof(Req));
    std::copy(reqs.begin(), reqs.end(), sr);
    sh->n_total = start;
    sh->nreq = nreq;
    sh->tiles0 = ft;
    const Work w = bind_layout(E.L, E.ws);
    e = hipMemcpyAsync(w.reqs, sr, nreq * sizeof(Req), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(w.hdr, sh, sizeof(Hdr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(E.staged, s);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    E.staged_pending = true;
    if ((e = hipGraphLaunch(E.exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return LEYENDA_OK;
}

}  // namespace

int batch_sort(const leyenda_segment *segs, uint64_t count, hipStream_t s) {
    if (count == 0) return LEYENDA_OK;
    if (!segs) return fail(LEYENDA_EINVAL, "leyenda_sort_batch: NULL segment table");
    uint64_t total = 0;
    for (uint64_t i = 0; i < count; i++) {
        const leyenda_segment &g = segs[i];
        if (g.n == 0) continue;
        int rc = check_records(g.in, g.out, g.n, "leyenda_sort_batch");
        if (rc) return rc;
        total += g.n;
    }
    (void)total;
    const Tune t = tune_of(current_params());
    // groups of at most 65535 requests (request ids are 16-bit on the device)
    if (count > 65535 && batch_is_split(s))
        return fail(LEYENDA_EINVAL, "leyenda_sort_batch: a two-part engine takes at most 65535 requests");
    for (uint64_t i = 0; i < count; i += 65535) {
        int rc = batch_group(segs + i, std::min<uint64_t>(65535, count - i), s, t);
        if (rc) return rc;
    }
    return LEYENDA_OK;
}

// Pre-sizes the batch engine of stream s (used by the serving engine so that
// its device memory is fixed when it is created).
int batch_reserve(hipStream_t s, uint64_t n, uint32_t r, size_t *bytes, bool split) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    const Tune t = tune_of(current_params());
    std::lock_guard<std::mutex> lk(g_batch_mu);
    BatchEngine &E = g_batch[{dev, s}];
    E.split = split;
    int rc = engine_build(E, s, n, std::min<uint32_t>(r, 65535u), t);
    if (rc) { E.release(); return rc; }
    if (bytes) *bytes = E.L.total;
    return LEYENDA_OK;
}

bool batch_is_split(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batch.find({dev, s});
    return it != g_batch.end() && it->second.split;
}

// After the first part of a batch on stream s has completed: replays the
// second part if the first reported deeper levels (returns 1), else 0.
int batch_continue_if_needed(hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batch.find({dev, s});
    if (it == g_batch.end() || !it->second.split || !it->second.exec2) return 0;
    BatchEngine &E = it->second;
    const uint32_t deep = __atomic_load_n(E.flag(), __ATOMIC_ACQUIRE);
    if (!deep) return 0;
    *E.flag() = 0;
    if ((e = hipGraphLaunch(E.exec2, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch (second part)");
    return 1;
}

uint64_t batch_bytes(uint64_t n, uint32_t r) {
    return plan_layout(std::max<uint64_t>(n, 1 << 12), std::max<uint32_t>(r, 16), tune_of(current_params())).total;
}

void batch_forget(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batch.find({dev, s});
    if (it != g_batch.end()) {
        it->second.release();
        g_batch.erase(it);
    }
}

bool batch_holds_any() {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    return !g_batch.empty();
}

void batch_release_all() {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto &kv : g_batch) kv.second.release();
    g_batch.clear();
}

}  // namespace ley

using namespace ley;

extern "C" int leyenda_sort_batch(const leyenda_segment *segs, uint64_t count, void *stream) {
    return batch_sort(segs, count, static_cast<hipStream_t>(stream));
}
