// Serving engine: sort requests arrive over time and are admitted, batched
// and run on one GPU while earlier batches are still in flight (continuous
// batching), under a fixed device-memory budget.
//
// The budget covers everything the engine allocates: one workspace per slot
// (a slot is a stream running one batch at a time) and an arena holding the
// output buffer of every admitted request until the client releases it.  A
// dispatcher thread retires finished batches, then, for every free slot,
// admits queued requests in arrival order while their outputs fit the arena
// and the batch stays under its size caps, and launches them as one batched
// sort (leyenda_sort_batch's captured launch sequence).  With batching off,
// the same loop admits one request at a time and runs one plain leyenda_sort
// per request on a single stream: the baseline it is compared with.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime.h"

namespace ley {

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size), 256-byte granules, coalescing frees.
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> length
    void init(size_t s) {
        free_.clear();
        if (s) free_[0] = s;
    }
    static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
    bool alloc(size_t bytes, size_t *off) {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, o2 = it->first + bytes;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SReq {
    const void *in = nullptr;
    uint64_t n = 0;
    size_t off = 0, bytes = 0;
    double t_submit = 0, t_start = 0, t_done = 0;
    int status = 0;
    bool done = false;
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> tags;
    bool busy = false;
};

}  // namespace

}  // namespace ley

struct leyenda_server {
    leyenda_server_config cfg{};
    int dev = 0;
    ley::Tune tune{};
    void *arena_dev = nullptr;
    ley::Arena arena;
    std::vector<ley::Slot> slots;
    std::deque<uint64_t> queue;
    std::map<uint64_t, ley::SReq> reqs;
    std::deque<uint64_t> done_q;
    std::mutex mu;
    std::condition_variable cv_done;
    std::thread th;
    std::atomic<bool> stop{false};

    void loop();
};

namespace ley {

// The dispatcher: retire finished batches, then fill every free slot.
static void dispatch_once(leyenda_server &S, bool *did) {
    std::vector<leyenda_segment> segs;
    std::unique_lock<std::mutex> lk(S.mu);
    bool retired = false;
    for (Slot &sl : S.slots) {
        if (!sl.busy) continue;
        hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q == hipSuccess && S.cfg.batched) {
            // the first part of a two-part batch: the second part if needed
            const int c = batch_continue_if_needed(sl.s);
            if (c == 1 && hipEventRecord(sl.done, sl.s) == hipSuccess) {
                *did = true;
                continue;
            }
            if (c != 0) q = hipErrorUnknown;
        }
        const double t = now_s();
        for (uint64_t tag : sl.tags) {
            SReq &r = S.reqs[tag];
            r.t_done = t;
            r.done = true;
            if (q != hipSuccess) r.status = LEYENDA_EHIP;
            S.done_q.push_back(tag);
        }
        sl.tags.clear();
        sl.busy = false;
        retired = true;
    }
    if (retired) {
        S.cv_done.notify_all();
        *did = true;
    }
    for (Slot &sl : S.slots) {
        if (sl.busy || S.queue.empty()) continue;
        segs.clear();
        uint64_t recs = 0;
        const double t = now_s();
        while (!S.queue.empty() && sl.tags.size() < S.cfg.max_batch) {
            const uint64_t tag = S.queue.front();
            SReq &r = S.reqs[tag];
            if (recs + r.n > S.cfg.max_batch_records) break;
            size_t off = 0;
            if (!S.arena.alloc(r.n * kRec, &off)) break;  // admission waits for memory
            r.off = off;
            r.bytes = r.n * kRec;
            r.t_start = t;
            segs.push_back(leyenda_segment{r.in, static_cast<char *>(S.arena_dev) + off, r.n});
            sl.tags.push_back(tag);
            S.queue.pop_front();
            recs += r.n;
            if (!S.cfg.batched) break;
        }
        if (sl.tags.empty()) break;  // the oldest request does not fit yet
        int rc = S.cfg.batched ? batch_sort(segs.data(), segs.size(), sl.s)
                               : sort_device(segs[0].in, segs[0].n, segs[0].out, sl.s, S.tune);
        if (hipEventRecord(sl.done, sl.s) != hipSuccess && rc == 0) rc = LEYENDA_EHIP;
        if (rc) {
            for (uint64_t tag : sl.tags) S.reqs[tag].status = rc;
        }
        sl.busy = true;
        *did = true;
    }
}

}  // namespace ley

void leyenda_server::loop() {
    (void)hipSetDevice(dev);
    while (!stop.load()) {
        bool did = false;
        ley::dispatch_once(*this, &did);
        if (!did) std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
}

using namespace ley;

extern "C" int leyenda_server_create(const leyenda_server_config *cfg, leyenda_server **out) {
    if (!cfg || !out) return fail(LEYENDA_EINVAL, "leyenda_server_create: NULL");
    *out = nullptr;
    if (cfg->slots == 0 || cfg->max_batch == 0 || cfg->max_batch_records == 0 ||
        cfg->max_batch_records > LEYENDA_MAX_RECORDS || cfg->max_batch > 65535)
        return fail(LEYENDA_EINVAL, "leyenda_server_create: bad configuration");
    auto *S = new leyenda_server();
    S->cfg = *cfg;
    if (!S->cfg.batched) {
        S->cfg.slots = 1;
        S->cfg.max_batch = 1;
    }
    S->tune = tune_of(current_params());
    hipError_t e = hipGetDevice(&S->dev);
    if (e != hipSuccess) { delete S; return hip_fail(e, "hipGetDevice"); }
    // fixed per-slot workspaces first, the rest of the budget is the output arena
    size_t ws_total = 0;
    for (uint32_t i = 0; i < S->cfg.slots; i++) {
        Slot sl;
        if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
            S->slots.push_back(sl);
            leyenda_server_destroy(S);
            return hip_fail(e, "leyenda_server_create: stream");
        }
        S->slots.push_back(sl);
        const size_t ws = S->cfg.batched ? batch_bytes(S->cfg.max_batch_records, S->cfg.max_batch)
                                         : plan_layout(S->cfg.max_batch_records, 1, S->tune).total;
        ws_total += ws;
    }
    const size_t min_arena = (size_t)S->cfg.max_batch_records * kRec;
    if (ws_total + min_arena > cfg->budget_bytes) {
        leyenda_server_destroy(S);
        return fail(LEYENDA_EBUDGET, "leyenda_server_create: budget below the slot workspaces plus one full batch");
    }
    for (Slot &sl : S->slots) {
        int rc;
        if (S->cfg.batched) {
            rc = batch_reserve(sl.s, S->cfg.max_batch_records, S->cfg.max_batch, nullptr, true);
        } else {
            void *ws = nullptr;
            rc = get_workspace(sl.s, plan_layout(S->cfg.max_batch_records, 1, S->tune).total, &ws);
        }
        if (rc) { leyenda_server_destroy(S); return rc; }
    }
    const size_t arena_bytes = cfg->budget_bytes - ws_total;
    if ((e = hipMalloc(&S->arena_dev, arena_bytes)) != hipSuccess) {
        (void)hipGetLastError();
        S->arena_dev = nullptr;
        leyenda_server_destroy(S);
        return fail(LEYENDA_ENOMEM, "leyenda_server_create: output arena of %zu bytes", arena_bytes);
    }
    S->arena.init(arena_bytes);
    S->th = std::thread([S] { S->loop(); });
    *out = S;
    return LEYENDA_OK;
}

extern "C" int leyenda_server_submit(leyenda_server *S, const void *in_dev, uint64_t n, uint64_t tag) {
    if (!S || (!in_dev && n)) return fail(LEYENDA_EINVAL, "leyenda_server_submit: NULL");
    if (n == 0 || n > S->cfg.max_batch_records)
        return fail(LEYENDA_EINVAL, "leyenda_server_submit: request size must be 1..max_batch_records");
    if (reinterpret_cast<uintptr_t>(in_dev) & 3u) return fail(LEYENDA_EINVAL, "leyenda_server_submit: misaligned");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->reqs.count(tag)) return fail(LEYENDA_EINVAL, "leyenda_server_submit: tag already in use");
    SReq r;
    r.in = in_dev;
    r.n = n;
    r.t_submit = now_s();
    S->reqs[tag] = r;
    S->queue.push_back(tag);
    return LEYENDA_OK;
}

extern "C" int leyenda_server_poll(leyenda_server *S, leyenda_done *out, uint64_t cap, uint64_t *count,
                                   double timeout_s) {
    if (!S || !count || (!out && cap)) return fail(LEYENDA_EINVAL, "leyenda_server_poll: NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->done_q.empty() && timeout_s > 0)
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [S] { return !S->done_q.empty(); });
    uint64_t k = 0;
    while (k < cap && !S->done_q.empty()) {
        const uint64_t tag = S->done_q.front();
        S->done_q.pop_front();
        const SReq &r = S->reqs[tag];
        leyenda_done d;
        d.tag = tag;
        d.out_dev = static_cast<char *>(S->arena_dev) + r.off;
        d.n = r.n;
        d.submit_s = r.t_submit;
        d.start_s = r.t_start;
        d.done_s = r.t_done;
        d.status = r.status;
        out[k++] = d;
    }
    *count = k;
    return LEYENDA_OK;
}

extern "C" int leyenda_server_release(leyenda_server *S, uint64_t tag) {
    if (!S) return fail(LEYENDA_EINVAL, "leyenda_server_release: NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(tag);
    if (it == S->reqs.end() || !it->second.done) return fail(LEYENDA_EINVAL, "leyenda_server_release: not completed");
    S->arena.release(it->second.off, it->second.bytes);
    S->reqs.erase(it);
    return LEYENDA_OK;
}

extern "C" int leyenda_server_destroy(leyenda_server *S) {
    if (!S) return LEYENDA_OK;
    S->stop.store(true);
    if (S->th.joinable()) S->th.join();
    for (Slot &sl : S->slots) {
        if (sl.s) {
            (void)hipStreamSynchronize(sl.s);
            if (S->cfg.batched) batch_forget(sl.s);
            else pool_forget(sl.s);
            (void)hipStreamDestroy(sl.s);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (S->arena_dev) (void)hipFree(S->arena_dev);
    delete S;
    return LEYENDA_OK;
}

extern "C" int leyenda_serve_replay(const leyenda_server_config *cfg, uint64_t count, const void *const *in_dev,
                                    const uint64_t *n, const double *arrival_s, double *latency_s,
                                    double *makespan_s) {
    if (!cfg || (count && (!in_dev || !n || !arrival_s || !latency_s)) || !makespan_s)
        return fail(LEYENDA_EINVAL, "leyenda_serve_replay: NULL");
    for (uint64_t i = 1; i < count; i++)
        if (arrival_s[i] < arrival_s[i - 1]) return fail(LEYENDA_EINVAL, "leyenda_serve_replay: arrivals not sorted");
    leyenda_server *S = nullptr;
    int rc = leyenda_server_create(cfg, &S);
    if (rc) return rc;
    std::vector<leyenda_done> got(256);
    const double t0 = now_s() + 0.005;
    uint64_t next = 0, completed = 0;
    double last_done = t0;
    while (completed < count) {
        const double t = now_s() - t0;
        while (next < count && arrival_s[next] <= t) {
            if ((rc = leyenda_server_submit(S, in_dev[next], n[next], next))) {
                leyenda_server_destroy(S);
                return rc;
            }
            next++;
        }
        double wait = 0.0002;
        if (next < count) wait = std::min(wait, std::max(0.0, arrival_s[next] - (now_s() - t0)));
        uint64_t k = 0;
        if ((rc = leyenda_server_poll(S, got.data(), got.size(), &k, wait))) break;
        for (uint64_t j = 0; j < k; j++) {
            const leyenda_done &d = got[j];
            if (d.status) rc = d.status;
            latency_s[d.tag] = (d.done_s - t0) - arrival_s[d.tag];
            last_done = std::max(last_done, d.done_s);
            (void)leyenda_server_release(S, d.tag);
            completed++;
        }
        if (rc) break;
    }
    *makespan_s = last_done - t0;
    leyenda_server_destroy(S);
    return rc;
}
