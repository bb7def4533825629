// Host-side parallel copy used by the external sorts' pageable outputs.
// Plain C++ (no HIP), so it also builds and is tested on its own.
#pragma once
#include <sched.h>

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

namespace ley {

// A fixed team of host threads that copies one byte range in parallel (the
// pageable destination of the external outputs); the threads sleep between
// copies.  Up to 16 threads, at most one per CPU this process may run on.
class CopyTeam {
  public:
    CopyTeam() {
        cpu_set_t cs;
        unsigned cpus = std::thread::hardware_concurrency();
        if (sched_getaffinity(0, sizeof(cs), &cs) == 0) cpus = (unsigned)CPU_COUNT(&cs);
        n_ = std::max(1u, std::min(16u, cpus));
        for (unsigned t = 1; t < n_; t++) th_.emplace_back([this, t] { work(t); });
    }
    ~CopyTeam() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &x : th_) x.join();
    }
    // Copies `bytes` from src to dst; returns when every thread is done.
    void copy(uint8_t *dst, const uint8_t *src, size_t bytes) {
        if (bytes < (8u << 20) || n_ == 1) { std::memcpy(dst, src, bytes); return; }
        {
            std::lock_guard<std::mutex> lk(mu_);
            dst_ = dst; src_ = src; bytes_ = bytes; left_ = n_ - 1;
            gen_++;
        }
        cv_.notify_all();
        part(0);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return left_ == 0; });
    }

  private:
    void part(unsigned t) {
        const size_t per = (bytes_ + n_ - 1) / n_ / 64 * 64 + 64;
        const size_t a = std::min(bytes_, t * per), b = std::min(bytes_, a + per);
        if (a < b) std::memcpy(dst_ + a, src_ + a, b - a);
    }
    void work(unsigned t) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            part(t);
            std::lock_guard<std::mutex> lk(mu_);
            if (--left_ == 0) done_cv_.notify_one();
        }
    }
    unsigned n_ = 1;
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    uint64_t gen_ = 0;
    bool stop_ = false;
    unsigned left_ = 0;
    uint8_t *dst_ = nullptr;
    const uint8_t *src_ = nullptr;
    size_t bytes_ = 0;
};

}  // namespace ley
