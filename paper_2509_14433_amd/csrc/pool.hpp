// A small fork-join thread pool for the host forest work of a batch
// (relabelling merged trees, listing the members of many trees): run(n, fn)
// calls fn(i, worker) for every i in [0, n) on the calling thread and the
// pool's workers, and returns when all calls have returned.  `worker` is in
// [0, size()): per-worker scratch can be indexed by it.  Calls of run() must
// not overlap (one batch's host work at a time, as the library's context
// lock guarantees).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace cupk {

class Pool {
  public:
    explicit Pool(unsigned workers = 0)
    {
        unsigned n = workers;
        if (n == 0) {
            const unsigned hw = std::thread::hardware_concurrency();
            n = hw > 2 ? hw / 2 : 1;
            if (n > 8) n = 8;
        }
        size_ = n;
        for (unsigned w = 1; w < n; w++) th_.emplace_back([this, w] { loop(w); });
    }
    ~Pool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    Pool(const Pool &) = delete;
    Pool &operator=(const Pool &) = delete;

    unsigned size() const { return size_; }

    void run(size_t n, const std::function<void(size_t, unsigned)> &fn)
    {
        if (n == 0) return;
        if (n == 1 || size_ == 1) {
            for (size_t i = 0; i < n; i++) fn(i, 0);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(m_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            busy_ = (unsigned)th_.size();
            gen_++;
        }
        cv_.notify_all();
        work(0);
        std::unique_lock<std::mutex> lk(m_);
        done_.wait(lk, [this] { return busy_ == 0; });
        fn_ = nullptr;
    }

  private:
    void work(unsigned w)
    {
        for (;;) {
            const size_t i = next_.fetch_add(1);
            if (i >= n_) break;
            (*fn_)(i, w);
        }
    }
    void loop(unsigned w)
    {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work(w);
            {
                std::lock_guard<std::mutex> lk(m_);
                if (--busy_ == 0) done_.notify_one();
            }
        }
    }

    unsigned size_ = 1;
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(size_t, unsigned)> *fn_ = nullptr;
    size_t n_ = 0;
    std::atomic<size_t> next_{0};
    unsigned busy_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

}  // namespace cupk
