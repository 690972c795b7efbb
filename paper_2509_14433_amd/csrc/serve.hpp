// Serving loop (see serve.cpp).
#pragma once

#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <hip/hip_runtime.h>

#include "cupk.h"

namespace cupk {

class Server {
  public:
    // apply: one batch of packed updates already in device memory, whose
    // upload is complete once `ready` has been reached (the context's
    // stream must wait for it); conn: Connected(u, v) on the context.  Both
    // run on the worker thread.
    using ApplyFn = int (*)(cupk_ctx *, const uint64_t *, size_t, hipEvent_t ready);
    using ConnFn = int (*)(cupk_ctx *, uint32_t, uint32_t);

    Server(cupk_ctx *ctx, const cupk_serve_opts &o, ApplyFn apply, ConnFn conn);
    ~Server();
    // Allocate the request rings and start the worker; CUPK_OK or an error.
    int start();

    int submit_updates(const uint32_t *u, const uint32_t *v, const uint8_t *del, size_t n,
                       uint32_t V, uint64_t *ticket);
    int submit_query(uint32_t u, uint32_t v, uint32_t V, uint64_t *ticket);
    int submit_queries(const uint32_t *u, const uint32_t *v, size_t n, int32_t *out, uint32_t V,
                       uint64_t *ticket);
    int wait(uint64_t ticket, int32_t *result);
    void get_stats(cupk_serve_stats_t *out);
    void reset_stats();

  private:
    struct Req;
    void loop();

    cupk_ctx *ctx_;
    cupk_serve_opts opts_;
    ApplyFn apply_;
    ConnFn conn_;
    std::thread th_;
    std::mutex m_;
    std::condition_variable cv_work_, cv_done_, cv_space_;
    bool reserve(size_t n, size_t *slot);  // ring words for a request (lock held)
    std::deque<std::unique_ptr<Req>> queue_;
    // Admission by device memory: every admitted update request holds a
    // contiguous slot of a device ring (and of its pinned host staging twin),
    // uploaded on a copy stream at submission; slots are freed in order.
    uint64_t *d_ring_ = nullptr, *h_ring_ = nullptr;
    size_t cap_ = 0;          // ring capacity, words
    size_t head_ = 0;         // next free word
    std::deque<std::pair<size_t, size_t>> slots_;  // in-use (start, words), oldest first
    hipStream_t copy_s_ = nullptr;
    hipEvent_t copied_ = nullptr;
    std::unordered_map<uint64_t, int32_t> results_;
    std::vector<double> latencies_;
    cupk_serve_stats_t stats_ = {};
    size_t pending_bytes_ = 0;  // device ring bytes held by pending requests
    uint64_t next_ticket_ = 0;
    bool stop_ = false;
};

}  // namespace cupk
