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

#include "cupk.h"

namespace cupk {

class Server {
  public:
    // apply: one batch of packed updates (host memory) on the context;
    // conn: Connected(u, v) on the context.  Both run on the worker thread.
    using ApplyFn = int (*)(cupk_ctx *, const uint64_t *, size_t);
    using ConnFn = int (*)(cupk_ctx *, uint32_t, uint32_t);

    Server(cupk_ctx *ctx, const cupk_serve_opts &o, ApplyFn apply, ConnFn conn);
    ~Server();

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
    std::deque<std::unique_ptr<Req>> queue_;
    std::unordered_map<uint64_t, int32_t> results_;
    std::vector<double> latencies_;
    cupk_serve_stats_t stats_ = {};
    size_t pending_bytes_ = 0;
    uint64_t next_ticket_ = 0;
    bool stop_ = false;
};

}  // namespace cupk
