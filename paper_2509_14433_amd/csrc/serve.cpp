// Serving loop: continuous batching of interleaved update and query
// requests over one resident context.
//
// Clients submit update requests (copied at submission, validated
// all-or-nothing) and connectivity queries, each getting a ticket in
// submission order.  A worker thread owns the context.  It repeatedly takes
// the longest prefix of pending update requests that fits one device batch
// (and stops at the first query), applies it as one batch, then answers the
// queries that follow it.  Requests submitted while a batch is on the GPU
// wait in the queue and join the next batch, so a query observes exactly
// the updates submitted before it (queries flush pending updates first,
// Sec. 4.3 of arXiv 2509.14433).
//
// Admission is by memory: pending update requests hold host staging memory
// (8 bytes per update); a submission that would exceed the budget blocks
// until the worker frees space, or fails with CUPK_EBUSY in non-blocking
// mode.  Query latency is measured from submission to answer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "cupk.h"
#include "serve.hpp"

#include <exception>

namespace cupk {

namespace {
double now_us()
{
    return std::chrono::duration<double, std::micro>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}
}  // namespace

struct Server::Req {
    uint64_t ticket;
    bool query;
    uint32_t qu, qv;
    bool burst = false;            // a burst of queries (bu, bv; answers go to bout)
    std::vector<uint32_t> bu, bv;
    int32_t *bout = nullptr;
    std::vector<uint64_t> packed;  // update requests: packed updates
    size_t done_upd = 0;           // updates of this request already applied
    double t_submit;
};

Server::Server(cupk_ctx *ctx, const cupk_serve_opts &o, ApplyFn apply, ConnFn conn)
    : ctx_(ctx), opts_(o), apply_(apply), conn_(conn)
{
    if (opts_.max_batch == 0) opts_.max_batch = 1u << 20;
    if (opts_.mem_budget_bytes == 0) opts_.mem_budget_bytes = (size_t)64 << 20;
    th_ = std::thread([this] { loop(); });
}

Server::~Server()
{
    {
        std::lock_guard<std::mutex> g(m_);
        stop_ = true;
    }
    cv_work_.notify_all();
    cv_space_.notify_all();
    if (th_.joinable()) th_.join();
}

int Server::submit_updates(const uint32_t *u, const uint32_t *v, const uint8_t *del, size_t n,
                           uint32_t V, uint64_t *ticket)
{
    for (size_t i = 0; i < n; i++)
        if (u[i] == v[i] || u[i] >= V || v[i] >= V) return CUPK_EINVAL;
    const size_t bytes = n * 8;
    if (bytes > opts_.mem_budget_bytes) return CUPK_EINVAL;  // can never be admitted
    auto r = std::make_unique<Req>();
    r->query = false;
    r->packed.resize(n);
    for (size_t i = 0; i < n; i++)
        r->packed[i] =
            (uint64_t)u[i] | ((uint64_t)v[i] << 32) | ((uint64_t)(del[i] != 0) << 63);
    std::unique_lock<std::mutex> g(m_);
    if (pending_bytes_ + bytes > opts_.mem_budget_bytes) {
        if (opts_.nonblocking) return CUPK_EBUSY;
        stats_.admission_waits++;
        cv_space_.wait(g, [&] { return stop_ || pending_bytes_ + bytes <= opts_.mem_budget_bytes; });
        if (stop_) return CUPK_EBUSY;
    }
    pending_bytes_ += bytes;
    r->ticket = next_ticket_++;
    r->t_submit = now_us();
    *ticket = r->ticket;
    queue_.push_back(std::move(r));
    stats_.update_requests++;
    g.unlock();
    cv_work_.notify_one();
    return CUPK_OK;
}

int Server::submit_query(uint32_t u, uint32_t v, uint32_t V, uint64_t *ticket)
{
    if (u >= V || v >= V) return CUPK_EINVAL;
    auto r = std::make_unique<Req>();
    r->query = true;
    r->qu = u;
    r->qv = v;
    std::unique_lock<std::mutex> g(m_);
    r->ticket = next_ticket_++;
    r->t_submit = now_us();
    *ticket = r->ticket;
    queue_.push_back(std::move(r));
    stats_.queries++;
    g.unlock();
    cv_work_.notify_one();
    return CUPK_OK;
}

int Server::submit_queries(const uint32_t *u, const uint32_t *v, size_t n, int32_t *out,
                           uint32_t V, uint64_t *ticket)
{
    for (size_t i = 0; i < n; i++)
        if (u[i] >= V || v[i] >= V) return CUPK_EINVAL;
    auto r = std::make_unique<Req>();
    r->query = true;
    r->burst = true;
    r->bu.assign(u, u + n);
    r->bv.assign(v, v + n);
    r->bout = out;
    std::unique_lock<std::mutex> g(m_);
    r->ticket = next_ticket_++;
    r->t_submit = now_us();
    *ticket = r->ticket;
    queue_.push_back(std::move(r));
    stats_.queries += n;
    g.unlock();
    cv_work_.notify_one();
    return CUPK_OK;
}

int Server::wait(uint64_t ticket, int32_t *result)
{
    std::unique_lock<std::mutex> g(m_);
    if (ticket >= next_ticket_) return CUPK_EINVAL;
    cv_done_.wait(g, [&] { return results_.count(ticket) != 0; });
    auto it = results_.find(ticket);
    if (result) *result = it->second;
    results_.erase(it);
    return CUPK_OK;
}

void Server::get_stats(cupk_serve_stats_t *out)
{
    std::lock_guard<std::mutex> g(m_);
    *out = stats_;
    std::vector<double> lat = latencies_;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) -> double {
        if (lat.empty()) return 0.0;
        size_t i = (size_t)(p * (lat.size() - 1) + 0.5);
        return lat[std::min(i, lat.size() - 1)];
    };
    out->query_p50_us = pct(0.50);
    out->query_p99_us = pct(0.99);
    out->query_max_us = lat.empty() ? 0.0 : lat.back();
}

void Server::reset_stats()
{
    std::lock_guard<std::mutex> g(m_);
    stats_ = cupk_serve_stats_t{};
    latencies_.clear();
}

void Server::loop()
{
    std::vector<uint64_t> batch;
    for (;;) {
        // gather the next batch: a prefix of update requests, up to max_batch
        // updates, stopping at the first query
        std::vector<Req *> part;  // requests contributing to this batch
        std::vector<std::pair<Req *, size_t>> takes;
        {
            std::unique_lock<std::mutex> g(m_);
            cv_work_.wait(g, [&] { return stop_ || !queue_.empty(); });
            if (queue_.empty() && stop_) return;
            batch.clear();
            for (auto &rp : queue_) {
                Req *r = rp.get();
                if (r->query) break;
                const size_t left = r->packed.size() - r->done_upd;
                const size_t room = opts_.max_batch - batch.size();
                const size_t take = std::min(left, room);
                takes.push_back({r, take});
                if (take == 0) break;
                batch.insert(batch.end(), r->packed.begin() + r->done_upd,
                             r->packed.begin() + r->done_upd + take);
                if (batch.size() >= opts_.max_batch) break;
            }
        }
        int rc = CUPK_OK;
        if (!batch.empty()) {
            // no exception may leave the worker thread
            try {
                rc = apply_(ctx_, batch.data(), batch.size());
            } catch (const std::exception &) {
                rc = CUPK_ENOMEM;
            }
            std::lock_guard<std::mutex> g(m_);
            stats_.batches++;
            stats_.updates += batch.size();
        }
        // retire finished update requests and answer the queries that now
        // head the queue
        {
            std::unique_lock<std::mutex> g(m_);
            size_t freed = 0;
            for (auto &t : takes) {
                t.first->done_upd += t.second;
                freed += t.second * 8;
            }
            while (!queue_.empty()) {
                Req *r = queue_.front().get();
                if (!r->query) {
                    if (r->done_upd < r->packed.size()) break;
                    results_[r->ticket] = rc;
                    queue_.pop_front();
                    continue;
                }
                if (r->burst) {
                    // a burst: every answer, then one completion
                    int c = CUPK_OK;
                    for (size_t i = 0; i < r->bu.size(); i++) {
                        const int a = conn_(ctx_, r->bu[i], r->bv[i]);
                        r->bout[i] = a;
                        if (a < 0) c = a;
                    }
                    results_[r->ticket] = c;
                    const double lat = now_us() - r->t_submit;
                    for (size_t i = 0; i < r->bu.size(); i++) latencies_.push_back(lat);
                } else {
                    const int c = conn_(ctx_, r->qu, r->qv);
                    results_[r->ticket] = c;
                    latencies_.push_back(now_us() - r->t_submit);
                }
                queue_.pop_front();
            }
            pending_bytes_ -= freed;
        }
        cv_space_.notify_all();
        cv_done_.notify_all();
    }
}

}  // namespace cupk
