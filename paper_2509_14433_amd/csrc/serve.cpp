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
// Admission is by device memory: an admitted update request takes a
// contiguous slot of a device ring of mem_budget_bytes (8 bytes per update),
// packed into the slot's pinned host twin and uploaded on a copy stream at
// once, so that its upload overlaps the batch the worker has on the GPU.
// A submission that does not fit blocks until the worker retires requests
// (slots are freed in submission order), or fails with CUPK_EBUSY in
// non-blocking mode.  The worker applies a batch straight from its device
// slots after the context's stream has waited for their uploads.  Query
// latency is measured from submission to answer.
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
    size_t slot = 0, n = 0;        // update requests: device ring slot, updates
    size_t done_upd = 0;           // updates of this request already applied
    double t_submit;
};

Server::Server(cupk_ctx *ctx, const cupk_serve_opts &o, ApplyFn apply, ConnFn conn)
    : ctx_(ctx), opts_(o), apply_(apply), conn_(conn)
{
    if (opts_.max_batch == 0) opts_.max_batch = 1u << 20;
    if (opts_.mem_budget_bytes == 0) opts_.mem_budget_bytes = (size_t)64 << 20;
}

int Server::start()
{
    cap_ = opts_.mem_budget_bytes / 8;
    if (cap_ == 0) return CUPK_EINVAL;
    if (hipStreamCreateWithFlags(&copy_s_, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&copied_, hipEventDisableTiming) != hipSuccess)
        return CUPK_EDEVICE;
    if (hipMalloc((void **)&d_ring_, cap_ * 8) != hipSuccess) return CUPK_ENOMEM;
    if (hipHostMalloc((void **)&h_ring_, cap_ * 8, hipHostMallocDefault) != hipSuccess)
        return CUPK_ENOMEM;
    th_ = std::thread([this] { loop(); });
    return CUPK_OK;
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
    if (copy_s_) (void)hipStreamSynchronize(copy_s_);
    if (d_ring_) (void)hipFree(d_ring_);
    if (h_ring_) (void)hipHostFree(h_ring_);
    if (copied_) (void)hipEventDestroy(copied_);
    if (copy_s_) (void)hipStreamDestroy(copy_s_);
}

// A contiguous slot of n words after the newest one, wrapping to the start
// of the ring when the end is too short; false when it does not fit yet.
// In use: slots_ from its oldest (tail) to the newest, which ends at head_.
bool Server::reserve(size_t n, size_t *slot)
{
    if (slots_.empty()) {
        head_ = 0;
        if (n > cap_) return false;
        *slot = 0;
        return true;
    }
    const size_t tail = slots_.front().first;
    if (head_ > tail) {  // free: [head_, cap_) and [0, tail)
        if (cap_ - head_ >= n) {
            *slot = head_;
            return true;
        }
        if (tail >= n) {
            *slot = 0;
            return true;
        }
        return false;
    }
    if (tail - head_ >= n) {  // wrapped: free [head_, tail)
        *slot = head_;
        return true;
    }
    return false;
}

int Server::submit_updates(const uint32_t *u, const uint32_t *v, const uint8_t *del, size_t n,
                           uint32_t V, uint64_t *ticket)
{
    for (size_t i = 0; i < n; i++)
        if (u[i] == v[i] || u[i] >= V || v[i] >= V) return CUPK_EINVAL;
    if (n > cap_) return CUPK_EINVAL;  // can never be admitted
    auto r = std::make_unique<Req>();
    r->query = false;
    r->n = n;
    std::unique_lock<std::mutex> g(m_);
    size_t slot = 0;
    if (n && !reserve(n, &slot)) {
        if (opts_.nonblocking) return CUPK_EBUSY;
        stats_.admission_waits++;
        cv_space_.wait(g, [&] { return stop_ || reserve(n, &slot); });
        if (stop_) return CUPK_EBUSY;
    }
    // pack into the slot's pinned twin and upload it now (its previous
    // contents were uploaded and applied before the slot was freed)
    if (n) {
        uint64_t *h = h_ring_ + slot;
        for (size_t i = 0; i < n; i++)
            h[i] = (uint64_t)u[i] | ((uint64_t)v[i] << 32) | ((uint64_t)(del[i] != 0) << 63);
        if (hipMemcpyAsync(d_ring_ + slot, h, n * 8, hipMemcpyHostToDevice, copy_s_) !=
            hipSuccess)
            return CUPK_EDEVICE;
        slots_.push_back({slot, n});
        head_ = slot + n;
        pending_bytes_ += n * 8;
    }
    r->slot = slot;
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
    for (;;) {
        // gather the next batch: a prefix of update requests whose device
        // slots are contiguous, up to max_batch updates, stopping at the
        // first query
        std::vector<std::pair<Req *, size_t>> takes;
        size_t start = 0, nb = 0;
        {
            std::unique_lock<std::mutex> g(m_);
            cv_work_.wait(g, [&] { return stop_ || !queue_.empty(); });
            if (queue_.empty() && stop_) return;
            for (auto &rp : queue_) {
                Req *r = rp.get();
                if (r->query) break;
                if (r->n == 0) continue;  // nothing to apply; retired below
                const size_t from = r->slot + r->done_upd;
                if (nb && from != start + nb) break;  // the ring wrapped here
                const size_t left = r->n - r->done_upd;
                const size_t take = std::min(left, (size_t)opts_.max_batch - nb);
                if (take == 0) break;
                if (!nb) start = from;
                takes.push_back({r, take});
                nb += take;
                if (take < left || nb >= opts_.max_batch) break;
            }
            // every gathered request's upload was queued before this event
            if (nb && hipEventRecord(copied_, copy_s_) != hipSuccess) nb = 0, takes.clear();
        }
        int rc = CUPK_OK;
        if (nb) {
            // no exception may leave the worker thread
            try {
                rc = apply_(ctx_, d_ring_ + start, nb, copied_);
            } catch (const std::exception &) {
                rc = CUPK_ENOMEM;
            }
            std::lock_guard<std::mutex> g(m_);
            stats_.batches++;
            stats_.updates += nb;
        }
        // retire finished update requests (freeing their slots, oldest
        // first) and answer the queries that now head the queue
        {
            std::unique_lock<std::mutex> g(m_);
            for (auto &t : takes) t.first->done_upd += t.second;
            while (!queue_.empty()) {
                Req *r = queue_.front().get();
                if (!r->query) {
                    if (r->done_upd < r->n) break;
                    results_[r->ticket] = rc;
                    if (r->n) {
                        pending_bytes_ -= r->n * 8;
                        slots_.pop_front();
                    }
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
        }
        cv_space_.notify_all();
        cv_done_.notify_all();
    }
}

}  // namespace cupk
