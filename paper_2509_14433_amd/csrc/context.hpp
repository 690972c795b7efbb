// Context of the C ABI and helpers shared by the library's translation
// units (api.cpp: batches, rounds, ABI; levels.cpp: the multi-level
// hierarchy).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "cupk.h"
#include "contract.hpp"
#include "forest.hpp"
#include "kernels.hpp"
#include "serve.hpp"

namespace cupk {

constexpr uint32_t kRedChunk = 16;          // members per reduction work item
constexpr size_t kMaxBatchPerLaunch = 1u << 28;
constexpr int kTimerRing = 64;

inline double now_ms()
{
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
};
template <class T>
struct HostBuf {
    T *p = nullptr;
    size_t cap = 0;
};

struct Levels;  // multi-level hierarchy state (levels.cpp)

}  // namespace cupk

struct cupk_ctx {
    uint32_t V = 0, C = 0, D = 0;
    uint64_t S = 0;
    uint64_t seeds[64] = {};
    uint32_t W = 0;  // words per vertex slab = 2*C*D
    cupk_opts opts = {};
    hipStream_t s = nullptr, cs = nullptr;
    bool own_stream = false;
    uint32_t hdr_seq = 0;          // headers published by the device so far (expected)
    uint32_t *hdr_word = nullptr;  // where the current pass publishes its sequence number
    bool query_often = false;      // the pass's batch was uploaded from host memory
    // timed pass: t0 after classification, tb after binning, tc before the
    // scatter (split passes only: reflagging and the wait for the previous
    // batch's rounds come between), t1 after the scatter
    struct TimerSlot {
        hipEvent_t t0, tb, tc, t1;
        bool busy, split;
    };
    TimerSlot timers[cupk::kTimerRing] = {};
    int timer_head = 0;

    uint64_t *d_sk = nullptr;
    bool own_sk = false;
    uint64_t *d_seeds = nullptr;
    uint32_t *d_lbl = nullptr, *d_par = nullptr;
    uint64_t *d_lp = nullptr;  // label | parent << 32 per vertex
    uint32_t *d_blk = nullptr; // per 64 vertex ids: their common label, or kBlkMixed
    uint32_t *h_lbl = nullptr, *h_par = nullptr;
    bool forest_dev_stale = false;
    // page-wise uploads of the forest: the pages written since the last
    // upload, their staging block (pinned, then device) and whether its
    // last copy (ev_stage) may still be in flight
    std::vector<uint32_t> up_pages;
    cupk::HostBuf<uint32_t> h_stage;
    cupk::DevBuf<uint32_t> d_stage;
    hipEvent_t ev_stage = nullptr;
    bool stage_busy = false;

    // batch buffers
    cupk::DevBuf<uint64_t> d_upd;
    cupk::HostBuf<uint64_t> h_upd;
    uint32_t *d_hdr = nullptr, *h_hdr = nullptr;
    cupk::DevBuf<uint32_t> d_fcnt, d_foff;
    cupk::DevBuf<uint32_t> d_fdel;  // flagged deletes per classify block  // flagged updates: per-block counts and offsets,
    cupk::DevBuf<uint64_t> d_fupd, d_oupd;  // per-block regions, the compacted ordered list
    cupk::HostBuf<uint64_t> h_fupd;  // coherent: short flag lists are written there by the device
    cupk::DevBuf<uint32_t> d_fpos, d_opos;  // positions of flagged updates (exact mode)
    cupk::HostBuf<uint32_t> h_fpos;

    // staged scatter
    uint32_t tile_shift = 5, rows = 8, chunk = 4096, ntiles = 0, tile_grid = 0;
    uint32_t layout = CUPK_LAYOUT_RECORD;  // staged-scatter lane layout
    cupk::DevBuf<uint32_t> d_tcnt, d_toff, d_tcur, d_items;
    cupk::DevBuf<uint32_t> d_tsum;  // chunk totals of the multi-block tile scan
    cupk::DevBuf<uint32_t> d_trel;  // per (classify block, tile): start inside the tile's bin
    cupk::DevBuf<uint32_t> d_tgoff; // per (count copy, tile): where the copy's records start
    cupk::DevBuf<uint64_t> d_bins;
    // two-level binning (more than kFillStageTiles tiles): coarse bins of
    // 2^fshift tiles (fshift 0: one level), their counts, count-copy
    // starts, offsets and cursors, the coarse-binned records, and a sink
    // for the coarse scan's (unused) work items
    uint32_t fshift = 0, ncoarse = 0;
    cupk::DevBuf<uint32_t> d_ccnt, d_cgoff, d_coff, d_ccur, d_csink;
    cupk::DevBuf<uint64_t> d_bins1;
    uint32_t *d_nitems = nullptr;
    unsigned long long *d_touched = nullptr;  // buckets changed by timed staged launches

    // reductions / samples
    cupk::DevBuf<uint32_t> d_ridx;   // members, then the work items, of a reduction
    cupk::HostBuf<uint32_t> h_ridx;
    cupk::DevBuf<uint64_t> d_sig[2];
    cupk::DevBuf<int32_t> d_res;
    cupk::HostBuf<int32_t> h_res;
    cupk::DevBuf<uint64_t> d_tmp;
    uint64_t *d_misc = nullptr, *h_misc = nullptr;
    cupk::SmallResult *d_small = nullptr, *h_small = nullptr;  // small-batch pass results
    bool small_pass = false;   // the last pass took the small-batch path
    // cupk_apply_updates_device leaves the host part of its batch (flag
    // walk, replacement rounds) pending until the next call that needs it
    bool pending = false;
    uint32_t pending_n = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;  // ordering with a caller's stream
    // Overlapped passes: the pending batch's replacement rounds reduce on
    // cs (after ev_scat, its scatter) while s classifies and bins the next
    // batch (after ev_up, the forest's upload on cs); rstream is the stream
    // the rounds use (s otherwise)
    hipStream_t rstream = nullptr;
    hipEvent_t ev_scat = nullptr, ev_up = nullptr;
    hipEvent_t ev_cls = nullptr;  // after the split pass's classification
    TimerSlot *split_ts = nullptr;  // timer of the split pass in flight
    bool scat_marked = false;       // ev_scat follows the pending batch's scatter
    bool flags_packed = false;      // the last pass packed its flag list on the device
    // device address of the allocation-free entry point's scratch array on
    // this context's device (taken at init)
    uint64_t *noalloc_scratch = nullptr;
    cupk::BatchDesc *d_desc = nullptr, *h_desc = nullptr;
    // The batch of the pass being enqueued, passed to the kernels by value;
    // while graphs are captured they read d_desc instead.
    cupk::BatchDesc cur_desc = {};
    bool capturing = false;

    // captured step (use_graph): classify + header copy, bin, tile
    hipStream_t gs = nullptr;  // capture stream
    hipGraphExec_t gx_cls = nullptr, gx_bin = nullptr, gx_tile = nullptr, gx_all = nullptr;
    uint32_t graph_cap = 0;    // batch capacity the graphs were captured for
    size_t batch_cap = 0;      // updates per batch every batch buffer holds
    uint32_t tuned_batch = 0;  // the autotuner's batch target (0: not tuned)


    int device = 0;
    bool trace = false;  // CUPK_TRACE=1: per-batch host timings on stderr
    std::unique_ptr<cupk::Server> server;
    std::vector<int32_t> round_gmap;  // label -> round group, -1 elsewhere
    // first round over pieces (stamped per use)
    std::vector<uint32_t> piece_id, piece_stamp, piece_label_stamp, piece_of_label, piece_mem;
    uint32_t piece_epoch = 0;
    std::unique_ptr<cupk::Levels> levels;  // multi-level hierarchy (opts.levels)
    cupk::Forest forest;
    std::unique_ptr<cupk::Pool> pool;  // host worker threads (large V only)
    cupk::Contraction contract;  // contracted walks of flagged runs
    std::vector<uint8_t> cand_linked;  // which round candidates linked
    // a carried set of the last round whose sketch was not reduced (the old
    // root's piece of the one broken tree; kNone: none)
    uint32_t virtual_set = 0xffffffffu;
    cupk_counters_t ctr = {};
    std::string err;

    int fail(hipError_t e, const char *what, int line)
    {
        char buf[256];
        snprintf(buf, sizeof buf, "%s failed at api.cpp:%d: %s", what, line, hipGetErrorString(e));
        err = buf;
        return e == hipErrorOutOfMemory ? CUPK_ENOMEM : CUPK_EDEVICE;
    }
    int invalid(const char *why)
    {
        err = why;
        return CUPK_EINVAL;
    }
};

#define HIPCHK(x)                                                   \
    do {                                                            \
        hipError_t e_ = (x);                                        \
        if (e_ != hipSuccess) return ctx->fail(e_, #x, __LINE__);   \
    } while (0)

// No C++ exception crosses the C ABI: a failed host allocation inside an
// entry point becomes CUPK_ENOMEM with a message.
template <class F>
inline int guarded(cupk_ctx *ctx, F &&f)
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        ctx->err = "host memory allocation failed";
        return CUPK_ENOMEM;
    } catch (const std::length_error &) {
        ctx->err = "host allocation too large";
        return CUPK_ENOMEM;
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return CUPK_EDEVICE;
    }
}

namespace cupk {

template <class T>
inline hipError_t grow(DevBuf<T> &b, size_t need)
{
    if (need <= b.cap) return hipSuccess;
    size_t cap = std::max(need, 2 * b.cap);
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc((void **)&b.p, cap * sizeof(T));
    if (e != hipSuccess) return e;
    b.cap = cap;
    return hipSuccess;
}

template <class T>
inline hipError_t grow(HostBuf<T> &b, size_t need, unsigned flags = hipHostMallocDefault)
{
    if (need <= b.cap) return hipSuccess;
    size_t cap = std::max(need, 2 * b.cap);
    if (b.p) {
        hipError_t e = hipHostFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipHostMalloc((void **)&b.p, cap * sizeof(T), flags);
    if (e != hipSuccess) return e;
    b.cap = cap;
    return hipSuccess;
}

template <class T>
inline void release(DevBuf<T> &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}
template <class T>
inline void release(HostBuf<T> &b)
{
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
}

// Shared by the translation units (api.cpp).
DevSketch dev_sketch(cupk_ctx *ctx);
int upload_forest(cupk_ctx *ctx);
int reduce_and_sample(cupk_ctx *ctx, int slot, const std::vector<uint32_t> &vmem,
                      const std::vector<uint32_t> &voff, const std::vector<uint32_t> &fmem,
                      const std::vector<uint32_t> &foff);
int run_rounds(cupk_ctx *ctx);
int flush_pending(cupk_ctx *ctx);

}  // namespace cupk
