// Multi-level hierarchy (Gibb's cutset levels, Sec. 2.2.2 and Alg. 1 of
// arXiv 2509.14433) over the one resident sketch.
//
// Levels 0..C.  Level i < C queries components of its forest F_i with sketch
// column i alone (its own independent sampler); the top level C is the
// context's forest, which answers connectivity, and queries with all C
// columns.  F_0 has no edges (implicit), F_1..F_(C-1) are kept here, and
// F_i is contained in F_(i+1).  The weight of a forest edge is the lowest
// level that holds it.
//
// Per batch: the scatter updates every column; deletes of top-forest edges
// (in stream order) leave every level from the edge's weight up; then
// restore() re-establishes Invariant 3 (a level-i component whose query
// succeeds is a proper subset of its level-(i+1) component) in passes, each
// one GPU launch pair (one-column reduce + query) over every component that
// could violate it, repairs at the lowest violating level as in Alg. 1
// (cycle edge = heaviest edge of the top-forest path, removed from its
// weight up; the sampled edge joins every level above), and finally
// completes the top forest with replacement rounds on the all-column
// sampler.
#pragma once

#include "context.hpp"

namespace cupk {

struct Level {
    std::vector<uint32_t> lbl, par;  // the forest's label / parent words
    Forest F;
};

struct Levels {
    uint32_t top = 0;                       // = C
    std::vector<std::unique_ptr<Level>> lv; // lv[j] for j = 1..top-1 (lv[0] empty)
    DevBuf<uint32_t> d_col, d_idx, d_items;
    HostBuf<uint32_t> h_col, h_idx, h_items;
    DevBuf<uint64_t> d_agg;
    std::vector<uint32_t> mark;             // scratch of path searches
    uint32_t epoch = 0;
};

// Set up the inner levels (opts.levels).
int levels_init(cupk_ctx *ctx);
void levels_release(cupk_ctx *ctx);
// Delete walk: a delete of a top-forest edge leaves every level from its
// weight up.  Returns true when it was a forest edge.
bool levels_delete(cupk_ctx *ctx, uint32_t a, uint32_t b);
// Batch end: restoration passes, then top completion.
int levels_restore(cupk_ctx *ctx);
// Edges of the forest at `level` (1..C) as (u < v) pairs.
void levels_edges(cupk_ctx *ctx, uint32_t level, std::vector<uint32_t> &eu,
                  std::vector<uint32_t> &ev);

}  // namespace cupk
