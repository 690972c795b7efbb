// Contracted walk of a run of flagged updates.
//
// Walking a batch's flagged updates one by one on the forest (an insert
// links two different trees, a delete of a forest edge removes it, pieces
// split before the next insert) costs a relabelling of the smaller tree per
// link and a piece search per split.  When the same few edges are linked
// and cut again and again inside one run (bridges between large trees
// toggled many times), most of that work is undone within the run.
//
// The contracted walk gives exactly the same result with work proportional
// to the net change:
//   1. T0 = the forest at the start of the run.  The T0 edges the run
//      deletes are D0; the pieces are the components of T0 - D0.  Every
//      edge of T0 - D0 stays in the forest throughout the run, so each
//      piece stays connected, and two vertices are connected at any moment
//      exactly when their pieces are connected by the forest edges that
//      join different pieces (D0 edges not yet deleted, and edges the run
//      linked).  The piece of a vertex is named by its top vertex: the
//      first vertex at or above it whose parent edge is in D0, or the root.
//      Only the run's endpoints need a piece, found by walking parent
//      pointers up, each vertex once (a walk that would exceed a budget
//      proportional to the run gives up and the caller walks the run one
//      update at a time instead; no edge has been changed then).
//   2. The run is replayed on a small forest over the pieces, starting
//      with the D0 edges: links and removals happen there exactly when they
//      would happen on the whole forest, so the counts of links and cuts
//      are the same.
//   3. The net change is applied to the whole forest: D0 edges that ended
//      removed are removed, the pieces split once, and the edges the replay
//      added that were not in T0 are linked (Forest::link_many: each merged
//      tree relabelled once).
//   4. Dirty marks: one by one, a tree ends dirty exactly when it holds an
//      endpoint of an edge removed during the run (each removal makes both
//      sides dirty, marks follow links, and every piece of a split holds
//      such an endpoint) or a vertex of a tree already dirty.  Step 3 sets
//      a subset of those marks; the endpoints of every edge the replay
//      removed mark the rest.
#pragma once

#include <stdint.h>

#include <chrono>
#include <unordered_set>
#include <vector>

#include "forest.hpp"

namespace cupk {

class Contraction {
  public:
    // Walk the flagged updates upd[k0, k1) (packed: u in bits 0..31, v in
    // 32..62, delete flag in bit 63) into F.  Pending splits are done first.
    // Returns false, with F's edges untouched, when the piece search
    // exceeds its budget.  *links and *cuts get the links and forest-edge
    // removals of the one-by-one walk; *changed tells whether the forest's
    // edges changed.
    bool run(Forest &F, const uint64_t *upd, uint32_t k0, uint32_t k1, uint64_t *links,
             uint64_t *cuts, bool *changed)
    {
        const uint32_t V = F.V();
        if (cut_.size() != V) {
            cut_.assign(V, 0);
            seen_.assign(V, 0);
            top_.assign(V, 0);
            pid_.assign(V, 0);
            epoch_ = 0;
        }
        if (++epoch_ == 0) {
            std::fill(cut_.begin(), cut_.end(), 0);
            std::fill(seen_.begin(), seen_.end(), 0);
            std::fill(pstamp_.begin(), pstamp_.end(), 0);
            epoch_ = 1;
        }
        const auto t0 = std::chrono::steady_clock::now();
        // labels exact, so that T0 is the current forest
        F.split_pending();
        // D0: T0 edges the run deletes (child endpoint marked)
        d0_.clear();
        for (uint32_t k = k0; k < k1; k++) {
            const uint64_t p = upd[k];
            if ((p >> 63) == 0) continue;
            uint32_t a, b;
            ends(p, a, b);
            if (!F.is_edge(a, b)) continue;
            const uint32_t child = F.parent(a) == b ? a : b;
            if (cut_[child] == epoch_) continue;  // deleted again after a re-insert
            cut_[child] = epoch_;
            d0_.push_back(key(a, b));
        }
        // pieces of the run's endpoints
        size_t budget = budget_per_update_ * (k1 - k0) + budget_base_;
        uint32_t P = 0;
        for (uint32_t k = k0; k < k1; k++) {
            uint32_t a, b;
            ends(upd[k], a, b);
            for (uint32_t x : {a, b}) {
                if (seen_[x] == epoch_) continue;
                const uint32_t t = find_top(F, x, budget);
                if (t == kNone) return false;
                if (pid_[t] >= P || piece_top_[pid_[t]] != t) {
                    pid_[t] = P++;
                    if (piece_top_.size() < P) piece_top_.resize(P);
                    piece_top_[P - 1] = t;
                }
            }
        }
        const auto t1 = std::chrono::steady_clock::now();
        // replay on the piece forest
        plbl_.resize(P);
        ppar_.resize(P);
        PF_.init(P, plbl_.data(), ppar_.data());
        live_.clear();
        live_.reserve(2 * (d0_.size() + (k1 - k0)));
        for (uint64_t e : d0_) {
            const uint32_t a = (uint32_t)e, b = (uint32_t)(e >> 32);
            PF_.link(piece(a), piece(b));
            live_.insert(e);
        }
        added_.clear();
        removed_.clear();
        uint64_t nl = 0, nc = 0;
        for (uint32_t k = k0; k < k1; k++) {
            const uint64_t p = upd[k];
            uint32_t a, b;
            ends(p, a, b);
            const uint32_t pa = piece(a), pb = piece(b);
            if ((p >> 63) == 0) {
                if (PF_.has_pending()) PF_.split_pending();
                if (pa != pb && !PF_.same_tree(pa, pb)) {
                    PF_.link(pa, pb);
                    live_.insert(key(a, b));
                    added_.push_back(key(a, b));
                    nl++;
                }
            } else if (live_.erase(key(a, b))) {
                PF_.remove_edge(pa, pb);
                removed_.push_back(a);
                removed_.push_back(b);
                nc++;
            }
        }
        const auto t2 = std::chrono::steady_clock::now();
        // net change on the whole forest: the removals, then every piece of
        // the broken trees (and every tree a net edge joins) settled into its
        // final tree at once, the final trees being the piece forest's
        bool ch = false;
        for (uint64_t e : d0_)
            if (!live_.count(e)) {
                F.remove_edge((uint32_t)e, (uint32_t)(e >> 32));
                ch = true;
            }
        const auto t3 = std::chrono::steady_clock::now();
        net_.clear();
        for (uint64_t e : added_) {
            if (!live_.count(e)) continue;
            const uint32_t a = (uint32_t)e, b = (uint32_t)(e >> 32);
            if (F.is_edge(a, b)) continue;  // a D0 edge deleted and linked again
            net_.push_back({a, b});
            live_.erase(e);  // linked once, even if added more than once
        }
        if (F.has_pending() || !net_.empty()) {
            if (PF_.has_pending()) PF_.split_pending();
            if (pstamp_.size() != V) pstamp_.assign(V, 0);
            pieces_.clear();
            uint32_t extra = P;  // group ids past the piece forest's labels
            auto add = [&](uint32_t t) {
                if (pstamp_[t] == epoch_) return;
                pstamp_[t] = epoch_;
                uint32_t g;
                size_t big = (size_t)-1;
                if (seen_[t] == epoch_ || find_top(F, t, big) != kNone) {
                    const uint32_t q = pid_[top_[t]];
                    g = (q < P && piece_top_[q] == top_[t]) ? PF_.label(q) : extra++;
                } else {
                    g = extra++;
                }
                pieces_.push_back({t, g});
            };
            for (const auto &pr : F.pending()) {
                add(pr.second);
                add(F.tree_root(pr.first));
            }
            for (const auto &e : net_) {
                add(F.tree_root(F.label(e.first)));
                add(F.tree_root(F.label(e.second)));
            }
            F.settle_regroup(pieces_, net_);
            ch = true;
        }
        for (uint32_t x : removed_) F.set_dirty(F.label(x));
        const auto t4 = std::chrono::steady_clock::now();
        auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        last_ms[0] = ms(t0, t1);  // pending splits, D0, pieces
        last_ms[1] = ms(t1, t2);  // replay on the piece forest
        last_ms[2] = ms(t2, t3);  // removals
        last_ms[3] = ms(t3, t4);  // settling the pieces into their final trees
        last_pieces = P;
        *links += nl;
        *cuts += nc;
        *changed = ch;
        return true;
    }

    // Host time of the last run's phases (ms) and its number of pieces.
    double last_ms[4] = {0, 0, 0, 0};
    uint32_t last_pieces = 0;

    // Parent steps the piece search may take: per update of the run, plus
    // a constant.
    void set_budget(size_t per_update, size_t base)
    {
        budget_per_update_ = per_update;
        budget_base_ = base;
    }

  private:
    static uint64_t key(uint32_t a, uint32_t b) { return (uint64_t)b << 32 | a; }
    static void ends(uint64_t p, uint32_t &a, uint32_t &b)
    {
        a = (uint32_t)p;
        b = (uint32_t)(p >> 32) & 0x7fffffffu;
        if (a > b) std::swap(a, b);
    }
    uint32_t piece(uint32_t x) const { return pid_[top_[x]]; }
    // Top vertex of x's piece; kNone when the budget runs out.  Every
    // vertex on the way up is remembered for this run.
    uint32_t find_top(const Forest &F, uint32_t x, size_t &budget)
    {
        path_.clear();
        uint32_t y = x, t;
        for (;;) {
            if (seen_[y] == epoch_) {
                t = top_[y];
                break;
            }
            path_.push_back(y);
            const uint32_t up = F.parent(y);
            if (up == kNone || cut_[y] == epoch_) {
                t = y;
                break;
            }
            if (budget == 0) return kNone;
            budget--;
            y = up;
        }
        for (uint32_t w : path_) {
            seen_[w] = epoch_;
            top_[w] = t;
        }
        return t;
    }

    std::vector<uint32_t> cut_, seen_, top_, pid_, pstamp_;  // by vertex; stamps are epochs
    std::vector<std::pair<uint32_t, uint32_t>> pieces_;  // (top, final group) to settle
    uint32_t epoch_ = 0;
    size_t budget_per_update_ = 64, budget_base_ = 4096;
    std::vector<uint32_t> piece_top_, path_;
    std::vector<uint64_t> d0_, added_;
    std::vector<std::pair<uint32_t, uint32_t>> net_;
    std::vector<uint8_t> net_linked_;
    std::vector<uint32_t> removed_;
    std::unordered_set<uint64_t> live_;  // edges between pieces, by original endpoints
    std::vector<uint32_t> plbl_, ppar_;
    Forest PF_;
};

}  // namespace cupk
