// Host spanning forest with exact component labels.
//
// The paper answers connectivity queries from a sketchless dynamic tree on
// the top level (Sec. 4.1) and links / cuts forest edges as updates demand
// (cutset Link / Cut, Sec. 2.2.1).  Here the forest is a rooted forest:
// parent pointers, doubly linked child lists (an edge is removed in O(1)),
// and one label per vertex naming its tree:
//   - link(a, b): the smaller tree is relabelled; the endpoint whose path
//     to its root is shorter is made its tree's root (parent pointers
//     reversed along that path) and hung below the other endpoint (work
//     proportional to the smaller tree plus the shorter path);
//   - cut(a, b): the edge is removed and the two sides are searched
//     top-down (from the old root and from the child endpoint), interleaved
//     edge by edge, so the work is proportional to the smaller side (even
//     next to a high-degree vertex); the smaller side gets a fresh label.
//     A run of cuts can remove all its edges first and split each tree once
//     into all its pieces (remove_edge / split_pending).
// Labels come from a free list in [0, V), so label arrays are V words and
// the device can classify updates against them (lbl[u] != lbl[v] means u
// and v are in different trees; par[] identifies forest edges).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "pool.hpp"

namespace cupk {

constexpr uint32_t kNone = 0xffffffffu;

class Forest {
  public:
    // lbl and par are caller-owned arrays of V words (pinned host memory in
    // the library, so they can be copied to the device asynchronously).
    void init(uint32_t V, uint32_t *lbl, uint32_t *par)
    {
        V_ = V;
        lbl_ = lbl;
        par_ = par;
        first_kid_.assign(V, kNone);
        next_sib_.assign(V, kNone);
        prev_sib_.assign(V, kNone);
        size_.assign(V, 1);
        root_.resize(V);
        dirty_.assign(V, 0);
        free_.clear();
        live_.resize(V);
        live_pos_.resize(V);
        for (uint32_t w = 0; w < V; w++) {
            lbl_[w] = w;
            par_[w] = kNone;
            root_[w] = w;
            live_[w] = w;
            live_pos_[w] = w;
        }
        n_trees_ = V;
        n_edges_ = 0;
        dirty_list_.clear();
        pending_.clear();
    }

    uint32_t V() const { return V_; }
    uint32_t label(uint32_t w) const { return lbl_[w]; }
    bool same_tree(uint32_t a, uint32_t b) const { return lbl_[a] == lbl_[b]; }
    bool is_edge(uint32_t a, uint32_t b) const { return par_[a] == b || par_[b] == a; }
    uint64_t n_trees() const { return n_trees_; }
    uint64_t n_edges() const { return n_edges_; }
    uint32_t tree_size(uint32_t label) const { return size_[label]; }
    uint32_t tree_root(uint32_t label) const { return root_[label]; }

    bool is_dirty(uint32_t label) const { return dirty_[label] != 0; }
    void set_dirty(uint32_t label)
    {
        if (!dirty_[label]) {
            dirty_[label] = 1;
            dirty_list_.push_back(label);
        }
    }
    void clear_dirty(uint32_t label) { dirty_[label] = 0; }
    // Mark every tree dirty (one pass over the vertices).
    void mark_all_dirty()
    {
        for (uint32_t w = 0; w < V_; w++)
            if (root_[lbl_[w]] == w) set_dirty(lbl_[w]);
    }
    // Forget all dirty marks (forests whose marks nobody reads).
    void discard_dirty()
    {
        for (uint32_t l : dirty_list_) dirty_[l] = 0;
        dirty_list_.clear();
    }
    uint32_t parent(uint32_t w) const { return par_[w]; }
    // Labels of the current trees (one each, in no particular order).
    const std::vector<uint32_t> &live_labels() const { return live_; }
    // Labels currently dirty (deduplicated; stale entries dropped).
    std::vector<uint32_t> dirty_labels()
    {
        std::vector<uint32_t> out;
        std::vector<uint32_t> keep;
        for (uint32_t l : dirty_list_) {
            if (dirty_[l] == 1) {
                dirty_[l] = 2;  // mark as collected
                out.push_back(l);
            }
        }
        for (uint32_t l : out) dirty_[l] = 1;
        dirty_list_ = out;
        return out;
    }

    // Link two vertices of different trees.  Returns the merged label.
    uint32_t link(uint32_t a, uint32_t b)
    {
        uint32_t la = lbl_[a], lb = lbl_[b];
        if (size_[la] > size_[lb]) {
            std::swap(a, b);
            std::swap(la, lb);
        }
        // relabel a's (smaller) tree, top-down from its root
        queue_.clear();
        queue_.push_back(root_[la]);
        for (size_t qi = 0; qi < queue_.size(); qi++) {
            const uint32_t x = queue_[qi];
            lbl_[x] = lb;
            touch(x);
            for (uint32_t y = first_kid_[x]; y != kNone; y = next_sib_[y]) queue_.push_back(y);
        }
        // re-root the endpoint with the shorter path to its root (the paths
        // are walked in lockstep) and hang it below the other one (the
        // structural link counts the merge)
        const uint32_t ra = root_[la];
        if (!link_structural_short(a, b)) root_[lb] = ra;  // b's tree hangs below a
        size_[lb] += size_[la];
        if (dirty_[la]) set_dirty(lb);
        dirty_[la] = 0;
        free_.push_back(la);
        live_remove(la);
        return lb;
    }

    // Replace forest edge {a, b} by {x, y}, where x and y are in the same
    // tree and their tree path runs through {a, b}: the tree keeps its
    // vertices (no relabelling); the side below {a, b} is re-rooted at its
    // endpoint of {x, y} (one path reversed) and hung below the other one.
    void swap_edge(uint32_t a, uint32_t b, uint32_t x, uint32_t y)
    {
        const uint32_t child = par_[a] == b ? a : b;
        const uint32_t parent = child == a ? b : a;
        // which of x, y lies below the removed edge
        uint32_t s = x, t = y;
        {
            uint32_t c = x;
            while (c != kNone && c != child) c = par_[c];
            if (c != child) std::swap(s, t);
        }
        remove_kid(parent, child);
        par_[child] = kNone;
        touch(child);
        for (uint32_t c = s, below = kNone; c != kNone;) {
            const uint32_t up = par_[c];
            if (up != kNone) remove_kid(up, c);
            if (below != kNone) {
                par_[c] = below;
                touch(c);
                add_kid(below, c);
            }
            below = c;
            c = up;
        }
        par_[s] = t;
        touch(s);
        add_kid(t, s);
    }

    // Cut forest edge {a, b}.  Returns (label of a's side, label of b's side).
    std::pair<uint32_t, uint32_t> cut(uint32_t a, uint32_t b)
    {
        remove_edge(a, b);
        split_pending();
        return {lbl_[a], lbl_[b]};
    }

    // Remove forest edge {a, b} from the structure (parent pointer and
    // child list) and leave the labels to split_pending().  A run of
    // removals followed by one split costs about as much as splitting each
    // tree once into all its pieces.  Until split_pending() runs, labels,
    // sizes and roots still describe the trees before the removals: only
    // is_edge() and remove_edge() may be called in between.
    void remove_edge(uint32_t a, uint32_t b)
    {
        const uint32_t child = par_[a] == b ? a : b;
        const uint32_t parent = child == a ? b : a;
        remove_kid(parent, child);
        par_[child] = kNone;
        touch(child);
        pending_.push_back({lbl_[child], child});
        n_trees_++;
        n_edges_--;
    }
    bool has_pending() const { return !pending_.empty(); }

    // Relabel the trees split by remove_edge().  Every piece of a split tree
    // is the subtree below its top vertex (the old root, or the child
    // endpoint of a removed edge), so the pieces are searched top-down,
    // interleaved one tree edge at a time; all but the last piece to finish
    // get fresh labels, and the work is about twice the size of the pieces
    // that finish.  Every piece is dirty.
    void split_pending()
    {
        if (pending_.empty()) return;
        std::sort(pending_.begin(), pending_.end());
        for (size_t g0 = 0; g0 < pending_.size();) {
            const uint32_t old = pending_[g0].first;
            size_t g1 = g0;
            while (g1 < pending_.size() && pending_[g1].first == old) g1++;
            const size_t k = g1 - g0 + 1;  // pieces: the old root's, then one per removal
            if (pq_.size() < k) pq_.resize(k);
            pw_.assign(k, Walk{0, kNone});
            active_.clear();
            for (size_t i = 0; i < k; i++) {
                pq_[i].clear();
                pq_[i].push_back(i == 0 ? root_[old] : pending_[g0 + i - 1].second);
                active_.push_back((uint32_t)i);
            }
            uint32_t moved = 0;
            while (active_.size() > 1) {
                for (size_t j = 0; j < active_.size();) {
                    const uint32_t i = active_[j];
                    // a few edges per turn keep the switching cost low
                    bool more = true;
                    for (int t = 0; t < 16 && more; t++) more = step_down(pq_[i], pw_[i]);
                    if (more) {
                        j++;
                        continue;
                    }
                    // piece i is complete: it takes a fresh label
                    const uint32_t nl = free_.back();
                    free_.pop_back();
                    live_add(nl);
                    for (uint32_t x : pq_[i]) {
                        lbl_[x] = nl;
                        touch(x);
                    }
                    size_[nl] = (uint32_t)pq_[i].size();
                    root_[nl] = pq_[i][0];
                    dirty_[nl] = 0;
                    set_dirty(nl);
                    moved += (uint32_t)pq_[i].size();
                    active_[j] = active_.back();
                    active_.pop_back();
                    if (active_.size() == 1) break;
                }
            }
            // the last piece keeps the old label
            size_[old] -= moved;
            root_[old] = pq_[active_[0]][0];
            set_dirty(old);
            g0 = g1;
        }
        pending_.clear();
    }

    // ---- pieces of pending removals, settled without a split ------------
    //
    // After a run of remove_edge(), the trees they broke can be worked on as
    // their pieces (each the subtree below its top: the old root or a
    // removed edge's child endpoint) without relabelling: pending() names
    // them, link_structural() joins pieces by parent pointers only, and
    // settle_*() then assigns the final labels, sizes, roots and dirty
    // marks.  Labels, sizes and roots describe the trees before the
    // removals until the settle.
    const std::vector<std::pair<uint32_t, uint32_t>> &pending() const { return pending_; }
    uint32_t first_child(uint32_t x) const { return first_kid_[x]; }
    uint32_t next_sibling(uint32_t x) const { return next_sib_[x]; }
    // Re-root x's tree at x (one path reversed) and hang it below y.
    void link_structural(uint32_t x, uint32_t y)
    {
        for (uint32_t c = x, below = kNone; c != kNone;) {
            const uint32_t up = par_[c];
            if (up != kNone) remove_kid(up, c);
            if (below != kNone) {
                par_[c] = below;
                touch(c);
                add_kid(below, c);
            }
            below = c;
            c = up;
        }
        par_[x] = y;
        touch(x);
        add_kid(y, x);
        n_trees_--;
        n_edges_++;
    }
    // Link a and b (different trees) by parent pointers only, re-rooting the
    // endpoint whose path to its root is shorter (both paths are walked in
    // lockstep, so the work is about twice the shorter path).  Returns true
    // when a's tree was re-rooted (the root of b's tree is the new root).
    bool link_structural_short(uint32_t a, uint32_t b)
    {
        for (uint32_t x = a, y = b;; x = par_[x], y = par_[y]) {
            if (par_[x] == kNone) {
                link_structural(a, b);
                return true;
            }
            if (par_[y] == kNone) {
                link_structural(b, a);
                return false;
            }
        }
    }
    // Root of x's tree, by parent pointers.
    uint32_t root_of(uint32_t x) const
    {
        while (par_[x] != kNone) x = par_[x];
        return x;
    }
    // A fresh label (a new tree), and giving one back.
    uint32_t settle_take_label()
    {
        const uint32_t l = free_.back();
        free_.pop_back();
        live_add(l);
        dirty_[l] = 0;
        return l;
    }
    void settle_drop_label(uint32_t l)
    {
        dirty_[l] = 0;
        free_.push_back(l);
        live_remove(l);
    }
    void settle_relabel(const uint32_t *v, size_t n, uint32_t l)
    {
        for (size_t i = 0; i < n; i++) lbl_[v[i]] = l;
    }
    // Settle a set of pieces into their final trees in one step (instead of
    // split_pending() and then link_many()).  pieces: (top, group) for every
    // piece of the trees broken by the pending removals (each the subtree
    // below its top: the old root or a removed edge's child endpoint) and
    // the root of every unbroken tree that a link joins; group ids name the
    // final trees (any values).  links: the edges joining the pieces of a
    // group into a tree (they must do so; no other piece is touched).
    //   - A group keeps the label of the largest old tree whose root piece
    //     it holds (ties: the smaller label), else takes a fresh label; only
    //     the pieces whose label changes are relabelled (on the pool when
    //     their vertices are many), so a tree whose pieces all end together
    //     keeps its label and costs nothing.
    //   - Labels no group keeps are freed.  Sizes follow from the relabelled
    //     pieces' sizes (a kept label loses what left and gains what came).
    //   - A group is dirty when one of its pieces was in a broken tree or in
    //     a dirty one (as every piece of a split is dirty, and a link keeps
    //     its parts' marks).
    //   - The links are made by parent pointers; roots follow.
    void settle_regroup(std::vector<std::pair<uint32_t, uint32_t>> &pieces,
                        const std::vector<std::pair<uint32_t, uint32_t>> &links)
    {
        // old trees broken by the pending removals
        for (const auto &pr : pending_) rg_broken_.push_back(pr.first);
        std::sort(rg_broken_.begin(), rg_broken_.end());
        rg_broken_.erase(std::unique(rg_broken_.begin(), rg_broken_.end()), rg_broken_.end());
        auto broken = [&](uint32_t l) {
            return std::binary_search(rg_broken_.begin(), rg_broken_.end(), l);
        };
        std::sort(pieces.begin(), pieces.end(),
                  [](const std::pair<uint32_t, uint32_t> &a, const std::pair<uint32_t, uint32_t> &b) {
                      return a.second != b.second ? a.second < b.second : a.first < b.first;
                  });
        // per group: its target label and dirty mark; per piece: the job
        rg_target_.assign(pieces.size(), kNone);
        rg_jobs_.clear();
        rg_group_end_.clear();
        rg_kept_.clear();
        for (size_t g0 = 0; g0 < pieces.size();) {
            size_t g1 = g0;
            while (g1 < pieces.size() && pieces[g1].second == pieces[g0].second) g1++;
            uint32_t keep = kNone;
            bool dirty = false;
            for (size_t i = g0; i < g1; i++) {
                const uint32_t t = pieces[i].first, l = lbl_[t];
                dirty = dirty || dirty_[l] || broken(l);
                if (root_[l] != t) continue;  // not the old tree's root piece
                if (keep == kNone || size_[l] > size_[keep] || (size_[l] == size_[keep] && l < keep))
                    keep = l;
            }
            const bool fresh = keep == kNone;
            if (fresh) keep = settle_take_label();
            else rg_kept_.push_back(keep);
            for (size_t i = g0; i < g1; i++) {
                rg_target_[i] = keep;
                if (lbl_[pieces[i].first] != keep) rg_jobs_.push_back((uint32_t)i);
            }
            if (fresh) size_[keep] = 0;
            rg_group_end_.push_back({(uint32_t)g1, dirty ? 1u : 0u});
            g0 = g1;
        }
        std::sort(rg_kept_.begin(), rg_kept_.end());
        // relabel the pieces that change tree (disjoint subtrees)
        rg_size_.assign(rg_jobs_.size(), 0);
        rg_old_.assign(rg_jobs_.size(), 0);
        size_t work = 0;
        for (size_t j = 0; j < rg_jobs_.size(); j++) {
            const uint32_t t = pieces[rg_jobs_[j]].first;
            rg_old_[j] = lbl_[t];
            work += size_[rg_old_[j]];  // a bound: the piece is part of its old tree
        }
        auto one = [&](size_t j, unsigned w) {
            const uint32_t i = rg_jobs_[j];
            std::vector<uint32_t> &q = pool_ ? wq_[w] : queue_;
            relabel_tree_with(q, pieces[i].first, rg_target_[i]);
            rg_size_[j] = (uint32_t)q.size();
        };
        if (pool_ && rg_jobs_.size() > 1 && work >= par_work_)
            pool_->run(rg_jobs_.size(), one);
        else
            for (size_t j = 0; j < rg_jobs_.size(); j++) one(j, 0);
        // sizes: what left each old tree, what came to each target
        for (size_t j = 0; j < rg_jobs_.size(); j++) {
            size_[rg_old_[j]] -= rg_size_[j];
            size_[rg_target_[rg_jobs_[j]]] += rg_size_[j];
        }
        // labels no group keeps (all their pieces left) are freed once
        for (size_t j = 0; j < rg_jobs_.size(); j++) {
            const uint32_t l = rg_old_[j];
            if (size_[l] == 0 && !std::binary_search(rg_kept_.begin(), rg_kept_.end(), l) &&
                live_pos_[l] < live_.size() && live_[live_pos_[l]] == l) {
                settle_drop_label(l);
            }
        }
        // links by parent pointers, then roots and dirty marks per group
        for (const auto &e : links) link_structural_short(e.first, e.second);
        size_t g0 = 0;
        for (const auto &ge : rg_group_end_) {
            const uint32_t l = rg_target_[g0];
            root_[l] = root_of(pieces[g0].first);
            if (ge.second) set_dirty(l);
            g0 = ge.first;
        }
        pending_.clear();
        rg_broken_.clear();
    }

    // Relabel every vertex of the tree rooted at r (top-down).
    void settle_relabel_tree(uint32_t r, uint32_t l) { relabel_tree_with(queue_, r, l); }
    // Label every vertex of the tree rooted at r with l (q: scratch).
    void relabel_tree_with(std::vector<uint32_t> &q, uint32_t r, uint32_t l)
    {
        q.clear();
        q.push_back(r);
        for (size_t qi = 0; qi < q.size(); qi++) {
            const uint32_t x = q[qi];
            lbl_[x] = l;
            touch(x);
            for (uint32_t y = first_kid_[x]; y != kNone; y = next_sib_[y]) q.push_back(y);
        }
    }
    void settle_tree(uint32_t l, uint32_t root, uint32_t size, bool dirty)
    {
        root_[l] = root;
        size_[l] = size;
        dirty_[l] = 0;
        if (dirty) set_dirty(l);
    }
    void settle_done() { pending_.clear(); }

    // Link, in order, every pair (a, b) of `cand` whose endpoints are in
    // different trees at its turn: the same links as calling link() for
    // each pair that same_tree() rejects not, but decided on a union-find
    // over the trees' labels, and each merged tree is labelled once (it
    // keeps its largest part's label, whose vertices are not touched), so a
    // vertex is relabelled at most once however many merges it takes part
    // in.  Marks the pairs that linked in `linked` (same length as cand) and
    // returns their number.  Must not be called with removals pending.
    size_t link_many(const std::vector<std::pair<uint32_t, uint32_t>> &cand,
                     std::vector<uint8_t> &linked)
    {
        linked.assign(cand.size(), 0);
        if (lm_st_.size() != V_ || lm_ep_ == 0xffffffffu) {
            lm_up_.assign(V_, 0);
            lm_sz_.assign(V_, 0);
            lm_st_.assign(V_, 0);
            lm_best_.assign(V_, 0);
            lm_ep_ = 0;
        }
        lm_ep_++;
        lm_touched_.clear();
        lm_edges_.clear();
        auto node = [&](uint32_t l) {
            if (lm_st_[l] != lm_ep_) {
                lm_st_[l] = lm_ep_;
                lm_up_[l] = l;
                lm_sz_[l] = size_[l];
                lm_touched_.push_back(l);
            }
            return l;
        };
        auto find = [&](uint32_t l) {
            while (lm_up_[l] != l) l = lm_up_[l] = lm_up_[lm_up_[l]];
            return l;
        };
        for (size_t i = 0; i < cand.size(); i++) {
            uint32_t a = cand[i].first, b = cand[i].second;
            uint32_t ra = find(node(lbl_[a])), rb = find(node(lbl_[b]));
            if (ra == rb) continue;
            if (lm_sz_[ra] > lm_sz_[rb]) {  // the smaller side is re-rooted
                std::swap(a, b);
                std::swap(ra, rb);
            }
            lm_edges_.push_back({a, b});
            lm_up_[ra] = rb;
            lm_sz_[rb] += lm_sz_[ra];
            linked[i] = 1;
        }
        if (lm_edges_.empty()) return 0;
        // the label each merged tree keeps: its largest part's (ties: the
        // smaller label); dirty when a part is
        for (uint32_t l : lm_touched_)
            if (find(l) == l) lm_best_[l] = kNone;
        for (uint32_t l : lm_touched_) {
            const uint32_t r = find(l), c = lm_best_[r];
            if (c == kNone || size_[l] > size_[c] || (size_[l] == size_[c] && l < c))
                lm_best_[r] = l;
        }
        for (uint32_t l : lm_touched_)
            if (dirty_[l]) set_dirty(lm_best_[find(l)]);
        // relabel the other parts in the structure before the links (the
        // trees are disjoint: in parallel when there is enough of them)
        lm_jobs_.clear();
        size_t lm_work = 0;
        for (uint32_t l : lm_touched_) {
            const uint32_t keep = lm_best_[find(l)];
            if (l != keep) {
                lm_jobs_.push_back({root_[l], keep});
                lm_work += size_[l];
            }
        }
        relabel_trees(lm_jobs_, lm_work);
        for (const auto &e : lm_edges_) link_structural_short(e.first, e.second);
        for (uint32_t l : lm_touched_) {
            const uint32_t r = find(l), keep = lm_best_[r];
            if (l != keep) {
                dirty_[l] = 0;
                free_.push_back(l);
                live_remove(l);
            } else {
                size_[keep] = lm_sz_[r];
            }
        }
        for (uint32_t l : lm_touched_) {
            const uint32_t keep = lm_best_[find(l)];
            if (l == keep) root_[keep] = root_of(root_[keep]);
        }
        return lm_edges_.size();
    }

    // Vertices of the tree with the given label (BFS from its root); also
    // returns the smallest vertex id.
    // Use `p` (may be null) for the host work that splits over trees.
    void set_pool(Pool *p)
    {
        pool_ = p;
        wq_.resize(p ? p->size() : 1);
    }
    Pool *pool() const { return pool_; }

    // Relabel whole trees: jobs (root, new label); `work` = their total
    // size, which decides whether the pool is worth waking.
    void relabel_trees(const std::vector<std::pair<uint32_t, uint32_t>> &jobs, size_t work)
    {
        if (pool_ && jobs.size() > 1 && work >= par_work_) {
            pool_->run(jobs.size(), [&](size_t i, unsigned w) {
                relabel_tree_with(wq_[w], jobs[i].first, jobs[i].second);
            });
        } else {
            for (const auto &j : jobs) relabel_tree_with(queue_, j.first, j.second);
        }
    }
    // Vertices from which splitting host work over the pool pays.
    size_t parallel_work() const { return par_work_; }
    void set_parallel_work(size_t n) { par_work_ = n; }

    uint32_t collect(uint32_t label, std::vector<uint32_t> &out) const
    {
        const uint32_t r = root_[label];
        const size_t start = out.size();
        out.push_back(r);
        uint32_t mn = r;
        for (size_t qi = start; qi < out.size(); qi++) {
            const uint32_t x = out[qi];
            for (uint32_t y = first_kid_[x]; y != kNone; y = next_sib_[y]) {
                out.push_back(y);
                mn = std::min(mn, y);
            }
        }
        return mn;
    }

    void edges(std::vector<uint32_t> &eu, std::vector<uint32_t> &ev) const
    {
        for (uint32_t w = 0; w < V_; w++)
            if (par_[w] != kNone) {
                eu.push_back(std::min(w, par_[w]));
                ev.push_back(std::max(w, par_[w]));
            }
    }

    // ---- pages written since the last take_pages() -----------------------
    // With tracking on, every label or parent write marks its page of
    // 2^shift vertices (from the pool's workers too), so that a copy
    // elsewhere can be refreshed page by page.  Turning it on marks every
    // page.
    void track_pages(uint32_t shift)
    {
        pshift_ = shift;
        pages_.assign(((size_t)V_ >> shift) + 1, 1);
        track_ = true;
    }
    uint32_t page_shift() const { return pshift_; }
    size_t n_pages() const { return pages_.size(); }
    // Append the marked pages to `out` and clear their marks.
    void take_pages(std::vector<uint32_t> &out)
    {
        for (size_t p = 0; p < pages_.size(); p++)
            if (pages_[p]) {
                out.push_back((uint32_t)p);
                pages_[p] = 0;
            }
    }

  private:
    void touch(uint32_t x)
    {
        // read first: a page is written many times between two takes, and
        // stores to the few cache lines of marks from every pool worker
        // would bounce those lines between cores
        if (!track_) return;
        uint8_t *m = &pages_[x >> pshift_];
        if (!__atomic_load_n(m, __ATOMIC_RELAXED)) __atomic_store_n(m, (uint8_t)1, __ATOMIC_RELAXED);
    }
    std::vector<uint8_t> pages_;
    uint32_t pshift_ = 0;
    bool track_ = false;

    // position of a top-down piece search: queue index, and the next child
    // of that vertex to look at (kNone: start at its first child)
    struct Walk {
        size_t qi;
        uint32_t next;
    };
    // Advance a top-down search of one piece by one tree edge.  Returns
    // false when the piece is complete.
    bool step_down(std::vector<uint32_t> &q, Walk &w)
    {
        for (;;) {
            if (w.qi == q.size()) return false;
            const uint32_t y = w.next == kNone ? first_kid_[q[w.qi]] : w.next;
            if (y != kNone) {
                q.push_back(y);
                w.next = next_sib_[y];
                if (w.next == kNone) {
                    w.qi++;
                }
                return true;
            }
            w.qi++;
            w.next = kNone;
        }
    }
    // children of a vertex form a doubly linked list (insert and remove in
    // O(1), one memory access per child when walking it)
    void live_add(uint32_t l)
    {
        live_pos_[l] = (uint32_t)live_.size();
        live_.push_back(l);
    }
    void live_remove(uint32_t l)
    {
        const uint32_t i = live_pos_[l], last = live_.back();
        live_[i] = last;
        live_pos_[last] = i;
        live_.pop_back();
    }
    void add_kid(uint32_t p, uint32_t c)
    {
        const uint32_t f = first_kid_[p];
        next_sib_[c] = f;
        prev_sib_[c] = kNone;
        if (f != kNone) prev_sib_[f] = c;
        first_kid_[p] = c;
    }
    void remove_kid(uint32_t p, uint32_t c)
    {
        const uint32_t pv = prev_sib_[c], nx = next_sib_[c];
        if (pv == kNone)
            first_kid_[p] = nx;
        else
            next_sib_[pv] = nx;
        if (nx != kNone) prev_sib_[nx] = pv;
    }

    uint32_t V_ = 0;
    uint32_t *lbl_ = nullptr;
    uint32_t *par_ = nullptr;
    std::vector<uint32_t> first_kid_, next_sib_, prev_sib_;  // child lists
    std::vector<uint32_t> size_;   // by label
    std::vector<uint32_t> root_;   // by label
    std::vector<uint8_t> dirty_;   // by label
    std::vector<uint32_t> dirty_list_;
    std::vector<uint32_t> free_;
    std::vector<uint32_t> live_, live_pos_;  // labels in use, and each one's slot
    std::vector<uint32_t> queue_;
    Pool *pool_ = nullptr;
    size_t par_work_ = 16384;
    std::vector<std::vector<uint32_t>> wq_ = std::vector<std::vector<uint32_t>>(1);  // per worker
    std::vector<std::pair<uint32_t, uint32_t>> lm_jobs_;
    // settle_regroup
    std::vector<uint32_t> rg_broken_, rg_target_, rg_jobs_, rg_size_, rg_old_, rg_kept_;
    std::vector<std::pair<uint32_t, uint32_t>> rg_group_end_;
    std::vector<uint32_t> lm_up_, lm_sz_, lm_st_, lm_best_, lm_touched_;  // link_many, by label
    uint32_t lm_ep_ = 0;
    std::vector<std::pair<uint32_t, uint32_t>> lm_edges_;
    std::vector<std::pair<uint32_t, uint32_t>> pending_;  // (old label, top) per removal
    std::vector<std::vector<uint32_t>> pq_;              // per-piece search queues
    std::vector<Walk> pw_;
    std::vector<uint32_t> active_;
    uint64_t n_trees_ = 0;
    uint64_t n_edges_ = 0;
};

}  // namespace cupk
