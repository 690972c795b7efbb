// Host spanning forest with exact component labels.
//
// The paper answers connectivity queries from a sketchless dynamic tree on
// the top level (Sec. 4.1) and links / cuts forest edges as updates demand
// (cutset Link / Cut, Sec. 2.2.1).  Here the forest is a rooted forest:
// parent pointers, child lists (each child knows its slot in its parent's
// list, so an edge is removed in O(1)), and one label per vertex naming its
// tree:
//   - link(a, b): the smaller tree is re-rooted at its endpoint, hung below
//     the other endpoint and relabelled (work proportional to the smaller
//     tree);
//   - cut(a, b): the edge is removed and the two sides are explored by
//     breadth-first searches interleaved edge by edge, so the work is
//     proportional to the smaller side (even next to a high-degree
//     vertex); the smaller side gets a fresh label.
// Labels come from a free list in [0, V), so label arrays are V words and
// the device can classify updates against them (lbl[u] != lbl[v] means u
// and v are in different trees; par[] identifies forest edges).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

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
        kids_.assign(V, {});
        // most tree vertices have a few children: reserving them keeps
        // relinking free of small reallocations
        for (auto &k : kids_) k.reserve(2);
        kid_pos_.assign(V, 0);
        bfs_par_.assign(V, kNone);
        size_.assign(V, 1);
        root_.resize(V);
        dirty_.assign(V, 0);
        free_.clear();
        for (uint32_t w = 0; w < V; w++) {
            lbl_[w] = w;
            par_[w] = kNone;
            root_[w] = w;
        }
        stamp_.assign(V, 0);
        epoch_ = 0;
        n_trees_ = V;
        n_edges_ = 0;
        dirty_list_.clear();
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
        // re-root a's (smaller) tree at a: breadth-first search over its
        // undirected tree edges, remembering each vertex's search parent
        const uint32_t ep = next_epoch();
        queue_.clear();
        queue_.push_back(a);
        stamp_[a] = ep;
        bfs_par_[a] = kNone;
        for (size_t qi = 0; qi < queue_.size(); qi++) {
            const uint32_t x = queue_[qi];
            const uint32_t px = par_[x];
            if (px != kNone && stamp_[px] != ep) {
                stamp_[px] = ep;
                bfs_par_[px] = x;
                queue_.push_back(px);
            }
            for (uint32_t y : kids_[x]) {
                if (stamp_[y] == ep) continue;
                stamp_[y] = ep;
                bfs_par_[y] = x;
                queue_.push_back(y);
            }
        }
        // rebuild parent pointers and child lists from the search tree, hang
        // a below b and relabel
        for (uint32_t x : queue_) kids_[x].clear();
        for (uint32_t x : queue_) {
            lbl_[x] = lb;
            const uint32_t p = bfs_par_[x];
            if (p == kNone) continue;
            par_[x] = p;
            add_kid(p, x);
        }
        par_[a] = b;
        add_kid(b, a);
        size_[lb] += size_[la];
        if (dirty_[la]) set_dirty(lb);
        dirty_[la] = 0;
        free_.push_back(la);
        n_trees_--;
        n_edges_++;
        return lb;
    }

    // Cut forest edge {a, b}.  Returns (label of a's side, label of b's side).
    std::pair<uint32_t, uint32_t> cut(uint32_t a, uint32_t b)
    {
        const uint32_t old = lbl_[a];
        // the child endpoint becomes the root of its side
        const uint32_t child = par_[a] == b ? a : b;
        const uint32_t parent = child == a ? b : a;
        remove_kid(parent, child);
        par_[child] = kNone;
        // breadth-first searches from a and b, interleaved one edge at a
        // time; the side that finishes first is the smaller one
        const uint32_t ea = next_epoch();
        const uint32_t eb = next_epoch();
        qa_.clear();
        qb_.clear();
        qa_.push_back(a);
        qb_.push_back(b);
        stamp_[a] = ea;
        stamp_[b] = eb;
        Walk wa{0, 0}, wb{0, 0};
        bool a_small;
        for (;;) {
            if (!step(qa_, wa, ea)) {
                a_small = true;
                break;
            }
            if (!step(qb_, wb, eb)) {
                a_small = false;
                break;
            }
        }
        const std::vector<uint32_t> &small = a_small ? qa_ : qb_;
        const uint32_t nl = free_.back();
        free_.pop_back();
        for (uint32_t x : small) lbl_[x] = nl;
        size_[nl] = (uint32_t)small.size();
        size_[old] -= (uint32_t)small.size();
        // roots: the side holding the old root keeps it; the other side is
        // rooted at the child endpoint
        const uint32_t small_end = a_small ? a : b;
        const bool small_has_child = small_end == child;
        if (small_has_child) {
            root_[nl] = child;
        } else {
            root_[nl] = root_[old];
            root_[old] = child;
        }
        dirty_[nl] = 0;
        set_dirty(old);
        set_dirty(nl);
        n_trees_++;
        n_edges_--;
        const uint32_t la = lbl_[a], lb2 = lbl_[b];
        return {la, lb2};
    }

    // Vertices of the tree with the given label (BFS from its root); also
    // returns the smallest vertex id.
    uint32_t collect(uint32_t label, std::vector<uint32_t> &out)
    {
        const uint32_t r = root_[label];
        const uint32_t ep = next_epoch();
        const size_t start = out.size();
        out.push_back(r);
        stamp_[r] = ep;
        uint32_t mn = r;
        (void)ep;
        for (size_t qi = start; qi < out.size(); qi++) {
            const uint32_t x = out[qi];
            for (uint32_t y : kids_[x]) {
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

  private:
    uint32_t next_epoch()
    {
        if (++epoch_ == 0) {
            std::fill(stamp_.begin(), stamp_.end(), 0u);
            epoch_ = 1;
        }
        return epoch_;
    }
    // position of an interleaved search: queue index, and the next
    // neighbour of that vertex to look at (0 = its parent, 1+k = child k)
    struct Walk {
        size_t qi;
        size_t ni;
    };
    // Advance a search by one tree edge.  Returns false when the search has
    // no vertex left to expand (its side is complete).
    bool step(std::vector<uint32_t> &q, Walk &w, uint32_t ep)
    {
        for (;;) {
            if (w.qi == q.size()) return false;
            const uint32_t x = q[w.qi];
            const auto &k = kids_[x];
            if (w.ni == 0) {
                w.ni = 1;
                const uint32_t p = par_[x];
                if (p != kNone && stamp_[p] != ep) {
                    stamp_[p] = ep;
                    q.push_back(p);
                    return true;
                }
                continue;
            }
            if (w.ni - 1 < k.size()) {
                const uint32_t y = k[w.ni - 1];
                w.ni++;
                if (stamp_[y] != ep) {
                    stamp_[y] = ep;
                    q.push_back(y);
                }
                return true;
            }
            w.qi++;
            w.ni = 0;
        }
    }
    void add_kid(uint32_t p, uint32_t c)
    {
        kid_pos_[c] = (uint32_t)kids_[p].size();
        kids_[p].push_back(c);
    }
    void remove_kid(uint32_t p, uint32_t c)
    {
        auto &k = kids_[p];
        const uint32_t i = kid_pos_[c];
        const uint32_t last = k.back();
        k[i] = last;
        kid_pos_[last] = i;
        k.pop_back();
    }

    uint32_t V_ = 0;
    uint32_t *lbl_ = nullptr;
    uint32_t *par_ = nullptr;
    std::vector<std::vector<uint32_t>> kids_;  // children of each vertex
    std::vector<uint32_t> kid_pos_;            // slot of a vertex in its parent's list
    std::vector<uint32_t> bfs_par_;            // scratch of link
    std::vector<uint32_t> size_;   // by label
    std::vector<uint32_t> root_;   // by label
    std::vector<uint8_t> dirty_;   // by label
    std::vector<uint32_t> dirty_list_;
    std::vector<uint32_t> free_;
    std::vector<uint32_t> stamp_;
    std::vector<uint32_t> queue_, qa_, qb_;
    uint32_t epoch_ = 0;
    uint64_t n_trees_ = 0;
    uint64_t n_edges_ = 0;
};

}  // namespace cupk
