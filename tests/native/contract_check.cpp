// Randomized check of the contracted walk (paper_2509_14433_amd/csrc/
// contract.hpp) against the one-by-one walk of the same runs of updates on
// a copy of the same forest: forest edges, trees, dirty trees and the counts
// of links and cuts must agree after every run, and every label or parent
// written must lie in a page the forest marked.  Runs toggle a small pool of
// edges between trees many times (links and cuts undone within the run),
// delete forest edges and insert random pairs; some runs get a piece-search
// budget too small to finish, so the fallback is exercised as well.  Built
// and run by tests/test_forest_host.py (host code only, with sanitizers).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <memory>
#include <set>
#include <vector>

#include "contract.hpp"
#include "forest.hpp"

using cupk::Contraction;
using cupk::Forest;

static uint64_t pack(uint32_t a, uint32_t b, bool del)
{
    // either endpoint order, as a batch may hold it
    return (uint64_t)a | (uint64_t)b << 32 | (uint64_t)(del ? 1 : 0) << 63;
}

// The one-by-one walk: inserts link two different trees (pending pieces
// split first), deletes of forest edges are removed.
static void walk_plain(Forest &F, const std::vector<uint64_t> &run, uint64_t &links,
                       uint64_t &cuts)
{
    for (uint64_t p : run) {
        uint32_t a = (uint32_t)p, b = (uint32_t)(p >> 32) & 0x7fffffffu;
        if (a > b) std::swap(a, b);
        if ((p >> 63) == 0) {
            if (F.has_pending()) F.split_pending();
            if (!F.same_tree(a, b)) {
                F.link(a, b);
                links++;
            }
        } else if (F.is_edge(a, b)) {
            F.remove_edge(a, b);
            cuts++;
        }
    }
}

static int fail(const char *what, uint64_t run)
{
    fprintf(stderr, "FAIL %s after run %llu\n", what, (unsigned long long)run);
    return 1;
}

// Every vertex whose label or parent changed since the last call lies in a
// page the forest marked; then the marks are cleared and the copies
// refreshed.
static bool pages_cover(Forest &F, const std::vector<uint32_t> &l, const std::vector<uint32_t> &p,
                        std::vector<uint32_t> &lc, std::vector<uint32_t> &pc)
{
    std::vector<uint32_t> pg;
    F.take_pages(pg);
    std::vector<uint8_t> mark(F.n_pages(), 0);
    for (uint32_t x : pg) mark[x] = 1;
    for (size_t w = 0; w < l.size(); w++)
        if ((l[w] != lc[w] || p[w] != pc[w]) && !mark[w >> F.page_shift()]) return false;
    lc = l;
    pc = p;
    return true;
}

static std::vector<uint32_t> canon(const Forest &F)
{
    // smallest vertex of each vertex's tree
    const uint32_t V = F.V();
    std::map<uint32_t, uint32_t> low;
    std::vector<uint32_t> c(V);
    for (uint32_t w = 0; w < V; w++) {
        auto it = low.find(F.label(w));
        if (it == low.end()) it = low.insert({F.label(w), w}).first;
        c[w] = it->second;
    }
    return c;
}

static int compare(Forest &A, Forest &B, uint64_t r)
{
    A.split_pending();
    B.split_pending();
    std::vector<uint32_t> au, av, bu, bv;
    A.edges(au, av);
    B.edges(bu, bv);
    std::set<std::pair<uint32_t, uint32_t>> ea, eb;
    for (size_t i = 0; i < au.size(); i++) ea.insert({au[i], av[i]});
    for (size_t i = 0; i < bu.size(); i++) eb.insert({bu[i], bv[i]});
    if (ea != eb) return fail("forest edges", r);
    if (A.n_trees() != B.n_trees()) return fail("tree count", r);
    if (canon(A) != canon(B)) return fail("trees", r);
    for (uint32_t w = 0; w < A.V(); w++)
        if (A.is_dirty(A.label(w)) != B.is_dirty(B.label(w))) return fail("dirty trees", r);
    for (uint32_t w = 0; w < A.V(); w++)
        if (A.tree_size(A.label(w)) != B.tree_size(B.label(w))) return fail("tree sizes", r);
    // child lists agree with the parent pointers
    for (const Forest *F : {&A, &B}) {
        size_t kids = 0, nonroots = 0;
        for (uint32_t w = 0; w < F->V(); w++) {
            if (F->parent(w) != cupk::kNone) nonroots++;
            for (uint32_t y = F->first_child(w); y != cupk::kNone; y = F->next_sibling(y)) {
                if (F->parent(y) != w) return fail("child lists", r);
                if (++kids > F->V()) return fail("child lists (cycle)", r);
            }
        }
        if (kids != nonroots) return fail("child list count", r);
    }
    // the live label list names exactly the labels in use
    for (const Forest *F : {&A, &B}) {
        std::set<uint32_t> used, live(F->live_labels().begin(), F->live_labels().end());
        for (uint32_t w = 0; w < F->V(); w++) used.insert(F->label(w));
        if (used != live || live.size() != F->live_labels().size())
            return fail("live labels", r);
    }
    // each tree's recorded root is a root of that tree
    for (const Forest *F : {&A, &B})
        for (uint32_t w = 0; w < F->V(); w++) {
            const uint32_t rt = F->tree_root(F->label(w));
            if (F->parent(rt) != cupk::kNone || F->label(rt) != F->label(w))
                return fail("tree roots", r);
        }
    return 0;
}

int main(int argc, char **argv)
{
    const uint32_t V = argc > 1 ? (uint32_t)atoi(argv[1]) : 200;
    const uint64_t runs = argc > 2 ? (uint64_t)atoll(argv[2]) : 300;
    const uint64_t seed = argc > 3 ? (uint64_t)atoll(argv[3]) : 1;
    // threads > 0: B relabels merged trees on a pool of that many workers,
    // whatever their size
    const unsigned threads = argc > 4 ? (unsigned)atoi(argv[4]) : 0;
    std::mt19937_64 rng(seed);
    std::vector<uint32_t> la(V), pa(V), lb(V), pb(V);
    Forest A, B;
    A.init(V, la.data(), pa.data());
    B.init(V, lb.data(), pb.data());
    // pages of 4 vertices: every write must mark its page
    A.track_pages(2);
    B.track_pages(2);
    std::vector<uint32_t> lac(V, ~0u), pac(V, ~0u), lbc(V, ~0u), pbc(V, ~0u);
    auto pages_ok = [&]() {
        return pages_cover(A, la, pa, lac, pac) && pages_cover(B, lb, pb, lbc, pbc);
    };
    if (!pages_ok()) return fail("page marks after init", 0);
    std::unique_ptr<cupk::Pool> workers;
    if (threads) {
        workers.reset(new cupk::Pool(threads));
        B.set_pool(workers.get());
        B.set_parallel_work(1);
    }
    Contraction C;
    uint64_t many_runs = 0;
    // the graph's edges (what a valid stream toggles)
    std::set<std::pair<uint32_t, uint32_t>> G;
    // a pool of edges toggled again and again
    std::vector<std::pair<uint32_t, uint32_t>> pool;
    for (uint32_t i = 0; i < std::max<uint32_t>(4, V / 8); i++) {
        uint32_t a = (uint32_t)(rng() % V), b = (uint32_t)(rng() % V);
        if (a == b) continue;
        pool.push_back({std::min(a, b), std::max(a, b)});
    }
    // a start forest: random links from singletons, one by one on A and in
    // one link_many on B
    {
        std::vector<std::pair<uint32_t, uint32_t>> cand;
        for (uint32_t i = 0; i < V; i++) {
            const uint32_t a = (uint32_t)(rng() % V), b = (uint32_t)(rng() % V);
            if (a != b) cand.push_back({a, b});
        }
        std::vector<uint8_t> got;
        size_t nw = 0;
        for (const auto &e : cand)
            if (!A.same_tree(e.first, e.second)) {
                A.link(e.first, e.second);
                G.insert({std::min(e.first, e.second), std::max(e.first, e.second)});
                nw++;
            }
        if (B.link_many(cand, got) != nw) return fail("link_many: start forest", 0);
        if (compare(A, B, 0)) return 1;
        if (!pages_ok()) return fail("page marks: start forest", 0);
    }
    uint64_t fallbacks = 0, contracted = 0;
    for (uint64_t r = 0; r < runs; r++) {
        // some trees dirty when the run starts (failed queries keep them)
        for (uint32_t l : A.dirty_labels()) A.clear_dirty(l);
        for (uint32_t l : B.dirty_labels()) B.clear_dirty(l);
        for (uint32_t t = 0; t < 3; t++) {
            const uint32_t w = (uint32_t)(rng() % V);
            if (rng() % 2) {
                A.set_dirty(A.label(w));
                B.set_dirty(B.label(w));
            }
        }
        if (rng() % 4 == 0) {
            // a list of candidate links (as a replacement round produces):
            // Forest::link_many against link() one pair at a time
            A.split_pending();
            B.split_pending();
            std::vector<std::pair<uint32_t, uint32_t>> cand;
            const uint32_t len = 1 + (uint32_t)(rng() % (2 * V));
            for (uint32_t i = 0; i < len; i++) {
                const uint32_t a = (uint32_t)(rng() % V), b = (uint32_t)(rng() % V);
                if (a != b) cand.push_back({a, b});
            }
            std::vector<uint8_t> want(cand.size(), 0), got;
            size_t nw = 0;
            for (size_t i = 0; i < cand.size(); i++)
                if (!A.same_tree(cand[i].first, cand[i].second)) {
                    A.link(cand[i].first, cand[i].second);
                    want[i] = 1;
                    nw++;
                }
            const size_t ng = B.link_many(cand, got);
            if (ng != nw || got != want) return fail("link_many: links", r);
            for (size_t i = 0; i < cand.size(); i++)
                if (want[i]) G.insert({std::min(cand[i].first, cand[i].second),
                                       std::max(cand[i].first, cand[i].second)});
            if (compare(A, B, r)) return 1;
            if (!pages_ok()) return fail("page marks: link_many", r);
            many_runs++;
            continue;
        }
        std::vector<uint64_t> run;
        const uint32_t len = 1 + (uint32_t)(rng() % 64);
        for (uint32_t i = 0; i < len; i++) {
            const uint32_t mode = (uint32_t)(rng() % 10);
            uint32_t a, b;
            if (mode < 6 && !pool.empty()) {
                const auto &e = pool[rng() % pool.size()];
                a = e.first;
                b = e.second;
            } else if (mode < 8 && !G.empty()) {
                auto it = G.begin();
                std::advance(it, rng() % G.size());
                a = it->first;
                b = it->second;
            } else {
                a = (uint32_t)(rng() % V);
                b = (uint32_t)(rng() % V);
                if (a == b) continue;
                if (a > b) std::swap(a, b);
            }
            const bool present = G.count({a, b}) != 0;
            if (present)
                G.erase({a, b});
            else
                G.insert({a, b});
            // occasionally an invalid update (delete of an absent edge, or
            // insert of a present one): both walks must still agree
            const bool del = (rng() % 50 == 0) ? !present : present;
            run.push_back(rng() % 2 ? pack(a, b, del) : pack(b, a, del));
        }
        // a run sometimes starts with removals still pending
        if (rng() % 4 == 0) {
            std::vector<uint32_t> eu, ev;
            A.edges(eu, ev);
            if (!eu.empty()) {
                const size_t k = rng() % eu.size();
                A.remove_edge(eu[k], ev[k]);
                B.remove_edge(eu[k], ev[k]);
                G.erase({eu[k], ev[k]});
            }
        }
        uint64_t l0 = 0, c0 = 0, l1 = 0, c1 = 0;
        walk_plain(A, run, l0, c0);
        if (rng() % 5 == 0)
            C.set_budget(0, rng() % 8);
        else
            C.set_budget(64, 4096);
        bool changed = false;
        std::vector<uint32_t> eb0, ev0;
        B.edges(eb0, ev0);
        if (C.run(B, run.data(), 0, (uint32_t)run.size(), &l1, &c1, &changed)) {
            contracted++;
        } else {
            // nothing but pending splits done: the edges are as before
            std::vector<uint32_t> eb1, ev1;
            B.edges(eb1, ev1);
            if (eb0 != eb1 || ev0 != ev1) return fail("fallback changed edges", r);
            fallbacks++;
            walk_plain(B, run, l1, c1);
        }
        if (l0 != l1 || c0 != c1) return fail("link / cut counts", r);
        if (compare(A, B, r)) return 1;
        if (!pages_ok()) return fail("page marks", r);
    }
    printf("ok V=%u runs=%llu contracted=%llu fallbacks=%llu link lists=%llu\n", V,
           (unsigned long long)runs, (unsigned long long)contracted,
           (unsigned long long)fallbacks, (unsigned long long)many_runs);
    // both paths must have run (tiny forests never exhaust a budget)
    return contracted && (fallbacks || V < 8 || runs < 20) ? 0 : 2;
}
