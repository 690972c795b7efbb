// Randomized check of the host forest (paper_2509_14433_amd/csrc/forest.hpp)
// against a naive model: adjacency sets and breadth-first search.  Built and
// run by tests/test_forest_host.py (host code only, with sanitizers).
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <set>
#include <vector>

#include "forest.hpp"

using cupk::Forest;

struct Naive {
    uint32_t V;
    std::vector<std::set<uint32_t>> adj;
    explicit Naive(uint32_t v) : V(v), adj(v) {}
    std::vector<uint32_t> comp() const
    {
        std::vector<uint32_t> c(V, UINT32_MAX);
        for (uint32_t s = 0; s < V; s++) {
            if (c[s] != UINT32_MAX) continue;
            std::deque<uint32_t> q{s};
            c[s] = s;
            while (!q.empty()) {
                uint32_t x = q.front();
                q.pop_front();
                for (uint32_t y : adj[x])
                    if (c[y] == UINT32_MAX) {
                        c[y] = s;
                        q.push_back(y);
                    }
            }
        }
        return c;
    }
};

static int fail(const char *what, uint64_t step)
{
    fprintf(stderr, "FAIL %s at step %llu\n", what, (unsigned long long)step);
    return 1;
}

static int check(Forest &F, Naive &N, uint64_t step)
{
    const std::vector<uint32_t> c = N.comp();
    std::set<uint32_t> roots(c.begin(), c.end());
    if (F.n_trees() != roots.size()) return fail("tree count", step);
    for (uint32_t w = 0; w < N.V; w++)
        for (uint32_t x : {0u, w / 3, (w * 7 + 1) % N.V})
            if (F.same_tree(w, x) != (c[w] == c[x])) return fail("same_tree", step);
    std::vector<uint32_t> eu, ev;
    F.edges(eu, ev);
    std::set<std::pair<uint32_t, uint32_t>> fe, ne;
    for (size_t i = 0; i < eu.size(); i++) fe.insert({eu[i], ev[i]});
    for (uint32_t a = 0; a < N.V; a++)
        for (uint32_t b : N.adj[a])
            if (a < b) ne.insert({a, b});
    if (fe != ne) return fail("edge set", step);
    for (auto &e : ne)
        if (!F.is_edge(e.first, e.second)) return fail("is_edge", step);
    // the live label list names every tree once
    {
        std::set<uint32_t> labels_of_vertices, live(F.live_labels().begin(), F.live_labels().end());
        for (uint32_t w = 0; w < N.V; w++) labels_of_vertices.insert(F.label(w));
        if (live.size() != F.live_labels().size()) return fail("live labels repeat", step);
        if (live != labels_of_vertices) return fail("live labels", step);
    }
    // every tree: collect() returns exactly its vertices and the minimum
    std::set<uint32_t> seen_labels;
    for (uint32_t w = 0; w < N.V; w++) {
        const uint32_t l = F.label(w);
        if (!seen_labels.insert(l).second) continue;
        std::vector<uint32_t> mem;
        const uint32_t mn = F.collect(l, mem);
        std::set<uint32_t> ms(mem.begin(), mem.end());
        if (ms.size() != mem.size()) return fail("collect duplicates", step);
        uint32_t want_min = UINT32_MAX;
        size_t want_n = 0;
        for (uint32_t x = 0; x < N.V; x++)
            if (c[x] == c[w]) {
                want_n++;
                want_min = std::min(want_min, x);
                if (!ms.count(x)) return fail("collect misses a vertex", step);
            }
        if (mem.size() != want_n || mn != want_min) return fail("collect", step);
        if (F.tree_size(l) != want_n) return fail("tree size", step);
        const uint32_t r = F.tree_root(l);
        if (c[r] != c[w]) return fail("root outside its tree", step);
    }
    return 0;
}

int main(int argc, char **argv)
{
    const uint32_t V = argc > 1 ? (uint32_t)atoi(argv[1]) : 60;
    const uint64_t steps = argc > 2 ? (uint64_t)atoll(argv[2]) : 3000;
    const uint64_t seed = argc > 3 ? (uint64_t)atoll(argv[3]) : 1;
    std::mt19937_64 rng(seed);
    std::vector<uint32_t> lbl(V), par(V);
    Forest F;
    F.init(V, lbl.data(), par.data());
    Naive N(V);
    for (uint64_t s = 0; s < steps; s++) {
        const uint32_t mode = (uint32_t)(rng() % 10);
        if (mode < 6) {
            // link: sometimes to a hub (vertex 0) to grow a high-degree node,
            // sometimes along a path
            uint32_t a = (uint32_t)(rng() % V), b = (uint32_t)(rng() % V);
            if (mode == 0) a = 0;
            if (mode == 1) b = (a + 1) % V;
            if (a == b || F.same_tree(a, b)) continue;
            F.link(a, b);
            N.adj[a].insert(b);
            N.adj[b].insert(a);
        } else if (mode == 8 && (rng() & 1)) {
            // swap a tree edge for a non-tree pair whose path crosses it
            const uint32_t x = (uint32_t)(rng() % V), y = (uint32_t)(rng() % V);
            if (x == y || !F.same_tree(x, y) || F.is_edge(x, y)) continue;
            // the naive path x .. y
            std::vector<uint32_t> prev(V, UINT32_MAX);
            std::deque<uint32_t> q{x};
            prev[x] = x;
            while (!q.empty()) {
                const uint32_t a = q.front();
                q.pop_front();
                for (uint32_t b : N.adj[a])
                    if (prev[b] == UINT32_MAX) {
                        prev[b] = a;
                        q.push_back(b);
                    }
            }
            std::vector<uint32_t> path{y};
            while (path.back() != x) path.push_back(prev[path.back()]);
            const size_t k = rng() % (path.size() - 1);
            const uint32_t ea = std::min(path[k], path[k + 1]);
            const uint32_t eb = std::max(path[k], path[k + 1]);
            const uint64_t trees = F.n_trees();
            const uint32_t lx = F.label(x);
            F.swap_edge(ea, eb, x, y);
            N.adj[ea].erase(eb);
            N.adj[eb].erase(ea);
            N.adj[x].insert(y);
            N.adj[y].insert(x);
            if (F.n_trees() != trees || F.label(x) != lx || F.label(y) != lx)
                return fail("swap changed the trees", s);
        } else if (mode < 9) {
            std::vector<uint32_t> eu, ev;
            F.edges(eu, ev);
            if (eu.empty()) continue;
            const size_t k = rng() % eu.size();
            F.cut(eu[k], ev[k]);
            N.adj[eu[k]].erase(ev[k]);
            N.adj[ev[k]].erase(eu[k]);
        } else {
            // a run of removals, then one split of every tree they broke
            for (uint32_t l : F.dirty_labels()) F.clear_dirty(l);
            const std::vector<uint32_t> before = N.comp();
            std::set<uint32_t> broken;  // components (naive ids) that lost an edge
            const uint32_t run = 1 + (uint32_t)(rng() % 8);
            for (uint32_t r = 0; r < run; r++) {
                std::vector<uint32_t> eu, ev;
                F.edges(eu, ev);
                if (eu.empty()) break;
                const size_t k = rng() % eu.size();
                if (!F.is_edge(eu[k], ev[k])) return fail("is_edge during a run", s);
                F.remove_edge(eu[k], ev[k]);
                broken.insert(before[eu[k]]);
                N.adj[eu[k]].erase(ev[k]);
                N.adj[ev[k]].erase(eu[k]);
            }
            F.split_pending();
            // exactly the pieces of the broken trees are dirty
            for (uint32_t w = 0; w < V; w++)
                if (F.is_dirty(F.label(w)) != (broken.count(before[w]) != 0))
                    return fail("dirty pieces", s);
        }
        if (check(F, N, s)) return 1;
    }
    printf("ok V=%u steps=%llu\n", V, (unsigned long long)steps);
    return 0;
}
