// C ABI, context and per-batch orchestration of the sketch hot path.
//
// One batch (cupk_apply_updates / cupk_apply_updates_device):
//   1. upload the forest's label / parent arrays if they changed;
//   2. classify (validate, flag structural candidates, count tile records);
//   3. scatter: plain atomic kernel, or bin + LDS-staged kernel;
//   4. meanwhile on the host: read the flagged updates (copy stream), sort
//      them back into stream order and apply links / cuts to the forest;
//   5. replacement rounds for trees broken by cuts: segmented XOR reduction
//      of every dirty tree but the largest in one launch, verify/sample in
//      one launch, host links in ascending order of each tree's smallest
//      vertex; merged trees are reduced from their fragments' sketches in
//      the next round.
// The batch semantics match the tests' CPU oracle bit for bit: same sketch,
// same forest edges, same samples.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "context.hpp"
#include "levels.hpp"

using namespace cupk;

namespace {

// Message of the last failed cupk_sketch_init (no context survives it).
thread_local std::string g_init_error;

// SplitMix64 (Steele, Lea, Flood 2014): state += golden gamma, then the
// Stafford "Mix13" finalizer.
uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint32_t ceil_log2(uint32_t V)
{
    uint32_t L = 0;
    while ((uint64_t(1) << L) < V) L++;
    return L < 1 ? 1 : L;
}

}  // namespace

namespace cupk {

void drop_graphs(cupk_ctx *ctx);
int ensure_rel(cupk_ctx *ctx);

DevSketch dev_sketch(cupk_ctx *ctx)
{
    DevSketch d;
    d.b = ctx->d_sk;
    d.seeds = ctx->d_seeds;
    d.V = ctx->V;
    d.C = ctx->C;
    d.D = ctx->D;
    return d;
}

// Harvest finished kernel timers; with `all`, wait for every pending one.
int harvest_timers(cupk_ctx *ctx, bool all)
{
    for (int k = 0; k < kTimerRing; k++) {
        auto &t = ctx->timers[k];
        if (!t.busy) continue;
        if (all) {
            HIPCHK(hipEventSynchronize(t.t1));
        } else if (hipEventQuery(t.t1) != hipSuccess) {
            continue;
        }
        float ms_b = 0.f, ms_s = 0.f;
        HIPCHK(hipEventElapsedTime(&ms_b, t.t0, t.tb));
        HIPCHK(hipEventElapsedTime(&ms_s, t.split ? t.tc : t.tb, t.t1));
        ctx->ctr.bin_ms += ms_b;
        ctx->ctr.scatter_ms += ms_s;
        t.busy = false;
    }
    return CUPK_OK;
}

// Bring the device forest (labels, parents, packed words) up to date on
// stream st: the pages the host forest wrote since the last upload, through
// a pinned staging block, when they are fewer than a quarter of all pages;
// else the whole arrays, copied from the host forest itself (which must then
// not change until the copy is done).
int upload_forest_on(cupk_ctx *ctx, hipStream_t st)
{
    if (!ctx->forest_dev_stale) return CUPK_OK;
    ctx->forest_dev_stale = false;
    std::vector<uint32_t> &pg = ctx->up_pages;
    pg.clear();
    ctx->forest.take_pages(pg);
    if (pg.empty()) return CUPK_OK;
    const uint32_t sh = ctx->forest.page_shift(), pv = 1u << sh;
    if (pg.size() * 4 >= ctx->forest.n_pages()) {
        const size_t bytes = (size_t)ctx->V * sizeof(uint32_t);
        HIPCHK(hipMemcpyAsync(ctx->d_lbl, ctx->h_lbl, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->d_par, ctx->h_par, bytes, hipMemcpyHostToDevice, st));
        HIPCHK(launch_pack_forest(st, ctx->d_lbl, ctx->d_par, ctx->d_lp, ctx->V));
        HIPCHK(launch_block_labels(st, ctx->d_lbl, ctx->V, ctx->d_blk, nullptr, 0, 0));
        return CUPK_OK;
    }
    // the previous staging block has been copied
    if (ctx->stage_busy) {
        HIPCHK(hipEventSynchronize(ctx->ev_stage));
        ctx->stage_busy = false;
    }
    const size_t np = pg.size(), words = np * (1 + 2 * (size_t)pv);
    HIPCHK(grow(ctx->h_stage, words));
    HIPCHK(grow(ctx->d_stage, words));
    uint32_t *h = ctx->h_stage.p;
    std::copy(pg.begin(), pg.end(), h);
    uint32_t *hl = h + np, *hp = hl + np * pv;
    for (size_t i = 0; i < np; i++) {
        const size_t base = (size_t)pg[i] << sh;
        const size_t m = base < ctx->V ? std::min<size_t>(pv, ctx->V - base) : 0;
        std::memcpy(hl + i * pv, ctx->h_lbl + base, m * 4);
        std::memcpy(hp + i * pv, ctx->h_par + base, m * 4);
    }
    HIPCHK(hipMemcpyAsync(ctx->d_stage.p, h, words * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(ctx->ev_stage, st));
    ctx->stage_busy = true;
    HIPCHK(launch_forest_pages(st, ctx->d_stage.p, (uint32_t)np, sh, ctx->V, ctx->d_lbl,
                               ctx->d_par, ctx->d_lp));
    HIPCHK(launch_block_labels(st, ctx->d_lbl, ctx->V, ctx->d_blk, ctx->d_stage.p, (uint32_t)np,
                               sh));
    return CUPK_OK;
}

int upload_forest(cupk_ctx *ctx) { return upload_forest_on(ctx, ctx->s); }

// One replacement-search set: a tree of the forest, reduced either from its
// vertices or from fragment sketches of the previous round.
struct RoundSet {
    uint32_t label;
    uint32_t minv;
    uint32_t size;
    bool sampled;  // false: the left-out tree, reduced only to serve as a fragment
    uint8_t kind = 0;  // reduced from: 0 vertices, 1 fragments, 2 the other fragments
};

// Reduce k sets into d_sig[slot] (internal layout, W words per set) and
// sample them into h_res.  Vertex sets come as (members, offsets) over
// vertex ids; fragment sets as (members, offsets) over slots of
// d_sig[1-slot].  Set order: vertex sets first, then fragment sets.
int reduce_and_sample(cupk_ctx *ctx, int slot, const std::vector<uint32_t> &vmem,
                      const std::vector<uint32_t> &voff, const std::vector<uint32_t> &fmem,
                      const std::vector<uint32_t> &foff)
{
    const uint32_t kv = voff.empty() ? 0 : (uint32_t)voff.size() - 1;
    const uint32_t kf = foff.empty() ? 0 : (uint32_t)foff.size() - 1;
    const uint32_t k = kv + kf;
    if (k == 0) return CUPK_OK;
    const uint32_t W = ctx->W;
    const hipStream_t rs = ctx->rstream;
    HIPCHK(grow(ctx->d_sig[slot], (size_t)k * W));
    HIPCHK(grow(ctx->d_res, (size_t)3 * k));
    HIPCHK(grow(ctx->h_res, (size_t)3 * k));
    // work items
    std::vector<uint32_t> items;
    auto add_items = [&](const std::vector<uint32_t> &off, uint32_t set0, uint32_t mem0) {
        for (size_t j = 0; j + 1 < off.size(); j++)
            for (uint32_t b = off[j]; b < off[j + 1]; b += kRedChunk) {
                items.push_back(set0 + (uint32_t)j);
                items.push_back(mem0 + b);
                items.push_back(mem0 + std::min(off[j + 1], b + kRedChunk));
            }
    };
    add_items(voff, 0, 0);
    const size_t nvi = items.size() / 3;
    add_items(foff, kv, (uint32_t)vmem.size());
    const size_t nitems = items.size() / 3;
    // members, then the work items, in one buffer and one copy
    const size_t nmem = vmem.size() + fmem.size();
    const size_t nall = nmem + items.size();
    HIPCHK(grow(ctx->h_ridx, nall + 1));
    HIPCHK(grow(ctx->d_ridx, nall + 1));
    std::copy(vmem.begin(), vmem.end(), ctx->h_ridx.p);
    std::copy(fmem.begin(), fmem.end(), ctx->h_ridx.p + vmem.size());
    std::copy(items.begin(), items.end(), ctx->h_ridx.p + nmem);
    if (nall)
        HIPCHK(hipMemcpyAsync(ctx->d_ridx.p, ctx->h_ridx.p, nall * 4, hipMemcpyHostToDevice,
                              rs));
    const uint32_t *d_items = ctx->d_ridx.p + nmem;
    uint64_t *sig = ctx->d_sig[slot].p;
    HIPCHK(launch_zero(rs, sig, (size_t)k * W));
    if (nvi)
        HIPCHK(launch_reduce(rs, ctx->d_sk, W, ctx->d_ridx.p, d_items, (uint32_t)nvi,
                             sig));
    if (nitems > nvi)
        HIPCHK(launch_reduce(rs, ctx->d_sig[1 - slot].p, W, ctx->d_ridx.p,
                             d_items + 3 * nvi, (uint32_t)(nitems - nvi), sig));
    HIPCHK(launch_sample(rs, sig, k, ctx->V, ctx->C, ctx->D, 1, ctx->C, W, ctx->d_seeds,
                         ctx->d_res.p));
    HIPCHK(hipMemcpyAsync(ctx->h_res.p, ctx->d_res.p, (size_t)3 * k * 4, hipMemcpyDeviceToHost,
                          rs));
    HIPCHK(hipStreamSynchronize(rs));
    ctx->ctr.sets_reduced += k;
    ctx->ctr.slabs_reduced += nmem;
    return CUPK_OK;
}

// First replacement round over the pieces of the trees that pending
// removals broke, without splitting them first.
//
// Splitting relabels every piece but the largest, and when the first round
// links most pieces back together each link relabels one side again.  Here
// the pieces below removed edges are listed top-down into one buffer (their
// members are the round's vertex sets anyway); the old root's piece is
// sized by subtraction and listed only when it is sampled or carried.  The
// round decides its links on a union-find over pieces and applies them to
// the parent pointers only, and the final trees are labelled once: a tree
// holding a broken tree's unvisited piece keeps that tree's label, the
// others keep the label most of their vertices already have or take a fresh
// one, and only the vertices of listed pieces whose label changes are
// written.  The round is the regular first round (same sets, order,
// samples, links and dirty marks), so the forest is the one a split would
// give.
//
// Applies only when the broken trees are the only dirty ones.  Returns 1
// when the round ran (*done: no further round), 0 when the caller should
// split and run the regular round instead, or a negative error.
static int round_one_pieces(cupk_ctx *ctx, int slot, std::vector<RoundSet> &nsets, bool *linked,
                            bool *done)
{
    Forest &F = ctx->forest;
    if (F.pending().empty() || !F.dirty_labels().empty()) return 0;
    const double tr0 = now_ms();
    const uint32_t V = F.V();
    auto &pid = ctx->piece_id;    // vertex -> listed piece (stamped)
    auto &pst = ctx->piece_stamp;
    auto &lst = ctx->piece_label_stamp;  // broken label -> its unvisited piece (stamped)
    auto &lpc = ctx->piece_of_label;
    // stamps: ep marks this call's pieces, ep + 1 the labels it has given
    if (pid.size() != V || ctx->piece_epoch >= 0xfffffff0u) {
        pid.assign(V, 0);
        pst.assign(V, 0);
        lst.assign(V, 0);
        lpc.assign(V, 0);
        ctx->piece_epoch = 0;
    }
    ctx->piece_epoch += 2;
    const uint32_t ep = ctx->piece_epoch;
    struct Piece {
        uint32_t label, top, size, minv;
        size_t off;  // members at mem[off, off + size) once listed
        bool listed;
    };
    std::vector<Piece> P;
    std::vector<uint32_t> &mem = ctx->piece_mem;
    mem.clear();
    // one piece top-down into mem, stamping its vertices
    auto list = [&](uint32_t i) {
        Piece &p = P[i];
        const size_t b = mem.size();
        mem.push_back(p.top);
        uint32_t mn = kNone;
        for (size_t qi = b; qi < mem.size(); qi++) {
            const uint32_t x = mem[qi];
            mn = std::min(mn, x);
            pid[x] = i;
            pst[x] = ep;
            for (uint32_t y = F.first_child(x); y != kNone; y = F.next_sibling(y)) mem.push_back(y);
        }
        p.off = b;
        p.size = (uint32_t)(mem.size() - b);
        p.minv = mn;
        p.listed = true;
    };
    // Pieces of each broken tree: one per removal, listed, and the old
    // root's, sized by subtraction and listed only when needed.
    std::vector<std::pair<uint32_t, uint32_t>> pend(F.pending().begin(), F.pending().end());
    std::sort(pend.begin(), pend.end());
    for (size_t g0 = 0; g0 < pend.size();) {
        const uint32_t old = pend[g0].first;
        size_t g1 = g0;
        while (g1 < pend.size() && pend[g1].first == old) g1++;
        uint32_t listed = 0;
        for (size_t i = g0; i < g1; i++) {
            P.push_back({old, pend[i].second, 0, kNone, 0, false});
            list((uint32_t)P.size() - 1);
            listed += P.back().size;
        }
        P.push_back({old, F.tree_root(old), F.tree_size(old) - listed, kNone, 0, false});
        lst[old] = ep;
        lpc[old] = (uint32_t)P.size() - 1;
        g0 = g1;
    }
    const uint32_t np = (uint32_t)P.size();
    // One broken tree holding a large share of V: the old root's piece is
    // not listed when it is the left-out one.  Its vertices and the other
    // pieces' make up the tree as it was before the cuts, a union of whole
    // components of the graph after the batch (no other tree is dirty, and
    // every insert between two trees was linked), so no edge leaves that
    // union and the XOR of all its vertex sketches is zero (App. A.1's stream
    // contract: no insert of a present edge, no delete of an absent one).
    // The piece is carried without a sketch; the next round reduces a tree
    // that holds it from the pieces it does not hold instead.  Its smallest
    // vertex is the first vertex of the tree that no listed piece holds.
    const uint32_t rp = np - 1;
    bool virtual_root = pend.back().first == pend.front().first && !ctx->opts.exact &&
                        !ctx->levels && (uint64_t)F.tree_size(P[rp].label) * 16 >= V;
    if (virtual_root) {
        const uint32_t old = P[rp].label;
        for (uint32_t x = 0; x < V; x++)
            if (pst[x] != ep && F.label(x) == old) {
                P[rp].minv = x;
                break;
            }
    }
    // the left-out piece: largest, ties by smallest vertex (pieces in a tie
    // are listed to know their smallest vertex)
    uint32_t maxs = 0;
    uint64_t total = 0;
    for (const Piece &p : P) {
        maxs = std::max(maxs, p.size);
        total += p.size;
    }
    uint32_t nmax = 0;
    for (const Piece &p : P) nmax += p.size == maxs;
    if (nmax > 1 && !virtual_root)
        for (uint32_t i = 0; i < np; i++)
            if (P[i].size == maxs && !P[i].listed) list(i);
    uint32_t skip = kNone;
    for (uint32_t i = 0; i < np; i++)
        if (P[i].size == maxs && (skip == kNone || P[i].minv < P[skip].minv)) skip = i;
    virtual_root = virtual_root && skip == rp;
    // every other piece is sampled: list the unvisited ones; the left-out one
    // is listed too (and carried, so that the next round can be built from
    // this round's sets) when it is no larger than the others together
    for (uint32_t i = 0; i < np; i++)
        if (i != skip && !P[i].listed) list(i);
    if (!P[skip].listed && !virtual_root && 2 * (uint64_t)P[skip].size <= total) list(skip);
    const bool carry = P[skip].listed || virtual_root;
    // sets in ascending order of smallest vertex, the carried left-out last
    std::vector<uint32_t> gord;
    for (uint32_t i = 0; i < np; i++)
        if (i != skip) gord.push_back(i);
    std::sort(gord.begin(), gord.end(), [&](uint32_t a, uint32_t b) { return P[a].minv < P[b].minv; });
    if (carry) gord.push_back(skip);
    std::vector<uint32_t> vmem, voff{0}, none;
    vmem.reserve(mem.size());
    nsets.clear();
    for (uint32_t i : gord) {
        nsets.push_back({P[i].label, P[i].minv, P[i].size, i != skip});
        if (P[i].listed)
            vmem.insert(vmem.end(), mem.begin() + P[i].off, mem.begin() + P[i].off + P[i].size);
        voff.push_back((uint32_t)vmem.size());
    }
    // the carried old root's piece is last: a set without a sketch
    ctx->virtual_set = virtual_root ? (uint32_t)nsets.size() - 1 : kNone;
    if (virtual_root) ctx->ctr.pieces_sketchless++;
    ctx->ctr.rounds++;
    const double tr1 = now_ms();
    int rc = reduce_and_sample(ctx, slot, vmem, voff, none, none);
    if (rc != CUPK_OK) return rc;
    const double tr2 = now_ms();
    const int32_t *res = ctx->h_res.p;
    const size_t k = nsets.size();
    // the piece of a vertex: listed (stamped), or its broken tree's unvisited one
    auto piece_of = [&](uint32_t v) -> uint32_t {
        if (pst[v] == ep) return pid[v];
        const uint32_t l = F.label(v);
        return lst[l] == ep ? lpc[l] : kNone;
    };
    for (size_t i = 0; i < k; i++) {
        if (!nsets[i].sampled || res[3 * i] != CUPK_OK) continue;
        if (piece_of((uint32_t)res[3 * i + 1]) == kNone ||
            piece_of((uint32_t)res[3 * i + 2]) == kNone) {
            ctx->ctr.rounds--;  // an edge out of the broken trees: the regular round
            return 0;           // runs instead (nothing has been changed)
        }
    }
    if (ctx->trace)
        fprintf(stderr,
                "cupk   pieces=%u sets=%zu left_out=%u vmembers=%zu search=%.3f gpu=%.3f ms\n",
                np, k, P[skip].size, vmem.size(), tr1 - tr0, tr2 - tr1);
    // links on a union-find over pieces (sets are already in ascending order
    // of smallest vertex); parent pointers follow at once
    std::vector<uint32_t> up(np), groot(np), gsize(np);
    std::vector<uint8_t> gclean(np, 0);
    for (uint32_t i = 0; i < np; i++) {
        up[i] = i;
        groot[i] = P[i].top;
        gsize[i] = P[i].size;
    }
    auto find = [&](uint32_t a) {
        while (up[a] != a) a = up[a] = up[up[a]];
        return a;
    };
    const double tl0 = now_ms();
    bool lk = false, failed = false;
    uint32_t nlinks = 0;
    for (size_t i = 0; i < k; i++) {
        if (!nsets[i].sampled || res[3 * i] != CUPK_OK) continue;
        const uint32_t x = (uint32_t)res[3 * i + 1], y = (uint32_t)res[3 * i + 2];
        const uint32_t rx = find(piece_of(x)), ry = find(piece_of(y));
        if (rx == ry) continue;
        // the endpoint with the shorter path to its root is re-rooted and
        // hangs below the other: the other tree's root is the new root
        const uint32_t nr = F.link_structural_short(x, y) ? groot[ry] : groot[rx];
        const uint32_t r = gsize[rx] > gsize[ry] ? rx : ry, o = r == rx ? ry : rx;
        up[o] = r;
        groot[r] = nr;
        gsize[r] = gsize[rx] + gsize[ry];
        ctx->ctr.links++;
        nlinks++;
        lk = true;
    }
    if (ctx->trace) fprintf(stderr, "cupk   links=%u in %.3f ms\n", nlinks, now_ms() - tl0);
    for (size_t i = 0; i < k; i++) {
        if (!nsets[i].sampled) continue;
        const int st = res[3 * i];
        if (st == CUPK_EMPTY) {
            // a whole component: clean, unless it was merged this round
            const uint32_t r = find(gord[i]);
            if (gsize[r] == nsets[i].size) gclean[r] = 1;
        } else if (st == CUPK_SAMPLE_FAILED) {
            ctx->ctr.sample_failed++;
            failed = true;
            if (ctx->trace)
                fprintf(stderr, "cupk   failed: first round set %zu of %zu size %u minv %u\n", i,
                        k, nsets[i].size, nsets[i].minv);
        }
    }
    if (!lk) {
        if (!failed) gclean[find(skip)] = 1;
        *done = true;
    }
    // Final labels.  A broken tree's unvisited piece cannot be relabelled:
    // its tree keeps that label.  Other trees keep the old label with the
    // most of their listed vertices when no other tree has it, else take a
    // fresh one.
    std::vector<uint32_t> glabel(np, kNone), weight(np, 0), best(np, kNone);
    std::vector<uint32_t> roots;
    for (uint32_t i = 0; i < np; i++) {
        const uint32_t r = find(i);
        if (r == i) roots.push_back(r);
    }
    std::vector<uint32_t> used;  // labels given to trees (stamped via lst = ep + 1)
    auto take = [&](uint32_t r, uint32_t l) {
        glabel[r] = l;
        used.push_back(l);
        lst[l] = ep + 1;  // marks the label as given (no piece lookup needs it any more)
    };
    for (uint32_t i = 0; i < np; i++)
        if (!P[i].listed) {
            const uint32_t r = find(i);
            if (glabel[r] == kNone) take(r, P[i].label);
            else return ctx->invalid("two unvisited pieces in one tree");  // cannot happen
        }
    {
        // per tree, the old label of its largest listed share
        std::vector<std::pair<uint64_t, uint32_t>> share;  // ((root << 32) | label, size)
        for (uint32_t i = 0; i < np; i++)
            if (P[i].listed) share.push_back({(uint64_t)find(i) << 32 | P[i].label, P[i].size});
        std::sort(share.begin(), share.end());
        std::vector<std::pair<uint32_t, uint32_t>> cand;  // (weight, root)
        for (size_t a = 0; a < share.size();) {
            size_t b = a;
            uint32_t w = 0;
            while (b < share.size() && share[b].first == share[a].first) w += share[b++].second;
            const uint32_t r = (uint32_t)(share[a].first >> 32), l = (uint32_t)share[a].first;
            if (glabel[r] == kNone && w > weight[r]) {
                weight[r] = w;
                best[r] = l;
            }
            a = b;
        }
        for (uint32_t r : roots)
            if (glabel[r] == kNone) cand.push_back({weight[r], r});
        std::sort(cand.begin(), cand.end(), std::greater<>());
        for (auto &c : cand) {
            const uint32_t r = c.second, l = best[r];
            if (lst[l] != ep + 1) take(r, l);
        }
        for (uint32_t r : roots)
            if (glabel[r] == kNone) take(r, F.settle_take_label());
    }
    for (uint32_t i = 0; i < np; i++) {
        const uint32_t l = glabel[find(i)];
        if (P[i].listed && P[i].label != l) F.settle_relabel(mem.data() + P[i].off, P[i].size, l);
    }
    // broken trees' labels that no final tree kept are given back
    for (size_t g = 0; g < pend.size(); g++) {
        const uint32_t l = pend[g].first;
        if (lst[l] == ep) {
            lst[l] = ep + 1;
            F.settle_drop_label(l);
        }
    }
    for (uint32_t r : roots) F.settle_tree(glabel[r], groot[r], gsize[r], gclean[r] == 0);
    F.settle_done();
    if (lk) *linked = true;
    return 1;
}

// Replacement rounds over the dirty trees.
//
// Clean trees are whole components, so every edge that leaves a dirty tree
// ends in another dirty tree.  Each round therefore leaves out the largest
// dirty tree (ties: smallest vertex id) and samples all the others, each
// reduced from its vertices or, when it is a union of trees sampled in the
// previous round, from their sketches; links go in ascending order of each
// tree's smallest vertex.  A tree that samples EMPTY is a whole component;
// so is a lone dirty tree, and so is the left-out tree once a round links
// nothing and no sample failed.  Trees whose sample failed stay dirty.
int run_rounds(cupk_ctx *ctx)
{
    Forest &F = ctx->forest;
    std::vector<RoundSet> sets;  // sets of the previous round, in d_sig order
    std::vector<uint32_t> vmem, voff, fmem, foff;
    struct Group {
        uint32_t label, minv, size;
        std::vector<uint32_t> frags;  // previous-round sets forming the tree
        bool from_frags, have_minv;
        bool complemented = false;    // frags are the previous-round sets it does not hold
    };
    int slot = 0;
    bool linked_any = false;
    bool done = false;
    ctx->virtual_set = kNone;
    const int r1 = ctx->opts.split_rounds ? 0 : round_one_pieces(ctx, slot, sets, &linked_any, &done);
    if (r1 < 0) return r1;
    if (r1 == 1) {
        slot = 1 - slot;
    } else {
        sets.clear();
        ctx->virtual_set = kNone;
        const double ts0 = now_ms();
        F.split_pending();
        if (ctx->trace) fprintf(stderr, "cupk   split=%.3f ms\n", now_ms() - ts0);
    }
    double tr0 = now_ms();
    for (; !done;) {
        const std::vector<uint32_t> labels = F.dirty_labels();
        if (labels.empty()) break;
        if (labels.size() == 1) {
            F.clear_dirty(labels[0]);
            break;
        }
        // previous-round sets grouped by the tree they now belong to
        std::vector<std::pair<uint32_t, uint32_t>> frag;  // (label, set index)
        frag.reserve(sets.size());
        for (size_t i = 0; i < sets.size(); i++)
            frag.push_back({F.label(sets[i].minv), (uint32_t)i});
        std::sort(frag.begin(), frag.end());
        std::vector<Group> groups(labels.size());
        uint32_t maxs = 0;
        for (size_t gi = 0; gi < labels.size(); gi++) {
            Group &g = groups[gi];
            g.label = labels[gi];
            g.size = F.tree_size(g.label);
            g.minv = 0xffffffffu;
            uint32_t tot = 0;
            auto it = std::lower_bound(frag.begin(), frag.end(), std::make_pair(g.label, 0u));
            for (; it != frag.end() && it->first == g.label; ++it) {
                g.frags.push_back(it->second);
                tot += sets[it->second].size;
                g.minv = std::min(g.minv, sets[it->second].minv);
            }
            g.from_frags = g.have_minv = (tot == g.size);
            if (!g.from_frags) g.frags.clear();
            maxs = std::max(maxs, g.size);
        }
        // A tree holding the previous round's set without a sketch (the old
        // root's piece of the one broken tree) is reduced from all the other
        // previous-round sets, the pieces it does not hold: the pieces
        // together XOR to zero.
        const uint32_t vs = ctx->virtual_set;
        ctx->virtual_set = kNone;
        if (vs != kNone)
            for (Group &g : groups)
                if (g.from_frags && std::find(g.frags.begin(), g.frags.end(), vs) != g.frags.end()) {
                    std::vector<uint8_t> in(sets.size(), 0);
                    for (uint32_t f : g.frags) in[f] = 1;
                    g.frags.clear();
                    for (uint32_t i = 0; i < sets.size(); i++)
                        if (!in[i]) g.frags.push_back(i);
                    g.complemented = true;
                    ctx->ctr.sets_complemented++;
                }
        // the left-out tree: largest, ties broken by smallest vertex id
        std::vector<std::vector<uint32_t>> lists(groups.size());
        size_t skip = groups.size();
        for (size_t gi = 0; gi < groups.size(); gi++) {
            if (groups[gi].size != maxs) continue;
            if (skip == groups.size()) {
                skip = gi;
                continue;
            }
            for (size_t t : {skip, gi})
                if (!groups[t].have_minv) {
                    groups[t].minv = F.collect(groups[t].label, lists[t]);
                    groups[t].have_minv = true;
                }
            if (groups[gi].minv < groups[skip].minv) skip = gi;
        }
        // members of the trees reduced from their vertices: one pass over
        // the labels when these trees hold a large share of all vertices
        // (members then come in ascending order), else a search of each
        size_t need = 0;
        for (size_t gi = 0; gi < groups.size(); gi++)
            if (gi != skip && !groups[gi].from_frags && lists[gi].empty()) need += groups[gi].size;
        // The left-out tree is not sampled, but when it merges with sampled
        // trees the merged tree can be reduced from fragments only if its
        // sketch is known too.  It is carried along (reduced, not sampled)
        // when that is cheap: from fragments, or in the same pass over the
        // labels when it is no larger than the trees collected anyway.
        bool carry = groups[skip].from_frags || !lists[skip].empty();
        if (need * 4 >= F.V()) {
            std::vector<int32_t> &gmap = ctx->round_gmap;
            if (gmap.size() != F.V()) gmap.assign(F.V(), -1);
            if (!carry && lists[skip].empty() && groups[skip].size <= need) carry = true;
            for (size_t gi = 0; gi < groups.size(); gi++)
                if ((gi != skip || carry) && !groups[gi].from_frags && lists[gi].empty()) {
                    gmap[groups[gi].label] = (int32_t)gi;
                    lists[gi].reserve(groups[gi].size);
                }
            for (uint32_t w = 0; w < F.V(); w++) {
                const int32_t g = gmap[F.label(w)];
                if (g >= 0) lists[g].push_back(w);
            }
            for (size_t gi = 0; gi < groups.size(); gi++)
                if (gmap[groups[gi].label] >= 0) {
                    gmap[groups[gi].label] = -1;
                    groups[gi].minv = lists[gi][0];
                }
        } else {
            // one search per tree, the trees split over the pool when their
            // members are many (each writes its own list)
            std::vector<size_t> todo;
            for (size_t gi = 0; gi < groups.size(); gi++)
                if (gi != skip && !groups[gi].from_frags && lists[gi].empty()) todo.push_back(gi);
            auto one = [&](size_t i, unsigned) {
                Group &g = groups[todo[i]];
                g.minv = F.collect(g.label, lists[todo[i]]);
            };
            if (F.pool() && todo.size() > 1 && need >= F.parallel_work())
                F.pool()->run(todo.size(), one);
            else
                for (size_t i = 0; i < todo.size(); i++) one(i, 0);
        }
        std::vector<size_t> gord;
        gord.reserve(groups.size());
        for (size_t gi = 0; gi < groups.size(); gi++)
            if (gi != skip) gord.push_back(gi);
        std::sort(gord.begin(), gord.end(),
                  [&](size_t a, size_t b) { return groups[a].minv < groups[b].minv; });
        // vertex-reduced sets first, then fragment sets (see
        // reduce_and_sample); each group in ascending smallest-vertex order
        std::vector<RoundSet> nsets;
        vmem.clear();
        voff.clear();
        fmem.clear();
        foff.clear();
        voff.push_back(0);
        foff.push_back(0);
        if (carry) gord.push_back(skip);
        for (size_t gi : gord)
            if (!groups[gi].from_frags) {
                nsets.push_back({groups[gi].label, groups[gi].minv, groups[gi].size, gi != skip});
                vmem.insert(vmem.end(), lists[gi].begin(), lists[gi].end());
                voff.push_back((uint32_t)vmem.size());
            }
        for (size_t gi : gord)
            if (groups[gi].from_frags) {
                nsets.push_back({groups[gi].label, groups[gi].minv, groups[gi].size, gi != skip,
                                 (uint8_t)(groups[gi].complemented ? 2 : 1)});
                fmem.insert(fmem.end(), groups[gi].frags.begin(), groups[gi].frags.end());
                foff.push_back((uint32_t)fmem.size());
            }
        if (voff.size() == 1) voff.clear();
        if (foff.size() == 1) foff.clear();
        sets.swap(nsets);
        const uint32_t skip_label = groups[skip].label;

        ctx->ctr.rounds++;
        const double tr1 = now_ms();
        int rc = reduce_and_sample(ctx, slot, vmem, voff, fmem, foff);
        if (rc != CUPK_OK) return rc;
        const double tr2 = now_ms();
        if (ctx->trace)
            fprintf(stderr,
                    "cupk   round sets=%zu left_out=%u vmembers=%zu fmembers=%zu prep=%.3f "
                    "gpu=%.3f ms\n",
                    sets.size(), groups[skip].size, vmem.size(), fmem.size(), tr1 - tr0,
                    tr2 - tr1);
        const int32_t *res = ctx->h_res.p;
        const size_t k = sets.size();
        std::vector<size_t> ord(k);
        for (size_t i = 0; i < k; i++) ord[i] = i;
        std::sort(ord.begin(), ord.end(),
                  [&](size_t a, size_t b) { return sets[a].minv < sets[b].minv; });
        bool linked = false, failed = false;
        const double tl0 = now_ms();
        // the sampled edges, in ascending order of their tree's smallest
        // vertex, link when their endpoints are in different trees at their
        // turn (each merged tree relabelled once)
        std::vector<std::pair<uint32_t, uint32_t>> cand;
        for (size_t i : ord) {
            if (!sets[i].sampled || res[3 * i] != CUPK_OK) continue;
            cand.push_back({(uint32_t)res[3 * i + 1], (uint32_t)res[3 * i + 2]});
        }
        const uint32_t nlinks = (uint32_t)F.link_many(cand, ctx->cand_linked);
        ctx->ctr.links += nlinks;
        linked = nlinks > 0;
        if (ctx->trace) fprintf(stderr, "cupk   links=%u in %.3f ms\n", nlinks, now_ms() - tl0);
        for (size_t i = 0; i < k; i++) {
            if (!sets[i].sampled) continue;
            const int st = res[3 * i];
            if (st == CUPK_EMPTY) {
                // a whole component: clean, unless it was merged this round
                const uint32_t l = F.label(sets[i].minv);
                if (l == sets[i].label && F.tree_size(l) == sets[i].size) F.clear_dirty(l);
            } else if (st == CUPK_SAMPLE_FAILED) {
                ctx->ctr.sample_failed++;
                failed = true;
                if (ctx->trace)
                    fprintf(stderr, "cupk   failed: round %llu set %zu of %zu kind %u size %u minv %u\n",
                            (unsigned long long)ctx->ctr.rounds, i, k, (unsigned)sets[i].kind,
                            sets[i].size, sets[i].minv);
            }
        }
        if (!linked) {
            if (!failed) F.clear_dirty(skip_label);
            break;
        }
        linked_any = true;
        slot = 1 - slot;
        tr0 = now_ms();
    }
    if (linked_any) ctx->forest_dev_stale = true;
    return CUPK_OK;
}

// Apply flagged updates [k0, k1) of one batch (host copies, stream order) to
// the forest.  Returns true when the rest of the list cannot change the
// forest: without flagged deletes nothing splits a tree during the walk, so
// once one tree is left no later insert can link.
bool apply_flags(cupk_ctx *ctx, const uint64_t *upd, uint32_t k0, uint32_t k1, bool all_inserts)
{
    Forest &F = ctx->forest;
    if (ctx->levels) {
        // the hierarchy links only through its restoration passes
        for (uint32_t k = k0; k < k1; k++) {
            const uint64_t p = upd[k];
            if ((p >> 63) == 0) continue;
            uint32_t a = (uint32_t)p, b = (uint32_t)(p >> 32) & 0x7fffffffu;
            if (a > b) std::swap(a, b);
            levels_delete(ctx, a, b);
        }
        return false;
    }
    // Contract only runs where an insert follows a delete: without one, the
    // one-by-one walk removes edges in O(1) each and splits once at the end.
    bool insert_after_delete = false;
    if (!all_inserts && !ctx->opts.walk_plain) {
        bool seen_delete = false;
        for (uint32_t k = k0; k < k1 && !insert_after_delete; k++) {
            if (upd[k] >> 63)
                seen_delete = true;
            else
                insert_after_delete = seen_delete;
        }
    }
    if (insert_after_delete) {
        uint64_t nl = 0, nc = 0;
        bool changed = false;
        if (ctx->contract.run(F, upd, k0, k1, &nl, &nc, &changed)) {
            if (ctx->trace)
                fprintf(stderr,
                        "cupk   contract k=%u pieces=%u links=%llu cuts=%llu: pieces %.3f "
                        "replay %.3f removals %.3f settle %.3f ms\n",
                        k1 - k0, ctx->contract.last_pieces, (unsigned long long)nl,
                        (unsigned long long)nc, ctx->contract.last_ms[0],
                        ctx->contract.last_ms[1], ctx->contract.last_ms[2],
                        ctx->contract.last_ms[3]);
            ctx->ctr.links += nl;
            ctx->ctr.cuts += nc;
            ctx->ctr.walks_contracted++;
            if (changed) ctx->forest_dev_stale = true;
            return false;
        }
        ctx->ctr.walks_fallback++;
    }
    bool done = false;
    for (uint32_t k = k0; k < k1; k++) {
        if (all_inserts && F.n_trees() == 1) {
            done = true;
            break;
        }
        const uint64_t p = upd[k];
        uint32_t a = (uint32_t)p, b = (uint32_t)(p >> 32) & 0x7fffffffu;
        const bool del = (p >> 63) != 0;
        if (a > b) std::swap(a, b);
        if (!del) {
            // labels are exact again before an insert looks at them
            if (F.has_pending()) F.split_pending();
            if (!F.same_tree(a, b)) {
                F.link(a, b);
                ctx->ctr.links++;
                ctx->forest_dev_stale = true;
            }
        } else if (F.is_edge(a, b)) {
            // a run of cuts removes its edges now and splits the trees once
            // (before the next insert or the rounds)
            F.remove_edge(a, b);
            ctx->ctr.cuts++;
            ctx->forest_dev_stale = true;
        }
    }
    return done || (all_inserts && F.n_trees() == 1);
}

// Size every per-batch buffer for one capacity (updates per batch); growth
// is geometric.  Captured graphs embed buffer pointers and are dropped.
int ensure_batch_buffers(cupk_ctx *ctx, size_t n)
{
    if (n <= ctx->batch_cap) return CUPK_OK;
    const size_t cap = std::max(n, ctx->batch_cap + ctx->batch_cap / 2);
    drop_graphs(ctx);
    const size_t nb = (cap + 4095) / 4096;
    HIPCHK(grow(ctx->d_fupd, nb * 4096));
    HIPCHK(grow(ctx->d_fcnt, nb + 1));
    HIPCHK(grow(ctx->d_fdel, nb + 1));
    HIPCHK(grow(ctx->d_foff, nb + 1));
    HIPCHK(grow(ctx->d_oupd, cap));
    HIPCHK(grow(ctx->h_fupd, cap, hipHostMallocCoherent));
    if (ctx->opts.exact) {
        HIPCHK(grow(ctx->d_fpos, nb * 4096));
        HIPCHK(grow(ctx->d_opos, cap));
        HIPCHK(grow(ctx->h_fpos, cap));
    }
    if (ctx->opts.scatter_mode == CUPK_SCATTER_STAGED) {
        HIPCHK(grow(ctx->d_bins, 2 * cap));
        if (ctx->fshift) HIPCHK(grow(ctx->d_bins1, 2 * cap));
        const size_t icap = 2 * cap / ctx->chunk + ctx->ntiles + 1;
        HIPCHK(grow(ctx->d_items, 2 * icap));
    }
    ctx->batch_cap = cap;
    return ensure_rel(ctx);
}

// Block starts inside the tile bins (one word per classify block and tile)
// for the batch capacity and geometry in force, when they fit a modest
// buffer; otherwise the fill reserves its ranges with atomics.
constexpr size_t kRelMaxWords = (size_t)1 << 25;
static size_t rel_words(cupk_ctx *ctx, size_t n)
{
    // the fill that uses them bins by coarse bin in two-level mode
    const uint32_t nt = ctx->fshift ? ctx->ncoarse : ctx->ntiles;
    if (ctx->opts.scatter_mode != CUPK_SCATTER_STAGED || ctx->opts.fill_reserve ||
        nt > kRelMaxTiles)
        return 0;
    const size_t w = (size_t)classify_blocks((uint32_t)std::min<size_t>(n, kMaxBatchPerLaunch)) *
                     nt;
    return w <= kRelMaxWords ? w : 0;
}

int ensure_rel(cupk_ctx *ctx)
{
    const size_t w = rel_words(ctx, ctx->batch_cap);
    if (w) HIPCHK(grow(ctx->d_trel, w));
    return CUPK_OK;
}

static uint32_t *rel_ptr(cupk_ctx *ctx, uint32_t grid_n)
{
    const size_t w = rel_words(ctx, grid_n);
    return w && w <= ctx->d_trel.cap ? ctx->d_trel.p : nullptr;
}

void drop_graphs(cupk_ctx *ctx)
{
    for (hipGraphExec_t *g : {&ctx->gx_cls, &ctx->gx_bin, &ctx->gx_tile, &ctx->gx_all})
        if (*g) {
            (void)hipGraphExecDestroy(*g);
            *g = nullptr;
        }
    ctx->graph_cap = 0;
}

StagedParams staged_params(cupk_ctx *ctx, uint32_t grid_n)
{
    StagedParams p;
    p.tile_shift = ctx->tile_shift;
    p.rows = ctx->rows;
    p.layout = ctx->layout == CUPK_LAYOUT_PAIR ? kLayoutPair : kLayoutRecord;
    p.ntiles = ctx->ntiles;
    p.chunk = ctx->chunk;
    p.items_cap = (uint32_t)(2 * (size_t)grid_n / ctx->chunk + ctx->ntiles + 1);
    p.grid = ctx->tile_grid;
    return p;
}

// Device work of one batch, in three parts.  Grids are sized for grid_n;
// the kernels read the batch from ctx->cur_desc (by value) or, while graphs
// are captured, from ctx->d_desc.  The header is left zeroed by the previous
// batch's scatter (and at init).
static const BatchDesc *desc_ptr(cupk_ctx *ctx) { return ctx->capturing ? ctx->d_desc : nullptr; }

// Where the scan after classification finds the flag regions (and puts a
// short flag list: straight into host memory, except in exact mode, which
// also needs the flags' positions).
static FlagInline flag_inline(cupk_ctx *ctx, uint32_t grid_n)
{
    FlagInline fi = {};
    fi.fupd = ctx->d_fupd.p;
    fi.fcnt = ctx->d_fcnt.p;
    fi.fdel = ctx->d_fdel.p;
    fi.nb = classify_blocks(grid_n);
    fi.hflags = ctx->opts.exact ? nullptr : ctx->h_fupd.p;
    return fi;
}

// tiles_only: leave the flags unpublished (an overlapped pass checks them
// again against the forest after the previous batch's rounds).
int enqueue_classify(cupk_ctx *ctx, hipStream_t s, uint32_t grid_n, bool tiles_only = false)
{
    const bool staged = ctx->opts.scatter_mode == CUPK_SCATTER_STAGED;
    ScanArgs sa = {};
    if (staged) {
        sa.off = ctx->d_toff.p;
        sa.cur = ctx->d_tcur.p;
        sa.items = ctx->d_items.p;
        sa.nitems = ctx->d_nitems;
        sa.chunk = ctx->chunk;
        sa.items_cap = staged_params(ctx, grid_n).items_cap;
        sa.groups = 1;
        if (ctx->ntiles > kScanOneBlockTiles) sa.sums = ctx->d_tsum.p;
    }
    uint32_t *rel = staged ? rel_ptr(ctx, grid_n) : nullptr;
    uint32_t *cnt = staged ? ctx->d_tcnt.p : nullptr;
    uint32_t cls_shift = ctx->tile_shift, cls_tiles = ctx->ntiles;
    if (staged && ctx->fshift) {
        // two-level: the classify kernel and its scan work on coarse bins
        // (the tile counts come later, from the coarse-binned records)
        sa = {};
        sa.off = ctx->d_coff.p;
        sa.cur = ctx->d_ccur.p;
        sa.items = ctx->d_csink.p;
        sa.nitems = ctx->d_csink.p + 2;
        sa.chunk = 1u << 30;
        sa.items_cap = 0;
        sa.groups = 1;
        cnt = ctx->d_ccnt.p;
        cls_shift = ctx->tile_shift + ctx->fshift;
        cls_tiles = ctx->ncoarse;
    }
    if (rel) {
        sa.groups = kCntGroups;
        sa.goff = ctx->fshift ? ctx->d_cgoff.p : ctx->d_tgoff.p;
    }
    FlagInline fi = flag_inline(ctx, grid_n);
    fi.tiles_only = tiles_only ? 1u : 0u;
    HIPCHK(launch_classify(s, desc_ptr(ctx), ctx->cur_desc, grid_n, ctx->V, ctx->d_lp,
                           ctx->d_blk, ctx->d_hdr, ctx->d_fupd.p,
                           ctx->opts.exact ? ctx->d_fpos.p : nullptr, ctx->d_fcnt.p,
                           cnt, cls_shift, cls_tiles, sa, ctx->h_hdr, fi, rel));
    return CUPK_OK;
}

int enqueue_bin(cupk_ctx *ctx, hipStream_t s, uint32_t grid_n)
{
    if (ctx->opts.scatter_mode != CUPK_SCATTER_STAGED) return CUPK_OK;
    const StagedParams p = staged_params(ctx, grid_n);
    if (!ctx->fshift) {
        HIPCHK(launch_bin(s, desc_ptr(ctx), ctx->cur_desc, grid_n, dev_sketch(ctx), ctx->d_hdr, p,
                          ctx->d_tcur.p, ctx->d_bins.p, ctx->d_tgoff.p, rel_ptr(ctx, grid_n)));
        return CUPK_OK;
    }
    // two-level: records by coarse bin into bins1, then by tile into bins
    StagedParams pc = p;
    pc.tile_shift = ctx->tile_shift + ctx->fshift;
    pc.ntiles = ctx->ncoarse;
    HIPCHK(launch_bin(s, desc_ptr(ctx), ctx->cur_desc, grid_n, dev_sketch(ctx), ctx->d_hdr, pc,
                      ctx->d_ccur.p, ctx->d_bins1.p, ctx->d_cgoff.p, rel_ptr(ctx, grid_n)));
    ScanArgs sa = {};
    sa.off = ctx->d_toff.p;
    sa.cur = ctx->d_tcur.p;
    sa.items = ctx->d_items.p;
    sa.nitems = ctx->d_nitems;
    sa.chunk = ctx->chunk;
    sa.items_cap = p.items_cap;
    sa.groups = 1;
    sa.sums = ctx->d_tsum.p;
    HIPCHK(launch_fine(s, grid_n, ctx->d_hdr, ctx->d_bins1.p, ctx->d_coff.p + ctx->ncoarse,
                       ctx->tile_shift, ctx->fshift, ctx->ntiles, ctx->d_tcnt.p, sa,
                       ctx->d_bins.p));
    return CUPK_OK;
}

// count: the staged kernel adds the buckets it changes to ctx->d_touched
// (timed passes).
int enqueue_tile(cupk_ctx *ctx, hipStream_t s, uint32_t grid_n, bool count)
{
    if (ctx->opts.scatter_mode == CUPK_SCATTER_STAGED) {
        HIPCHK(launch_tile(s, dev_sketch(ctx), ctx->d_hdr, staged_params(ctx, grid_n),
                           ctx->d_toff.p, ctx->d_bins.p, ctx->d_items.p, ctx->d_nitems,
                           count ? ctx->d_touched : nullptr));
    } else {
        HIPCHK(launch_scatter_atomic(s, desc_ptr(ctx), ctx->cur_desc, grid_n, dev_sketch(ctx),
                                     ctx->d_hdr));
    }
    return CUPK_OK;
}

// Capture the three parts as graphs sized for the current batch capacity.
// Captured on an internal stream; replayed on the context's stream.
int capture_graphs(cupk_ctx *ctx)
{
    drop_graphs(ctx);
    if (!ctx->gs) HIPCHK(hipStreamCreateWithFlags(&ctx->gs, hipStreamNonBlocking));
    const uint32_t cap = (uint32_t)std::min<size_t>(ctx->batch_cap, kMaxBatchPerLaunch);
    // parts 0..2: classify, bin, scatter (launched apart when the pass is
    // timed, with events between them); part 3: all three in one graph (the
    // host needs nothing between them: the header reaches it by itself)
    for (int part = 0; part < 4; part++) {
        HIPCHK(hipStreamBeginCapture(ctx->gs, hipStreamCaptureModeThreadLocal));
        ctx->capturing = true;
        int rc = CUPK_OK;
        if (part == 0 || part == 3) rc = enqueue_classify(ctx, ctx->gs, cap);
        if (rc == CUPK_OK && (part == 1 || part == 3)) rc = enqueue_bin(ctx, ctx->gs, cap);
        if (rc == CUPK_OK && (part == 2 || part == 3)) rc = enqueue_tile(ctx, ctx->gs, cap, false);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->gs, &g);
        if (rc != CUPK_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return ctx->fail(e, "hipStreamEndCapture", __LINE__);
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return ctx->fail(e, "hipGraphInstantiate", __LINE__);
        (part == 0 ? ctx->gx_cls : part == 1 ? ctx->gx_bin : part == 2 ? ctx->gx_tile : ctx->gx_all) = x;
    }
    ctx->graph_cap = cap;
    return CUPK_OK;
}

// Device work of one pass over the updates [0, n) at d_upd: forest upload,
// batch descriptor, classification (with the header copy) and scatter.  A
// revert pass applies updates again to undo a speculative scatter (XOR
// toggles back); it leaves the forest mirror alone and its flags are not
// read.
// The timer slot of the pass being enqueued (every time_kernels-th pass),
// or null.
static int take_timer(cupk_ctx *ctx, uint32_t n, cupk_ctx::TimerSlot **out)
{
    *out = nullptr;
    if (!ctx->opts.time_kernels || ctx->ctr.scatter_launches % ctx->opts.time_kernels != 0)
        return CUPK_OK;
    ctx->ctr.timed_launches++;
    ctx->ctr.timed_updates += n;
    cupk_ctx::TimerSlot *ts = &ctx->timers[ctx->timer_head];
    ctx->timer_head = (ctx->timer_head + 1) % kTimerRing;
    if (ts->busy) {
        HIPCHK(hipEventSynchronize(ts->t1));
        const int rc = harvest_timers(ctx, false);
        if (rc != CUPK_OK) return rc;
    }
    ts->split = false;
    *out = ts;
    return CUPK_OK;
}

// An overlapped pass in two halves.  Front: classify the batch against the
// forest on the device (which the caller uploaded after the previous
// batch's flag walk) without publishing its flags, and bin it.  Back (after
// the previous batch's rounds): upload the forest as the rounds left it,
// keep the flags that forest still gives, publish them with the header,
// and scatter.
static int enqueue_split_front(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n)
{
    int rc = harvest_timers(ctx, false);
    if (rc != CUPK_OK) return rc;
    ctx->small_pass = false;
    ctx->cur_desc.upd = d_upd;
    ctx->cur_desc.n = n;
    cupk_ctx::TimerSlot *ts = nullptr;
    rc = take_timer(ctx, n, &ts);
    if (rc != CUPK_OK) return rc;
    rc = enqueue_classify(ctx, ctx->s, n, true);
    if (rc != CUPK_OK) return rc;
    // the last reader of the uploaded forest until the back half
    HIPCHK(hipEventRecord(ctx->ev_cls, ctx->s));
    if (ts) HIPCHK(hipEventRecord(ts->t0, ctx->s));
    rc = enqueue_bin(ctx, ctx->s, n);
    if (rc != CUPK_OK) return rc;
    if (ts) HIPCHK(hipEventRecord(ts->tb, ctx->s));
    ctx->split_ts = ts;
    return CUPK_OK;
}

static int enqueue_split_back(cupk_ctx *ctx, uint32_t n)
{
    // the forest as the rounds left it, uploaded on the copy stream (idle
    // now) once the classification has read the previous upload, so that it
    // overlaps the binning still running on the main stream
    const bool changed = ctx->forest_dev_stale;
    if (changed) {
        HIPCHK(hipStreamWaitEvent(ctx->cs, ctx->ev_cls, 0));
        const int rc = upload_forest_on(ctx, ctx->cs);
        if (rc != CUPK_OK) return rc;
        HIPCHK(hipEventRecord(ctx->ev_up, ctx->cs));
        HIPCHK(hipStreamWaitEvent(ctx->s, ctx->ev_up, 0));
    }
    // the flags are packed on this stream before the header: packed by the
    // walk on the copy stream, they would wait for the scatter's blocks.
    // When the rounds changed nothing, the forest the batch was classified
    // against is the one after the rounds: no check.
    HIPCHK(launch_reflag(ctx->s, ctx->V, ctx->d_lp, ctx->d_hdr, ctx->d_fupd.p, ctx->h_hdr,
                         flag_inline(ctx, n), ctx->d_foff.p, ctx->d_oupd.p, changed));
    ctx->flags_packed = true;
    cupk_ctx::TimerSlot *ts = ctx->split_ts;
    ctx->split_ts = nullptr;
    if (ts) HIPCHK(hipEventRecord(ts->tc, ctx->s));
    const int rc = enqueue_tile(ctx, ctx->s, n, ts != nullptr);
    if (rc != CUPK_OK) return rc;
    ctx->hdr_seq++;
    ctx->hdr_word = &ctx->h_hdr[HDR_SEQ];
    if (ts) {
        HIPCHK(hipEventRecord(ts->t1, ctx->s));
        ts->split = true;
        ts->busy = true;
    }
    ctx->ctr.scatter_launches++;
    return CUPK_OK;
}

int enqueue_pass(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n, bool revert)
{
    int rc = harvest_timers(ctx, false);
    if (rc != CUPK_OK) return rc;
    ctx->flags_packed = false;
    if (!revert) {
        rc = upload_forest(ctx);
        if (rc != CUPK_OK) return rc;
    }
    const bool graph = ctx->opts.use_graph != 0 && !ctx->opts.exact;
    ctx->small_pass = !graph && n <= kSmallMax;
    if (ctx->small_pass) {
        // two launches and one copy: classify into the result block, copy
        // header + flags + positions to the host, scatter with device
        // atomics (the previous small result was read before this pass:
        // every pass waits for its header or for the whole stream)
        uint32_t *derr = &ctx->d_small->hdr[HDR_ERR];
        HIPCHK(launch_small_classify(ctx->s, d_upd, n, ctx->V, ctx->d_lbl, ctx->d_par,
                                     ctx->h_small, derr, ctx->d_hdr + HDR_SEQ,
                                     ctx->opts.exact != 0));
        ctx->hdr_seq++;
        ctx->hdr_word = &ctx->h_small->hdr[HDR_SEQ];
        // the host walks the flags while the scatter runs
        HIPCHK(launch_small_scatter(ctx->s, d_upd, n, dev_sketch(ctx), derr));
        ctx->ctr.scatter_launches++;
        return CUPK_OK;
    }
    // the batch descriptor: kernel arguments, or for captured graphs device
    // memory (pinned staging; the previous pass's copy has completed: every
    // pass is followed by a wait for its classify step or for the whole
    // stream)
    ctx->cur_desc.upd = d_upd;
    ctx->cur_desc.n = n;
    if (graph) {
        ctx->h_desc->upd = d_upd;
        ctx->h_desc->n = n;
        HIPCHK(hipMemcpyAsync(ctx->d_desc, ctx->h_desc, sizeof(BatchDesc), hipMemcpyHostToDevice,
                              ctx->s));
    }
    if (graph && (ctx->graph_cap < n || !ctx->gx_cls)) {
        rc = capture_graphs(ctx);
        if (rc != CUPK_OK) return rc;
    }
    // Timed passes (every time_kernels-th) get events around the binning and
    // the scatter; captured graphs are then launched in their three parts.
    cupk_ctx::TimerSlot *ts = nullptr;
    rc = take_timer(ctx, n, &ts);
    if (rc != CUPK_OK) return rc;
    // The classify step publishes the header to pinned host memory itself,
    // and the host waits for it by its sequence number, not an event: every
    // event recorded between two kernels leaves the GPU idle for a few
    // microseconds.  (Flag compaction on the copy stream is launched only
    // after the header has arrived, so after classification has finished.)
    if (graph && !ts) {
        HIPCHK(hipGraphLaunch(ctx->gx_all, ctx->s));
    } else if (graph) {
        HIPCHK(hipGraphLaunch(ctx->gx_cls, ctx->s));
        HIPCHK(hipEventRecord(ts->t0, ctx->s));
        HIPCHK(hipGraphLaunch(ctx->gx_bin, ctx->s));
        HIPCHK(hipEventRecord(ts->tb, ctx->s));
        HIPCHK(hipGraphLaunch(ctx->gx_tile, ctx->s));
    } else {
        // scatter skipped on the device if the batch was rejected
        rc = enqueue_classify(ctx, ctx->s, n);
        if (rc != CUPK_OK) return rc;
        if (ts) HIPCHK(hipEventRecord(ts->t0, ctx->s));
        rc = enqueue_bin(ctx, ctx->s, n);
        if (rc != CUPK_OK) return rc;
        if (ts) HIPCHK(hipEventRecord(ts->tb, ctx->s));
        rc = enqueue_tile(ctx, ctx->s, n, ts != nullptr);
        if (rc != CUPK_OK) return rc;
    }
    ctx->hdr_seq++;
    ctx->hdr_word = &ctx->h_hdr[HDR_SEQ];
    if (ts) {
        HIPCHK(hipEventRecord(ts->t1, ctx->s));
        ts->busy = true;
    }
    ctx->ctr.scatter_launches++;
    return CUPK_OK;
}

// Walk flagged updates [k0, k1) of an exact-mode pass: inserts link as
// usual; the walk stops before the first delete of a current forest edge
// and returns its index in *kc.  Returns 0 (list done), 1 (stop: insert-only
// list and one tree left) or 2 (a cut at *kc).
int walk_exact(cupk_ctx *ctx, const uint64_t *upd, uint32_t k0, uint32_t k1, bool all_inserts,
               uint32_t *kc)
{
    Forest &F = ctx->forest;
    for (uint32_t k = k0; k < k1; k++) {
        if (all_inserts && F.n_trees() == 1) return 1;
        const uint64_t p = upd[k];
        uint32_t a = (uint32_t)p, b = (uint32_t)(p >> 32) & 0x7fffffffu;
        if (a > b) std::swap(a, b);
        if ((p >> 63) == 0) {
            if (!F.same_tree(a, b)) {
                F.link(a, b);
                ctx->ctr.links++;
                ctx->forest_dev_stale = true;
            }
        } else if (F.is_edge(a, b)) {
            *kc = k;
            return 2;
        }
    }
    return 0;
}

// Wait until the header with sequence number `seq` has been published to
// host memory.  The stream is queried now and then: if it has drained and
// the header is still missing, or it reports an error, the wait fails
// instead of spinning on.
// A batch already in device memory: the stream is queried only after a
// millisecond without the header, then once per millisecond (a query of a
// busy stream can queue a marker, which idles the GPU for a few
// microseconds between two kernels).  A batch uploaded from host memory:
// every 256 spins, which kept the served query latency lower.
static int wait_header(cupk_ctx *ctx, uint32_t seq)
{
    uint32_t *w = ctx->hdr_word;
    const double every = ctx->query_often ? 0.0 : 1.0;
    double next_query = 0;
    for (uint32_t spin = 1;; spin++) {
        if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return CUPK_OK;
        if ((spin & 255) == 0) {
            const double t = now_ms();
            if (next_query == 0) next_query = t + every;
            if (t < next_query) {
                __builtin_ia32_pause();
                continue;
            }
            next_query = t + every;
            const hipError_t e = hipStreamQuery(ctx->s);
            if (e == hipSuccess) {
                if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == seq) return CUPK_OK;
                return ctx->fail(hipErrorUnknown, "classification header was not published",
                                 __LINE__);
            }
            if (e != hipErrorNotReady) return ctx->fail(e, "hipStreamQuery", __LINE__);
        }
        __builtin_ia32_pause();
    }
}

// Host side of a pass: wait for the classification header, pack and fetch
// the flagged updates in growing chunks and walk them into the forest.
// exact: stop at the first cut and report its position in the pass and its
// endpoints (*cut_pos = UINT32_MAX when the pass has no cut).
int walk_pass(cupk_ctx *ctx, uint32_t n, bool exact, uint32_t *cut_pos, uint32_t *cut_a,
              uint32_t *cut_b, uint32_t *nflag_out, double *t_wait, double *t_copy)
{
    double t0 = now_ms();
    {
        int rw = wait_header(ctx, ctx->hdr_seq);
        if (rw != CUPK_OK) return rw;
    }
    double t1 = now_ms();
    ctx->ctr.host_wait_ms += t1 - t0;
    *t_wait = t1 - t0;
    // a small pass left header, flags and positions in one host block
    const bool small = ctx->small_pass;
    const uint32_t *hdr = small ? ctx->h_small->hdr : ctx->h_hdr;
    if (hdr[HDR_ERR]) {
        HIPCHK(hipStreamSynchronize(ctx->s));
        return ctx->invalid("batch holds an update with u == v or an endpoint >= V");
    }
    const uint32_t nflag = hdr[HDR_NFLAG];
    const uint32_t nflag_del = hdr[HDR_NFLAG_DEL];
    *nflag_out = nflag;
    if (cut_pos) *cut_pos = UINT32_MAX;
    double tcopy = t1;
    const uint64_t *fl = small ? ctx->h_small->fupd : ctx->h_fupd.p;
    const uint32_t *fp = small ? ctx->h_small->fpos : ctx->h_fpos.p;
    // the flags are already in host memory after a small pass and when the
    // device wrote a short list with the header
    const bool have = small || hdr[HDR_INLINE] != 0;
    if (nflag && !(ctx->levels && nflag_del == 0)) {
        // pack the per-block regions into one ordered list (copy stream,
        // already ordered after the classify kernel), then fetch and walk it
        // in growing chunks: the walk may stop early
        uint32_t *opos = exact ? ctx->d_opos.p : nullptr;
        if (!have && !ctx->flags_packed)
            HIPCHK(launch_flag_compact(ctx->cs, n, ctx->d_fupd.p, exact ? ctx->d_fpos.p : nullptr,
                                       ctx->d_fcnt.p, ctx->d_foff.p, ctx->d_oupd.p, opos));
        uint32_t k0 = 0, step = have ? nflag : 1u << 16;
        while (k0 < nflag) {
            const uint32_t m = std::min(step, nflag - k0);
            if (!have) {
                HIPCHK(hipMemcpyAsync(ctx->h_fupd.p + k0, ctx->d_oupd.p + k0, (size_t)m * 8,
                                      hipMemcpyDeviceToHost, ctx->cs));
                if (exact)
                    HIPCHK(hipMemcpyAsync(ctx->h_fpos.p + k0, opos + k0, (size_t)m * 4,
                                          hipMemcpyDeviceToHost, ctx->cs));
                HIPCHK(hipStreamSynchronize(ctx->cs));
            }
            if (k0 == 0) tcopy = now_ms();
            if (exact) {
                uint32_t kc = 0;
                const int r = walk_exact(ctx, fl, k0, k0 + m, nflag_del == 0, &kc);
                if (r == 2) {
                    const uint64_t p = fl[kc];
                    *cut_pos = fp[kc];
                    *cut_a = std::min((uint32_t)p, (uint32_t)(p >> 32) & 0x7fffffffu);
                    *cut_b = std::max((uint32_t)p, (uint32_t)(p >> 32) & 0x7fffffffu);
                    break;
                }
                if (r == 1) break;
            } else if (apply_flags(ctx, fl, k0, k0 + m, nflag_del == 0)) {
                break;
            }
            k0 += m;
            step *= 2;
        }
    }
    *t_copy = tcopy - t1;
    ctx->ctr.host_flags_ms += now_ms() - t1;
    ctx->ctr.flagged += nflag;
    return CUPK_OK;
}

// Host part of a batch-semantics pass whose device work is enqueued: wait
// for the classification header, walk the flagged updates into the forest,
// then run the replacement rounds (or, in levels mode, the restoration).
static int finish_pass(cupk_ctx *ctx, uint32_t n)
{
    uint32_t nflag = 0;
    double tw = 0, tc = 0;
    const double t0 = now_ms();
    int rc = walk_pass(ctx, n, false, nullptr, nullptr, nullptr, &nflag, &tw, &tc);
    if (rc != CUPK_OK) return rc;
    const double t2 = now_ms();
    rc = ctx->levels ? levels_restore(ctx) : run_rounds(ctx);
    const double t3 = now_ms();
    ctx->ctr.host_rounds_ms += t3 - t2;
    if (ctx->trace)
        fprintf(stderr,
                "cupk batch %llu n=%u nflag=%u wait=%.3f copy=%.3f flags=%.3f rounds=%.3f ms\n",
                (unsigned long long)ctx->ctr.batches, n, nflag, tw, tc, t2 - t0 - tw - tc,
                t3 - t2);
    return rc;
}

// The host part of the last enqueued batch, if it has not run yet.  Every
// entry point that reads the forest, the sketch or the counters, or enqueues
// more work, calls this first.
int flush_pending(cupk_ctx *ctx)
{
    if (!ctx->pending) return CUPK_OK;
    ctx->pending = false;
    return finish_pass(ctx, ctx->pending_n);
}

// Leave the host part of the batch just enqueued (n updates) pending.  A
// large batch's scatter is marked for the replacement rounds of an
// overlapped next batch (which reduce on another stream after it).
static int set_pending(cupk_ctx *ctx, uint32_t n)
{
    ctx->scat_marked = false;
    if (n > kSmallMax && !ctx->opts.serial_rounds) {
        HIPCHK(hipEventRecord(ctx->ev_scat, ctx->s));
        ctx->scat_marked = true;
    }
    ctx->pending = true;
    ctx->pending_n = n;
    return CUPK_OK;
}

// Whether batch k+1 (n updates) can be classified and binned while the
// pending batch k's replacement rounds run: batch semantics, no captured
// graphs, a batch of at least overlap_min_batch updates (smaller ones leave
// the GPU idle during the rounds anyway), and batch buffers that already
// hold it (a reallocation could free buffers that k's scatter still uses).
constexpr uint32_t kOverlapMinBatch = 1u << 22;
static bool can_overlap(cupk_ctx *ctx, uint32_t n)
{
    const uint32_t lo = ctx->opts.overlap_min_batch ? ctx->opts.overlap_min_batch
                                                    : kOverlapMinBatch;
    return ctx->pending && !ctx->opts.serial_rounds && !ctx->opts.exact && !ctx->levels &&
           ctx->opts.use_graph == 0 && n > kSmallMax && n >= lo && n <= ctx->batch_cap;
}

static int apply_flushed(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n, bool defer);

// Pending batch k, new batch k+1 (n updates at d_upd).  Walk k's flags into
// the forest; upload that forest on the copy stream; classify and bin k+1
// against it on the main stream while k's replacement rounds run on the
// host, their reductions on the copy stream after k's scatter (the copy
// stream is idle meanwhile: k's flags have been fetched, k+1's are not
// published yet; a stream of their own would cost a hardware queue, and
// streams that share one run in one order); then the
// back half of k+1 (enqueue_split_back).  The rounds only link trees, so
// the forest after the walk has finer trees and a subset of the edges of
// the forest after the rounds: every update the classify rule flags against
// the latter it also flags against the former (a delete of an edge the
// rounds added joins two trees of the former), and the check against the
// latter in the back half leaves exactly the serial order's flags.  This
// needs exact labels after the walk: when it ends with removals whose trees
// are not split yet (their pieces still share a label until the rounds
// split them), k's rounds run first and k+1 takes the serial order.  So it
// does when the walk leaves fewer than two dirty trees: the rounds then
// have nothing to search, and the split pass's extra launches and stream
// waits would only cost time.  An error of k's rounds is this call's, and
// k+1 is then still applied.
static int apply_overlapped(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n, bool defer)
{
    ctx->pending = false;
    const uint32_t nk = ctx->pending_n;
    const unsigned long long bk = (unsigned long long)ctx->ctr.batches;
    uint32_t nflag = 0;
    double tw = 0, tc = 0;
    const double t0 = now_ms();
    int rc = walk_pass(ctx, nk, false, nullptr, nullptr, nullptr, &nflag, &tw, &tc);
    if (rc != CUPK_OK) return rc;
    const double t1 = now_ms();
    if (ctx->forest.has_pending() || ctx->forest.dirty_labels().size() < 2) {
        ctx->scat_marked = false;
        const int rr = run_rounds(ctx);
        const double t3 = now_ms();
        ctx->ctr.host_rounds_ms += t3 - t1;
        if (ctx->trace)
            fprintf(stderr,
                    "cupk batch %llu n=%u nflag=%u wait=%.3f copy=%.3f flags=%.3f rounds=%.3f ms\n",
                    bk, nk, nflag, tw, tc, t1 - t0 - tw - tc, t3 - t1);
        if (rr != CUPK_OK) return rr;
        return apply_flushed(ctx, d_upd, n, defer);
    }
    if (!ctx->scat_marked) HIPCHK(hipEventRecord(ctx->ev_scat, ctx->s));
    ctx->scat_marked = false;
    // the forest after the walk, for k+1's classification (every earlier
    // reader of the device forest has finished: k's header, which the walk
    // waited for, is published after them)
    const bool up = ctx->forest_dev_stale;
    if (up) {
        rc = upload_forest_on(ctx, ctx->cs);
        if (rc != CUPK_OK) return rc;
        HIPCHK(hipEventRecord(ctx->ev_up, ctx->cs));
        HIPCHK(hipStreamWaitEvent(ctx->s, ctx->ev_up, 0));
    }
    ctx->ctr.updates += n;
    ctx->ctr.batches++;
    ctx->ctr.overlapped++;
    rc = enqueue_split_front(ctx, d_upd, n);
    if (rc != CUPK_OK) return rc;
    // the rounds write the host forest the copies read
    if (up) HIPCHK(hipEventSynchronize(ctx->ev_up));
    HIPCHK(hipStreamWaitEvent(ctx->cs, ctx->ev_scat, 0));
    ctx->rstream = ctx->cs;
    const double t2 = now_ms();
    const int rr = run_rounds(ctx);
    const double t3 = now_ms();
    ctx->rstream = ctx->s;
    ctx->ctr.host_rounds_ms += t3 - t2;
    if (ctx->trace)
        fprintf(stderr,
                "cupk batch %llu n=%u nflag=%u wait=%.3f copy=%.3f flags=%.3f rounds=%.3f ms "
                "(next batch classified and binned meanwhile)\n",
                bk, nk, nflag, tw, tc, t1 - t0 - tw - tc, t3 - t2);
    rc = enqueue_split_back(ctx, n);
    if (rr != CUPK_OK) return rr;
    if (rc != CUPK_OK) return rc;
    if (defer) return set_pending(ctx, n);
    return finish_pass(ctx, n);
}

// One batch of at most kMaxBatchPerLaunch updates.  defer: leave the host
// part pending (batch semantics only; exact mode always completes).
int apply_device_one(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n, bool defer)
{
    if (can_overlap(ctx, n)) return apply_overlapped(ctx, d_upd, n, defer);
    const int rc = flush_pending(ctx);
    if (rc != CUPK_OK) return rc;
    return apply_flushed(ctx, d_upd, n, defer);
}

// The rest of apply_device_one once no host part is pending.
static int apply_flushed(cupk_ctx *ctx, const uint64_t *d_upd, uint32_t n, bool defer)
{
    int rc = ensure_batch_buffers(ctx, n);
    if (rc != CUPK_OK) return rc;
    ctx->ctr.updates += n;
    ctx->ctr.batches++;
    if (!ctx->opts.exact) {
        rc = enqueue_pass(ctx, d_upd, n, false);
        if (rc != CUPK_OK) return rc;
        if (defer && !ctx->levels) return set_pending(ctx, n);
        return finish_pass(ctx, n);
    }
    // exact mode: speculate over the rest of the batch, stop at the first
    // cut, undo the speculation past it, cut and search replacements on the
    // sketch as of that update, then go on after it
    uint32_t nflag = 0;
    double tw = 0, tc = 0;
    uint32_t s = 0;
    while (s < n) {
        rc = enqueue_pass(ctx, d_upd + s, n - s, false);
        if (rc != CUPK_OK) return rc;
        uint32_t pos, a = 0, b = 0;
        rc = walk_pass(ctx, n - s, true, &pos, &a, &b, &nflag, &tw, &tc);
        if (rc != CUPK_OK) return rc;
        if (pos == UINT32_MAX) break;
        const uint32_t next = s + pos + 1;
        if (next < n) {
            rc = enqueue_pass(ctx, d_upd + next, n - next, true);
            if (rc != CUPK_OK) return rc;
            ctx->ctr.reverts++;
            // the descriptor staging is written again by the next pass
            HIPCHK(hipStreamSynchronize(ctx->s));
        }
        ctx->forest.cut(a, b);
        ctx->ctr.cuts++;
        ctx->forest_dev_stale = true;
        const double t2 = now_ms();
        rc = run_rounds(ctx);
        ctx->ctr.host_rounds_ms += now_ms() - t2;
        if (rc != CUPK_OK) return rc;
        s = next;
    }
    const double t2 = now_ms();
    rc = run_rounds(ctx);
    ctx->ctr.host_rounds_ms += now_ms() - t2;
    return rc;
}

int apply_device(cupk_ctx *ctx, const uint64_t *d_upd, size_t n, bool defer)
{
    for (size_t off = 0; off < n; off += kMaxBatchPerLaunch) {
        const uint32_t m = (uint32_t)std::min(kMaxBatchPerLaunch, n - off);
        int rc = apply_device_one(ctx, d_upd + off, m, defer);
        if (rc != CUPK_OK) return rc;
    }
    return CUPK_OK;
}

int connected_impl(cupk_ctx *ctx, uint32_t u, uint32_t v)
{
    return ctx->forest.same_tree(u, v) ? 1 : 0;
}

void destroy(cupk_ctx *ctx)
{
    ctx->server.reset();
    levels_release(ctx);
    if (ctx->s) (void)hipStreamSynchronize(ctx->s);
    if (ctx->cs) (void)hipStreamSynchronize(ctx->cs);
    if (ctx->own_sk && ctx->d_sk) (void)hipFree(ctx->d_sk);
    if (ctx->d_seeds) (void)hipFree(ctx->d_seeds);
    if (ctx->d_lbl) (void)hipFree(ctx->d_lbl);
    if (ctx->d_par) (void)hipFree(ctx->d_par);
    if (ctx->d_lp) (void)hipFree(ctx->d_lp);
    if (ctx->d_blk) (void)hipFree(ctx->d_blk);
    if (ctx->h_lbl) (void)hipHostFree(ctx->h_lbl);
    if (ctx->h_par) (void)hipHostFree(ctx->h_par);
    if (ctx->d_hdr) (void)hipFree(ctx->d_hdr);
    if (ctx->h_hdr) (void)hipHostFree(ctx->h_hdr);
    if (ctx->d_nitems) (void)hipFree(ctx->d_nitems);
    if (ctx->d_touched) (void)hipFree(ctx->d_touched);
    drop_graphs(ctx);
    if (ctx->gs) (void)hipStreamDestroy(ctx->gs);
    if (ctx->d_desc) (void)hipFree(ctx->d_desc);
    if (ctx->h_desc) (void)hipHostFree(ctx->h_desc);
    if (ctx->d_misc) (void)hipFree(ctx->d_misc);
    if (ctx->d_small) (void)hipFree(ctx->d_small);
    if (ctx->h_small) (void)hipHostFree(ctx->h_small);
    if (ctx->h_misc) (void)hipHostFree(ctx->h_misc);
    release(ctx->d_upd);
    release(ctx->h_upd);
    release(ctx->d_fupd);
    release(ctx->d_oupd);
    release(ctx->d_foff);
    release(ctx->d_fcnt);
    release(ctx->d_fdel);
    release(ctx->h_fupd);
    release(ctx->d_fpos);
    release(ctx->d_opos);
    release(ctx->h_fpos);
    release(ctx->d_tcnt);
    release(ctx->d_toff);
    release(ctx->d_tsum);
    release(ctx->d_tcur);
    release(ctx->d_trel);
    release(ctx->d_tgoff);
    release(ctx->d_items);
    release(ctx->d_bins);
    release(ctx->d_bins1);
    release(ctx->d_ccnt);
    release(ctx->d_cgoff);
    release(ctx->d_coff);
    release(ctx->d_ccur);
    release(ctx->d_csink);
    release(ctx->d_ridx);
    release(ctx->h_ridx);
    release(ctx->d_sig[0]);
    release(ctx->d_sig[1]);
    release(ctx->d_res);
    release(ctx->h_res);
    release(ctx->d_tmp);
    release(ctx->h_stage);
    release(ctx->d_stage);
    for (auto &t : ctx->timers) {
        if (t.t0) (void)hipEventDestroy(t.t0);
        if (t.tb) (void)hipEventDestroy(t.tb);
        if (t.tc) (void)hipEventDestroy(t.tc);
        if (t.t1) (void)hipEventDestroy(t.t1);
    }
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->ev_scat) (void)hipEventDestroy(ctx->ev_scat);
    if (ctx->ev_up) (void)hipEventDestroy(ctx->ev_up);
    if (ctx->ev_cls) (void)hipEventDestroy(ctx->ev_cls);
    if (ctx->ev_stage) (void)hipEventDestroy(ctx->ev_stage);
    if (ctx->cs) (void)hipStreamDestroy(ctx->cs);
    if (ctx->own_stream && ctx->s) (void)hipStreamDestroy(ctx->s);
    delete ctx;
}

// Staged-scatter geometry: tv vertices per tile (power of two), `rows` depth
// rows in LDS, `chunk` records per work item; `coarse` tiles per coarse bin
// of the two-level binning (a power of two; 0: the default).
int set_geometry(cupk_ctx *ctx, uint32_t tv, uint32_t rows, uint32_t chunk, uint32_t layout,
                 uint32_t coarse)
{
    if (layout != CUPK_LAYOUT_RECORD && layout != CUPK_LAYOUT_PAIR)
        return ctx->invalid("tile_layout must be CUPK_LAYOUT_RECORD or CUPK_LAYOUT_PAIR");
    drop_graphs(ctx);  // captured graphs embed the geometry and buffers
    uint32_t sh = 0;
    while ((1u << sh) < tv) sh++;
    if (tv == 0 || (1u << sh) != tv) return ctx->invalid("tile_vertices must be a power of two");
    if (rows < 1 || rows > ctx->D) return ctx->invalid("lds_rows must be in [1, D]");
    if (!tile_geometry_fits(rows, ctx->C, tv, layout))
        return ctx->invalid("staged tile does not fit 64 KiB of LDS (with the record stage of "
                            "the pair layout)");
    if (chunk < 64) return ctx->invalid("chunk_records must be >= 64");
    ctx->tile_shift = sh;
    ctx->rows = rows;
    ctx->chunk = chunk;
    ctx->layout = layout;
    ctx->ntiles = (uint32_t)(((uint64_t)ctx->V + tv - 1) >> sh);
    // two-level binning beyond kFillStageTiles tiles.  Both fills write runs
    // of records per (block, bin): about 8192 / ncoarse records per coarse
    // bin in the first, about 4096 / (tiles per coarse bin) per tile in the
    // second; by default the coarse count is the power of two nearest
    // sqrt(2 * ntiles), which evens out the two when records fall on every
    // tile, within [64, 2048].  When they fall on a few tiles only (dense
    // clusters), smaller coarse bins keep the second fill's runs long, and
    // the autotuner tries them.
    ctx->fshift = 0;
    ctx->ncoarse = 0;
    if (coarse && (coarse < 2 || coarse > kFineLdsTiles || (coarse & (coarse - 1))))
        return ctx->invalid("coarse_tiles must be a power of two in [2, 8192]");
    if (ctx->opts.scatter_mode == CUPK_SCATTER_STAGED && ctx->ntiles > kFillStageTiles) {
        uint32_t f = 1;
        if (coarse) {
            while ((1u << f) < coarse) f++;
            // the classify kernel counts coarse bins in LDS: at most 8192
            if ((((uint64_t)ctx->ntiles + (1u << f) - 1) >> f) > kLdsHistMax)
                return ctx->invalid("coarse_tiles too small: more than 8192 coarse bins");
        } else {
            uint32_t target = 64;
            while (target < 2048 &&
                   (uint64_t)(2 * target) * (2 * target) <= 2 * (uint64_t)ctx->ntiles)
                target *= 2;
            while ((((uint64_t)ctx->ntiles + (1u << f) - 1) >> f) > target) f++;
        }
        ctx->fshift = f;
        ctx->ncoarse = (uint32_t)(((uint64_t)ctx->V + (1ull << (sh + f)) - 1) >> (sh + f));
        const size_t nc = (size_t)kCntGroups * ctx->ncoarse + 1;
        HIPCHK(grow(ctx->d_ccnt, nc));
        HIPCHK(grow(ctx->d_cgoff, nc));
        HIPCHK(grow(ctx->d_coff, ctx->ncoarse + 1));
        HIPCHK(grow(ctx->d_ccur, ctx->ncoarse + 1));
        HIPCHK(grow(ctx->d_csink, 4));
        HIPCHK(launch_zero32(ctx->s, ctx->d_ccnt.p, nc));
        if (ctx->batch_cap) HIPCHK(grow(ctx->d_bins1, 2 * ctx->batch_cap));
    }
    if (ctx->opts.scatter_mode == CUPK_SCATTER_STAGED) {
        // counts: kCntGroups copies (one in use unless classify blocks also
        // store where their records start)
        const size_t ncnt = (size_t)kCntGroups * ctx->ntiles + 1;
        HIPCHK(grow(ctx->d_tcnt, ncnt));
        HIPCHK(grow(ctx->d_tgoff, ncnt));
        HIPCHK(grow(ctx->d_toff, ctx->ntiles + 1));
        HIPCHK(grow(ctx->d_tsum, 2 * (size_t)tile_scan_chunks(ctx->ntiles) + 2));
        HIPCHK(grow(ctx->d_tcur, ctx->ntiles + 1));
        // the scan kernel re-zeroes the counts after every batch
        HIPCHK(launch_zero32(ctx->s, ctx->d_tcnt.p, ncnt));
        // work-item capacity depends on ntiles and chunk
        const size_t icap = 2 * ctx->batch_cap / chunk + ctx->ntiles + 1;
        HIPCHK(grow(ctx->d_items, 2 * icap));
    }
    return ensure_rel(ctx);
}

int init_impl(cupk_ctx *ctx, const cupk_opts *opts)
{
    const uint32_t V = ctx->V, C = ctx->C, D = ctx->D;
    if (opts) ctx->opts = *opts;
    else ctx->opts.scatter_mode = CUPK_SCATTER_STAGED;
    if (ctx->opts.scatter_mode > CUPK_SCATTER_STAGED) return ctx->invalid("unknown scatter_mode");
    if (ctx->opts.levels && ctx->opts.exact)
        return ctx->invalid("levels and exact modes do not combine");
    uint64_t st = ctx->S;
    for (uint32_t c = 0; c < C; c++) {
        st += 0x9E3779B97F4A7C15ull;
        ctx->seeds[c] = sm64_mix(st);
    }
    ctx->W = 2 * C * D;
    HIPCHK(hipGetDevice(&ctx->device));
    // the allocation-free entry point's scratch array on this device
    HIPCHK(noalloc_scratch_address(ctx->device, &ctx->noalloc_scratch));
    {
        const char *tr = getenv("CUPK_TRACE");
        ctx->trace = tr && tr[0] == '1';
    }
    if (ctx->opts.use_given_stream) {
        ctx->s = (hipStream_t)ctx->opts.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&ctx->s, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&ctx->cs, hipStreamNonBlocking));
    ctx->rstream = ctx->s;
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_scat, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_up, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_cls, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ctx->ev_stage, hipEventDisableTiming));
    if (ctx->opts.time_kernels)
        for (auto &t : ctx->timers) {
            HIPCHK(hipEventCreate(&t.t0));
            HIPCHK(hipEventCreate(&t.tb));
            HIPCHK(hipEventCreate(&t.tc));
            HIPCHK(hipEventCreate(&t.t1));
        }
    const size_t sk_bytes = cupk_sketch_bytes(V, C, D);
    if (ctx->opts.sketch_device_ptr) {
        ctx->d_sk = (uint64_t *)ctx->opts.sketch_device_ptr;
    } else {
        HIPCHK(hipMalloc((void **)&ctx->d_sk, sk_bytes));
        ctx->own_sk = true;
    }
    HIPCHK(launch_zero(ctx->s, ctx->d_sk, sk_bytes / 8));
    HIPCHK(hipMalloc((void **)&ctx->d_seeds, 64 * 8));
    HIPCHK(hipMemcpy(ctx->d_seeds, ctx->seeds, 64 * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMalloc((void **)&ctx->d_lbl, (size_t)V * 4));
    HIPCHK(hipMalloc((void **)&ctx->d_par, (size_t)V * 4));
    HIPCHK(hipMalloc((void **)&ctx->d_lp, (size_t)V * 8));
    HIPCHK(hipMalloc((void **)&ctx->d_blk, (((size_t)V + 63) >> kBlkShift) * 4));
    HIPCHK(hipHostMalloc((void **)&ctx->h_lbl, (size_t)V * 4, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&ctx->h_par, (size_t)V * 4, hipHostMallocDefault));
    HIPCHK(hipMalloc((void **)&ctx->d_hdr, HDR_WORDS * 4));
    HIPCHK(hipMemset(ctx->d_hdr, 0, HDR_WORDS * 4));
    // coherent: the scan kernel's stores reach the host without a flush
    HIPCHK(hipHostMalloc((void **)&ctx->h_hdr, HDR_WORDS * 4, hipHostMallocCoherent));
    memset(ctx->h_hdr, 0, HDR_WORDS * 4);
    HIPCHK(hipMalloc((void **)&ctx->d_nitems, 4));
    HIPCHK(hipMalloc((void **)&ctx->d_touched, 8));
    HIPCHK(hipMemset(ctx->d_touched, 0, 8));
    HIPCHK(hipMalloc((void **)&ctx->d_desc, sizeof(BatchDesc)));
    HIPCHK(hipHostMalloc((void **)&ctx->h_desc, sizeof(BatchDesc), hipHostMallocDefault));
    HIPCHK(hipMalloc((void **)&ctx->d_misc, 64));
    HIPCHK(hipMalloc((void **)&ctx->d_small, sizeof(SmallResult)));
    // coherent: the small classify kernel writes its result here directly
    HIPCHK(hipHostMalloc((void **)&ctx->h_small, sizeof(SmallResult), hipHostMallocCoherent));
    memset(ctx->h_small, 0, sizeof(SmallResult));
    HIPCHK(hipHostMalloc((void **)&ctx->h_misc, 64, hipHostMallocDefault));
    ctx->forest.init(V, ctx->h_lbl, ctx->h_par);
    ctx->forest.track_pages(10);  // 4 KiB of labels (and of parents) per page
    if (V >= (1u << 17)) {
        // host forest work of a batch (relabels, member lists) is split
        // over a few threads when trees are large
        ctx->pool.reset(new (std::nothrow) cupk::Pool());
        if (ctx->pool) ctx->forest.set_pool(ctx->pool.get());
    }
    if (ctx->opts.levels) {
        int rc = levels_init(ctx);
        if (rc != CUPK_OK) return rc;
    }
    ctx->forest_dev_stale = true;

    // staged scatter geometry: LDS delta of `rows` depth rows x C columns x
    // 2 words per vertex, at most 64 KiB per block
    uint32_t rows = ctx->opts.lds_rows ? ctx->opts.lds_rows : 8;
    rows = std::min(rows, D);
    uint32_t tv = ctx->opts.tile_vertices;
    if (tv == 0) {
        // measured best on the V=16384, C=14 workload: 16 vertices per tile
        // (about 28 KiB of LDS, several blocks per CU); smaller when C*rows
        // does not fit
        tv = 1;
        while ((size_t)2 * rows * C * (tv * 2) * 8 <= 32768 && tv < 16) tv *= 2;
    }
    ctx->tile_grid = ctx->opts.tile_grid;
    uint32_t layout = ctx->opts.tile_layout;
    if (layout == 0)
        layout = ctx->opts.max_batch >= (4u << 20) ? CUPK_LAYOUT_PAIR : CUPK_LAYOUT_RECORD;
    int rc0 = set_geometry(ctx, tv, rows, ctx->opts.chunk_records ? ctx->opts.chunk_records : 4096,
                           layout, ctx->opts.coarse_tiles);
    if (rc0 != CUPK_OK) return rc0;
    const size_t mb = ctx->opts.max_batch ? ctx->opts.max_batch : (1u << 20);
    int rc = ensure_batch_buffers(ctx, mb);
    if (rc != CUPK_OK) return rc;
    // replacement-round buffers sized up front (every vertex as a member,
    // up to 1024 sets), so rounds do not allocate (allocation and free can
    // synchronise the device)
    {
        const size_t sets = std::min<size_t>(V, 1024);
        const size_t items = V / kRedChunk + sets + 1;
        HIPCHK(grow(ctx->d_sig[0], sets * ctx->W));
        HIPCHK(grow(ctx->d_sig[1], sets * ctx->W));
        HIPCHK(grow(ctx->d_res, 3 * sets));
        HIPCHK(grow(ctx->h_res, 3 * sets));
        HIPCHK(grow(ctx->d_ridx, (size_t)V + 1 + 3 * items));
        HIPCHK(grow(ctx->h_ridx, (size_t)V + 1 + 3 * items));
    }
    HIPCHK(hipStreamSynchronize(ctx->s));
    return CUPK_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// Whether p is device memory (anything else is taken as host memory).  The
// query of an unregistered host pointer may report an error; it is cleared
// so that the next launch check does not see it.
static bool is_device_ptr(const void *p)
{
    hipPointerAttribute_t a = {};
    const hipError_t e = hipPointerGetAttributes(&a, p);
    (void)hipGetLastError();
    return e == hipSuccess && a.type == hipMemoryTypeDevice;
}

// Entry points that read the forest, the sketch or the counters, or that
// enqueue other work, first complete the host part of a device batch left
// pending by cupk_apply_updates_device; its error is theirs.
#define CUPK_FLUSH()                                  \
    do {                                              \
        const int frc_ = flush_pending(ctx);          \
        if (frc_ != CUPK_OK) return frc_;             \
    } while (0)

extern "C" {

size_t cupk_sketch_bytes(uint32_t V, uint32_t C, uint32_t D)
{
    return (size_t)V * C * D * 2 * sizeof(uint64_t);
}

int cupk_sketch_init(cupk_ctx **out, uint32_t V, uint32_t C, uint32_t D, uint64_t seed,
                     const cupk_opts *opts)
{
    if (!out) return CUPK_EINVAL;
    *out = nullptr;
    if (V < 2 || V > (1u << 31)) return CUPK_EINVAL;
    const uint32_t L = ceil_log2(V);
    if (C == 0) C = L;
    if (D == 0) D = 2 * L;
    if (C < 1 || C > 64 || D < 2 || D > 64) return CUPK_EINVAL;
    cupk_ctx *ctx = new (std::nothrow) cupk_ctx();
    if (!ctx) return CUPK_ENOMEM;
    ctx->V = V;
    ctx->C = C;
    ctx->D = D;
    ctx->S = seed;
    int rc = guarded(ctx, [&] { return init_impl(ctx, opts); });
    if (rc != CUPK_OK) {
        g_init_error = ctx->err;
        destroy(ctx);
        return rc;
    }
    *out = ctx;
    return CUPK_OK;
}

void cupk_free(cupk_ctx *ctx)
{
    if (ctx) destroy(ctx);
}

int cupk_apply_updates(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v,
                       const uint8_t *is_delete, size_t n)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        if (n == 0) return CUPK_OK;
        if (!u || !v || !is_delete) return ctx->invalid("null array");
        for (size_t i = 0; i < n; i++)
            if (u[i] == v[i] || u[i] >= ctx->V || v[i] >= ctx->V)
                return ctx->invalid("batch holds an update with u == v or an endpoint >= V");
        int rc = flush_pending(ctx);
        if (rc != CUPK_OK) return rc;
        HIPCHK(grow(ctx->h_upd, n));
        HIPCHK(grow(ctx->d_upd, n));
        // the previous batch's upload from h_upd finished: every call waits for
        // its classify kernel, which follows the upload on the stream
        uint64_t *h = ctx->h_upd.p;
        for (size_t i = 0; i < n; i++)
            h[i] = (uint64_t)u[i] | ((uint64_t)v[i] << 32) | ((uint64_t)(is_delete[i] != 0) << 63);
        HIPCHK(hipMemcpyAsync(ctx->d_upd.p, h, n * 8, hipMemcpyHostToDevice, ctx->s));
        ctx->query_often = true;
        rc = apply_device(ctx, ctx->d_upd.p, n, false);
        ctx->query_often = false;
        return rc;
    });
}

int cupk_apply_updates_device(cupk_ctx *ctx, const uint64_t *d_packed, size_t n,
                              void *hip_stream)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        if (n == 0) return CUPK_OK;
        if (!d_packed) return ctx->invalid("null device pointer");
        // the host part of the previous batch comes first, or overlaps the
        // new batch's classification (apply_device_one): its error is this
        // call's
        const hipStream_t cs = (hipStream_t)hip_stream;
        // the batch is read on the library's stream after what the caller's
        // stream has queued so far, and the caller's stream waits for the
        // scatter (the last kernel that reads the batch)
        if (cs != ctx->s) {
            HIPCHK(hipEventRecord(ctx->ev_in, cs));
            HIPCHK(hipStreamWaitEvent(ctx->s, ctx->ev_in, 0));
        }
        const int rc = apply_device(ctx, d_packed, n, true);
        if (cs != ctx->s) {
            // also after a failure: whatever was enqueued is ordered
            if (hipEventRecord(ctx->ev_out, ctx->s) == hipSuccess)
                (void)hipStreamWaitEvent(cs, ctx->ev_out, 0);
        }
        return rc;
    });
}

int cupk_component_sketch_batch(cupk_ctx *ctx, const uint64_t *offsets, size_t k,
                                const uint32_t *verts, cupk_bucket *out)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (k == 0) return CUPK_OK;
        if (!offsets || !out) return ctx->invalid("null array");
        if (offsets[0] != 0) return ctx->invalid("offsets[0] must be 0");
        for (size_t j = 0; j < k; j++)
            if (offsets[j + 1] < offsets[j]) return ctx->invalid("offsets must be non-decreasing");
        const size_t nv = offsets[k];
        if (nv && !verts) return ctx->invalid("null verts");
        if (nv >= (1ull << 32) || k >= (1ull << 31)) return ctx->invalid("too many members");
        for (size_t i = 0; i < nv; i++)
            if (verts[i] >= ctx->V) return ctx->invalid("vertex id >= V");
        std::vector<uint32_t> vmem(verts, verts + nv), voff(k + 1), none;
        for (size_t j = 0; j <= k; j++) voff[j] = (uint32_t)offsets[j];
        int rc = reduce_and_sample(ctx, 0, vmem, voff, none, none);
        if (rc != CUPK_OK) return rc;
        if (is_device_ptr(out)) {
            HIPCHK(launch_to_canonical(ctx->s, ctx->d_sig[0].p, ctx->C, ctx->D, k,
                                       (uint64_t *)out));
        } else {
            HIPCHK(grow(ctx->d_tmp, (size_t)k * ctx->W));
            HIPCHK(launch_to_canonical(ctx->s, ctx->d_sig[0].p, ctx->C, ctx->D, k, ctx->d_tmp.p));
            HIPCHK(hipMemcpyAsync(out, ctx->d_tmp.p, (size_t)k * ctx->W * 8,
                                  hipMemcpyDeviceToHost, ctx->s));
        }
        HIPCHK(hipStreamSynchronize(ctx->s));
        return CUPK_OK;
    });
}

int cupk_component_sketch_batch_noalloc(cupk_ctx *ctx, const uint64_t *offsets, size_t k,
                                        const uint32_t *verts, cupk_bucket *out_device)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        if (k == 0) return CUPK_OK;
        if (!offsets || !out_device) return ctx->invalid("null array");
        if (ctx->server) return ctx->invalid("component sketches while the serving loop runs");
        // completing a pending batch may allocate: the caller does it first
        if (ctx->pending)
            return ctx->invalid("a device batch is pending: call cupk_sync first");
        if (k > kNoAllocMaxSets) return ctx->invalid("more sets than the scratch holds (4096)");
        if ((uint64_t)k * ctx->W > kNoAllocAggWords)
            return ctx->invalid("k * 2*C*D words exceed the scratch's 2^21 aggregate words");
        if (offsets[0] != 0) return ctx->invalid("offsets[0] must be 0");
        for (size_t j = 0; j < k; j++)
            if (offsets[j + 1] < offsets[j]) return ctx->invalid("offsets must be non-decreasing");
        const uint64_t nv = offsets[k];
        if (nv > kNoAllocMaxMembers)
            return ctx->invalid("more members than the scratch holds (2^20)");
        if (nv && !verts) return ctx->invalid("null verts");
        for (uint64_t i = 0; i < nv; i++)
            if (verts[i] >= ctx->V) return ctx->invalid("vertex id >= V");
        if (!is_device_ptr(out_device)) return ctx->invalid("out_device is not device memory");
        uint64_t *agg = ctx->noalloc_scratch;
        uint64_t *offs = agg + kNoAllocOffsWord;
        uint32_t *mem = (uint32_t *)(agg + kNoAllocMemWord);
        // inputs into the scratch (copies from the caller's host arrays), a
        // zero fill of the aggregates, the reduction, canonical order into out
        HIPCHK(hipMemcpyAsync(offs, offsets, (k + 1) * sizeof(uint64_t), hipMemcpyHostToDevice,
                              ctx->s));
        if (nv)
            HIPCHK(hipMemcpyAsync(mem, verts, nv * sizeof(uint32_t), hipMemcpyHostToDevice,
                                  ctx->s));
        HIPCHK(launch_zero(ctx->s, agg, (size_t)k * ctx->W));
        HIPCHK(launch_reduce_csr(ctx->s, ctx->d_sk, ctx->W, mem, offs, (uint32_t)k, (uint32_t)nv,
                                 agg));
        HIPCHK(launch_to_canonical(ctx->s, agg, ctx->C, ctx->D, k, (uint64_t *)out_device));
        HIPCHK(hipStreamSynchronize(ctx->s));
        return CUPK_OK;
    });
}

int cupk_component_sketch(cupk_ctx *ctx, const uint32_t *verts, size_t n, cupk_bucket *out)
{
    const uint64_t off[2] = {0, n};
    return cupk_component_sketch_batch(ctx, off, 1, verts, out);
}

int cupk_sample_cut_edge_batch(cupk_ctx *ctx, const cupk_bucket *sketches, size_t k,
                               int32_t *status, uint32_t *u, uint32_t *v)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        if (k == 0) return CUPK_OK;
        if (!sketches || !status || !u || !v) return ctx->invalid("null array");
        if (k >= (1ull << 31)) return ctx->invalid("too many sketches");
        const size_t words = (size_t)k * ctx->W;
        HIPCHK(grow(ctx->d_tmp, words));
        HIPCHK(grow(ctx->d_res, 3 * k));
        HIPCHK(grow(ctx->h_res, 3 * k));
        HIPCHK(hipMemcpyAsync(ctx->d_tmp.p, sketches, words * 8, hipMemcpyHostToDevice, ctx->s));
        // canonical layout: bucket (c, d) at word (c*D + d)*2
        HIPCHK(launch_sample(ctx->s, ctx->d_tmp.p, (uint32_t)k, ctx->V, ctx->C, ctx->D, ctx->D, 1,
                             ctx->W, ctx->d_seeds, ctx->d_res.p));
        HIPCHK(hipMemcpyAsync(ctx->h_res.p, ctx->d_res.p, 3 * k * 4, hipMemcpyDeviceToHost, ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->s));
        for (size_t j = 0; j < k; j++) {
            status[j] = ctx->h_res.p[3 * j];
            u[j] = (uint32_t)ctx->h_res.p[3 * j + 1];
            v[j] = (uint32_t)ctx->h_res.p[3 * j + 2];
        }
        return CUPK_OK;
    });
}

int cupk_sample_cut_edge(cupk_ctx *ctx, const cupk_bucket *sketch, uint32_t *u, uint32_t *v)
{
    int32_t st = 0;
    uint32_t a = 0, b = 0;
    int rc = cupk_sample_cut_edge_batch(ctx, sketch, 1, &st, &a, &b);
    if (rc != CUPK_OK) return rc;
    if (u) *u = a;
    if (v) *v = b;
    return st;
}

int cupk_connected(cupk_ctx *ctx, uint32_t u, uint32_t v)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (u >= ctx->V || v >= ctx->V) return ctx->invalid("vertex id >= V");
        // the forest is complete once pending host work has run; the sketch
        // may still be in flight but queries do not read it
        return ctx->forest.same_tree(u, v) ? 1 : 0;
    });
}

int cupk_get_sketch(cupk_ctx *ctx, uint32_t w0, uint32_t nv, cupk_bucket *out)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (nv == 0) return CUPK_OK;
        if (!out) return ctx->invalid("null out");
        if ((uint64_t)w0 + nv > ctx->V) return ctx->invalid("vertex range beyond V");
        const uint32_t step = 4096;
        HIPCHK(grow(ctx->d_tmp, (size_t)step * ctx->W));
        for (uint32_t o = 0; o < nv; o += step) {
            const uint32_t m = std::min(step, nv - o);
            HIPCHK(launch_to_canonical(ctx->s, ctx->d_sk + (uint64_t)(w0 + o) * ctx->W, ctx->C, ctx->D,
                                       m, ctx->d_tmp.p));
            HIPCHK(hipMemcpyAsync(out + (size_t)o * ctx->C * ctx->D, ctx->d_tmp.p,
                                  (size_t)m * ctx->W * 8, hipMemcpyDeviceToHost, ctx->s));
            HIPCHK(hipStreamSynchronize(ctx->s));
        }
        return CUPK_OK;
    });
}

int cupk_digest(cupk_ctx *ctx, uint64_t *out)
{
    if (!ctx || !out) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        HIPCHK(launch_zero(ctx->s, ctx->d_misc, 1));
        HIPCHK(launch_digest(ctx->s, dev_sketch(ctx), ctx->S, ctx->d_misc));
        HIPCHK(hipMemcpyAsync(ctx->h_misc, ctx->d_misc, 8, hipMemcpyDeviceToHost, ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->s));
        *out = ctx->h_misc[0];
        return CUPK_OK;
    });
}

int cupk_num_components(cupk_ctx *ctx, uint64_t *out)
{
    if (!ctx || !out) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        *out = ctx->forest.n_trees();
        return CUPK_OK;
    });
}

int cupk_forest_edges(cupk_ctx *ctx, uint32_t *u, uint32_t *v, size_t cap, size_t *n)
{
    if (!ctx || !n) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        std::vector<uint32_t> eu, ev;
        ctx->forest.edges(eu, ev);
        *n = eu.size();
        if (cap < eu.size()) return ctx->invalid("forest edge buffer too small");
        if (eu.size() && (!u || !v)) return ctx->invalid("null array");
        std::copy(eu.begin(), eu.end(), u);
        std::copy(ev.begin(), ev.end(), v);
        return CUPK_OK;
    });
}

int cupk_level_forest_edges(cupk_ctx *ctx, uint32_t level, uint32_t *u, uint32_t *v, size_t cap,
                            size_t *n)
{
    if (!ctx || !n) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (!ctx->levels) return ctx->invalid("not in levels mode");
        if (level < 1 || level > ctx->levels->top) return ctx->invalid("level out of range");
        std::vector<uint32_t> eu, ev;
        levels_edges(ctx, level, eu, ev);
        *n = eu.size();
        if (cap < eu.size()) return ctx->invalid("forest edge buffer too small");
        if (eu.size() && (!u || !v)) return ctx->invalid("null array");
        std::copy(eu.begin(), eu.end(), u);
        std::copy(ev.begin(), ev.end(), v);
        return CUPK_OK;
    });
}

int cupk_component_labels(cupk_ctx *ctx, uint32_t *out)
{
    if (!ctx || !out) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        for (uint32_t w = 0; w < ctx->V; w++) out[w] = ctx->forest.label(w);
        return CUPK_OK;
    });
}

int cupk_counters(cupk_ctx *ctx, cupk_counters_t *out)
{
    if (!ctx || !out) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        int rc = harvest_timers(ctx, true);
        if (rc != CUPK_OK) return rc;
        HIPCHK(hipMemcpyAsync(ctx->h_misc + 1, ctx->d_touched, 8, hipMemcpyDeviceToHost,
                              ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->s));
        ctx->ctr.timed_buckets = ctx->h_misc[1];
        *out = ctx->ctr;
        return CUPK_OK;
    });
}

int cupk_sync(cupk_ctx *ctx)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        HIPCHK(hipStreamSynchronize(ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->cs));
        return harvest_timers(ctx, true);
    });
}

// Time the bin + scatter of `n` sample updates (one application) with the
// geometry in force, reading the tile counts from a classify pass.
static int time_scatter_once(cupk_ctx *ctx, const uint64_t *d, uint32_t n, hipEvent_t e0,
                             hipEvent_t e1, float *ms)
{
    int rc = ensure_batch_buffers(ctx, n);
    if (rc != CUPK_OK) return rc;
    ctx->cur_desc.upd = d;
    ctx->cur_desc.n = n;
    HIPCHK(hipEventRecord(e0, ctx->s));
    rc = enqueue_classify(ctx, ctx->s, n);
    ctx->hdr_seq++;  // published by the scan kernel (read after the sync below)
    if (rc != CUPK_OK) return rc;
    rc = enqueue_bin(ctx, ctx->s, n);
    if (rc == CUPK_OK) rc = enqueue_tile(ctx, ctx->s, n, false);
    if (rc != CUPK_OK) return rc;
    HIPCHK(hipEventRecord(e1, ctx->s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    if (ctx->h_hdr[HDR_ERR]) return ctx->invalid("sample batch holds an invalid update");
    return CUPK_OK;
}

// Median over `reps` pairs of applications (each pair cancels out).
static int time_scatter(cupk_ctx *ctx, const uint64_t *d, uint32_t n, int reps, hipEvent_t e0,
                        hipEvent_t e1, double *out_ms)
{
    std::vector<float> t;
    for (int r = 0; r < reps; r++)
        for (int k = 0; k < 2; k++) {
            float ms = 0;
            int rc = time_scatter_once(ctx, d, n, e0, e1, &ms);
            if (rc != CUPK_OK) return rc;
            t.push_back(ms);
        }
    std::sort(t.begin(), t.end());
    *out_ms = t[t.size() / 2];
    return CUPK_OK;
}

// Boruvka over supernodes on the resident sketch (see cupk.h).  Round 1
// samples every vertex sketch in place; round 2 reduces the new supernodes
// from their vertices, later rounds from the previous round's supernode
// sketches (each new supernode is a union of previous active ones).
static int static_components(cupk_ctx *ctx, uint32_t *labels, uint32_t *eu, uint32_t *ev,
                             cupk_static_info *info)
{
    const uint32_t V = ctx->V, W = ctx->W;
    std::vector<uint32_t> parent(V), size(V, 1);
    for (uint32_t w = 0; w < V; w++) parent[w] = w;
    auto find = [&](uint32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    };
    std::vector<uint32_t> edges_u, edges_v;
    uint32_t rounds = 0, failed = 0;
    // active sets of the current round, ascending smallest vertex
    std::vector<uint32_t> set_min, set_size;
    std::vector<uint32_t> vmem, voff, fmem, foff;
    int slot = 0;
    bool first = true;
    for (;;) {
        uint32_t k;
        const int32_t *res;
        rounds++;
        if (first) {
            k = V;
            set_min.resize(V);
            set_size.assign(V, 1);
            for (uint32_t w = 0; w < V; w++) set_min[w] = w;
            HIPCHK(grow(ctx->d_res, (size_t)3 * V));
            HIPCHK(grow(ctx->h_res, (size_t)3 * V));
            HIPCHK(launch_sample(ctx->s, ctx->d_sk, V, V, ctx->C, ctx->D, 1, ctx->C, W,
                                 ctx->d_seeds, ctx->d_res.p));
            HIPCHK(hipMemcpyAsync(ctx->h_res.p, ctx->d_res.p, (size_t)3 * V * 4,
                                  hipMemcpyDeviceToHost, ctx->s));
            HIPCHK(hipStreamSynchronize(ctx->s));
        } else {
            k = (uint32_t)set_min.size();
            int rc = reduce_and_sample(ctx, slot, vmem, voff, fmem, foff);
            if (rc != CUPK_OK) return rc;
        }
        res = ctx->h_res.p;
        bool merged = false;
        for (uint32_t i = 0; i < k; i++) {
            if (res[3 * i] != CUPK_OK) continue;
            const uint32_t x = (uint32_t)res[3 * i + 1], y = (uint32_t)res[3 * i + 2];
            const uint32_t rx = find(x), ry = find(y);
            if (rx == ry) continue;
            parent[rx] = ry;
            size[ry] += size[rx];
            edges_u.push_back(std::min(x, y));
            edges_v.push_back(std::max(x, y));
            merged = true;
        }
        // next round: every supernode with an active part, except EMPTY
        // ones that nothing joined.  Sets are kept in ascending order of
        // smallest vertex, so numbering the supernodes in order of their
        // first part numbers them in that order too.
        std::vector<int32_t> &gid = ctx->round_gmap;  // by root vertex
        if (gid.size() != V) gid.assign(V, -1);
        std::vector<uint32_t> part_gid(k), gcount, nmin, nsize;
        uint32_t ng = 0;
        for (uint32_t i = 0; i < k; i++) {
            const int st = res[3 * i];
            const uint32_t r = find(set_min[i]);
            if (st == CUPK_SAMPLE_FAILED) failed++;
            if (st == CUPK_EMPTY && size[r] == set_size[i]) {
                part_gid[i] = UINT32_MAX;
                continue;
            }
            if (gid[r] < 0) {
                gid[r] = (int32_t)ng++;
                gcount.push_back(0);
                nmin.push_back(set_min[i]);
                nsize.push_back(0);
            }
            const uint32_t g = (uint32_t)gid[r];
            part_gid[i] = g;
            gcount[g]++;
            nsize[g] += set_size[i];
        }
        for (uint32_t i = 0; i < k; i++)
            if (part_gid[i] != UINT32_MAX) gid[find(set_min[i])] = -1;
        if (!merged || ng == 0) break;
        vmem.clear();
        voff.clear();
        fmem.clear();
        foff.clear();
        std::vector<uint32_t> &mem = first ? vmem : fmem;
        std::vector<uint32_t> &off = first ? voff : foff;
        off.assign(ng + 1, 0);
        for (uint32_t g = 0; g < ng; g++) off[g + 1] = off[g] + gcount[g];
        mem.resize(off[ng]);
        std::vector<uint32_t> fill(off.begin(), off.end() - 1);
        for (uint32_t i = 0; i < k; i++)
            if (part_gid[i] != UINT32_MAX)
                mem[fill[part_gid[i]]++] = first ? set_min[i] : i;  // round 1 sets are vertices
        set_min.swap(nmin);
        set_size.swap(nsize);
        if (!first) slot = 1 - slot;
        first = false;
    }
    // labels: smallest vertex of each final supernode
    std::vector<uint32_t> low(V, 0xffffffffu);
    uint32_t ncomp = 0;
    for (uint32_t w = 0; w < V; w++) {
        const uint32_t r = find(w);
        if (low[r] == 0xffffffffu) {
            low[r] = w;
            ncomp++;
        }
        if (labels) labels[w] = low[r];
    }
    if (eu && ev) {
        std::copy(edges_u.begin(), edges_u.end(), eu);
        std::copy(edges_v.begin(), edges_v.end(), ev);
    }
    if (info) {
        info->n_components = ncomp;
        info->rounds = rounds;
        info->sample_failed = failed;
        info->n_edges = (uint32_t)edges_u.size();
    }
    return CUPK_OK;
}

int cupk_static_components(cupk_ctx *ctx, uint32_t *labels, uint32_t *eu, uint32_t *ev,
                           cupk_static_info *info)
{
    if (!ctx) return CUPK_EINVAL;
    if (ctx->server) return ctx->invalid("static components while the serving loop runs");
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        return static_components(ctx, labels, eu, ev, info);
    });
}

int cupk_autotune(cupk_ctx *ctx, const uint64_t *d_sample, size_t n, cupk_tune_result *out)
{
    if (!ctx || !out || !d_sample) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (ctx->server) return ctx->invalid("autotune while the serving loop runs");
        if (ctx->opts.scatter_mode != CUPK_SCATTER_STAGED) return ctx->invalid("autotune needs staged mode");
        if (n == 0 || n > kMaxBatchPerLaunch) return ctx->invalid("bad sample size");
        *out = cupk_tune_result{};
        HIPCHK(hipStreamSynchronize(ctx->s));
        int rc = upload_forest(ctx);
        if (rc != CUPK_OK) return rc;
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const uint32_t tv0 = 1u << ctx->tile_shift, rows0 = ctx->rows, chunk0 = ctx->chunk;
        const uint32_t lay0 = ctx->layout;
        const uint32_t co0 = ctx->fshift ? 1u << ctx->fshift : 0u;
        const uint32_t m = (uint32_t)n;
        double before = 0;
        rc = time_scatter(ctx, d_sample, m, 1, e0, e1, &before);  // also warms up
        if (rc == CUPK_OK) rc = time_scatter(ctx, d_sample, m, 2, e0, e1, &before);
        double best = before;
        uint32_t btv = tv0, brows = rows0, bchunk = chunk0, blay = lay0, tried = 1;
        struct Cand {
            double ms;
            uint32_t tv, rows, chunk, lay;
        };
        std::vector<Cand> cands;
        cands.push_back({before, tv0, rows0, chunk0, lay0});
        const uint32_t lays[] = {CUPK_LAYOUT_RECORD, CUPK_LAYOUT_PAIR};
        const uint32_t tvs[] = {4, 8, 16, 32, 64};
        const uint32_t rowss[] = {6, 8, 10, 12};
        const uint32_t chunks[] = {2048, 4096, 8192};
        for (uint32_t lay : lays)
            for (uint32_t tv : tvs)
                for (uint32_t rows : rowss)
                    for (uint32_t ch : chunks) {
                        if (rc != CUPK_OK) break;
                        if (rows > ctx->D || !tile_geometry_fits(rows, ctx->C, tv,
                                                                 lay == CUPK_LAYOUT_PAIR
                                                                     ? kLayoutPair
                                                                     : kLayoutRecord))
                            continue;
                        if (tv == tv0 && rows == rows0 && ch == chunk0 && lay == lay0 && !co0)
                            continue;
                        rc = set_geometry(ctx, tv, rows, ch, lay, 0);
                        if (rc != CUPK_OK) break;
                        double ms = 0;
                        rc = time_scatter(ctx, d_sample, m, 2, e0, e1, &ms);
                        tried++;
                        if (ctx->trace)
                            fprintf(stderr, "cupk tune layout=%u tv=%u rows=%u chunk=%u %.4f ms\n",
                                    lay, tv, rows, ch, ms);
                        if (rc == CUPK_OK) cands.push_back({ms, tv, rows, ch, lay});
                        if (rc == CUPK_OK && ms < best) {
                            best = ms;
                            btv = tv;
                            brows = rows;
                            bchunk = ch;
                            blay = lay;
                        }
                    }
        // The best few again, in two alternating passes of twice the
        // repetitions: settings within a few percent of each other are
        // within the noise of one short timing, and a wrong pick among them
        // (say 10 LDS rows instead of 12) costs as much on every batch.
        if (rc == CUPK_OK && cands.size() > 1) {
            std::sort(cands.begin(), cands.end(),
                      [](const Cand &a, const Cand &b) { return a.ms < b.ms; });
            const size_t top = std::min<size_t>(4, cands.size());
            std::vector<double> sum(top, 0.0);
            for (int pass = 0; pass < 2 && rc == CUPK_OK; pass++)
                for (size_t i = 0; i < top && rc == CUPK_OK; i++) {
                    const Cand &c = cands[i];
                    rc = set_geometry(ctx, c.tv, c.rows, c.chunk, c.lay, 0);
                    double ms = 0;
                    if (rc == CUPK_OK) rc = time_scatter(ctx, d_sample, m, 2, e0, e1, &ms);
                    sum[i] += ms;
                    tried++;
                    if (ctx->trace)
                        fprintf(stderr, "cupk tune again layout=%u tv=%u rows=%u chunk=%u %.4f ms\n",
                                c.lay, c.tv, c.rows, c.chunk, ms);
                }
            if (rc == CUPK_OK) {
                size_t bi = 0;
                for (size_t i = 1; i < top; i++)
                    if (sum[i] < sum[bi]) bi = i;
                btv = cands[bi].tv;
                brows = cands[bi].rows;
                bchunk = cands[bi].chunk;
                blay = cands[bi].lay;
                best = sum[bi] / 2;
            }
        }
        if (rc == CUPK_OK) rc = set_geometry(ctx, btv, brows, bchunk, blay, 0);
        // two-level binning: coarse bins from the default size down to 1/32
        // of it, and twice it (where the records fall on a few tiles, smaller
        // coarse bins keep the second fill's runs long)
        uint32_t bco = 0;
        if (rc == CUPK_OK && ctx->fshift) {
            const uint32_t f0 = ctx->fshift;
            double best_co = 0;
            rc = time_scatter(ctx, d_sample, m, 2, e0, e1, &best_co);
            best = std::min(best, best_co);
            bco = 1u << f0;
            for (uint32_t f = f0 + 1; rc == CUPK_OK && f + 5 >= f0 && f >= 1; f--) {
                if (f == f0) continue;
                const uint32_t co = 1u << f;
                if (co > kFineLdsTiles ||
                    (((uint64_t)ctx->ntiles + co - 1) >> f) > kLdsHistMax)
                    continue;
                rc = set_geometry(ctx, btv, brows, bchunk, blay, co);
                if (rc != CUPK_OK) break;
                double ms = 0;
                rc = time_scatter(ctx, d_sample, m, 2, e0, e1, &ms);
                tried++;
                if (ctx->trace)
                    fprintf(stderr, "cupk tune coarse_tiles=%u %.4f ms\n", co, ms);
                if (rc == CUPK_OK && ms < best_co) {
                    best_co = ms;
                    bco = co;
                }
                if (f == 1) break;
            }
            best = std::min(best, best_co);
            if (rc == CUPK_OK) rc = set_geometry(ctx, btv, brows, bchunk, blay, bco);
        }
        // batch-size schedule: device time of prefixes n/128 .. n, plus the
        // host time per batch (flag walk and replacement rounds, which cost
        // about the same whatever the batch size) measured on this
        // context's batches so far; the target is the smallest prefix whose
        // whole-path rate reaches 80% of the best one
        const double host_ms = ctx->ctr.batches
                                   ? (ctx->ctr.host_flags_ms + ctx->ctr.host_rounds_ms) /
                                         (double)ctx->ctr.batches
                                   : 0.0;
        out->host_ms_per_batch = host_ms;
        double best_rate = 0;
        for (int k = 0; k < 8 && rc == CUPK_OK; k++) {
            const uint32_t sz = std::max<uint32_t>(1, m >> (7 - k));
            double ms = 0;
            rc = time_scatter(ctx, d_sample, sz, 2, e0, e1, &ms);
            out->batch_sizes[k] = sz;
            out->batch_ms[k] = ms;
            if (ms + host_ms > 0) best_rate = std::max(best_rate, sz / (ms + host_ms));
        }
        if (rc == CUPK_OK) {
            out->batch_target = m;
            for (int k = 0; k < 8; k++)
                if (out->batch_ms[k] + host_ms > 0 &&
                    out->batch_sizes[k] / (out->batch_ms[k] + host_ms) >= 0.8 * best_rate) {
                    out->batch_target = out->batch_sizes[k];
                    break;
                }
            ctx->tuned_batch = out->batch_target;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != CUPK_OK) {
            (void)set_geometry(ctx, tv0, rows0, chunk0, lay0, co0);
            return rc;
        }
        out->tile_layout = blay;
        out->tile_vertices = btv;
        out->lds_rows = brows;
        out->chunk_records = bchunk;
        out->coarse_tiles = bco;
        out->candidates = tried;
        out->best_ms = best;
        out->before_ms = before;
        return CUPK_OK;
    });
}

int cupk_serve_start(cupk_ctx *ctx, const cupk_serve_opts *opts)
{
    if (!ctx) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        CUPK_FLUSH();
        if (ctx->server) return ctx->invalid("serving loop already running");
        cupk_serve_opts o = {};
        if (opts) o = *opts;
        // the autotuner's batch-size schedule, unless the caller sets one
        if (o.max_batch == 0 && ctx->tuned_batch) o.max_batch = ctx->tuned_batch;
        HIPCHK(hipStreamSynchronize(ctx->s));
        const int dev = ctx->device;
        ctx->server.reset(new (std::nothrow) Server(
            ctx, o,
            [](cupk_ctx *c, const uint64_t *d, size_t n, hipEvent_t ready) -> int {
                static thread_local int bound = -1;
                if (bound != c->device) {
                    if (hipSetDevice(c->device) != hipSuccess) return CUPK_EDEVICE;
                    bound = c->device;
                }
                // the batch sits in the server's device ring once its
                // upload (on the server's copy stream) is done
                if (ready && hipStreamWaitEvent(c->s, ready, 0) != hipSuccess)
                    return CUPK_EDEVICE;
                c->query_often = true;
                const int rc = apply_device(c, d, n, false);
                c->query_often = false;
                return rc;
            },
            connected_impl));
        (void)dev;
        if (!ctx->server) return CUPK_ENOMEM;
        const int src = ctx->server->start();
        if (src != CUPK_OK) {
            ctx->server.reset();
            return src == CUPK_ENOMEM ? ctx->fail(hipErrorOutOfMemory, "serving ring", __LINE__)
                                      : ctx->fail(hipErrorUnknown, "serving ring", __LINE__);
        }
        return CUPK_OK;
    });
}

int cupk_submit_updates(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v,
                        const uint8_t *is_delete, size_t n, uint64_t *ticket)
{
    if (!ctx || !ctx->server || !ticket) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        if (n && (!u || !v || !is_delete)) return CUPK_EINVAL;
        return ctx->server->submit_updates(u, v, is_delete, n, ctx->V, ticket);
    });
}

int cupk_submit_query(cupk_ctx *ctx, uint32_t u, uint32_t v, uint64_t *ticket)
{
    if (!ctx || !ctx->server || !ticket) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        return ctx->server->submit_query(u, v, ctx->V, ticket);
    });
}

int cupk_submit_queries(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v, size_t n,
                        int32_t *out, uint64_t *ticket)
{
    if (!ctx || !ctx->server || !ticket) return CUPK_EINVAL;
    if (n && (!u || !v || !out)) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        return ctx->server->submit_queries(u, v, n, out, ctx->V, ticket);
    });
}

int cupk_wait(cupk_ctx *ctx, uint64_t ticket, int32_t *result)
{
    if (!ctx || !ctx->server) return CUPK_EINVAL;
    return ctx->server->wait(ticket, result);
}

int cupk_serve_stats(cupk_ctx *ctx, cupk_serve_stats_t *out)
{
    if (!ctx || !ctx->server || !out) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        ctx->server->get_stats(out);
        return CUPK_OK;
    });
}

int cupk_serve_reset_stats(cupk_ctx *ctx)
{
    if (!ctx || !ctx->server) return CUPK_EINVAL;
    ctx->server->reset_stats();
    return CUPK_OK;
}

int cupk_serve_stop(cupk_ctx *ctx)
{
    if (!ctx || !ctx->server) return CUPK_EINVAL;
    return guarded(ctx, [&]() -> int {
        ctx->server.reset();  // drains the queue, joins the worker
        HIPCHK(hipStreamSynchronize(ctx->s));
        return CUPK_OK;
    });
}

const char *cupk_strerror(int code)
{
    switch (code) {
    case CUPK_OK: return "ok";
    case CUPK_EMPTY: return "empty: the aggregate sketch is zero";
    case CUPK_SAMPLE_FAILED: return "sample failed: no bucket verifies";
    case CUPK_EINVAL: return "invalid argument";
    case CUPK_ENOMEM: return "out of memory";
    case CUPK_EDEVICE: return "HIP device error";
    case CUPK_EBUSY: return "busy: admission refused";
    default: return "unknown code";
    }
}

const char *cupk_last_error(cupk_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

}  // extern "C"
