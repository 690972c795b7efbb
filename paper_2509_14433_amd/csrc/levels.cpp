// Multi-level hierarchy: see levels.hpp.
#include "levels.hpp"

namespace cupk {

namespace {

Forest &level_forest(cupk_ctx *ctx, uint32_t j)
{
    return j == ctx->levels->top ? ctx->forest : ctx->levels->lv[j]->F;
}

// Weight of top-forest edge {a, b}: the lowest level whose forest holds it.
uint32_t weight_of(cupk_ctx *ctx, uint32_t a, uint32_t b)
{
    Levels &L = *ctx->levels;
    for (uint32_t j = 1; j < L.top; j++)
        if (L.lv[j]->F.is_edge(a, b)) return j;
    return L.top;
}

// Remove forest edge {a, b} from every level from its weight w up.
void remove_from(cupk_ctx *ctx, uint32_t a, uint32_t b, uint32_t w)
{
    Levels &L = *ctx->levels;
    for (uint32_t j = w; j < L.top; j++) L.lv[j]->F.cut(a, b);
    ctx->forest.cut(a, b);
    ctx->ctr.cuts++;
    ctx->forest_dev_stale = true;
}

// The heaviest edge on the top-forest path between x and y (ties: the
// smaller edge (a, b), a < b): its weight, or 0 when x and y are not
// connected.  The path meets at the lowest common ancestor of the rooted
// top forest.
uint32_t heaviest_on_path(cupk_ctx *ctx, uint32_t x, uint32_t y, uint32_t &ea, uint32_t &eb)
{
    Forest &T = ctx->forest;
    if (!T.same_tree(x, y)) return 0;
    Levels &L = *ctx->levels;
    if (++L.epoch == 0) {
        std::fill(L.mark.begin(), L.mark.end(), 0u);
        L.epoch = 1;
    }
    const uint32_t ep = L.epoch;
    for (uint32_t a = x; a != kNone; a = T.parent(a)) L.mark[a] = ep;
    uint32_t lca = y;
    while (L.mark[lca] != ep) lca = T.parent(lca);
    uint32_t best = 0;
    ea = eb = 0;
    auto consider = [&](uint32_t c) {
        const uint32_t p = T.parent(c);
        const uint32_t lo = std::min(c, p), hi = std::max(c, p);
        const uint32_t w = weight_of(ctx, lo, hi);
        if (w > best || (w == best && (lo < ea || (lo == ea && hi < eb)))) {
            best = w;
            ea = lo;
            eb = hi;
        }
    };
    for (uint32_t c = x; c != lca; c = T.parent(c)) consider(c);
    for (uint32_t c = y; c != lca; c = T.parent(c)) consider(c);
    return best;
}

// A component that may violate Invariant 3 at its level; members
// mem[mb, me).
struct Cand {
    uint32_t level, minv, size, mb, me;
};

// Components of F_i, i in [lo, top), that are as large as their level-(i+1)
// component (the others satisfy Invariant 3 whatever their query returns);
// level by level, each in ascending order of smallest vertex.
void gather(cupk_ctx *ctx, uint32_t lo, std::vector<Cand> &cands, std::vector<uint32_t> &mem)
{
    Levels &L = *ctx->levels;
    for (uint32_t i = lo; i < L.top; i++) {
        Forest &N = level_forest(ctx, i + 1);
        const size_t c0 = cands.size();
        if (i == 0) {
            // singletons of F_1
            for (uint32_t l : N.live_labels())
                if (N.tree_size(l) == 1) {
                    const uint32_t w = N.tree_root(l);
                    const uint32_t mb = (uint32_t)mem.size();
                    mem.push_back(w);
                    cands.push_back({0, w, 1, mb, mb + 1});
                }
        } else {
            Forest &F = L.lv[i]->F;
            uint32_t giant = kNone, giant_sz = 0;
            for (uint32_t l : F.live_labels()) {
                const uint32_t w = F.tree_root(l);
                const uint32_t sz = F.tree_size(l);
                if (N.tree_size(N.label(w)) != sz) continue;
                if (2 * (uint64_t)sz > ctx->V) {
                    giant = l;
                    giant_sz = sz;
                    continue;
                }
                const uint32_t mb = (uint32_t)mem.size();
                const uint32_t mn = F.collect(l, mem);
                cands.push_back({i, mn, sz, mb, (uint32_t)mem.size()});
            }
            if (giant != kNone) {
                // Every edge adds the same words to both endpoints, so the
                // sketches of all vertices XOR to zero and a set's aggregate
                // equals its complement's: a tree holding most vertices is
                // reduced over the other trees' vertices.
                const uint32_t mb = (uint32_t)mem.size();
                for (uint32_t l : F.live_labels())
                    if (l != giant) F.collect(l, mem);
                if (++L.epoch == 0) {
                    std::fill(L.mark.begin(), L.mark.end(), 0u);
                    L.epoch = 1;
                }
                for (size_t q = mb; q < mem.size(); q++) L.mark[mem[q]] = L.epoch;
                uint32_t mn = 0;
                while (L.mark[mn] == L.epoch) mn++;  // smallest vertex of the giant
                cands.push_back({i, mn, giant_sz, mb, (uint32_t)mem.size()});
            }
        }
        std::sort(cands.begin() + (long)c0, cands.end(),
                  [](const Cand &a, const Cand &b) { return a.minv < b.minv; });
    }
}

// One launch pair over all candidates: one-column reduction of each
// candidate's members, then its level's query; results in ctx->h_res.
int query_cands(cupk_ctx *ctx, const std::vector<Cand> &cands, const std::vector<uint32_t> &mem)
{
    Levels &L = *ctx->levels;
    const uint32_t k = (uint32_t)cands.size();
    const uint32_t W2 = 2 * ctx->D;
    size_t nitems = 0;
    for (const Cand &c : cands) nitems += (c.me - c.mb + kRedChunk - 1) / kRedChunk;
    HIPCHK(grow(L.h_col, k));
    HIPCHK(grow(L.d_col, k));
    HIPCHK(grow(L.h_idx, mem.size() + 1));
    HIPCHK(grow(L.d_idx, mem.size() + 1));
    HIPCHK(grow(L.h_items, 3 * nitems + 1));
    HIPCHK(grow(L.d_items, 3 * nitems + 1));
    HIPCHK(grow(L.d_agg, (size_t)k * W2));
    HIPCHK(grow(ctx->d_res, (size_t)3 * k));
    HIPCHK(grow(ctx->h_res, (size_t)3 * k));
    uint32_t *it = L.h_items.p;
    for (uint32_t j = 0; j < k; j++) {
        L.h_col.p[j] = cands[j].level;
        for (uint32_t b = cands[j].mb; b < cands[j].me; b += kRedChunk) {
            *it++ = j;
            *it++ = b;
            *it++ = std::min(cands[j].me, b + kRedChunk);
        }
    }
    std::copy(mem.begin(), mem.end(), L.h_idx.p);
    hipStream_t s = ctx->s;
    HIPCHK(hipMemcpyAsync(L.d_col.p, L.h_col.p, (size_t)k * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(L.d_idx.p, L.h_idx.p, mem.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(L.d_items.p, L.h_items.p, 3 * nitems * 4, hipMemcpyHostToDevice, s));
    HIPCHK(launch_zero(s, L.d_agg.p, (size_t)k * W2));
    HIPCHK(launch_reduce_col(s, ctx->d_sk, ctx->C, ctx->D, L.d_idx.p, L.d_items.p,
                             (uint32_t)nitems, L.d_col.p, L.d_agg.p));
    HIPCHK(launch_sample_col(s, L.d_agg.p, k, ctx->V, ctx->D, L.d_col.p, ctx->d_seeds,
                             ctx->d_res.p));
    HIPCHK(hipMemcpyAsync(ctx->h_res.p, ctx->d_res.p, (size_t)3 * k * 4, hipMemcpyDeviceToHost,
                          s));
    // the pinned staging above is written again by the next pass
    HIPCHK(hipStreamSynchronize(s));
    ctx->ctr.sets_reduced += k;
    ctx->ctr.slabs_reduced += mem.size();
    return CUPK_OK;
}

}  // namespace

int levels_init(cupk_ctx *ctx)
{
    std::unique_ptr<Levels> L(new Levels());
    L->top = ctx->C;
    L->lv.resize(ctx->C);
    for (uint32_t j = 1; j < ctx->C; j++) {
        std::unique_ptr<Level> lv(new Level());
        lv->lbl.resize(ctx->V);
        lv->par.resize(ctx->V);
        lv->F.init(ctx->V, lv->lbl.data(), lv->par.data());
        L->lv[j] = std::move(lv);
    }
    L->mark.assign(ctx->V, 0);
    ctx->levels = std::move(L);
    return CUPK_OK;
}

void levels_release(cupk_ctx *ctx)
{
    if (!ctx->levels) return;
    Levels &L = *ctx->levels;
    release(L.d_col);
    release(L.d_idx);
    release(L.d_items);
    release(L.h_col);
    release(L.h_idx);
    release(L.h_items);
    release(L.d_agg);
}

bool levels_delete(cupk_ctx *ctx, uint32_t a, uint32_t b)
{
    if (!ctx->forest.is_edge(a, b)) return false;
    remove_from(ctx, a, b, weight_of(ctx, a, b));
    return true;
}

int levels_restore(cupk_ctx *ctx)
{
    Levels &L = *ctx->levels;
    std::vector<Cand> cands;
    std::vector<uint32_t> mem;
    uint32_t lo = 0;
    while (lo < L.top) {
        ctx->ctr.level_passes++;
        const double t0 = now_ms();
        cands.clear();
        mem.clear();
        gather(ctx, lo, cands, mem);
        if (cands.empty()) break;
        const double t1 = now_ms();
        int rc = query_cands(ctx, cands, mem);
        if (rc != CUPK_OK) return rc;
        const double t2 = now_ms();
        const int32_t *res = ctx->h_res.p;
        uint32_t found = UINT32_MAX;
        for (size_t j = 0; j < cands.size(); j++)
            if (res[3 * j] == CUPK_OK) found = std::min(found, cands[j].level);
        // failed queries at the levels this pass looked at: up to the
        // repaired level (levels above it are queried again next pass)
        for (size_t j = 0; j < cands.size(); j++)
            if (res[3 * j] == CUPK_SAMPLE_FAILED && cands[j].level <= found)
                ctx->ctr.level_failed++;
        if (found == UINT32_MAX) break;
        const uint32_t i = found;
        Forest &N = level_forest(ctx, i + 1);
        for (size_t j = 0; j < cands.size(); j++) {
            if (cands[j].level != i || res[3 * j] != CUPK_OK) continue;
            const uint32_t x = (uint32_t)res[3 * j + 1], y = (uint32_t)res[3 * j + 2];
            // the sampled edge leaves the component: find its endpoint inside
            uint32_t inside;
            if (i == 0) {
                inside = x == cands[j].minv ? x : y;
            } else {
                Forest &F = L.lv[i]->F;
                inside = F.label(x) == F.label(cands[j].minv) ? x : y;
            }
            // joined by an earlier repair of this pass
            if (N.tree_size(N.label(inside)) != cands[j].size) continue;
            uint32_t ea, eb;
            const uint32_t w = heaviest_on_path(ctx, x, y, ea, eb);
            // from the cycle edge's weight up, (x, y) replaces it inside one
            // tree (no split, no relabelling); below that it joins two trees
            const uint32_t swap_from = w ? w : L.top + 1;
            for (uint32_t l = i + 1; l <= L.top; l++) {
                Forest &G = level_forest(ctx, l);
                if (l >= swap_from)
                    G.swap_edge(ea, eb, x, y);
                else
                    G.link(x, y);
            }
            if (w) ctx->ctr.cuts++;
            ctx->forest_dev_stale = true;
            ctx->ctr.links++;
            ctx->ctr.level_repairs++;
        }
        if (ctx->trace)
            fprintf(stderr,
                    "cupk   levels pass lo=%u level=%u cands=%zu members=%zu gather=%.3f "
                    "gpu=%.3f repairs=%.3f ms\n",
                    lo, i, cands.size(), mem.size(), t1 - t0, t2 - t1, now_ms() - t2);
        lo = i + 1;
    }
    for (uint32_t j = 1; j < L.top; j++) L.lv[j]->F.discard_dirty();
    // top completion: replacement rounds over every top-level tree
    ctx->forest.mark_all_dirty();
    return run_rounds(ctx);
}

void levels_edges(cupk_ctx *ctx, uint32_t level, std::vector<uint32_t> &eu,
                  std::vector<uint32_t> &ev)
{
    if (level == 0) return;
    level_forest(ctx, level).edges(eu, ev);
}

}  // namespace cupk
