/*
 * Seeded synthetic update streams that are too long to draw in Python.
 * Input generation only: no hashing, sketching or forest logic of the
 * method lives here.  Randomness: xoshiro256** (Blackman, Vigna 2018),
 * state filled from the 64-bit seed with SplitMix64 as its authors suggest.
 *
 * Every stream is legal in the graph-stream model: an edge is inserted only
 * when absent and deleted only when present, u < v, no self loops.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s[4];
} rng_t;

static uint64_t sm_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed)
{
    uint64_t x = seed;
    for (int i = 0; i < 4; i++) r->s[i] = sm_next(&x);
}

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r)
{
    uint64_t *s = r->s;
    const uint64_t out = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return out;
}

static double rng_unif(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform in [0, n) (n > 0), by rejection */
static uint64_t rng_below(rng_t *r, uint64_t n)
{
    const uint64_t lim = UINT64_MAX - UINT64_MAX % n;
    uint64_t x;
    do {
        x = rng_next(r);
    } while (x >= lim);
    return x % n;
}

static int bit_get(const uint64_t *bm, uint64_t k) { return (bm[k >> 6] >> (k & 63)) & 1; }
static void bit_set(uint64_t *bm, uint64_t k) { bm[k >> 6] |= 1ULL << (k & 63); }
static void bit_clr(uint64_t *bm, uint64_t k) { bm[k >> 6] &= ~(1ULL << (k & 63)); }

/*
 * R-MAT stream with interleaved deletions, drawn in resumable pieces.
 * At each step, with probability del_prob (if any edge is live) a uniformly
 * random live edge is deleted; otherwise an R-MAT edge (quadrant
 * probabilities a, b, c, 1-a-b-c over logV levels) is drawn, canonicalised
 * to u < v and inserted; self loops and live pairs are re-drawn (after 64
 * failed R-MAT draws, uniform pairs are drawn instead).
 */
typedef struct {
    rng_t r;
    uint32_t logV;
    uint64_t V;
    uint64_t *bm;   /* live pairs, V*V bits */
    uint64_t *live; /* live edge keys */
    size_t nlive, cap;
} rmat_t;

void *sg_rmat_new(uint32_t logV, uint64_t seed, size_t max_live)
{
    rmat_t *g = (rmat_t *)calloc(1, sizeof(rmat_t));
    if (!g) return NULL;
    g->logV = logV;
    g->V = 1ULL << logV;
    g->bm = (uint64_t *)calloc((g->V * g->V + 63) / 64, 8);
    g->cap = max_live ? max_live : 1;
    g->live = (uint64_t *)malloc(sizeof(uint64_t) * g->cap);
    if (!g->bm || !g->live) {
        free(g->bm);
        free(g->live);
        free(g);
        return NULL;
    }
    rng_seed(&g->r, seed);
    return g;
}

void sg_rmat_free(void *h)
{
    rmat_t *g = (rmat_t *)h;
    if (!g) return;
    free(g->bm);
    free(g->live);
    free(g);
}

/* Next n updates; returns n, or 0 if the live list would overflow. */
size_t sg_rmat_next(void *h, size_t n, double del_prob, double a, double b, double c,
                    uint32_t *u, uint32_t *v, uint8_t *d)
{
    rmat_t *g = (rmat_t *)h;
    rng_t *r = &g->r;
    const uint64_t V = g->V;
    const double ab = a + b, abc = a + b + c;
    for (size_t i = 0; i < n; i++) {
        if (g->nlive > 0 && rng_unif(r) < del_prob) {
            const uint64_t j = rng_below(r, g->nlive);
            const uint64_t key = g->live[j];
            g->live[j] = g->live[--g->nlive];
            bit_clr(g->bm, key);
            u[i] = (uint32_t)(key / V);
            v[i] = (uint32_t)(key % V);
            d[i] = 1;
            continue;
        }
        if (g->nlive >= g->cap) return 0;
        uint64_t x, y, key;
        int tries = 0;
        for (;;) {
            if (tries < 64) {
                x = 0;
                y = 0;
                for (uint32_t l = 0; l < g->logV; l++) {
                    const double q = rng_unif(r);
                    const int bx = q >= ab;                       /* quadrants c, d */
                    const int by = (q >= a && q < ab) || q >= abc; /* quadrants b, d */
                    x = (x << 1) | (uint64_t)bx;
                    y = (y << 1) | (uint64_t)by;
                }
            } else {
                x = rng_below(r, V);
                y = rng_below(r, V);
            }
            tries++;
            if (x == y) continue;
            if (x > y) {
                const uint64_t t = x;
                x = y;
                y = t;
            }
            key = x * V + y;
            if (!bit_get(g->bm, key)) break;
        }
        bit_set(g->bm, key);
        g->live[g->nlive++] = key;
        u[i] = (uint32_t)x;
        v[i] = (uint32_t)y;
        d[i] = 0;
    }
    return n;
}

/* G(V, p) pairs u < v by geometric skipping over each row; returns the
 * number of edges written (at most cap). */
static size_t er_edges(rng_t *r, uint32_t V, double p, uint32_t *eu, uint32_t *ev, size_t cap)
{
    size_t m = 0;
    const double lq = p < 1.0 ? __builtin_log(1.0 - p) : 0.0;
    for (uint32_t x = 0; x + 1 < V; x++) {
        int64_t y = x;
        for (;;) {
            if (p >= 1.0) {
                y += 1;
            } else {
                double uu = rng_unif(r);
                if (uu <= 0.0) uu = 0x1.0p-53;
                y += 1 + (int64_t)(__builtin_log(uu) / lq);
            }
            if (y >= (int64_t)V) break;
            if (m >= cap) return m;
            eu[m] = x;
            ev[m] = (uint32_t)y;
            m++;
        }
    }
    return m;
}

static void shuffle2(rng_t *r, uint32_t *a, uint32_t *b, size_t m)
{
    for (size_t i = m; i > 1; i--) {
        const size_t j = (size_t)rng_below(r, i);
        uint32_t t = a[i - 1];
        a[i - 1] = a[j];
        a[j] = t;
        t = b[i - 1];
        b[i - 1] = b[j];
        b[j] = t;
    }
}

static uint32_t uf_find(uint32_t *p, uint32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

/*
 * Clustered churn.  Vertices [0, K*S) form K clusters of S vertices, each a
 * G(S, p_in); the other n_sparse vertices carry a sparse G(n, m = 2n).
 * Stream:
 *   1. the sparse edges, random order;
 *   2. bridges: a random tree over the clusters (cluster i to a random
 *      earlier cluster) plus extra_bridges random ones, each between random
 *      vertices of two different clusters;
 *   3. each cluster's first-arrival spanning forest (fixed forest);
 *   4. `rounds` times: insert every other cluster edge in random order, then
 *      delete them all in random order.
 * During phases 3-4, after every adv_every updates, adv_k bridges drawn
 * uniformly are toggled (deleted if present, re-inserted if absent).
 * Returns the number of updates written (at most cap), 0 on failure.
 */
size_t sg_clustered(uint32_t K, uint32_t S, double p_in, uint32_t n_sparse,
                    uint32_t extra_bridges, uint32_t rounds, uint32_t adv_every, uint32_t adv_k,
                    uint64_t seed, size_t cap, uint32_t *u, uint32_t *v, uint8_t *d)
{
    rng_t r;
    rng_seed(&r, seed);
    const uint32_t Vc = K * S;
    const uint32_t nb = K > 1 ? (K - 1) + extra_bridges : 0;
    const size_t per = (size_t)S * (S > 0 ? S - 1 : 0) / 2;
    const size_t mcap = (size_t)K * per + 1;
    const size_t msp = n_sparse >= 2 ? 2 * (size_t)n_sparse : 0;
    size_t hcap = 1;
    while (hcap < 4 * msp + 1) hcap <<= 1;
    size_t w = 0, since = 0, m = 0;
    int ok = 0;
    uint32_t *bu = (uint32_t *)malloc(sizeof(uint32_t) * (nb + 1));
    uint32_t *bv = (uint32_t *)malloc(sizeof(uint32_t) * (nb + 1));
    uint8_t *blive = (uint8_t *)calloc(nb + 1, 1);
    uint32_t *ce_u = (uint32_t *)malloc(sizeof(uint32_t) * mcap);
    uint32_t *ce_v = (uint32_t *)malloc(sizeof(uint32_t) * mcap);
    uint8_t *inf = (uint8_t *)calloc(mcap, 1);
    uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * (Vc + 1));
    uint64_t *hs = (uint64_t *)malloc(sizeof(uint64_t) * hcap);
    if (!bu || !bv || !blive || !ce_u || !ce_v || !inf || !par || !hs) goto done;
#define EMIT(a_, b_, del_)                   \
    do {                                     \
        if (w >= cap) goto done;             \
        const uint32_t x_ = (a_), y_ = (b_); \
        u[w] = x_ < y_ ? x_ : y_;            \
        v[w] = x_ < y_ ? y_ : x_;            \
        d[w] = (del_);                       \
        w++;                                 \
    } while (0)
#define ADV_TICK()                                                \
    do {                                                          \
        if (adv_every && nb && ++since >= adv_every) {            \
            since = 0;                                            \
            for (uint32_t t_ = 0; t_ < adv_k; t_++) {             \
                const uint32_t bi_ = (uint32_t)rng_below(&r, nb); \
                EMIT(bu[bi_], bv[bi_], blive[bi_] ? 1 : 0);       \
                blive[bi_] ^= 1;                                  \
            }                                                     \
        }                                                         \
    } while (0)
    /* 1. sparse part: m = 2n distinct random pairs (open-addressing set) */
    for (size_t i = 0; i < hcap; i++) hs[i] = UINT64_MAX;
    {
        const uint64_t nn = n_sparse;
        size_t got = 0;
        while (got < msp && (uint64_t)got < nn * (nn - 1) / 2) {
            uint64_t x = rng_below(&r, nn), y = rng_below(&r, nn);
            if (x == y) continue;
            if (x > y) {
                const uint64_t t = x;
                x = y;
                y = t;
            }
            const uint64_t key = x * nn + y;
            size_t h = (size_t)((key * 0x9E3779B97F4A7C15ULL) >> 17) & (hcap - 1);
            int dup = 0;
            while (hs[h] != UINT64_MAX) {
                if (hs[h] == key) {
                    dup = 1;
                    break;
                }
                h = (h + 1) & (hcap - 1);
            }
            if (dup) continue;
            hs[h] = key;
            got++;
            EMIT(Vc + (uint32_t)x, Vc + (uint32_t)y, 0);
        }
    }
    /* 2. bridges */
    {
        uint32_t q = 0;
        for (uint32_t i = 1; i < K; i++) {
            const uint32_t j = (uint32_t)rng_below(&r, i);
            bu[q] = i * S + (uint32_t)rng_below(&r, S);
            bv[q] = j * S + (uint32_t)rng_below(&r, S);
            q++;
        }
        while (q < nb) {
            const uint32_t i = (uint32_t)rng_below(&r, K), j = (uint32_t)rng_below(&r, K);
            if (i == j) continue;
            const uint32_t x = i * S + (uint32_t)rng_below(&r, S);
            const uint32_t y = j * S + (uint32_t)rng_below(&r, S);
            int dup = 0;
            for (uint32_t t = 0; t < q; t++)
                if ((bu[t] == x && bv[t] == y) || (bu[t] == y && bv[t] == x)) dup = 1;
            if (dup) continue;
            bu[q] = x;
            bv[q] = y;
            q++;
        }
        for (uint32_t t = 0; t < nb; t++) {
            EMIT(bu[t], bv[t], 0);
            blive[t] = 1;
        }
    }
    /* 3. clusters: edges, shuffled; first-arrival forest inserted once */
    for (uint32_t c = 0; c < K; c++) {
        const size_t m0 = m;
        m += er_edges(&r, S, p_in, ce_u + m, ce_v + m, mcap - m);
        for (size_t i = m0; i < m; i++) {
            ce_u[i] += c * S;
            ce_v[i] += c * S;
        }
    }
    shuffle2(&r, ce_u, ce_v, m);
    for (uint32_t x = 0; x < Vc; x++) par[x] = x;
    for (size_t i = 0; i < m; i++) {
        const uint32_t ra = uf_find(par, ce_u[i]), rb = uf_find(par, ce_v[i]);
        if (ra == rb) continue;
        par[ra] = rb;
        inf[i] = 1;
        EMIT(ce_u[i], ce_v[i], 0);
        ADV_TICK();
    }
    /* 4. churn of the other cluster edges, fresh random order each pass */
    for (uint32_t rd = 0; rd < rounds; rd++) {
        for (int pass = 0; pass < 2; pass++) {
            for (size_t i = m; i > 1; i--) {
                const size_t j = (size_t)rng_below(&r, i);
                uint32_t t = ce_u[i - 1];
                ce_u[i - 1] = ce_u[j];
                ce_u[j] = t;
                t = ce_v[i - 1];
                ce_v[i - 1] = ce_v[j];
                ce_v[j] = t;
                const uint8_t tf = inf[i - 1];
                inf[i - 1] = inf[j];
                inf[j] = tf;
            }
            for (size_t i = 0; i < m; i++) {
                if (inf[i]) continue;
                EMIT(ce_u[i], ce_v[i], pass);
                ADV_TICK();
            }
        }
    }
    ok = 1;
#undef ADV_TICK
#undef EMIT
done:
    free(bu);
    free(bv);
    free(blive);
    free(ce_u);
    free(ce_v);
    free(inf);
    free(par);
    free(hs);
    return ok ? w : 0;
}

/*
 * First-arrival spanning forest of an edge sequence: mask[i] = 1 iff edge i
 * joins two components of the edges before it (union-find).  Returns the
 * number of forest edges, or (size_t)-1 when out of memory.
 */
size_t sg_forest_mask(uint32_t V, size_t n, const uint32_t *u, const uint32_t *v, uint8_t *mask)
{
    uint32_t *p = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
    if (!p) return (size_t)-1;
    for (uint32_t w = 0; w < V; w++) p[w] = w;
    size_t k = 0;
    for (size_t i = 0; i < n; i++) {
        const uint32_t a = uf_find(p, u[i]), b = uf_find(p, v[i]);
        mask[i] = a != b;
        if (a != b) {
            p[a] = b;
            k++;
        }
    }
    free(p);
    return k;
}
