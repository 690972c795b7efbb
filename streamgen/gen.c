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
 * probabilities a, b, c, 1-a-b-c over logV levels, each level's quadrant
 * from a 16-bit uniform, four levels per 64-bit draw) is drawn, canonicalised
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
    /* quadrant thresholds on 16-bit uniforms: four levels per 64-bit draw */
    const uint32_t ta = (uint32_t)(a * 65536.0 + 0.5), tab = (uint32_t)((a + b) * 65536.0 + 0.5);
    const uint32_t tabc = (uint32_t)((a + b + c) * 65536.0 + 0.5);
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
                uint64_t bits = 0;
                for (uint32_t l = 0; l < g->logV; l++) {
                    if ((l & 3) == 0) bits = rng_next(r);
                    const uint32_t q = (uint32_t)(bits & 0xFFFF);
                    bits >>= 16;
                    const int bx = q >= tab;                         /* quadrants c, d */
                    const int by = (q >= ta && q < tab) || q >= tabc; /* quadrants b, d */
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

static uint32_t uf_find(uint32_t *p, uint32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]];
        x = p[x];
    }
    return x;
}

/* MurmurHash3's 64-bit finalizer (Appleby): the counter-based hash behind
 * the parallel shuffle below (bucket choice and per-bucket seeds). */
static uint64_t fmix64(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

/*
 * Uniformly random permutation of in[0..m) into out, the same for any
 * number of threads: one level of the Rao-Sandelius method.  Element i goes
 * to bucket fmix64(key + (i+1)*golden) >> 54 (1024 buckets), buckets are laid
 * out in order (elements in input order inside each), and every bucket is
 * then Fisher-Yates shuffled with its own xoshiro256** stream seeded from
 * (key, bucket).  Input chunks are fixed, so threads only share the work.
 */
enum { PS_BUCKETS = 1024, PS_CHUNKS = 256 };

static uint32_t ps_bucket(uint64_t key, size_t i)
{
    return (uint32_t)(fmix64(key + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ULL) >> 54);
}

static int par_shuffle(const uint64_t *in, uint64_t *out, size_t m, uint64_t key)
{
    size_t *cnt = (size_t *)calloc((size_t)PS_CHUNKS * PS_BUCKETS, sizeof(size_t));
    size_t *bstart = (size_t *)malloc(sizeof(size_t) * (PS_BUCKETS + 1));
    if (!cnt || !bstart) {
        free(cnt);
        free(bstart);
        return 0;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < PS_CHUNKS; c++) {
        const size_t lo = m * (size_t)c / PS_CHUNKS, hi = m * (size_t)(c + 1) / PS_CHUNKS;
        size_t *cc = cnt + (size_t)c * PS_BUCKETS;
        for (size_t i = lo; i < hi; i++) cc[ps_bucket(key, i)]++;
    }
    /* start of (bucket b, chunk c) = elements of earlier buckets, then of
     * earlier chunks inside bucket b */
    size_t acc = 0;
    for (int b = 0; b < PS_BUCKETS; b++) {
        bstart[b] = acc;
        for (int c = 0; c < PS_CHUNKS; c++) {
            const size_t x = cnt[(size_t)c * PS_BUCKETS + b];
            cnt[(size_t)c * PS_BUCKETS + b] = acc;
            acc += x;
        }
    }
    bstart[PS_BUCKETS] = acc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < PS_CHUNKS; c++) {
        const size_t lo = m * (size_t)c / PS_CHUNKS, hi = m * (size_t)(c + 1) / PS_CHUNKS;
        size_t *cc = cnt + (size_t)c * PS_BUCKETS;
        for (size_t i = lo; i < hi; i++) out[cc[ps_bucket(key, i)]++] = in[i];
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int b = 0; b < PS_BUCKETS; b++) {
        rng_t r;
        rng_seed(&r, fmix64(key ^ ((uint64_t)(b + 1) << 40)));
        uint64_t *a = out + bstart[b];
        for (size_t i = bstart[b + 1] - bstart[b]; i > 1; i--) {
            const size_t j = (size_t)rng_below(&r, i);
            const uint64_t t = a[i - 1];
            a[i - 1] = a[j];
            a[j] = t;
        }
    }
    free(cnt);
    free(bstart);
    return 1;
}

/*
 * Clustered churn, drawn one phase at a time.  Vertices [0, K*S) form K
 * clusters of S vertices, each a G(S, p_in); the other n_sparse vertices
 * carry a sparse G(n, m = 2n).
 *   setup:  the sparse edges (random order); bridges: a random tree over the
 *           clusters (cluster i to a random earlier cluster) plus
 *           extra_bridges random ones between random vertices of two
 *           different clusters; then every cluster's first-arrival spanning
 *           forest under one random order of all cluster edges (the fixed
 *           forest, never deleted).
 *   round:  every other cluster edge inserted in a fresh random order, then
 *           all of them deleted in another one.
 * From the forest on, after every adv_every updates, adv_k bridges drawn
 * uniformly are toggled (deleted if present, re-inserted if absent); rounds
 * must therefore be drawn in order.  Updates are written packed: u | v<<32
 * | is_delete<<63 with u < v.
 */
typedef struct {
    rng_t r;           /* sequential stream: sparse part, bridges, bridge picks */
    uint64_t seed;
    uint32_t K, S, n_sparse, nb, adv_every, adv_k;
    uint32_t *bu, *bv;
    uint8_t *blive;
    uint64_t *sp;      /* sparse edges */
    size_t nsp;
    uint64_t *fe;      /* forest edges, arrival order */
    size_t nf;
    uint64_t *ce;      /* the other cluster edges */
    size_t m2;
    uint64_t *tmp;     /* shuffle output */
    uint64_t since;
    uint32_t next_round;
    int setup_done;
} clu_t;

static uint64_t pk(uint32_t a, uint32_t b, int del)
{
    const uint32_t x = a < b ? a : b, y = a < b ? b : a;
    return (uint64_t)x | ((uint64_t)y << 32) | ((uint64_t)(del != 0) << 63);
}

void sg_clu_free(void *h)
{
    clu_t *g = (clu_t *)h;
    if (!g) return;
    free(g->bu);
    free(g->bv);
    free(g->blive);
    free(g->sp);
    free(g->fe);
    free(g->ce);
    free(g->tmp);
    free(g);
}

void *sg_clu_new(uint32_t K, uint32_t S, double p_in, uint32_t n_sparse, uint32_t extra_bridges,
                 uint32_t adv_every, uint32_t adv_k, uint64_t seed)
{
    clu_t *g = (clu_t *)calloc(1, sizeof(clu_t));
    if (!g) return NULL;
    rng_seed(&g->r, seed);
    g->seed = seed;
    g->K = K;
    g->S = S;
    g->n_sparse = n_sparse;
    g->adv_every = adv_every;
    g->adv_k = adv_k;
    g->nb = K > 1 ? (K - 1) + extra_bridges : 0;
    const uint32_t Vc = K * S;
    const size_t per = (size_t)S * (S > 0 ? S - 1 : 0) / 2;
    const size_t msp = n_sparse >= 2 ? 2 * (size_t)n_sparse : 0;
    g->bu = (uint32_t *)malloc(sizeof(uint32_t) * (g->nb + 1));
    g->bv = (uint32_t *)malloc(sizeof(uint32_t) * (g->nb + 1));
    g->blive = (uint8_t *)calloc(g->nb + 1, 1);
    g->sp = (uint64_t *)malloc(sizeof(uint64_t) * (msp + 1));
    size_t hcap = 1;
    while (hcap < 4 * msp + 1) hcap <<= 1;
    uint64_t *hs = (uint64_t *)malloc(sizeof(uint64_t) * hcap);
    size_t *cm = (size_t *)calloc((size_t)K + 1, sizeof(size_t));
    uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)K * per + 1));
    uint32_t *par = (uint32_t *)malloc(sizeof(uint32_t) * ((size_t)Vc + 1));
    if (!g->bu || !g->bv || !g->blive || !g->sp || !hs || !cm || !all || !par) goto fail;
    /* sparse part: m = 2n distinct random pairs (open-addressing set) */
    for (size_t i = 0; i < hcap; i++) hs[i] = UINT64_MAX;
    {
        const uint64_t nn = n_sparse;
        while (g->nsp < msp && (uint64_t)g->nsp < nn * (nn - 1) / 2) {
            uint64_t x = rng_below(&g->r, nn), y = rng_below(&g->r, nn);
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
            g->sp[g->nsp++] = pk(Vc + (uint32_t)x, Vc + (uint32_t)y, 0);
        }
    }
    /* bridges */
    {
        uint32_t q = 0;
        for (uint32_t i = 1; i < K; i++) {
            const uint32_t j = (uint32_t)rng_below(&g->r, i);
            g->bu[q] = i * S + (uint32_t)rng_below(&g->r, S);
            g->bv[q] = j * S + (uint32_t)rng_below(&g->r, S);
            q++;
        }
        while (q < g->nb) {
            const uint32_t i = (uint32_t)rng_below(&g->r, K), j = (uint32_t)rng_below(&g->r, K);
            if (i == j) continue;
            const uint32_t x = i * S + (uint32_t)rng_below(&g->r, S);
            const uint32_t y = j * S + (uint32_t)rng_below(&g->r, S);
            int dup = 0;
            for (uint32_t t = 0; t < q; t++)
                if ((g->bu[t] == x && g->bv[t] == y) || (g->bu[t] == y && g->bv[t] == x)) dup = 1;
            if (dup) continue;
            g->bu[q] = x;
            g->bv[q] = y;
            q++;
        }
    }
    /* cluster graphs, one xoshiro stream per cluster, drawn in parallel
     * into fixed slots and packed in cluster order */
#pragma omp parallel for schedule(dynamic, 1)
    for (uint32_t c = 0; c < K; c++) {
        rng_t rc;
        rng_seed(&rc, fmix64(seed ^ (0xC1u + ((uint64_t)c << 32))));
        uint64_t *slot = all + (size_t)c * per;
        const double lq = p_in < 1.0 ? __builtin_log(1.0 - p_in) : 0.0;
        size_t k = 0;
        for (uint32_t x = 0; x + 1 < S; x++) {
            int64_t y = x;
            for (;;) {
                if (p_in >= 1.0) {
                    y += 1;
                } else {
                    double uu = rng_unif(&rc);
                    if (uu <= 0.0) uu = 0x1.0p-53;
                    y += 1 + (int64_t)(__builtin_log(uu) / lq);
                }
                if (y >= (int64_t)S) break;
                slot[k++] = pk(c * S + x, c * S + (uint32_t)y, 0);
            }
        }
        cm[c] = k;
    }
    size_t m = 0;
    for (uint32_t c = 0; c < K; c++) {
        memmove(all + m, all + (size_t)c * per, cm[c] * sizeof(uint64_t));
        m += cm[c];
    }
    g->tmp = (uint64_t *)malloc(sizeof(uint64_t) * (m + 1));
    g->fe = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)Vc + 1));
    g->ce = (uint64_t *)malloc(sizeof(uint64_t) * (m + 1));
    if (!g->tmp || !g->fe || !g->ce) goto fail;
    /* first-arrival forest of one random order of all cluster edges */
    if (!par_shuffle(all, g->tmp, m, fmix64(seed ^ 0xF0F0F0F0ULL))) goto fail;
    for (uint32_t x = 0; x < Vc; x++) par[x] = x;
    for (size_t i = 0; i < m; i++) {
        const uint64_t e = g->tmp[i];
        const uint32_t ra = uf_find(par, (uint32_t)e), rb = uf_find(par, (uint32_t)(e >> 32));
        if (ra != rb) {
            par[ra] = rb;
            g->fe[g->nf++] = e;
        } else {
            g->ce[g->m2++] = e;
        }
    }
    free(hs);
    free(cm);
    free(all);
    free(par);
    return g;
fail:
    free(hs);
    free(cm);
    free(all);
    free(par);
    sg_clu_free(g);
    return NULL;
}

/* Updates in the setup phase and in one churn round (upper bound: the
 * number of bridge toggles depends on where the ticks fall). */
size_t sg_clu_setup_len(void *h)
{
    clu_t *g = (clu_t *)h;
    const size_t base = g->nsp + g->nb + g->nf;
    return base + (g->adv_every ? (g->nf / g->adv_every + 1) * g->adv_k : 0);
}

size_t sg_clu_round_cap(void *h)
{
    clu_t *g = (clu_t *)h;
    return 2 * g->m2 + (g->adv_every ? (2 * g->m2 / g->adv_every + 2) * g->adv_k : 0);
}

size_t sg_clu_m2(void *h) { return ((clu_t *)h)->m2; }

/* one update, then the bridge-toggle tick */
static size_t clu_emit(clu_t *g, uint64_t *out, size_t w, uint64_t p)
{
    out[w++] = p;
    if (g->adv_every && g->nb && ++g->since >= g->adv_every) {
        g->since = 0;
        for (uint32_t t = 0; t < g->adv_k; t++) {
            const uint32_t bi = (uint32_t)rng_below(&g->r, g->nb);
            out[w++] = pk(g->bu[bi], g->bv[bi], g->blive[bi]);
            g->blive[bi] ^= 1;
        }
    }
    return w;
}

/* The setup phase into out (sg_clu_setup_len(h) words); returns its length. */
size_t sg_clu_setup(void *h, uint64_t *out)
{
    clu_t *g = (clu_t *)h;
    if (g->setup_done) return 0;
    size_t w = 0;
    for (size_t i = 0; i < g->nsp; i++) out[w++] = g->sp[i];
    for (uint32_t t = 0; t < g->nb; t++) {
        out[w++] = pk(g->bu[t], g->bv[t], 0);
        g->blive[t] = 1;
    }
    for (size_t i = 0; i < g->nf; i++) w = clu_emit(g, out, w, g->fe[i]);
    g->setup_done = 1;
    return w;
}

/* Churn round `rd` (rounds in order, after the setup) into out
 * (sg_clu_round_cap(h) words); returns its length, 0 on misuse or when out
 * of memory. */
size_t sg_clu_round(void *h, uint32_t rd, uint64_t *out)
{
    clu_t *g = (clu_t *)h;
    if (!g->setup_done || rd != g->next_round) return 0;
    size_t w = 0;
    for (int pass = 0; pass < 2; pass++) {
        const uint64_t key = fmix64(g->seed ^ (((uint64_t)rd << 8) | (uint64_t)(pass + 1)) << 20);
        if (!par_shuffle(g->ce, g->tmp, g->m2, key)) return 0;
        const uint64_t del = pass ? 1ULL << 63 : 0;
        for (size_t i = 0; i < g->m2; i++) w = clu_emit(g, out, w, g->tmp[i] | del);
    }
    g->next_round++;
    return w;
}

/*
 * G(V, p) inserts in random order, then deletions of a fraction of the
 * inserted edges in chunks, part of each chunk on current forest edges that
 * the caller supplies (the forest of whatever engine replays the stream).
 *   - edges: row x's neighbours y > x by geometric skipping, one xoshiro
 *     stream per block of 64 rows (drawn in parallel), in row order, then
 *     put in a random order by par_shuffle;
 *   - a chunk of `size` deletions: Binomial(size, forest_frac) distinct
 *     uniform edges of the supplied forest (at most all of them), the rest
 *     uniform live edges outside it (rejection over the insertion order),
 *     the whole chunk in random order.
 * A live bitmap over keys u*V + v (V*V bits) keeps the stream legal.
 * Updates are packed: u | v<<32 | is_delete<<63 with u < v.
 */
typedef struct {
    rng_t r;
    uint32_t V;
    double forest_frac;
    uint64_t *ins;    /* packed inserts, stream order */
    size_t m;
    uint64_t *bm;     /* live keys */
    size_t k, deleted;
    uint64_t *fset;   /* open-addressing set of the supplied forest's keys */
    size_t fcap;
    size_t inserted;  /* inserts drawn so far (a prefix of ins) */
} ftd_t;

static int ftd_live(const ftd_t *g, uint64_t key) { return bit_get(g->bm, key); }

void sg_ftd_free(void *h)
{
    ftd_t *g = (ftd_t *)h;
    if (!g) return;
    free(g->ins);
    free(g->bm);
    free(g->fset);
    free(g);
}

void *sg_ftd_new(uint32_t V, double p, double del_frac, double forest_frac, uint64_t seed)
{
    ftd_t *g = (ftd_t *)calloc(1, sizeof(ftd_t));
    if (!g || V < 2) {
        free(g);
        return NULL;
    }
    rng_seed(&g->r, seed);
    g->V = V;
    g->forest_frac = forest_frac;
    const uint32_t RB = 64;
    const uint32_t nblk = (V + RB - 1) / RB;
    size_t *cnt = (size_t *)calloc((size_t)nblk + 1, sizeof(size_t));
    uint64_t **part = (uint64_t **)calloc(nblk, sizeof(uint64_t *));
    int ok = cnt && part;
    const double lq = p < 1.0 ? __builtin_log(1.0 - p) : 0.0;
#pragma omp parallel for schedule(dynamic, 4)
    for (uint32_t b = 0; b < nblk; b++) {
        if (!ok) continue;
        rng_t rb;
        rng_seed(&rb, fmix64(seed ^ (0xE5u + ((uint64_t)b << 32))));
        const uint32_t x0 = b * RB, x1 = x0 + RB < V ? x0 + RB : V;
        size_t cap = 1024, k = 0;
        uint64_t *buf = (uint64_t *)malloc(cap * sizeof(uint64_t));
        for (uint32_t x = x0; x < x1 && buf; x++) {
            int64_t y = x;
            for (;;) {
                if (p >= 1.0) {
                    y += 1;
                } else {
                    double uu = rng_unif(&rb);
                    if (uu <= 0.0) uu = 0x1.0p-53;
                    y += 1 + (int64_t)(__builtin_log(uu) / lq);
                }
                if (y >= (int64_t)V) break;
                if (k == cap) {
                    cap *= 2;
                    uint64_t *nb = (uint64_t *)realloc(buf, cap * sizeof(uint64_t));
                    if (!nb) {
                        free(buf);
                        buf = NULL;
                        break;
                    }
                    buf = nb;
                }
                buf[k++] = (uint64_t)x | ((uint64_t)y << 32);
            }
        }
        if (!buf) ok = 0;
        part[b] = buf;
        cnt[b] = k;
    }
    size_t m = 0;
    for (uint32_t b = 0; ok && b < nblk; b++) m += cnt[b];
    uint64_t *all = ok ? (uint64_t *)malloc(sizeof(uint64_t) * (m + 1)) : NULL;
    g->ins = ok ? (uint64_t *)malloc(sizeof(uint64_t) * (m + 1)) : NULL;
    g->bm = ok ? (uint64_t *)calloc(((uint64_t)V * V + 63) / 64, 8) : NULL;
    if (!all || !g->ins || !g->bm) ok = 0;
    size_t w = 0;
    for (uint32_t b = 0; b < nblk; b++) {
        if (ok) memcpy(all + w, part[b], cnt[b] * sizeof(uint64_t));
        w += ok ? cnt[b] : 0;
        free(part ? part[b] : NULL);
    }
    free(part);
    free(cnt);
    if (ok && !par_shuffle(all, g->ins, m, fmix64(seed ^ 0x1A5E27ULL))) ok = 0;
    free(all);
    if (!ok) {
        sg_ftd_free(g);
        return NULL;
    }
    g->m = m;
    g->k = (size_t)(del_frac * (double)m);
    return g;
}

size_t sg_ftd_m(void *h) { return ((ftd_t *)h)->m; }
size_t sg_ftd_k(void *h) { return ((ftd_t *)h)->k; }
size_t sg_ftd_deleted(void *h) { return ((ftd_t *)h)->deleted; }

/* Inserts [k0, k1) of the insert phase, packed, into out; marks them live. */
size_t sg_ftd_inserts(void *h, size_t k0, size_t k1, uint64_t *out)
{
    ftd_t *g = (ftd_t *)h;
    if (k1 > g->m) k1 = g->m;
    if (k0 != g->inserted || k1 < k0) return 0;  /* in order, once */
    size_t w = 0;
    for (size_t i = k0; i < k1; i++) {
        const uint64_t e = g->ins[i];
        bit_set(g->bm, (e & 0xFFFFFFFFu) * g->V + (e >> 32));
        out[w++] = e;
    }
    g->inserted = k1;
    return w;
}

static int fset_has(const ftd_t *g, uint64_t key)
{
    size_t i = (size_t)(fmix64(key) & (g->fcap - 1));
    while (g->fset[i] != UINT64_MAX) {
        if (g->fset[i] == key) return 1;
        i = (i + 1) & (g->fcap - 1);
    }
    return 0;
}

/* The next chunk of at most `size` deletions, given the current forest
 * (nf edges as keys u*V + v, u < v, all live) in `forest` (reordered in
 * place).  Writes packed deletions to out; returns their number (0 when
 * every deletion has been drawn), or (size_t)-1 when out of memory. */
size_t sg_ftd_delete_chunk(void *h, size_t size, uint64_t *forest, size_t nf, uint64_t *out)
{
    ftd_t *g = (ftd_t *)h;
    const uint64_t V = g->V;
    if (g->deleted + size > g->k) size = g->k - g->deleted;
    if (size == 0) return 0;
    size_t want = 0;
    for (size_t i = 0; i < size; i++) want += rng_unif(&g->r) < g->forest_frac;
    if (want > nf) want = nf;
    /* at most every live edge outside the forest (nf forest edges are live) */
    const size_t live = g->inserted - g->deleted;
    const size_t avail = live > nf ? live - nf : 0;
    if (size - want > avail) size = want + avail;
    /* forest keys: a set for the rejection test below */
    size_t cap = 16;
    while (cap < 2 * nf + 16) cap <<= 1;
    if (cap > g->fcap) {
        free(g->fset);
        g->fset = (uint64_t *)malloc(cap * sizeof(uint64_t));
        if (!g->fset) {
            g->fcap = 0;
            return (size_t)-1;
        }
        g->fcap = cap;
    }
    for (size_t i = 0; i < g->fcap; i++) g->fset[i] = UINT64_MAX;
    for (size_t i = 0; i < nf; i++) {
        size_t j = (size_t)(fmix64(forest[i]) & (g->fcap - 1));
        while (g->fset[j] != UINT64_MAX && g->fset[j] != forest[i]) j = (j + 1) & (g->fcap - 1);
        g->fset[j] = forest[i];
    }
    size_t w = 0;
    /* distinct uniform forest edges: a partial Fisher-Yates over the list */
    for (size_t i = 0; i < want; i++) {
        const size_t j = i + (size_t)rng_below(&g->r, nf - i);
        const uint64_t t = forest[i];
        forest[i] = forest[j];
        forest[j] = t;
        const uint64_t key = forest[i];
        bit_clr(g->bm, key);
        out[w++] = (key / V) | ((key % V) << 32) | (1ULL << 63);
    }
    /* uniform live non-forest edges (each drawn edge is dead at once, so
     * the picks are distinct) */
    while (w < size) {
        const uint64_t e = g->ins[rng_below(&g->r, g->m)];
        const uint64_t key = (e & 0xFFFFFFFFu) * V + (e >> 32);
        if (!ftd_live(g, key) || fset_has(g, key)) continue;
        bit_clr(g->bm, key);
        out[w++] = e | (1ULL << 63);
    }
    for (size_t i = w; i > 1; i--) {
        const size_t j = (size_t)rng_below(&g->r, i);
        const uint64_t t = out[i - 1];
        out[i - 1] = out[j];
        out[j] = t;
    }
    g->deleted += w;
    return w;
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
