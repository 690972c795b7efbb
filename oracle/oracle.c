/*
 * Oracle for sketch-based dynamic connectivity: a plain, slow, single-thread
 * CPU implementation of what the GPU hot path computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * What it computes (paper references are sections / equations / theorems of
 * "Fast and Compact Sketch-Based Dynamic Connectivity", arXiv 2509.14433):
 *
 *  - Per-vertex l0-sketch of the vertex's characteristic vector (App. A.1.1,
 *    "The AGM algorithm"): f_u has a 1 at index (u,v) for every incident
 *    edge.  The sampler is a CameoSketch-style F2 sampler (Thm. "CameoSketch",
 *    App. A.1.1; Sec. 3.1): C independent columns, each update touches one
 *    bucket per column, each bucket holds the XOR of the indices (alpha) and
 *    the XOR of their checksums (gamma).
 *  - Sketch addition is word-wise XOR (App. A.1.1), so the sketch of a vertex
 *    set is the XOR of its members' sketches; internal edges cancel and what
 *    remains is exactly the sketch of the cut (App. A.1.1, cancellation).
 *  - A query returns an edge from a bucket that holds exactly one index
 *    (Sec. 2.1; l0-sampling in App. A.1.1), or fails.
 *
 * Readings of points the paper leaves open (the hash family, depth rule,
 * checksum, the order in which good buckets are scanned) are fixed as:
 *   seed_c   = c-th output of SplitMix64 started at state S
 *              (Steele, Lea, Flood, OOPSLA 2014)
 *   mix(z)   = SplitMix64 output finalizer
 *   h_c(x)   = mix(x ^ seed_c)
 *   d_c(x)   = min(ctz(h_c(x)), D-1), ctz(0) = 64
 *   bucket (c, d) of a vertex sketch:
 *            alpha = XOR of x_e over incident live edges e with d_c(x_e) = d
 *            gamma = XOR of h_c(x_e) over the same edges
 *   x_e      = u*V + v for edge {u,v} with u < v
 *   good(c,d)= alpha != 0 and alpha decodes to u < v < V
 *              and h_c(alpha) == gamma and d_c(alpha) == d
 *   sample   = first good bucket scanning c = 0..C-1, and inside a column
 *              d = D-1 down to 0; EMPTY if every word is zero, else FAILED.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EMPTY 1
#define ORC_FAILED 2

/* ---- hash ------------------------------------------------------------- */

uint64_t orc_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* c-th output (c = 0, 1, ...) of SplitMix64 whose state starts at S:
 * the state advances by the golden-ratio increment before each output. */
uint64_t orc_seed(uint64_t S, uint32_t c)
{
    uint64_t state = S;
    uint64_t out = 0;
    for (uint32_t i = 0; i <= c; i++) {
        state += 0x9E3779B97F4A7C15ULL;
        out = orc_mix(state);
    }
    return out;
}

uint64_t orc_hash(uint64_t S, uint32_t c, uint64_t x)
{
    return orc_mix(x ^ orc_seed(S, c));
}

static uint32_t ctz64(uint64_t h)
{
    if (h == 0) return 64;
    uint32_t n = 0;
    while ((h & 1ULL) == 0) { h >>= 1; n++; }
    return n;
}

uint32_t orc_depth_of_hash(uint64_t h, uint32_t D)
{
    uint32_t z = ctz64(h);
    return z < D - 1 ? z : D - 1;
}

uint64_t orc_edge_index(uint32_t V, uint32_t a, uint32_t b)
{
    uint32_t u = a < b ? a : b;
    uint32_t v = a < b ? b : a;
    return (uint64_t)u * V + v;
}

/* valid(x): x decodes to u < v < V */
int orc_valid_index(uint32_t V, uint64_t x)
{
    if (x == 0) return 0;
    uint64_t u = x / V, v = x % V;
    return u < v && v < V;
}

/* ---- sketch state ----------------------------------------------------- */

/* Bucket (c, d) of vertex w lives at [(w*C + c)*D + d]: the canonical
 * order.  alpha and gamma are separate arrays. */
typedef struct {
    uint32_t V, C, D;
    uint64_t S;
    uint64_t *seeds; /* seeds[c] */
    uint64_t *alpha;
    uint64_t *gamma;
} orc_sketch;

orc_sketch *orc_new(uint32_t V, uint32_t C, uint32_t D, uint64_t S)
{
    orc_sketch *s = (orc_sketch *)calloc(1, sizeof(orc_sketch));
    if (!s) return NULL;
    s->V = V; s->C = C; s->D = D; s->S = S;
    s->seeds = (uint64_t *)malloc(sizeof(uint64_t) * C);
    size_t nb = (size_t)V * C * D;
    s->alpha = (uint64_t *)calloc(nb, sizeof(uint64_t));
    s->gamma = (uint64_t *)calloc(nb, sizeof(uint64_t));
    if (!s->seeds || !s->alpha || !s->gamma) {
        free(s->seeds); free(s->alpha); free(s->gamma); free(s);
        return NULL;
    }
    for (uint32_t c = 0; c < C; c++) s->seeds[c] = orc_seed(S, c);
    return s;
}

void orc_free(orc_sketch *s)
{
    if (!s) return;
    free(s->seeds); free(s->alpha); free(s->gamma); free(s);
}

void orc_clear(orc_sketch *s)
{
    size_t nb = (size_t)s->V * s->C * s->D;
    memset(s->alpha, 0, nb * sizeof(uint64_t));
    memset(s->gamma, 0, nb * sizeof(uint64_t));
}

const uint64_t *orc_alpha(const orc_sketch *s) { return s->alpha; }
const uint64_t *orc_gamma(const orc_sketch *s) { return s->gamma; }

/* One stream update ((a,b), +-1).  Over F2 an insert and a delete are the
 * same operation: toggle index x in the characteristic vectors of both
 * endpoints, i.e. XOR (x, h_c(x)) into bucket (c, d_c(x)) of each endpoint
 * for every column c. */
void orc_toggle(orc_sketch *s, uint32_t a, uint32_t b)
{
    uint64_t x = orc_edge_index(s->V, a, b);
    for (uint32_t c = 0; c < s->C; c++) {
        uint64_t h = orc_mix(x ^ s->seeds[c]);
        uint32_t d = orc_depth_of_hash(h, s->D);
        size_t iu = ((size_t)a * s->C + c) * s->D + d;
        size_t iv = ((size_t)b * s->C + c) * s->D + d;
        s->alpha[iu] ^= x; s->gamma[iu] ^= h;
        s->alpha[iv] ^= x; s->gamma[iv] ^= h;
    }
}

void orc_apply(orc_sketch *s, const uint32_t *u, const uint32_t *v, size_t n)
{
    for (size_t i = 0; i < n; i++) orc_toggle(s, u[i], v[i]);
}

/* orc_apply on several host threads (the all-core CPU baseline): the
 * vertices are dealt to the T threads in blocks of 256 consecutive ids,
 * round-robin (thread t owns w with (w / 256) mod T == t, so that streams
 * whose busy vertices have nearby ids still spread over all threads), and
 * each thread, scanning the whole stream in order, applies the bucket
 * writes of the endpoints it owns.  Every bucket has one writer and sees its
 * updates in stream order, so the result is the one orc_apply gives.
 * Returns the number of threads used (1 when built without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_apply_threads(orc_sketch *s, const uint32_t *u, const uint32_t *v, size_t n,
                      int nthreads)
{
    int used = 1;
    if (nthreads < 1) nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
    {
        int T = 1, t = 0;
#ifdef _OPENMP
        T = omp_get_num_threads();
        t = omp_get_thread_num();
        if (t == 0) used = T;
#endif
        for (size_t i = 0; i < n; i++) {
            const uint32_t a = u[i], b = v[i];
            const int own_a = (int)((a >> 8) % (uint32_t)T) == t;
            const int own_b = (int)((b >> 8) % (uint32_t)T) == t;
            if (!own_a && !own_b) continue;
            const uint64_t x = orc_edge_index(s->V, a, b);
            for (uint32_t c = 0; c < s->C; c++) {
                const uint64_t h = orc_mix(x ^ s->seeds[c]);
                const uint32_t d = orc_depth_of_hash(h, s->D);
                if (own_a) {
                    const size_t ia = ((size_t)a * s->C + c) * s->D + d;
                    s->alpha[ia] ^= x;
                    s->gamma[ia] ^= h;
                }
                if (own_b) {
                    const size_t ib = ((size_t)b * s->C + c) * s->D + d;
                    s->alpha[ib] ^= x;
                    s->gamma[ib] ^= h;
                }
            }
        }
    }
    return used;
}

/* Sketch of one vertex w computed from the stream alone: apply only the
 * updates that touch w.  Output is C*D alpha and gamma words in canonical
 * order.  Used to check single vertices of streams too long to replay in
 * full. */
void orc_vertex_from_stream(uint32_t V, uint32_t C, uint32_t D, uint64_t S,
                            uint32_t w, const uint32_t *u, const uint32_t *v,
                            size_t n, uint64_t *out_alpha, uint64_t *out_gamma)
{
    uint64_t *seeds = (uint64_t *)malloc(sizeof(uint64_t) * C);
    for (uint32_t c = 0; c < C; c++) seeds[c] = orc_seed(S, c);
    memset(out_alpha, 0, sizeof(uint64_t) * C * D);
    memset(out_gamma, 0, sizeof(uint64_t) * C * D);
    for (size_t i = 0; i < n; i++) {
        if (u[i] != w && v[i] != w) continue;
        uint64_t x = orc_edge_index(V, u[i], v[i]);
        for (uint32_t c = 0; c < C; c++) {
            uint64_t h = orc_mix(x ^ seeds[c]);
            uint32_t d = orc_depth_of_hash(h, D);
            out_alpha[c * D + d] ^= x;
            out_gamma[c * D + d] ^= h;
        }
    }
    free(seeds);
}

/* Sketch of a vertex set: XOR of the members' sketches (App. A.1.1). */
void orc_set_sketch(const orc_sketch *s, const uint32_t *verts, size_t n,
                    uint64_t *out_alpha, uint64_t *out_gamma)
{
    size_t w = (size_t)s->C * s->D;
    memset(out_alpha, 0, sizeof(uint64_t) * w);
    memset(out_gamma, 0, sizeof(uint64_t) * w);
    for (size_t i = 0; i < n; i++) {
        const uint64_t *a = s->alpha + (size_t)verts[i] * w;
        const uint64_t *g = s->gamma + (size_t)verts[i] * w;
        for (size_t k = 0; k < w; k++) {
            out_alpha[k] ^= a[k];
            out_gamma[k] ^= g[k];
        }
    }
}

/* Query of an aggregate sketch (C*D buckets, canonical order). */
int orc_sample(uint32_t V, uint32_t C, uint32_t D, uint64_t S,
               const uint64_t *alpha, const uint64_t *gamma,
               uint32_t *out_u, uint32_t *out_v)
{
    for (uint32_t c = 0; c < C; c++) {
        uint64_t seed = orc_seed(S, c);
        for (uint32_t k = 0; k < D; k++) {
            uint32_t d = D - 1 - k;
            uint64_t a = alpha[c * D + d];
            uint64_t g = gamma[c * D + d];
            if (a == 0) continue;
            if (!orc_valid_index(V, a)) continue;
            uint64_t h = orc_mix(a ^ seed);
            if (h != g) continue;
            if (orc_depth_of_hash(h, D) != d) continue;
            *out_u = (uint32_t)(a / V);
            *out_v = (uint32_t)(a % V);
            return ORC_OK;
        }
    }
    for (uint32_t k = 0; k < C * D; k++)
        if (alpha[k] != 0 || gamma[k] != 0) return ORC_FAILED;
    return ORC_EMPTY;
}

/* The query of column c alone: the sampler of one level of the multi-level
 * hierarchy (Sec. 2.2.2; level c uses column c).  The column's depths are
 * scanned deepest first (the same order as inside a column of orc_sample);
 * the first bucket that verifies is returned.  EMPTY when every word of
 * the column is zero, FAILED when some word is not but nothing verified. */
int orc_sample_col(uint32_t V, uint32_t C, uint32_t D, uint64_t S, uint32_t c,
                   const uint64_t *alpha, const uint64_t *gamma,
                   uint32_t *out_u, uint32_t *out_v)
{
    const uint64_t seed_c = orc_seed(S, c);
    const uint64_t *col_a = alpha + (size_t)c * D; /* column c: D depths */
    const uint64_t *col_g = gamma + (size_t)c * D;
    int nonzero = 0;
    (void)C;
    for (int32_t d = (int32_t)D - 1; d >= 0; d--) { /* deepest first */
        const uint64_t a = col_a[d], g = col_g[d];
        if ((a | g) != 0) nonzero = 1;
        if (a == 0 || !orc_valid_index(V, a)) continue;
        const uint64_t hc = orc_mix(a ^ seed_c);
        if (hc != g || orc_depth_of_hash(hc, D) != (uint32_t)d) continue;
        *out_u = (uint32_t)(a / V);
        *out_v = (uint32_t)(a % V);
        return ORC_OK;
    }
    return nonzero ? ORC_FAILED : ORC_EMPTY;
}

/* ---- connectivity truth ------------------------------------------------ */

static uint32_t uf_root(uint32_t *p, uint32_t x)
{
    while (p[x] != x) {
        p[x] = p[p[x]]; /* path halving */
        x = p[x];
    }
    return x;
}

/* Connected components of the graph on V vertices with edges (u[i], v[i]):
 * label[w] = smallest vertex of w's component.  Union-find, for graphs too
 * large for the breadth-first search of the Python oracle.  Returns the
 * number of components, or 0 when out of memory. */
uint64_t orc_uf_components(uint32_t V, const uint32_t *u, const uint32_t *v, size_t n,
                           uint32_t *label)
{
    uint32_t *p = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)V);
    if (!p) return 0;
    for (uint32_t w = 0; w < V; w++) p[w] = w;
    for (size_t i = 0; i < n; i++) {
        const uint32_t a = uf_root(p, u[i]), b = uf_root(p, v[i]);
        if (a != b) p[a < b ? b : a] = a < b ? a : b; /* the smaller root survives */
    }
    uint64_t k = 0;
    for (uint32_t w = 0; w < V; w++) {
        label[w] = uf_root(p, w);
        if (label[w] == w) k++;
    }
    free(p);
    return k;
}

/* Incremental union-find for connectivity truth along a growing edge set. */
typedef struct {
    uint32_t V;
    uint32_t *p;
    uint64_t n_comp;
} orc_uf;

orc_uf *orc_uf_new(uint32_t V)
{
    orc_uf *h = (orc_uf *)calloc(1, sizeof(orc_uf));
    if (!h) return NULL;
    h->p = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)V);
    if (!h->p) {
        free(h);
        return NULL;
    }
    for (uint32_t w = 0; w < V; w++) h->p[w] = w;
    h->V = V;
    h->n_comp = V;
    return h;
}

void orc_uf_free(orc_uf *h)
{
    if (!h) return;
    free(h->p);
    free(h);
}

/* Add edges (u[i], v[i]); returns the number of components after them. */
uint64_t orc_uf_add(orc_uf *h, const uint32_t *u, const uint32_t *v, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        const uint32_t a = uf_root(h->p, u[i]), b = uf_root(h->p, v[i]);
        if (a != b) {
            h->p[a < b ? b : a] = a < b ? a : b;
            h->n_comp--;
        }
    }
    return h->n_comp;
}

int orc_uf_same(orc_uf *h, uint32_t a, uint32_t b)
{
    return uf_root(h->p, a) == uf_root(h->p, b);
}

/* Order-independent 64-bit digest of a whole sketch:
 *   sum over (w,c,d) of mix(alpha ^ rotl(gamma,32) ^ mix(((w*C+c)*D+d) ^ S))
 * modulo 2^64. */
uint64_t orc_digest(const orc_sketch *s)
{
    uint64_t acc = 0;
    size_t i = 0;
    for (uint64_t w = 0; w < s->V; w++)
        for (uint64_t c = 0; c < s->C; c++)
            for (uint64_t d = 0; d < s->D; d++, i++) {
                uint64_t pos = (w * s->C + c) * s->D + d;
                uint64_t g = s->gamma[i];
                uint64_t rg = (g << 32) | (g >> 32);
                acc += orc_mix(s->alpha[i] ^ rg ^ orc_mix(pos ^ s->S));
            }
    return acc;
}

/* Same digest over explicit arrays of a vertex range [w0, w0+nv): the
 * partial sum; partial sums of disjoint ranges add up to the whole. */
uint64_t orc_digest_arrays(uint32_t C, uint32_t D, uint64_t S, uint32_t w0,
                           uint32_t nv, const uint64_t *alpha,
                           const uint64_t *gamma)
{
    uint64_t acc = 0;
    size_t i = 0;
    for (uint64_t w = w0; w < (uint64_t)w0 + nv; w++)
        for (uint64_t c = 0; c < C; c++)
            for (uint64_t d = 0; d < D; d++, i++) {
                uint64_t pos = (w * C + c) * D + d;
                uint64_t g = gamma[i];
                uint64_t rg = (g << 32) | (g >> 32);
                acc += orc_mix(alpha[i] ^ rg ^ orc_mix(pos ^ S));
            }
    return acc;
}
