/*
 * cupk — sketch-based dynamic connectivity on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of the CUPCaKE method ("Fast and
 * Compact Sketch-Based Dynamic Connectivity", arXiv 2509.14433):
 *   - every vertex keeps a resident l0-sketch of its characteristic vector
 *     (App. A.1.1, AGM characteristic vectors; CameoSketch-style F2 sampler,
 *     Sec. 3.1 and the CameoSketch theorem of App. A.1.1);
 *   - a batch of edge inserts / deletes is hashed once per column and
 *     XOR-scattered into one bucket per column of both endpoints' sketches
 *     (cutset Update, Sec. 2.2.1; Alg. 1, first parallel loop);
 *   - the sketch of a vertex set is the XOR of its members' sketches, which
 *     cancels internal edges and leaves the cut (App. A.1.1);
 *   - a query returns an edge from a bucket holding exactly one index
 *     (cutset Query, Sec. 2.2.1);
 *   - a spanning forest is kept on the host; deleting a forest edge triggers
 *     replacement search by Boruvka-style rounds over the broken trees
 *     (App. A.1.1, AGM Boruvka; Alg. 1 restoration loop) and connectivity
 *     queries are answered from the forest (Sec. 2.1 problem statement,
 *     Sec. 4.1 query tree).
 * Modes beyond that path (cupk_opts): exact per-update semantics inside
 * batches (speculative buffering, Sec. 4.3), the multi-level hierarchy of
 * cutsets (Sec. 2.2.2, Alg. 1), and, as separate calls, components of the
 * whole graph from the sketch alone (App. A.1.1) and a serving loop with
 * query bursts.
 *
 * Sketch definition (bit-exact contract with the tests' CPU oracle):
 *   seed_c  = c-th output of SplitMix64 from state `seed`
 *   h_c(x)  = SplitMix64 finalizer of (x ^ seed_c)
 *   d_c(x)  = min(ctz(h_c(x)), D-1)          (ctz(0) = 64)
 *   x       = u*V + v for edge {u, v}, u < v
 *   bucket (c, d) of vertex w holds
 *           alpha = XOR of x over live edges at w with d_c(x) = d,
 *           gamma = XOR of h_c(x) over the same edges.
 *   good(c,d) iff alpha != 0, alpha decodes to u < v < V, h_c(alpha) == gamma
 *           and d_c(alpha) == d.
 *   sample  = the first good bucket scanning c = 0..C-1 and, inside a column,
 *           d = D-1 down to 0.
 *
 * Conventions
 *   - Return codes: 0 OK, positive = informational status, negative = error.
 *   - Buckets at this boundary are always in canonical order: bucket (c, d)
 *     of one sketch is element c*D + d of a cupk_bucket array.
 *   - Pointers are host pointers unless the name says "device".
 *   - No C++ exception crosses this boundary.
 *   - A context is used by one host thread at a time.
 */
#ifndef CUPK_H
#define CUPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status / error codes ---------------------------------------------- */
#define CUPK_OK 0
#define CUPK_EMPTY 1          /* aggregate sketch is all zero: the cut is empty */
#define CUPK_SAMPLE_FAILED 2  /* nonzero aggregate but no bucket verifies       */
#define CUPK_EINVAL (-1)      /* bad argument; nothing was changed              */
#define CUPK_ENOMEM (-2)      /* device or pinned-host allocation failed        */
#define CUPK_EDEVICE (-3)     /* a HIP call failed; see cupk_last_error         */
#define CUPK_EBUSY (-4)       /* admission refused (serving loop)               */

/* ---- scatter kernel selection ------------------------------------------ */
#define CUPK_SCATTER_ATOMIC 0 /* plain kernel: one device atomic XOR per word  */
#define CUPK_SCATTER_STAGED 1 /* vertex-binned, LDS-staged kernel              */

/* ---- staged-scatter lane layouts --------------------------------------- */
#define CUPK_LAYOUT_RECORD 1  /* one lane per record, its C columns in turn    */
#define CUPK_LAYOUT_PAIR 2    /* one lane per (record, column) pair            */

typedef struct cupk_ctx cupk_ctx;

/* One sketch bucket: XOR of indices and XOR of their checksums. */
typedef struct {
    uint64_t alpha;
    uint64_t gamma;
} cupk_bucket;

/* Options for cupk_sketch_init.  Zero-initialise and set what you need. */
typedef struct {
    /* CUPK_SCATTER_ATOMIC or CUPK_SCATTER_STAGED (default: STAGED). */
    uint32_t scatter_mode;
    /* Initial capacity of the device update buffers, in updates (default
     * 1<<20).  Larger batches grow the buffers on demand. */
    uint32_t max_batch;
    /* hipStream_t to launch on.  Used when use_given_stream is nonzero (a
     * NULL stream then means the default stream); otherwise the library
     * creates and owns a stream. */
    void *stream;
    uint32_t use_given_stream;
    /* Device memory for the sketch, >= cupk_sketch_bytes(V, C, D) bytes,
     * owned by the caller (e.g. a torch tensor) and kept alive until
     * cupk_free.  NULL = the library allocates it.  It is zeroed at init. */
    void *sketch_device_ptr;
    /* k > 0: record HIP events around every k-th scatter launch (1 = every
     * launch) so that cupk_counters reports the summed kernel time of the
     * timed launches (scatter_ms, bin_ms) and their number and updates
     * (timed_launches, timed_updates).  Every event recorded between two
     * kernels leaves the GPU idle for a few microseconds, so sampling keeps
     * the timed run close to an untimed one. */
    uint32_t time_kernels;
    /* Staged scatter tuning (0 = library default / autotuned value):
     * vertices per LDS tile and depth rows kept in LDS. */
    uint32_t tile_vertices;
    uint32_t lds_rows;
    /* Records per work item of the staged kernel (0 = default 4096) and
     * blocks of its persistent grid (0 = default 2048). */
    uint32_t chunk_records;
    uint32_t tile_grid;
    /* Nonzero: replay each batch's device work (classification with its
     * header copy, binning, scatter) as captured HIP graphs sized for the
     * batch capacity; the kernels read the batch size from device memory,
     * so one capture serves batches of any size up to the capacity. */
    uint32_t use_graph;
    /* Nonzero: per-update semantics inside every batch (speculative update
     * buffering, Sec. 4.3).  A batch is classified and scattered as a
     * whole; at the first update that cuts a forest edge, the scatter of
     * the updates after it is undone (applied again: XOR toggles back), the
     * cut and its replacement rounds run on the sketch as of that update,
     * and the rest of the batch is processed again the same way.  The
     * forest then equals the one obtained by applying the updates one at a
     * time (batches of one), whatever the batch size, as long as no
     * replacement query fails (a failed tree is retried at the next cut or
     * batch end rather than after every update).  Captured graphs
     * (use_graph) are not used in this mode. */
    uint32_t exact;
    /* Nonzero: multi-level hierarchy (Gibb's cutset levels, Sec. 2.2.2 and
     * Alg. 1).  Levels 0..C: level i < C keeps its own forest and queries
     * its components with sketch column i alone; level C is the forest that
     * answers connectivity.  Inserts only update the sketch; a delete of a
     * forest edge removes it from every level from its weight (the lowest
     * level holding it) up.  At the end of each batch, Invariant 3 (a
     * level-i component whose query returns an edge is a proper subset of
     * its level-(i+1) component) is restored pass by pass from the lowest
     * violating level, each pass one reduce + query launch over the
     * components that could violate it; a repair removes the heaviest edge
     * of the cycle it would close (ties: the smaller edge) from its weight
     * up and adds the sampled edge to every level above.  The top forest is
     * then completed with replacement rounds on the all-column sampler.
     * Not combinable with exact. */
    uint32_t levels;
    /* Nonzero: walk the flagged updates of a batch into the forest one at a
     * time.  Default: a run of flagged updates where an insert follows a
     * delete is walked contracted (the pieces the run's deletes leave of the
     * forest as vertices, the run replayed on that small forest, only the
     * net change applied), which gives the same forest, dirty trees and
     * counts. */
    uint32_t walk_plain;
    /* Nonzero: split the trees broken by a batch's cuts (relabel every piece
     * but the largest) before the first replacement round.  Default: the
     * first round works on the pieces as found by the same search, links
     * them by parent pointers only and labels the final trees once, which
     * gives the same forest and counts without relabelling pieces that the
     * round links back together. */
    uint32_t split_rounds;
    /* Nonzero: the staged fill reserves each (block, tile) range in the bins
     * with an atomic, and the classify kernel keeps one set of tile counts.
     * Default: each classify block adds its tile counts to one of four
     * copies and stores where its records start (one word per classify
     * block and tile, up to 2^25 words, at most 2048 tiles; beyond that the
     * fill reserves), so that the fill reserves nothing.  Same bins up to
     * the order of records inside a tile, same sketch. */
    uint32_t fill_reserve;
    /* Lane layout of the staged scatter: CUPK_LAYOUT_RECORD (each lane
     * hashes one record's C columns as independent chains; LDS address
     * conflicts grow with the records per vertex and batch) or
     * CUPK_LAYOUT_PAIR (each lane one (record, column) pair, records decoded
     * once into LDS; conflict-free, for large batches).  0 = default: PAIR
     * when max_batch is at least 4M updates, else RECORD.  The autotuner
     * tries both. */
    uint32_t tile_layout;
    /* Nonzero: finish each batch's replacement rounds before the next batch
     * is classified.  Default: when a device batch follows one whose host
     * part is still pending (cupk_apply_updates_device), the new batch is
     * classified against the forest as it stands after the pending batch's
     * flag walk and binned while that batch's replacement rounds run (their
     * reductions on a stream of their own).  The rounds only join trees, so
     * the flags found that way include every flag of the forest after the
     * rounds; they are checked again against that forest before the scatter,
     * which leaves exactly the flags, forest and sketch of the serial
     * order.  A walk that ends with cuts whose trees are not split yet
     * (their pieces share a label until the rounds split them), or that
     * leaves fewer than two dirty trees (nothing for the rounds to search),
     * has its rounds run first, and so do batches below overlap_min_batch. */
    uint32_t serial_rounds;
    /* Tiles per coarse bin of the two-level binning the staged scatter uses
     * beyond 2048 tiles (a power of two in [2, 8192], at most 8192 coarse
     * bins; 0 = default: about sqrt(2 * tiles) coarse bins, which suits
     * records spread over all tiles).  The autotuner tries smaller ones,
     * which suit records that fall on few tiles. */
    uint32_t coarse_tiles;
    /* Smallest batch (updates) that may be classified and binned while the
     * previous batch's replacement rounds run (serial_rounds above); 0 =
     * default 4,194,304.  Below it the host work of a batch outlasts its
     * device work, so the GPU idles during the rounds anyway, and running
     * the rounds' reductions beside the next batch's kernels would only
     * lengthen them. */
    uint32_t overlap_min_batch;
} cupk_opts;

/* Counters, cumulative since init. */
typedef struct {
    uint64_t updates;            /* updates applied                              */
    uint64_t batches;            /* batches applied                              */
    uint64_t flagged;            /* updates the device classified as structural  */
    uint64_t links;              /* forest links (inserts and replacements)      */
    uint64_t cuts;               /* forest cuts (deleted forest edges)           */
    uint64_t rounds;             /* replacement rounds run                       */
    uint64_t sets_reduced;       /* vertex sets / fragments reduced              */
    uint64_t slabs_reduced;      /* vertex sketches read by set reductions       */
    uint64_t sample_failed;      /* trees whose sample failed (kept dirty)       */
    uint64_t scatter_launches;   /* scatter kernel launches                      */
    double scatter_ms;           /* summed scatter kernel time of timed launches */
    double bin_ms;               /* summed binning time of timed launches        */
    double host_wait_ms;         /* host time waiting for classification results */
    double host_flags_ms;        /* host time applying flagged updates to forest */
    double host_rounds_ms;       /* host time in replacement rounds (incl. GPU)  */
    uint64_t reverts;            /* exact mode: batch tails scattered again to
                                    undo speculation past a cut                 */
    uint64_t level_passes;       /* levels mode: restoration passes              */
    uint64_t level_repairs;      /* levels mode: violating components repaired   */
    uint64_t level_failed;       /* levels mode: one-column queries that failed  */
    uint64_t walks_contracted;   /* runs of flagged updates walked contracted    */
    uint64_t walks_fallback;     /* runs whose piece search gave up (walked one
                                    update at a time)                           */
    uint64_t timed_launches;     /* scatter launches timed (time_kernels)        */
    uint64_t timed_updates;      /* updates in the timed launches                */
    uint64_t pieces_sketchless;  /* first rounds whose left-out old-root piece of
                                    the lone broken tree was carried unlisted,
                                    without a sketch                            */
    uint64_t sets_complemented;  /* trees holding such a piece reduced from the
                                    other pieces (all pieces XOR to zero)       */
    uint64_t timed_buckets;      /* buckets the timed staged scatter launches
                                    changed in HBM (nonzero folded delta, or a
                                    record's deep-row bucket): 32 B of
                                    compulsory traffic each (read + write)      */
    uint64_t overlapped;         /* batches classified and binned while the
                                    previous batch's rounds ran                 */
} cupk_counters_t;

/* Bytes of device memory the sketch of (V, C, D) occupies. */
size_t cupk_sketch_bytes(uint32_t V, uint32_t C, uint32_t D);

/* sketch_init — create a context holding V zeroed vertex sketches of C
 * columns x D depth buckets (Sec. 2.1 l0 sketches; App. A.1.1: O(log V)
 * sketches per vertex, each an array of machine words).
 *   V: vertex count, 2 <= V <= 2^31.
 *   C: columns; 0 means ceil(log2 V).  1 <= C <= 64.
 *   D: depth buckets per column; 0 means 2*ceil(log2 V).  2 <= D <= 64.
 *   seed: 64-bit master seed of the column hashes.
 *   opts: NULL for defaults.
 * On success *out owns device memory for the sketch (unless
 * opts->sketch_device_ptr is given), label and parent arrays and staging
 * buffers, and a host spanning forest of the empty graph.
 * Errors: CUPK_EINVAL (bad sizes), CUPK_ENOMEM, CUPK_EDEVICE. */
int cupk_sketch_init(cupk_ctx **out, uint32_t V, uint32_t C, uint32_t D,
                     uint64_t seed, const cupk_opts *opts);

/* Release everything the context owns.  NULL is a no-op. */
void cupk_free(cupk_ctx *ctx);

/* apply_updates — apply a batch of n stream updates ((u_i, v_i), +-1)
 * in order (App. A.1 graph-stream model; fully-dynamic connectivity problem,
 * App. A.1.2).  u, v, is_delete are host arrays of n elements, read before
 * return; endpoints may come in either order.
 * Every update toggles its edge in both endpoints' sketches (over F2 an
 * insert and a delete are the same operation; cutset Update, Sec. 2.2.1).
 * The forest is then brought up to date: inserts joining two trees link
 * them, deletes of forest edges cut them, and at the end of the batch
 * replacement rounds reconnect broken trees from their aggregate sketches.
 * After return, cupk_connected reflects all n updates.
 * Validation is all-or-nothing: u == v or an endpoint >= V returns
 * CUPK_EINVAL and applies nothing.  Inserting a present edge or deleting an
 * absent one breaks the stream contract (App. A.1) and is not detected.
 * n == 0 is a no-op. */
int cupk_apply_updates(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v,
                       const uint8_t *is_delete, size_t n);

/* apply_updates_device — cupk_apply_updates for a batch already in device
 * memory, ordered on streams (graph-stream model, App. A.1; cutset Update,
 * Sec. 2.2.1; updates buffered and flushed before queries, Sec. 4.3).
 *   d_packed: n packed words in device memory: lo32 = one endpoint, bits
 *     32..62 = the other, bit 63 = 1 for a delete.  Owned by the caller and
 *     only read.
 *   hip_stream: the hipStream_t on which the caller produced d_packed (NULL =
 *     the null stream).  The library reads the batch after the work queued
 *     on hip_stream before this call, and makes hip_stream wait for the
 *     last kernel that reads the batch: work the caller queues on hip_stream
 *     afterwards (freeing or reusing the buffer, reading the sketch) runs
 *     after it.  Used with any other stream, the caller keeps the buffer
 *     alive until cupk_sync returns.
 * The call returns once the batch's device work is queued; it does not
 * wait for the GPU.  The host part of the batch (links and cuts of the
 * flagged updates, replacement rounds) stays pending until the next call on
 * ctx that needs it: the next apply call, cupk_sync, cupk_connected and
 * every other call that reads the forest, the sketch or the counters.  The
 * next apply call of a large batch (cupk_opts.overlap_min_batch) overlaps
 * the two: it classifies and bins its batch while the pending batch's
 * replacement rounds run (cupk_opts.serial_rounds turns this off).
 * Validation runs on the GPU: a batch with u == v or an endpoint >= V
 * applies nothing, and CUPK_EINVAL is returned by the call that completes
 * its host part (the next such call).  In exact and levels modes the call
 * completes the batch before returning.  n == 0 is a no-op.
 * Errors: CUPK_EINVAL (null pointer; an earlier invalid batch),
 *   CUPK_ENOMEM, CUPK_EDEVICE. */
int cupk_apply_updates_device(cupk_ctx *ctx, const uint64_t *d_packed, size_t n,
                              void *hip_stream);

/* component_sketch — aggregate sketch of a vertex set U: XOR of the
 * members' sketches (App. A.1.1 sketch addition; the cutset's component
 * aggregate, Sec. 2.2.1).  By cancellation it equals the sketch of the cut
 * of U.  verts: n distinct vertex ids (host); duplicates cancel in pairs.
 * out: C*D buckets, canonical order, in host or device memory (the kind is
 * found with hipPointerGetAttributes; device memory is written on the
 * library's stream and the call waits for it).  Reflects all applied
 * updates.  Errors: CUPK_EINVAL for an id >= V. */
int cupk_component_sketch(cupk_ctx *ctx, const uint32_t *verts, size_t n,
                          cupk_bucket *out);

/* component_sketch_batch — k aggregate sketches in one launch.
 * offsets: k+1 host offsets into verts (CSR); set j is
 * verts[offsets[j] .. offsets[j+1]).  out: k*C*D buckets, set j at
 * out[j*C*D], host or device memory as for cupk_component_sketch.  Sets
 * may have any sizes, including 0. */
int cupk_component_sketch_batch(cupk_ctx *ctx, const uint64_t *offsets, size_t k,
                                const uint32_t *verts, cupk_bucket *out);

/* component_sketch_batch_noalloc — cupk_component_sketch_batch for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the call allocates no device or host
 * memory.  Its members, offsets and aggregates live in a file-scope device
 * array of about 20 MiB, one per GPU, taken when the library's code is
 * loaded on that GPU and held until the process ends; its address is looked
 * up once per device by cupk_sketch_init.
 *   offsets, k, verts: as for cupk_component_sketch_batch (host arrays).
 *   out_device: k*C*D buckets in device memory, canonical order.
 * Limits: k <= 4096 sets, offsets[k] <= 2^20 members, k*2*C*D <= 2^21
 * aggregate words; beyond them CUPK_EINVAL with nothing done.  A device
 * batch still pending from cupk_apply_updates_device is also CUPK_EINVAL
 * (completing it may allocate: call cupk_sync first).  The call returns
 * when out_device is written.  Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (other threads, other contexts
 * on the same device) race; the array keeps the last call's contents and
 * each call zero-fills the part it uses.
 * Errors: CUPK_EINVAL, CUPK_EDEVICE. */
int cupk_component_sketch_batch_noalloc(cupk_ctx *ctx, const uint64_t *offsets, size_t k,
                                        const uint32_t *verts, cupk_bucket *out_device);

/* sample_cut_edge — query one aggregate sketch (cutset Query, Sec. 2.2.1;
 * l0 sampling, App. A.1.1).  sketch: C*D buckets (host), canonical order.
 * Returns CUPK_OK with *u < *v the edge of the first good bucket,
 * CUPK_EMPTY when every word is zero, CUPK_SAMPLE_FAILED otherwise. */
int cupk_sample_cut_edge(cupk_ctx *ctx, const cupk_bucket *sketch, uint32_t *u,
                         uint32_t *v);

/* sample_cut_edge_batch — k queries in one launch; status[j], u[j], v[j]
 * receive the result of sketch j (host arrays of k). */
int cupk_sample_cut_edge_batch(cupk_ctx *ctx, const cupk_bucket *sketches, size_t k,
                               int32_t *status, uint32_t *u, uint32_t *v);

/* connected — Connected(u, v) on the current graph (Sec. 2.1): 1 or 0 after
 * every update applied so far; negative on error (CUPK_EINVAL for ids
 * >= V). */
int cupk_connected(cupk_ctx *ctx, uint32_t u, uint32_t v);

/* ---- introspection (parity, tests, benchmarks) ------------------------- */

/* Sketches of vertices w0 .. w0+nv-1 into out (host, nv*C*D buckets,
 * canonical order per vertex). */
int cupk_get_sketch(cupk_ctx *ctx, uint32_t w0, uint32_t nv, cupk_bucket *out);

/* Order-independent digest of the whole sketch:
 *   sum over (w,c,d) of mix(alpha ^ rotl(gamma, 32) ^ mix(((w*C+c)*D+d) ^ seed))
 * modulo 2^64, mix = SplitMix64 finalizer. */
int cupk_digest(cupk_ctx *ctx, uint64_t *out);

/* Number of trees in the forest (= components, w.h.p.). */
int cupk_num_components(cupk_ctx *ctx, uint64_t *out);

/* Forest edges: writes up to cap pairs (u < v) and sets *n to the number of
 * forest edges.  Returns CUPK_EINVAL if cap < *n (nothing written then). */
int cupk_forest_edges(cupk_ctx *ctx, uint32_t *u, uint32_t *v, size_t cap, size_t *n);

/* Component label of every vertex (host array of V).  Two vertices are
 * connected iff their labels are equal. */
int cupk_component_labels(cupk_ctx *ctx, uint32_t *out);

/* Levels mode: edges of the forest of `level` (1..C; C is the forest of
 * cupk_forest_edges), same contract as cupk_forest_edges.
 * Errors: CUPK_EINVAL (not in levels mode, level out of range, cap too
 * small: *n is then the count needed). */
int cupk_level_forest_edges(cupk_ctx *ctx, uint32_t level, uint32_t *u, uint32_t *v, size_t cap,
                            size_t *n);

int cupk_counters(cupk_ctx *ctx, cupk_counters_t *out);

/* Wait for all work the context queued. */
int cupk_sync(cupk_ctx *ctx);

/* ---- static connectivity from the sketch -----------------------------------
 * Connected components of the current graph computed from the vertex
 * sketches alone, ignoring the maintained forest: Boruvka's algorithm over
 * supernodes, where a supernode's incident edge is recovered by querying the
 * XOR of its members' sketches and merging supernodes merges their sketches
 * (App. A.1.1, the AGM connectivity sketch).  Rounds take the active
 * supernodes in ascending order of smallest vertex; each sampled edge merges
 * the two supernodes unless they are already one (recorded as a spanning
 * forest edge); an EMPTY supernode not merged in the round is a whole
 * component; a round that merges nothing ends the run (supernodes whose
 * query failed then stay as they are, counted in sample_failed).
 * labels: NULL or V host words, set to the smallest vertex of each vertex's
 *   component.
 * eu, ev: NULL or V-1 host words each; the merge edges (eu < ev) in merge
 *   order; info->n_edges of them are written.
 * info: NULL or filled with the counts below.
 * Reflects every update applied so far; the forest is not touched.  Uses
 * device scratch of up to V/2 set sketches.
 * Errors: CUPK_EINVAL (serving loop running), CUPK_ENOMEM, CUPK_EDEVICE. */
typedef struct {
    uint32_t n_components;
    uint32_t rounds;
    uint32_t sample_failed;
    uint32_t n_edges;
} cupk_static_info;

int cupk_static_components(cupk_ctx *ctx, uint32_t *labels, uint32_t *eu, uint32_t *ev,
                           cupk_static_info *info);

/* ---- autotuner ------------------------------------------------------------
 * Picks the staged scatter's tile geometry (lane layout, vertices per LDS
 * tile, depth rows in LDS, records per work item) by timing every
 * candidate's device work (classification, tile scan, binning, scatter) on
 * a sample batch and timing the best four again (two alternating passes,
 * which decide), then the tiles per coarse bin of the two-level binning for
 * that setting; and derives a batch-size schedule: the device time of prefixes n/128 .. n of
 * the sample plus the host time per batch this context has measured so far
 * (flag walk and replacement rounds, nearly independent of the batch size);
 * batch_target is the smallest prefix whose whole-path rate reaches 80% of
 * the best one.  The serving loop then uses batch_target as its batch size
 * unless cupk_serve_opts.max_batch is set.  Each candidate applies the
 * sample an even number of times, so the XOR toggles cancel and the sketch
 * is left exactly as it was; the forest is not touched.
 * d_sample: n packed updates in device memory (format of
 * cupk_apply_updates_device).  The chosen setting stays in force on ctx.
 * Errors: CUPK_EINVAL (not in staged mode, n == 0, invalid sample). */
typedef struct {
    uint32_t tile_vertices;    /* chosen                                       */
    uint32_t lds_rows;
    uint32_t chunk_records;
    uint32_t candidates;       /* settings timed                               */
    double best_ms;            /* device time of the sample, chosen setting
                                  (its second timing)                          */
    double before_ms;          /* same with the setting in force before (its
                                  first timing)                                */
    uint32_t batch_target;     /* smallest timed batch reaching 80% of the
                                  best whole-path rate (batch-size schedule)  */
    double batch_ms[8];        /* device time of prefixes n/128, ... , n       */
    uint32_t batch_sizes[8];
    double host_ms_per_batch;  /* host time per batch the schedule assumed     */
    uint32_t tile_layout;      /* chosen CUPK_LAYOUT_*                         */
    uint32_t coarse_tiles;     /* chosen tiles per coarse bin (0: one level)   */
} cupk_tune_result;

int cupk_autotune(cupk_ctx *ctx, const uint64_t *d_sample, size_t n, cupk_tune_result *out);

/* ---- serving loop -------------------------------------------------------
 * Continuous batching of interleaved update and query requests.  While the
 * loop runs, a worker thread owns the context: use only the calls below on
 * it until cupk_serve_stop.  Requests are ordered by submission; a query
 * observes exactly the updates submitted before it (queries flush pending
 * updates first, Sec. 4.3).  Update requests submitted while a batch is on
 * the GPU join the next batch.  Admission is by device memory: an admitted
 * request holds a slot of a device ring (mem_budget_bytes) and is uploaded
 * at once on a copy stream, overlapping the batch on the GPU; the worker
 * applies each batch straight from the ring. */

typedef struct {
    uint32_t max_batch;        /* updates per device batch (0 = the autotuned
                                  batch target if cupk_autotune ran, else
                                  1<<20)                                       */
    uint32_t nonblocking;      /* 1: refuse with CUPK_EBUSY instead of waiting */
    size_t mem_budget_bytes;   /* device ring holding admitted update requests
                                  until applied, 8 B per update (0 = 64 MiB;
                                  as much pinned host staging again);
                                  admission waits for room                    */
} cupk_serve_opts;

typedef struct {
    uint64_t update_requests;  /* update requests admitted                     */
    uint64_t queries;          /* queries admitted                             */
    uint64_t batches;          /* device batches applied                       */
    uint64_t updates;          /* updates applied                              */
    uint64_t admission_waits;  /* submissions that waited for memory           */
    double query_p50_us;       /* query latency, submission to answer          */
    double query_p99_us;
    double query_max_us;
} cupk_serve_stats_t;

/* Start the loop.  CUPK_EINVAL if it already runs. */
int cupk_serve_start(cupk_ctx *ctx, const cupk_serve_opts *opts);

/* Submit n updates (host arrays, copied before return; validated
 * all-or-nothing: CUPK_EINVAL for u == v or an endpoint >= V, or for a
 * request larger than the memory budget).  *ticket identifies it.  Blocks
 * for admission unless the loop is non-blocking (then CUPK_EBUSY).  Safe to
 * call from several threads. */
int cupk_submit_updates(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v,
                        const uint8_t *is_delete, size_t n, uint64_t *ticket);

/* Submit Connected(u, v). */
int cupk_submit_query(cupk_ctx *ctx, uint32_t u, uint32_t v, uint64_t *ticket);

/* A burst of n connectivity queries (the paper's streams interleave bursts
 * of queries between update periods, App. C.1).  The burst is one request:
 * it observes exactly the updates submitted before it, and its answers
 * (1 connected, 0 not, < 0 error) are written to out[0..n-1], a host array
 * the caller keeps alive until cupk_wait on *ticket returns (its result is
 * CUPK_OK or the first error).  Every query of the burst is counted with
 * the burst's latency (submission to last answer).
 * Errors: CUPK_EINVAL (loop not running, an endpoint >= V). */
int cupk_submit_queries(cupk_ctx *ctx, const uint32_t *u, const uint32_t *v, size_t n,
                        int32_t *out, uint64_t *ticket);

/* Wait for a ticket; *result = 1/0 for a query, the apply status (0 or a
 * negative error) for an update request.  Each ticket is waited for once. */
int cupk_wait(cupk_ctx *ctx, uint64_t ticket, int32_t *result);

int cupk_serve_stats(cupk_ctx *ctx, cupk_serve_stats_t *out);
int cupk_serve_reset_stats(cupk_ctx *ctx);

/* Drain the queue and stop the loop; the context is usable again. */
int cupk_serve_stop(cupk_ctx *ctx);

/* Static text of a return code. */
const char *cupk_strerror(int code);

/* Text of the last error on ctx (empty if none); with ctx == NULL, the
 * text of the last failed cupk_sketch_init on this thread. */
const char *cupk_last_error(cupk_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* CUPK_H */
