// Launch wrappers of the gfx950 kernels.  Host code calls only these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cupk {

// Device view of the resident sketch.
// Internal layout: bucket (w, d, c) of vertex w at word ((w*D + d)*C + c)*2,
// alpha at +0 and gamma at +1 ("depth-major inside a vertex": the shallow
// rows that take most updates are contiguous at the front of a vertex).
struct DevSketch {
    uint64_t *b;           // 2*V*C*D words
    const uint64_t *seeds; // C column seeds
    uint32_t V, C, D;
};

// The batch a step works on, read by the kernels from device memory so that
// one captured graph serves batches of any size up to its capacity.
struct BatchDesc {
    const uint64_t *upd;  // packed updates
    uint32_t n;           // number of updates
    uint32_t pad;
};

// Header words.  ERR / NFLAG / NFLAG_DEL are accumulated by the classify
// kernel; SCAT_DONE counts finished blocks of the scatter kernel, whose last
// block clears ERR / NFLAG / NFLAG_DEL (and SCAT_DONE) for the next batch.
// SEQ counts published headers: the one-block kernel after classify copies
// ERR / NFLAG / NFLAG_DEL to the host, then the incremented SEQ (release
// store), which the host waits for.
enum {
    HDR_ERR = 0,
    HDR_NFLAG = 1,
    HDR_NFLAG_DEL = 2,
    HDR_SCAT_DONE = 3,
    HDR_SEQ = 4,
    HDR_INLINE = 5,  // host copy only: the flagged updates came with the header
    HDR_WORDS = 8
};

// Flagged updates of a batch with at most kInlineFlags of them (and at most
// kInlineMaxBlocks classify blocks) are compacted in stream order straight
// into host memory by the one-block kernel after classification, before it
// publishes the header (HDR_INLINE set): no compaction kernels, no copy.
constexpr uint32_t kInlineFlags = 16384;
constexpr uint32_t kInlineMaxBlocks = 8192;
struct FlagInline {
    const uint64_t *fupd;  // per-block regions (the classify kernel's output)
    const uint32_t *fcnt;  // flags per classify block
    uint32_t *fdel;        // flagged deletes per classify block
    uint32_t nb;           // classify blocks
    uint64_t *hflags;      // coherent pinned host memory; null: never inline
    // 1: the scan after the classify kernel leaves the flags and the header
    // alone (launch_reflag checks the flags against a newer forest and
    // publishes them later); 0: it publishes them
    uint32_t tiles_only;
};

// Where the one-block tile scan writes: bin offsets and fill cursors
// (ntiles + 1 words each), work items (tile, chunk) and their number.
// Tile counts are kept in `groups` copies of ntiles words (1, or
// kCntGroups when classify blocks also store where their records start:
// block b adds to copy b % kCntGroups, so that fewer blocks meet on one
// counter).  goff (groups * ntiles words, may be null) receives where each
// copy's records start in every tile's bin.
constexpr uint32_t kCntGroups = 4;
// sums (2 * tile_scan_chunks(ntiles) words, may be null): scratch of the
// multi-block scan, used (and required) when ntiles > kScanOneBlockTiles:
// the one-block kernel then only publishes the header and two multi-block
// kernels scan the counts (one count copy only).
constexpr uint32_t kScanOneBlockTiles = 4096;
struct ScanArgs {
    uint32_t *off, *cur, *items, *nitems;
    uint32_t chunk, items_cap;
    uint32_t groups;
    uint32_t *goff;
    uint32_t *sums;
};
uint32_t tile_scan_chunks(uint32_t ntiles);

// Staged-scatter lane layouts: one lane per record (its C columns in turn)
// or one lane per (record, column) pair.
constexpr uint32_t kLayoutRecord = 1;
constexpr uint32_t kLayoutPair = 2;

struct StagedParams {
    uint32_t tile_shift;   // vertices per tile = 1 << tile_shift
    uint32_t rows;         // depth rows held in LDS (d < rows)
    uint32_t layout;       // kLayoutRecord or kLayoutPair
    uint32_t ntiles;
    uint32_t chunk;        // max records per work item
    uint32_t items_cap;    // capacity of the work-item array
    uint32_t grid;         // blocks of the persistent tile kernel (0 = default)
};

// Per-batch: validation, structural classification and compaction of the
// flagged updates.  hdr's ERR / NFLAG / NFLAG_DEL words must be zero (as
// the previous batch's scatter leaves them).  A one-block kernel after it
// writes their final values to `hout` (coherent pinned host memory,
// HDR_WORDS words: no copy needed), then the next sequence number at
// hout[HDR_SEQ].  When `tile_cnt` is non-null the classify kernel
// also counts how many endpoint records each vertex tile gets, and the
// one-block kernel scans the counts into `sa` (sa.off set).  Flagged updates of
// classify block b (positions [b*4096, (b+1)*4096)) land in stream order at
// offsets b*4096.. of fupd (capacity: the batch rounded up to a multiple of
// 4096); fcnt[b] receives their number.  fpos (may be null) receives each
// flagged update's position in the batch, alongside.  grid_n sizes the
// grids (the batch size, or the capacity of a captured graph); the kernels
// read the batch from device memory at `desc` (captured graphs) or, when
// desc is null, from `dv`.  When `tile_rel` is non-null (tile counts on, at
// most kRelMaxTiles tiles; classify_blocks(grid_n) * ntiles words; tile_cnt
// of kCntGroups * ntiles words and sa.groups == kCntGroups), block b also
// stores at tile_rel[b*ntiles + t] where its records start among the
// records of count copy b % kCntGroups in tile t (written only for tiles it
// has records in), so that the fill reserves nothing.
// blk (may be null): the block labels (launch_block_labels) of the forest
// in lp; inserts between two uniform blocks then skip the forest words.
constexpr uint32_t kRelMaxTiles = 2048;
hipError_t launch_classify(hipStream_t s, const BatchDesc *desc, BatchDesc dv, uint32_t grid_n,
                           uint32_t V, const uint64_t *lp, const uint32_t *blk, uint32_t *hdr,
                           uint64_t *fupd, uint32_t *fpos, uint32_t *fcnt, uint32_t *tile_cnt,
                           uint32_t tile_shift, uint32_t ntiles, const ScanArgs &sa,
                           uint32_t *hout, const FlagInline &fi, uint32_t *tile_rel);
uint32_t classify_blocks(uint32_t n);
// lp[w] = lbl[w] | par[w] << 32 (the forest as the classify kernel reads it:
// one 8-byte load per endpoint gives its label and its parent).
hipError_t launch_pack_forest(hipStream_t s, const uint32_t *lbl, const uint32_t *par, uint64_t *lp,
                              uint32_t V);
// Block labels: blk[b] (b < ceil(V / 64)) = the label that all vertex ids
// [64 b, 64 b + 64) below V share, or kBlkMixed.  With `pages` (np page ids
// in device memory, pages of 2^pshift ids, pshift in [6, 16]) only the
// blocks of those pages are recomputed.  The classify kernel (blk non-null)
// decides an insert whose endpoints both lie in uniform blocks by them.
constexpr uint32_t kBlkShift = 6;
constexpr uint32_t kBlkMixed = 0xffffffffu;
hipError_t launch_block_labels(hipStream_t s, const uint32_t *lbl, uint32_t V, uint32_t *blk,
                               const uint32_t *pages, uint32_t np, uint32_t pshift);
// Refresh np pages of 2^pshift vertices of the device forest from a staging
// block: np page ids, then each page's labels in turn, then each page's
// parents in turn (2^pshift words per page; entries past V are ignored).
hipError_t launch_forest_pages(hipStream_t s, const uint32_t *stage, uint32_t np, uint32_t pshift,
                               uint32_t V, uint32_t *lbl, uint32_t *par, uint64_t *lp);
// Second half of a classification launched with fi.tiles_only = 1: with
// `check`, keep, in each classify block's region of fi.fupd (in place,
// stream order kept), only the updates the classify kernel's rule flags
// against the forest in `lp`, and rewrite fi.fcnt and fi.fdel; pack the
// regions into one ordered list at oupd (foff: fi.nb words of scratch), as
// launch_flag_compact does; then publish the flag counts, the short flag
// lists and the header as launch_classify does otherwise.  Exact when `lp`
// is a coarsening of the forest the regions were flagged against that keeps
// all its edges (it then flags a subset of what that forest flagged).  A
// rejected batch (header error) keeps its regions.
hipError_t launch_reflag(hipStream_t s, uint32_t V, const uint64_t *lp, uint32_t *hdr,
                         uint64_t *fupd, uint32_t *hout, const FlagInline &fi, uint32_t *foff,
                         uint64_t *oupd, bool check);

// Pack the per-block flag regions into one list in stream order (foff:
// classify_blocks(n) words of scratch); positions too when fpos and opos
// are not null.
hipError_t launch_flag_compact(hipStream_t s, uint32_t n, const uint64_t *fupd,
                               const uint32_t *fpos, const uint32_t *fcnt, uint32_t *foff,
                               uint64_t *oupd, uint32_t *opos);

// Small batches: header, flagged updates (stream order) and their positions
// of one batch of at most kSmallMax updates, written by one kernel straight
// into host memory.
constexpr uint32_t kSmallMax = 4096;
struct SmallResult {
    uint32_t hdr[HDR_WORDS];
    uint64_t fupd[kSmallMax];
    uint32_t fpos[kSmallMax];
};
// Classify (one block) a batch of 1..kSmallMax packed updates given in the
// arguments into `out` (coherent pinned host memory; with_pos: also
// positions), set *derr (device) to the error flag, and publish the next
// value of the counter *seqp at out->hdr[HDR_SEQ] (release store) once the
// rest of `out` is written.  Then scatter it with device atomics; the
// scatter does nothing if an update was invalid (*derr set).
hipError_t launch_small_classify(hipStream_t s, const uint64_t *upd, uint32_t n, uint32_t V,
                                 const uint32_t *lbl, const uint32_t *par, SmallResult *out,
                                 uint32_t *derr, uint32_t *seqp, bool with_pos);
hipError_t launch_small_scatter(hipStream_t s, const uint64_t *upd, uint32_t n, DevSketch sk,
                                const uint32_t *derr);

// Plain scatter: device-scope atomic XOR of (x, h) into both endpoints.
// Its last block clears the header for the next batch.
hipError_t launch_scatter_atomic(hipStream_t s, const BatchDesc *desc, BatchDesc dv,
                                 uint32_t grid_n, DevSketch sk, uint32_t *hdr);

// Staged scatter: launch_bin = fill of the per-tile bins (at the offsets
// the classify kernel's tile scan wrote: the count copy's start in
// tile_goff plus the classify block's tile_rel entry when tile_rel is
// non-null, else reserved from tile_cur);
// launch_tile = LDS-staged XOR per work item, whose last block clears the
// header for the next batch; touched (may be null) is incremented by the
// number of buckets the launch changes in HBM.
hipError_t launch_bin(hipStream_t s, const BatchDesc *desc, BatchDesc dv, uint32_t grid_n,
                      DevSketch sk, const uint32_t *hdr, const StagedParams &p,
                      uint32_t *tile_cur, uint64_t *bins, const uint32_t *tile_goff,
                      const uint32_t *tile_rel);
hipError_t launch_tile(hipStream_t s, DevSketch sk, uint32_t *hdr, const StagedParams &p,
                       const uint32_t *tile_off, const uint64_t *bins, const uint32_t *items,
                       const uint32_t *nitems, unsigned long long *touched);
// Second level of the two-level binning (used when there are more tiles
// than kFillStageTiles): bins1 holds the batch's records binned by coarse
// bin (2^fshift tiles each; the classify kernel counted them and the fill
// wrote them), total points at their number (the coarse scan's last
// offset).  Counts them per tile into tile_cnt, scans with the multi-block
// tile scan into sa (one count copy, sa.sums set) and writes them into
// their tile bins in `bins`.
constexpr uint32_t kFillStageTiles = 2048;
// Most bins the classify kernel counts in LDS (beyond, with device atomics),
// and most tiles per coarse bin (launch_fine).
constexpr uint32_t kLdsHistMax = 8192;
constexpr uint32_t kFineLdsTiles = 8192;
hipError_t launch_fine(hipStream_t s, uint32_t grid_n, const uint32_t *hdr, const uint64_t *bins1,
                       const uint32_t *total, uint32_t tile_shift, uint32_t fshift,
                       uint32_t ntiles, uint32_t *tile_cnt, const ScanArgs &sa, uint64_t *bins);
// Whether a staged-scatter geometry fits one block's LDS: the delta of
// `rows` depth rows x C columns x tv vertices (alpha and gamma), plus, in
// the pair layout, room to stage one block's worth of decoded records.
bool tile_geometry_fits(uint32_t rows, uint32_t C, uint32_t tv, uint32_t layout);

// Fill n words with zero.
hipError_t launch_zero(hipStream_t s, uint64_t *p, size_t n);
hipError_t launch_zero32(hipStream_t s, uint32_t *p, size_t n);

// Segmented XOR reduction: out[set] = XOR of src slabs listed by `idx`.
// items: triples (set, begin, end) into idx; slab = W words.
hipError_t launch_reduce(hipStream_t s, const uint64_t *src, uint32_t W, const uint32_t *idx,
                         const uint32_t *items, uint32_t nitems, uint64_t *out);

// Allocation-free aggregates (cupk_component_sketch_batch_noalloc): the
// members, set offsets and aggregates of one call live in a file-scope
// device array of kNoAllocScratchWords words, one per GPU for the life of
// the process.  Layout in words: aggregates [0, kNoAllocAggWords), then the
// kNoAllocMaxSets + 1 set offsets (uint64), then the members (uint32, two
// per word).
constexpr uint32_t kNoAllocMaxMembers = 1u << 20;
constexpr uint32_t kNoAllocMaxSets = 4096;
constexpr uint32_t kNoAllocAggWords = 1u << 21;  // 16 MiB of aggregates
constexpr size_t kNoAllocOffsWord = kNoAllocAggWords;
constexpr size_t kNoAllocMemWord = kNoAllocOffsWord + kNoAllocMaxSets + 1;
constexpr size_t kNoAllocScratchWords = kNoAllocMemWord + kNoAllocMaxMembers / 2;
// Device address of the scratch array on `device`, which must be current.
// Taken with hipGetSymbolAddress on the first call per device and kept.
hipError_t noalloc_scratch_address(int device, uint64_t **out);

// Segmented XOR reduction over CSR sets: out[j] = XOR of the slabs of
// mem[offs[j] .. offs[j+1]) for j < k (nv = offs[k] members).  Blocks take
// 16 consecutive members at a time and find their set by binary search, so
// no work-item list is needed.  out (k*W words) must be zeroed first.
hipError_t launch_reduce_csr(hipStream_t s, const uint64_t *src, uint32_t W,
                             const uint32_t *mem, const uint64_t *offs, uint32_t k,
                             uint32_t nv, uint64_t *out);

// Query each of k aggregate sketches (bucket (c,d) at word (c*sc + d*sd)*2).
// res: 3 words per set (status, u, v).
hipError_t launch_sample(hipStream_t s, const uint64_t *sig, uint32_t k, uint32_t V, uint32_t C,
                         uint32_t D, uint32_t sc, uint32_t sd, uint64_t set_stride,
                         const uint64_t *seeds, int32_t *res);

// Digest of the whole sketch, added into *out (zero it first).
hipError_t launch_digest(hipStream_t s, DevSketch sk, uint64_t master_seed, uint64_t *out);

// Copy nv sketches from internal layout (first vertex w0) or from an
// internal-layout aggregate array (w0 ignored when `agg` is set) into
// canonical (c, d) order.
hipError_t launch_to_canonical(hipStream_t s, const uint64_t *src, uint32_t C, uint32_t D,
                               uint64_t nv, uint64_t *dst);

// Multi-level hierarchy: reduce set k over column col[k] only (items:
// (set, begin, end) triples over idx, vertex ids; out: k sets x 2D words,
// [depth][alpha, gamma], zeroed by the caller), then query each set's one
// column (res: status, u, v per set, as launch_sample).  D <= 64.
hipError_t launch_reduce_col(hipStream_t s, const uint64_t *sk, uint32_t C, uint32_t D,
                             const uint32_t *idx, const uint32_t *items, uint32_t nitems,
                             const uint32_t *col, uint64_t *out);
hipError_t launch_sample_col(hipStream_t s, const uint64_t *agg, uint32_t k, uint32_t V,
                             uint32_t D, const uint32_t *col, const uint64_t *seeds,
                             int32_t *res);

}  // namespace cupk
