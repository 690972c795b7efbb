// gfx950 kernels of the sketch hot path.
//
// All arithmetic is integer / GF(2): the sketch is a set of 64-bit words
// combined by XOR (App. A.1.1 of arXiv 2509.14433), so there is no matrix
// work and no floating point.  What bounds these kernels is HBM (and L2/LDS)
// traffic and, for the staged scatter, the 64-bit integer hashing.
//
// Bucket layout in HBM: bucket (w, d, c) at word ((w*D + d)*C + c)*2, alpha
// then gamma.  A vertex's shallow depth rows, which receive almost all
// updates (depth d is hit with probability 2^-(d+1)), are contiguous.
#include "kernels.hpp"

#include <mutex>

namespace cupk {

#define DEVI __device__ __forceinline__

// SplitMix64 output finalizer (Steele, Lea, Flood 2014).
DEVI uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The same finalizer after its first step.  That step, z ^ (z >> 30), is
// linear over XOR, so for z = x ^ seed it equals (x ^ (x >> 30)) ^
// (seed ^ (seed >> 30)): callers hashing one x under many seeds compute
// the two halves once each.
DEVI uint64_t mix64_tail(uint64_t z)
{
    z *= 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

DEVI uint64_t mix64_head(uint64_t z) { return z ^ (z >> 30); }

// Depth of a column hash: trailing zero count, capped at D-1.
DEVI uint32_t depth_of(uint64_t h, uint32_t D)
{
    uint32_t z = h ? (uint32_t)__builtin_ctzll(h) : 64u;
    return z < D - 1 ? z : D - 1;
}

// Packed update: lo32 = one endpoint, bits 32..62 = the other, bit 63 = delete.
DEVI bool unpack(uint64_t p, uint32_t V, uint32_t &u, uint32_t &v, bool &del)
{
    uint32_t a = (uint32_t)p;
    uint32_t b = (uint32_t)(p >> 32) & 0x7fffffffu;
    del = (p >> 63) != 0;
    u = a < b ? a : b;
    v = a < b ? b : a;
    return a != b && v < V;
}

// Number of set bits of m below this lane.
DEVI uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

DEVI void gxor(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DEVI void lxor(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// Classification: validate the batch, flag structural candidates and count
// endpoint records per vertex tile.
//
// Flagged (using the forest as it stood at the start of the batch):
//   insert {u,v} with lbl[u] != lbl[v]               (may join two trees)
//   delete {u,v} that is a forest edge (par[u]==v or par[v]==u), or with
//   lbl[u] != lbl[v] (an edge linked earlier in this same batch)
// Everything else can only touch the sketch.  Block b covers positions
// [b*4096, (b+1)*4096) with 512 threads; each thread issues the loads of
// all its 8 updates (and their label words) before using any, since the
// kernel is bound by the latency of those dependent loads.  The block
// writes its flagged updates in
// stream order into its own region of the flag buffers (same offsets), at
// positions from one prefix over (step, wave) counts; cnt[b] gets their
// number.  k_flag_compact later packs the regions into one ordered list.
// ---------------------------------------------------------------------------
constexpr uint32_t kClsThreads = 512;  // 8 updates per thread: 16 label loads in flight
constexpr uint32_t kClsPerBlock = 4096;
constexpr uint32_t kClsPerThread = kClsPerBlock / kClsThreads;
constexpr uint32_t kClsWaves = kClsThreads / 64;
static_assert(kClsPerThread * kClsWaves == 64, "one wave scans the (step, wave) counts");

constexpr uint32_t kScanThreads = 1024;

// Block-wide exclusive scan of one value per thread; returns the prefix and
// sets `total`.
template <uint32_t NT>
DEVI uint32_t block_exscan(uint32_t x, uint32_t &total, uint32_t *sh)
{
    const uint32_t lane = __lane_id();
    const uint32_t wid = threadIdx.x / 64;
    uint32_t inc = x;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    if (threadIdx.x < 64) {
        uint32_t w = threadIdx.x < NT / 64 ? sh[threadIdx.x] : 0u;
        uint32_t wi = w;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(wi, o);
            if (lane >= o) wi += y;
        }
        if (threadIdx.x < NT / 64) sh[64 + threadIdx.x] = wi - w;
        if (threadIdx.x == NT / 64 - 1) sh[128] = wi;
    }
    __syncthreads();
    const uint32_t ex = sh[64 + wid] + inc - x;
    total = sh[128];
    __syncthreads();
    return ex;
}

// Tile scan (one block, after the classify kernel): publishes the header
// to the host, then (staged path, a.off set) scans the per-tile record
// counts into bin offsets (and fill cursors) and lists the work items
// (tile, chunk), a chunk being at most `chunk` records of one tile's bin.
// The counts are zeroed for the next batch.
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint32_t *__restrict__ cnt,
                                                            uint32_t ntiles, ScanArgs a,
                                                            uint32_t *__restrict__ hdr,
                                                            uint32_t *__restrict__ hout,
                                                            FlagInline fi)
{
    __shared__ uint32_t sh[160];
    __shared__ uint32_t boff[kInlineMaxBlocks];
    static_assert(kInlineFlags < 65536 && kClsPerBlock < 65536, "packed region words");
    const bool err = hdr[HDR_ERR] != 0;
    if (!fi.tiles_only) {
        // the batch's flag counts: sums of the classify blocks' counts
        uint32_t nflag, nflag_del;
        {
            uint32_t a = 0, b = 0;
            for (uint32_t i = threadIdx.x; i < fi.nb; i += kScanThreads) {
                a += fi.fcnt[i];
                b += fi.fdel[i];
            }
            block_exscan<kScanThreads>(a, nflag, sh);
            block_exscan<kScanThreads>(b, nflag_del, sh);
        }
        // few flagged updates: compact them into host memory in stream order
        // (one wave per classify block's region)
        const bool inl = fi.hflags && !err && nflag <= kInlineFlags && fi.nb <= kInlineMaxBlocks;
        if (inl && nflag) {
            uint32_t carry = 0;
            for (uint32_t base = 0; base < fi.nb; base += kScanThreads) {
                const uint32_t b = base + threadIdx.x;
                const uint32_t c = b < fi.nb ? fi.fcnt[b] : 0u;
                uint32_t tot;
                const uint32_t ex = block_exscan<kScanThreads>(c, tot, sh);
                // count (<= 4096) and start (<= kInlineFlags) of the region,
                // packed: the copy below reads no global count again
                if (b < fi.nb) boff[b] = c << 16 | (carry + ex);
                carry += tot;
            }
            __syncthreads();
            const uint32_t lane = __lane_id();
            for (uint32_t b = threadIdx.x / 64; b < fi.nb; b += kScanThreads / 64) {
                const uint32_t w = boff[b];
                const uint32_t c = w >> 16, o = w & 0xffffu;
                for (uint32_t k = lane; k < c; k += 64)
                    fi.hflags[o + k] = fi.fupd[(size_t)b * kClsPerBlock + k];
            }
            // every wave waits until its stores have been acknowledged; thread
            // 0's system-scope release of the sequence number below then writes
            // back L2 once for the whole block (a system fence in every wave
            // would write it back once per wave)
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        // the header goes straight to host memory (no copy, no event): words
        // first, then the sequence number with release semantics
        if (threadIdx.x == 0) {
            hout[HDR_ERR] = hdr[HDR_ERR];
            hdr[HDR_NFLAG] = nflag;
            hdr[HDR_NFLAG_DEL] = nflag_del;
            hout[HDR_NFLAG] = nflag;
            hout[HDR_NFLAG_DEL] = nflag_del;
            hout[HDR_INLINE] = inl ? 1u : 0u;
            const uint32_t seq = hdr[HDR_SEQ] + 1;
            hdr[HDR_SEQ] = seq;
            __hip_atomic_store(&hout[HDR_SEQ], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
    if (!a.off || a.sums) return;  // no tile counts, or the multi-block kernels scan them
    const uint32_t ng = a.groups;  // count copies (1 or kCntGroups)
    if (err) {
        // rejected batch: leave the counts zeroed for the next one
        for (uint32_t t = threadIdx.x; t < ng * ntiles; t += blockDim.x) cnt[t] = 0;
        if (threadIdx.x == 0) *a.nitems = 0;
        return;
    }
    const uint32_t chunk = a.chunk, items_cap = a.items_cap;
    uint32_t *off = a.off, *cur = a.cur, *items = a.items;
    uint32_t carry_r = 0, carry_i = 0;
    for (uint32_t base = 0; base < ntiles; base += kScanThreads) {
        const uint32_t t = base + threadIdx.x;
        uint32_t c = 0;
        uint32_t cg[kCntGroups];
#pragma unroll
        for (uint32_t g = 0; g < kCntGroups; g++) {
            cg[g] = 0;
            if (t < ntiles && g < ng) {
                cg[g] = cnt[g * ntiles + t];
                cnt[g * ntiles + t] = 0;  // ready for the next batch's counts
                c += cg[g];
            }
        }
        const uint32_t k = (c + chunk - 1) / chunk;
        uint32_t tot_c, tot_k;
        const uint32_t ex_c = block_exscan<kScanThreads>(c, tot_c, sh);
        const uint32_t ex_k = block_exscan<kScanThreads>(k, tot_k, sh);
        if (t < ntiles) {
            off[t] = carry_r + ex_c;
            cur[t] = carry_r + ex_c;
            if (a.goff) {
                // where each copy's records start: after the copies before it
                uint32_t o = carry_r + ex_c;
#pragma unroll
                for (uint32_t g = 0; g < kCntGroups; g++)
                    if (g < ng) {
                        a.goff[g * ntiles + t] = o;
                        o += cg[g];
                    }
            }
            for (uint32_t j = 0; j < k; j++) {
                const uint32_t q = carry_i + ex_k + j;
                if (q < items_cap) {
                    items[2 * q] = t;
                    items[2 * q + 1] = j;
                }
            }
        }
        carry_r += tot_c;
        carry_i += tot_k;
    }
    if (threadIdx.x == 0) {
        off[ntiles] = carry_r;
        *a.nitems = min(carry_i, items_cap);
    }
}

// Multi-block tile scan (more than kScanOneBlockTiles tiles, one count
// copy): block b covers tiles [b*kScanChunk, (b+1)*kScanChunk).
// k_tile_sums writes each chunk's record total and work-item total;
// k_tile_offsets adds the totals of the chunks before its own, scans its
// chunk (kScanChunk / kScanThreads consecutive tiles per thread) into bin
// offsets, fill cursors and work items, and zeroes the counts for the next
// batch.  A rejected batch (header error) gets no work items.
constexpr uint32_t kScanChunk = 4096;
constexpr uint32_t kScanPer = kScanChunk / kScanThreads;
static_assert(kScanPer * kScanThreads == kScanChunk, "whole tiles per thread");

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint32_t *__restrict__ cnt,
                                                            uint32_t ntiles, uint32_t chunk,
                                                            uint32_t *__restrict__ sums)
{
    __shared__ uint32_t sh[160];
    const uint32_t t0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    uint32_t c = 0, k = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; j++) {
        const uint32_t t = t0 + j;
        const uint32_t x = t < ntiles ? cnt[t] : 0u;
        c += x;
        k += (x + chunk - 1) / chunk;
    }
    uint32_t tc, tk;
    block_exscan<kScanThreads>(c, tc, sh);
    block_exscan<kScanThreads>(k, tk, sh);
    if (threadIdx.x == 0) {
        sums[2 * blockIdx.x] = tc;
        sums[2 * blockIdx.x + 1] = tk;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_tile_offsets(uint32_t *__restrict__ cnt,
                                                               uint32_t ntiles, ScanArgs a,
                                                               const uint32_t *__restrict__ hdr)
{
    __shared__ uint32_t sh[160];
    const bool err = hdr[HDR_ERR] != 0;
    const uint32_t b = blockIdx.x;
    // totals of the chunks before this one
    uint32_t pc = 0, pk = 0;
    for (uint32_t i = threadIdx.x; i < b; i += kScanThreads) {
        pc += a.sums[2 * i];
        pk += a.sums[2 * i + 1];
    }
    uint32_t carry_r, carry_i;
    block_exscan<kScanThreads>(pc, carry_r, sh);
    block_exscan<kScanThreads>(pk, carry_i, sh);
    const uint32_t t0 = b * kScanChunk + threadIdx.x * kScanPer;
    uint32_t c[kScanPer], k[kScanPer], lc = 0, lk = 0;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; j++) {
        const uint32_t t = t0 + j;
        c[j] = t < ntiles ? cnt[t] : 0u;
        if (t < ntiles) cnt[t] = 0;  // ready for the next batch's counts
        k[j] = err ? 0u : (c[j] + a.chunk - 1) / a.chunk;
        lc += c[j];
        lk += k[j];
    }
    uint32_t tot_c, tot_k;
    const uint32_t ex_c = block_exscan<kScanThreads>(lc, tot_c, sh);
    const uint32_t ex_k = block_exscan<kScanThreads>(lk, tot_k, sh);
    uint32_t o = carry_r + ex_c, q = carry_i + ex_k;
#pragma unroll
    for (uint32_t j = 0; j < kScanPer; j++) {
        const uint32_t t = t0 + j;
        if (t < ntiles) {
            a.off[t] = o;
            a.cur[t] = o;
            for (uint32_t i = 0; i < k[j]; i++, q++)
                if (q < a.items_cap) {
                    a.items[2 * q] = t;
                    a.items[2 * q + 1] = i;
                }
        }
        o += c[j];
    }
    if (b == gridDim.x - 1 && threadIdx.x == 0) {
        a.off[ntiles] = carry_r + tot_c;
        *a.nitems = err ? 0u : min(carry_i + tot_k, a.items_cap);
    }
}

__global__ __launch_bounds__(kClsThreads) void k_classify(
    const BatchDesc *__restrict__ desc, BatchDesc dv, uint32_t V, const uint64_t *__restrict__ lp,
    const uint32_t *__restrict__ blk, uint32_t *__restrict__ hdr, uint64_t *__restrict__ fupd,
    uint32_t *__restrict__ fpos, uint32_t *__restrict__ fcnt, uint32_t *__restrict__ fdel,
    uint32_t *__restrict__ tile_cnt, uint32_t tile_shift, uint32_t ntiles,
    uint32_t *__restrict__ tile_rel)
{
    __shared__ uint32_t hist[kLdsHistMax];
    __shared__ uint32_t pre[64 + 1];  // flagged per (step, wave) -> exclusive prefix; total
    __shared__ uint32_t wdel[kClsWaves];  // flagged deletes per wave
    const bool count = tile_cnt != nullptr;
    const bool use_lds = count && ntiles <= kLdsHistMax;
    if (use_lds)
        for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) hist[t] = 0;

    const uint64_t *__restrict__ upd = desc ? desc->upd : dv.upd;
    const uint32_t n = desc ? desc->n : dv.n;
    const uint32_t begin = blockIdx.x * kClsPerBlock;
    const uint32_t lane = __lane_id();
    const uint32_t wid = threadIdx.x / 64;
    uint64_t p[kClsPerThread];
    uint64_t lu[kClsPerThread], lv[kClsPerThread];  // label | parent << 32
    uint32_t bu[kClsPerThread], bv[kClsPerThread];  // block labels (inserts)
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        const uint32_t i = begin + k * kClsThreads + threadIdx.x;
        p[k] = i < n ? upd[i] : 0;
    }
    // bit k of `ok`: update k exists and is valid.  An insert whose
    // endpoints both lie in blocks of one label each is decided by those
    // labels (a table of V/64 words); the others load both forest words.
    uint32_t ok = 0;
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        const uint32_t i = begin + k * kClsThreads + threadIdx.x;
        uint32_t u, v;
        bool del;
        bu[k] = bv[k] = kBlkMixed;
        if (i < n && unpack(p[k], V, u, v, del)) {
            ok |= 1u << k;
            if (blk && !del) {
                bu[k] = blk[u >> kBlkShift];
                bv[k] = blk[v >> kBlkShift];
            }
        }
    }
    uint32_t gath = 0;  // bit k: update k is decided by its forest words
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        lu[k] = lv[k] = 0;
        if (!((ok >> k) & 1u)) continue;
        if (bu[k] != kBlkMixed && bv[k] != kBlkMixed) continue;
        uint32_t u, v;
        bool del;
        unpack(p[k], V, u, v, del);
        gath |= 1u << k;
        lu[k] = lp[u];
        lv[k] = lp[v];
    }
    bool bad = false;
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        const uint32_t i = begin + k * kClsThreads + threadIdx.x;
        if (i < n && !((ok >> k) & 1u)) bad = true;
    }
    uint32_t fl = 0;  // bit k: update k flagged
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        if (!((ok >> k) & 1u)) continue;
        bool f;
        if (!((gath >> k) & 1u)) {
            f = bu[k] != bv[k];  // an insert between two uniform blocks
        } else {
            uint32_t u, v;
            bool del;
            unpack(p[k], V, u, v, del);
            f = (uint32_t)lu[k] != (uint32_t)lv[k];
            if (!f && del) f = (uint32_t)(lu[k] >> 32) == v || (uint32_t)(lv[k] >> 32) == u;
        }
        if (f) fl |= 1u << k;
    }
    __syncthreads();  // hist zeroed
    if (count) {
        uint32_t *h = use_lds ? hist : tile_cnt;
#pragma unroll
        for (uint32_t k = 0; k < kClsPerThread; k++) {
            if (!((ok >> k) & 1u)) continue;
            uint32_t u, v;
            bool del;
            unpack(p[k], V, u, v, del);
            atomicAdd(&h[u >> tile_shift], 1u);
            atomicAdd(&h[v >> tile_shift], 1u);
        }
    }
    uint32_t ndel = 0;  // flagged deletes of this lane, then of this wave
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        const bool f = (fl >> k) & 1u;
        const uint64_t m = __ballot(f);
        if (lane == 0) pre[k * kClsWaves + wid] = (uint32_t)__popcll(m);
        ndel += (f && (p[k] >> 63)) ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t o = 32; o > 0; o >>= 1) ndel += __shfl_xor(ndel, o);
    if (lane == 0) wdel[wid] = ndel;
    const uint64_t mb = __ballot(bad);
    if (mb && lane == (uint32_t)__builtin_ctzll(mb)) atomicOr(&hdr[HDR_ERR], 1u);
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t x = pre[threadIdx.x];
        uint32_t inc = x;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        pre[threadIdx.x] = inc - x;
        if (threadIdx.x == 63) pre[64] = inc;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kClsPerThread; k++) {
        const bool f = (fl >> k) & 1u;
        const uint64_t m = __ballot(f);
        if (f) {
            const uint32_t q = begin + pre[k * kClsWaves + wid] + lanes_below(m);
            fupd[q] = p[k];
            if (fpos) fpos[q] = begin + k * kClsThreads + threadIdx.x;
        }
    }
    // per-block counts only: the one-block scan after this kernel sums them
    // (device atomics of every block on one header word would serialize)
    const uint32_t total = pre[64];
    if (threadIdx.x == 0) {
        uint32_t dsum = 0;
#pragma unroll
        for (uint32_t w = 0; w < kClsWaves; w++) dsum += wdel[w];
        fcnt[blockIdx.x] = total;
        fdel[blockIdx.x] = dsum;
    }
    if (use_lds) {
        __syncthreads();
        if (tile_rel) {
            // the returned count is where this block's records start among
            // its count copy's records in the tile's bin
            uint32_t *rb = tile_rel + (size_t)blockIdx.x * ntiles;
            uint32_t *tc = tile_cnt + (blockIdx.x % kCntGroups) * ntiles;
            for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
                const uint32_t h = hist[t];
                if (h) rb[t] = atomicAdd(&tc[t], h);
            }
        } else {
            for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x)
                if (hist[t]) atomicAdd(&tile_cnt[t], hist[t]);
        }
    }
}

uint32_t classify_blocks(uint32_t n) { return (n + kClsPerBlock - 1) / kClsPerBlock; }

__global__ void k_pack_forest(const uint32_t *__restrict__ lbl, const uint32_t *__restrict__ par,
                              uint64_t *__restrict__ lp, uint32_t V)
{
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < V; w += gridDim.x * blockDim.x)
        lp[w] = (uint64_t)lbl[w] | (uint64_t)par[w] << 32;
}

// One wave per block of 2^kBlkShift = 64 vertex ids: the label they all
// share, or kBlkMixed.  pages null: every block; else the blocks of the np
// pages (2^pshift ids each) listed there.
__global__ void k_block_labels(const uint32_t *__restrict__ lbl, uint32_t V,
                               uint32_t *__restrict__ blk, const uint32_t *__restrict__ pages,
                               uint32_t np, uint32_t pshift)
{
    const uint32_t nblk = (V + 63) >> kBlkShift;
    const uint32_t per = pages ? 1u << (pshift - kBlkShift) : 0u;  // blocks per page
    const uint32_t nw = pages ? np * per : nblk;
    const uint32_t lane = __lane_id();
    for (uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / 64; w < nw;
         w += gridDim.x * blockDim.x / 64) {
        const uint32_t b = pages ? (pages[w / per] << (pshift - kBlkShift)) + w % per : w;
        if (b >= nblk) continue;  // (wave-uniform) past the last vertex
        const uint32_t x = (b << kBlkShift) + lane;
        const uint32_t l = x < V ? lbl[x] : 0u;
        const uint32_t first = __shfl(l, 0);
        const uint64_t differ = __ballot(x < V && l != first);
        if (lane == 0) blk[b] = differ ? kBlkMixed : first;
    }
}

hipError_t launch_block_labels(hipStream_t s, const uint32_t *lbl, uint32_t V, uint32_t *blk,
                               const uint32_t *pages, uint32_t np, uint32_t pshift)
{
    if (V == 0 || (pages && np == 0)) return hipSuccess;
    if (pages && (pshift < kBlkShift || pshift > 16)) return hipErrorInvalidValue;
    const uint32_t nw = pages ? np << (pshift - kBlkShift) : (V + 63) >> kBlkShift;
    const uint32_t grid = min((nw + 3) / 4, 8192u);
    k_block_labels<<<grid, 256, 0, s>>>(lbl, V, blk, pages, np, pshift);
    return hipGetLastError();
}

hipError_t launch_pack_forest(hipStream_t s, const uint32_t *lbl, const uint32_t *par, uint64_t *lp,
                              uint32_t V)
{
    if (V == 0) return hipSuccess;
    const uint32_t grid = min((V + 255) / 256, 8192u);
    k_pack_forest<<<grid, 256, 0, s>>>(lbl, par, lp, V);
    return hipGetLastError();
}

// Page i of the staging block (id stage[i], then 2^pshift labels of each
// page in turn, then 2^pshift parents of each page in turn) into lbl, par
// and lp.
__global__ void k_forest_pages(const uint32_t *__restrict__ stage, uint32_t np, uint32_t pshift,
                               uint32_t V, uint32_t *__restrict__ lbl, uint32_t *__restrict__ par,
                               uint64_t *__restrict__ lp)
{
    const uint32_t i = blockIdx.x;
    const uint32_t pv = 1u << pshift;
    const uint32_t base = stage[i] << pshift;
    const uint32_t *sl = stage + np + (size_t)i * pv;
    const uint32_t *sp = stage + np + (size_t)np * pv + (size_t)i * pv;
    for (uint32_t j = threadIdx.x; j < pv && base + j < V; j += blockDim.x) {
        const uint32_t w = base + j, l = sl[j], q = sp[j];
        lbl[w] = l;
        par[w] = q;
        lp[w] = (uint64_t)l | (uint64_t)q << 32;
    }
}

hipError_t launch_forest_pages(hipStream_t s, const uint32_t *stage, uint32_t np, uint32_t pshift,
                               uint32_t V, uint32_t *lbl, uint32_t *par, uint64_t *lp)
{
    if (np == 0) return hipSuccess;
    if (pshift > 16 || ((size_t)(V - 1) >> pshift) >= (1u << 31)) return hipErrorInvalidValue;
    k_forest_pages<<<np, 256, 0, s>>>(stage, np, pshift, V, lbl, par, lp);
    return hipGetLastError();
}

hipError_t launch_classify(hipStream_t s, const BatchDesc *desc, BatchDesc dv, uint32_t grid_n,
                           uint32_t V, const uint64_t *lp, const uint32_t *blk, uint32_t *hdr,
                           uint64_t *fupd, uint32_t *fpos, uint32_t *fcnt, uint32_t *tile_cnt,
                           uint32_t tile_shift, uint32_t ntiles, const ScanArgs &sa,
                           uint32_t *hout, const FlagInline &fi, uint32_t *tile_rel)
{
    if (!fi.fdel || fi.fcnt != fcnt || fi.nb != classify_blocks(grid_n)) return hipErrorInvalidValue;
    if (grid_n == 0) return hipSuccess;
    if (tile_rel && (!tile_cnt || ntiles > kRelMaxTiles || sa.groups != kCntGroups || !sa.goff))
        return hipErrorInvalidValue;
    if (!tile_rel && tile_cnt && sa.groups != 1) return hipErrorInvalidValue;
    if (sa.sums && (tile_rel || sa.groups != 1 || ntiles <= kScanOneBlockTiles))
        return hipErrorInvalidValue;
    k_classify<<<classify_blocks(grid_n), kClsThreads, 0, s>>>(
        desc, dv, V, lp, blk, hdr, fupd, fpos, fcnt, fi.fdel, tile_cnt, tile_shift, ntiles,
        tile_rel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // (nothing to do for the one-block scan when it only scans tiles and
    // the multi-block kernels do that, or there are no tile counts)
    if (!fi.tiles_only || (tile_cnt && sa.off && !sa.sums)) {
        k_tile_scan<<<1, kScanThreads, 0, s>>>(tile_cnt, ntiles, sa, hdr, hout, fi);
        e = hipGetLastError();
    }
    if (e != hipSuccess || !tile_cnt || !sa.sums) return e;
    const uint32_t nch = tile_scan_chunks(ntiles);
    k_tile_sums<<<nch, kScanThreads, 0, s>>>(tile_cnt, ntiles, sa.chunk, sa.sums);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tile_offsets<<<nch, kScanThreads, 0, s>>>(tile_cnt, ntiles, sa, hdr);
    return hipGetLastError();
}

uint32_t tile_scan_chunks(uint32_t ntiles) { return (ntiles + kScanChunk - 1) / kScanChunk; }

// Last block of a scatter kernel to finish: clear the header for the next
// batch.  Every block used its read of ERR before taking its ticket, so the
// ticket needs no fence (a device-scope fence would write back L2).
DEVI void scatter_done(uint32_t *hdr)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        if (__hip_atomic_fetch_add(&hdr[HDR_SCAT_DONE], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
            hdr[HDR_ERR] = 0;
            hdr[HDR_NFLAG] = 0;
            hdr[HDR_NFLAG_DEL] = 0;
            hdr[HDR_SCAT_DONE] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// Plain scatter: one thread per update, hashing the edge index once per
// column and XOR-ing (x, h) into bucket (c, d) of both endpoints with
// device-scope atomics (4 per column).  Skipped when the batch was rejected.
// ---------------------------------------------------------------------------
// All C columns of one update into both endpoints, with device atomics.
DEVI void scatter_one(const DevSketch &sk, uint64_t p)
{
    uint32_t u, v;
    bool del;
    unpack(p, sk.V, u, v, del);
    const uint64_t x = (uint64_t)u * sk.V + v;
    const uint64_t ru = (uint64_t)u * sk.D, rv = (uint64_t)v * sk.D;
    for (uint32_t c = 0; c < sk.C; c++) {
        const uint64_t h = mix64(x ^ sk.seeds[c]);
        const uint32_t d = depth_of(h, sk.D);
        uint64_t *bu = sk.b + ((ru + d) * sk.C + c) * 2;
        uint64_t *bv = sk.b + ((rv + d) * sk.C + c) * 2;
        gxor(bu, x);
        gxor(bu + 1, h);
        gxor(bv, x);
        gxor(bv + 1, h);
    }
}

__global__ __launch_bounds__(256) void k_scatter_atomic(const BatchDesc *__restrict__ desc,
                                                        BatchDesc dv, DevSketch sk,
                                                        uint32_t *__restrict__ hdr)
{
    const bool err = hdr[HDR_ERR] != 0;
    const uint32_t n = desc ? desc->n : dv.n;
    const uint64_t *upd = desc ? desc->upd : dv.upd;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (!err && i < n) scatter_one(sk, upd[i]);
    scatter_done(hdr);
}

// ---------------------------------------------------------------------------
// Small batches (n <= kSmallMax): one block classifies the whole batch and
// writes the header and the flagged updates (with positions) straight into
// a result block in coherent pinned host memory, then publishes the next
// sequence number; a second kernel scatters with device atomics.  The batch
// comes in the arguments, so no descriptor copy, header clearing,
// compaction, binning, copy or event is needed: the latency of a small
// batch is two launches.
// ---------------------------------------------------------------------------
constexpr uint32_t kSmallThreads = 1024;
constexpr uint32_t kSmallPerThread = kSmallMax / kSmallThreads;
static_assert(kSmallPerThread * (kSmallThreads / 64) == 64, "one wave scans the step counts");

__global__ __launch_bounds__(kSmallThreads) void k_small_classify(
    const uint64_t *__restrict__ upd, uint32_t n, uint32_t V, const uint32_t *__restrict__ lbl,
    const uint32_t *__restrict__ par, SmallResult *__restrict__ out, uint32_t *__restrict__ derr,
    uint32_t *__restrict__ seqp, uint32_t with_pos)
{
    __shared__ uint32_t pre[64 + 1];
    __shared__ uint32_t s_bad, s_del;
    const uint32_t lane = __lane_id();
    const uint32_t wid = threadIdx.x / 64;
    constexpr uint32_t kWaves = kSmallThreads / 64;
    if (threadIdx.x == 0) {
        s_bad = 0;
        s_del = 0;
    }
    uint64_t p[kSmallPerThread];
    uint32_t fl = 0, bad = 0, ndel = 0;
#pragma unroll
    for (uint32_t k = 0; k < kSmallPerThread; k++) {
        const uint32_t i = k * kSmallThreads + threadIdx.x;
        p[k] = i < n ? upd[i] : 0;
    }
#pragma unroll
    for (uint32_t k = 0; k < kSmallPerThread; k++) {
        const uint32_t i = k * kSmallThreads + threadIdx.x;
        if (i >= n) continue;
        uint32_t u, v;
        bool del;
        if (!unpack(p[k], V, u, v, del)) {
            bad = 1;
            continue;
        }
        bool f = lbl[u] != lbl[v];
        if (!f && del) f = par[u] == v || par[v] == u;
        if (f) {
            fl |= 1u << k;
            ndel += del ? 1u : 0u;
        }
    }
    __syncthreads();  // s_bad, s_del cleared
    if (bad) atomicOr(&s_bad, 1u);
    if (ndel) atomicAdd(&s_del, ndel);
#pragma unroll
    for (uint32_t k = 0; k < kSmallPerThread; k++) {
        const uint64_t m = __ballot((fl >> k) & 1u);
        if (lane == 0) pre[k * kWaves + wid] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t x = pre[threadIdx.x];
        uint32_t inc = x;
#pragma unroll
        for (uint32_t o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        pre[threadIdx.x] = inc - x;
        if (threadIdx.x == 63) pre[64] = inc;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kSmallPerThread; k++) {
        const bool f = (fl >> k) & 1u;
        const uint64_t m = __ballot(f);
        if (f) {
            const uint32_t q = pre[k * kWaves + wid] + lanes_below(m);
            out->fupd[q] = p[k];
            if (with_pos) out->fpos[q] = k * kSmallThreads + threadIdx.x;
        }
    }
    // the result is in host memory before the sequence number says so:
    // every wave waits until its stores have been acknowledged, and thread
    // 0's system-scope release below writes back L2 once for the block
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        *derr = s_bad;  // for the scatter
        out->hdr[HDR_ERR] = s_bad;
        out->hdr[HDR_NFLAG] = s_bad ? 0u : pre[64];
        out->hdr[HDR_NFLAG_DEL] = s_bad ? 0u : s_del;
        const uint32_t seq = *seqp + 1;
        *seqp = seq;
        __hip_atomic_store(&out->hdr[HDR_SEQ], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ __launch_bounds__(256) void k_small_scatter(const uint64_t *__restrict__ upd,
                                                       uint32_t n, DevSketch sk,
                                                       const uint32_t *__restrict__ derr)
{
    if (*derr) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    scatter_one(sk, upd[i]);
}

hipError_t launch_small_classify(hipStream_t s, const uint64_t *upd, uint32_t n, uint32_t V,
                                 const uint32_t *lbl, const uint32_t *par, SmallResult *out,
                                 uint32_t *derr, uint32_t *seqp, bool with_pos)
{
    if (n == 0 || n > kSmallMax) return hipErrorInvalidValue;
    k_small_classify<<<1, kSmallThreads, 0, s>>>(upd, n, V, lbl, par, out, derr, seqp,
                                                with_pos ? 1u : 0u);
    return hipGetLastError();
}

hipError_t launch_small_scatter(hipStream_t s, const uint64_t *upd, uint32_t n, DevSketch sk,
                                const uint32_t *derr)
{
    if (n == 0 || n > kSmallMax) return hipErrorInvalidValue;
    k_small_scatter<<<(n + 255) / 256, 256, 0, s>>>(upd, n, sk, derr);
    return hipGetLastError();
}

hipError_t launch_scatter_atomic(hipStream_t s, const BatchDesc *desc, BatchDesc dv,
                                 uint32_t grid_n, DevSketch sk, uint32_t *hdr)
{
    if (grid_n == 0) return hipSuccess;
    k_scatter_atomic<<<(grid_n + 255) / 256, 256, 0, s>>>(desc, dv, sk, hdr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Staged scatter.
//
// 1. tile scan (the last block of k_classify, once all counts are in):
//    exclusive scan of the per-tile record counts into bin offsets, and a
//    list of work items (tile, chunk) where a chunk is at most `chunk`
//    records of one tile's bin.
// 2. k_tile_fill: each update writes one record per endpoint into the bin
//    of that endpoint's tile: u | v << 32, with bit 63 set (kRecV) in the
//    record of v.  Slots are reserved per block in LDS first, so global
//    atomics are per (block, tile), not per record.
// 3. k_tile_scatter: one work item per block iteration.  The block keeps a
//    zeroed LDS delta of depth rows 0..rows-1 for the tile's vertices,
//    decodes the chunk's records into LDS, XORs every (record, column)
//    pair into the delta (LDS atomics, one lane per pair; depths >= rows
//    go straight to HBM with device atomics), then folds the nonzero delta
//    words into HBM: a plain read-XOR-write when the chunk is the tile's
//    whole bin (no other block touches these vertices), a device atomic XOR
//    otherwise.  LDS holds alpha and gamma in separate planes ordered
//    [d][vertex][c], so the C lanes of one record hit consecutive words.
// ---------------------------------------------------------------------------
constexpr uint64_t kRecV = 1ull << 63;  // the record is for endpoint v

constexpr uint32_t kFillThreads = 1024;
constexpr uint32_t kFillPerBlock = 4096;
constexpr uint32_t kFillPerThread = kFillPerBlock / kFillThreads;

__global__ __launch_bounds__(kFillThreads) void k_tile_fill(
    const BatchDesc *__restrict__ desc, BatchDesc dv, uint32_t V, uint32_t tile_shift,
    uint32_t ntiles, uint32_t *__restrict__ cur, uint64_t *__restrict__ bins,
    const uint32_t *__restrict__ hdr)
{
    __shared__ uint32_t lcnt[kLdsHistMax];
    if (hdr[HDR_ERR]) return;
    const uint64_t *__restrict__ upd = desc ? desc->upd : dv.upd;
    const uint32_t n = desc ? desc->n : dv.n;
    const uint32_t begin = blockIdx.x * kFillPerBlock;
    if (begin >= n) return;
    // all of this thread's updates are loaded once, up front
    uint64_t p[kFillPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        const uint32_t i = begin + k * kFillThreads + threadIdx.x;
        p[k] = i < n ? upd[i] : 0;
    }
    if (ntiles > kLdsHistMax) {
        // Many small tiles: contention is low, reserve per record.
#pragma unroll
        for (uint32_t k = 0; k < kFillPerThread; k++) {
            if (begin + k * kFillThreads + threadIdx.x >= n) continue;
            uint32_t u, v;
            bool del;
            unpack(p[k], V, u, v, del);
            const uint64_t rec = (uint64_t)u | ((uint64_t)v << 32);
            bins[atomicAdd(&cur[u >> tile_shift], 1u)] = rec;
            bins[atomicAdd(&cur[v >> tile_shift], 1u)] = rec | kRecV;
        }
        return;
    }
    for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) lcnt[t] = 0;
    __syncthreads();
    // ranks of each record inside its tile's share of this block
    uint32_t ru[kFillPerThread], rv[kFillPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        ru[k] = rv[k] = 0;
        if (begin + k * kFillThreads + threadIdx.x >= n) continue;
        uint32_t u, v;
        bool del;
        unpack(p[k], V, u, v, del);
        ru[k] = atomicAdd(&lcnt[u >> tile_shift], 1u);
        rv[k] = atomicAdd(&lcnt[v >> tile_shift], 1u);
    }
    __syncthreads();
    // reserve one contiguous range per tile present in this block
    for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
        const uint32_t c = lcnt[t];
        if (c) lcnt[t] = atomicAdd(&cur[t], c);
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        if (begin + k * kFillThreads + threadIdx.x >= n) continue;
        uint32_t u, v;
        bool del;
        unpack(p[k], V, u, v, del);
        const uint64_t rec = (uint64_t)u | ((uint64_t)v << 32);
        bins[lcnt[u >> tile_shift] + ru[k]] = rec;
        bins[lcnt[v >> tile_shift] + rv[k]] = rec | kRecV;
    }
}

// Fill for up to kFillStageTiles tiles: the block's 2*kFillPerBlock records
// are first counting-sorted by tile in LDS, then written out in that order,
// so that the lanes of a wave store one (block, tile) run after another into
// consecutive bin words (coalesced) instead of 8-byte words scattered over
// all tiles.  Dynamic LDS: fill_stage_lds(ntiles) bytes.
static_assert(kFillStageTiles == 2 * kFillThreads, "two tiles per fill thread");
static size_t fill_stage_lds(uint32_t ntiles)
{
    return (size_t)2 * kFillPerBlock * 8 + (size_t)2 * ntiles * 4 + 160 * 4;
}

__global__ __launch_bounds__(kFillThreads) void k_tile_fill_staged(
    const BatchDesc *__restrict__ desc, BatchDesc dv, uint32_t V, uint32_t tile_shift,
    uint32_t ntiles, uint32_t *__restrict__ cur, uint64_t *__restrict__ bins,
    const uint32_t *__restrict__ hdr, const uint32_t *__restrict__ goff,
    const uint32_t *__restrict__ rel)
{
    extern __shared__ uint64_t fsm[];
    uint64_t *stage = fsm;                                   // records in tile order
    uint32_t *lcnt = (uint32_t *)(fsm + 2 * kFillPerBlock);  // per tile: count, then bin base
    uint32_t *lpre = lcnt + ntiles;                          // per tile: first stage slot
    uint32_t *sh = lpre + ntiles;                            // scan scratch (160 words)
    if (hdr[HDR_ERR]) return;
    const uint64_t *__restrict__ upd = desc ? desc->upd : dv.upd;
    const uint32_t n = desc ? desc->n : dv.n;
    const uint32_t begin = blockIdx.x * kFillPerBlock;
    if (begin >= n) return;
    uint64_t p[kFillPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        const uint32_t i = begin + k * kFillThreads + threadIdx.x;
        p[k] = i < n ? upd[i] : 0;
    }
    for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) lcnt[t] = 0;
    __syncthreads();
    // ranks of each record inside its tile's share of this block
    uint32_t ru[kFillPerThread], rv[kFillPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        ru[k] = rv[k] = 0;
        if (begin + k * kFillThreads + threadIdx.x >= n) continue;
        uint32_t u, v;
        bool del;
        unpack(p[k], V, u, v, del);
        ru[k] = atomicAdd(&lcnt[u >> tile_shift], 1u);
        rv[k] = atomicAdd(&lcnt[v >> tile_shift], 1u);
    }
    __syncthreads();
    // first stage slot of each tile (two tiles per thread), and one
    // contiguous bin range per tile present in this block
    const uint32_t t0 = 2 * threadIdx.x;
    const uint32_t c0 = t0 < ntiles ? lcnt[t0] : 0u;
    const uint32_t c1 = t0 + 1 < ntiles ? lcnt[t0 + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exscan<kFillThreads>(c0 + c1, tot, sh);
    // with `rel`, the classify block of the same updates has already taken
    // this block's place in every tile, among the records of its count copy
    const uint32_t *rb = rel ? rel + (size_t)blockIdx.x * ntiles : nullptr;
    const uint32_t *go = rel ? goff + (blockIdx.x % kCntGroups) * ntiles : nullptr;
    if (t0 < ntiles) {
        lpre[t0] = ex;
        lcnt[t0] = c0 ? (rb ? go[t0] + rb[t0] : atomicAdd(&cur[t0], c0)) : 0u;
    }
    if (t0 + 1 < ntiles) {
        lpre[t0 + 1] = ex + c0;
        lcnt[t0 + 1] = c1 ? (rb ? go[t0 + 1] + rb[t0 + 1] : atomicAdd(&cur[t0 + 1], c1)) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kFillPerThread; k++) {
        if (begin + k * kFillThreads + threadIdx.x >= n) continue;
        uint32_t u, v;
        bool del;
        unpack(p[k], V, u, v, del);
        const uint64_t rec = (uint64_t)u | ((uint64_t)v << 32);
        stage[lpre[u >> tile_shift] + ru[k]] = rec;
        stage[lpre[v >> tile_shift] + rv[k]] = rec | kRecV;
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < tot; j += blockDim.x) {
        const uint64_t rec = stage[j];
        const uint32_t e = (rec & kRecV) ? (uint32_t)(rec >> 32) & 0x7fffffffu : (uint32_t)rec;
        const uint32_t t = e >> tile_shift;
        bins[lcnt[t] + (j - lpre[t])] = rec;
    }
}

// ---------------------------------------------------------------------------
// Two-level binning, for more tiles than one block's LDS histogram serves.
// The classify kernel counts records per coarse bin (2^fshift consecutive
// tiles) and the fill bins them by coarse bin into `bins1` (k_tile_fill_staged
// on coarse bins).  Then every chunk of kFinePerBlock coarse-binned records
// spans few tiles: k_fine_count counts the chunk's records per tile in LDS
// and adds the counts to the tile counts (one global atomic per (chunk,
// tile)), the multi-block tile scan turns them into bin offsets and work
// items, and k_fine_fill ranks each chunk's records per tile in LDS,
// reserves one range per (chunk, tile) from the tile's cursor and writes
// the records there, staged in tile order in LDS so that each (chunk, tile)
// run is written as consecutive words.  A tile more than kFineLdsTiles
// (count) or kFillLdsTiles (fill) past the chunk's first coarse bin is
// counted and reserved per record instead.
// ---------------------------------------------------------------------------
constexpr uint32_t kFineThreads = 1024;
constexpr uint32_t kFinePer = 8;
constexpr uint32_t kFinePerBlock = kFineThreads * kFinePer;

DEVI uint32_t rec_endpoint(uint64_t rec)
{
    return (rec & kRecV) ? (uint32_t)(rec >> 32) & 0x7fffffffu : (uint32_t)rec;
}

__global__ __launch_bounds__(kFineThreads) void k_fine_count(
    const uint64_t *__restrict__ bins1, const uint32_t *__restrict__ total, uint32_t tile_shift,
    uint32_t fshift, uint32_t *__restrict__ cnt, const uint32_t *__restrict__ hdr)
{
    __shared__ uint32_t hist[kFineLdsTiles];
    if (hdr[HDR_ERR]) return;
    const uint32_t n = *total;
    const uint32_t begin = blockIdx.x * kFinePerBlock;
    if (begin >= n) return;
    const uint32_t t_lo = (rec_endpoint(bins1[begin]) >> (tile_shift + fshift)) << fshift;
    for (uint32_t j = threadIdx.x; j < kFineLdsTiles; j += kFineThreads) hist[j] = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kFinePer; k++) {
        const uint32_t i = begin + k * kFineThreads + threadIdx.x;
        if (i >= n) continue;
        const uint32_t t = rec_endpoint(bins1[i]) >> tile_shift;
        if (t - t_lo < kFineLdsTiles)
            atomicAdd(&hist[t - t_lo], 1u);
        else
            atomicAdd(&cnt[t], 1u);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < kFineLdsTiles; j += kFineThreads) {
        const uint32_t c = hist[j];
        if (c) atomicAdd(&cnt[t_lo + j], c);
    }
}

// The fill takes half as many records per block as the count, so that its
// LDS (the block's records staged in tile order, and per tile the count,
// stage start and reserved bin start) stays within 64 KiB.
constexpr uint32_t kFillPer2 = 4;
constexpr uint32_t kFillPerBlock2 = kFineThreads * kFillPer2;
constexpr uint32_t kFillLdsTiles = 2 * kFineThreads;

__global__ __launch_bounds__(kFineThreads) void k_fine_fill(
    const uint64_t *__restrict__ bins1, const uint32_t *__restrict__ total, uint32_t tile_shift,
    uint32_t fshift, uint32_t *__restrict__ cur, uint64_t *__restrict__ bins,
    const uint32_t *__restrict__ hdr)
{
    __shared__ uint64_t stage[kFillPerBlock2];  // local records in tile order
    __shared__ uint32_t lcnt[kFillLdsTiles];    // per tile: count, then reserved bin start
    __shared__ uint32_t lpre[kFillLdsTiles];    // per tile: first stage slot
    __shared__ uint32_t sh[160];
    if (hdr[HDR_ERR]) return;
    const uint32_t n = *total;
    const uint32_t begin = blockIdx.x * kFillPerBlock2;
    if (begin >= n) return;
    const uint32_t t_lo = (rec_endpoint(bins1[begin]) >> (tile_shift + fshift)) << fshift;
    for (uint32_t j = threadIdx.x; j < kFillLdsTiles; j += kFineThreads) lcnt[j] = 0;
    __syncthreads();
    uint64_t rec[kFillPer2];
    uint32_t rk[kFillPer2];  // rank in the block's share of its tile, or the final position
#pragma unroll
    for (uint32_t k = 0; k < kFillPer2; k++) {
        const uint32_t i = begin + k * kFineThreads + threadIdx.x;
        rec[k] = i < n ? bins1[i] : 0;
        rk[k] = 0;
        if (i >= n) continue;
        const uint32_t t = rec_endpoint(rec[k]) >> tile_shift;
        rk[k] = t - t_lo < kFillLdsTiles ? atomicAdd(&lcnt[t - t_lo], 1u) : atomicAdd(&cur[t], 1u);
    }
    __syncthreads();
    // stage starts (a block scan, two tiles per thread) and one reserved bin
    // range per tile present in this block
    const uint32_t t0 = 2 * threadIdx.x;
    const uint32_t c0 = lcnt[t0], c1 = lcnt[t0 + 1];
    uint32_t tot;
    const uint32_t ex = block_exscan<kFineThreads>(c0 + c1, tot, sh);
    lpre[t0] = ex;
    lpre[t0 + 1] = ex + c0;
    lcnt[t0] = c0 ? atomicAdd(&cur[t_lo + t0], c0) : 0u;
    lcnt[t0 + 1] = c1 ? atomicAdd(&cur[t_lo + t0 + 1], c1) : 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kFillPer2; k++) {
        const uint32_t i = begin + k * kFineThreads + threadIdx.x;
        if (i >= n) continue;
        const uint32_t t = rec_endpoint(rec[k]) >> tile_shift;
        if (t - t_lo < kFillLdsTiles)
            stage[lpre[t - t_lo] + rk[k]] = rec[k];
        else
            bins[rk[k]] = rec[k];
    }
    __syncthreads();
    // out in tile order: the lanes of a wave store runs of consecutive words
    for (uint32_t j = threadIdx.x; j < tot; j += kFineThreads) {
        const uint64_t r = stage[j];
        const uint32_t t = (rec_endpoint(r) >> tile_shift) - t_lo;
        bins[lcnt[t] + (j - lpre[t])] = r;
    }
}

hipError_t launch_fine(hipStream_t s, uint32_t grid_n, const uint32_t *hdr, const uint64_t *bins1,
                       const uint32_t *total, uint32_t tile_shift, uint32_t fshift,
                       uint32_t ntiles, uint32_t *tile_cnt, const ScanArgs &sa, uint64_t *bins)
{
    if (grid_n == 0) return hipSuccess;
    if (!sa.sums || sa.groups != 1 || fshift == 0 || (1u << fshift) > kFineLdsTiles)
        return hipErrorInvalidValue;
    const uint32_t nb = (uint32_t)((2 * (uint64_t)grid_n + kFinePerBlock - 1) / kFinePerBlock);
    k_fine_count<<<nb, kFineThreads, 0, s>>>(bins1, total, tile_shift, fshift, tile_cnt, hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t nch = tile_scan_chunks(ntiles);
    k_tile_sums<<<nch, kScanThreads, 0, s>>>(tile_cnt, ntiles, sa.chunk, sa.sums);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_tile_offsets<<<nch, kScanThreads, 0, s>>>(tile_cnt, ntiles, sa, hdr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t nf = (uint32_t)((2 * (uint64_t)grid_n + kFillPerBlock2 - 1) / kFillPerBlock2);
    k_fine_fill<<<nf, kFineThreads, 0, s>>>(bins1, total, tile_shift, fshift, sa.cur, bins, hdr);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Record layout of the staged scatter (StagedParams.layout == kLayoutRecord):
// one lane per record, looping over the C columns (unrolled at compile time
// for C <= CMAX, seeds in scalar registers), so each lane hashes its record
// C times as independent chains.  LDS planes ordered [d][c][vertex]: the
// lanes of a wave hit the same column of up to 64 records of one tile, so
// many records per vertex mean LDS address conflicts; with few records per
// tile and batch this layout still wins on its instruction-level
// parallelism.  Everything else is as in the pair layout below.
// ---------------------------------------------------------------------------
constexpr uint32_t kRecThreads = 256;

// XOR one (record, column) pair into the endpoint's LDS delta, or into HBM
// for depths beyond the rows held in LDS.  lq = c*TV + (local vertex index),
// CTV = C*TV (words per LDS depth row); gb = the endpoint's first bucket in
// HBM; y = mix64_head(x), seed1 = mix64_head(column seed).  Index products
// use the full-rate 24-bit multiply (d < 64 and C*TV, C < 2^24).
DEVI void rec_column(uint64_t *la, uint64_t *lg, uint64_t *gb, uint32_t C, uint32_t D,
                     uint32_t CTV, uint32_t rows, uint32_t rfast, uint32_t stop, uint32_t c,
                     uint64_t seed1, uint64_t x, uint64_t y, uint32_t lq, uint32_t &deep)
{
    const uint64_t h = mix64_tail(y ^ seed1);
    uint32_t d = (uint32_t)__builtin_ctz((uint32_t)h | stop);
    if (d == rfast) {
        d = depth_of(h, D);
        if (d >= rows) {
            uint64_t *bp = gb + 2 * (__umul24(d & 63u, C & 0xffffffu) + c);
            gxor(bp, x);
            gxor(bp + 1, h);
            deep++;
            return;
        }
    }
    const uint32_t q = __umul24(d & 63u, CTV) + lq;
    lxor(&la[q], x);
    lxor(&lg[q], h);
}

template <uint32_t CMAX>
__global__ __launch_bounds__(kRecThreads) void k_tile_scatter_rec(
    DevSketch sk, const uint64_t *__restrict__ bins, const uint32_t *__restrict__ off,
    const uint32_t *__restrict__ items, const uint32_t *__restrict__ nitems_p, uint32_t tile_shift,
    uint32_t rows, uint32_t chunk, uint32_t *__restrict__ hdr,
    unsigned long long *__restrict__ touched)
{
    uint32_t nchanged = 0;  // buckets this thread changed in HBM
    extern __shared__ uint64_t lds[];
    const bool err = hdr[HDR_ERR] != 0;
    const uint32_t TV = 1u << tile_shift;
    const uint32_t C = sk.C, D = sk.D, V = sk.V;
    const uint32_t plane = rows * C * TV;  // words per LDS plane
    const uint32_t CTV = (C * TV) & 0xffffffu;  // words per LDS depth row
    const uint64_t DC2 = (uint64_t)D * C * 2;   // words per vertex in HBM
    const uint32_t rfast = min(min(rows, D - 1), 31u);
    const uint32_t stop = 1u << rfast;
    uint64_t *la = lds;          // alpha plane [d][c][vl]
    uint64_t *lg = lds + plane;  // gamma plane
    const uint32_t nitems = err ? 0u : *nitems_p;
    uint64_t seed1[CMAX > 0 ? CMAX : 1];
    if (CMAX > 0) {
#pragma unroll
        for (uint32_t c = 0; c < CMAX; c++) seed1[c] = c < C ? mix64_head(sk.seeds[c]) : 0;
    }

    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t tile = items[2 * it];
        const uint32_t j = items[2 * it + 1];
        const uint32_t rb = off[tile], re = off[tile + 1];
        const uint32_t cb = rb + j * chunk;
        const uint32_t ce = min(re, cb + chunk);
        const bool single = (re - rb) <= chunk;
        const uint32_t w0 = tile << tile_shift;

        for (uint32_t q = threadIdx.x; q < 2 * plane; q += blockDim.x) lds[q] = 0;
        __syncthreads();

        for (uint32_t r = cb + threadIdx.x; r < ce; r += blockDim.x) {
            const uint64_t rec = bins[r];
            const uint32_t u = (uint32_t)rec, v = (uint32_t)(rec >> 32) & 0x7fffffffu;
            const uint64_t x = (uint64_t)u * V + v;
            const uint64_t y = mix64_head(x);
            const uint32_t p = (rec & kRecV) ? v : u;  // the record's endpoint in this tile
            uint64_t *gb = sk.b + (uint64_t)p * DC2;
            if (CMAX > 0) {
#pragma unroll
                for (uint32_t c = 0; c < (CMAX > 0 ? CMAX : 1); c++)
                    if (c < C)
                        rec_column(la, lg, gb, C, D, CTV, rows, rfast, stop, c, seed1[c], x, y,
                                   c * TV + (p - w0), nchanged);
            } else {
                for (uint32_t c = 0; c < C; c++)
                    rec_column(la, lg, gb, C, D, CTV, rows, rfast, stop, c,
                               mix64_head(sk.seeds[c]), x, y, c * TV + (p - w0), nchanged);
            }
        }
        __syncthreads();

        // Fold the delta into HBM, walking buckets in HBM order
        // (vertex, d, c) so that consecutive lanes touch consecutive words.
        const uint32_t nvt = min(TV, V - w0);
        const uint32_t per_v = rows * C;
        const uint32_t nb = nvt * per_v;
        for (uint32_t q = threadIdx.x; q < nb; q += blockDim.x) {
            const uint32_t vl = q / per_v;
            const uint32_t rc = q - vl * per_v;  // d*C + c
            const uint64_t da = la[rc * TV + vl];
            const uint64_t dg = lg[rc * TV + vl];
            if ((da | dg) == 0) continue;
            nchanged++;
            uint64_t *g = sk.b + (((uint64_t)(w0 + vl) * D) * C + rc) * 2;
            if (single) {
                g[0] ^= da;
                g[1] ^= dg;
            } else {
                if (da) gxor(g, da);
                if (dg) gxor(g + 1, dg);
            }
        }
        __syncthreads();
    }
    if (touched) {
        uint32_t t = nchanged;
#pragma unroll
        for (uint32_t o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (__lane_id() == 0 && t) atomicAdd(touched, (unsigned long long)t);
    }
    scatter_done(hdr);
}

constexpr uint32_t kTileThreads = 512;
constexpr uint32_t kTileWaves = kTileThreads / 64;
constexpr uint32_t kTileLdsMax = 65536;  // dynamic LDS per block, bytes
constexpr uint32_t kTileStage = 512;     // records staged per pass

// The staged records (24 B each: edge index and the first step of its
// hash, byte offset of the endpoint's words in an LDS depth row, local
// vertex) must fit beside the LDS delta.
constexpr uint32_t kStagedRecBytes = 24;
static bool tile_stage_fits(size_t delta_bytes)
{
    return delta_bytes + (size_t)kTileStage * kStagedRecBytes <= kTileLdsMax;
}

bool tile_geometry_fits(uint32_t rows, uint32_t C, uint32_t tv, uint32_t layout)
{
    const size_t delta = (size_t)2 * rows * C * tv * sizeof(uint64_t);
    if (C < 1 || C > 64 || rows < 1) return false;
    return layout == kLayoutRecord ? delta <= kTileLdsMax : tile_stage_fits(delta);
}

struct StagedRec {
    uint64_t x;   // edge index u*V + v of the record's update
    uint64_t y;   // mix64_head(x)
    uint32_t qb;  // vl*C*8: byte offset of the endpoint's words in a depth row
    uint32_t vl;  // endpoint - first vertex of the tile
};

// XOR one (record, column) pair into the LDS delta (or HBM for a deep row).
// colb = column * 8; RSB = bytes per LDS depth row; pg = gamma plane offset
// in bytes; seed1 = mix64_head(column seed).  The depth is ctz of the hash's low word with a stop bit at
// rfast = min(rows, D-1, 31); only when no bit below rfast is set (odds
// 2^-rfast) is the full depth taken, and a depth >= rows goes to HBM with
// device atomics.
DEVI void tile_pair(uint8_t *lds8, uint32_t RSB, uint32_t pg, uint32_t rows, uint32_t rfast,
                    uint32_t stop, uint32_t colb, uint64_t seed1, const StagedRec &r,
                    const DevSketch &sk, uint32_t w0, uint64_t DC2, uint32_t &nchanged)
{
    const uint64_t h = mix64_tail(r.y ^ seed1);
    const uint32_t d0 = (uint32_t)__builtin_ctz((uint32_t)h | stop);  // <= 31
    if (d0 != rfast) {
        const uint32_t a = __umul24(d0, RSB) + r.qb + colb;
        lxor((uint64_t *)(lds8 + a), r.x);
        lxor((uint64_t *)(lds8 + a + pg), h);
        return;
    }
    const uint32_t d = depth_of(h, sk.D);
    if (d < rows) {
        // (d < 64 and RSB < 2^24: the masks let the compiler use the
        // 24-bit multiply)
        const uint32_t a = __umul24(d & 63u, RSB & 0xffffffu) + r.qb + colb;
        lxor((uint64_t *)(lds8 + a), r.x);
        lxor((uint64_t *)(lds8 + a + pg), h);
    } else {
        uint64_t *bp = sk.b + (uint64_t)(w0 + r.vl) * DC2 + 2 * (uint64_t)d * sk.C + colb / 4;
        gxor(bp, r.x);
        gxor(bp + 1, h);
        nchanged++;
    }
}

// One (record, column) pair per lane: the edge index x = u*V + v of the
// record's update is hashed for column c and (x, h) is XOR-ed into bucket
// (d, c) of the record's endpoint.  Lane l of a wave takes column l mod C of
// record l / C (G = 64 / C records per wave step, lanes l >= G*C idle), so
// the C lanes of a record hit C consecutive LDS words and the hash seed is a
// per-lane constant.
//
// LDS: the delta's alpha and gamma planes, word d*TV*C + vl*C + c for depth
// row d < rows, local vertex vl, column c; then the staged records.
//
// touched (may be null) receives the number of buckets the launch changes
// in HBM: folded buckets with a nonzero delta, plus one per pair that goes
// to a deep row directly.
__global__ __launch_bounds__(kTileThreads) void k_tile_scatter(
    DevSketch sk, const uint64_t *__restrict__ bins, const uint32_t *__restrict__ off,
    const uint32_t *__restrict__ items, const uint32_t *__restrict__ nitems_p, uint32_t tile_shift,
    uint32_t rows, uint32_t chunk, uint32_t *__restrict__ hdr,
    unsigned long long *__restrict__ touched)
{
    uint32_t nchanged = 0;  // buckets this thread changed in HBM
    extern __shared__ uint64_t lds[];
    uint8_t *lds8 = (uint8_t *)lds;
    const bool err = hdr[HDR_ERR] != 0;
    const uint32_t TV = 1u << tile_shift;
    const uint32_t C = sk.C, V = sk.V;
    const uint32_t RS = TV * C;             // words per LDS depth row (< 2^12)
    const uint32_t plane = rows * RS;       // words per LDS plane
    const uint64_t DC2 = (uint64_t)sk.D * C * 2;  // words per vertex in HBM
    const uint32_t rfast = min(min(rows, sk.D - 1), 31u);
    const uint32_t stop = 1u << rfast;
    const uint64_t *la = lds;               // alpha plane
    const uint64_t *lg = lds + plane;       // gamma plane
    StagedRec *st = (StagedRec *)(lds + 2 * plane);
    const uint32_t nitems = err ? 0u : *nitems_p;

    const uint32_t lane = __lane_id(), wid = threadIdx.x / 64;
    const uint32_t G = 64 / C;              // records (or rows) per wave step
    const uint32_t WG = kTileWaves * G;     // records per block step
    const uint32_t slot = lane / C;
    const uint32_t col = lane - slot * C;
    const bool active = slot < G;
    const uint32_t colb = col * 8;
    const uint64_t seed1 = active ? mix64_head(sk.seeds[col]) : 0;

    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t tile = items[2 * it];
        const uint32_t j = items[2 * it + 1];
        const uint32_t rb = off[tile], re = off[tile + 1];
        const uint32_t cb = rb + j * chunk;
        const uint32_t ce = min(re, cb + chunk);
        const bool single = (re - rb) <= chunk;
        const uint32_t w0 = tile << tile_shift;
        if (cb >= ce) continue;  // (block-uniform) nothing to fold

        for (uint32_t q = threadIdx.x; q < 2 * plane; q += kTileThreads) lds[q] = 0;

        for (uint32_t sb = cb; sb < ce; sb += kTileStage) {
            const uint32_t ns = min(kTileStage, ce - sb);
            // stage: decode each record once
            for (uint32_t i = threadIdx.x; i < ns; i += kTileThreads) {
                const uint64_t rec = bins[sb + i];
                const uint32_t u = (uint32_t)rec, v = (uint32_t)(rec >> 32) & 0x7fffffffu;
                const uint32_t vl = ((rec & kRecV) ? v : u) - w0;
                StagedRec r;
                r.x = (uint64_t)u * V + v;
                r.y = mix64_head(r.x);
                r.qb = __umul24(vl, C) * 8;
                r.vl = vl;
                st[i] = r;
            }
            __syncthreads();
            if (active) {
                // full block steps need no bound check; the last one does
                const uint32_t full = ns / WG * WG;
                uint32_t i = wid * G + slot;
                for (; i + WG < full; i += 2 * WG) {
                    const StagedRec r0 = st[i], r1 = st[i + WG];
                    tile_pair(lds8, RS * 8, plane * 8, rows, rfast, stop, colb, seed1, r0, sk,
                              w0, DC2, nchanged);
                    tile_pair(lds8, RS * 8, plane * 8, rows, rfast, stop, colb, seed1, r1, sk,
                              w0, DC2, nchanged);
                }
                if (i < full) {
                    tile_pair(lds8, RS * 8, plane * 8, rows, rfast, stop, colb, seed1, st[i], sk,
                              w0, DC2, nchanged);
                    i += WG;
                }
                if (i < ns)
                    tile_pair(lds8, RS * 8, plane * 8, rows, rfast, stop, colb, seed1, st[i], sk,
                              w0, DC2, nchanged);
            }
            __syncthreads();
        }

        // Fold the delta into HBM: lanes (slot, column) of a wave take G
        // vertices at a time and walk their depth rows, so each step reads
        // C consecutive words per row in LDS and C consecutive buckets
        // (16 B each) per row in HBM.
        if (active) {
            const uint32_t nvt = min(TV, V - w0);
            for (uint32_t vl = wid * G + slot; vl < nvt; vl += WG) {
                uint32_t q = __umul24(vl, C) + col;
                uint64_t *g = sk.b + (uint64_t)(w0 + vl) * DC2 + 2 * col;
                for (uint32_t d = 0; d < rows; d++, q += RS, g += 2 * C) {
                    const uint64_t da = la[q], dg = lg[q];
                    if ((da | dg) == 0) continue;
                    nchanged++;
                    if (single) {
                        ulonglong2 *g2 = (ulonglong2 *)g;
                        ulonglong2 b = *g2;
                        b.x ^= da;
                        b.y ^= dg;
                        *g2 = b;
                    } else {
                        if (da) gxor(g, da);
                        if (dg) gxor(g + 1, dg);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (touched) {
        uint32_t t = nchanged;
#pragma unroll
        for (uint32_t o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (__lane_id() == 0 && t) atomicAdd(touched, (unsigned long long)t);
    }
    scatter_done(hdr);
}

hipError_t launch_bin(hipStream_t s, const BatchDesc *desc, BatchDesc dv, uint32_t grid_n,
                      DevSketch sk, const uint32_t *hdr, const StagedParams &p,
                      uint32_t *tile_cur, uint64_t *bins, const uint32_t *tile_goff,
                      const uint32_t *tile_rel)
{
    if (grid_n == 0) return hipSuccess;
    const uint32_t fb = (grid_n + kFillPerBlock - 1) / kFillPerBlock;
    // the fill's blocks cover the same updates as the classify blocks
    static_assert(kFillPerBlock == kClsPerBlock,
                  "fill and classify blocks must cover the same updates");
    static_assert(kRelMaxTiles <= kFillStageTiles && kRelMaxTiles <= kLdsHistMax,
                  "tile_rel needs the classify's LDS counts and the staged fill");
    if (tile_rel && (p.ntiles > kRelMaxTiles || !tile_goff)) return hipErrorInvalidValue;
    if (p.ntiles <= kFillStageTiles)
        k_tile_fill_staged<<<fb, kFillThreads, fill_stage_lds(p.ntiles), s>>>(
            desc, dv, sk.V, p.tile_shift, p.ntiles, tile_cur, bins, hdr, tile_goff, tile_rel);
    else
        k_tile_fill<<<fb, kFillThreads, 0, s>>>(desc, dv, sk.V, p.tile_shift, p.ntiles, tile_cur,
                                                bins, hdr);
    return hipGetLastError();
}

hipError_t launch_tile(hipStream_t s, DevSketch sk, uint32_t *hdr, const StagedParams &p,
                       const uint32_t *tile_off, const uint64_t *bins, const uint32_t *items,
                       const uint32_t *nitems, unsigned long long *touched)
{
    const size_t delta = (size_t)2 * p.rows * sk.C * (1u << p.tile_shift) * sizeof(uint64_t);
    if (!tile_geometry_fits(p.rows, sk.C, 1u << p.tile_shift, p.layout))
        return hipErrorInvalidValue;
    // Persistent grid: a few blocks per CU, each looping over work items.
    const uint32_t grid = min(p.items_cap, p.grid ? p.grid : 256u * 8u);
    if (p.layout == kLayoutRecord) {
#define CUPK_REC_LAUNCH(CM)                                                                    \
    k_tile_scatter_rec<CM><<<grid, kRecThreads, delta, s>>>(sk, bins, tile_off, items, nitems, \
                                                            p.tile_shift, p.rows, p.chunk, hdr, \
                                                            touched)
        if (sk.C <= 8) CUPK_REC_LAUNCH(8);
        else if (sk.C <= 16) CUPK_REC_LAUNCH(16);
        else if (sk.C <= 24) CUPK_REC_LAUNCH(24);
        else if (sk.C <= 32) CUPK_REC_LAUNCH(32);
        else CUPK_REC_LAUNCH(0);
#undef CUPK_REC_LAUNCH
        return hipGetLastError();
    }
    const size_t lds = delta + (size_t)kTileStage * kStagedRecBytes;
    k_tile_scatter<<<grid, kTileThreads, lds, s>>>(sk, bins, tile_off, items, nitems, p.tile_shift,
                                                   p.rows, p.chunk, hdr, touched);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Flag compaction: exclusive scan of the per-block flag counts (one block),
// then every classify block's region is copied to its offset, giving the
// flagged updates of the batch in stream order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanThreads) void k_flag_scan(const uint32_t *__restrict__ fcnt,
                                                            uint32_t nb,
                                                            uint32_t *__restrict__ foff)
{
    __shared__ uint32_t sh[160];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += kScanThreads) {
        const uint32_t b = base + threadIdx.x;
        const uint32_t c = b < nb ? fcnt[b] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exscan<kScanThreads>(c, tot, sh);
        if (b < nb) foff[b] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void k_flag_compact(const uint64_t *__restrict__ fupd,
                                                      const uint32_t *__restrict__ fpos,
                                                      const uint32_t *__restrict__ fcnt,
                                                      const uint32_t *__restrict__ foff,
                                                      uint64_t *__restrict__ oupd,
                                                      uint32_t *__restrict__ opos)
{
    const uint32_t b = blockIdx.x;
    const uint32_t c = fcnt[b], o = foff[b];
    const uint32_t src = b * kClsPerBlock;
    for (uint32_t k = threadIdx.x; k < c; k += blockDim.x) {
        oupd[o + k] = fupd[src + k];
        if (opos) opos[o + k] = fpos[src + k];
    }
}

hipError_t launch_flag_compact(hipStream_t s, uint32_t n, const uint64_t *fupd,
                               const uint32_t *fpos, const uint32_t *fcnt, uint32_t *foff,
                               uint64_t *oupd, uint32_t *opos)
{
    const uint32_t nb = classify_blocks(n);
    if (nb == 0) return hipSuccess;
    k_flag_scan<<<1, kScanThreads, 0, s>>>(fcnt, nb, foff);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_flag_compact<<<nb, 256, 0, s>>>(fupd, fpos, fcnt, foff, oupd, opos);
    return hipGetLastError();
}

// Flag check against a newer forest, one wave per classify block's region:
// each step reads 64 flagged updates, keeps those the classify rule still
// flags against `lp`, and writes them back packed at the front of the
// region (a step writes below the next step's reads: in place is safe).
constexpr uint32_t kReflagThreads = 256;

__global__ __launch_bounds__(kReflagThreads) void k_reflag(uint32_t V, const uint64_t *__restrict__ lp,
                                                           const uint32_t *__restrict__ hdr,
                                                           uint64_t *__restrict__ fupd,
                                                           uint32_t *__restrict__ fcnt,
                                                           uint32_t *__restrict__ fdel, uint32_t nb)
{
    const uint32_t b = blockIdx.x * (kReflagThreads / 64) + threadIdx.x / 64;
    if (b >= nb || hdr[HDR_ERR] != 0) return;  // whole waves
    const uint32_t lane = __lane_id();
    const uint32_t c = fcnt[b];
    uint64_t *r = fupd + (size_t)b * kClsPerBlock;
    uint32_t w = 0, nd = 0;
    for (uint32_t k0 = 0; k0 < c; k0 += 64) {
        const uint32_t k = k0 + lane;
        bool keep = false, del = false;
        uint64_t p = 0;
        if (k < c) {
            p = r[k];
            uint32_t u, v;
            unpack(p, V, u, v, del);
            const uint64_t lu = lp[u], lv = lp[v];
            keep = (uint32_t)lu != (uint32_t)lv;
            if (!keep && del) keep = (uint32_t)(lu >> 32) == v || (uint32_t)(lv >> 32) == u;
        }
        const uint64_t m = __ballot(keep);
        if (keep) r[w + lanes_below(m)] = p;
        w += (uint32_t)__popcll(m);
        nd += (uint32_t)__popcll(__ballot(keep && del));
    }
    if (lane == 0) {
        fcnt[b] = w;
        fdel[b] = nd;
    }
}

hipError_t launch_reflag(hipStream_t s, uint32_t V, const uint64_t *lp, uint32_t *hdr,
                         uint64_t *fupd, uint32_t *hout, const FlagInline &fi, uint32_t *foff,
                         uint64_t *oupd, bool check)
{
    if (!fi.fdel || !fi.fcnt || fi.fupd != fupd || fi.tiles_only || !foff || !oupd)
        return hipErrorInvalidValue;
    if (fi.nb) {
        hipError_t e = hipSuccess;
        if (check) {
            const uint32_t per = kReflagThreads / 64;
            k_reflag<<<(fi.nb + per - 1) / per, kReflagThreads, 0, s>>>(
                V, lp, hdr, fupd, const_cast<uint32_t *>(fi.fcnt), fi.fdel, fi.nb);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        // the ordered list, before the header: the host only copies it
        k_flag_scan<<<1, kScanThreads, 0, s>>>(fi.fcnt, fi.nb, foff);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        k_flag_compact<<<fi.nb, 256, 0, s>>>(fupd, nullptr, fi.fcnt, foff, oupd, nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // header only: no tile counts
    k_tile_scan<<<1, kScanThreads, 0, s>>>(nullptr, 0, ScanArgs{}, hdr, hout, fi);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Utility fills.
// ---------------------------------------------------------------------------
__global__ void k_zero64(uint64_t *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero32(uint32_t *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero(hipStream_t s, uint64_t *p, size_t n)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_zero64<<<(uint32_t)blocks, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_zero32(hipStream_t s, uint32_t *p, size_t n)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_zero32<<<(uint32_t)blocks, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Segmented XOR reduction (component sketches).  A work item is
// (set, begin, end) over the member list; the block streams the members'
// slabs (W words each, coalesced across lanes) and XORs them into
// registers, then folds the nonzero words into out[set] with device
// atomics (a set may span several work items).
// ---------------------------------------------------------------------------
constexpr uint32_t kRedThreads = 256;

// KMAX words per lane: slabs of up to KMAX*256 words (C*D*2 <= KMAX*256).
template <uint32_t KMAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const uint64_t *__restrict__ src,
                                                        uint32_t W,
                                                        const uint32_t *__restrict__ idx,
                                                        const uint32_t *__restrict__ items,
                                                        uint32_t nitems,
                                                        uint64_t *__restrict__ out)
{
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const uint32_t set = items[3 * it];
        const uint32_t b = items[3 * it + 1];
        const uint32_t e = items[3 * it + 2];
        uint64_t acc[KMAX];
#pragma unroll
        for (uint32_t k = 0; k < KMAX; k++) acc[k] = 0;
        uint32_t j = b;
        // two slabs per step: twice the loads in flight
        for (; j + 2 <= e; j += 2) {
            const uint64_t *s0 = src + (uint64_t)idx[j] * W;
            const uint64_t *s1 = src + (uint64_t)idx[j + 1] * W;
#pragma unroll
            for (uint32_t k = 0; k < KMAX; k++) {
                const uint32_t w = k * kRedThreads + threadIdx.x;
                if (w < W) acc[k] ^= s0[w] ^ s1[w];
            }
        }
        if (j < e) {
            const uint64_t *s0 = src + (uint64_t)idx[j] * W;
#pragma unroll
            for (uint32_t k = 0; k < KMAX; k++) {
                const uint32_t w = k * kRedThreads + threadIdx.x;
                if (w < W) acc[k] ^= s0[w];
            }
        }
        uint64_t *o = out + (uint64_t)set * W;
#pragma unroll
        for (uint32_t k = 0; k < KMAX; k++) {
            const uint32_t w = k * kRedThreads + threadIdx.x;
            if (w < W && acc[k]) gxor(&o[w], acc[k]);
        }
    }
}

hipError_t launch_reduce(hipStream_t s, const uint64_t *src, uint32_t W, const uint32_t *idx,
                         const uint32_t *items, uint32_t nitems, uint64_t *out)
{
    if (nitems == 0) return hipSuccess;
    const uint32_t grid = min(nitems, 8192u);
    if (W <= 4 * kRedThreads)
        k_reduce<4><<<grid, kRedThreads, 0, s>>>(src, W, idx, items, nitems, out);
    else if (W <= 8 * kRedThreads)
        k_reduce<8><<<grid, kRedThreads, 0, s>>>(src, W, idx, items, nitems, out);
    else if (W <= 16 * kRedThreads)
        k_reduce<16><<<grid, kRedThreads, 0, s>>>(src, W, idx, items, nitems, out);
    else if (W <= 32 * kRedThreads)
        k_reduce<32><<<grid, kRedThreads, 0, s>>>(src, W, idx, items, nitems, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Reduction over CSR sets for the allocation-free entry point: a block takes
// members [16q, 16q + 16) of the concatenated member list, finds the set of
// the first one by binary search over the offsets (sets may be empty), and
// walks forward, folding its accumulator into a set's aggregate whenever it
// leaves that set.
constexpr uint32_t kCsrChunk = 16;

template <uint32_t KMAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce_csr(const uint64_t *__restrict__ src,
                                                            uint32_t W,
                                                            const uint32_t *__restrict__ mem,
                                                            const uint64_t *__restrict__ offs,
                                                            uint32_t k, uint32_t nv,
                                                            uint64_t *__restrict__ out)
{
    const uint32_t nchunks = (nv + kCsrChunk - 1) / kCsrChunk;
    for (uint32_t q = blockIdx.x; q < nchunks; q += gridDim.x) {
        const uint32_t b = q * kCsrChunk, e = min(nv, b + kCsrChunk);
        // the last set j with offs[j] <= b; offs[0] = 0 <= b < nv = offs[k]
        uint32_t lo = 0, hi = k;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) / 2;
            if (offs[mid] <= b) lo = mid;
            else hi = mid;
        }
        uint32_t j = lo;
        uint64_t end = offs[j + 1];
        uint64_t acc[KMAX];
#pragma unroll
        for (uint32_t t = 0; t < KMAX; t++) acc[t] = 0;
        for (uint32_t m = b; m < e; m++) {
            if (m >= end) {
                uint64_t *o = out + (uint64_t)j * W;
#pragma unroll
                for (uint32_t t = 0; t < KMAX; t++) {
                    const uint32_t w = t * kRedThreads + threadIdx.x;
                    if (w < W && acc[t]) gxor(&o[w], acc[t]);
                    acc[t] = 0;
                }
                do {
                    j++;
                    end = offs[j + 1];
                } while (m >= end);
            }
            const uint64_t *s0 = src + (uint64_t)mem[m] * W;
#pragma unroll
            for (uint32_t t = 0; t < KMAX; t++) {
                const uint32_t w = t * kRedThreads + threadIdx.x;
                if (w < W) acc[t] ^= s0[w];
            }
        }
        uint64_t *o = out + (uint64_t)j * W;
#pragma unroll
        for (uint32_t t = 0; t < KMAX; t++) {
            const uint32_t w = t * kRedThreads + threadIdx.x;
            if (w < W && acc[t]) gxor(&o[w], acc[t]);
        }
    }
}

hipError_t launch_reduce_csr(hipStream_t s, const uint64_t *src, uint32_t W,
                             const uint32_t *mem, const uint64_t *offs, uint32_t k,
                             uint32_t nv, uint64_t *out)
{
    if (k == 0 || nv == 0) return hipSuccess;
    const uint32_t grid = min((nv + kCsrChunk - 1) / kCsrChunk, 8192u);
    if (W <= 4 * kRedThreads)
        k_reduce_csr<4><<<grid, kRedThreads, 0, s>>>(src, W, mem, offs, k, nv, out);
    else if (W <= 8 * kRedThreads)
        k_reduce_csr<8><<<grid, kRedThreads, 0, s>>>(src, W, mem, offs, k, nv, out);
    else if (W <= 16 * kRedThreads)
        k_reduce_csr<16><<<grid, kRedThreads, 0, s>>>(src, W, mem, offs, k, nv, out);
    else if (W <= 32 * kRedThreads)
        k_reduce_csr<32><<<grid, kRedThreads, 0, s>>>(src, W, mem, offs, k, nv, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Scratch of the allocation-free entry point: one array per GPU, held until
// the process ends.  In host code its name is a host-side stand-in, not a
// device address: host code uses only the address hipGetSymbolAddress
// returns for the current device, kept per device below.
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchWords];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static uint64_t *g_scratch_addr[kMaxDevices];

hipError_t noalloc_scratch_address(int device, uint64_t **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        uint64_t *p = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Verify and sample.  One block per aggregate sketch: every lane checks its
// buckets (alpha != 0, checksum and depth re-derived from alpha, alpha
// decodes to u < v < V) and the block takes the minimum canonical rank
// c*D + (D-1-d) among the good ones; a block-wide OR detects the all-zero
// (EMPTY) case.
// ---------------------------------------------------------------------------
constexpr uint32_t kSmpThreads = 256;

__global__ __launch_bounds__(kSmpThreads) void k_sample(const uint64_t *__restrict__ sig,
                                                        uint32_t k, uint32_t V, uint32_t C,
                                                        uint32_t D, uint32_t sc, uint32_t sd,
                                                        uint64_t set_stride,
                                                        const uint64_t *__restrict__ seeds,
                                                        int32_t *__restrict__ res)
{
    __shared__ uint32_t s_best[kSmpThreads / 64];
    __shared__ uint64_t s_any[kSmpThreads / 64];
    const uint32_t set = blockIdx.x;
    if (set >= k) return;
    const uint64_t *S = sig + (uint64_t)set * set_stride;
    uint32_t best = 0xffffffffu;
    uint64_t any = 0;
    const uint32_t nb = C * D;
    for (uint32_t q = threadIdx.x; q < nb; q += blockDim.x) {
        const uint32_t c = q / D, d = q - c * D;
        const uint64_t o = ((uint64_t)c * sc + (uint64_t)d * sd) * 2;
        const uint64_t a = S[o], g = S[o + 1];
        any |= a | g;
        if (a == 0) continue;
        const uint64_t h = mix64(a ^ seeds[c]);
        if (h != g || depth_of(h, D) != d) continue;
        const uint64_t uu = a / V, vv = a - uu * V;
        if (!(uu < vv)) continue;
        const uint32_t key = c * D + (D - 1 - d);
        best = key < best ? key : best;
    }
    // wave reductions
    for (uint32_t o = 32; o > 0; o >>= 1) {
        const uint32_t ob = __shfl_xor(best, o);
        best = ob < best ? ob : best;
        any |= __shfl_xor(any, o);
    }
    const uint32_t wid = threadIdx.x / 64;
    if (__lane_id() == 0) {
        s_best[wid] = best;
        s_any[wid] = any;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / 64; w++) {
            best = s_best[w] < best ? s_best[w] : best;
            any |= s_any[w];
        }
        int32_t *r = res + 3 * (uint64_t)set;
        if (best != 0xffffffffu) {
            const uint32_t c = best / D, d = D - 1 - (best - c * D);
            const uint64_t a = S[((uint64_t)c * sc + (uint64_t)d * sd) * 2];
            r[0] = 0;
            r[1] = (int32_t)(uint32_t)(a / V);
            r[2] = (int32_t)(uint32_t)(a % V);
        } else {
            r[0] = any ? 2 : 1;
            r[1] = 0;
            r[2] = 0;
        }
    }
}

hipError_t launch_sample(hipStream_t s, const uint64_t *sig, uint32_t k, uint32_t V, uint32_t C,
                         uint32_t D, uint32_t sc, uint32_t sd, uint64_t set_stride,
                         const uint64_t *seeds, int32_t *res)
{
    if (k == 0) return hipSuccess;
    k_sample<<<k, kSmpThreads, 0, s>>>(sig, k, V, C, D, sc, sd, set_stride, seeds, res);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One-column aggregates for the multi-level hierarchy: set k is reduced over
// column col[k] only (level col[k]'s sampler).  A wave takes one work item
// (set, members [b, e)) at a time; lane l < 2D holds word l of the
// aggregate (depth l/2, alpha or gamma), read from each member's slab with a
// stride of one bucket row; the result is XORed into out[k*2D + l].
// ---------------------------------------------------------------------------
constexpr uint32_t kColThreads = 256;

__global__ __launch_bounds__(kColThreads) void k_reduce_col(
    const uint64_t *__restrict__ sk, uint32_t C, uint32_t D, const uint32_t *__restrict__ idx,
    const uint32_t *__restrict__ items, uint32_t nitems, const uint32_t *__restrict__ col,
    uint64_t *__restrict__ out)
{
    const uint32_t lane = __lane_id();
    const uint32_t waves = kColThreads / 64;
    const uint32_t W2 = 2 * D;
    for (uint32_t it = blockIdx.x * waves + threadIdx.x / 64; it < nitems;
         it += gridDim.x * waves) {
        const uint32_t set = items[3 * it], b = items[3 * it + 1], e = items[3 * it + 2];
        const uint32_t c = col[set];
        for (uint32_t l = lane; l < W2; l += 64) {
            const uint32_t d = l >> 1;
            uint64_t acc = 0;
            for (uint32_t m = b; m < e; m++) {
                const uint64_t w = idx[m];
                acc ^= sk[((w * D + d) * C + c) * 2 + (l & 1)];
            }
            if (acc) gxor(out + (uint64_t)set * W2 + l, acc);
        }
    }
}

hipError_t launch_reduce_col(hipStream_t s, const uint64_t *sk, uint32_t C, uint32_t D,
                             const uint32_t *idx, const uint32_t *items, uint32_t nitems,
                             const uint32_t *col, uint64_t *out)
{
    if (nitems == 0) return hipSuccess;
    const uint32_t waves = kColThreads / 64;
    const uint32_t grid = min((nitems + waves - 1) / waves, 8192u);
    k_reduce_col<<<grid, kColThreads, 0, s>>>(sk, C, D, idx, items, nitems, col, out);
    return hipGetLastError();
}

// Query of one column: a wave per set; lane d checks bucket d of the
// set's one-column aggregate; the deepest good bucket wins (depths are
// scanned from D-1 down).
__global__ __launch_bounds__(kColThreads) void k_sample_col(
    const uint64_t *__restrict__ agg, uint32_t k, uint32_t V, uint32_t D,
    const uint32_t *__restrict__ col, const uint64_t *__restrict__ seeds, int32_t *__restrict__ res)
{
    const uint32_t lane = __lane_id();
    const uint32_t set = blockIdx.x * (kColThreads / 64) + threadIdx.x / 64;
    if (set >= k) return;
    const uint64_t *A = agg + (uint64_t)set * 2 * D;
    const uint64_t seed = seeds[col[set]];
    uint64_t a = 0, g = 0;
    bool good = false;
    if (lane < D) {
        a = A[2 * lane];
        g = A[2 * lane + 1];
        if (a != 0) {
            const uint64_t h = mix64(a ^ seed);
            const uint64_t uu = a / V, vv = a - uu * V;
            good = h == g && depth_of(h, D) == lane && uu < vv;
        }
    }
    const uint64_t mg = __ballot(good);
    const uint64_t mz = __ballot((a | g) != 0);
    const uint32_t top = mg ? 63u - (uint32_t)__builtin_clzll(mg) : 0u;
    const uint64_t pick = __shfl(a, (int)top);
    if (lane == 0) {
        int32_t *r = res + 3 * (uint64_t)set;
        if (mg) {
            r[0] = 0;
            r[1] = (int32_t)(uint32_t)(pick / V);
            r[2] = (int32_t)(uint32_t)(pick % V);
        } else {
            r[0] = mz ? 2 : 1;
            r[1] = 0;
            r[2] = 0;
        }
    }
}

hipError_t launch_sample_col(hipStream_t s, const uint64_t *agg, uint32_t k, uint32_t V,
                             uint32_t D, const uint32_t *col, const uint64_t *seeds,
                             int32_t *res)
{
    if (k == 0) return hipSuccess;
    const uint32_t waves = kColThreads / 64;
    k_sample_col<<<(k + waves - 1) / waves, kColThreads, 0, s>>>(agg, k, V, D, col, seeds, res);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Digest: order-independent sum over all buckets of
// mix(alpha ^ rotl(gamma, 32) ^ mix(canonical_position ^ seed)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_digest(DevSketch sk, uint64_t S, uint64_t *out)
{
    const uint32_t C = sk.C, D = sk.D;
    const uint32_t per_v = C * D;
    uint64_t acc = 0;
    for (uint32_t w = blockIdx.x; w < sk.V; w += gridDim.x) {
        const uint64_t *b = sk.b + (uint64_t)w * per_v * 2;
        for (uint32_t r = threadIdx.x; r < per_v; r += blockDim.x) {
            const uint32_t d = r / C, c = r - d * C;
            const uint64_t pos = ((uint64_t)w * C + c) * D + d;
            const uint64_t a = b[2 * r], g = b[2 * r + 1];
            const uint64_t rg = (g << 32) | (g >> 32);
            acc += mix64(a ^ rg ^ mix64(pos ^ S));
        }
    }
    for (uint32_t o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (__lane_id() == 0) atomicAdd((unsigned long long *)out, (unsigned long long)acc);
}

hipError_t launch_digest(hipStream_t s, DevSketch sk, uint64_t master_seed, uint64_t *out)
{
    const uint32_t grid = min(sk.V, 8192u);
    k_digest<<<grid, 256, 0, s>>>(sk, master_seed, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Internal layout -> canonical (c, d) order.
// ---------------------------------------------------------------------------
__global__ void k_to_canonical(const uint64_t *__restrict__ src, uint32_t C, uint32_t D,
                               uint64_t nv, uint64_t *__restrict__ dst)
{
    const uint32_t per_v = C * D;
    const uint64_t total = nv * per_v;
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < total;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t i = q / per_v;
        const uint32_t r = (uint32_t)(q - i * per_v);
        const uint32_t c = r / D, d = r - c * D;
        const uint64_t s = (i * per_v + (uint64_t)d * C + c) * 2;
        dst[2 * q] = src[s];
        dst[2 * q + 1] = src[s + 1];
    }
}

hipError_t launch_to_canonical(hipStream_t s, const uint64_t *src, uint32_t C, uint32_t D,
                               uint64_t nv, uint64_t *dst)
{
    const uint64_t total = nv * C * D;
    if (total == 0) return hipSuccess;
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_to_canonical<<<(uint32_t)blocks, 256, 0, s>>>(src, C, D, nv, dst);
    return hipGetLastError();
}

}  // namespace cupk
