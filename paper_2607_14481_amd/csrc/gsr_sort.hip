// gsr_sort.hip -- binning stages of the rasterizer on gfx950:
//   A2 scans: visible-item compaction and per-item pair offsets (exclusive
//      scans in u32 with saturating adds, reduce-then-scan, no spin waits)
//   A3 emission: (tile, item) pairs, written in ascending item order
//   A4 radix sort: LSD passes of up to 8 bits over (tile u32, item u32)
//   A4c per-tile depth order: each tile's list sorted by (depth bits, item)
//   A5 tile ranges: [start, end) of each tile in the sorted pairs
//
// Order of work.  The pairs must end up sorted by (tile, depth bits, item).
// Rather than sorting 48-bit (tile, depth) keys over all M pairs (six 8-bit
// passes over the pairs), the pairs are emitted in ascending item order, an
// LSD sort on the tile id alone (ceil(tile_bits / 8) passes, two at 1080p)
// groups them by tile, and one workgroup per tile sorts its short list by
// (depth bits, item) in LDS.  The result is the (tile, depth, item) order
// exactly, whatever order a tile's list had before; so the first radix pass
// need not keep equal digits in input order (only the later ones must).
//
// Every kernel reads its element count from the workspace header, so the
// launch grid can be sized for a capacity and the call needs no host
// synchronisation (graph capture).
#include "gsr_internal.h"

namespace gsr {

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;
    return s < a ? 0xffffffffu : s;
}

// Block-wide exclusive scan of one value per thread (256 threads), saturating.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *lds /* [4] */, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive_scan(x, sat_add);
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before = sat_add(before, lds[k]);
    total = sat_add(sat_add(lds[0], lds[1]), sat_add(lds[2], lds[3]));
    __syncthreads();
    return sat_add(before, inc - x);
}

// ---------------------------------------------------------------------------
// Generic reduce-then-scan.  Phase 1: per-block sums of a per-element value.
// Phase 2: one block scans the block sums.  Phase 3: per-block scan + offset,
// handing each element its exclusive prefix to an epilogue.
// ---------------------------------------------------------------------------
template <class F>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(F f, const uint32_t *__restrict__ n_dev, uint64_t n_host,
                                                              uint32_t *__restrict__ block_sums) {
    __shared__ uint32_t lds[4];
    const uint64_t n = n_dev ? (uint64_t)*n_dev : n_host;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t acc = 0;
    if (base < n) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const uint64_t i = base + (uint64_t)threadIdx.x * kScanItems + k;
            if (i < n) acc = sat_add(acc, f(i));
        }
    }
    uint32_t total;
    block_exclusive_scan(acc, lds, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of nb block sums in place; total -> *out_total.
// With `cap_hdr` set the total is the pair count and the overflow decision
// (total > capacity) is taken here too.
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *__restrict__ block_sums, uint32_t nb,
                                                      uint32_t *__restrict__ out_total, WsHeader *cap_hdr) {
    __shared__ uint32_t lds[16];
    __shared__ uint32_t carry;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nb ? block_sums[i] : 0u;
        const uint32_t inc = wave_inclusive_scan(x, sat_add);
        if (lane == 63) lds[w] = inc;
        __syncthreads();
        uint32_t before = carry;
        for (int k = 0; k < w; ++k) before = sat_add(before, lds[k]);
        if (i < nb) block_sums[i] = sat_add(before, inc - x);
        __syncthreads();
        if (threadIdx.x == 1023) carry = sat_add(before, inc);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out_total = carry;
        if (cap_hdr) cap_hdr->overflow = carry > cap_hdr->pair_capacity ? 1u : 0u;
    }
}

// Ordered compaction of byte flags: out_idx receives, in ascending order, the
// indices i < n with flags[i] != 0; their number goes to *out_count.
struct ByteFlag {
    const uint8_t *f;
    __device__ uint32_t operator()(uint64_t i) const { return f[i] ? 1u : 0u; }
};

__global__ __launch_bounds__(kScanThreads) void k_flag_compact_apply(const uint8_t *__restrict__ flags, uint64_t n,
                                                                     const uint32_t *__restrict__ block_sums,
                                                                     uint32_t *__restrict__ out_idx) {
    __shared__ uint32_t lds[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t bits = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const bool on = base + k < n && flags[base + k] != 0;
        bits |= (on ? 1u : 0u) << k;
        cnt += on;
    }
    uint32_t total;
    uint32_t pos = block_sums[blockIdx.x] + block_exclusive_scan(cnt, lds, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (bits & (1u << k)) out_idx[pos++] = (uint32_t)(base + k);
}

void launch_compact_flags(const uint8_t *flags, uint64_t n, uint32_t *out_idx, uint32_t *block_tmp,
                          uint32_t *out_count, hipStream_t st) {
    const uint32_t nb = (uint32_t)((n + kScanTile - 1) / kScanTile);
    if (nb == 0) return;
    hipLaunchKernelGGL(k_scan_reduce<ByteFlag>, dim3(nb), dim3(kScanThreads), 0, st, ByteFlag{flags},
                       (const uint32_t *)nullptr, n, block_tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, st, block_tmp, nb, out_count, (WsHeader *)nullptr);
    hipLaunchKernelGGL(k_flag_compact_apply, dim3(nb), dim3(kScanThreads), 0, st, flags, n, block_tmp, out_idx);
}

// ---------------------------------------------------------------------------
// A2 in one reduce-then-scan over the items, with two values per item: visible
// (tiles touched > 0) and its tile count.  An invisible item counts zero tiles,
// so the pair offset of the k-th visible item is the prefix of the counts over
// all items before it.  Phase 1 sums each block of kScanTile items; phase 2
// gives each block the sums of the blocks before it (each block adds them up
// itself: at most a few thousand L2-resident values, no extra launch) and
// writes the k-th visible item's id, pair offset and box word and, for each
// chunk of kChunkPairs pair slots whose first pair the item holds, k.  The
// last block writes the visible and pair counts and the overflow decision
// (pairs > capacity).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kScanThreads) void k_vis_reduce(const uint32_t *__restrict__ count, uint64_t n,
                                                             uint32_t *__restrict__ block_vis,
                                                             uint32_t *__restrict__ block_pairs) {
    __shared__ uint32_t lds[4];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t nv = 0, np = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t c = base + k < n ? count[base + k] : 0u;
        nv += c > 0u ? 1u : 0u;
        np = sat_add(np, c);
    }
    uint32_t tv, tp;
    block_exclusive_scan(nv, lds, tv);
    block_exclusive_scan(np, lds, tp);
    if (threadIdx.x == 0) {
        block_vis[blockIdx.x] = tv;
        block_pairs[blockIdx.x] = tp;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_vis_apply(ViewTable vt, uint64_t n_view,
                                                            const uint32_t *__restrict__ count,
                                                            Rec *__restrict__ rec,
                                                            const uint32_t *__restrict__ zkey, uint64_t n,
                                                            const uint32_t *__restrict__ block_vis,
                                                            const uint32_t *__restrict__ block_pairs,
                                                            uint32_t *__restrict__ vis, uint32_t *__restrict__ poff,
                                                            uint4 *__restrict__ item_box,
                                                            uint32_t *__restrict__ chunk_item, uint64_t chunks_cap,
                                                            WsHeader *__restrict__ hdr) {
    // The block's kScanTile items in kScanItems rounds of kScanThreads
    // consecutive ones (round k, thread t: item base + k kScanThreads + t), so
    // that every load and store of a round is row-contiguous across the wave.
    // Per wave and round: the inclusive totals of the visible flags and the
    // pair counts; last, the wave's part of the sums of the blocks before.
    constexpr int kV = kScanItems * 2;
    __shared__ uint32_t s_w[4][kV + 2];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t c[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint64_t it = base + (uint64_t)k * kScanThreads + tid;
        c[k] = it < n ? count[it] : 0u;
    }
    // the visible items' boxes and depth keys, all requested before the scans
    // (the stores below into the same records would otherwise order each load
    // after the previous item's store)
    float4 r2[kScanItems];
    uint32_t z[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (c[k] > 0u) {
            const uint64_t it = base + (uint64_t)k * kScanThreads + tid;
            r2[k] = rec[it].r2;
            z[k] = zkey[it];
        }
    }
    // the sums of the blocks before this one
    uint32_t bv = 0, bp = 0;
    for (uint32_t j = tid; j < blockIdx.x; j += kScanThreads) {
        bv += block_vis[j];
        bp = sat_add(bp, block_pairs[j]);
    }
    bv = wave_reduce(bv, 0u, sat_add);
    bp = wave_reduce(bp, 0u, sat_add);
    uint32_t fv[kScanItems], fp[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        fv[k] = wave_inclusive_scan(c[k] > 0u ? 1u : 0u, sat_add);
        fp[k] = wave_inclusive_scan(c[k], sat_add);
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) s_w[w][k] = fv[k], s_w[w][kScanItems + k] = fp[k];
        s_w[w][kV] = bv;
        s_w[w][kV + 1] = bp;
    }
    __syncthreads();
    uint32_t v0 = 0, p0 = 0;  // visible items and pairs before the current round
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) v0 = sat_add(v0, s_w[ww][kV]), p0 = sat_add(p0, s_w[ww][kV + 1]);
    uint32_t kv[kScanItems], run[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        uint32_t ov = 0, op = 0, tv = 0, tp = 0;  // waves before this one; the whole round
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
            if (ww < w) ov = sat_add(ov, s_w[ww][k]), op = sat_add(op, s_w[ww][kScanItems + k]);
            tv = sat_add(tv, s_w[ww][k]);
            tp = sat_add(tp, s_w[ww][kScanItems + k]);
        }
        kv[k] = sat_add(sat_add(v0, ov), fv[k] - (c[k] > 0u ? 1u : 0u));
        run[k] = sat_add(sat_add(p0, op), fp[k] - c[k]);
        v0 = sat_add(v0, tv);
        p0 = sat_add(p0, tp);
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        hdr->n_visible = v0;
        hdr->n_pairs = p0;
        hdr->overflow = p0 > hdr->pair_capacity ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (c[k] > 0u) {
            const uint32_t item = (uint32_t)(base + (uint64_t)k * kScanThreads + tid);
            vis[kv[k]] = item;
            poff[kv[k]] = run[k];
            item_box[kv[k]] = item_box_word(vt, n_view, item, r2[k], z[k]);
            rec[item].r2.w = __uint_as_float(run[k]);  // the item's first pair, for the later passes
            // chunks whose first pair lies in [run, run + c)
            const uint32_t end = sat_add(run[k], c[k]);
            for (uint64_t ch = chunk_count(run[k]); ch < chunks_cap && ch * kChunkPairs < end; ++ch)
                chunk_item[ch] = kv[k];
        }
    }
}

void launch_visible_offsets(const ViewTable &vt, uint64_t n, const uint32_t *count, Rec *rec,
                            const uint32_t *zkey, uint64_t items, uint32_t *vis, uint32_t *poff, uint4 *item_box,
                            uint32_t *chunk_item, uint64_t chunks_cap, uint32_t *block_tmp, WsHeader *hdr,
                            hipStream_t st) {
    const uint32_t nb = (uint32_t)((items + kScanTile - 1) / kScanTile);
    if (nb == 0) return;
    uint32_t *bv = block_tmp, *bp = block_tmp + nb;
    hipLaunchKernelGGL(k_vis_reduce, dim3(nb), dim3(kScanThreads), 0, st, count, items, bv, bp);
    hipLaunchKernelGGL(k_vis_apply, dim3(nb), dim3(kScanThreads), 0, st, vt, n, count, rec, zkey, items, bv, bp, vis,
                       poff, item_box, chunk_item, chunks_cap, hdr);
}

// ---------------------------------------------------------------------------
// A4: LSD radix sort, one 8-bit digit per pass.
//   k_radix_hist    per-block digit histogram -> hist[digit][block]
//   k_radix_scan    per digit: exclusive scan over blocks (in place) + total
//   k_radix_scatter rank within the block (wave ballots, stable; or LDS
//                   atomics for a first pass that need not be), scatter
// The element count is read on the device: either *n_dev or, for the pair
// sort, 0 when the header flags an overflow.
// ---------------------------------------------------------------------------
// A block sorts TILE consecutive elements.
// Rounds of 64 consecutive elements per wave: wave w of a block owns the
// block's elements [w * TILE / 4, (w + 1) * TILE / 4), which keeps the block's
// order (wave, round, lane) equal to the input order.
template <int TILE>
struct SortShape {
    static constexpr int kWaveSpan = TILE / (kSortThreads / 64);
    static constexpr int kRounds = kWaveSpan / 64;
    static constexpr int kItems = TILE / kSortThreads;
};

// Lanes of the wave holding the same digit (of `bits` <= 8 bits) as this lane.
__device__ __forceinline__ unsigned long long digit_peers(bool ok, uint32_t d, int bits) {
    unsigned long long match = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (b >= bits) break;
        const unsigned long long bal = __ballot(ok && ((d >> b) & 1u));
        match &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return match;
}

// Per-block digit histogram (LDS atomics; all loads are issued first).
template <int TILE>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *__restrict__ keys, SortCount sc,
                                                             int shift, uint32_t mask, uint32_t *__restrict__ hist,
                                                             uint32_t hist_blocks) {
    __shared__ uint32_t h[256];
    const uint64_t n = sc();
    const uint64_t blk = (uint64_t)blockIdx.x * TILE;
    if (blk >= n) return;  // blocks past the end are never scanned
    const uint32_t m = (uint32_t)min((uint64_t)TILE, n - blk);
    uint32_t k[SortShape<TILE>::kItems];
#pragma unroll
    for (int r = 0; r < SortShape<TILE>::kItems; ++r) {
        const uint32_t li = (uint32_t)r * kSortThreads + threadIdx.x;
        k[r] = li < m ? keys[blk + li] : 0u;
    }
    h[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SortShape<TILE>::kItems; ++r)
        if ((uint32_t)r * kSortThreads + threadIdx.x < m) atomicAdd(&h[(k[r] >> shift) & mask], 1u);
    __syncthreads();
    hist[(size_t)threadIdx.x * hist_blocks + blockIdx.x] = h[threadIdx.x];
}

// One workgroup per digit: exclusive scan of hist[d][0..nb) in place, each
// thread taking kScanRun consecutive blocks per sweep (one sweep covers 2048
// blocks, 6.3M elements at 3072 per block).
constexpr int kScanRun = 8;
template <int TILE>
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t *__restrict__ hist, uint32_t hist_blocks, SortCount sc,
                                                    uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t lds[4];
    const uint64_t n = sc();
    const uint32_t nb = (uint32_t)((n + TILE - 1) / TILE);
    uint32_t *row = hist + (size_t)blockIdx.x * hist_blocks;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += 256 * kScanRun) {
        const uint32_t bt = b0 + threadIdx.x * kScanRun;
        uint32_t x[kScanRun], sum = 0;
#pragma unroll
        for (int j = 0; j < kScanRun; ++j) {
            x[j] = bt + j < nb ? row[bt + j] : 0u;
            sum += x[j];
        }
        uint32_t total;
        uint32_t ex = carry + block_exclusive_scan(sum, lds, total);
#pragma unroll
        for (int j = 0; j < kScanRun; ++j) {
            if (bt + j < nb) row[bt + j] = ex;
            ex += x[j];
        }
        carry += total;
    }
    if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// Stable scatter of one block's TILE elements.  Each wave loads its TILE / 4
// consecutive elements up front, then ranks them round by round against its
// own running digit counts (ballot peers; no block barrier inside the loop).
// One barrier later the waves' counts become offsets, the block's elements
// are placed in LDS in digit order, and written out in contiguous runs per
// digit (coalesced, instead of one random 4-byte write per element).  With
// STABLE false (a first pass whose caller does not need equal keys kept in
// input order) each element takes its rank from an LDS atomic on its wave's
// digit count instead of the ballots.
template <int TILE, bool STABLE>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                const uint32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout,
                                                                uint32_t *__restrict__ vout, SortCount sc, int shift,
                                                                int bits, const uint32_t *__restrict__ hist,
                                                                uint32_t hist_blocks,
                                                                const uint32_t *__restrict__ digit_total) {
    __shared__ uint32_t gbase[256];      // global position of this block's first element of each digit
    __shared__ uint32_t lbase[256];      // block-local position of the same
    __shared__ uint32_t wcnt[4][256];    // per-wave running digit counts, then per-wave block-local offsets
    __shared__ uint32_t lds[4];
    __shared__ uint32_t skey[TILE], sval[TILE];
    const uint64_t n = sc();
    const uint32_t nb = (uint32_t)((n + TILE - 1) / TILE);
    if (blockIdx.x >= nb) return;
    // neighbouring blocks write neighbouring parts of each digit's output
    // range (often the same cache lines): keep them on one XCD
    const uint32_t tb = xcd_contiguous(blockIdx.x, nb);
    const uint64_t blk = (uint64_t)tb * TILE;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t t = threadIdx.x;
    const uint32_t m = (uint32_t)min((uint64_t)TILE, n - blk);
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t key[SortShape<TILE>::kRounds], val[SortShape<TILE>::kRounds];
#pragma unroll
    for (int r = 0; r < SortShape<TILE>::kRounds; ++r) {
        const uint32_t li = (uint32_t)(w * SortShape<TILE>::kWaveSpan + r * 64 + lane);
        key[r] = li < m ? kin[blk + li] : 0u;
        val[r] = li < m ? vin[blk + li] : 0u;
    }
    {
        uint32_t total;
        // digits above the mask do not occur in this pass (their totals were not scanned)
        const bool used = t <= mask;
        const uint32_t tot = used ? digit_total[t] : 0u;
        const uint32_t ex = block_exclusive_scan(tot, lds, total);
        const uint32_t mine = used ? hist[(size_t)t * hist_blocks + tb] : 0u;
        const uint32_t next = !used ? 0u : tb + 1 < nb ? hist[(size_t)t * hist_blocks + tb + 1] : tot;
        gbase[t] = ex + mine;
        lbase[t] = block_exclusive_scan(next - mine, lds, total);
    }
    for (int k = 0; k < 4; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const unsigned long long lt_mask = (1ull << lane) - 1ull;
    uint32_t pos[SortShape<TILE>::kRounds];
#pragma unroll
    for (int r = 0; r < SortShape<TILE>::kRounds; ++r) {
        const uint32_t li = (uint32_t)(w * SortShape<TILE>::kWaveSpan + r * 64 + lane);
        const bool ok = li < m;
        const uint32_t d = (key[r] >> shift) & mask;
        if constexpr (!STABLE) {
            pos[r] = ok ? atomicAdd(&wcnt[w][d], 1u) : 0u;
            continue;
        }
        const unsigned long long peers = digit_peers(ok, d, bits);
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const uint32_t before = ok ? wcnt[w][d] : 0u;
        pos[r] = before + rank;
        // the digit's last lane advances the wave's count (read above by every lane first)
        __builtin_amdgcn_wave_barrier();
        if (ok && (peers >> lane) == 1ull) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const uint32_t c0 = wcnt[0][t], c1 = wcnt[1][t], c2 = wcnt[2][t];
        const uint32_t b = lbase[t];
        wcnt[0][t] = b;
        wcnt[1][t] = b + c0;
        wcnt[2][t] = b + c0 + c1;
        wcnt[3][t] = b + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SortShape<TILE>::kRounds; ++r) {
        const uint32_t li = (uint32_t)(w * SortShape<TILE>::kWaveSpan + r * 64 + lane);
        if (li < m) {
            const uint32_t p = wcnt[w][(key[r] >> shift) & mask] + pos[r];
            skey[p] = key[r];
            sval[p] = val[r];
        }
    }
    __syncthreads();
    // write out in local order: runs of one digit go to consecutive addresses
    for (uint32_t p = t; p < m; p += kSortThreads) {
        const uint32_t k = skey[p];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t g = gbase[d] + (p - lbase[d]);
        kout[g] = k;
        vout[g] = sval[p];
    }
}

template <int TILE>
static void radix_passes(uint32_t *keys[2], uint32_t *vals[2], SortCount sc, uint64_t n_cap, int begin_bit,
                         int end_bit, uint32_t *hist, uint32_t hist_blocks, uint32_t *digit_total, int &cur,
                         bool stable, hipStream_t st) {
    const uint32_t nb = (uint32_t)((n_cap + TILE - 1) / TILE);
    // as many 8-bit passes as the key needs, with the bits spread evenly over
    // them (13 bits: 7 + 6): fewer digits per pass means longer runs per digit
    // in each block's output, so better coalesced writes
    const int total_bits = end_bit - begin_bit;
    const int passes = (total_bits + 7) / 8;
    for (int pass = 0, shift = begin_bit; pass < passes; ++pass) {
        const int bits = (end_bit - shift + (passes - pass) - 1) / (passes - pass);
        // the result buffer depends only on the number of passes, not on n
        if (nb == 0) {
            cur ^= 1;
            shift += bits;
            continue;
        }
        const uint32_t mask = (1u << bits) - 1u;
        hipLaunchKernelGGL(k_radix_hist<TILE>, dim3(nb), dim3(kSortThreads), 0, st, keys[cur], sc, shift, mask, hist,
                           hist_blocks);
        hipLaunchKernelGGL(k_radix_scan<TILE>, dim3(1u << bits), dim3(256), 0, st, hist, hist_blocks, sc, digit_total);
        // only the first pass may break ties: every later one keeps the order of the digits below
        if (pass == 0 && !stable)
            hipLaunchKernelGGL((k_radix_scatter<TILE, false>), dim3(nb), dim3(kSortThreads), 0, st, keys[cur],
                               vals[cur], keys[cur ^ 1], vals[cur ^ 1], sc, shift, bits, hist, hist_blocks,
                               digit_total);
        else
            hipLaunchKernelGGL((k_radix_scatter<TILE, true>), dim3(nb), dim3(kSortThreads), 0, st, keys[cur],
                               vals[cur], keys[cur ^ 1], vals[cur ^ 1], sc, shift, bits, hist, hist_blocks,
                               digit_total);
        cur ^= 1;
        shift += bits;
    }
}

void radix_sort_u32(uint32_t *keys[2], uint32_t *vals[2], SortCount sc, uint64_t n_cap, int begin_bit, int end_bit,
                    uint32_t *hist, uint32_t hist_blocks, uint32_t *digit_total, int &cur, bool stable,
                    hipStream_t st) {
    radix_passes<kSortTile>(keys, vals, sc, n_cap, begin_bit, end_bit, hist, hist_blocks, digit_total, cur, stable,
                            st);
}

// ---------------------------------------------------------------------------
// A3: emission.  The k-th visible item (ascending item id) owns pairs
// [poff[k], poff[k] + count) in row-major order over its tile box.  A workgroup
// writes one chunk of 1024 consecutive pair slots, 4 per thread (16-byte
// stores, so the writes are coalesced and equal per thread however the tile
// counts are spread): the chunk's items are staged in LDS and each thread finds
// its pairs' item by binary search there.  The items' box words come from the
// compaction pass (by visible index: coalesced loads).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kChunkThreads) void k_emit(const uint32_t *__restrict__ poff,
                                                        const uint32_t *__restrict__ chunk_item,
                                                        const uint4 *__restrict__ item_box,
                                                        uint32_t *__restrict__ pkey, uint32_t *__restrict__ pval,
                                                        uint32_t *__restrict__ pflag, const WsHeader *__restrict__ hdr) {
    __shared__ ChunkItems ci;
    if (hdr->overflow) return;
    const uint32_t m = hdr->n_pairs, nvis = hdr->n_visible;
    const uint32_t c0 = blockIdx.x * kChunkPairs;
    if (c0 >= m) return;  // uniform per workgroup
    const uint32_t cend = min(c0 + kChunkPairs, m);
    uint32_t i_lo;
    const uint32_t nloc = load_chunk_items(poff, chunk_item, item_box, blockIdx.x, m, nvis, ci, i_lo);
    const uint32_t pb = c0 + threadIdx.x * kChunkPerThread;
    if (pb >= cend) return;
    pflag[pb / 4] = 0u;  // the four slots' "moments written" flags, set by the backward compositing
    uint32_t key[kChunkPerThread], val[kChunkPerThread];
    PairWalker pw;
    pw.start(ci, nloc, pb);
#pragma unroll
    for (uint32_t u = 0; u < kChunkPerThread; ++u) {
        if (u > 0) pw.next(ci, nloc, pb + u);
        key[u] = pw.tile(ci);
        val[u] = ci.item[pw.k];
    }
    if (pb + kChunkPerThread <= cend) {
        *reinterpret_cast<uint4 *>(pkey + pb) = make_uint4(key[0], key[1], key[2], key[3]);
        *reinterpret_cast<uint4 *>(pval + pb) = make_uint4(val[0], val[1], val[2], val[3]);
    } else {
        for (uint32_t u = 0; pb + u < cend; ++u) {
            pkey[pb + u] = key[u];
            pval[pb + u] = val[u];
        }
    }
}

void launch_emit_pairs(const uint32_t *poff, const uint32_t *chunk_item, const uint4 *item_box, uint64_t pair_grid,
                       uint32_t *pkey, uint32_t *pval, uint32_t *pflag, const WsHeader *hdr, hipStream_t st) {
    static_assert(kChunkPerThread == 4, "one 32-bit word of slot flags per thread");
    const uint64_t chunks = chunk_count(pair_grid);
    if (chunks == 0) return;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)chunks), dim3(kChunkThreads), 0, st, poff, chunk_item, item_box, pkey,
                       pval, pflag, hdr);
}

// ---------------------------------------------------------------------------
// A4c: per-tile depth order.  After the tile sort each tile's list holds its
// items in no particular order; it is sorted here by the 64-bit key
// (depth key << 32 | item), the unique order of the compositing definition.
//
// The network is bitonic with every comparator oriented low-to-high: each
// merge starts with a "flip" that pairs mirrored positions, then half-cleaners
// at halving distances.  Lists are padded to a power of two with keys above
// every real key, which the network leaves at the end.
//
// A workgroup of four waves takes one tile.  A list of up to 1024 entries (most
// tiles) is sorted by a bucket pass (below) when the depths allow, else by the
// network in registers.  There each lane holds E (1..16) consecutive entries,
// so comparators closer than E are register operations and the others pair
// lane l with lane l ^ m, fetched with DPP or ds_swizzle (within 32 lanes) or
// ds_bpermute, or, across waves, exchanged through LDS; a flip also mirrors
// the register index.  Lists of 1025..4096 entries take the network with 16
// entries per lane; longer lists run the multi-workgroup path (below) or, when
// it is off, the same network over global memory, one comparator per thread
// and step.
// ---------------------------------------------------------------------------
typedef unsigned long long u64;
constexpr u64 kPadKey = ~0ull;
constexpr int kBlockBucketMax = 1024;  // bucket path: four waves, up to 4 entries per lane

// v from lane (lane ^ M)
template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane) {
    if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
    else if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x1B, 0xF, 0xF, false);  // quad_perm 3,2,1,0
    else if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false); // row_half_mirror
    else if constexpr (M == 8) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false); // row_ror 8
    else if constexpr (M == 15) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false); // row_mirror
    else if constexpr (M < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (M << 10));  // xor in 32 lanes
    else return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ M) << 2, (int)v);
}

template <int M>
__device__ __forceinline__ u64 lane_xor64(u64 v, int lane) {
    const uint32_t lo = lane_xor<M>((uint32_t)v, lane), hi = lane_xor<M>((uint32_t)(v >> 32), lane);
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ void order_regs(u64 &a, u64 &b) {
    const u64 x = a, y = b;
    a = x < y ? x : y;
    b = x < y ? y : x;
}

// keep the smaller of (mine, other) when `low`, else the larger
__device__ __forceinline__ u64 keep(u64 mine, u64 other, bool low) { return (other < mine) == low ? other : mine; }

// One comparator step of the network over P = 64 * E * W keys: merge size K,
// distance J (J == K / 2 is the flip).  key[r] of lane `lane` in wave `wave`
// is entry wave * 64E + lane * E + r.  W > 1 exchanges across waves through
// `xs` (64 * E * W words) and requires every thread of the W waves.
template <int E, int W, int K, int J>
__device__ __forceinline__ void bitonic_step(u64 (&key)[E], int lane, int wave, uint32_t *xs) {
    constexpr bool kFlip = J == K / 2;
    if constexpr (J < E) {  // both entries in this lane's registers
#pragma unroll
        for (int r = 0; r < E; ++r) {
            if constexpr (kFlip) {
                if ((r ^ (K - 1)) > r) order_regs(key[r], key[r ^ (K - 1)]);
            } else {
                if (!(r & J)) order_regs(key[r], key[r + J]);
            }
        }
    } else if constexpr (J < 64 * E) {  // another lane of this wave
        if constexpr (kFlip) {
            const bool low = !(lane & (K / (2 * E)));
            u64 o[E];
#pragma unroll
            for (int r = 0; r < E; ++r) o[r] = lane_xor64<K / E - 1>(key[E - 1 - r], lane);
#pragma unroll
            for (int r = 0; r < E; ++r) key[r] = keep(key[r], o[r], low);
        } else {
            const bool low = !(lane & (J / E));
#pragma unroll
            for (int r = 0; r < E; ++r) key[r] = keep(key[r], lane_xor64<J / E>(key[r], lane), low);
        }
    } else {  // another wave: through LDS, one 32-bit half at a time
        static_assert(W > 1, "cross-wave steps need several waves");
        constexpr int M = kFlip ? K / (64 * E) - 1 : J / (64 * E);
        const bool low = !(wave & (kFlip ? K / (128 * E) : M));
        const int pw = wave ^ M, pl = kFlip ? lane ^ 63 : lane;
        uint32_t half[2][E];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int r = 0; r < E; ++r) xs[(r * W + wave) * 64 + lane] = (uint32_t)(key[r] >> (32 * h));
            __syncthreads();
#pragma unroll
            for (int r = 0; r < E; ++r) half[h][r] = xs[((kFlip ? E - 1 - r : r) * W + pw) * 64 + pl];
            __syncthreads();
        }
#pragma unroll
        for (int r = 0; r < E; ++r) key[r] = keep(key[r], ((u64)half[1][r] << 32) | half[0][r], low);
    }
}

template <int E, int W, int K, int J>
__device__ __forceinline__ void bitonic_merge(u64 (&key)[E], int lane, int wave, uint32_t *xs) {
    bitonic_step<E, W, K, J>(key, lane, wave, xs);
    if constexpr (J > 1) bitonic_merge<E, W, K, J / 2>(key, lane, wave, xs);
}

template <int E, int W, int K = 2>
__device__ __forceinline__ void register_bitonic(u64 (&key)[E], int lane, int wave, uint32_t *xs) {
    bitonic_merge<E, W, K, K / 2>(key, lane, wave, xs);
    if constexpr (K < 64 * E * W) register_bitonic<E, W, 2 * K>(key, lane, wave, xs);
}

// Sort list[0, len) of item ids by (zkey[item], item); the caller's threads
// are `W` whole waves and 64 * E * W >= len.  The result goes back to list,
// or, with out_hi non-null, as keys to out_hi (depth key) / out_lo (item).
template <int E, int W>
__device__ __forceinline__ void sort_list_regs(uint32_t *__restrict__ list, uint32_t len,
                                               const uint32_t *__restrict__ zkey, int lane, int wave, uint32_t *xs,
                                               uint32_t *__restrict__ out_hi = nullptr,
                                               uint32_t *__restrict__ out_lo = nullptr) {
    u64 key[E];
    const uint32_t base = (uint32_t)(wave * 64 + lane) * E;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = base + r;
        const uint32_t item = i < len ? list[i] : 0u;
        key[r] = i < len ? (((u64)zkey[item] << 32) | item) : kPadKey;
    }
    register_bitonic<E, W>(key, lane, wave, xs);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if (base + r < len) {
            if (out_hi) {
                out_hi[base + r] = (uint32_t)(key[r] >> 32);
                out_lo[base + r] = (uint32_t)key[r];
            } else {
                list[base + r] = (uint32_t)key[r];
            }
        }
    }
}

// Fast path: a counting sort on a bucket index that is a monotone function of
// the depth key, b = floor((z - zmin) * NB / (zmax - zmin + 1)) in FP32
// (conversion, product and truncation are all non-decreasing, so bucket order
// never contradicts key order).  Entries are dropped into their bucket in
// arrival order; each then counts the bucket-mates with a smaller 64-bit key
// and stores itself at bucket start + that count.  For depths spread over the
// tile's range a bucket holds about one entry, so the ranking costs a read or
// two per entry, all independent.  Returns false, having written nothing, when
// some bucket holds more than kMaxBucket entries (clustered depths): the
// caller then sorts with the network, whose cost does not depend on the keys.
// Runs on the whole workgroup (256 threads, E entries each: NB = 256 E).
constexpr uint32_t kMaxBucket = 16;

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    return wave_reduce(v, 0xffffffffu, [](uint32_t a, uint32_t b) { return min(a, b); });
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    return wave_reduce(v, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
}

template <int E>
__device__ bool bucket_sort_block(uint32_t *__restrict__ list, uint32_t len, const uint32_t *__restrict__ zkey,
                                  u64 *buf, uint32_t *cnt, uint32_t *red /* [8] */) {
    constexpr uint32_t NB = 256 * E;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int r = 0; r < E; ++r) cnt[r * 256 + tid] = 0u;
    u64 key[E];
    uint32_t zmin = 0xffffffffu, zmax = 0u;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = (uint32_t)r * 256 + tid;
        const uint32_t item = i < len ? list[i] : 0u;
        const uint32_t z = i < len ? zkey[item] : 0u;
        key[r] = ((u64)z << 32) | item;
        if (i < len) zmin = min(zmin, z), zmax = max(zmax, z);
    }
    zmin = wave_min_u32(zmin);
    zmax = wave_max_u32(zmax);
    if (lane == 0) red[wave] = zmin, red[4 + wave] = zmax;
    __syncthreads();
    zmin = min(min(red[0], red[1]), min(red[2], red[3]));
    zmax = max(max(red[4], red[5]), max(red[6], red[7]));
    const float scale = (float)NB / ((float)(zmax - zmin) + 1.0f);
    uint32_t bk[E], slot[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((uint32_t)r * 256 + tid < len) {
            const uint32_t z = (uint32_t)(key[r] >> 32);
            bk[r] = min(NB - 1, (uint32_t)((float)(z - zmin) * scale));
            slot[r] = atomicAdd(&cnt[bk[r]], 1u);
        }
    }
    __syncthreads();
    // thread owns buckets [tid * E, tid * E + E): their exclusive starts
    uint32_t c[E], run = 0, big = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        c[j] = cnt[tid * E + j];
        run += c[j];
        big = max(big, c[j]);
    }
    big = wave_max_u32(big);
    if (lane == 0) red[wave] = big;  // (red was last read before the barrier above)
    uint32_t total;
    uint32_t st = block_exclusive_scan(run, red + 4, total);  // ends with a barrier
    big = max(max(red[0], red[1]), max(red[2], red[3]));
    if (big > kMaxBucket) return false;  // uniform
#pragma unroll
    for (int j = 0; j < E; ++j) {
        cnt[tid * E + j] = (st << 16) | c[j];  // start < 2^16, count <= kMaxBucket
        st += c[j];
    }
    __syncthreads();
    uint32_t sc[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((uint32_t)r * 256 + tid < len) {
            sc[r] = cnt[bk[r]];
            buf[(sc[r] >> 16) + slot[r]] = key[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((uint32_t)r * 256 + tid < len) {
            const uint32_t s0 = sc[r] >> 16, n = sc[r] & 0xffffu;
            uint32_t rank = 0;
            for (uint32_t q = 0; q < n; ++q) rank += buf[s0 + q] < key[r] ? 1u : 0u;
            list[s0 + rank] = (uint32_t)key[r];
        }
    }
    return true;
}

template <int E>
__device__ __forceinline__ void sort_list_block(uint32_t *__restrict__ list, uint32_t len,
                                                const uint32_t *__restrict__ zkey, u64 *buf, uint32_t *cnt,
                                                uint32_t *red, uint32_t *xs) {
    if (!bucket_sort_block<E>(list, len, zkey, buf, cnt, red)) {
        __syncthreads();  // the network reuses the exchange area
        sort_list_regs<E, 4>(list, len, zkey, threadIdx.x & 63, threadIdx.x >> 6, xs);
    }
}

// The same network over global memory, for lists beyond kGroupSortMax
// (comparators with an entry past the end are skipped: those entries act as
// +infinity).  Runs on the whole workgroup.
__device__ void sort_list_global(uint32_t *__restrict__ list, uint32_t len, const uint32_t *__restrict__ zkey,
                                 uint32_t *__restrict__ hi, uint32_t *__restrict__ lo) {
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        const uint32_t item = list[i];
        hi[i] = zkey[item];
        lo[i] = item;
    }
    __syncthreads();
    uint32_t p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (uint32_t k = 2; k <= p2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t c = threadIdx.x; c < p2 / 2; c += blockDim.x) {
                const uint32_t a = ((c & ~(j - 1)) << 1) | (c & (j - 1));
                const uint32_t b = j == (k >> 1) ? (a ^ (k - 1)) : (a + j);
                if (b < len) {
                    const uint32_t ha = hi[a], hb = hi[b], la = lo[a], lb = lo[b];
                    if (ha > hb || (ha == hb && la > lb)) hi[a] = hb, hi[b] = ha, lo[a] = lb, lo[b] = la;
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) list[i] = lo[i];
    __syncthreads();
}

// Lists longer than kGroupSortMax, when the multi-workgroup path takes them:
// every listed long tile of at most kLongWindow << passes entries (all of them
// once they fit the list).  k_long_windows numbers their windows (of
// kLongWindow entries for the run sort, of kMergeWindow outputs for the merge
// passes) in list order once per forward; a workgroup then finds its window
// by a binary search over those offsets.
__device__ __forceinline__ bool long_path_on(const WsHeader *hdr, int passes) {
    return passes > 0 && passes <= kMaxLongPasses && hdr->n_long <= kMaxLongTiles;
}

__global__ __launch_bounds__(256) void k_long_windows(const uint2 *__restrict__ ranges,
                                                      uint32_t *__restrict__ long_tiles, int passes,
                                                      const WsHeader *__restrict__ hdr) {
    constexpr int kPer = kMaxLongTiles / 256;
    __shared__ uint32_t lds[4];
    if (hdr->overflow || !long_path_on(hdr, passes)) return;  // uniform
    const uint32_t n_long = hdr->n_long;
    const uint64_t cover = (uint64_t)kLongWindow << passes;
    uint32_t na[kPer], nm[kPer], sa = 0, sm = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const uint32_t k = threadIdx.x * kPer + j;
        na[j] = nm[j] = 0;
        if (k < n_long) {
            const uint2 rg = ranges[long_tiles[k]];
            const uint32_t len = rg.y - rg.x;
            if ((uint64_t)len <= cover) {
                na[j] = (len + kLongWindow - 1) / kLongWindow;
                nm[j] = (len + kMergeWindow - 1) / kMergeWindow;
            }
        }
        sa += na[j];
        sm += nm[j];
    }
    uint32_t ta, tm;
    uint32_t ea = block_exclusive_scan(sa, lds, ta);
    uint32_t em = block_exclusive_scan(sm, lds, tm);
    uint32_t *wa = long_tiles + kMaxLongTiles, *wm = wa + kMaxLongTiles + 1;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const uint32_t k = threadIdx.x * kPer + j;
        if (k < n_long) wa[k] = ea, wm[k] = em;
        ea += na[j];
        em += nm[j];
    }
    if (threadIdx.x == 0) wa[n_long] = ta, wm[n_long] = tm;
}

void launch_long_windows(const uint2 *ranges, uint32_t *long_tiles, int long_passes, const WsHeader *hdr,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_long_windows, dim3(1), dim3(256), 0, st, ranges, long_tiles, long_passes, hdr);
}

// Window e of all the long lists' windows (offsets `first`: one of the two
// tables above) as (tile, window within its list); false past the last.
__device__ __forceinline__ bool long_tile_window(const uint32_t *__restrict__ long_tiles,
                                                 const uint32_t *__restrict__ first, uint32_t n_long, uint32_t e,
                                                 uint32_t &tile, uint32_t &w) {
    if (n_long == 0 || e >= first[n_long]) return false;
    // the last list whose first window is at or before e (it has windows: the
    // next offset, or the total, is above e)
    uint32_t lo = 0, hi = n_long - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= e)
            lo = mid;
        else
            hi = mid - 1;
    }
    tile = long_tiles[lo];
    w = e - first[lo];
    return true;
}

// The fused compositing's schedule, filed by one workgroup: every tile in the
// bucket of min(its list length, cost_hint[t]).  Each bucket has room for
// every tile, so filing needs only a slot counter per bucket, kept in LDS
// (`slots`): returning atomics on global counters serialise across the chip
// when most tiles share a few buckets, as they do, while LDS atomics resolve
// the lanes that collide within one instruction.  kSched tiles per thread are
// loaded together.
constexpr int kSched = 16;
__device__ void file_schedule(const uint2 *__restrict__ ranges, const uint32_t *__restrict__ cost_hint,
                              uint32_t total_tiles, uint32_t *__restrict__ order, uint32_t *slots) {
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid < (int)kCostBuckets) slots[tid] = 0u;
    __syncthreads();
    for (uint32_t base = 0; base < total_tiles; base += (uint32_t)(nt * kSched)) {
        uint32_t b[kSched];
#pragma unroll
        for (int q = 0; q < kSched; ++q) {
            const uint32_t t = base + (uint32_t)(q * nt + tid);
            b[q] = kCostBuckets;  // none
            if (t < total_tiles) {
                const uint2 rg = ranges[t];
                b[q] = cost_bucket(min(rg.y - rg.x, cost_hint[t]));
            }
        }
#pragma unroll
        for (int q = 0; q < kSched; ++q) {
            if (b[q] < kCostBuckets) {
                const uint32_t slot = atomicAdd(&slots[b[q]], 1u);
                order[kCostBuckets + (size_t)b[q] * total_tiles + slot] = base + (uint32_t)(q * nt + tid);
            }
        }
    }
    __syncthreads();
    if (tid < (int)kCostBuckets) order[tid] = slots[tid];
}

__global__ __launch_bounds__(256) void k_tile_depth_sort(const uint2 *__restrict__ ranges, uint32_t total_tiles,
                                                         uint32_t *__restrict__ pval, const uint32_t *__restrict__ zkey,
                                                         uint32_t *__restrict__ x_hi, uint32_t *__restrict__ x_lo,
                                                         uint32_t *__restrict__ y_hi, uint32_t *__restrict__ y_lo,
                                                         const uint32_t *__restrict__ long_tiles, int passes,
                                                         uint32_t *__restrict__ sched,
                                                         const uint32_t *__restrict__ cost_hint,
                                                         const WsHeader *__restrict__ hdr) {
    __shared__ u64 s_buf[kGroupSortMax / 2];  // bucket entries; the network's exchange area (16 KB)
    __shared__ uint32_t s_cnt[kBlockBucketMax];
    __shared__ uint32_t s_red[8];
    if (hdr->overflow) return;  // uniform (no schedule either: the fused compositing falls back to tile order)
    uint32_t *xs = reinterpret_cast<uint32_t *>(s_buf);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool multi = long_path_on(hdr, passes);
    // with a schedule to file, workgroup 0 files it (overlapping the sorts)
    // and the tiles start at workgroup 1
    if (sched && blockIdx.x == 0) {
        file_schedule(ranges, cost_hint, total_tiles, sched, s_cnt);
        return;
    }
    const uint32_t bid = blockIdx.x - (sched ? 1u : 0u);
    if (bid >= total_tiles) {
        // a window of a long list, sorted into a run of the first merge pass's input
        if (!multi) return;
        uint32_t t, w;
        if (!long_tile_window(long_tiles, long_tiles + kMaxLongTiles, hdr->n_long, bid - total_tiles, t, w))
            return;
        const uint2 rg = ranges[t];
        const uint32_t off = rg.x + w * kLongWindow;
        const uint32_t n = min(kLongWindow, rg.y - off);
        uint32_t *oh = (passes & 1) ? x_hi : y_hi, *ol = (passes & 1) ? x_lo : y_lo;
        sort_list_regs<16, 4>(pval + off, n, zkey, lane, wave, xs, oh + off, ol + off);
        return;
    }
    const uint32_t t = bid;
    const uint2 rg = ranges[t];
    const uint32_t len = rg.y - rg.x;
    uint32_t *list = pval + rg.x;
    if (len <= 1) return;
    if (len <= 256)
        sort_list_block<1>(list, len, zkey, s_buf, s_cnt, s_red, xs);
    else if (len <= 512)
        sort_list_block<2>(list, len, zkey, s_buf, s_cnt, s_red, xs);
    else if (len <= (uint32_t)kBlockBucketMax)
        sort_list_block<4>(list, len, zkey, s_buf, s_cnt, s_red, xs);
    else if (len <= (uint32_t)kGroupSortMax)
        sort_list_regs<16, 4>(list, len, zkey, lane, wave, xs);
    else if (!multi || (uint64_t)len > ((uint64_t)kLongWindow << passes))
        sort_list_global(list, len, zkey, x_hi + rg.x, x_lo + rg.x);
    // else: the window workgroups and the merge passes sort it
}

void launch_tile_depth_sort(const uint2 *ranges, uint32_t total_tiles, uint32_t *pval, const uint32_t *zkey,
                            uint32_t *x_hi, uint32_t *x_lo, uint32_t *y_hi, uint32_t *y_lo,
                            const uint32_t *long_tiles, int long_passes, uint32_t chunk_wgs, uint32_t *sched,
                            const uint32_t *cost_hint, const WsHeader *hdr, hipStream_t st) {
    if (total_tiles == 0) return;
    const uint32_t grid = total_tiles + (long_passes > 0 ? chunk_wgs : 0u) + (sched ? 1u : 0u);
    hipLaunchKernelGGL(k_tile_depth_sort, dim3(grid), dim3(256), 0, st, ranges, total_tiles, pval, zkey, x_hi, x_lo,
                       y_hi, y_lo, long_tiles, long_passes, sched, cost_hint, hdr);
}

// ---------------------------------------------------------------------------
// A4d: merge passes over the long lists' sorted runs.  Pass p merges runs of
// kLongWindow << p pairwise; a workgroup makes kMergeWindow consecutive
// outputs of one merge.  Its inputs start where the merge path crosses its
// first and last output (found by one wave each, 64 probes per round), are
// staged in LDS, and each thread merges 8 outputs from its own crossing.
// Keys are unique, so every split is unambiguous.
// ---------------------------------------------------------------------------
__device__ __forceinline__ u64 load_key(const uint32_t *__restrict__ hi, const uint32_t *__restrict__ lo, uint32_t i) {
    return ((u64)hi[i] << 32) | lo[i];
}

// Number of elements of A among the first d outputs of merge(A, B): the
// smallest a in [max(0, d - nB), min(d, nA)] with not (A[a] < B[d - 1 - a]).
// One whole wave calls it.
__device__ uint32_t wave_merge_split(const uint32_t *a_hi, const uint32_t *a_lo, uint32_t nA, const uint32_t *b_hi,
                                     const uint32_t *b_lo, uint32_t nB, uint32_t d, int lane) {
    uint32_t lo = d > nB ? d - nB : 0u, hi = min(d, nA);
    while (lo < hi) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t m = lo + (uint32_t)lane * step;
        const bool probe = m < hi;
        const bool before = probe && load_key(a_hi, a_lo, m) < load_key(b_hi, b_lo, d - 1 - m);
        const uint32_t c = (uint32_t)__popcll(__ballot(before));  // probes before the split: a prefix of the lanes
        const uint32_t nlo = c > 0 ? lo + (c - 1) * step + 1 : lo;
        const uint32_t nhi = min(hi, lo + c * step);
        lo = nlo;
        hi = nhi;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_long_merge(const uint2 *__restrict__ ranges,
                                                    const uint32_t *__restrict__ long_tiles,
                                                    const WsHeader *__restrict__ hdr, int p, int passes,
                                                    const uint32_t *__restrict__ src_hi,
                                                    const uint32_t *__restrict__ src_lo, uint32_t *__restrict__ dst_hi,
                                                    uint32_t *__restrict__ dst_lo, uint32_t *__restrict__ pval) {
    __shared__ u64 sA[kMergeWindow], sB[kMergeWindow];
    __shared__ uint32_t s_split[2];
    if (hdr->overflow || !long_path_on(hdr, passes)) return;  // uniform
    uint32_t t, w;
    if (!long_tile_window(long_tiles, long_tiles + 2 * kMaxLongTiles + 1, hdr->n_long, blockIdx.x, t, w)) return;
    const uint2 rg = ranges[t];
    const uint32_t L = rg.y - rg.x;
    const uint32_t o0 = w * kMergeWindow, o1 = min(o0 + kMergeWindow, L);
    const uint64_t R64 = (uint64_t)kLongWindow << p;  // p < kMaxLongPasses: R < 2^29
    const uint32_t R = (uint32_t)R64;
    const uint32_t base = (uint32_t)((o0 / (2 * R64)) * (2 * R64));
    const uint32_t nA = min(R, L - base), nB = L - base > R ? min(R, L - base - R) : 0u;
    const uint32_t *ah = src_hi + rg.x + base, *al = src_lo + rg.x + base;
    const uint32_t *bh = ah + R, *bl = al + R;
    const bool last = p == passes - 1;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t d0 = o0 - base, d1 = o1 - base;
    if (wave < 2) {
        const uint32_t a = wave_merge_split(ah, al, nA, bh, bl, nB, wave == 0 ? d0 : d1, (int)lane);
        if (lane == 0) s_split[wave] = a;
    }
    __syncthreads();
    const uint32_t a0 = s_split[0], a1 = s_split[1], b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t na = a1 - a0, nb = b1 - b0;
    for (uint32_t k = tid; k < na; k += 256) sA[k] = load_key(ah, al, a0 + k);
    for (uint32_t k = tid; k < nb; k += 256) sB[k] = load_key(bh, bl, b0 + k);
    __syncthreads();
    constexpr uint32_t kPer = kMergeWindow / 256;
    const uint32_t q = tid * kPer;
    if (q >= na + nb) return;
    // this thread's crossing of the staged merge
    uint32_t lo = q > nb ? q - nb : 0u, hi = min(q, na);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sA[mid] < sB[q - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo, j = q - lo;
    const uint32_t out = rg.x + o0 + q;
    const uint32_t nq = min(kPer, na + nb - q);
    for (uint32_t k = 0; k < nq; ++k) {
        const bool take_b = i >= na || (j < nb && sB[j] < sA[i]);
        const u64 v = take_b ? sB[j] : sA[i];
        i += take_b ? 0u : 1u;
        j += take_b ? 1u : 0u;
        if (last) {
            pval[out + k] = (uint32_t)v;
        } else {
            dst_hi[out + k] = (uint32_t)(v >> 32);
            dst_lo[out + k] = (uint32_t)v;
        }
    }
}

void launch_long_merge(const uint2 *ranges, const uint32_t *long_tiles, const WsHeader *hdr, int p, int long_passes,
                       const uint32_t *src_hi, const uint32_t *src_lo, uint32_t *dst_hi, uint32_t *dst_lo,
                       uint32_t *pval, uint32_t merge_wgs, hipStream_t st) {
    if (merge_wgs == 0) return;
    hipLaunchKernelGGL(k_long_merge, dim3(merge_wgs), dim3(256), 0, st, ranges, long_tiles, hdr, p, long_passes,
                       src_hi, src_lo, dst_hi, dst_lo, pval);
}

// Tile id at every position of the sorted pairs (the export of the lists).
__global__ __launch_bounds__(256) void k_expand_ranges(const uint2 *__restrict__ ranges, uint32_t total_tiles,
                                                       uint32_t *__restrict__ pair_tiles,
                                                       const WsHeader *__restrict__ hdr) {
    const uint32_t t = blockIdx.x;
    if (t >= total_tiles || hdr->overflow) return;
    const uint2 rg = ranges[t];
    for (uint32_t i = rg.x + threadIdx.x; i < rg.y; i += 256) pair_tiles[i] = t;
}

void launch_expand_ranges(const uint2 *ranges, uint32_t total_tiles, uint32_t *pair_tiles, const WsHeader *hdr,
                          hipStream_t st) {
    if (total_tiles == 0) return;
    hipLaunchKernelGGL(k_expand_ranges, dim3(total_tiles), dim3(256), 0, st, ranges, total_tiles, pair_tiles, hdr);
}

// ---------------------------------------------------------------------------
// A5: per-tile [start, end) over the sorted pairs.  Where the tile key changes
// (and once more at i = m) the previous tile is closed, the new one opened, and
// the tiles in between marked empty, so no pre-clearing pass is needed.  Each
// thread takes kRangeRun consecutive pairs (16-byte loads).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tile_boundary(const uint32_t *__restrict__ pkey, uint2 *__restrict__ ranges,
                                              uint32_t *__restrict__ long_tiles, WsHeader *__restrict__ hdr,
                                              uint64_t i, uint64_t m, int64_t prev, int64_t t) {
    for (int64_t u = prev + 1; u < t; ++u) ranges[u] = make_uint2((uint32_t)i, (uint32_t)i);
    if (i < m) ranges[t].x = (uint32_t)i;
    if (i == 0) return;
    ranges[prev].y = (uint32_t)i;
    // a list longer than kGroupSortMax: find where it starts (the keys are
    // sorted) and register it for the multi-workgroup sort
    if (i > (uint64_t)kGroupSortMax && pkey[i - kGroupSortMax - 1] == (uint32_t)prev) {
        uint64_t lo = 0, hi = i - kGroupSortMax - 1;  // first position holding prev lies in [lo, hi]
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (pkey[mid] < (uint32_t)prev) lo = mid + 1;
            else hi = mid;
        }
        const uint32_t len = (uint32_t)(i - lo);
        const uint32_t k = atomicAdd(&hdr->n_long, 1u);
        if (k < kMaxLongTiles) long_tiles[k] = (uint32_t)prev;
        atomicAdd(&hdr->long_pairs, len);
        atomicMax(&hdr->max_long, len);
    }
}

constexpr int kRangeRun = 4;
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t *__restrict__ pkey, uint64_t cap,
                                                     uint2 *__restrict__ ranges, uint32_t total_tiles,
                                                     uint32_t *__restrict__ long_tiles,
                                                     uint32_t *__restrict__ tile_order, WsHeader *__restrict__ hdr) {
    if (blockIdx.x == 0 && threadIdx.x < kCostBuckets) tile_order[threadIdx.x] = 0u;  // filled by the forward
    const uint64_t i0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * kRangeRun;
    // a whole run inside the buffer is loaded while the pair count is still
    // in flight (entries past the count are ignored below)
    uint32_t k[kRangeRun];
    const bool whole = i0 + kRangeRun <= cap;
    if (whole) {
#pragma unroll
        for (int q = 0; q < kRangeRun / 4; ++q) {
            const uint4 kk = *reinterpret_cast<const uint4 *>(pkey + i0 + 4 * q);
            k[4 * q] = kk.x, k[4 * q + 1] = kk.y, k[4 * q + 2] = kk.z, k[4 * q + 3] = kk.w;
        }
    }
    const uint32_t prev_key = i0 > 0 && i0 <= cap ? pkey[i0 - 1] : 0u;
    const uint64_t m = hdr->overflow ? 0ull : (uint64_t)hdr->n_pairs;
    if (i0 > m) return;
    if (!whole || i0 + kRangeRun > m) {
#pragma unroll
        for (int j = 0; j < kRangeRun; ++j) k[j] = i0 + j < m ? pkey[i0 + j] : total_tiles;
    }
    // positions of this run where the tile changes (and i = m)
    uint32_t edges = 0;
    int64_t prev = i0 > 0 ? (int64_t)prev_key : -1;
#pragma unroll
    for (int j = 0; j < kRangeRun; ++j) {
        const int64_t t = i0 + j <= m ? (int64_t)k[j] : prev;  // (k[j] = total_tiles at i = m)
        edges |= (t != prev ? 1u : 0u) << j;
        prev = t;
    }
    while (edges) {
        const int j = __builtin_ctz(edges);
        edges &= edges - 1;
        // k[j] and the key before it, selected without indexing the array by j
        int64_t t = 0, before = i0 > 0 ? (int64_t)prev_key : -1;
#pragma unroll
        for (int q = 0; q < kRangeRun; ++q) {
            if (q == j) t = (int64_t)k[q];
            if (q + 1 == j) before = (int64_t)k[q];
        }
        tile_boundary(pkey, ranges, long_tiles, hdr, i0 + j, m, before, t);
    }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = value;
}

void launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st) {
    if (n == 0) return;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n);
}

__global__ void k_reset_header(WsHeader *h, uint32_t cap) {
    const uint32_t t = threadIdx.x;
    uint32_t *w = reinterpret_cast<uint32_t *>(h);
    if (t < sizeof(WsHeader) / 4) w[t] = 0u;
    __syncthreads();
    if (t == 0) h->pair_capacity = cap;
}

void launch_reset_header(WsHeader *h, uint32_t cap, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_header, dim3(1), dim3(64), 0, st, h, cap);
}

// Start of a backward pass: its work queue.
__global__ void k_reset_queue(WsHeader *h, int which) { h->queue[which] = 0u; }

void launch_reset_queue(WsHeader *h, int which, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(1), 0, st, h, which);
}

void launch_tile_ranges(const uint32_t *pkey, uint64_t cap, uint2 *ranges, uint32_t total_tiles,
                        uint32_t *long_tiles, uint32_t *tile_order, WsHeader *hdr, hipStream_t st) {
    if (total_tiles == 0) return;
    const uint64_t groups = cap / kRangeRun + 1;  // positions 0..cap, kRangeRun per thread
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, st, pkey, cap, ranges,
                       total_tiles, long_tiles, tile_order, hdr);
}

}  // namespace gsr
