// Monte-Carlo shuffles binned by genome region (Sec. 3.2) for gfx950.
//
// A shuffle's total is a sum over its placements of first - last (Algorithm 1),
// so the placements may be counted in any order.  This path orders them by
// region of the genome, so that the slice of B_S and B_E a region needs is
// read from HBM once per batch of shuffles into LDS and every search runs in
// LDS, with no per-search memory request:
//   regions  each chromosome is cut into cells of 2^S bp; a region is a run of
//            consecutive cells of one chromosome, cut where the merged count of
//            B_S and B_E keys since the chromosome's start crosses a multiple
//            of kRegionKeys, so regions follow B's density;
//   binning  per (shuffle, chromosome): the placements of the chromosome's
//            queries are made (the Philox stream of the other Monte-Carlo
//            kernels), counted per region, made again and written, with their
//            ends, in region order: one segment per (shuffle, region).  When
//            the chromosome has many regions, the second sweep goes in chunks
//            that are counting-sorted by region in LDS and written out in
//            region runs, so that a record line is filled in one go;
//   search   per region (or per share of a region's records when regions
//            are few): both slices are staged in LDS (B_S with kMargin keys
//            past the region's end, for ends that cross it), with a table of
//            slice ranks at equally spaced coordinates (a piecewise-constant
//            CDF of the slice), and each placement of each shuffle of the
//            batch is counted by two table lookups, each followed by a
//            bisection of the few keys of its bucket, all in LDS; the
//            per-shuffle sums are written out;
//   reduce   per shuffle: the sums over regions (and shares) are added to the
//            totals.
// A region whose slices exceed the LDS capacity (very dense or duplicated
// keys) is searched in HBM by the same bisections; an end past the staged
// margin continues by galloping search in HBM.  Both only cost speed.
#include <algorithm>

#include "bits_internal.hpp"

namespace bits {

namespace {

constexpr uint32_t kMaxCells = 8192;       // cells per chromosome (LDS table of the binning kernel)
constexpr uint32_t kMinShift = 10;         // cells are at least 1 kbp
constexpr uint32_t kRegionKeys = 8192;     // merged B_S + B_E keys per region (target)
constexpr uint32_t kMargin = 256;          // B_S keys staged past a region's end
constexpr uint32_t kSliceWords = 12800;    // LDS slice capacity of the search kernel (50 KiB)
// Bucket tables of the search kernel: a region's coordinate range is cut
// into at most kBuckets equal power-of-two buckets; word b of a table is the
// slice rank of bucket b's first coordinate (b = 0 .. buckets, the last one
// closing the final bucket).
constexpr uint32_t kBuckets = 1536;
constexpr uint32_t kBinThreads = 1024;
constexpr int ILP = 4;   // table entries each binning thread loads before it places them
// A reference with few regions (a small B) would leave most of the chip idle
// in the search; each region's records are then split over up to kMaxSplits
// workgroups, aiming at kSearchWorkgroups per pass.
constexpr uint32_t kSearchWorkgroups = 2048;
constexpr uint32_t kMaxSplits = 16;

// Per-chromosome geometry, passed by value: off[k] = first coordinate of
// chromosome k (off[n] = genome size), cb[k] = its first cell (cb[n] = cells).
struct BinGeom {
    uint32_t n_chrom, shift;
    uint32_t off[BITS_MAX_CHROM + 1];
    uint32_t cb[BITS_MAX_CHROM + 1];
};

// The first key of region r, and #{B_S < key_lo}, #{B_E < key_lo}.
struct RegionDesc {
    uint32_t key_lo, s_lo, e_lo, pad;
};

__device__ __forceinline__ uint32_t chrom_of_cell(const BinGeom& g, uint32_t c) {
    uint32_t lo = 0, hi = g.n_chrom;   // last k with cb[k] <= c (chromosomes without cells are skipped)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (g.cb[mid] <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// #{K[0..m) < x} (STRICT) or #{K[0..m) <= x}; the same number of steps for
// every lane at a given m.  (Staging the slices with a spare word per 32
// keys spreads the probes over more LDS banks, but its two extra VALU
// operations per probe cost more than the conflicts it saves.)
template <bool STRICT>
__device__ __forceinline__ uint32_t rank_in(const uint32_t* K, uint32_t m, uint32_t x) {
    if (m == 0) return 0;
    uint32_t base = 0, len = m;
    while (len > 1) {
        const uint32_t half = len >> 1;
        const uint32_t k = K[base + half];
        if (STRICT ? (k < x) : (k <= x)) base += half;
        len -= half;
    }
    const uint32_t k = K[base];
    return base + (STRICT ? (k < x) : (k <= x));
}

// rank_in for the few keys of one bucket: no early exit for m = 0 (K[0] is
// then still read, at most one word past the slices, and ignored), so that
// the lanes of a wave do not branch around each other.
template <bool STRICT>
__device__ __forceinline__ uint32_t rank_bucket(const uint32_t* K, uint32_t m, uint32_t x) {
    uint32_t base = 0, len = m;
    while (len > 1) {
        const uint32_t half = len >> 1;
        const uint32_t k = K[base + half];
        if (STRICT ? (k < x) : (k <= x)) base += half;
        len -= half;
    }
    const uint32_t k = K[base];
    return base + ((m != 0u) & (STRICT ? (k < x) : (k <= x)));
}

// #{bs <= x} over the whole array, given that bs[j - 1] <= x (j >= 1) or j = 0.
__device__ uint32_t gallop_le(const uint32_t* __restrict__ bs, uint32_t n, uint32_t j, uint32_t x) {
    uint32_t lo = j, hi = n;
    uint64_t step = 1;
    while (true) {
        const uint64_t probe = (uint64_t)lo + step - 1;
        if (probe >= n) break;
        if (bs[probe] <= x) {
            lo = (uint32_t)probe + 1u;
            step <<= 1;
        } else {
            hi = (uint32_t)probe;
            break;
        }
    }
    return lo + rank_in<false>(bs + lo, hi - lo, x);
}

// Exclusive scan of h[0..m) in place (m <= per * blockDim with per <= 8);
// returns the total.  wsum holds blockDim / 64 words.
__device__ uint32_t block_scan_u32(uint32_t* h, uint32_t m, uint32_t* wsum) {
    const uint32_t per = (m + blockDim.x - 1) / blockDim.x;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t mine = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (b0 + k < m) mine += h[b0 + k];
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t x = mine;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t k = 0; k < blockDim.x / kWave; ++k) {
        if (k < w) pre += wsum[k];
        tot += wsum[k];
    }
    pre += x - mine;
    for (uint32_t k = 0; k < per; ++k) {
        if (b0 + k < m) {
            const uint32_t v = h[b0 + k];
            h[b0 + k] = pre;
            pre += v;
        }
    }
    __syncthreads();
    return tot;
}

// Ranks of every cell's first coordinate in B_S and B_E.
__global__ void __launch_bounds__(256) k_bin_cells(BinGeom g, const uint32_t* __restrict__ bs,
                                                   const uint32_t* __restrict__ be, uint32_t n,
                                                   uint32_t* __restrict__ rs, uint32_t* __restrict__ re) {
    const uint32_t ncells = g.cb[g.n_chrom];
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x) {
        const uint32_t k = chrom_of_cell(g, c);
        const uint32_t lo = g.off[k] + ((c - g.cb[k]) << g.shift);
        rs[c] = rank_in<true>(bs, n, lo);
        re[c] = rank_in<true>(be, n, lo);
    }
}

// flag[c] = 1 where a region starts: the first cell of a chromosome, or the
// merged count since the chromosome's start enters a new multiple of kRegionKeys.
__global__ void __launch_bounds__(256) k_bin_flags(BinGeom g, const uint32_t* __restrict__ rs,
                                                   const uint32_t* __restrict__ re, uint32_t* __restrict__ flag) {
    const uint32_t ncells = g.cb[g.n_chrom];
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x) {
        const uint32_t k = chrom_of_cell(g, c), c0 = g.cb[k];
        uint32_t f = 1u;
        if (c != c0) {
            const uint64_t base = (uint64_t)rs[c0] + re[c0];
            const uint64_t p = (uint64_t)rs[c] + re[c] - base, q = (uint64_t)rs[c - 1] + re[c - 1] - base;
            f = (p / kRegionKeys) != (q / kRegionKeys) ? 1u : 0u;
        }
        flag[c] = f;
    }
}

// cell -> region (offsets = exclusive scan of the flags), region descriptors,
// and the sentinel after the last region: {genome size, n, n}.
__global__ void __launch_bounds__(256) k_bin_regions(BinGeom g, const uint32_t* __restrict__ rs,
                                                     const uint32_t* __restrict__ re,
                                                     const uint32_t* __restrict__ flag,
                                                     const uint64_t* __restrict__ offsets, uint32_t n,
                                                     uint32_t nreg_max, uint32_t* __restrict__ cell_region,
                                                     RegionDesc* __restrict__ desc, uint32_t* status) {
    const uint32_t ncells = g.cb[g.n_chrom];
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncells; c += gridDim.x * blockDim.x) {
        uint32_t rid = (uint32_t)(offsets[c + 1] - 1u);
        if (rid >= nreg_max) {          // cannot happen (nreg_max bounds the count); never index past it
            atomicOr(status, BITS_FLAG_CHROM);
            rid = nreg_max - 1u;
        }
        cell_region[c] = rid;
        if (flag[c]) {
            const uint32_t k = chrom_of_cell(g, c);
            desc[rid] = RegionDesc{g.off[k] + ((c - g.cb[k]) << g.shift), rs[c], re[c], 0u};
        }
        if (c == ncells - 1) desc[rid + 1] = RegionDesc{g.off[g.n_chrom], n, n, 0u};   // desc has nreg_max + 1
    }
}

// The per-query table the binning kernel reads: {input index, length}, the
// length 0 for a query outside its chromosome (span 0).  A query's legal
// starts follow from its chromosome's length: span = len_k - L + 1.
__global__ void __launch_bounds__(256) k_bin_pack(const uint32_t* __restrict__ span, const uint32_t* __restrict__ len,
                                                  const uint32_t* __restrict__ idx, uint64_t na,
                                                  uint2* __restrict__ packed) {
    for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; p < na; p += (uint64_t)gridDim.x * blockDim.x)
        packed[p] = make_uint2(idx[p], span[p] ? len[p] : 0u);
}

// Inclusive prefix sum over the 64 lanes of a wave, moving data between lanes
// with DPP only (no LDS instruction, so it does not queue behind the
// bisections): four row_shr steps (1, 2, 4, 8) build the prefix inside each
// row of 16 lanes, then row_bcast:15 adds row 0's total to row 1 and row 2's
// to row 3, and row_bcast:31 adds the total of rows 0-1 to rows 2 and 3.
// Lanes whose source lies outside the row, and rows the row mask leaves out,
// receive 0 (the `old` operand), so every step is a plain add.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_in0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void scan_step(uint32_t& x) {
    x += dpp_in0<CTRL, ROWS>(x);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void scan_step(uint64_t& x) {
    const uint32_t lo = dpp_in0<CTRL, ROWS>((uint32_t)x), hi = dpp_in0<CTRL, ROWS>((uint32_t)(x >> 32));
    x += ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    scan_step<0x111, 0xF>(x);   // row_shr:1
    scan_step<0x112, 0xF>(x);   // row_shr:2
    scan_step<0x114, 0xF>(x);   // row_shr:4
    scan_step<0x118, 0xF>(x);   // row_shr:8
    scan_step<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    scan_step<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// Staged binning (second sweep): chromosomes with kStageMinRegions..kStageRegions
// regions; kStageRecs records per chunk, so that the workgroup's LDS (about 76 KB)
// still lets two workgroups share a CU.
constexpr uint32_t kStageRegions = 2048;
constexpr uint32_t kStageMinRegions = 128;
constexpr uint32_t kStageRecs = 5632;      // 44 KB
constexpr int kStagePer = (kStageRecs + kBinThreads - 1) / kBinThreads;
static_assert(kStageRegions <= 2 * kBinThreads, "one thread owns two regions' chunk counters");
static_assert(kStageRecs < (1u << 16), "chunk counts and offsets are 16-bit");
static_assert(kMaxCells <= (1u << 16), "cell-to-region table entries are 16-bit");

// Entry j of an array of 16-bit values packed two per word.
__device__ __forceinline__ uint32_t half16(const uint32_t* w, uint32_t j) {
    return (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

// Binning of shuffles [sb, sb + nb): workgroup (k, s) makes the placements of
// chromosome k's queries (table positions [cursor[k] - hist[k], cursor[k]))
// in shuffle sb + s, counts them per region, writes the segment table of
// (s, every region of k), and writes the records {start, end} in region
// order to recs[s * na + table position range], either one by one (few
// regions, or more than kStageRegions) or chunk by chunk through LDS.  A
// group that fits one chunk is placed only once: its chunk's region counts
// are the segment table and the chunk is its final layout.
// (8 waves per SIMD: two workgroups per CU, at most 64 VGPRs.)
__global__ void __launch_bounds__(kBinThreads, 8) k_bin_place(
    BinGeom g, const uint2* __restrict__ packed, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ cursor,
    uint64_t na, uint64_t seed, uint64_t sb, uint32_t nb, const uint32_t* __restrict__ cell_region,
    const uint64_t* __restrict__ offsets, uint32_t nreg_max, uint32_t* __restrict__ seg_start,
    uint32_t* __restrict__ seg_cnt, uint2* __restrict__ recs) {
    __shared__ uint16_t cr[kMaxCells];
    __shared__ uint32_t hs[kStageRegions];          // segment cursors (staged path)
    __shared__ uint32_t cc[kStageRegions / 2];      // chunk counts, 16 bits each
    __shared__ uint32_t co[kStageRegions / 2];      // chunk offsets (exclusive), 16 bits each
    __shared__ uint2 stage[kStageRecs];             // the chunk's records in region order; h of the direct path
    __shared__ uint32_t wsum[kBinThreads / kWave];
    __shared__ uint32_t staged_total;
    const uint32_t k = blockIdx.x / nb, s = blockIdx.x - k * nb;
    const uint32_t c0 = g.cb[k], nc = g.cb[k + 1] - c0;
    if (nc == 0) return;
    const uint32_t nreg = (uint32_t)offsets[g.cb[g.n_chrom]];
    const uint32_t rb = cell_region[c0];
    const uint32_t rl = (k + 1 < g.n_chrom && g.cb[k + 1] < g.cb[g.n_chrom]) ? cell_region[g.cb[k + 1]] : nreg;
    const uint32_t nr = rl > rb ? min(min(rl - rb, nc), nreg_max - rb) : 0u;
    // staging pays when a chromosome spreads its records over many regions (many open
    // record lines); with few regions the direct writes already merge in L2
    const bool staged = nr >= kStageMinRegions && nr <= kStageRegions;
    uint32_t* h = staged ? hs : reinterpret_cast<uint32_t*>(stage);   // kMaxCells words fit the stage buffer
    for (uint32_t j = threadIdx.x; j < nc; j += blockDim.x) cr[j] = (uint16_t)(cell_region[c0 + j] - rb);
    for (uint32_t j = threadIdx.x; j < nr; j += blockDim.x) h[j] = 0u;
    __syncthreads();
    const uint32_t g1 = cursor[k], g0 = g1 - hist[k];
    const uint32_t ok = g.off[k], sh = g.shift, clen = g.off[k + 1] - g.off[k];
    const uint64_t gs = (sb + s) * na;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (g1 - g0 <= kStageRecs && nr <= kStageRegions) {
        // The group fits one LDS chunk: every entry is placed once and ranked in its
        // region, the counts give the segment table directly, and the chunk in region
        // order is the group's final layout (written out sequentially).
        const uint32_t nw2 = (nr + 1) >> 1;
        const bool owner = threadIdx.x < nw2;
        if (owner) cc[threadIdx.x] = 0u;
        __syncthreads();
        uint32_t st_[kStagePer], len_[kStagePer], key_[kStagePer];   // key = lr << 16 | rank, or ~0
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            const uint32_t p = g0 + threadIdx.x + (uint32_t)u * blockDim.x;
            const uint2 q = p < g1 ? packed[p] : make_uint2(0u, 0u);
            key_[u] = 0xFFFFFFFFu;
            st_[u] = 0u;
            len_[u] = q.y;
            if (!q.y) continue;
            const uint32_t st = mc_place(gs + q.x, k0, k1, ok, clen - q.y + 1u);
            const uint32_t lr = cr[(st - ok) >> sh];
            if (lr >= nr) continue;
            const uint32_t sft = 16u * (lr & 1u);
            const uint32_t old = atomicAdd(&cc[lr >> 1], 1u << sft);
            st_[u] = st;
            key_[u] = (lr << 16) | ((old >> sft) & 0xFFFFu);
        }
        __syncthreads();
        {
            const uint32_t wv = owner ? cc[threadIdx.x] : 0u;
            const uint32_t a0 = wv & 0xFFFFu, a1 = wv >> 16, tsum = a0 + a1;
            const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
            const uint32_t x = wave_inclusive_scan<uint32_t>(tsum);
            if (lane == kWave - 1) wsum[w] = x;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
            for (uint32_t j = 0; j < kBinThreads / kWave; ++j) {
                if (j < w) pre += wsum[j];
                tot += wsum[j];
            }
            pre += x - tsum;
            if (owner) {
                uint32_t* ss = seg_start + (uint64_t)s * nreg_max + rb;
                uint32_t* sc = seg_cnt + (uint64_t)s * nreg_max + rb;
                const uint32_t r0 = 2u * threadIdx.x, lo1 = pre + a0;
                co[threadIdx.x] = pre | (lo1 << 16);
                ss[r0] = g0 + pre;
                sc[r0] = a0;
                if (r0 + 1u < nr) {
                    ss[r0 + 1u] = g0 + lo1;
                    sc[r0 + 1u] = a1;
                }
            }
            if (threadIdx.x == 0) staged_total = tot;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            if (key_[u] == 0xFFFFFFFFu) continue;
            const uint32_t lr = key_[u] >> 16;
            stage[half16(co, lr) + (key_[u] & 0xFFFFu)] = make_uint2(st_[u], st_[u] + (len_[u] - 1u));
        }
        __syncthreads();
        uint2* out = recs + (uint64_t)s * na + g0;
        const uint32_t tot = staged_total;
        for (uint32_t j = threadIdx.x; j < tot; j += blockDim.x) out[j] = stage[j];
        return;
    }
    for (uint32_t p0 = g0 + threadIdx.x; p0 < g1; p0 += ILP * blockDim.x) {
        uint2 q[ILP];
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            const uint32_t p = p0 + u * blockDim.x;
            q[u] = p < g1 ? packed[p] : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < ILP; ++u) {
            if (!q[u].y) continue;
            const uint32_t st = mc_place(gs + q[u].x, k0, k1, ok, clen - q[u].y + 1u);
            const uint32_t lr = cr[(st - ok) >> sh];
            if (lr < nr) atomicAdd(&h[lr], 1u);
        }
    }
    __syncthreads();
    uint32_t* ss = seg_start + (uint64_t)s * nreg_max + rb;
    uint32_t* sc = seg_cnt + (uint64_t)s * nreg_max + rb;
    for (uint32_t j = threadIdx.x; j < nr; j += blockDim.x) sc[j] = h[j];
    __syncthreads();
    block_scan_u32(h, nr, wsum);
    for (uint32_t j = threadIdx.x; j < nr; j += blockDim.x) ss[j] = g0 + h[j];
    __syncthreads();
    uint2* out = recs + (uint64_t)s * na;
    if (!staged) {
        for (uint32_t p0 = g0 + threadIdx.x; p0 < g1; p0 += ILP * blockDim.x) {
            uint2 q[ILP];
#pragma unroll
            for (int u = 0; u < ILP; ++u) {
                const uint32_t p = p0 + u * blockDim.x;
                q[u] = p < g1 ? packed[p] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int u = 0; u < ILP; ++u) {
                if (!q[u].y) continue;
                const uint32_t st = mc_place(gs + q[u].x, k0, k1, ok, clen - q[u].y + 1u);
                const uint32_t lr = cr[(st - ok) >> sh];
                if (lr >= nr) continue;
                const uint32_t at = atomicAdd(&h[lr], 1u);
                out[g0 + at] = make_uint2(st, st + (q[u].y - 1u));
            }
        }
        return;
    }
    // staged: chunks of kStageRecs table entries are placed, counting-sorted by region in
    // LDS, and written out in region runs.  Thread t < nw2 owns regions 2t and 2t + 1
    // (counter word t) for the whole loop.  During a chunk, hs[r] holds region r's cursor
    // minus the offset of r's run in the chunk, so the chunk's record j goes to
    // g0 + hs[r] + j; the next chunk's scan adds back the end of that run (kept in the
    // owner's registers) to get the cursor again.  Four barriers a chunk: the next
    // chunk's ranking touches only the counters, so it may overlap this write-out.
    const uint32_t nw2 = (nr + 1) >> 1;
    const bool owner = threadIdx.x < nw2;
    if (owner) cc[threadIdx.x] = 0u;
    uint32_t end0 = 0u, end1 = 0u;   // the owner's run ends in the previous chunk
    __syncthreads();
    for (uint32_t cb = g0; cb < g1; cb += kStageRecs) {
        const uint32_t ce = min(g1, cb + kStageRecs);
        uint32_t st_[kStagePer], len_[kStagePer], key_[kStagePer];   // key = lr << 16 | rank, or ~0
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            const uint32_t p = cb + threadIdx.x + (uint32_t)u * blockDim.x;
            const uint2 q = p < ce ? packed[p] : make_uint2(0u, 0u);
            key_[u] = 0xFFFFFFFFu;
            st_[u] = 0u;
            len_[u] = q.y;
            if (!q.y) continue;
            const uint32_t st = mc_place(gs + q.x, k0, k1, ok, clen - q.y + 1u);
            const uint32_t lr = cr[(st - ok) >> sh];
            if (lr >= nr) continue;
            const uint32_t sft = 16u * (lr & 1u);
            const uint32_t old = atomicAdd(&cc[lr >> 1], 1u << sft);
            st_[u] = st;
            key_[u] = (lr << 16) | ((old >> sft) & 0xFFFFu);
        }
        __syncthreads();   // counts complete; the previous chunk is written out
        // exclusive offsets of the chunk's region counts (two per word) into co, and the
        // owners' cursors turned into this chunk's deltas
        {
            const uint32_t wv = owner ? cc[threadIdx.x] : 0u;
            if (owner) cc[threadIdx.x] = 0u;   // ready for the next chunk
            const uint32_t a0 = wv & 0xFFFFu, a1 = wv >> 16, tsum = a0 + a1;
            const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
            const uint32_t x = wave_inclusive_scan<uint32_t>(tsum);
            if (lane == kWave - 1) wsum[w] = x;
            __syncthreads();
            uint32_t pre = 0, tot = 0;
            for (uint32_t j = 0; j < kBinThreads / kWave; ++j) {
                if (j < w) pre += wsum[j];
                tot += wsum[j];
            }
            pre += x - tsum;
            if (owner) {
                const uint32_t r0 = 2u * threadIdx.x, lo1 = pre + a0;
                co[threadIdx.x] = pre | (lo1 << 16);
                hs[r0] = hs[r0] + end0 - pre;
                end0 = lo1;
                if (r0 + 1u < nr) {
                    hs[r0 + 1u] = hs[r0 + 1u] + end1 - lo1;
                    end1 = lo1 + a1;
                }
            }
            if (threadIdx.x == 0) staged_total = tot;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kStagePer; ++u) {
            if (key_[u] == 0xFFFFFFFFu) continue;
            const uint32_t lr = key_[u] >> 16;
            stage[half16(co, lr) + (key_[u] & 0xFFFFu)] = make_uint2(st_[u], st_[u] + (len_[u] - 1u));
        }
        __syncthreads();
        const uint32_t tot = staged_total;
        for (uint32_t j = threadIdx.x; j < tot; j += blockDim.x) {
            const uint2 rec = stage[j];
            const uint32_t lr = cr[(rec.x - ok) >> sh];
            out[g0 + hs[lr] + j] = rec;
        }
    }
}

// Wave-level segmented sum: lanes carry (key, value) with the keys of the
// valid lanes non-decreasing in lane order; each run of equal keys adds its
// sum to acc[key] with at most two LDS atomics (the run's inclusive prefix at
// its last lane, minus the prefix before its first lane, which is that lane's
// inclusive prefix minus its own value).  T = uint32_t only when 64 values
// cannot reach 2^32.
template <typename T>
__device__ __forceinline__ void wave_segment_add(uint32_t key, T v, bool valid, unsigned long long* acc) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const T x = wave_inclusive_scan<T>(v);
    // the neighbours' keys by whole-wave DPP shifts (wave_shr:1, wave_shl:1); lane 0's kp and
    // lane 63's kn are never used
    const uint32_t kp = dpp_in0<0x138, 0xF>(key), kn = dpp_in0<0x130, 0xF>(key);
    if (!valid) return;
    if (lane == kWave - 1 || kn != key) atomicAdd(&acc[key], (unsigned long long)x);
    if (lane != 0 && kp != key) atomicAdd(&acc[key], 0ull - (unsigned long long)(x - v));
}

// R[b] = #{K[0..m) < key_lo + b 2^sh} for b = 0 .. nb, K sorted with
// K[0] >= key_lo.  With F(x) = (x - key_lo) >> sh, the largest b whose
// coordinate is <= x, key j writes j to the buckets in (F(K[j - 1]), F(K[j])]
// and a final step j = m fills the rest up to nb: every bucket is written
// once, in one pass over the keys.
__device__ void bucket_ranks(const uint32_t* K, uint32_t m, uint32_t key_lo, uint32_t sh, uint32_t nb, uint32_t* R) {
    for (uint32_t j = threadIdx.x; j <= m; j += blockDim.x) {
        const uint32_t lo = j == 0 ? 0u : min((K[j - 1] - key_lo) >> sh, nb) + 1u;
        const uint32_t hi = j == m ? nb : min((K[j] - key_lo) >> sh, nb);
        for (uint32_t b = lo; b <= hi; ++b) R[b] = j;
    }
}

// The placements of one region, counted against slices S = B_S[s_lo, s_lo + ns)
// and E = B_E[e_lo, e_lo + ne) (in LDS, or in HBM for an oversize region):
// the workgroup's share [q0, q1) of the region's records.  Each wave takes a
// contiguous range of it, 64 records per step; records are grouped by
// shuffle (pre[s] = first record of shuffle s), so a wave tracks its shuffle
// by a forward scan and adds per-shuffle sums with wave_segment_add.
// Bucket geometry of a region [key_lo, key_hi): bucket of x = (x - key_lo) >> sh.
// On the LDS path, TS / TE hold word b = rank(v_b), v_b = key_lo + b 2^sh,
// the ranks being #{S < v} and #{E < v} in the slices; bucket b's keys are
// ranks [TS[b], TS[b + 1]).
struct Buckets {
    const uint32_t* TS;
    const uint32_t* TE;
    uint32_t key_lo, key_hi, sh;
};

template <bool LDS, typename T>
__device__ __forceinline__ void bin_count_region(const uint32_t* S, uint32_t ns, const uint32_t* E, uint32_t ne,
                                                 const uint32_t* __restrict__ bs, uint32_t n, uint32_t s_lo,
                                                 uint32_t e_lo, const Buckets& bk, const uint2* __restrict__ recs,
                                                 const uint32_t* pre, const uint32_t* base, uint32_t nb,
                                                 uint64_t q0, uint64_t q1, unsigned long long* acc) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    const uint64_t steps = (q1 - q0 + kWave - 1) / kWave, per = (steps + nw - 1) / nw;
    const uint64_t p0 = q0 + (uint64_t)wv * per * kWave, p1 = min(q1, p0 + per * kWave);
    if (p0 >= p1) return;
    // record p of the pass (p < pre[nb] < 2^32) is recs[base[s] + p], s its shuffle
    const uint32_t s_end = s_lo + ns;
    // shuffle of the wave's first record: the last s with pre[s] <= p0
    uint32_t sw = 0, hi = nb;
    while (hi - sw > 1) {
        const uint32_t mid = (sw + hi) >> 1;
        if (pre[mid] <= p0) sw = mid; else hi = mid;
    }
    // Software pipeline: the record of the next step is loaded before this
    // step's searches, so a wave has two record loads in flight.  A lane's
    // shuffle only moves forward, as its record index grows by 64 a step.
    uint32_t sl = sw;
    uint2 rn = make_uint2(0u, 0u);
    if (p0 + lane < p1) {
        const uint32_t p = (uint32_t)p0 + lane;
        while (pre[sl + 1] <= p) ++sl;   // ends at sl < nb: p < pre[nb]
        rn = recs[base[sl] + p];
    }
    for (uint64_t b = p0; b < p1; b += kWave) {
        const bool valid = b + lane < p1;
        const uint32_t slc = sl;
        const uint2 r = rn;
        if (b + kWave + lane < p1) {
            const uint32_t p = (uint32_t)(b + kWave) + lane;
            while (pre[sl + 1] <= p) ++sl;
            rn = recs[base[sl] + p];
        }
        T v = 0;
        if (valid) {
            uint32_t first, last;
            if (LDS && r.y < bk.key_hi) {
                // every key <= r.y is below key_hi, so inside the slice: the bucket's keys decide
                const uint32_t b = (r.y - bk.key_lo) >> bk.sh, lo = bk.TS[b];
                first = s_lo + lo + rank_bucket<false>(S + lo, bk.TS[b + 1] - lo, r.y);
            } else if (r.y == 0xFFFFFFFFu) {
                first = n;
            } else {
                const uint32_t c = rank_in<false>(S, ns, r.y);
                first = (c == ns && s_end < n) ? gallop_le(bs, n, s_end, r.y) : s_lo + c;
            }
            if (LDS) {   // key_lo <= r.x < key_hi: the start lies in the region
                const uint32_t b = (r.x - bk.key_lo) >> bk.sh, lo = bk.TE[b];
                last = e_lo + lo + rank_bucket<true>(E + lo, bk.TE[b + 1] - lo, r.x);
            } else {
                last = e_lo + rank_in<true>(E, ne, r.x);
            }
            v = (T)(first - last);
        }
        wave_segment_add<T>(valid ? slc : 0xFFFFFFFFu, v, valid, acc);
    }
}

// `splits` workgroups per region r < nreg (nreg on the device; workgroups past
// it return): stage the slices, count the workgroup's share of the placements
// of the batch that start in the region, write partial[(r * splits + part) * nb + s].
// SPLIT = false is the one-workgroup-per-region form (splits = 1).
template <bool SPLIT>
__global__ void __launch_bounds__(kBinThreads) k_bin_search(
    const uint32_t* __restrict__ bs, const uint32_t* __restrict__ be, uint32_t n,
    const RegionDesc* __restrict__ desc, const uint64_t* __restrict__ nreg_p, const uint32_t* __restrict__ seg_start,
    const uint32_t* __restrict__ seg_cnt, uint32_t nreg_max, uint32_t nb, const uint2* __restrict__ recs,
    uint64_t na, uint32_t splits, unsigned long long* __restrict__ partial) {
    __shared__ uint32_t slice[kSliceWords + 1];   // + 1: the word an empty last bucket reads
    __shared__ uint32_t tabs[2 * (kBuckets + 1)];
    __shared__ uint32_t pre[BITS_MC_BIN_MAX_BATCH + 1];
    __shared__ uint32_t base[BITS_MC_BIN_MAX_BATCH];
    __shared__ unsigned long long acc[BITS_MC_BIN_MAX_BATCH];
    __shared__ uint32_t w32[kBinThreads / kWave];
    const uint32_t r = SPLIT ? blockIdx.x / splits : blockIdx.x, part = SPLIT ? blockIdx.x - r * splits : 0u;
    if (r >= *nreg_p) return;
    const RegionDesc d0 = desc[r], d1 = desc[r + 1];
    const uint32_t s_lo = d0.s_lo, e_lo = d0.e_lo;
    const uint32_t s_end = (uint32_t)min((uint64_t)d1.s_lo + kMargin, (uint64_t)n);
    const uint32_t ns = s_end - s_lo, ne = d1.e_lo - e_lo;
    // per-shuffle prefix of the segment lengths, and each shuffle's record base: record p of
    // the pass (in shuffle s) is recs[s * na + seg_start + (p - pre[s])]; nb * na < 2^32
    uint32_t cnt = 0, sst = 0;
    if (threadIdx.x < nb) {
        sst = seg_start[(uint64_t)threadIdx.x * nreg_max + r];
        cnt = seg_cnt[(uint64_t)threadIdx.x * nreg_max + r];
        acc[threadIdx.x] = 0ull;
    }
    {
        const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
        uint32_t x = cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= (uint32_t)o) x += y;
        }
        if (lane == kWave - 1) w32[w] = x;
        __syncthreads();
        uint32_t before = 0;
        for (uint32_t j = 0; j < w; ++j) before += w32[j];
        const uint32_t pr = before + x - cnt;
        if (threadIdx.x < nb) {
            pre[threadIdx.x] = pr;
            base[threadIdx.x] = threadIdx.x * (uint32_t)na + sst - pr;
        }
        if (threadIdx.x == nb - 1) pre[nb] = before + x;
    }
    const uint32_t eo = ns;   // E's first word
    const bool in_lds = (uint64_t)ns + ne <= kSliceWords;
    // buckets: the least power-of-two width that cuts [key_lo, key_hi) into at most kBuckets
    Buckets bk{tabs, tabs + kBuckets + 1, d0.key_lo, d1.key_lo, 0u};
    const uint32_t span = bk.key_hi - bk.key_lo;   // > 0: a region holds at least one cell
    while (((span - 1u) >> bk.sh) >= kBuckets) ++bk.sh;
    const uint32_t nbk = ((span - 1u) >> bk.sh) + 1u;
    if (in_lds) {
        for (uint32_t j = threadIdx.x; j < ns; j += blockDim.x) slice[j] = bs[s_lo + j];
        for (uint32_t j = threadIdx.x; j < ne; j += blockDim.x) slice[eo + j] = be[e_lo + j];
        __syncthreads();
        bucket_ranks(slice, ns, bk.key_lo, bk.sh, nbk, tabs);
        bucket_ranks(slice + eo, ne, bk.key_lo, bk.sh, nbk, tabs + kBuckets + 1);
    }
    __syncthreads();
    // this workgroup's share of the region's records
    const uint64_t total = pre[nb];
    const uint64_t q0 = SPLIT ? total * part / splits : 0ull, q1 = SPLIT ? total * (part + 1) / splits : total;
    // per-step sums fit 32 bits when 64 counts of at most n cannot reach 2^32
    const bool narrow = n < (1u << 26);
    if (in_lds && narrow)
        bin_count_region<true, uint32_t>(slice, ns, slice + eo, ne, bs, n, s_lo, e_lo, bk, recs, pre, base, nb,
                                         q0, q1, acc);
    else if (in_lds)
        bin_count_region<true, uint64_t>(slice, ns, slice + eo, ne, bs, n, s_lo, e_lo, bk, recs, pre, base, nb,
                                         q0, q1, acc);
    else if (narrow)
        bin_count_region<false, uint32_t>(bs + s_lo, ns, be + e_lo, ne, bs, n, s_lo, e_lo, bk, recs, pre, base,
                                          nb, q0, q1, acc);
    else
        bin_count_region<false, uint64_t>(bs + s_lo, ns, be + e_lo, ne, bs, n, s_lo, e_lo, bk, recs, pre, base,
                                          nb, q0, q1, acc);
    __syncthreads();
    if (threadIdx.x < nb)
        partial[(SPLIT ? (uint64_t)r * splits + part : (uint64_t)r) * nb + threadIdx.x] = acc[threadIdx.x];
}

// totals[s] += sum over the nreg * splits region shares j of partial[j * nb + s];
// blockIdx.y takes every gridDim.y-th share.
__global__ void __launch_bounds__(256) k_bin_reduce(const unsigned long long* __restrict__ partial,
                                                    const uint64_t* __restrict__ nreg_p, uint32_t splits,
                                                    uint32_t nb, unsigned long long* __restrict__ totals) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nb) return;
    const uint64_t shares = *nreg_p * splits;
    unsigned long long v = 0ull;
    for (uint64_t j = blockIdx.y; j < shares; j += gridDim.y) v += partial[j * nb + s];
    if (v) atomicAdd(totals + s, v);
}

// Cell shift and per-chromosome cell bases of a genome; false if no shift
// keeps every chromosome within kMaxCells cells (impossible below 2^32 bp).
bool bin_geometry(const uint32_t* chrom_len, uint32_t n_chrom, BinGeom* g) {
    uint64_t maxlen = 0, acc = 0;
    for (uint32_t k = 0; k < n_chrom; ++k) maxlen = chrom_len[k] > maxlen ? chrom_len[k] : maxlen;
    uint32_t sh = kMinShift;
    while (sh < 32 && ((maxlen + (1ull << sh) - 1) >> sh) > kMaxCells) ++sh;
    if (sh >= 32) return false;
    g->n_chrom = n_chrom;
    g->shift = sh;
    uint64_t cells = 0;
    for (uint32_t k = 0; k < n_chrom; ++k) {
        g->off[k] = (uint32_t)acc;
        g->cb[k] = (uint32_t)cells;
        acc += chrom_len[k];
        cells += ((uint64_t)chrom_len[k] + (1ull << sh) - 1) >> sh;
    }
    if (acc > 0xFFFFFFFFull || cells > 0xFFFFFFFFull) return false;
    for (uint32_t k = n_chrom; k <= BITS_MAX_CHROM; ++k) {
        g->off[k] = (uint32_t)acc;
        g->cb[k] = (uint32_t)cells;
    }
    return true;
}

}  // namespace

bool bin_layout(const uint32_t* chrom_len, uint32_t n_chrom, uint64_t n, BinLayout* L) {
    BinGeom g;
    if (!bin_geometry(chrom_len, n_chrom, &g)) return false;
    L->ncells = g.cb[n_chrom];
    uint64_t with_cells = 0;
    for (uint32_t k = 0; k < n_chrom; ++k) with_cells += g.cb[k + 1] > g.cb[k];
    const uint64_t bound = with_cells + (2 * n) / kRegionKeys;
    L->nreg_max = L->ncells < bound ? L->ncells : bound;
    const uint64_t sp = L->nreg_max ? (kSearchWorkgroups + L->nreg_max - 1) / L->nreg_max : 1;
    L->splits = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(sp, 1), kMaxSplits);
    return true;
}

hipError_t launch_bin_pack(const McTable& tab, uint64_t na, const BinWs& w, hipStream_t s) {
    if (!na) return hipSuccess;
    const uint32_t gr = (uint32_t)std::min<uint64_t>((na + 255) / 256, 8192);
    hipLaunchKernelGGL(k_bin_pack, dim3(gr), dim3(256), 0, s, tab.span, tab.len, tab.idx, na,
                       reinterpret_cast<uint2*>(w.packed));
    return hipGetLastError();
}

hipError_t launch_bin_regions(const uint32_t* chrom_len, uint32_t n_chrom, const uint32_t* bs, const uint32_t* be,
                              uint32_t n, const BinWs& w, uint32_t* status, hipStream_t s) {
    BinGeom g;
    if (!bin_geometry(chrom_len, n_chrom, &g)) return hipErrorInvalidValue;
    const uint32_t ncells = g.cb[n_chrom];
    if (!ncells) return hipErrorInvalidValue;
    const uint32_t gr = (uint32_t)std::min<uint64_t>((ncells + 255) / 256, 4096);
    hipLaunchKernelGGL(k_bin_cells, dim3(gr), dim3(256), 0, s, g, bs, be, n, w.rs, w.re);
    hipLaunchKernelGGL(k_bin_flags, dim3(gr), dim3(256), 0, s, g, w.rs, w.re, w.flag);
    hipError_t e = launch_scan_counts(w.flag, ncells, w.offsets, w.scan_tiles, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_regions, dim3(gr), dim3(256), 0, s, g, w.rs, w.re, w.flag, w.offsets, n, w.nreg_max,
                       w.cell_region, reinterpret_cast<RegionDesc*>(w.desc), status);
    return hipGetLastError();
}

hipError_t launch_bin_batch(const uint32_t* chrom_len, uint32_t n_chrom, const McTable& tab, uint64_t na,
                            const uint32_t* bs, const uint32_t* be, uint32_t n, uint64_t seed, uint64_t sb,
                            uint32_t nb, const BinWs& w, unsigned long long* totals, hipStream_t s,
                            hipEvent_t* ev) {
    BinGeom g;
    if (!bin_geometry(chrom_len, n_chrom, &g)) return hipErrorInvalidValue;
    if (nb == 0 || nb > BITS_MC_BIN_MAX_BATCH) return hipErrorInvalidValue;
    const uint32_t ncells = g.cb[n_chrom];
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_place, dim3(n_chrom * nb), dim3(kBinThreads), 0, s, g,
                       reinterpret_cast<const uint2*>(w.packed), tab.hist, tab.cursor, na, seed, sb, nb,
                       w.cell_region, w.offsets, w.nreg_max, w.seg_start, w.seg_cnt, reinterpret_cast<uint2*>(w.recs));
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (w.splits > 1)
        hipLaunchKernelGGL(k_bin_search<true>, dim3(w.nreg_max * w.splits), dim3(kBinThreads), 0, s, bs, be, n,
                           reinterpret_cast<const RegionDesc*>(w.desc), w.offsets + ncells, w.seg_start, w.seg_cnt,
                           w.nreg_max, nb, reinterpret_cast<const uint2*>(w.recs), na, w.splits, w.partial);
    else
        hipLaunchKernelGGL(k_bin_search<false>, dim3(w.nreg_max), dim3(kBinThreads), 0, s, bs, be, n,
                           reinterpret_cast<const RegionDesc*>(w.desc), w.offsets + ncells, w.seg_start, w.seg_cnt,
                           w.nreg_max, nb, reinterpret_cast<const uint2*>(w.recs), na, 1u, w.partial);
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    // about 8 region shares per thread, at most 512 partial sums per shuffle into the atomics
    const uint32_t gy = (uint32_t)std::min<uint64_t>(std::max<uint64_t>((uint64_t)w.nreg_max * w.splits / 8, 1), 512);
    hipLaunchKernelGGL(k_bin_reduce, dim3((nb + 255) / 256, gy), dim3(256), 0, s, w.partial, w.offsets + ncells,
                       w.splits, nb, totals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace bits
