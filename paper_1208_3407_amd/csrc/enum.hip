// Enumeration (Sec. 1.1, sub-problem 4) for gfx950: the pairs behind the
// per-query counts.
//
// Sec. 2.1 notes that the count of a query is what makes enumeration cheap:
// every b intersecting a has b.start <= a.end, i.e. lies before position
// first = #{B_S <= a.end} of B sorted by start, so scanning that prefix
// backwards and keeping the intervals with b.end >= a.start finds them all,
// and the scan can stop as soon as count(a) of them have been found.  Intervals
// contained in an earlier one are stepped over without being counted, which is
// the extra work the paper describes for nested intervals.
//
// Pieces:
//   - the index: B_S sorted with each interval's input index carried along by
//     the segmented radix sort (stable), then the ends gathered into that order;
//   - an exclusive scan of the per-query counts into uint64 output offsets;
//   - the enumeration kernel, one query per lane.
#include "bits_internal.hpp"

namespace bits {

namespace {

constexpr uint32_t kScanThreads = 256;
constexpr uint32_t kScanPer = 16;                             // counts per thread per tile
constexpr uint32_t kScanTile = kScanThreads * kScanPer;       // 4096 counts per tile

__global__ void k_gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx, uint64_t n,
                             uint32_t* __restrict__ dst) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (uint64_t)gridDim.x * blockDim.x)
        dst[j] = src[idx[j]];
}

// Inclusive scan of one uint64 per thread over the block; returns the
// thread's exclusive prefix and the block total in *total.
__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t* tmp, uint64_t* total) {
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t y = __shfl_up(x, o);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == kWave - 1) tmp[w] = x;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (uint32_t k = 0; k < blockDim.x / kWave; ++k) {
        if (k < w) pre += tmp[k];
        tot += tmp[k];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

// Tile sums of the counts.
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t* __restrict__ counts, uint64_t n,
                                                              uint64_t* __restrict__ tile_sum) {
    __shared__ uint64_t tmp[kScanThreads / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (uint32_t k = threadIdx.x; k < kScanTile; k += kScanThreads) {
        const uint64_t i = base + k;
        if (i < n) s += counts[i];
    }
    uint64_t tot = 0;
    block_scan_u64(s, tmp, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place (one workgroup, any number of tiles).
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(uint64_t* __restrict__ tile_sum, uint64_t ntiles) {
    __shared__ uint64_t tmp[kScanThreads / kWave];
    uint64_t carry = 0;
    for (uint64_t b = 0; b < ntiles; b += kScanThreads) {
        const uint64_t i = b + threadIdx.x;
        const uint64_t v = i < ntiles ? tile_sum[i] : 0ull;
        uint64_t tot = 0;
        const uint64_t pre = block_scan_u64(v, tmp, &tot);
        if (i < ntiles) tile_sum[i] = carry + pre;
        carry += tot;
    }
}

// offsets[i] = tile prefix + prefix inside the tile; offsets[n] = total.
// Thread t of a tile owns counts [t * kScanPer, (t + 1) * kScanPer).
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const uint32_t* __restrict__ counts, uint64_t n,
                                                            const uint64_t* __restrict__ tile_pre,
                                                            uint64_t* __restrict__ offsets) {
    __shared__ uint64_t tmp[kScanThreads / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? counts[base + k] : 0u;
        s += v[k];
    }
    uint64_t tot = 0;
    uint64_t run = tile_pre[blockIdx.x] + block_scan_u64(s, tmp, &tot);
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        if (base + k < n) offsets[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) offsets[n] = run;
}

__global__ void k_scan_empty(uint64_t* offsets) { offsets[0] = 0ull; }

// One query per lane.  first = #{starts <= a.end}, given (the counting
// search computes it on the way) or found here by bisection; then the
// backward scan of Sec. 2.1 until count(a) pairs are out.  Pairs land at
// [offsets[i], offsets[i] + counts[i]), never at or past max_pairs; a query
// whose scan ends short of its count (counts not from this B) sets
// BITS_FLAG_ENUM.
__global__ void __launch_bounds__(256) k_enumerate(const uint32_t* __restrict__ starts,
                                                   const uint32_t* __restrict__ ends,
                                                   const uint32_t* __restrict__ ids, uint32_t n,
                                                   const uint32_t* __restrict__ a_start,
                                                   const uint32_t* __restrict__ a_end, uint64_t na,
                                                   const uint32_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ firsts,
                                                   const uint64_t* __restrict__ offsets, uint32_t* __restrict__ pa,
                                                   uint32_t* __restrict__ pb, uint64_t max_pairs, uint32_t* status) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t s = a_start[i], e = a_end[i], c = counts[i];
        if (c == 0u) continue;
        if (s > e) {
            bad |= BITS_FLAG_INTERVAL;
            continue;
        }
        uint32_t first;
        if (firsts) {
            first = min(firsts[i], n);
        } else if (e == 0xFFFFFFFFu) {
            first = n;
        } else {
            uint32_t lo = 0, len = n;   // #{starts < e + 1}
            while (len) {
                const uint32_t h = len >> 1;
                if (starts[lo + h] <= e) {
                    lo += h + 1;
                    len -= h + 1;
                } else {
                    len = h;
                }
            }
            first = lo;
        }
        const uint64_t off = offsets[i];
        uint32_t found = 0, j = first;
        while (found < c && j > 0) {
            --j;
            if (ends[j] >= s) {
                const uint64_t at = off + found;
                if (at < max_pairs) {
                    pa[at] = (uint32_t)i;
                    pb[at] = ids[j];
                } else {
                    bad |= BITS_FLAG_ENUM;
                }
                ++found;
            }
        }
        if (found < c) bad |= BITS_FLAG_ENUM;
    }
    if (bad && status) atomicOr(status, bad);
}

}  // namespace

uint64_t scan_tiles(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint64_t n, uint32_t* dst, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_gather_u32, dim3((uint32_t)g), dim3(256), 0, s, src, idx, n, dst);
    return hipGetLastError();
}

hipError_t launch_scan_counts(const uint32_t* counts, uint64_t n, uint64_t* offsets, uint64_t* tile_sum,
                              hipStream_t s) {
    if (!n) {
        hipLaunchKernelGGL(k_scan_empty, dim3(1), dim3(1), 0, s, offsets);
        return hipGetLastError();
    }
    const uint64_t nt = scan_tiles(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nt), dim3(kScanThreads), 0, s, counts, n, tile_sum);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, tile_sum, nt);
    hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)nt), dim3(kScanThreads), 0, s, counts, n, tile_sum, offsets);
    return hipGetLastError();
}

hipError_t launch_enumerate(const uint32_t* starts, const uint32_t* ends, const uint32_t* ids, uint32_t n,
                            const uint32_t* as, const uint32_t* ae, uint64_t na, const uint32_t* counts,
                            const uint32_t* firsts, const uint64_t* offsets, uint32_t* pa, uint32_t* pb,
                            uint64_t max_pairs, uint32_t* status, hipStream_t s) {
    if (!na) return hipSuccess;
    uint64_t g = (na + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 32;
    if (g > cap) g = cap;
    hipLaunchKernelGGL(k_enumerate, dim3((uint32_t)g), dim3(256), 0, s, starts, ends, ids, n, as, ae, na, counts,
                       firsts, offsets, pa, pb, max_pairs, status);
    return hipGetLastError();
}

}  // namespace bits
