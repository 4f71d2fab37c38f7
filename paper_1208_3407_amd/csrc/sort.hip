// On-device LSD radix sort of uint32 keys (the two Sort steps of Algorithm 2)
// and the Eytzinger top-tree build.
//
// Segmented: every segment (e.g. B_S and B_E of one or many references) is
// sorted independently in the same launches, keys only or with one uint32
// value per key carried along (explicit, or the implicit 0..n-1 input order;
// the sort is stable, so equal keys keep their input order).  One read of
// the input counts all four 8-bit digits of every segment; then each pass is
// a single kernel over tiles of 16384 keys taken in order from a counter:
// the tile ranks its keys by digit, publishes its digit counts, adds up the
// counts of the tiles before it in its segment by decoupled look-back (the
// nearest tile that has published its inclusive prefix ends the walk), and
// writes its keys out in digit runs.  Every key is read once and written
// once per pass.  A digit that is constant over every segment is skipped
// (decided on the device, so the sort never waits for the host).  Inputs
// are never written.
#include <string.h>

#include <vector>

#include "bits_internal.hpp"

namespace bits {

namespace {

constexpr int kThreads = 256;                  // histogram, scan and copy kernels
constexpr int kWaves = kThreads / kWave;
constexpr int kSweepThreads = 1024;            // one pass of the sort
constexpr int kSweepWaves = kSweepThreads / kWave;
// Keys per wave per tile: 20 rounds of 64 keys held in registers (20480-key
// tiles) for a keys-only sort; 16 rounds (16384-key tiles) when values ride
// along, so that keys and values both fit the tile's LDS.
template <bool VALS>
struct TileShape {
    static constexpr uint32_t kPerWave = VALS ? 1024u : 1280u;
    static constexpr uint32_t kTile = kPerWave * kSweepWaves;
    static constexpr int kRounds = (int)(kPerWave / kWave);
};
__host__ __device__ constexpr uint32_t tile_keys(bool vals) {
    return vals ? TileShape<true>::kTile : TileShape<false>::kTile;
}
// Look-back words, one per (tile, digit): bits 0-31 the count, bits 32-39
// the pass (1 + p; 0 = not yet published in this call), bit 40 set once the
// count is the inclusive prefix over the segment's tiles up to this one
// (else it is the tile's own count).
constexpr uint64_t kLbPrefix = 1ull << 40;
// Polls of a predecessor's word before giving up (the walk cannot deadlock:
// tiles are taken in order, so every tile waited on is held by a running
// workgroup; the bound only turns a fault into BITS_FLAG_SORT, not a hang).
constexpr uint32_t kLbSpinLimit = 1u << 20;
constexpr int kLbBatch = 8;   // predecessor words loaded at once

struct SegDesc {
    const uint32_t* in;
    uint32_t* ping;
    uint32_t* out;
    uint32_t n;
    uint32_t tile0;   // first global tile of the segment
    const uint32_t* vin;   // values: input (nullptr with vmode 2: the input index)
    uint32_t* vping;
    uint32_t* vout;
    uint32_t vmode;   // 0 keys only, 1 values from vin, 2 values = input index
    uint32_t pad;
};
static_assert(sizeof(SegDesc) == 64, "SegDesc layout");

struct SortPlan {
    uint32_t active[4];
    uint32_t src[4];   // 0 = input, 1 = ping, 2 = output
    uint32_t dst[4];
    uint32_t n_active;
    uint32_t next_tile[4];   // tile counter of each pass
    uint32_t error;          // nonzero: a look-back walk gave up (output invalid)
    uint32_t pad[2];
};

constexpr int kDescChunk = 48;   // 3 KB of kernel arguments
struct DescChunk {
    SegDesc d[kDescChunk];
};

__device__ __forceinline__ uint32_t seg_of_tile(const SegDesc* descs, uint32_t nseg, uint32_t t) {
    uint32_t lo = 0, hi = nseg;      // last s with tile0 <= t
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (descs[mid].tile0 <= t) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ const uint32_t* buf_ro(const SegDesc& d, uint32_t sel) {
    return sel == 0 ? d.in : sel == 1 ? d.ping : d.out;
}
__device__ __forceinline__ uint32_t* buf_rw(const SegDesc& d, uint32_t sel) {
    return sel == 1 ? d.ping : d.out;
}
__device__ __forceinline__ const uint32_t* vbuf_ro(const SegDesc& d, uint32_t sel) {
    return sel == 0 ? d.vin : sel == 1 ? d.vping : d.vout;
}
__device__ __forceinline__ uint32_t* vbuf_rw(const SegDesc& d, uint32_t sel) {
    return sel == 1 ? d.vping : d.vout;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) tmp[w] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        if (k < w) pre += tmp[k];
        tot += tmp[k];
    }
    __syncthreads();
    if (total) *total = tot;
    return pre + x - v;
}

__global__ void k_write_descs(SegDesc* dst, DescChunk chunk, uint32_t count) {
    const uint32_t i = threadIdx.x;
    if (i < count) dst[i] = chunk.d[i];
}

// All four digit histograms of every segment in one read of the input.
// Workgroup b walks a contiguous range of tiles, accumulating in LDS and
// flushing when the segment changes.
__global__ void __launch_bounds__(kThreads) k_hist_all(const SegDesc* __restrict__ descs, uint32_t nseg,
                                                       uint32_t ntiles, uint32_t tile,
                                                       uint32_t* __restrict__ seg_hist) {
    __shared__ uint32_t h[4][256];
    const uint32_t t0 = (uint32_t)((uint64_t)ntiles * blockIdx.x / gridDim.x);
    const uint32_t t1 = (uint32_t)((uint64_t)ntiles * (blockIdx.x + 1) / gridDim.x);
    for (int k = threadIdx.x; k < 1024; k += kThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    uint32_t cur = 0xFFFFFFFFu;
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t s = seg_of_tile(descs, nseg, t);
        if (s != cur) {
            if (cur != 0xFFFFFFFFu) {
                __syncthreads();
                for (int k = threadIdx.x; k < 1024; k += kThreads) {
                    const uint32_t v = (&h[0][0])[k];
                    if (v) atomicAdd(seg_hist + (size_t)cur * 1024 + k, v);
                    (&h[0][0])[k] = 0;
                }
                __syncthreads();
            }
            cur = s;
        }
        const SegDesc d = descs[s];
        const uint32_t begin = (t - d.tile0) * tile;
        const uint32_t cnt = min(tile, d.n - begin);
        const uint32_t* src = d.in + begin;
        // four independent loads per thread in flight, then their counts
        for (uint32_t k0 = threadIdx.x; k0 < cnt; k0 += 4 * kThreads) {
            uint32_t key[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t k = k0 + (uint32_t)u * kThreads;
                key[u] = src[min(k, cnt - 1u)];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (k0 + (uint32_t)u * kThreads >= cnt) break;
                atomicAdd(&h[0][key[u] & 255u], 1u);
                atomicAdd(&h[1][(key[u] >> 8) & 255u], 1u);
                atomicAdd(&h[2][(key[u] >> 16) & 255u], 1u);
                atomicAdd(&h[3][key[u] >> 24], 1u);
            }
        }
    }
    __syncthreads();
    if (cur != 0xFFFFFFFFu) {
        for (int k = threadIdx.x; k < 1024; k += kThreads) {
            const uint32_t v = (&h[0][0])[k];
            if (v) atomicAdd(seg_hist + (size_t)cur * 1024 + k, v);
        }
    }
}

// Block (s, p): exclusive prefix over digits of segment s's pass-p histogram;
// marks pass p active when the digit takes two or more values in s.
__global__ void __launch_bounds__(kThreads) k_seg_scan(const uint32_t* __restrict__ seg_hist,
                                                       uint32_t* __restrict__ seg_pre, SortPlan* plan) {
    __shared__ uint32_t tmp[kWaves];
    const uint32_t sp = blockIdx.x;   // s * 4 + p
    const uint32_t v = seg_hist[(size_t)sp * 256 + threadIdx.x];
    uint32_t tot = 0;
    seg_pre[(size_t)sp * 256 + threadIdx.x] = block_excl_scan(v, tmp, &tot);
    const uint64_t nz = __ballot(v != 0);
    __shared__ uint32_t nzc[kWaves];
    if ((threadIdx.x & (kWave - 1)) == 0) nzc[threadIdx.x / kWave] = (uint32_t)__popcll(nz);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int k = 0; k < kWaves; ++k) c += nzc[k];
        if (c >= 2) atomicOr(&plan->active[sp & 3u], 1u);
    }
}

// Buffer schedule: the last active pass writes the output, earlier ones
// alternate so that the first reads the input.
__global__ void k_plan(SortPlan* plan) {
    if (threadIdx.x != 0) return;
    uint32_t na = 0;
    for (int p = 0; p < 4; ++p) na += plan->active[p] ? 1u : 0u;
    plan->n_active = na;
    uint32_t r = 0, prev_dst = 0;
    for (int p = 0; p < 4; ++p) {
        if (!plan->active[p]) continue;
        const uint32_t dst = ((na - 1 - r) % 2 == 0) ? 2u : 1u;
        plan->src[p] = r == 0 ? 0u : prev_dst;
        plan->dst[p] = dst;
        prev_dst = dst;
        ++r;
    }
}

// The look-back word of (tile, digit).
__device__ __forceinline__ unsigned long long* lb_word(unsigned long long* lb, uint32_t ntiles, uint32_t tile,
                                                      uint32_t dg) {
    return lb + (size_t)tile * 256 + dg;
}

template <int WAVES>
__device__ __forceinline__ uint32_t block_excl_scan_n(uint32_t v, uint32_t* tmp) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) tmp[w] = x;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k)
        if (k < w) pre += tmp[k];
    __syncthreads();
    return pre + x - v;
}

// One pass of the sort over one tile (taken from the pass's counter).  Wave
// w ranks keys [w*kPerWave, (w+1)*kPerWave) of the tile in kRounds rounds; within a
// round, lanes holding the same digit are found with 8 ballots (each folded
// into the lane's peer mask by one v_bitop3 per half) and ranked by lane
// order.  The tile's digit counts are published, the exclusive prefix
// over the segment's earlier tiles is gathered by look-back (one thread per
// digit), and the tile, sorted by digit in LDS, is written out in digit runs.
template <bool VALS>
__global__ void __launch_bounds__(kSweepThreads) k_onesweep(const SegDesc* __restrict__ descs, uint32_t nseg,
                                                            SortPlan* plan, int p,
                                                            unsigned long long* __restrict__ lb, uint32_t ntiles,
                                                            const uint32_t* __restrict__ seg_pre) {
    if (!plan->active[p]) return;
    constexpr uint32_t kPerWave = TileShape<VALS>::kPerWave, kTile = TileShape<VALS>::kTile;
    constexpr int kRounds = TileShape<VALS>::kRounds;
    __shared__ uint32_t keys_lds[kTile];
    __shared__ uint32_t vals_lds[VALS ? kTile : 1];
    __shared__ uint32_t wcnt[kSweepWaves][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t tmp[kSweepWaves];
    __shared__ uint32_t tile_sh;
    if (threadIdx.x == 0) tile_sh = atomicAdd(&plan->next_tile[p], 1u);
    for (int k = threadIdx.x; k < kSweepWaves * 256; k += kSweepThreads) (&wcnt[0][0])[k] = 0;
    __syncthreads();
    const uint32_t t = tile_sh;
    const uint32_t s = seg_of_tile(descs, nseg, t);
    const SegDesc d = descs[s];
    const uint32_t begin = (t - d.tile0) * kTile;
    const uint32_t cnt = min(kTile, d.n - begin);
    const uint32_t* src = buf_ro(d, plan->src[p]) + begin;
    uint32_t* dst = buf_rw(d, plan->dst[p]);
    // values: vmode 2 reads the input index on the first active pass
    const bool vals = VALS && d.vmode != 0;
    const bool iota = d.vmode == 2 && plan->src[p] == 0;
    const uint32_t* vsrc = vals && !iota ? vbuf_ro(d, plan->src[p]) + begin : nullptr;
    uint32_t* vdst = vals ? vbuf_rw(d, plan->dst[p]) : nullptr;
    const uint32_t shift = 8u * p;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    uint32_t key[kRounds], rank[kRounds];
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const uint32_t idx = (uint32_t)w * kPerWave + (uint32_t)r * kWave + lane;
        key[r] = idx < cnt ? src[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const uint32_t idx = (uint32_t)w * kPerWave + (uint32_t)r * kWave + lane;
        const bool valid = idx < cnt;
        const uint32_t dg = (key[r] >> shift) & 255u;
        const uint64_t pv = __ballot(valid);
        uint32_t plo = (uint32_t)pv, phi = (uint32_t)(pv >> 32);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint32_t sb = 0u - ((dg >> b) & 1u);   // all ones where the bit is set
            const uint64_t m = __ballot(sb != 0u);
            // peers &= bit ? m : ~m, i.e. peers & ~(m ^ sb): one v_bitop3 per half
            plo = __builtin_amdgcn_bitop3_b32(plo, (uint32_t)m, sb, 0x90);
            phi = __builtin_amdgcn_bitop3_b32(phi, (uint32_t)(m >> 32), sb, 0x90);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t before = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid) old = wcnt[w][dg];
        rank[r] = old + before;
        if (valid && before == 0) wcnt[w][dg] = old + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: wave offsets within the tile, the tile's count, published at once
    uint32_t tot = 0;
    const uint32_t dg = threadIdx.x;
    const unsigned long long tag = (unsigned long long)(p + 1) << 32;
    if (dg < 256) {
#pragma unroll
        for (int k = 0; k < kSweepWaves; ++k) {
            const uint32_t c = wcnt[k][dg];
            wcnt[k][dg] = tot;
            tot += c;
        }
        __hip_atomic_store(lb_word(lb, ntiles, t, dg), (d.tile0 == t ? kLbPrefix : 0ull) | tag | tot, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t ds = block_excl_scan_n<kSweepWaves>(dg < 256 ? tot : 0u, tmp);
    if (dg < 256) {
        // wave offsets become tile offsets: each key then needs one LDS read
        dstart[dg] = ds;
#pragma unroll
        for (int k = 0; k < kSweepWaves; ++k) wcnt[k][dg] += ds;
    }
    __syncthreads();
    // the tile sorted by digit in LDS (needs only tile-local offsets)
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
        const uint32_t idx = (uint32_t)w * kPerWave + (uint32_t)r * kWave + lane;
        if (idx < cnt) {
            const uint32_t kd = (key[r] >> shift) & 255u;
            const uint32_t at = wcnt[w][kd] + rank[r];
            keys_lds[at] = key[r];
            if constexpr (VALS) {
                if (vals) vals_lds[at] = iota ? begin + idx : vsrc[idx];
            }
        }
    }
    if (dg < 256) {
        // look-back over the segment's earlier tiles, kLbBatch words loaded at
        // once (independent loads), then taken nearest first: a word not yet
        // published is polled until it is; the walk ends at an inclusive prefix
        uint32_t excl = 0;
        if (t != d.tile0) {
            uint32_t tp = t - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                unsigned long long v[kLbBatch];
#pragma unroll
                for (int k = 0; k < kLbBatch; ++k) {
                    const uint32_t tk = tp >= d.tile0 + (uint32_t)k ? tp - (uint32_t)k : d.tile0;
                    v[k] = __hip_atomic_load(lb_word(lb, ntiles, tk, dg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
                for (int k = 0; k < kLbBatch; ++k) {
                    if (done) break;
                    const uint32_t tk = tp - (uint32_t)k;
                    while ((v[k] & (0xFFull << 32)) != tag) {
                        if (++spins > kLbSpinLimit) {
                            atomicOr(&plan->error, 1u);
                            v[k] = kLbPrefix | tag;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        v[k] = __hip_atomic_load(lb_word(lb, ntiles, tk, dg), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                    }
                    excl += (uint32_t)v[k];
                    done = (v[k] & kLbPrefix) || tk == d.tile0;
                }
                tp -= kLbBatch;
            }
            __hip_atomic_store(lb_word(lb, ntiles, t, dg), kLbPrefix | tag | (excl + tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        goff[dg] = seg_pre[((size_t)s * 4 + p) * 256 + dg] + excl;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < cnt; k += kSweepThreads) {
        const uint32_t v = keys_lds[k];
        const uint32_t kd = (v >> shift) & 255u;
        const uint32_t at = goff[kd] + (k - dstart[kd]);
        dst[at] = v;
        if constexpr (VALS) {
            if (vals) vdst[at] = vals_lds[k];
        }
    }
}

// When no digit varies the input is already sorted (all keys equal): copy.
__global__ void k_copy_if_idle(const SegDesc* __restrict__ descs, uint32_t nseg, const SortPlan* __restrict__ plan,
                               uint32_t tile) {
    if (plan->n_active) return;
    const uint32_t t = blockIdx.x;
    const uint32_t s = seg_of_tile(descs, nseg, t);
    const SegDesc d = descs[s];
    const uint32_t begin = (t - d.tile0) * tile;
    const uint32_t cnt = min(tile, d.n - begin);
    for (uint32_t k = threadIdx.x; k < cnt; k += kThreads) {
        d.out[begin + k] = d.in[begin + k];
        if (d.vmode) d.vout[begin + k] = d.vmode == 2 ? begin + k : d.vin[begin + k];
    }
}

// Eytzinger top tree: node k (level l = floor(log2 k), j = k - 2^l) holds
// keys[p - 1] with p = floor((2j + 1) n / 2^(l + 1)), i.e. the last key of
// the bucket left of boundary p.  The first 2^d - 1 nodes form the depth-d
// tree for every d <= depth.
__global__ void k_build_tree(const uint32_t* __restrict__ keys, uint64_t n, uint32_t depth, uint32_t* __restrict__ tree) {
    const uint32_t m = 1u << depth;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < m; k += gridDim.x * blockDim.x) {
        if (k == 0) {
            tree[0] = 0u;
            continue;
        }
        const uint32_t l = 31u - __clz(k);
        const uint64_t j = k - (1u << l);
        const uint64_t pos = ((2 * j + 1) * n) >> (l + 1);
        tree[k] = keys[pos - 1];
    }
}

// Line heads: the first key of every 128-byte line, then +inf padding.
__global__ void k_build_heads(const uint32_t* __restrict__ keys, uint64_t n, uint64_t hl, uint32_t* __restrict__ heads) {
    const uint64_t m = (n + 31) / 32;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < hl; j += (uint64_t)gridDim.x * blockDim.x)
        heads[j] = j < m ? keys[32 * j] : 0xFFFFFFFFu;
}

struct WsLayout {
    size_t descs, plan, seg_hist, seg_pre, lb, ping, vping, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static WsLayout ws_layout(const uint64_t* n, uint32_t nseg, const uint32_t* vmode) {
    bool any_vals = false;
    for (uint32_t s = 0; s < nseg; ++s) any_vals |= vmode && vmode[s];
    const uint64_t tile = tile_keys(any_vals);
    uint64_t ntiles = 0, nkeys = 0, nvals = 0;
    for (uint32_t s = 0; s < nseg; ++s) {
        ntiles += (n[s] + tile - 1) / tile;
        nkeys += n[s];
        if (vmode && vmode[s]) nvals += n[s];
    }
    WsLayout L;
    size_t o = 0;
    L.plan = o; o = align256(o + sizeof(SortPlan));   // first: launch_sort_report finds it at 0
    L.descs = o; o = align256(o + sizeof(SegDesc) * nseg);
    L.seg_hist = o; o = align256(o + (size_t)nseg * 1024 * 4);
    L.seg_pre = o; o = align256(o + (size_t)nseg * 1024 * 4);
    L.lb = o; o = align256(o + (size_t)ntiles * 256 * 8);
    L.ping = o; o = align256(o + (size_t)nkeys * 4);
    L.vping = o; o = align256(o + (size_t)nvals * 4);
    L.total = o;
    return L;
}

}  // namespace

size_t sort_workspace_bytes(const uint64_t* n, uint32_t nseg, const uint32_t* vmode) {
    return ws_layout(n, nseg, vmode).total;
}

int launch_sort(const SortSeg* segs, uint32_t nseg, void* ws, size_t ws_bytes, hipStream_t s) {
    std::vector<uint64_t> ns(nseg);
    std::vector<uint32_t> vm(nseg);
    for (uint32_t i = 0; i < nseg; ++i) {
        if (segs[i].n > 0xFFFFFFFFull || segs[i].vmode > 2) return BITS_E_ARG;
        if ((segs[i].vmode == 1 && !segs[i].vin) || (segs[i].vmode && !segs[i].vout)) return BITS_E_ARG;
        ns[i] = segs[i].n;
        vm[i] = segs[i].vmode;
    }
    const WsLayout L = ws_layout(ns.data(), nseg, vm.data());
    bool any_vals = false;
    for (uint32_t i = 0; i < nseg; ++i) any_vals |= vm[i] != 0;
    const uint32_t tile = tile_keys(any_vals);
    if (ws_bytes < L.total) return BITS_E_WORKSPACE;
    char* base = (char*)ws;
    SegDesc* descs = (SegDesc*)(base + L.descs);
    SortPlan* plan = (SortPlan*)(base + L.plan);
    uint32_t* seg_hist = (uint32_t*)(base + L.seg_hist);
    uint32_t* seg_pre = (uint32_t*)(base + L.seg_pre);
    unsigned long long* lb = (unsigned long long*)(base + L.lb);
    uint32_t* ping = (uint32_t*)(base + L.ping);
    uint32_t* vping = (uint32_t*)(base + L.vping);

    // Descriptors, written by small kernels from by-value chunks so the call
    // stays asynchronous and capturable.
    uint32_t tile0 = 0;
    uint64_t koff = 0, voff = 0;
    for (uint32_t c0 = 0; c0 < nseg; c0 += kDescChunk) {
        DescChunk ch;
        memset(&ch, 0, sizeof(ch));
        const uint32_t cnt = (nseg - c0) < (uint32_t)kDescChunk ? (nseg - c0) : (uint32_t)kDescChunk;
        for (uint32_t i = 0; i < cnt; ++i) {
            const SortSeg& g = segs[c0 + i];
            ch.d[i].in = g.in;
            ch.d[i].out = g.out;
            ch.d[i].ping = ping + koff;
            ch.d[i].n = (uint32_t)g.n;
            ch.d[i].tile0 = tile0;
            ch.d[i].vmode = g.vmode;
            if (g.vmode) {
                ch.d[i].vin = g.vmode == 1 ? g.vin : nullptr;
                ch.d[i].vping = vping + voff;
                ch.d[i].vout = g.vout;
                voff += g.n;
            }
            tile0 += (uint32_t)((g.n + tile - 1) / tile);
            koff += g.n;
        }
        hipLaunchKernelGGL(k_write_descs, dim3(1), dim3(128), 0, s, descs + c0, ch, cnt);
    }
    const uint32_t ntiles = tile0;
    BITS_CHECK_HIP(launch_fill_u32((uint32_t*)plan, sizeof(SortPlan) / 4, 0u, s));
    BITS_CHECK_HIP(launch_fill_u32(seg_hist, (uint64_t)nseg * 1024, 0u, s));
    if (ntiles == 0) {
        BITS_CHECK_HIP(hipGetLastError());
        return BITS_OK;
    }

    BITS_CHECK_HIP(launch_fill_u64(lb, (uint64_t)ntiles * 256, 0ull, s));
    const uint32_t hg = ntiles < 2048u ? ntiles : 2048u;
    hipLaunchKernelGGL(k_hist_all, dim3(hg), dim3(kThreads), 0, s, descs, nseg, ntiles, tile, seg_hist);
    hipLaunchKernelGGL(k_seg_scan, dim3(nseg * 4), dim3(kThreads), 0, s, seg_hist, seg_pre, plan);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, s, plan);
    for (int p = 0; p < 4; ++p) {
        if (any_vals)
            hipLaunchKernelGGL(k_onesweep<true>, dim3(ntiles), dim3(kSweepThreads), 0, s, descs, nseg, plan, p, lb,
                               ntiles, seg_pre);
        else
            hipLaunchKernelGGL(k_onesweep<false>, dim3(ntiles), dim3(kSweepThreads), 0, s, descs, nseg, plan, p, lb,
                               ntiles, seg_pre);
    }
    hipLaunchKernelGGL(k_copy_if_idle, dim3(ntiles), dim3(kThreads), 0, s, descs, nseg, plan, tile);
    BITS_CHECK_HIP(hipGetLastError());
    return BITS_OK;
}

// Ors BITS_FLAG_SORT into *status if the last sort in ws gave up a look-back.
__global__ void k_sort_report(const SortPlan* plan, uint32_t* status) {
    if (threadIdx.x == 0 && plan->error) atomicOr(status, BITS_FLAG_SORT);
}

hipError_t launch_sort_report(const void* ws, uint32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_report, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<const SortPlan*>(ws), status);
    return hipGetLastError();
}

hipError_t launch_build_tree(const uint32_t* keys, uint64_t n, uint32_t depth, uint32_t* tree, hipStream_t s) {
    const uint32_t m = 1u << depth;
    const uint32_t g = (m + 255) / 256;
    hipLaunchKernelGGL(k_build_tree, dim3(g), dim3(256), 0, s, keys, n, depth, tree);
    return hipGetLastError();
}

hipError_t launch_build_heads(const uint32_t* keys, uint64_t n, uint32_t* heads, hipStream_t s) {
    const uint64_t hl = heads_len(n);
    uint64_t g = (hl + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_build_heads, dim3((uint32_t)g), dim3(256), 0, s, keys, n, hl, heads);
    return hipGetLastError();
}

}  // namespace bits
