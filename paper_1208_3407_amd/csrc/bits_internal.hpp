// Internal declarations of libbits.so (gfx950).  Device helpers used by the
// search, Monte-Carlo, batch and learned-index kernels, and the host-side
// launchers each translation unit exports to the C ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bits.h"

#define BITS_CHECK_HIP(expr)                                   \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return BITS_E_HIP;               \
    } while (0)

namespace bits {

constexpr int kWave = 64;
constexpr uint32_t kMaxTreeNodes = 1u << BITS_MAX_DEPTH;   // per array, entry 0 unused

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t olo = __shfl_xor(lo, o);
        uint32_t ohi = __shfl_xor(hi, o);
        uint32_t nlo = lo + olo;
        hi = hi + ohi + (nlo < lo ? 1u : 0u);
        lo = nlo;
    }
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// ------------------------------------------------------------------ Philox-4x32-10
// Counter-based generator of Salmon et al. (SC'11): ten rounds of two 32x32
// multiplies, word exchange and key xor, the key advancing by two Weyl
// increments after every round.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = c0 * 0xD2511F53u, hi0 = __umulhi(c0, 0xD2511F53u);
        const uint32_t lo1 = c2 * 0xCD9E8D57u, hi1 = __umulhi(c2, 0xCD9E8D57u);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ------------------------------------------------------------------ search arguments

struct SearchArgs {
    const uint32_t* bs;          // sorted starts
    const uint32_t* be;          // sorted ends
    const uint32_t* tree;        // [2][tree_stride] Eytzinger splitters
    const bits_rmi_model* rmi;   // [2] learned models or nullptr
    uint32_t* status;            // device status word
    unsigned long long* fallbacks;
    uint32_t n;                  // |B|
    uint32_t tree_stride;        // 2^built_depth
    uint32_t depth;              // levels searched from LDS (<= built depth)
};

// Number of LDS words a search kernel stages for depth d (both arrays).
__host__ __device__ constexpr uint32_t tree_lds_words(uint32_t d) { return d ? (2u << d) : 0u; }

// Copy the first 2^d - 1 nodes of both trees into LDS: lds[0..2^d) starts,
// lds[2^d..2^(d+1)) ends, 1-based BFS order (slot 0 unused).
__device__ __forceinline__ void stage_tree(uint32_t* lds, const uint32_t* tree, uint32_t stride, uint32_t d) {
    if (!d) return;
    const uint32_t m = 1u << d;
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
        lds[k] = tree[k];
        lds[m + k] = tree[stride + k];
    }
}

// ------------------------------------------------------------------ learned index

__device__ __forceinline__ uint32_t rmi_route(float a, float b, uint32_t x) {
    float r = floorf(fmaf(a, (float)x, b));
    r = fminf(fmaxf(r, 0.0f), (float)(BITS_RMI_LEAVES - 1));
    return (uint32_t)r;
}

// Rank offset predicted inside a leaf for a key x with kmin <= x (dx = x - kmin).
// The same arithmetic is used when the error windows are measured and when
// queries are answered.
__device__ __forceinline__ int32_t rmi_pred_offset(const float* p, uint32_t cnt, float kinv, uint32_t dx) {
    const float u = (float)dx * kinv;
    float y = p[48];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const float h = fmaxf(fmaf(p[j], u, p[16 + j]), 0.0f);
        y = fmaf(p[32 + j], h, y);
    }
    float r = rintf(y * (float)cnt);
    r = fminf(fmaxf(r, 0.0f), (float)cnt);
    return (int32_t)r;
}

// ------------------------------------------------------------------ host launchers

struct LaunchCfg {
    uint32_t block, qpl, depth, grid, path;
};

int device_cu_count();
int resolve_launch(const bits_ref* ref, const bits_launch* in, LaunchCfg* out);
SearchArgs make_search_args(const bits_ref* ref, const LaunchCfg& cfg);

// search.hip
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
hipError_t launch_count(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                        uint64_t na, uint32_t* counts, unsigned long long* total, hipStream_t s);
hipError_t launch_mc_prepare(const uint32_t* as, const uint32_t* ae, uint64_t na, const uint32_t* chrom_len,
                             uint32_t n_chrom, uint32_t* off, uint32_t* span, uint32_t* len, uint32_t* status,
                             hipStream_t s);
hipError_t launch_mc(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                     const uint32_t* off, const uint32_t* span, const uint32_t* len, uint64_t na,
                     uint64_t seed, uint64_t s0, uint64_t nshuf, unsigned long long* totals,
                     unsigned long long* observed, hipStream_t s);
hipError_t launch_mc_tail(const unsigned long long* totals, uint64_t nshuf, const unsigned long long* observed,
                          unsigned long long* n_ge, unsigned long long* n_le, hipStream_t s);
hipError_t launch_project(const uint32_t* chrom_len, uint32_t n_chrom, const uint32_t* chrom,
                          const uint32_t* ls, const uint32_t* le, uint64_t n, uint32_t* gs, uint32_t* ge,
                          uint32_t* status, hipStream_t s);

// Batched pairs (search.hip)
struct BatchRef {        // one reference in the batch table
    const uint32_t* bs;
    const uint32_t* be;
    const uint32_t* tree;
    uint32_t n, tree_stride, depth, pad;
};
struct BatchQuery {
    const uint32_t* as;
    const uint32_t* ae;
    uint64_t n;
};
struct BatchItem {       // a tile of one query set against one reference
    uint32_t q, r, begin, count;
};
hipError_t launch_batch(const BatchRef* refs, const BatchQuery* qs, const BatchItem* items,
                        const uint32_t* wg_begin, uint32_t n_wg, uint32_t n_ref, uint32_t max_depth,
                        const LaunchCfg& cfg, unsigned long long* pair_totals, uint32_t* status,
                        hipStream_t s);

// sort.hip
struct SortSeg {
    const uint32_t* in;
    uint32_t* out;
    uint64_t n;
};
size_t sort_workspace_bytes(const uint64_t* n, uint32_t nseg);
int launch_sort(const SortSeg* segs, uint32_t nseg, void* ws, size_t ws_bytes, hipStream_t s);
hipError_t launch_build_tree(const uint32_t* keys, uint64_t n, uint32_t depth, uint32_t* tree, hipStream_t s);

// rmi.hip
size_t rmi_workspace_bytes();
int launch_rmi_build2(const uint32_t* keys0, const uint32_t* keys1, uint64_t n, bits_rmi_model* m0,
                      bits_rmi_model* m1, const bits_train& tr, void* ws, hipStream_t s);
hipError_t launch_rmi_leaf_grad(const float* u, const float* t, uint32_t m, const float* params, float* grad,
                                float* loss, hipStream_t s);

}  // namespace bits
