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
    // Each 32 x 32 -> 64 product is one v_mad_u64_u32 and each three-way xor one
    // v_bitop3 (truth table 0x96), four VALU instructions per round.
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u, p1 = (uint64_t)c2 * 0xCD9E8D57u;
        c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        c1 = (uint32_t)p1;
        c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Start of a query's placement in shuffle s (Sec. 3.2): counter g = s * na + i
// (i the query's input index), key = the seed; the 64-bit draw u = (c1, c0)
// scaled to [0, span) by a high multiply, span > 0 being the number of legal
// starts of the query in its chromosome, which begins at `off`.
__device__ __forceinline__ uint32_t mc_place(uint64_t g, uint32_t k0, uint32_t k1, uint32_t off, uint32_t span) {
    uint32_t c0 = (uint32_t)g, c1 = (uint32_t)(g >> 32), c2 = 0u, c3 = 0u;
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    const uint64_t u = ((uint64_t)c1 << 32) | c0;
    return off + (uint32_t)__umul64hi(u, (uint64_t)span);
}

// ------------------------------------------------------------------ search arguments

struct SearchArgs {
    const uint32_t* bs;          // sorted starts
    const uint32_t* be;          // sorted ends
    const uint32_t* tree;        // [2][tree_stride] Eytzinger splitters
    const bits_rmi_model* rmi;   // [2] learned models or nullptr
    const uint32_t* hs;          // line heads of B_S (learned only): hs[j] = bs[32 j], 0xFFFFFFFF past the end
    const uint32_t* he;          // line heads of B_E
    uint32_t* status;            // device status word
    unsigned long long* fallbacks;
    uint32_t n;                  // |B|
    uint32_t tree_stride;        // 2^built_depth
    uint32_t depth;              // levels searched from LDS (<= built depth)
};

// Entries of one line-head array for n keys: ceil(n / 32) heads plus at
// least 32 entries of 0xFFFFFFFF, rounded up to whole 128-byte lines, so a
// 32-entry window starting at or before head ceil(n / 32) - 1 + 16 stays in bounds.
__host__ __device__ constexpr uint64_t heads_len(uint64_t n) { return ((n + 31) / 32 + 32 + 31) / 32 * 32; }

// Number of LDS words a search kernel stages for depth d (both arrays).
__host__ __device__ constexpr uint32_t tree_lds_words(uint32_t d) { return d ? (2u << d) : 0u; }

// LDS scratch of the learned search per chain: (leaf, x) of 64 owners, then
// 6 result words per owner; per wave: 2 * QPL chains.
constexpr uint32_t kLeafScr = 2 * kWave + 6 * kWave;
__host__ __device__ constexpr uint32_t probe_scratch_words(int qpl) { return 2u * (uint32_t)qpl * kLeafScr; }

// Dynamic LDS of a search kernel: the top trees (plain) or the per-wave
// scratch (learned).
__host__ __device__ constexpr size_t search_lds_bytes(bool learned, uint32_t depth, int qpl, uint32_t block) {
    return learned ? (size_t)(block / kWave) * probe_scratch_words(qpl) * 4u : (size_t)tree_lds_words(depth) * 4u;
}

// Line-probe scratch of the tiered search per wave: (start, x) of 64 owners
// and 64 counts (2 * 64 words each) per chain, 2 * QPL chains.
__host__ __device__ constexpr uint32_t tiered_scratch_words(int qpl) { return 4u * 2u * (uint32_t)qpl * kWave; }

// Counting kernel modes (k_count) and their dynamic LDS: the tiered search
// stages the top trees and, after them, its per-wave probe scratch.
enum : int { kModePlain = 0, kModeLearned = 1, kModeTiered = 2 };
__host__ __device__ constexpr size_t count_lds_bytes(uint32_t path, uint32_t depth, int qpl, uint32_t block) {
    return path == BITS_PATH_TIERED
               ? ((size_t)tree_lds_words(depth) + (size_t)(block / kWave) * tiered_scratch_words(qpl)) * 4u
               : search_lds_bytes(path == BITS_PATH_LEARNED, depth, qpl, block);
}

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

// Leaf prediction, in one fixed arithmetic order shared by the error-window
// measurement (sequential, rmi_pred_offset) and the queries (4 lanes per
// leaf, rmi_quad_partial + two lane-pair additions):
//   h_j = max(fma(w1_j, u, b1_j), 0),  s_q = fma-chain over j = 4q..4q+3 of w2_j h_j,
//   y   = b2 + ((s_0 + s_1) + (s_2 + s_3)).
__device__ __forceinline__ float rmi_quad_partial(const float* w1, const float* b1, const float* w2, float u) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) s = fmaf(w2[k], fmaxf(fmaf(w1[k], u, b1[k]), 0.0f), s);
    return s;
}

__device__ __forceinline__ int32_t rmi_offset_from_y(float y, uint32_t cnt) {
    float r = rintf(y * (float)cnt);
    r = fminf(fmaxf(r, 0.0f), (float)cnt);
    return (int32_t)r;
}

__device__ __forceinline__ float rmi_u(uint32_t dx, float kinv) { return (float)dx * kinv; }

// IEEE binary16 <-> fp32 (round to nearest even) for the stored leaf weights.
__device__ __forceinline__ float h2f(uint32_t bits) { return (float)__builtin_bit_cast(_Float16, (uint16_t)bits); }
__device__ __forceinline__ uint32_t f2h(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f); }

// Rank offset predicted inside a leaf for a key x with kmin <= x (dx = x - kmin);
// p holds the stored weights (w1, b1, w2 already rounded to binary16) and b2.
__device__ __forceinline__ int32_t rmi_pred_offset(const float* p, uint32_t cnt, float kinv, uint32_t dx) {
    const float u = rmi_u(dx, kinv);
    const float s0 = rmi_quad_partial(p + 0, p + 16, p + 32, u);
    const float s1 = rmi_quad_partial(p + 4, p + 20, p + 36, u);
    const float s2 = rmi_quad_partial(p + 8, p + 24, p + 40, u);
    const float s3 = rmi_quad_partial(p + 12, p + 28, p + 44, u);
    const float y = p[48] + ((s0 + s1) + (s2 + s3));
    return rmi_offset_from_y(y, cnt);
}

// ------------------------------------------------------------------ host launchers

struct LaunchCfg {
    uint32_t block, qpl, depth, grid, path;
};

int device_cu_count();
size_t device_lds_per_block();
int resolve_launch(const bits_ref* ref, const bits_launch* in, LaunchCfg* out);
SearchArgs make_search_args(const bits_ref* ref, const LaunchCfg& cfg);

// search.hip
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
// counts (nullable), firsts (nullable: #{B_S <= a.end} per query), total (nullable)
hipError_t launch_count(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                        uint64_t na, uint32_t* counts, unsigned long long* total, hipStream_t s,
                        uint32_t* firsts = nullptr);
// Monte-Carlo query table in the caller's workspace: uint32[na] each of
// chromosome offset, legal-start count, length and original index, grouped
// by chromosome; hist and cursor hold BITS_MAX_CHROM words each.
struct McTable {
    uint32_t *off, *span, *len, *idx, *hist, *cursor;
};
hipError_t launch_mc_prepare(const uint32_t* as, const uint32_t* ae, uint64_t na, const uint32_t* chrom_len,
                             uint32_t n_chrom, const McTable& tab, uint32_t* status, hipStream_t s);
hipError_t launch_mc(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                     const McTable& tab, uint64_t na, uint64_t seed, uint64_t s0, uint64_t nshuf,
                     unsigned long long* totals, unsigned long long* observed, hipStream_t s);
hipError_t launch_rmi_window(const SearchArgs& sa, uint32_t which, const uint32_t* xs, uint64_t n, uint32_t* lo,
                             uint32_t* hi, hipStream_t s);
hipError_t launch_decide(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                         uint64_t na, uint32_t* found, unsigned long long* witness, hipStream_t s);
hipError_t launch_select_u64(const unsigned long long* v, uint64_t n, uint64_t k0, uint64_t k1,
                             unsigned long long* out0, unsigned long long* out1, hipStream_t s);
hipError_t launch_place_rounds(const McTable& tab, const uint32_t* b_start, uint64_t nb, uint64_t seed, uint64_t s0,
                               uint32_t rounds, bool identity, uint32_t* S, uint32_t* E, hipStream_t s);
hipError_t launch_count_rounds(const uint32_t* S, const uint32_t* E, uint64_t nb, uint32_t rounds, const uint32_t* as,
                               const uint32_t* ae, uint64_t na, unsigned long long* totals, uint32_t* status,
                               hipStream_t s);
// binned.hip: the Monte-Carlo path binned by genome region.
struct BinLayout {
    uint64_t ncells, nreg_max;
    uint32_t splits;              // search workgroups per region
};
// Cell count and an upper bound on the region count for a genome and |B| = n;
// false if the genome cannot be cut (sizes past 2^32).
bool bin_layout(const uint32_t* chrom_len, uint32_t n_chrom, uint64_t n, BinLayout* L);
struct BinWs {                    // device buffers, carved from the caller's workspace
    uint32_t *rs, *re, *flag;     // [ncells]
    uint64_t* offsets;            // [ncells + 1]: region starts (exclusive scan of flag); offsets[ncells] = regions
    uint64_t* scan_tiles;         // scan_tiles(ncells)
    uint32_t* cell_region;        // [ncells]
    void* desc;                   // [nreg_max + 1] region descriptors (16 bytes)
    uint32_t *seg_start, *seg_cnt;    // [batch][nreg_max]
    unsigned long long* partial;      // [nreg_max * splits][batch]
    void* recs;                       // [batch][na] {start, end}
    void* packed;                     // [na] {input index, length or 0}
    uint32_t nreg_max, splits;
};
hipError_t launch_bin_pack(const McTable& tab, uint64_t na, const BinWs& w, hipStream_t s);
hipError_t launch_bin_regions(const uint32_t* chrom_len, uint32_t n_chrom, const uint32_t* bs, const uint32_t* be,
                              uint32_t n, const BinWs& w, uint32_t* status, hipStream_t s);
// Shuffles [sb, sb + nb) (absolute indices); totals points at shuffle sb's slot.
hipError_t launch_bin_batch(const uint32_t* chrom_len, uint32_t n_chrom, const McTable& tab, uint64_t na,
                            const uint32_t* bs, const uint32_t* be, uint32_t n, uint64_t seed, uint64_t sb,
                            uint32_t nb, const BinWs& w, unsigned long long* totals, hipStream_t s,
                            hipEvent_t* ev = nullptr);   // ev[4]: before binning, search, reduction, after
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
    const bits_rmi_model* rmi;       // learned path: the two models (else nullptr)
    const uint32_t* hs;              // learned path: line heads of B_S and B_E
    const uint32_t* he;
    unsigned long long* fallbacks;   // the reference's learned-path fallback counter
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
// cfg.path selects the plain (LDS tree + bisection) or the learned search for every pair;
// the learned path needs every reference learned.
hipError_t launch_batch(const BatchRef* refs, const BatchQuery* qs, const BatchItem* items,
                        const uint32_t* wg_begin, uint32_t n_wg, uint32_t n_ref, uint32_t max_depth,
                        const LaunchCfg& cfg, unsigned long long* pair_totals, uint32_t* status,
                        hipStream_t s);
int batch_blocks_per_cu(const LaunchCfg& cfg, uint32_t max_depth);

// sort.hip
// One segment to sort: n keys in -> out, optionally with one uint32 value per
// key moved along (vmode 1: values from vin; 2: the input index 0..n-1).
struct SortSeg {
    const uint32_t* in;
    uint32_t* out;
    uint64_t n;
    uint32_t vmode = 0;
    const uint32_t* vin = nullptr;
    uint32_t* vout = nullptr;
};
size_t sort_workspace_bytes(const uint64_t* n, uint32_t nseg, const uint32_t* vmode = nullptr);
int launch_sort(const SortSeg* segs, uint32_t nseg, void* ws, size_t ws_bytes, hipStream_t s);
// After launch_sort, before anything else writes ws: ORs BITS_FLAG_SORT into
// *status if a tile's look-back walk gave up (never expected; the sorted
// output is then invalid).
hipError_t launch_sort_report(const void* ws, uint32_t* status, hipStream_t s);
hipError_t launch_build_tree(const uint32_t* keys, uint64_t n, uint32_t depth, uint32_t* tree, hipStream_t s);
// Line heads of a sorted array: H[j] = keys[32 j] for j < ceil(n / 32), then
// 0xFFFFFFFF up to heads_len(n) entries.
hipError_t launch_build_heads(const uint32_t* keys, uint64_t n, uint32_t* heads, hipStream_t s);

// enum.hip
uint64_t scan_tiles(uint64_t n);
hipError_t launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint64_t n, uint32_t* dst, hipStream_t s);
hipError_t launch_scan_counts(const uint32_t* counts, uint64_t n, uint64_t* offsets, uint64_t* tile_sum,
                              hipStream_t s);
hipError_t launch_enumerate(const uint32_t* starts, const uint32_t* ends, const uint32_t* ids, uint32_t n,
                            const uint32_t* as, const uint32_t* ae, uint64_t na, const uint32_t* counts,
                            const uint32_t* firsts, const uint64_t* offsets, uint32_t* pa, uint32_t* pb,
                            uint64_t max_pairs, uint32_t* status, hipStream_t s);

// rmi.hip
size_t rmi_workspace_bytes();
// Also writes the line heads of both arrays (heads_len(n) words each).
int launch_rmi_build2(const uint32_t* keys0, const uint32_t* keys1, uint64_t n, bits_rmi_model* m0,
                      bits_rmi_model* m1, uint32_t* heads0, uint32_t* heads1, const bits_train& tr, void* ws,
                      hipStream_t s);
hipError_t launch_rmi_leaf_grad(const float* u, const float* t, uint32_t m, const float* params, float* grad,
                                float* loss, hipStream_t s);

}  // namespace bits
