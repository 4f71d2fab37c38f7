// Search kernels of libbits.so (gfx950): ICount (Algorithm 1) over the plain
// index (LDS Eytzinger top tree + bisection of the bucket in HBM) or the
// learned CDF index (route -> leaf model -> one cooperative 128-byte line
// probe at the predicted rank -> bisection of what is left of the error
// window -> verification), the per-query / total counters (Algorithm 2),
// the Monte-Carlo loop of Sec. 3.2 as one persistent launch, the
// batched-pairs kernel, projection and small helpers.
//
// Every lane carries QPL queries, i.e. 2*QPL independent search chains (one
// over B_S for a.end, one over B_E for a.start per query); the chains advance
// in lock-step so their dependent loads overlap.  Loads of the sorted arrays
// that have no reuse are non-temporal, so the learned leaf records and the
// shared top of the bisections stay in L2.
#include <mutex>
#include <unordered_map>

#include "bits_internal.hpp"

// Waves per SIMD the search kernels are compiled for (caps their VGPRs).
#ifndef BITS_SEARCH_WAVES_PER_EU
#define BITS_SEARCH_WAVES_PER_EU 4
#endif
#define BITS_SEARCH_KERNEL __global__ void __launch_bounds__(1024) \
    __attribute__((amdgpu_waves_per_eu(BITS_SEARCH_WAVES_PER_EU)))

namespace bits {

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ uint32_t ld_key(const uint32_t* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ bisection
// For each chain c: base[c] += #{K_c[base[c] .. base[c] + len[c]) < x[c]};
// K_c is B_S for even c and B_E for odd c.  Leaves len[c] == 0.  The first
// `hot` probes are ordinary (cached) loads, later ones non-temporal.
template <int NC>
__device__ __forceinline__ void bisect_multi(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ ke,
                                             uint32_t (&base)[NC], uint32_t (&len)[NC], const uint32_t (&x)[NC],
                                             uint32_t hot) {
    for (uint32_t step = 0;; ++step) {
        uint32_t v[NC];
        bool any = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t* K = (c & 1) ? ke : ks;
            const uint32_t half = len[c] >> 1;
            // a finished chain reads key 0 (always in bounds); its value is unused.
            // A probe is streamed (non-temporal) unless it is one of the shared
            // first probes or the range is down to ~2 lines, which the next
            // probes read again.
            const uint32_t idx = half ? base[c] + half - 1 : 0u;
            if (step < hot || len[c] <= 64u)
                v[c] = ld_key<false>(K + idx);
            else
                v[c] = ld_key<true>(K + idx);
            any |= half != 0;
        }
        if (!any) break;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t half = len[c] >> 1;
            if (half) {
                base[c] += (v[c] < x[c]) ? half : 0u;
                len[c] -= half;
            }
        }
    }
    uint32_t v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t* K = (c & 1) ? ke : ks;
        v[c] = len[c] ? ld_key<false>(K + base[c]) : 0u;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (len[c]) base[c] += (v[c] < x[c]) ? 1u : 0u;
        len[c] = 0;
    }
}

// ------------------------------------------------------------------ line probe
// For every lane's chains with start[c] != kNoLine:
//   cnt[c] = #{i in [start[c], start[c] + 32) : K_c[i] < x[c]},
// start a multiple of 4 (16-byte aligned).  On a sorted array probed at a
// 128-byte line (start = 32 line), 0 < cnt < 32 pins the global lower bound
// to start + cnt exactly.  The sorted arrays are 256-byte aligned inside the
// reference block and the rest of their last 128-byte line holds 0xFFFFFFFF
// (never < x), so every line read is in bounds and needs no masking; the
// line-head arrays are padded the same way.  The whole wave cooperates:
// kProbeLanes lanes read one 32-word window with 16-byte loads (each load
// instruction covering a contiguous 16 * kProbeLanes bytes of every window
// it touches) and their partial counts are summed with DPP lane moves.  NT
// selects non-temporal loads (data lines, no reuse) over cached ones (line
// heads, kept in L2).  `scr` is this wave's LDS scratch of 4 * NC * 64
// words.  Must be called by all 64 lanes.
constexpr uint32_t kNoLine = 0xFFFFFFFFu;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t count_lt4(u32x4 v, uint32_t x) {
    return (v.x < x ? 1u : 0u) + (v.y < x ? 1u : 0u) + (v.z < x ? 1u : 0u) + (v.w < x ? 1u : 0u);
}

#ifndef BITS_QUAD_SHFL
#define BITS_QUAD_SHFL 0
#endif
#ifndef BITS_PROBE_LANES
#define BITS_PROBE_LANES 8
#endif
constexpr int kProbeLanes = BITS_PROBE_LANES;        // lanes reading one line

// Sum over each aligned group of L lanes, in every lane of the group.
template <int L>
__device__ __forceinline__ uint32_t group_sum(uint32_t t) {
    if constexpr (L >= 2) t += dpp_u32<0xB1>(t);    // quad_perm [1,0,3,2]
    if constexpr (L >= 4) t += dpp_u32<0x4E>(t);    // quad_perm [2,3,0,1]
    if constexpr (L >= 8) t += dpp_u32<0x141>(t);   // row_half_mirror
    return t;
}

// WIN words per window (32: a 128-byte line; 16: half a line), read by
// LANES lanes with WIN / (4 LANES) 16-byte loads each.
template <int NC, bool NT, int WIN = 32, int LANES = kProbeLanes>
__device__ __forceinline__ void probe_lines(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ ke,
                                            const uint32_t (&start)[NC], const uint32_t (&x)[NC],
                                            uint32_t (&cnt)[NC], uint32_t* scr) {
    constexpr int kLanes = LANES;
    constexpr int kLoads = WIN / 4 / LANES;      // 16-byte loads per lane per window
    constexpr int kGroups = kWave / LANES;       // windows per instruction
    static_assert(kLoads >= 1 && WIN % (4 * LANES) == 0, "window geometry");
    const uint32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        // an idle lane probes words 0..31 against x = 0 (counts nothing, result unused)
        const bool on = start[c] != kNoLine;
        scr[(2 * c + 0) * 2 * kWave + 2 * lane] = on ? start[c] : 0u;
        scr[(2 * c + 0) * 2 * kWave + 2 * lane + 1] = on ? x[c] : 0u;
    }
    wave_lds_sync();
    const uint32_t sub = lane % kLanes, grp = lane / kLanes;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t* K = (c & 1) ? ke : ks;
        u32x4 v[kLanes][kLoads];
        uint32_t xx[kLanes];
#pragma unroll
        for (int j = 0; j < kLanes; ++j) {
            const uint32_t owner = (uint32_t)j * kGroups + grp;
            const uint2 lx = *reinterpret_cast<const uint2*>(scr + (2 * c + 0) * 2 * kWave + 2 * owner);
            xx[j] = lx.y;
            // load k covers bytes [16 k L, 16 (k + 1) L) of the window (L lanes), contiguous per group
            const u32x4* P = reinterpret_cast<const u32x4*>(K + lx.x) + sub;
#pragma unroll
            for (int k = 0; k < kLoads; ++k) {
                if constexpr (NT)
                    v[j][k] = __builtin_nontemporal_load(P + k * kLanes);
                else
                    v[j][k] = P[k * kLanes];
            }
        }
#pragma unroll
        for (int j = 0; j < kLanes; ++j) {
            const uint32_t owner = (uint32_t)j * kGroups + grp;
            uint32_t t = 0;
#pragma unroll
            for (int k = 0; k < kLoads; ++k) t += count_lt4(v[j][k], xx[j]);
            t = group_sum<LANES>(t);
            if (sub == 0) scr[(2 * c + 1) * 2 * kWave + owner] = t;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < NC; ++c) cnt[c] = scr[(2 * c + 1) * 2 * kWave + lane];
    wave_lds_sync();
}

// ------------------------------------------------------------------ leaf model
// Evaluates the leaf of every lane's chains cooperatively, 4 lanes per leaf:
// in pass p the quad k of the wave serves owner lane 16 p + k.  Lane q of
// the quad reads 16 bytes at 16 q and 16 bytes at 64 + 16 q of the owner's
// 128-byte leaf record (each instruction covers 64 contiguous bytes per
// quad): two header words and the binary16 weights of hidden units
// 4q..4q+3.  The quad adds its 4 partial sums with two lane-pair moves (the
// order b2 + ((s0 + s1) + (s2 + s3)) of rmi_pred_offset) and writes, per
// owner, {kmin, kmax, rlo, cnt, y, err} to LDS.  `scr` is this wave's
// scratch; chain c uses words [c * kLeafScr, (c + 1) * kLeafScr): 128 words
// of (leaf, x) pairs, then 6 result words per owner.  Must be called by all
// 64 lanes.

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_quad(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int NC>
__device__ __forceinline__ void quad_leaves(const bits_rmi_model* __restrict__ rmi, const uint32_t (&leaf)[NC],
                                            const uint32_t (&x)[NC], uint32_t* scr) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        scr[c * kLeafScr + 2 * lane] = leaf[c];
        scr[c * kLeafScr + 2 * lane + 1] = x[c];
    }
    wave_lds_sync();
    const uint32_t quad = lane >> 2, q = lane & 3u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const bits_rmi_model* M = rmi + (c & 1);
        uint4 A[4], B[4];
        uint32_t xo[4];
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const uint32_t owner = (uint32_t)pass * 16u + quad;
            const uint2 lx = *reinterpret_cast<const uint2*>(scr + c * kLeafScr + 2 * owner);
            xo[pass] = lx.y;
            const uint4* rec = reinterpret_cast<const uint4*>(M->leaf + lx.x);
            A[pass] = rec[q];
            B[pass] = rec[4 + q];
        }
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const uint32_t owner = (uint32_t)pass * 16u + quad;
            // kmin from quad lane 0, kinv from quad lane 2 (lane exchanges: a quad_perm
            // broadcast DPP folded into the using instruction gave wrong values here)
            const uint32_t kmin = (uint32_t)__shfl((int)A[pass].x, (int)(lane & ~3u));
            const uint32_t kinvb = (uint32_t)__shfl((int)A[pass].x, (int)((lane & ~3u) + 2u));
            const float u = rmi_u(xo[pass] - kmin, __uint_as_float(kinvb));
            const float w1[4] = {h2f(A[pass].z & 0xFFFFu), h2f(A[pass].z >> 16), h2f(A[pass].w & 0xFFFFu),
                                 h2f(A[pass].w >> 16)};
            const float b1[4] = {h2f(B[pass].x & 0xFFFFu), h2f(B[pass].x >> 16), h2f(B[pass].y & 0xFFFFu),
                                 h2f(B[pass].y >> 16)};
            const float w2[4] = {h2f(B[pass].z & 0xFFFFu), h2f(B[pass].z >> 16), h2f(B[pass].w & 0xFFFFu),
                                 h2f(B[pass].w >> 16)};
            float t = rmi_quad_partial(w1, b1, w2, u);
#if BITS_QUAD_SHFL
            t += __shfl_xor(t, 1);   // s0+s1, s2+s3
            t += __shfl_xor(t, 2);   // (s0+s1)+(s2+s3)
#else
            t += __uint_as_float(dpp_quad<0xB1>(__float_as_uint(t)));   // s0+s1, s2+s3
            t += __uint_as_float(dpp_quad<0x4E>(__float_as_uint(t)));   // (s0+s1)+(s2+s3)
#endif
            // lane 0: {kmin, kmax}; 1: {rlo, cnt}; 2: y = b2 + sum; 3: err
            uint32_t* res = scr + c * kLeafScr + 2 * kWave + 6 * owner;
            if (q < 2)
                *reinterpret_cast<uint2*>(res + 2 * q) = make_uint2(A[pass].x, A[pass].y);
            else if (q == 2)
                res[4] = __float_as_uint(__uint_as_float(A[pass].y) + t);
            else
                res[5] = A[pass].x;
        }
    }
    wave_lds_sync();
}


// ------------------------------------------------------------------ ICount
// first = #{B_S <= a.end} = #{B_S < a.end + 1}; last = #{B_E < a.start};
// count = first - last (Sec. 2.1).  a.end == 2^32-1 means first = |B|.
//
// A lane without a query (past the end of its tile or round, or a query
// left out) still runs the wave-cooperative searches with the interval
// [0, kIdleEnd]: both search keys are then 0, below every key routed to a
// leaf, so the learned searches resolve it from the leaf header without a
// single probe.  (An idle [0, 0] would search B_S for 1, which a reference
// with many intervals starting at 0 turns into a fallback bisection.)
constexpr uint32_t kIdleEnd = 0xFFFFFFFFu;

// Bisection probes kept in L2 on the plain path: the first few probes of a
// bucket are shared by every query landing in it.
constexpr uint32_t kPlainHotSteps = 3;

// The LDS top tree's bucket for each chain: the lower bound #{K_c < x[c]}
// lies in [base[c], base[c] + len[c]] (the whole array when depth is 0).
template <int NC>
__device__ __forceinline__ void tree_bucket(const SearchArgs& sa, const uint32_t* lds, const uint32_t (&x)[NC],
                                            uint32_t (&base)[NC], uint32_t (&len)[NC]) {
    const uint32_t d = sa.depth;
    if (d) {
        const uint32_t m = 1u << d;
        uint32_t k[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) k[c] = 1u;
        for (uint32_t l = 0; l < d; ++l) {
#pragma unroll
            for (int c = 0; c < NC; ++c) k[c] = 2u * k[c] + (lds[(c & 1) * m + k[c]] < x[c] ? 1u : 0u);
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint64_t qb = k[c] - m;
            base[c] = (uint32_t)((qb * sa.n) >> d);
            len[c] = (uint32_t)(((qb + 1) * sa.n) >> d) - base[c];
        }
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            base[c] = 0u;
            len[c] = sa.n;
        }
    }
}

template <int QPL>
__device__ __forceinline__ void icount_plain(const SearchArgs& sa, const uint32_t* lds,
                                             const uint32_t (&as)[QPL], const uint32_t (&ae)[QPL],
                                             uint32_t (&cnt)[QPL],
                                             uint32_t (&fst)[QPL]) {
    constexpr int NC = 2 * QPL;
    uint32_t x[NC], base[NC], len[NC];
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        x[2 * q] = ae[q] + 1u;
        x[2 * q + 1] = as[q];
    }
    tree_bucket<NC>(sa, lds, x, base, len);
    bisect_multi<NC>(sa.bs, sa.be, base, len, x, kPlainHotSteps);
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        const uint32_t first = (ae[q] == 0xFFFFFFFFu) ? sa.n : base[2 * q];
        cnt[q] = first - base[2 * q + 1];
        fst[q] = first;
    }
}

// Leaf stage of both learned searches for NC chains (even chains search B_S,
// odd ones B_E): route each key and evaluate its leaf model.  Per chain:
// the leaf's rank range [rlo, rhi]; inside = (kmin < x <= kmax); pred = the
// model's rank for an inside key, else the resolved rank (rhi if x > kmax,
// rlo if x <= kmin: routing is monotone, so no key of another leaf lies
// between); err = the leaf's packed error bounds.  Must be called by all 64
// lanes.
template <int NC>
__device__ __forceinline__ void leaf_stage(const SearchArgs& sa, uint32_t* scr, const uint32_t (&x)[NC],
                                           uint32_t (&rlo)[NC], uint32_t (&rhi)[NC], uint32_t (&pred)[NC],
                                           uint32_t (&err)[NC], bool (&inside)[NC]) {
    uint32_t leaf[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const bits_rmi_model* M = sa.rmi + (c & 1);
        leaf[c] = rmi_route(M->root_a, M->root_b, x[c]);
    }
    quad_leaves<NC>(sa.rmi, leaf, x, scr);
    const uint32_t lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t* res = scr + c * kLeafScr + 2 * kWave + 6 * lane;
        const uint2 ra = *reinterpret_cast<const uint2*>(res), rb = *reinterpret_cast<const uint2*>(res + 2),
                    rc = *reinterpret_cast<const uint2*>(res + 4);
        // ra = {kmin, kmax}, rb = {rlo, cnt}, rc = {y, err}
        // clamped to [0, n] so that no header value can send a search out of bounds
        rhi[c] = min(rb.x + rb.y, sa.n);
        rlo[c] = min(rb.x, rhi[c]);
        err[c] = rc.y;
        inside[c] = x[c] > ra.x && x[c] <= ra.y;
        if (inside[c])
            pred[c] = min(rlo[c] + (uint32_t)rmi_offset_from_y(__uint_as_float(rc.x), rb.y), rhi[c]);
        else
            pred[c] = x[c] > ra.y ? rhi[c] : rlo[c];
    }
}

// Learned search, leaf part: either the resolved rank (base, win = false) or
// the recorded error window [wl, wr] around the prediction (base = wl).  Must
// be called by all 64 lanes.
template <int NC>
__device__ __forceinline__ void learned_windows(const SearchArgs& sa, uint32_t* scr, const uint32_t (&x)[NC],
                                                uint32_t (&base)[NC], uint32_t (&wl)[NC], uint32_t (&wr)[NC],
                                                uint32_t (&rlo)[NC], uint32_t (&rhi)[NC], bool (&win)[NC]) {
    uint32_t pred[NC], err[NC];
    leaf_stage<NC>(sa, scr, x, rlo, rhi, pred, err, win);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        base[c] = pred[c];
        wl[c] = wr[c] = 0;
        if (win[c]) {
            const int32_t p = (int32_t)pred[c];
            const int32_t lo = p - (int32_t)(err[c] & 0xFFFFu), hi = p + (int32_t)(err[c] >> 16);
            wl[c] = (uint32_t)max(lo, (int32_t)rlo[c]);
            wr[c] = (uint32_t)min(hi, (int32_t)rhi[c]);
            if (wr[c] < wl[c]) wr[c] = wl[c];
            base[c] = wl[c];
        }
    }
}

// Learned search through the line heads (H[j] = K[32 j], the first key of
// every 128-byte line of a sorted array, padded with 0xFFFFFFFF).  With
// r = #{K < x} the lower bound and j = #{H < x} = ceil(r / 32), the lower
// bound lies in line j - 1: r = 32 (j - 1) + #{keys < x in that line}, or
// r = 0 when j = 0.  Per chain:
//   1. leaf model -> predicted rank -> line p = pred / 32;
//   2. one cooperative probe of a window of kHeadWin heads with p at least
//      kHeadLead lines from either end (cached loads: a workgroup that serves
//      one part of the key range keeps that part's heads in its L2) gives j
//      exactly when 0 < count < kHeadWin (or the window starts at 0);
//   3. otherwise the window next to it on the side the count points to is
//      probed (only if some lane of the wave needs it), and what is still
//      unresolved is bisected over the heads of the leaf's rank range (the
//      fallback counter counts these);
//   4. one cooperative non-temporal probe of line j - 1 gives r.
// Exact whatever the model predicts (no verification step), and every read
// stays inside the arrays whatever the leaf records hold.  Must be called by
// all 64 lanes.
#ifndef BITS_HEAD_WIN
#define BITS_HEAD_WIN 16
#endif
#ifndef BITS_HEAD_ALIGN
#define BITS_HEAD_ALIGN 8
#endif
#ifndef BITS_HEAD_LEAD
#define BITS_HEAD_LEAD 4
#endif
constexpr uint32_t kHeadWin = BITS_HEAD_WIN;      // heads per window
constexpr uint32_t kHeadAlign = BITS_HEAD_ALIGN;  // window start is a multiple of this (>= 4: 16-byte loads)
constexpr uint32_t kHeadLead = BITS_HEAD_LEAD;    // the predicted line sits >= this many lines into the window
constexpr int kHeadLanes = kHeadWin == 32 ? kProbeLanes : 4;
// windows reach at most 2 kHeadWin - kHeadLead heads past the predicted line
// (second window on the right), which the >= 32 padding heads cover
static_assert(kHeadLead + kHeadAlign <= kHeadWin && 2 * kHeadWin <= 32 + kHeadLead && kHeadAlign % 4 == 0,
              "head window");

// j from a window count: resolved (0 < cnt < kHeadWin, or cnt = 0 at the
// start of the array), else left (j <= w) or right (j >= w + kHeadWin).
enum : uint32_t { kHeadHit = 0, kHeadLeft = 1, kHeadRight = 2 };
__device__ __forceinline__ uint32_t head_outcome(uint32_t w, uint32_t cnt) {
    if (cnt >= kHeadWin) return kHeadRight;
    return (cnt == 0u && w != 0u) ? kHeadLeft : kHeadHit;
}

// Learned count: the leaf's recorded error window [wl, wr] holds the lower
// bound r = #{K < x}, so j = #{H < x} = ceil(r / 32) over the line heads
// (H[j] = K[32 j], kept in L2 / the Infinity Cache) lies in [ceil(wl / 32),
// ceil(wr / 32)].  One cooperative probe of the kHeadWin heads starting at
// or below ceil(wl / 32) - 1 resolves j when that range fits in the probe,
// else the heads of the leaf's whole range [rlo, rhi] are bisected; a probe
// whose count shows that j left the window (the model erred past its
// recorded error) falls back to that bisection too, and is counted.  One
// cooperative probe of line j - 1 then gives r (r = 0 when j = 0).  Must be
// called by all 64 lanes.
template <int QPL>
__device__ __forceinline__ void icount_learned(const SearchArgs& sa, uint32_t* scr, const uint32_t (&as)[QPL],
                                               const uint32_t (&ae)[QPL], uint32_t (&cnt)[QPL],
                                               uint32_t (&fst)[QPL]) {
    constexpr int NC = 2 * QPL;
    uint32_t x[NC], base[NC], wl[NC], wr[NC], rlo[NC], rhi[NC];
    bool win[NC];
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        x[2 * q] = ae[q] + 1u;
        x[2 * q + 1] = as[q];
    }
    learned_windows<NC>(sa, scr, x, base, wl, wr, rlo, rhi, win);
    const uint32_t m = (sa.n + 31u) >> 5;     // heads in use
    uint32_t w[NC], pc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t jlo = min((wl[c] + 31u) >> 5, m), jhi = min((wr[c] + 31u) >> 5, m);
        const uint32_t w0 = (jlo > 0u ? jlo - 1u : 0u) & ~(kHeadAlign - 1u);
        w[c] = (win[c] && jhi < w0 + kHeadWin) ? w0 : kNoLine;
    }
    probe_lines<NC, false, kHeadWin, kHeadLanes>(sa.hs, sa.he, w, x, pc, scr);
    uint32_t j[NC], jl[NC];
    bool again = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        j[c] = 0u;
        jl[c] = 0u;
        if (!win[c]) continue;
        if (w[c] != kNoLine && head_outcome(w[c], pc[c]) == kHeadHit) {
            j[c] = w[c] + pc[c];
            continue;
        }
        if (w[c] != kNoLine) atomicAdd(sa.fallbacks, 1ull);   // the window missed
        j[c] = min((rlo[c] + 31u) >> 5, m);
        jl[c] = min((rhi[c] + 31u) >> 5, m) - j[c];
        again = true;
    }
    if (__ballot(again)) bisect_multi<NC>(sa.hs, sa.he, j, jl, x, 32u);
    uint32_t dw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) dw[c] = (win[c] && j[c] != 0u) ? (min(j[c], m) - 1u) * 32u : kNoLine;
    probe_lines<NC, true>(sa.bs, sa.be, dw, x, pc, scr);
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (win[c]) base[c] = dw[c] == kNoLine ? 0u : dw[c] + pc[c];
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        const uint32_t first = (ae[q] == 0xFFFFFFFFu) ? sa.n : base[2 * q];
        cnt[q] = first - base[2 * q + 1];
        fst[q] = first;
    }
}

template <int QPL>
__device__ __forceinline__ void icount_heads(const SearchArgs& sa, uint32_t* scr, const uint32_t (&as)[QPL],
                                             const uint32_t (&ae)[QPL], uint32_t (&cnt)[QPL],
                                             uint32_t (&fst)[QPL]) {
    constexpr int NC = 2 * QPL;
    uint32_t x[NC], rlo[NC], rhi[NC], pred[NC], err[NC], w[NC], pc[NC], st[NC];
    bool inside[NC];
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        x[2 * q] = ae[q] + 1u;
        x[2 * q + 1] = as[q];
    }
    leaf_stage<NC>(sa, scr, x, rlo, rhi, pred, err, inside);
    const uint32_t m = (sa.n + 31u) >> 5;     // heads in use
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const uint32_t p = pred[c] >> 5;
        w[c] = inside[c] ? ((p > kHeadLead ? p - kHeadLead : 0u) & ~(kHeadAlign - 1u)) : kNoLine;
    }
    probe_lines<NC, false, kHeadWin, kHeadLanes>(sa.hs, sa.he, w, x, pc, scr);
    bool again = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        st[c] = w[c] == kNoLine ? kHeadHit : head_outcome(w[c], pc[c]);
        pc[c] = w[c] + pc[c];                 // j when resolved
        if (st[c] == kHeadLeft) w[c] = w[c] >= kHeadWin ? w[c] - kHeadWin : 0u;
        if (st[c] == kHeadRight) w[c] += kHeadWin;
        again |= st[c] != kHeadHit;
    }
    uint32_t j[NC], jl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        j[c] = pc[c];
        jl[c] = 0;
    }
    if (__ballot(again)) {
        uint32_t w2[NC], pc2[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) w2[c] = st[c] != kHeadHit ? w[c] : kNoLine;
        probe_lines<NC, false, kHeadWin, kHeadLanes>(sa.hs, sa.he, w2, x, pc2, scr);
        uint32_t nmiss = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (st[c] == kHeadHit) continue;
            const uint32_t o = head_outcome(w2[c], pc2[c]);
            if (o == kHeadHit) {
                j[c] = w2[c] + pc2[c];
                continue;
            }
            // still unresolved: j lies in [ceil(rlo/32), ceil(rhi/32)] (rlo <= r <= rhi),
            // on the side of w2 the count points to
            const uint32_t hi = min((rhi[c] + 31u) >> 5, m), lo = min((rlo[c] + 31u) >> 5, hi);
            uint32_t a = lo, b = hi;
            if (o == kHeadLeft && w2[c] >= lo && w2[c] <= hi) b = w2[c];
            if (o == kHeadRight && w2[c] + kHeadWin >= lo && w2[c] + kHeadWin <= hi) a = w2[c] + kHeadWin;
            j[c] = a;
            jl[c] = b - a;
            ++nmiss;
        }
        if (nmiss) {
            atomicAdd(sa.fallbacks, (unsigned long long)nmiss);
            bisect_multi<NC>(sa.hs, sa.he, j, jl, x, 32u);
        }
    }
    uint32_t dw[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        dw[c] = (inside[c] && j[c] != 0u) ? (min(j[c], m) - 1u) * 32u : kNoLine;
    probe_lines<NC, true>(sa.bs, sa.be, dw, x, pc, scr);
    uint32_t r[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) r[c] = !inside[c] ? pred[c] : (dw[c] == kNoLine ? 0u : dw[c] + pc[c]);
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        const uint32_t first = (ae[q] == 0xFFFFFFFFu) ? sa.n : r[2 * q];
        cnt[q] = first - r[2 * q + 1];
        fst[q] = first;
    }
}

// Plain search with the 32-key node tier, no model: the line heads
// H[j] = K[32 j] (1/32 of the array, cached in L2 / the Infinity Cache) sit
// between the LDS top tree and the sorted array.  The tree narrows the lower
// bound r = #{K < x} to its bucket [base, base + len]; then
// j = #{H < x} = ceil(r / 32) lies in [ceil(base / 32), ceil((base + len) / 32)]
// (every head before that range is < x, every head after it >= x), which is
// bisected over the heads; one cooperative probe of line j - 1 then gives r
// (r = 0 when j = 0), as in the head search of the Monte-Carlo path.  `scr`
// is this wave's probe scratch (tiered_scratch_words(QPL) words).  Must be
// called by all 64 lanes.
template <int QPL>
__device__ __forceinline__ void icount_tiered(const SearchArgs& sa, const uint32_t* lds, uint32_t* scr,
                                              const uint32_t (&as)[QPL], const uint32_t (&ae)[QPL],
                                              uint32_t (&cnt)[QPL], uint32_t (&fst)[QPL]) {
    constexpr int NC = 2 * QPL;
    uint32_t x[NC], base[NC], len[NC];
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        x[2 * q] = ae[q] + 1u;
        x[2 * q + 1] = as[q];
    }
    tree_bucket<NC>(sa, lds, x, base, len);
    uint32_t j[NC], jl[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        j[c] = (uint32_t)(((uint64_t)base[c] + 31u) >> 5);
        jl[c] = (uint32_t)(((uint64_t)base[c] + len[c] + 31u) >> 5) - j[c];
    }
    bisect_multi<NC>(sa.hs, sa.he, j, jl, x, 32u);
    uint32_t dw[NC], pc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) dw[c] = j[c] ? (j[c] - 1u) * 32u : kNoLine;
    probe_lines<NC, true>(sa.bs, sa.be, dw, x, pc, scr);
#pragma unroll
    for (int q = 0; q < QPL; ++q) {
        const uint32_t rs = dw[2 * q] == kNoLine ? 0u : dw[2 * q] + pc[2 * q];
        const uint32_t re = dw[2 * q + 1] == kNoLine ? 0u : dw[2 * q + 1] + pc[2 * q + 1];
        const uint32_t first = (ae[q] == 0xFFFFFFFFu) ? sa.n : rs;
        cnt[q] = first - re;
        fst[q] = first;
    }
}

template <int QPL, bool LEARNED>
__device__ __forceinline__ void icount(const SearchArgs& sa, uint32_t* lds, const uint32_t (&as)[QPL],
                                       const uint32_t (&ae)[QPL], uint32_t (&cnt)[QPL], uint32_t (&fst)[QPL]) {
    if constexpr (LEARNED)
        icount_learned<QPL>(sa, lds + (threadIdx.x / kWave) * probe_scratch_words(QPL), as, ae, cnt, fst);
    else
        icount_plain<QPL>(sa, lds, as, ae, cnt, fst);
}


// ------------------------------------------------------------------ counting kernel
// Persistent grid over tiles of blockDim*QPL queries; query i of a tile is
// loaded by lane (i mod blockDim), so every load of a query round is
// coalesced.  Totals: uint64 wave sum, one atomic per wave.

// MODE: kModePlain (LDS tree + bisection), kModeLearned (learned index,
// error-window head probe + one line) or kModeTiered (LDS tree + line-head tier + one line).
template <int QPL, int MODE>
BITS_SEARCH_KERNEL k_count(SearchArgs sa, const uint32_t* __restrict__ a_start,
                                                const uint32_t* __restrict__ a_end, uint64_t na,
                                                uint32_t* __restrict__ counts, uint32_t* __restrict__ firsts,
                                                unsigned long long* total) {
    extern __shared__ uint32_t lds[];
    if (MODE != kModeLearned) {
        stage_tree(lds, sa.tree, sa.tree_stride, sa.depth);
        __syncthreads();
    }
    const uint64_t tile = (uint64_t)blockDim.x * QPL;
    const uint64_t ntiles = (na + tile - 1) / tile;
    uint64_t acc = 0;
    uint32_t bad = 0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        uint32_t as[QPL], ae[QPL], cnt[QPL];
        bool valid[QPL];
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint64_t i = t * tile + (uint64_t)q * blockDim.x + threadIdx.x;
            valid[q] = i < na;
            as[q] = valid[q] ? a_start[i] : 0u;
            ae[q] = valid[q] ? a_end[i] : kIdleEnd;
            if (as[q] > ae[q]) {
                bad = 1;
                valid[q] = false;
                ae[q] = as[q];
            }
        }
        uint32_t fst[QPL];
        if constexpr (MODE == kModeTiered)
            icount_tiered<QPL>(sa, lds, lds + tree_lds_words(sa.depth) + (threadIdx.x / kWave) * tiered_scratch_words(QPL),
                               as, ae, cnt, fst);
        else
            icount<QPL, MODE == kModeLearned>(sa, lds, as, ae, cnt, fst);
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint64_t i = t * tile + (uint64_t)q * blockDim.x + threadIdx.x;
            const uint32_t c = valid[q] ? cnt[q] : 0u;
            if (counts && i < na) counts[i] = c;
            if (firsts && i < na) firsts[i] = fst[q];
            acc += c;
        }
    }
    if (bad) atomicOr(sa.status, BITS_FLAG_INTERVAL);
    if (total) {
        acc = wave_sum_u64(acc);
        if ((threadIdx.x & (kWave - 1)) == 0 && acc) atomicAdd(total, (unsigned long long)acc);
    }
}

// ------------------------------------------------------------------ decision
// Sec. 1.1, sub-problem 1: does any a intersect any b?  The counting loop
// with an early exit: a workgroup checks the shared flag before each tile
// and stops once some query has a non-zero count.  *witness receives the
// smallest index with a hit among the tiles that ran (initialised to
// 2^64 - 1 by the caller).
template <int QPL, bool LEARNED>
BITS_SEARCH_KERNEL k_decide(SearchArgs sa, const uint32_t* __restrict__ a_start, const uint32_t* __restrict__ a_end,
                            uint64_t na, uint32_t* found, unsigned long long* witness) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t stop;
    if (!LEARNED) stage_tree(lds, sa.tree, sa.tree_stride, sa.depth);
    __syncthreads();
    const uint64_t tile = (uint64_t)blockDim.x * QPL;
    const uint64_t ntiles = (na + tile - 1) / tile;
    uint32_t bad = 0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (threadIdx.x == 0) stop = __hip_atomic_load(found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (stop) break;
        uint32_t as[QPL], ae[QPL], cnt[QPL], fst[QPL];
        bool valid[QPL];
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint64_t i = t * tile + (uint64_t)q * blockDim.x + threadIdx.x;
            valid[q] = i < na;
            as[q] = valid[q] ? a_start[i] : 0u;
            ae[q] = valid[q] ? a_end[i] : kIdleEnd;
            if (as[q] > ae[q]) {
                bad = 1;
                valid[q] = false;
                ae[q] = as[q];
            }
        }
        icount<QPL, LEARNED>(sa, lds, as, ae, cnt, fst);
        bool hit = false;
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            if (valid[q] && cnt[q]) {
                atomicMin(witness, (unsigned long long)(t * tile + (uint64_t)q * blockDim.x + threadIdx.x));
                hit = true;
            }
        }
        if (hit) atomicOr(found, 1u);
        __syncthreads();   // every lane has read `stop` before it is rewritten
    }
    if (bad) atomicOr(sa.status, BITS_FLAG_INTERVAL);
}

// ------------------------------------------------------------------ Monte-Carlo
// The per-query table (off, span, len, idx) is grouped by chromosome (see
// k_mc_prepare): position j holds query idx[j].  Work item = (tile of
// blockDim*QPL table positions, chunk of consecutive shuffles), walked by a
// persistent grid.  A workgroup reads its tile's table entries once per item
// and runs every shuffle of the chunk on them.  Query i of shuffle s starts at
// off_i + floor(u * span_i / 2^64), u = the first two Philox words of counter
// g = (s0 + s) * na + i.  Per-shuffle wave sums are added in LDS and flushed
// with one global atomic per shuffle per item.  OBSERVED counts the
// unshuffled queries instead (same exclusion of queries with span 0, i.e.
// outside their chromosome).
//
// XCD-aware split: workgroups are dispatched round-robin over the 8 XCDs,
// so workgroup b runs on XCD b mod 8.  The tiles are cut into 8 contiguous
// groups and group x is served only by workgroups b = x (mod 8).  A shuffle
// keeps every query inside its chromosome, and the table is grouped by
// chromosome, so each XCD searches one contiguous part of B and its L2 holds
// that part's leaves and line heads.  (With another placement the split only
// costs locality, never correctness.)
constexpr uint32_t kMaxChunk = 64;
constexpr uint32_t kXcds = 8;

template <int QPL, bool LEARNED>
__device__ __forceinline__ void icount_mc(const SearchArgs& sa, uint32_t* lds, const uint32_t (&as)[QPL],
                                          const uint32_t (&ae)[QPL], uint32_t (&cnt)[QPL]) {
    uint32_t fst[QPL];
    if constexpr (LEARNED)
        icount_heads<QPL>(sa, lds + (threadIdx.x / kWave) * probe_scratch_words(QPL), as, ae, cnt, fst);
    else
        icount_plain<QPL>(sa, lds, as, ae, cnt, fst);
}

template <int QPL, bool LEARNED, bool OBSERVED>
BITS_SEARCH_KERNEL k_mc(SearchArgs sa, const uint32_t* __restrict__ a_start, const uint32_t* __restrict__ a_end,
         const uint32_t* __restrict__ off, const uint32_t* __restrict__ span, const uint32_t* __restrict__ len,
         const uint32_t* __restrict__ idx, uint64_t na, uint64_t seed, uint64_t s0, uint64_t nshuf, uint64_t tiles,
         uint32_t chunk, unsigned long long* __restrict__ totals) {
    extern __shared__ uint32_t lds[];
    __shared__ unsigned long long acc[kMaxChunk];
    if (!LEARNED) stage_tree(lds, sa.tree, sa.tree_stride, sa.depth);
    for (uint32_t k = threadIdx.x; k < kMaxChunk; k += blockDim.x) acc[k] = 0ull;
    __syncthreads();
    const uint64_t tile = (uint64_t)blockDim.x * QPL;
    const uint64_t nchunks = (nshuf + chunk - 1) / chunk;
    const uint32_t ng = (gridDim.x >= kXcds && tiles >= kXcds) ? kXcds : 1u;
    const uint32_t grp = blockIdx.x % ng, slot = blockIdx.x / ng;
    const uint32_t nslots = (gridDim.x - grp + ng - 1) / ng;   // workgroups b < gridDim with b = grp (mod ng)
    const uint64_t t_lo = tiles * grp / ng, gtiles = tiles * (grp + 1) / ng - t_lo;
    const uint64_t nitems = gtiles * nchunks;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint64_t it = slot; it < nitems; it += nslots) {
        const uint64_t kc = it / gtiles;
        const uint64_t t = t_lo + (it - kc * gtiles);
        uint32_t qo[QPL], qs[QPL], ql[QPL];
        uint64_t qi[QPL];
        bool valid[QPL];
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint64_t pos = t * tile + (uint64_t)q * blockDim.x + threadIdx.x;
            const bool in = pos < na;
            qs[q] = in ? span[pos] : 0u;
            qi[q] = in ? idx[pos] : 0u;
            valid[q] = qs[q] != 0u;
            if (OBSERVED) {
                qo[q] = valid[q] ? a_start[qi[q]] : 0u;
                ql[q] = valid[q] ? a_end[qi[q]] : kIdleEnd;
            } else {
                qo[q] = valid[q] ? off[pos] : 0u;
                ql[q] = valid[q] ? len[pos] : 1u;
            }
        }
        const uint64_t sb = kc * chunk;
        const uint64_t se = min(nshuf, sb + chunk);
        for (uint64_t s = sb; s < se; ++s) {
            uint32_t as[QPL], ae[QPL], cnt[QPL];
#pragma unroll
            for (int q = 0; q < QPL; ++q) {
                if (OBSERVED) {
                    as[q] = qo[q];
                    ae[q] = ql[q];
                } else {
                    const uint64_t g = (s0 + s) * na + qi[q];
                    uint32_t c0 = (uint32_t)g, c1 = (uint32_t)(g >> 32), c2 = 0u, c3 = 0u;
                    philox4x32_10(c0, c1, c2, c3, k0, k1);
                    const uint64_t u = ((uint64_t)c1 << 32) | c0;
                    const uint32_t local = (uint32_t)__umul64hi(u, (uint64_t)qs[q]);
                    as[q] = valid[q] ? qo[q] + local : 0u;
                    ae[q] = valid[q] ? as[q] + ql[q] - 1u : kIdleEnd;
                }
            }
            icount_mc<QPL, LEARNED>(sa, lds, as, ae, cnt);
            uint64_t sum = 0;
#pragma unroll
            for (int q = 0; q < QPL; ++q) sum += valid[q] ? cnt[q] : 0u;
            sum = wave_sum_u64(sum);
            if ((threadIdx.x & (kWave - 1)) == 0 && sum) atomicAdd(&acc[s - sb], (unsigned long long)sum);
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < (uint32_t)(se - sb); k += blockDim.x) {
            const unsigned long long v = acc[k];
            if (v) atomicAdd(totals + sb + k, v);
            acc[k] = 0ull;
        }
        __syncthreads();
    }
}

// Learned Monte-Carlo with placements sorted inside the work item.  An item
// (tile of blockDim/8 table positions, chunk of <= kMaxChunk shuffles)
// generates all its placements, counting-sorts them by start into
// kSortBuckets buckets over the tile's start range in LDS, and searches them
// in that order, so that lanes of a wave share leaf records and often head
// windows: the searches then take fewer L1/L2 requests, the resource that
// bounds the unsorted kernel.  Placements are made twice (histogram, then
// scatter) rather than staged unsorted, to fit LDS.  Totals are sums, so
// the order does not change them.  The placements (start, and query | shuffle
// << 8 in 16 bits) live in dynamic LDS after the per-wave probe scratch.
#ifndef BITS_MC_SORTED
#define BITS_MC_SORTED 1
#endif
#ifndef BITS_MC_SORTED_QPL
#define BITS_MC_SORTED_QPL 1
#endif
constexpr int kSortQpl = BITS_MC_SORTED_QPL;   // placements per lane per search round
constexpr uint32_t kSortBuckets = 1024;
constexpr uint32_t kSortMaxTileQ = 128;
constexpr uint32_t kSortQBits = 8;
__host__ __device__ constexpr uint32_t sort_tile_q(uint32_t block) { return block / 8u; }
__host__ __device__ constexpr size_t sort_lds_bytes(uint32_t block) {
    return (size_t)(block / kWave) * probe_scratch_words(kSortQpl) * 4u + (size_t)sort_tile_q(block) * kMaxChunk * 6u;
}
static_assert((kMaxChunk << kSortQBits) <= 65536, "sort meta");

// In-place exclusive scan of kSortBuckets counters by the whole workgroup;
// returns the total.
__device__ __forceinline__ uint32_t block_scan_buckets(uint32_t* h, uint32_t* wsum) {
    const uint32_t per = kSortBuckets / blockDim.x;            // 1, 2 or 4 (blocks of 1024, 512, 256)
    const uint32_t b0 = threadIdx.x * per;
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    uint32_t mine = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (k < per) v[k] = h[b0 + k];
        mine += v[k];
    }
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
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        if (k < per) h[b0 + k] = pre;
        pre += v[k];
    }
    __syncthreads();
    return tot;
}

BITS_SEARCH_KERNEL k_mc_sorted(SearchArgs sa, const uint32_t* __restrict__ off, const uint32_t* __restrict__ span,
                               const uint32_t* __restrict__ len, const uint32_t* __restrict__ idx, uint64_t na,
                               uint64_t seed, uint64_t s0, uint64_t nshuf, uint64_t tiles, uint32_t chunk,
                               unsigned long long* __restrict__ totals) {
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t hist[kSortBuckets];
    __shared__ uint32_t t_off[kSortMaxTileQ], t_span[kSortMaxTileQ], t_len[kSortMaxTileQ], t_idx[kSortMaxTileQ];
    __shared__ unsigned long long acc[kMaxChunk];
    __shared__ uint32_t wsum[16], lo_key, hi_key;
    const uint32_t tile_q = sort_tile_q(blockDim.x);           // 32, 64 or 128
    uint32_t* scr = lds + (threadIdx.x / kWave) * probe_scratch_words(kSortQpl);
    uint32_t* p_start = lds + (blockDim.x / kWave) * probe_scratch_words(kSortQpl);
    uint16_t* p_meta = reinterpret_cast<uint16_t*>(p_start + tile_q * kMaxChunk);
    for (uint32_t k = threadIdx.x; k < kMaxChunk; k += blockDim.x) acc[k] = 0ull;
    const uint64_t nchunks = (nshuf + chunk - 1) / chunk;
    const uint32_t ng = (gridDim.x >= kXcds && tiles >= kXcds) ? kXcds : 1u;
    const uint32_t grp = blockIdx.x % ng, slot = blockIdx.x / ng;
    const uint32_t nslots = (gridDim.x - grp + ng - 1) / ng;
    const uint64_t t_lo = tiles * grp / ng, gtiles = tiles * (grp + 1) / ng - t_lo;
    const uint64_t nitems = gtiles * nchunks;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    __syncthreads();
    for (uint64_t it = slot; it < nitems; it += nslots) {
        const uint64_t kc = it / gtiles;
        const uint64_t t = t_lo + (it - kc * gtiles);
        const uint64_t sb = kc * chunk;
        const uint32_t nsh = (uint32_t)min((uint64_t)chunk, nshuf - sb);
        // 1. the tile's table and its start range
        if (threadIdx.x == 0) {
            lo_key = 0xFFFFFFFFu;
            hi_key = 0u;
        }
        for (uint32_t k = threadIdx.x; k < kSortBuckets; k += blockDim.x) hist[k] = 0u;
        __syncthreads();
        if (threadIdx.x < tile_q) {
            const uint64_t pos = t * tile_q + threadIdx.x;
            const bool in = pos < na;
            const uint32_t sp = in ? span[pos] : 0u;
            t_span[threadIdx.x] = sp;
            t_off[threadIdx.x] = in ? off[pos] : 0u;
            t_len[threadIdx.x] = in ? len[pos] : 1u;
            t_idx[threadIdx.x] = in ? idx[pos] : 0u;
            if (sp) {
                atomicMin(&lo_key, t_off[threadIdx.x]);
                atomicMax(&hi_key, t_off[threadIdx.x] + (sp - 1u));
            }
        }
        __syncthreads();
        const uint32_t lo = lo_key;
        const uint32_t range = hi_key >= lo ? hi_key - lo : 0u;
        const uint32_t bits = range ? 32u - __clz(range) : 0u;
        const uint32_t shift = bits > 10u ? bits - 10u : 0u;   // (range >> shift) < 1024
        const uint32_t P = tile_q * nsh;
        // 2. histogram of the placements' buckets
        for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) {
            const uint32_t q = p & (tile_q - 1), sh = p / tile_q;
            if (!t_span[q]) continue;
            const uint32_t st = mc_place((s0 + sb + sh) * na + t_idx[q], k0, k1, t_off[q], t_span[q]);
            atomicAdd(&hist[(st - lo) >> shift], 1u);
        }
        __syncthreads();
        const uint32_t nvalid = block_scan_buckets(hist, wsum);
        // 3. the same placements again, scattered into bucket order
        for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) {
            const uint32_t q = p & (tile_q - 1), sh = p / tile_q;
            if (!t_span[q]) continue;
            const uint32_t st = mc_place((s0 + sb + sh) * na + t_idx[q], k0, k1, t_off[q], t_span[q]);
            const uint32_t at = atomicAdd(&hist[(st - lo) >> shift], 1u);
            p_start[at] = st;
            p_meta[at] = (uint16_t)(q | (sh << kSortQBits));
        }
        __syncthreads();
        // 4. the searches, in start order (every lane runs every round: the probes are wave-cooperative)
        for (uint32_t r0 = 0; r0 < nvalid; r0 += kSortQpl * blockDim.x) {
            uint32_t as[kSortQpl], ae[kSortQpl], cnt[kSortQpl], fst[kSortQpl], m[kSortQpl];
            bool valid[kSortQpl];
#pragma unroll
            for (uint32_t q = 0; q < kSortQpl; ++q) {
                const uint32_t p = r0 + q * blockDim.x + threadIdx.x;
                valid[q] = p < nvalid;
                as[q] = valid[q] ? p_start[p] : 0u;
                m[q] = valid[q] ? p_meta[p] : 0u;
                ae[q] = valid[q] ? as[q] + t_len[m[q] & (tile_q - 1)] - 1u : kIdleEnd;
            }
            icount_heads<kSortQpl>(sa, scr, as, ae, cnt, fst);
#pragma unroll
            for (uint32_t q = 0; q < kSortQpl; ++q)
                if (valid[q] && cnt[q]) atomicAdd(&acc[m[q] >> kSortQBits], (unsigned long long)cnt[q]);
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < nsh; k += blockDim.x) {
            const unsigned long long v = acc[k];
            if (v) atomicAdd(totals + sb + k, v);
            acc[k] = 0ull;
        }
        __syncthreads();
    }
}

struct ChromTab {
    uint32_t n;
    uint32_t off[BITS_MAX_CHROM + 1];   // off[c] = sum of lengths before c; off[n] = genome size
};

// Chromosome of a global coordinate: the last c with off[c] <= s.
__device__ __forceinline__ uint32_t chrom_of(const ChromTab& ct, uint32_t s) {
    uint32_t lo = 0, hi = ct.n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ct.off[mid] <= s) lo = mid; else hi = mid;
    }
    return lo;
}

// Per-chromosome query counts (hist zeroed by the caller).
__global__ void __launch_bounds__(256) k_mc_hist(const uint32_t* __restrict__ a_start, uint64_t na, ChromTab ct,
                                                 uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[BITS_MAX_CHROM];
    for (uint32_t k = threadIdx.x; k < BITS_MAX_CHROM; k += blockDim.x) h[k] = 0u;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[chrom_of(ct, a_start[i])], 1u);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < ct.n; k += blockDim.x)
        if (h[k]) atomicAdd(&hist[k], h[k]);
}

// cursor[c] = queries on chromosomes before c (one lane; at most 256 bins).
__global__ void k_mc_scan(const uint32_t* __restrict__ hist, uint32_t n, uint32_t* __restrict__ cursor) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        uint32_t acc = 0;
        for (uint32_t k = 0; k < n; ++k) {
            cursor[k] = acc;
            acc += hist[k];
        }
    }
}

// Per-query (chromosome offset, number of legal starts, length, index),
// computed once and reused by every shuffle, stored grouped by chromosome:
// each round of blockDim queries takes one slot range per chromosome from
// `cursor` and places its queries there.  The order inside a chromosome's
// range depends on scheduling; the totals do not (sums over the queries,
// each drawing from its own index).  span = 0 marks a query outside its
// chromosome (or start > end).
__global__ void __launch_bounds__(1024) k_mc_prepare(const uint32_t* __restrict__ a_start,
                                                     const uint32_t* __restrict__ a_end, uint64_t na, ChromTab ct,
                                                     uint32_t* __restrict__ cursor, uint32_t* __restrict__ off,
                                                     uint32_t* __restrict__ span, uint32_t* __restrict__ len,
                                                     uint32_t* __restrict__ idx, uint32_t* status) {
    __shared__ uint32_t cnt[BITS_MAX_CHROM], base[BITS_MAX_CHROM];
    uint32_t bad = 0;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < na; i0 += (uint64_t)gridDim.x * blockDim.x) {
        for (uint32_t k = threadIdx.x; k < ct.n; k += blockDim.x) cnt[k] = 0u;
        __syncthreads();
        const uint64_t i = i0 + threadIdx.x;
        uint32_t s = 0, e = 0, c = 0, r = 0;
        if (i < na) {
            s = a_start[i];
            e = a_end[i];
            c = chrom_of(ct, s);
            r = atomicAdd(&cnt[c], 1u);
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < ct.n; k += blockDim.x)
            if (cnt[k]) base[k] = atomicAdd(&cursor[k], cnt[k]);
        __syncthreads();
        if (i < na) {
            const bool ok = s <= e && s >= ct.off[c] && (uint64_t)e < (uint64_t)ct.off[c + 1];
            const uint32_t L = e - s + 1u;
            const uint32_t pos = base[c] + r;
            off[pos] = ct.off[c];
            len[pos] = ok ? L : 1u;
            span[pos] = ok ? (ct.off[c + 1] - ct.off[c]) - L + 1u : 0u;
            idx[pos] = (uint32_t)i;
            if (!ok) bad |= (s > e) ? BITS_FLAG_INTERVAL : BITS_FLAG_CHROM;
        }
        __syncthreads();
    }
    if (bad) atomicOr(status, bad);
}

// ------------------------------------------------------------------ paper orientation
// The Monte-Carlo loop as Sec. 3.2 runs it: every round randomises the
// database set B and sorts it again, then counts the fixed query set A.
// Round r of a batch places interval idx[p] of B (table position p) by the
// rule and stream of k_mc with the roles swapped, g = (s0 + r) * nb + idx[p],
// and writes keys S[r * nb + p], E[r * nb + p] as one segment per round for
// the segmented sort.  An interval outside its chromosome (span 0) becomes
// the sentinel [2^32 - 1, 2^32 - 1], which no query with end < 2^32 - 1
// counts.  identity = true writes the unshuffled set (the observed round).
__global__ void k_place_rounds(const uint32_t* __restrict__ off, const uint32_t* __restrict__ span,
                               const uint32_t* __restrict__ len, const uint32_t* __restrict__ idx,
                               const uint32_t* __restrict__ b_start, uint64_t nb, uint64_t seed, uint64_t s0,
                               uint32_t rounds, uint32_t identity, uint32_t* __restrict__ S, uint32_t* __restrict__ E) {
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint64_t total = (uint64_t)rounds * nb;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = t / nb, p = t - r * nb;
        const uint32_t sp = span[p];
        uint32_t st = 0xFFFFFFFFu, en = 0xFFFFFFFFu;
        if (sp) {
            if (identity) {
                st = b_start[idx[p]];
            } else {
                const uint64_t g = (s0 + r) * nb + idx[p];
                uint32_t c0 = (uint32_t)g, c1 = (uint32_t)(g >> 32), c2 = 0u, c3 = 0u;
                philox4x32_10(c0, c1, c2, c3, k0, k1);
                const uint64_t u = ((uint64_t)c1 << 32) | c0;
                st = off[p] + (uint32_t)__umul64hi(u, (uint64_t)sp);
            }
            en = st + len[p] - 1u;
        }
        S[t] = st;
        E[t] = en;
    }
}

// Counts the fixed query set A against every sorted round of a batch
// (segments S[r * nb ..], E[r * nb ..]) by plain bisection of the whole
// segment (no top tree: the arrays change every round).  Work item = (round,
// tile of A); one atomic per wave per item into totals[r].
template <int QPL>
BITS_SEARCH_KERNEL k_count_rounds(SearchArgs sa0, const uint32_t* __restrict__ S, const uint32_t* __restrict__ E,
                                  uint64_t nb, uint32_t rounds, const uint32_t* __restrict__ a_start,
                                  const uint32_t* __restrict__ a_end, uint64_t na, uint64_t tiles,
                                  unsigned long long* __restrict__ totals) {
    const uint64_t tile = (uint64_t)blockDim.x * QPL;
    uint32_t bad = 0;
    for (uint64_t item = blockIdx.x; item < (uint64_t)rounds * tiles; item += gridDim.x) {
        const uint64_t r = item / tiles, t = item - r * tiles;
        SearchArgs sa = sa0;
        sa.bs = S + r * nb;
        sa.be = E + r * nb;
        sa.n = (uint32_t)nb;
        sa.depth = 0;
        uint32_t as[QPL], ae[QPL], cnt[QPL], fst[QPL];
        bool valid[QPL];
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint64_t i = t * tile + (uint64_t)q * blockDim.x + threadIdx.x;
            valid[q] = i < na;
            as[q] = valid[q] ? a_start[i] : 0u;
            ae[q] = valid[q] ? a_end[i] : kIdleEnd;
            if (as[q] > ae[q]) {
                bad = 1;
                valid[q] = false;
                ae[q] = as[q];
            }
        }
        icount_plain<QPL>(sa, nullptr, as, ae, cnt, fst);
        uint64_t sum = 0;
#pragma unroll
        for (int q = 0; q < QPL; ++q) sum += valid[q] ? cnt[q] : 0u;
        sum = wave_sum_u64(sum);
        if ((threadIdx.x & (kWave - 1)) == 0 && sum) atomicAdd(totals + r, (unsigned long long)sum);
    }
    if (bad && sa0.status) atomicOr(sa0.status, BITS_FLAG_INTERVAL);
}

__global__ void k_mc_tail(const unsigned long long* __restrict__ totals, uint64_t nshuf,
                          const unsigned long long* observed, unsigned long long* n_ge,
                          unsigned long long* n_le) {
    __shared__ unsigned long long red[2][16];
    const unsigned long long obs = *observed;
    uint64_t ge = 0, le = 0;
    for (uint64_t s = threadIdx.x; s < nshuf; s += blockDim.x) {
        ge += totals[s] >= obs;
        le += totals[s] <= obs;
    }
    ge = wave_sum_u64(ge);
    le = wave_sum_u64(le);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][w] = ge;
        red[1][w] = le;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long g = 0, l = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
            g += red[0][k];
            l += red[1][k];
        }
        *n_ge = g;
        *n_le = l;
    }
}

// Order statistics of the per-shuffle totals (the median of Sec. 3.3):
// out[r] = the k[r]-th smallest (0-based) of v[0..n), by most-significant-
// digit radix selection over the 8 bytes: each pass histograms the values
// that match the digits fixed so far and keeps the bucket holding the rank.
// One workgroup; exact for any n < 2^32.
__global__ void __launch_bounds__(1024) k_select_u64(const unsigned long long* __restrict__ v, uint64_t n,
                                                     uint64_t k0, uint64_t k1, unsigned long long* out0,
                                                     unsigned long long* out1) {
    __shared__ uint32_t hist[256];
    __shared__ unsigned long long sh_prefix, sh_mask;
    __shared__ uint64_t sh_rank;
    for (int which = 0; which < 2; ++which) {
        if (threadIdx.x == 0) {
            sh_prefix = 0ull;
            sh_mask = 0ull;
            sh_rank = which ? k1 : k0;
        }
        __syncthreads();
        for (int p = 7; p >= 0; --p) {
            for (uint32_t d = threadIdx.x; d < 256u; d += blockDim.x) hist[d] = 0u;
            __syncthreads();
            const unsigned long long prefix = sh_prefix, mask = sh_mask;
            for (uint64_t i = threadIdx.x; i < n; i += blockDim.x) {
                const unsigned long long x = v[i];
                if ((x & mask) == prefix) atomicAdd(&hist[(uint32_t)(x >> (8 * p)) & 255u], 1u);
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                uint64_t r = sh_rank, cum = 0;
                uint32_t d = 0;
                while (d < 255u && cum + hist[d] <= r) cum += hist[d++];
                sh_rank = r - cum;
                sh_prefix = prefix | ((unsigned long long)d << (8 * p));
                sh_mask = mask | (0xFFull << (8 * p));
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) *(which ? out1 : out0) = sh_prefix;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ projection
__global__ void k_project(ChromTab ct, const uint32_t* __restrict__ chrom, const uint32_t* __restrict__ ls,
                          const uint32_t* __restrict__ le, uint64_t n, uint32_t* __restrict__ gs,
                          uint32_t* __restrict__ ge, uint32_t* status) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t c = chrom[i], s = ls[i], e = le[i];
        const bool cok = c < ct.n;
        const uint32_t o = cok ? ct.off[c] : 0u;
        const uint32_t clen = cok ? ct.off[c + 1] - ct.off[c] : 0u;
        if (!cok || e >= clen) bad |= BITS_FLAG_CHROM;
        if (s > e) bad |= BITS_FLAG_INTERVAL;
        gs[i] = o + s;
        ge[i] = o + e;
    }
    if (bad && status) atomicOr(status, bad);
}

// ------------------------------------------------------------------ batched pairs
// Each workgroup owns the contiguous item range [wg_begin[w], wg_begin[w+1]);
// items are sorted by reference, so (plain path) the LDS tree is re-staged
// only when the reference changes.  Consecutive logical workgroups run on the
// same XCD (hardware dispatches workgroups round-robin over the 8 XCDs), so
// an XCD's L2 sees few distinct references (and, on the learned path, their
// leaf records).  LEARNED searches every pair through the reference's learned
// index (leaf model, error-window head probe, one line), with the per-wave scratch in LDS.
template <int QPL, bool LEARNED>
__global__ void __launch_bounds__(1024)
    k_batch(const BatchRef* __restrict__ refs, const BatchQuery* __restrict__ qs, const BatchItem* __restrict__ items,
            const uint32_t* __restrict__ wg_begin, uint32_t n_wg, uint32_t n_ref, uint32_t max_depth,
            unsigned long long* __restrict__ pair_totals, uint32_t* status) {
    extern __shared__ uint32_t lds[];
    const uint32_t g = gridDim.x, b = blockIdx.x;
    const uint32_t per_xcd = g / 8u;
    const uint32_t w = (g % 8u == 0u) ? (b % 8u) * per_xcd + b / 8u : b;
    if (w >= n_wg) return;
    const uint32_t i0 = wg_begin[w], i1 = wg_begin[w + 1];
    uint32_t cur = 0xFFFFFFFFu;
    SearchArgs sa{};
    uint32_t bad = 0;
    for (uint32_t it = i0; it < i1; ++it) {
        const BatchItem item = items[it];
        if (item.r != cur) {
            const BatchRef R = refs[item.r];
            sa.bs = R.bs;
            sa.be = R.be;
            sa.tree = R.tree;
            sa.rmi = R.rmi;
            sa.hs = R.hs;
            sa.he = R.he;
            sa.status = status;
            sa.fallbacks = R.fallbacks;
            sa.n = R.n;
            sa.tree_stride = R.tree_stride;
            sa.depth = LEARNED ? 0u : min(R.depth, max_depth);
            if (!LEARNED) {
                __syncthreads();
                stage_tree(lds, sa.tree, sa.tree_stride, sa.depth);
                __syncthreads();
            }
            cur = item.r;
        }
        const BatchQuery Q = qs[item.q];
        uint32_t as[QPL], ae[QPL], cnt[QPL];
        bool valid[QPL];
#pragma unroll
        for (int q = 0; q < QPL; ++q) {
            const uint32_t k = (uint32_t)q * blockDim.x + threadIdx.x;
            const uint64_t i = (uint64_t)item.begin + k;
            valid[q] = k < item.count;
            as[q] = valid[q] ? Q.as[i] : 0u;
            ae[q] = valid[q] ? Q.ae[i] : kIdleEnd;
            if (as[q] > ae[q]) {
                bad = 1;
                valid[q] = false;
                ae[q] = as[q];
            }
        }
        if (sa.n) {   // uniform over the workgroup: every item of the loop is one reference
            uint32_t fst[QPL];
            icount<QPL, LEARNED>(sa, lds, as, ae, cnt, fst);
        } else {
#pragma unroll
            for (int q = 0; q < QPL; ++q) cnt[q] = 0;
        }
        uint64_t acc = 0;
#pragma unroll
        for (int q = 0; q < QPL; ++q) acc += valid[q] ? cnt[q] : 0u;
        acc = wave_sum_u64(acc);
        if ((threadIdx.x & (kWave - 1)) == 0 && acc)
            atomicAdd(pair_totals + (uint64_t)item.q * n_ref + item.r, (unsigned long long)acc);
    }
    if (bad) atomicOr(status, BITS_FLAG_INTERVAL);
}

// ------------------------------------------------------------------ window hook
// For keys x[i]: the learned path's window for array `which` (0 = B_S,
// 1 = B_E): lo = wl, hi = wr, or lo = hi = the resolved rank.
__global__ void __launch_bounds__(256) k_rmi_window(SearchArgs sa, uint32_t which, const uint32_t* __restrict__ xs,
                                                    uint64_t n, uint32_t* __restrict__ lo, uint32_t* __restrict__ hi) {
    extern __shared__ uint32_t lds[];
    uint32_t* scr = lds + (threadIdx.x / kWave) * probe_scratch_words(1);
    const uint64_t tiles = (n + blockDim.x - 1) / blockDim.x;
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t i = t * blockDim.x + threadIdx.x;
        const uint32_t xi = i < n ? xs[i] : 0u;
        uint32_t x[2] = {xi, xi}, base[2], wl[2], wr[2], rlo[2], rhi[2];
        bool win[2];
        learned_windows<2>(sa, scr, x, base, wl, wr, rlo, rhi, win);
        if (i < n) {
            lo[i] = win[which] ? wl[which] : base[which];
            hi[i] = win[which] ? wr[which] : base[which];
        }
    }
}

hipError_t launch_rmi_window(const SearchArgs& sa, uint32_t which, const uint32_t* xs, uint64_t n, uint32_t* lo,
                             uint32_t* hi, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_rmi_window, dim3((uint32_t)g), dim3(256), search_lds_bytes(true, 0, 1, 256), s, sa, which,
                       xs, n, lo, hi);
    return hipGetLastError();
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------ host side

int device_cu_count() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
        cached[dev] = cu;
    }
    return cached[dev];
}

size_t device_lds_per_block() {
    static size_t cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cached[dev] = (size_t)v;
    }
    return cached[dev];
}

// Workgroups resident per CU for a kernel/block/LDS combination (cached).
static int blocks_per_cu(const void* kernel, int block, size_t lds) {
    static std::mutex mu;
    static std::unordered_map<uint64_t, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint64_t key = ((uint64_t)(uintptr_t)kernel * 1315423911u) ^ ((uint64_t)block << 40) ^ ((uint64_t)lds << 8) ^ (uint64_t)dev;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, block, lds) != hipSuccess || nb <= 0) nb = 1;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = nb;
    return nb;
}

static uint32_t persistent_grid(const void* kernel, const LaunchCfg& cfg, size_t lds, uint64_t work_items) {
    uint64_t g = cfg.grid ? cfg.grid : (uint64_t)device_cu_count() * blocks_per_cu(kernel, cfg.block, lds);
    if (g > work_items) g = work_items;
    if (g < 1) g = 1;
    return (uint32_t)g;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template <int QPL, int MODE>
static hipError_t launch_count_t(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                                 uint64_t na, uint32_t* counts, uint32_t* firsts, unsigned long long* total,
                                 hipStream_t s) {
    const size_t lds = count_lds_bytes(cfg.path, sa.depth, QPL, cfg.block);
    const uint64_t tile = (uint64_t)cfg.block * QPL;
    const void* kern = (const void*)k_count<QPL, MODE>;
    const uint32_t grid = persistent_grid(kern, cfg, lds, (na + tile - 1) / tile);
    hipLaunchKernelGGL((k_count<QPL, MODE>), dim3(grid), dim3(cfg.block), lds, s, sa, as, ae, na, counts, firsts,
                       total);
    return hipGetLastError();
}

template <int QPL>
static hipError_t launch_count_q(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                                 uint64_t na, uint32_t* counts, uint32_t* firsts, unsigned long long* total,
                                 hipStream_t s) {
    switch (cfg.path) {
        case BITS_PATH_LEARNED:
            return launch_count_t<QPL, kModeLearned>(sa, cfg, as, ae, na, counts, firsts, total, s);
        case BITS_PATH_TIERED:
            return launch_count_t<QPL, kModeTiered>(sa, cfg, as, ae, na, counts, firsts, total, s);
        default:
            return launch_count_t<QPL, kModePlain>(sa, cfg, as, ae, na, counts, firsts, total, s);
    }
}

hipError_t launch_count(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                        uint64_t na, uint32_t* counts, unsigned long long* total, hipStream_t s, uint32_t* firsts) {
    if (!na) return hipSuccess;
    switch (cfg.qpl) {
        case 1: return launch_count_q<1>(sa, cfg, as, ae, na, counts, firsts, total, s);
        case 4: return launch_count_q<4>(sa, cfg, as, ae, na, counts, firsts, total, s);
        default: return launch_count_q<2>(sa, cfg, as, ae, na, counts, firsts, total, s);
    }
}

static int fill_chrom_tab(const uint32_t* chrom_len, uint32_t n_chrom, ChromTab* ct) {
    if (n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    uint64_t acc = 0;
    ct->n = n_chrom;
    for (uint32_t c = 0; c < n_chrom; ++c) {
        ct->off[c] = (uint32_t)acc;
        acc += chrom_len[c];
        if (acc > 0xFFFFFFFFull) return BITS_E_CHROM;
    }
    ct->off[n_chrom] = (uint32_t)acc;
    for (uint32_t c = n_chrom + 1; c <= BITS_MAX_CHROM; ++c) ct->off[c] = (uint32_t)acc;
    return BITS_OK;
}

hipError_t launch_mc_prepare(const uint32_t* as, const uint32_t* ae, uint64_t na, const uint32_t* chrom_len,
                             uint32_t n_chrom, const McTable& tab, uint32_t* status, hipStream_t s) {
    ChromTab ct;
    if (fill_chrom_tab(chrom_len, n_chrom, &ct) != BITS_OK) return hipErrorInvalidValue;
    if (!na) return hipSuccess;
    hipError_t e = launch_fill_u32(tab.hist, n_chrom, 0u, s);
    if (e != hipSuccess) return e;
    uint64_t g = (na + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_mc_hist, dim3((uint32_t)g), dim3(256), 0, s, as, na, ct, tab.hist);
    hipLaunchKernelGGL(k_mc_scan, dim3(1), dim3(64), 0, s, tab.hist, n_chrom, tab.cursor);
    g = (na + 1023) / 1024;
    if (g > 1024) g = 1024;
    hipLaunchKernelGGL(k_mc_prepare, dim3((uint32_t)g), dim3(1024), 0, s, as, ae, na, ct, tab.cursor, tab.off,
                       tab.span, tab.len, tab.idx, status);
    return hipGetLastError();
}

template <int QPL, bool LEARNED>
static hipError_t launch_mc_t(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                              const McTable& tab, uint64_t na, uint64_t seed, uint64_t s0, uint64_t nshuf,
                              unsigned long long* totals, unsigned long long* observed, hipStream_t s) {
    const size_t lds = search_lds_bytes(LEARNED, sa.depth, QPL, cfg.block);
    const uint64_t tile = (uint64_t)cfg.block * QPL;
    const uint64_t tps = (na + tile - 1) / tile;
    if (observed) {
        const void* ko = (const void*)k_mc<QPL, LEARNED, true>;
        const uint32_t go = persistent_grid(ko, cfg, lds, tps);
        hipLaunchKernelGGL((k_mc<QPL, LEARNED, true>), dim3(go), dim3(cfg.block), lds, s, sa, as, ae, tab.off,
                           tab.span, tab.len, tab.idx, na, seed, s0, (uint64_t)1, tps, 1u, observed);
    }
    // the sorted kernel when its LDS (dynamic + ~7 KB static) fits the device's per-workgroup limit
    if (nshuf && LEARNED && BITS_MC_SORTED && sort_lds_bytes(cfg.block) + 8192 <= device_lds_per_block()) {
        const size_t lds1 = sort_lds_bytes(cfg.block);
        const uint64_t tq = (na + sort_tile_q(cfg.block) - 1) / sort_tile_q(cfg.block);
        const void* km = (const void*)k_mc_sorted;
        const uint32_t gm = persistent_grid(km, cfg, lds1, nshuf * tq);
        uint32_t chunk = kMaxChunk;
        while (chunk > 1 && tq * ((nshuf + chunk - 1) / chunk) < 8ull * gm) chunk >>= 1;
        hipLaunchKernelGGL(k_mc_sorted, dim3(gm), dim3(cfg.block), lds1, s, sa, tab.off, tab.span, tab.len, tab.idx,
                           na, seed, s0, nshuf, tq, chunk, totals);
    } else if (nshuf) {
        const void* km = (const void*)k_mc<QPL, LEARNED, false>;
        const uint32_t gm = persistent_grid(km, cfg, lds, nshuf * tps);
        // shuffles per work item: as many as keep >= 8 items per workgroup
        uint32_t chunk = kMaxChunk;
        while (chunk > 1 && tps * ((nshuf + chunk - 1) / chunk) < 8ull * gm) chunk >>= 1;
        hipLaunchKernelGGL((k_mc<QPL, LEARNED, false>), dim3(gm), dim3(cfg.block), lds, s, sa, as, ae, tab.off,
                           tab.span, tab.len, tab.idx, na, seed, s0, nshuf, tps, chunk, totals);
    }
    return hipGetLastError();
}

hipError_t launch_mc(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                     const McTable& tab, uint64_t na, uint64_t seed, uint64_t s0, uint64_t nshuf,
                     unsigned long long* totals, unsigned long long* observed, hipStream_t s) {
    if (!na) return hipSuccess;
    const bool L = cfg.path == BITS_PATH_LEARNED;
    switch (cfg.qpl) {
        case 1: return L ? launch_mc_t<1, true>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s)
                         : launch_mc_t<1, false>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s);
        case 4: return L ? launch_mc_t<4, true>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s)
                         : launch_mc_t<4, false>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s);
        default: return L ? launch_mc_t<2, true>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s)
                          : launch_mc_t<2, false>(sa, cfg, as, ae, tab, na, seed, s0, nshuf, totals, observed, s);
    }
}

template <int QPL, bool LEARNED>
static hipError_t launch_decide_t(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                                  uint64_t na, uint32_t* found, unsigned long long* witness, hipStream_t s) {
    const size_t lds = search_lds_bytes(LEARNED, sa.depth, QPL, cfg.block);
    const uint64_t tile = (uint64_t)cfg.block * QPL;
    const void* kern = (const void*)k_decide<QPL, LEARNED>;
    const uint32_t grid = persistent_grid(kern, cfg, lds, (na + tile - 1) / tile);
    hipLaunchKernelGGL((k_decide<QPL, LEARNED>), dim3(grid), dim3(cfg.block), lds, s, sa, as, ae, na, found, witness);
    return hipGetLastError();
}

hipError_t launch_decide(const SearchArgs& sa, const LaunchCfg& cfg, const uint32_t* as, const uint32_t* ae,
                         uint64_t na, uint32_t* found, unsigned long long* witness, hipStream_t s) {
    if (!na) return hipSuccess;
    const bool L = cfg.path == BITS_PATH_LEARNED;
    switch (cfg.qpl) {
        case 1: return L ? launch_decide_t<1, true>(sa, cfg, as, ae, na, found, witness, s)
                         : launch_decide_t<1, false>(sa, cfg, as, ae, na, found, witness, s);
        case 4: return L ? launch_decide_t<4, true>(sa, cfg, as, ae, na, found, witness, s)
                         : launch_decide_t<4, false>(sa, cfg, as, ae, na, found, witness, s);
        default: return L ? launch_decide_t<2, true>(sa, cfg, as, ae, na, found, witness, s)
                          : launch_decide_t<2, false>(sa, cfg, as, ae, na, found, witness, s);
    }
}

hipError_t launch_select_u64(const unsigned long long* v, uint64_t n, uint64_t k0, uint64_t k1,
                             unsigned long long* out0, unsigned long long* out1, hipStream_t s) {
    hipLaunchKernelGGL(k_select_u64, dim3(1), dim3(1024), 0, s, v, n, k0, k1, out0, out1);
    return hipGetLastError();
}

hipError_t launch_place_rounds(const McTable& tab, const uint32_t* b_start, uint64_t nb, uint64_t seed, uint64_t s0,
                               uint32_t rounds, bool identity, uint32_t* S, uint32_t* E, hipStream_t s) {
    const uint64_t total = (uint64_t)rounds * nb;
    if (!total) return hipSuccess;
    uint64_t g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_place_rounds, dim3((uint32_t)g), dim3(256), 0, s, tab.off, tab.span, tab.len, tab.idx,
                       b_start, nb, seed, s0, rounds, identity ? 1u : 0u, S, E);
    return hipGetLastError();
}

hipError_t launch_count_rounds(const uint32_t* S, const uint32_t* E, uint64_t nb, uint32_t rounds, const uint32_t* as,
                               const uint32_t* ae, uint64_t na, unsigned long long* totals, uint32_t* status,
                               hipStream_t s) {
    if (!na || !rounds) return hipSuccess;
    constexpr int QPL = 2;
    const uint32_t block = 256;
    const uint64_t tile = (uint64_t)block * QPL;
    const uint64_t tiles = (na + tile - 1) / tile;
    SearchArgs sa{};
    sa.status = status;
    sa.n = (uint32_t)nb;
    LaunchCfg cfg{block, QPL, 0, 0, BITS_PATH_PLAIN};
    const void* kern = (const void*)k_count_rounds<QPL>;
    const uint32_t grid = persistent_grid(kern, cfg, 0, (uint64_t)rounds * tiles);
    hipLaunchKernelGGL(k_count_rounds<QPL>, dim3(grid), dim3(block), 0, s, sa, S, E, nb, rounds, as, ae, na, tiles,
                       totals);
    return hipGetLastError();
}

hipError_t launch_mc_tail(const unsigned long long* totals, uint64_t nshuf, const unsigned long long* observed,
                          unsigned long long* n_ge, unsigned long long* n_le, hipStream_t s) {
    hipLaunchKernelGGL(k_mc_tail, dim3(1), dim3(1024), 0, s, totals, nshuf, observed, n_ge, n_le);
    return hipGetLastError();
}

hipError_t launch_project(const uint32_t* chrom_len, uint32_t n_chrom, const uint32_t* chrom, const uint32_t* ls,
                          const uint32_t* le, uint64_t n, uint32_t* gs, uint32_t* ge, uint32_t* status,
                          hipStream_t s) {
    ChromTab ct;
    if (fill_chrom_tab(chrom_len, n_chrom, &ct) != BITS_OK) return hipErrorInvalidValue;
    if (!n) return hipSuccess;
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(k_project, dim3((uint32_t)g), dim3(256), 0, s, ct, chrom, ls, le, n, gs, ge, status);
    return hipGetLastError();
}

template <int QPL, bool LEARNED>
static const void* batch_kernel() {
    return (const void*)k_batch<QPL, LEARNED>;
}

static const void* batch_kernel(uint32_t qpl, bool learned) {
    switch (qpl) {
        case 1: return learned ? batch_kernel<1, true>() : batch_kernel<1, false>();
        case 4: return learned ? batch_kernel<4, true>() : batch_kernel<4, false>();
        default: return learned ? batch_kernel<2, true>() : batch_kernel<2, false>();
    }
}

static size_t batch_lds(const LaunchCfg& cfg, uint32_t max_depth) {
    return search_lds_bytes(cfg.path == BITS_PATH_LEARNED, max_depth, (int)cfg.qpl, cfg.block);
}

hipError_t launch_batch(const BatchRef* refs, const BatchQuery* qs, const BatchItem* items, const uint32_t* wg_begin,
                        uint32_t n_wg, uint32_t n_ref, uint32_t max_depth, const LaunchCfg& cfg,
                        unsigned long long* pair_totals, uint32_t* status, hipStream_t s) {
    const size_t lds = batch_lds(cfg, max_depth);
    const bool L = cfg.path == BITS_PATH_LEARNED;
    const void* k = batch_kernel(cfg.qpl, L);
    void* args[] = {(void*)&refs, (void*)&qs, (void*)&items, (void*)&wg_begin, (void*)&n_wg, (void*)&n_ref,
                    (void*)&max_depth, (void*)&pair_totals, (void*)&status};
    return hipLaunchKernel(k, dim3(n_wg), dim3(cfg.block), args, lds, s);
}

int batch_blocks_per_cu(const LaunchCfg& cfg, uint32_t max_depth) {
    return blocks_per_cu(batch_kernel(cfg.qpl, cfg.path == BITS_PATH_LEARNED), (int)cfg.block,
                         batch_lds(cfg, max_depth));
}

}  // namespace bits
