// Learned CDF index over a sorted uint32 array (an extension of the BITS
// index; not in the paper).  Two stages:
//   root:  least-squares line rank ~ a*key + b, fitted from exact integer
//          sums, routes a key to one of 4096 leaves (monotone in the key, so
//          every leaf owns a contiguous rank range [rlo, rlo + cnt));
//   leaf:  y(u) = b2 + sum_j w2_j relu(w1_j u + b1_j), 16 hidden units, u the
//          key normalised to the leaf's key range, y the normalised rank.
// Each leaf is trained on the device by full-batch Adam on up to 2048
// stride-sampled keys (one wave per leaf, all state in registers, fixed-order
// reductions, hence deterministic).  After training, the same wave measures the largest over- and under-prediction of the rank over all of
// the leaf's keys with the query-time prediction code; queries search that
// window, verify the result and fall back to bisection of the leaf's range.
#include "bits_internal.hpp"

namespace bits {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kSumBlocks = 512;
constexpr int kNP = BITS_RMI_PARAMS;   // 49

// Exact partial sums of one block, each a plain uint64 that cannot wrap for
// n < 2^32: sum x; the low and high 32-bit halves of x^2 and of x*i (i =
// rank), summed separately (each half < 2^32, so any n < 2^32 of them fit).
struct Sums {
    unsigned long long sx, xx_lo, xx_hi, xi_lo, xi_hi;
    unsigned long long pad[3];
};

struct Pair2 {
    const uint32_t* keys[2];
    bits_rmi_model* model[2];
    uint32_t* bounds[2];   // [4097] first rank of every leaf, bounds[4096] = n
    Sums* sums[2];
    uint32_t* heads[2];    // line heads of the array, heads_len(n) words
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void add_key(unsigned long long (&v)[5], uint32_t x, uint32_t i) {
    const uint64_t xx = (uint64_t)x * x, xi = (uint64_t)x * i;   // i < n < 2^32
    v[0] += x;
    v[1] += (uint32_t)xx;
    v[2] += (uint32_t)(xx >> 32);
    v[3] += (uint32_t)xi;
    v[4] += (uint32_t)(xi >> 32);
}

// One read of the sorted keys: exact sums x, x^2, x*i (i = rank) as split
// halves (Sums), and the line heads (heads[j] = keys[32 j], then 0xFFFFFFFF
// up to hl), four keys per 16-byte load.
__global__ void __launch_bounds__(kThreads) k_rmi_sums(Pair2 P, uint64_t n, uint64_t hl) {
    const int a = blockIdx.y;
    const uint32_t* K = P.keys[a];
    uint32_t* H = P.heads[a];
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long v[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
    const uint64_t nq = n / 4;
    const uint4* K4 = reinterpret_cast<const uint4*>(K);   // the sorted arrays are 256-byte aligned
    for (uint64_t c = gid; c < nq; c += stride) {
        const uint4 x = K4[c];
        const uint32_t i0 = (uint32_t)(4 * c);
        add_key(v, x.x, i0);
        add_key(v, x.y, i0 + 1u);
        add_key(v, x.z, i0 + 2u);
        add_key(v, x.w, i0 + 3u);
        if ((c & 7u) == 0) H[c >> 3] = x.x;
    }
    for (uint64_t i = 4 * nq + gid; i < n; i += stride) {
        const uint32_t x = K[i];
        add_key(v, x, (uint32_t)i);
        if ((i & 31u) == 0) H[i >> 5] = x;
    }
    for (uint64_t j = (n + 31) / 32 + gid; j < hl; j += stride) H[j] = 0xFFFFFFFFu;
    __shared__ unsigned long long r[kWaves][5];
    const uint32_t lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long t = wave_sum_u64(v[k]);
        if (lane == 0) r[w][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long t = 0;
        for (int k = 0; k < kWaves; ++k) t += r[k][threadIdx.x];
        (&P.sums[a][blockIdx.x].sx)[threadIdx.x] = t;
    }
}

// Root line from the exact sums; routing slope/intercept pre-scaled by 4096/n.
// One wave per array (blockDim 128): the block partials are summed per lane,
// then over the wave, then combined exactly in 128 bits.
__global__ void __launch_bounds__(2 * kWave) k_rmi_root(Pair2 P, uint64_t n, uint32_t nblocks) {
    const int a = threadIdx.x / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1);
    unsigned long long v[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
    for (uint32_t b = lane; b < nblocks; b += kWave) {
        const Sums& S = P.sums[a][b];
        v[0] += S.sx;
        v[1] += S.xx_lo;
        v[2] += S.xx_hi;
        v[3] += S.xi_lo;
        v[4] += S.xi_hi;
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = wave_sum_u64(v[k]);
    if (lane != 0) return;
    const __int128 N = (__int128)n;
    const __int128 Sx = (__int128)v[0];
    const __int128 Sxx = (__int128)(((unsigned __int128)v[2] << 32) + v[1]);
    const __int128 Sxi = (__int128)(((unsigned __int128)v[4] << 32) + v[3]);
    const __int128 Si = N * (N - 1) / 2;
    const __int128 num = N * Sxi - Sx * Si;
    const __int128 den = N * Sxx - Sx * Sx;
    double fa = den > 0 ? (double)num / (double)den : 0.0;
    if (fa < 0.0) fa = 0.0;
    const double fb = n ? ((double)Si - fa * (double)Sx) / (double)n : 0.0;
    bits_rmi_model* M = P.model[a];
    const double scale = n ? (double)BITS_RMI_LEAVES / (double)n : 0.0;
    M->fit_a = fa;
    M->fit_b = fb;
    M->root_a = (float)(fa * scale);
    M->root_b = (float)(fb * scale);
    M->n = n;
}

// bounds[l] = first rank whose key routes to a leaf >= l, for l = 0..4096:
// routing is monotone in the key (slope >= 0), so one bisection per leaf.
__global__ void __launch_bounds__(256) k_rmi_bounds(Pair2 P, uint64_t n) {
    const int a = blockIdx.y;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > BITS_RMI_LEAVES) return;
    const uint32_t* K = P.keys[a];
    const bits_rmi_model* M = P.model[a];
    const float ra = M->root_a, rb = M->root_b;
    uint64_t lo = 0, len = n;   // first i in [0, n) with route(K[i]) >= l, else n
    while (len > 0) {
        const uint64_t half = len >> 1;
        if (rmi_route(ra, rb, K[lo + half]) < l) {
            lo += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    P.bounds[a][l] = (uint32_t)lo;
}

// ---------------------------------------------------------------- leaf training
// One wave trains one leaf.  Its training points sit in the wave's LDS
// slice; the 49 parameters are uniform across the wave.  The 50 per-lane
// partial sums of an epoch (49 gradients and the squared residual) are
// reduce-scattered over the wave in a fixed order, so lane l ends with the
// whole sum of one of them (rs_index(l)); it updates that parameter's Adam
// moments, and every lane reads the new parameters back from their owners.
// Training is therefore deterministic.

// Which of the 50 sums lane l holds after wave_reduce_scatter, or -1.  The
// halvings go by lane bit 5, 4, 2, 3, 1, 0, keeping lists of 25, 13, 7, 4, 2
// and 1 values (the upper part of an odd list is padded with zero).
constexpr int rs_index(int l) {
    const int b0 = l & 1, b1 = (l >> 1) & 1, b2 = (l >> 2) & 1, b3 = (l >> 3) & 1, b4 = (l >> 4) & 1,
              b5 = (l >> 5) & 1;
    const int k4 = 4 * b3 + 2 * b1 + b0;
    if (k4 >= 7) return -1;
    const int k3 = 7 * b2 + k4;
    if (k3 >= 13) return -1;
    const int k2 = 13 * b4 + k3;
    if (k2 >= 25) return -1;
    return 25 * b5 + k2;
}

struct LaneOf {
    int v[kNP + 1];
};
constexpr LaneOf make_lane_of() {
    LaneOf t{};
    for (int l = 0; l < kWave; ++l)
        if (rs_index(l) >= 0) t.v[rs_index(l)] = l;
    return t;
}
constexpr LaneOf kLaneOf = make_lane_of();
static_assert(kLaneOf.v[0] == 0 && kLaneOf.v[kNP] == 60, "reduce-scatter lane map");

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// One halving inside rows of 16 lanes: lanes with bit BIT clear keep the
// first N_OUT values, the others the rest (zero past N_IN); each lane adds
// what its partner, read through the DPP pattern CTRL, does not keep.
template <int N_IN, int N_OUT, int BIT, int CTRL>
__device__ __forceinline__ void rs_halve(const float* in, float* out, uint32_t lane) {
    const bool hi = (lane >> BIT) & 1u;
#pragma unroll
    for (int k = 0; k < N_OUT; ++k) {
        const float a = in[k], b = N_OUT + k < N_IN ? in[N_OUT + k] : 0.0f;
        out[k] = (hi ? b : a) + dpp_f<CTRL>(hi ? a : b);
    }
}

// Wave sum of g[0..49] (each lane's partial sums), scattered: returns in lane
// l the sum of g[rs_index(l)] over the 64 lanes.  v_permlane32_swap and
// v_permlane16_swap exchange the halves of the wave and of each 32 lanes;
// DPP row_ror:4, row_ror:8 and two quad permutations do the rest.
__device__ __forceinline__ float wave_reduce_scatter(const float (&g)[kNP + 1]) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    float a[25], b[13], c[7], d[4], e[2], f[1];
#pragma unroll
    for (int j = 0; j < 25; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[j]), __float_as_uint(g[25 + j]), false,
                                                        false);
        a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int k = 0; k < 13; ++k) {
        const float hi = 13 + k < 25 ? a[13 + k] : 0.0f;
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[k]), __float_as_uint(hi), false, false);
        b[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    rs_halve<13, 7, 2, 0x124>(b, c, lane);   // row_ror:4
    rs_halve<7, 4, 3, 0x128>(c, d, lane);    // row_ror:8
    rs_halve<4, 2, 1, 0x4E>(d, e, lane);     // quad_perm [2,3,0,1]
    rs_halve<2, 1, 0, 0xB1>(e, f, lane);     // quad_perm [1,0,3,2]
    return f[0];
}

// One training point's contribution to the per-lane partial sums (see
// wave_grad).  FIRST assigns instead of adding, which gives the same values
// as adding to zeros without the 50 clears.
template <bool FIRST>
__device__ __forceinline__ void add_point(const float (&p)[kNP], float uk, float tk, float scale,
                                          float (&g)[kNP + 1]) {
    float pre[16], h[16];
    float y = p[48];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        pre[q] = fmaf(p[q], uk, p[16 + q]);
        h[q] = fmaxf(pre[q], 0.0f);
        y = fmaf(p[32 + q], h[q], y);
    }
    const float r = y - tk;
    const float dy = r * scale;
    g[kNP] = FIRST ? r * r : fmaf(r, r, g[kNP]);
    g[48] = FIRST ? dy : g[48] + dy;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float dh = pre[q] > 0.0f ? dy * p[32 + q] : 0.0f;
        g[32 + q] = FIRST ? dy * h[q] : fmaf(dy, h[q], g[32 + q]);
        g[q] = FIRST ? dh * uk : fmaf(dh, uk, g[q]);
        g[16 + q] = FIRST ? dh : g[16 + q] + dh;
    }
}

// Loss gradient of the leaf model over points (u[j], t[j]), j < m: lane l
// takes points l, l + 64, ... in order.  The per-lane partial sums are the
// gradients of mean (y - t)^2 with respect to the 49 parameters and, as
// value 49, the summed squared residual; the return value is lane l's
// reduce-scattered sum (of value rs_index(l)).
__device__ __forceinline__ float wave_grad(const float (&p)[kNP], const float* u, const float* t, uint32_t m) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const float scale = m ? 2.0f / (float)m : 0.0f;
    float g[kNP + 1];
    if (__builtin_amdgcn_readfirstlane(m) >= kWave) {   // every lane has a first point (m is wave-uniform)
        add_point<true>(p, u[lane], t[lane], scale, g);
#pragma unroll 1
        for (uint32_t j = lane + kWave; j < m; j += kWave) add_point<false>(p, u[j], t[j], scale, g);
        return wave_reduce_scatter(g);
    }
#pragma unroll
    for (int k = 0; k <= kNP; ++k) g[k] = 0.0f;
#pragma unroll 1
    for (uint32_t j = lane; j < m; j += kWave) add_point<false>(p, u[j], t[j], scale, g);
    return wave_reduce_scatter(g);
}

__device__ __forceinline__ uint32_t lower_bound_in(const uint32_t* K, uint32_t lo, uint32_t hi, uint32_t x) {
    uint32_t base = lo, len = hi - lo;
    while (len > 0) {
        const uint32_t half = len >> 1;
        if (K[base + half] < x) {
            base += half + 1;
            len -= half + 1;
        } else {
            len = half;
        }
    }
    return base;
}

__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

struct TrainCfg {
    uint32_t epochs, max_points;
    float lr, beta1, beta2;
};

constexpr int kTrainWaves = 2;
constexpr int kErrBatch = 8;   // keys per lane loaded together in the error-window pass

// Dynamic LDS: 2 * tc.max_points floats per wave.
__global__ void __launch_bounds__(kTrainWaves * kWave) k_rmi_train(Pair2 P, TrainCfg tc) {
    extern __shared__ float pts[];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    const int a = blockIdx.y;
    const uint32_t leaf = blockIdx.x * kTrainWaves + wv;
    const uint32_t* K = P.keys[a];
    bits_rmi_leaf* L = &P.model[a]->leaf[leaf];
    const uint32_t rlo = P.bounds[a][leaf];
    const uint32_t cnt = P.bounds[a][leaf + 1] - rlo;
    uint32_t* Lw = reinterpret_cast<uint32_t*>(L);
    if (cnt == 0) {
        if (lane < 32) Lw[lane] = lane == 0 ? 0xFFFFFFFFu : lane == 4 ? rlo : 0u;
        return;
    }
    const uint32_t kmin = K[rlo], kmax = K[rlo + cnt - 1];
    const uint32_t span = kmax - kmin;
    const float kinv = 1.0f / (float)(span > 1u ? span : 1u);
    const uint32_t m = cnt < tc.max_points ? cnt : tc.max_points;

    // training point j: the key at rank rlo + floor(j * cnt / m), target its
    // lower-bound rank normalised to the leaf
    float* u = pts + (size_t)wv * 2 * tc.max_points;
    float* t = u + tc.max_points;
    for (uint32_t j = lane; j < m; j += kWave) {
        const uint32_t i = rlo + (uint32_t)(((uint64_t)j * cnt) / m);
        const uint32_t x = K[i];
        u[j] = (float)(x - kmin) * kinv;
        t[j] = (float)(lower_bound_in(K, rlo, i, x) - rlo) / (float)cnt;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Initial network: piecewise-linear interpolation of the sampled CDF at
    // 16 quantile knots (unit j is relu(u - knot_j), w2 the slope changes).
    float ku = 0.0f, kt = 0.0f;
    if (lane <= 16) {
        const uint32_t sidx = lane < 16 ? (uint32_t)(((uint64_t)lane * m) / 16u) : m - 1;
        ku = u[sidx];
        kt = t[sidx];
    }
    float p[kNP];
    {
        float kn[17], tv[17];
#pragma unroll
        for (int j = 0; j < 17; ++j) {
            kn[j] = bcast(ku, j);
            tv[j] = bcast(kt, j);
        }
        if (!(kn[16] > kn[15])) kn[16] = kn[15] + 1e-3f;
        float prev = 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const float du = fmaxf(kn[j + 1] - kn[j], 1e-6f);
            const float slope = fminf((tv[j + 1] - tv[j]) / du, 1e4f);
            p[j] = 1.0f;
            p[16 + j] = -kn[j];
            p[32 + j] = slope - prev;
            prev = slope;
        }
        p[48] = tv[0];
    }

    // Full-batch Adam; lane l updates parameter rs_index(l) (when < 49), then
    // every lane reads the new parameters back from their owners.
    const int mine = rs_index((int)lane);
    const bool owner = mine >= 0 && mine < kNP;
    float own = 0.0f;
#pragma unroll
    for (int j = 0; j < kNP; ++j)
        if (mine == j) own = p[j];
    float mom = 0.0f, vel = 0.0f, b1t = 1.0f, b2t = 1.0f;
    for (uint32_t e = 0; e < tc.epochs; ++e) {
        const float gk = wave_grad(p, u, t, m);
        mom = tc.beta1 * mom + (1.0f - tc.beta1) * gk;
        vel = tc.beta2 * vel + (1.0f - tc.beta2) * gk * gk;
        b1t *= tc.beta1;
        b2t *= tc.beta2;
        const float mh = mom / (1.0f - b1t);
        const float vh = vel / (1.0f - b2t);
        if (owner) own -= tc.lr * mh / (sqrtf(vh) + 1e-8f);
#pragma unroll
        for (int j = 0; j < kNP; ++j) p[j] = bcast(own, kLaneOf.v[j]);
    }
    const float last_loss = bcast(wave_grad(p, u, t, m), kLaneOf.v[kNP]) / (float)m;

    // The stored model: w1, b1, w2 rounded to binary16, b2 kept in fp32.
    float q[kNP];
#pragma unroll
    for (int j = 0; j < 48; ++j) q[j] = h2f(f2h(p[j]));
    q[48] = p[48];
    // Error window over every key of the leaf (first occurrence of each
    // value; x == kmin is answered without a search), with the query-time
    // prediction arithmetic on the stored model.
    // kErrBatch keys (and their predecessors) are loaded per lane before any is
    // evaluated, so the loads of a batch are in flight together.
    int32_t over = 0, under = 0;
    const uint32_t rend = rlo + cnt;
    for (uint32_t i0 = rlo + lane; i0 < rend; i0 += kErrBatch * kWave) {
        uint32_t xs[kErrBatch], xp[kErrBatch];
#pragma unroll
        for (int k = 0; k < kErrBatch; ++k) {
            const uint32_t i = i0 + (uint32_t)k * kWave;
            xs[k] = i < rend ? K[i] : kmin;
            xp[k] = (i < rend && i > rlo) ? K[i - 1] : kmin;
        }
#pragma unroll
        for (int k = 0; k < kErrBatch; ++k) {
            const uint32_t i = i0 + (uint32_t)k * kWave, x = xs[k];
            if (x == kmin || xp[k] == x) continue;   // past the leaf, the leaf's first key, or a repeat
            const int32_t e = rmi_pred_offset(q, cnt, kinv, x - kmin) - (int32_t)(i - rlo);
            over = max(over, e);
            under = max(under, -e);
        }
    }
    over = min(wave_max_i32(over), 65535);
    under = min(wave_max_i32(under), 65535);
    if (lane == 0) {
        uint32_t w[32];
        w[0] = kmin;
        w[1] = kmax;
        w[4] = rlo;
        w[5] = cnt;
        w[8] = __float_as_uint(kinv);
        w[9] = __float_as_uint(q[48]);
        w[12] = (uint32_t)over | ((uint32_t)under << 16);
        w[13] = __float_as_uint(last_loss);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            w[4 * g + 2] = f2h(q[4 * g + 0]) | (f2h(q[4 * g + 1]) << 16);          // w1
            w[4 * g + 3] = f2h(q[4 * g + 2]) | (f2h(q[4 * g + 3]) << 16);
            w[16 + 4 * g + 0] = f2h(q[16 + 4 * g + 0]) | (f2h(q[16 + 4 * g + 1]) << 16);   // b1
            w[16 + 4 * g + 1] = f2h(q[16 + 4 * g + 2]) | (f2h(q[16 + 4 * g + 3]) << 16);
            w[16 + 4 * g + 2] = f2h(q[32 + 4 * g + 0]) | (f2h(q[32 + 4 * g + 1]) << 16);   // w2
            w[16 + 4 * g + 3] = f2h(q[32 + 4 * g + 2]) | (f2h(q[32 + 4 * g + 3]) << 16);
        }
        uint4* dst = reinterpret_cast<uint4*>(L);
#pragma unroll
        for (int k = 0; k < 8; ++k) dst[k] = make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
    }
}

// Gradient entry point: the training kernel's own wave_grad on given points.
__global__ void __launch_bounds__(kWave) k_leaf_grad(const float* u_in, const float* t_in, uint32_t m,
                                                      const float* params, float* grad, float* loss) {
    __shared__ float pts[2][BITS_RMI_MAX_POINTS];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    for (uint32_t j = lane; j < m; j += kWave) {
        pts[0][j] = u_in[j];
        pts[1][j] = t_in[j];
    }
    __syncthreads();
    float p[kNP];
#pragma unroll
    for (int j = 0; j < kNP; ++j) p[j] = params[j];
    const float gs = wave_grad(p, pts[0], pts[1], m);
    const int mine = rs_index((int)lane);
    if (mine >= 0 && mine < kNP) grad[mine] = gs;
    if (mine == kNP) *loss = m ? gs / (float)m : 0.0f;
}

}  // namespace

size_t rmi_workspace_bytes() {
    // two arrays: bounds (4097 uint32, rounded) + kSumBlocks partial sums
    return 2 * (4352 * sizeof(uint32_t) + kSumBlocks * sizeof(Sums));
}

// Builds the learned index of BOTH sorted arrays in the same launches.
int launch_rmi_build2(const uint32_t* keys0, const uint32_t* keys1, uint64_t n, bits_rmi_model* m0,
                      bits_rmi_model* m1, uint32_t* heads0, uint32_t* heads1, const bits_train& tr, void* ws,
                      hipStream_t s) {
    Pair2 P;
    P.heads[0] = heads0;
    P.heads[1] = heads1;
    char* b = (char*)ws;
    P.keys[0] = keys0;
    P.keys[1] = keys1;
    P.model[0] = m0;
    P.model[1] = m1;
    P.bounds[0] = (uint32_t*)b;
    P.bounds[1] = (uint32_t*)(b + 4352 * sizeof(uint32_t));
    P.sums[0] = (Sums*)(b + 2 * 4352 * sizeof(uint32_t));
    P.sums[1] = P.sums[0] + kSumBlocks;
    uint32_t nb = (uint32_t)((n + kThreads - 1) / kThreads);
    if (nb > (uint32_t)kSumBlocks) nb = kSumBlocks;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_rmi_sums, dim3(nb, 2), dim3(kThreads), 0, s, P, n, heads_len(n));
    hipLaunchKernelGGL(k_rmi_root, dim3(1), dim3(2 * kWave), 0, s, P, n, nb);
    hipLaunchKernelGGL(k_rmi_bounds, dim3((BITS_RMI_LEAVES + 256) / 256, 2), dim3(256), 0, s, P, n);
    TrainCfg tc{tr.epochs, tr.max_points, tr.lr, tr.beta1, tr.beta2};
    const size_t lds = (size_t)kTrainWaves * 2 * tc.max_points * sizeof(float);
    hipLaunchKernelGGL(k_rmi_train, dim3(BITS_RMI_LEAVES / kTrainWaves, 2), dim3(kTrainWaves * kWave), lds, s, P, tc);
    BITS_CHECK_HIP(hipGetLastError());
    return BITS_OK;
}

hipError_t launch_rmi_leaf_grad(const float* u, const float* t, uint32_t m, const float* params, float* grad,
                                float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_grad, dim3(1), dim3(kWave), 0, s, u, t, m, params, grad, loss);
    return hipGetLastError();
}

}  // namespace bits
