// Learned CDF index over a sorted uint32 array (an extension of the BITS
// index; not in the paper).  Two stages:
//   root:  least-squares line rank ~ a*key + b, fitted from exact integer
//          sums, routes a key to one of 4096 leaves (monotone in the key, so
//          every leaf owns a contiguous rank range [rlo, rlo + cnt));
//   leaf:  y(u) = b2 + sum_j w2_j relu(w1_j u + b1_j), 16 hidden units, u the
//          key normalised to the leaf's key range, y the normalised rank.
// Each leaf is trained on the device by full-batch Adam on up to 4096
// stride-sampled keys (one workgroup per leaf, all state on chip, fixed-order
// reductions, hence deterministic).  After training, the same workgroup
// measures the largest over- and under-prediction of the rank over all of
// the leaf's keys with the query-time prediction code; queries search that
// window, verify the result and fall back to bisection of the leaf's range.
#include "bits_internal.hpp"

namespace bits {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr uint32_t kMaxPoints = 4096;
constexpr int kSumBlocks = 512;
constexpr int kNP = BITS_RMI_PARAMS;   // 49

struct Sums {   // exact partial sums of one block
    unsigned long long sx;
    unsigned long long sxx_lo, sxx_hi;
    unsigned long long sxi_lo, sxi_hi;
    unsigned long long pad[3];
};

struct Pair2 {
    const uint32_t* keys[2];
    bits_rmi_model* model[2];
    uint32_t* bounds[2];   // [4097] first rank of every leaf, bounds[4096] = n
    Sums* sums[2];
};

__device__ __forceinline__ void add128(unsigned long long& lo, unsigned long long& hi, unsigned __int128 v) {
    const unsigned __int128 cur = ((unsigned __int128)hi << 64) | lo;
    const unsigned __int128 r = cur + v;
    lo = (unsigned long long)r;
    hi = (unsigned long long)(r >> 64);
}

// Exact sums over the keys: sum x, sum x^2, sum x*i (i = rank).
__global__ void __launch_bounds__(kThreads) k_rmi_sums(Pair2 P, uint64_t n) {
    const int a = blockIdx.y;
    const uint32_t* K = P.keys[a];
    unsigned long long sx = 0;
    unsigned __int128 sxx = 0, sxi = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = K[i];
        sx += x;
        sxx += (unsigned __int128)(x * x);
        sxi += (unsigned __int128)x * i;
    }
    __shared__ unsigned long long r[5][kThreads];
    r[0][threadIdx.x] = sx;
    r[1][threadIdx.x] = (unsigned long long)sxx;
    r[2][threadIdx.x] = (unsigned long long)(sxx >> 64);
    r[3][threadIdx.x] = (unsigned long long)sxi;
    r[4][threadIdx.x] = (unsigned long long)(sxi >> 64);
    __syncthreads();
    if (threadIdx.x == 0) {
        Sums S{};
        for (int t = 0; t < kThreads; ++t) {
            S.sx += r[0][t];
            add128(S.sxx_lo, S.sxx_hi, ((unsigned __int128)r[2][t] << 64) | r[1][t]);
            add128(S.sxi_lo, S.sxi_hi, ((unsigned __int128)r[4][t] << 64) | r[3][t]);
        }
        P.sums[a][blockIdx.x] = S;
    }
}

// Root line from the exact sums; routing slope/intercept pre-scaled by 4096/n.
__global__ void k_rmi_root(Pair2 P, uint64_t n, uint32_t nblocks) {
    const int a = threadIdx.x;
    if (a >= 2) return;
    unsigned long long sx = 0, xx_lo = 0, xx_hi = 0, xi_lo = 0, xi_hi = 0;
    for (uint32_t b = 0; b < nblocks; ++b) {
        const Sums S = P.sums[a][b];
        sx += S.sx;
        add128(xx_lo, xx_hi, ((unsigned __int128)S.sxx_hi << 64) | S.sxx_lo);
        add128(xi_lo, xi_hi, ((unsigned __int128)S.sxi_hi << 64) | S.sxi_lo);
    }
    const __int128 N = (__int128)n;
    const __int128 Sx = (__int128)sx;
    const __int128 Sxx = (__int128)(((unsigned __int128)xx_hi << 64) | xx_lo);
    const __int128 Sxi = (__int128)(((unsigned __int128)xi_hi << 64) | xi_lo);
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

// bounds[l] = first rank whose key routes to a leaf >= l.
__global__ void k_rmi_bounds(Pair2 P, uint64_t n) {
    const int a = blockIdx.y;
    const uint32_t* K = P.keys[a];
    const bits_rmi_model* M = P.model[a];
    uint32_t* B = P.bounds[a];
    const float ra = M->root_a, rb = M->root_b;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const int l = (int)rmi_route(ra, rb, K[i]);
        const int lp = i ? (int)rmi_route(ra, rb, K[i - 1]) : -1;
        for (int m = lp + 1; m <= l; ++m) B[m] = (uint32_t)i;
        if (i == n - 1)
            for (int m = l + 1; m <= (int)BITS_RMI_LEAVES; ++m) B[m] = (uint32_t)n;
    }
}

// Block-wide loss gradient of the leaf model over points (u[k], t[k]),
// k < m.  Every thread of the block returns; threads 0..49 hold the totals
// in out[0..49] (48 gradients, b2's, then the summed squared residual).
__device__ void block_grad(const float* u, const float* t, uint32_t m, const float* p, float (*red)[52],
                           float* out) {
    float g[kNP + 1];
#pragma unroll
    for (int k = 0; k <= kNP; ++k) g[k] = 0.0f;
    const float scale = m ? 2.0f / (float)m : 0.0f;
    for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
        const float uk = u[k];
        float pre[16], h[16];
        float y = p[48];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            pre[j] = fmaf(p[j], uk, p[16 + j]);
            h[j] = fmaxf(pre[j], 0.0f);
            y = fmaf(p[32 + j], h[j], y);
        }
        const float r = y - t[k];
        g[kNP] = fmaf(r, r, g[kNP]);
        const float dy = r * scale;
        g[48] += dy;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            g[32 + j] = fmaf(dy, h[j], g[32 + j]);
            const float dh = pre[j] > 0.0f ? dy * p[32 + j] : 0.0f;
            g[j] = fmaf(dh, uk, g[j]);
            g[16 + j] += dh;
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k <= kNP; ++k) {
        const float v = wave_sum_f32(g[k]);
        if (lane == 0) red[w][k] = v;
    }
    __syncthreads();
    if (threadIdx.x <= kNP) {
        float s = 0.0f;
        for (int ww = 0; ww < (int)(blockDim.x / kWave); ++ww) s += red[ww][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
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

struct TrainCfg {
    uint32_t epochs, max_points;
    float lr, beta1, beta2;
};

__global__ void __launch_bounds__(kThreads) k_rmi_train(Pair2 P, TrainCfg tc) {
    const int a = blockIdx.y;
    const uint32_t leaf = blockIdx.x;
    const uint32_t* K = P.keys[a];
    bits_rmi_leaf* L = &P.model[a]->leaf[leaf];
    const uint32_t rlo = P.bounds[a][leaf];
    const uint32_t cnt = P.bounds[a][leaf + 1] - rlo;
    __shared__ float su[kMaxPoints], st[kMaxPoints];
    __shared__ float prm[kNP];
    __shared__ float gsum[kNP + 1];
    __shared__ float red[kWaves][52];
    __shared__ int32_t ered[2][kWaves];

    if (cnt == 0) {
        for (int k = threadIdx.x; k < 64; k += blockDim.x) reinterpret_cast<uint32_t*>(L)[k] = 0u;
        __syncthreads();
        if (threadIdx.x == 0) {
            L->kmin = 0xFFFFFFFFu;
            L->kmax = 0u;
            L->rlo = rlo;
            L->cnt = 0u;
        }
        return;
    }
    const uint32_t kmin = K[rlo], kmax = K[rlo + cnt - 1];
    const uint32_t span = kmax - kmin;
    const float kinv = 1.0f / (float)(span > 1u ? span : 1u);
    const uint32_t m = cnt < tc.max_points ? cnt : tc.max_points;
    for (uint32_t j = threadIdx.x; j < m; j += blockDim.x) {
        const uint32_t i = rlo + (uint32_t)(((uint64_t)j * cnt) / m);
        const uint32_t x = K[i];
        const uint32_t lb = lower_bound_in(K, rlo, i, x);
        su[j] = (float)(x - kmin) * kinv;
        st[j] = (float)(lb - rlo) / (float)cnt;
    }
    __syncthreads();
    // Initial network: piecewise-linear interpolation of the sampled CDF at
    // 16 quantile knots (unit j is relu(u - knot_j), w2 the slope changes).
    if (threadIdx.x == 0) {
        float kn[17], tv[17];
        for (int j = 0; j < 16; ++j) {
            const uint32_t s = (uint32_t)(((uint64_t)j * m) / 16u);
            kn[j] = su[s];
            tv[j] = st[s];
        }
        kn[16] = su[m - 1] > kn[15] ? su[m - 1] : kn[15] + 1e-3f;
        tv[16] = st[m - 1];
        float prev = 0.0f;
        for (int j = 0; j < 16; ++j) {
            const float du = fmaxf(kn[j + 1] - kn[j], 1e-6f);
            float slope = (tv[j + 1] - tv[j]) / du;
            slope = fminf(slope, 1e4f);
            prm[j] = 1.0f;
            prm[16 + j] = -kn[j];
            prm[32 + j] = slope - prev;
            prev = slope;
        }
        prm[48] = tv[0];
    }
    __syncthreads();

    // Full-batch Adam; thread k < 49 owns parameter k and its moments.
    float mom = 0.0f, vel = 0.0f, b1t = 1.0f, b2t = 1.0f;
    float last_loss = 0.0f;
    for (uint32_t e = 0; e < tc.epochs; ++e) {
        float p[kNP];
#pragma unroll
        for (int k = 0; k < kNP; ++k) p[k] = prm[k];
        block_grad(su, st, m, p, red, gsum);
        if (threadIdx.x < kNP) {
            const float g = gsum[threadIdx.x];
            mom = tc.beta1 * mom + (1.0f - tc.beta1) * g;
            vel = tc.beta2 * vel + (1.0f - tc.beta2) * g * g;
            b1t *= tc.beta1;
            b2t *= tc.beta2;
            const float mh = mom / (1.0f - b1t);
            const float vh = vel / (1.0f - b2t);
            prm[threadIdx.x] -= tc.lr * mh / (sqrtf(vh) + 1e-8f);
        }
        __syncthreads();
    }
    {
        float p[kNP];
#pragma unroll
        for (int k = 0; k < kNP; ++k) p[k] = prm[k];
        block_grad(su, st, m, p, red, gsum);
        last_loss = gsum[kNP] / (float)m;
    }

    // Error window over every key of the leaf (first occurrence of each value;
    // x == kmin is answered without a search).
    float p[kNP];
#pragma unroll
    for (int k = 0; k < kNP; ++k) p[k] = prm[k];
    int32_t over = 0, under = 0;
    for (uint32_t i = rlo + threadIdx.x; i < rlo + cnt; i += blockDim.x) {
        const uint32_t x = K[i];
        if (x == kmin) continue;
        if (K[i - 1] == x) continue;   // i > rlo here because x > kmin
        const int32_t e = rmi_pred_offset(p, cnt, kinv, x - kmin) - (int32_t)(i - rlo);
        over = max(over, e);
        under = max(under, -e);
    }
    over = wave_max_i32(over);
    under = wave_max_i32(under);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) {
        ered[0][w] = over;
        ered[1][w] = under;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t o = 0, u = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
            o = max(o, ered[0][k]);
            u = max(u, ered[1][k]);
        }
        L->kmin = kmin;
        L->kmax = kmax;
        L->rlo = rlo;
        L->cnt = cnt;
        L->kinv = kinv;
        L->err_lo = o;
        L->err_hi = u;
        L->loss = last_loss;
    }
    if (threadIdx.x < kNP) L->p[threadIdx.x] = prm[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads) k_leaf_grad(const float* u, const float* t, uint32_t m,
                                                         const float* params, float* grad, float* loss) {
    __shared__ float red[kWaves][52];
    __shared__ float gsum[kNP + 1];
    float p[kNP];
#pragma unroll
    for (int k = 0; k < kNP; ++k) p[k] = params[k];
    block_grad(u, t, m, p, red, gsum);
    if (threadIdx.x < kNP) grad[threadIdx.x] = gsum[threadIdx.x];
    if (threadIdx.x == 0) *loss = m ? gsum[kNP] / (float)m : 0.0f;
}

}  // namespace

size_t rmi_workspace_bytes() {
    // two arrays: bounds (4097 uint32, rounded) + kSumBlocks partial sums
    return 2 * (4352 * sizeof(uint32_t) + kSumBlocks * sizeof(Sums));
}

// Builds the learned index of BOTH sorted arrays in the same launches.
int launch_rmi_build2(const uint32_t* keys0, const uint32_t* keys1, uint64_t n, bits_rmi_model* m0,
                      bits_rmi_model* m1, const bits_train& tr, void* ws, hipStream_t s) {
    Pair2 P;
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
    hipLaunchKernelGGL(k_rmi_sums, dim3(nb, 2), dim3(kThreads), 0, s, P, n);
    hipLaunchKernelGGL(k_rmi_root, dim3(1), dim3(64), 0, s, P, n, nb);
    uint32_t gb = (uint32_t)((n + 255) / 256);
    if (gb > 8192u) gb = 8192u;
    if (gb < 1) gb = 1;
    hipLaunchKernelGGL(k_rmi_bounds, dim3(gb, 2), dim3(256), 0, s, P, n);
    TrainCfg tc{tr.epochs, tr.max_points, tr.lr, tr.beta1, tr.beta2};
    hipLaunchKernelGGL(k_rmi_train, dim3(BITS_RMI_LEAVES, 2), dim3(kThreads), 0, s, P, tc);
    BITS_CHECK_HIP(hipGetLastError());
    return BITS_OK;
}

hipError_t launch_rmi_leaf_grad(const float* u, const float* t, uint32_t m, const float* params, float* grad,
                                float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_leaf_grad, dim3(1), dim3(kThreads), 0, s, u, t, m, params, grad, loss);
    return hipGetLastError();
}

}  // namespace bits
