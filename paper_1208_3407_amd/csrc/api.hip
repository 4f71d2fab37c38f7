// C ABI of libbits.so: argument checks, workspace carving and launch
// sequencing for the entry points declared in include/bits.h.  No entry
// point allocates device memory; every call only enqueues work on the
// caller's stream (bits_batch_create and the *_info/status readers, which
// wait on it, excepted).
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "bits_internal.hpp"

using namespace bits;

namespace {

constexpr size_t kStatusBytes = 256;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint32_t clamp_depth(uint64_t n, uint32_t depth) {
    if (n == 0) return 0;
    uint32_t lg = 0;
    while (lg < 63 && (2ull << lg) <= n) ++lg;   // floor(log2 n)
    uint32_t d = depth < BITS_MAX_DEPTH ? depth : BITS_MAX_DEPTH;
    return d < lg ? d : lg;
}

struct RefLayout {
    size_t status, tree, rmi, heads, bs, be, total;
};

RefLayout ref_layout(uint64_t n, uint32_t depth, int learned) {
    RefLayout L;
    size_t o = 0;
    L.status = o; o = align256(o + kStatusBytes);
    L.tree = o; o = align256(o + (size_t)2 * ((size_t)1 << depth) * sizeof(uint32_t));
    L.rmi = o; o = align256(o + (learned ? 2 * sizeof(bits_rmi_model) : 0));
    L.heads = o; o = align256(o + 2 * heads_len(n) * sizeof(uint32_t));
    L.bs = o; o = align256(o + (size_t)n * sizeof(uint32_t));
    L.be = o; o = align256(o + (size_t)n * sizeof(uint32_t));
    L.total = o;
    return L;
}

bool ref_ok(const bits_ref* r) {
    if (!r || !r->status || !r->tree || !r->heads || r->n > 0xFFFFFFFFull) return false;
    if (r->n && (!r->bs || !r->be)) return false;
    if (r->learned && !r->rmi) return false;
    return r->depth <= BITS_MAX_DEPTH;
}

bits_train train_defaults(const bits_train* t) {
    bits_train d{300u, 256u, 2e-3f, 0.9f, 0.999f};
    if (!t) return d;
    bits_train r = *t;
    if (r.max_points == 0) r.max_points = d.max_points;
    if (r.max_points > BITS_RMI_MAX_POINTS) r.max_points = BITS_RMI_MAX_POINTS;
    if (!(r.lr > 0.0f)) r.lr = d.lr;
    if (!(r.beta1 > 0.0f && r.beta1 < 1.0f)) r.beta1 = d.beta1;
    if (!(r.beta2 > 0.0f && r.beta2 < 1.0f)) r.beta2 = d.beta2;
    return r;
}

unsigned long long* fallback_counter(const bits_ref* r) {
    return reinterpret_cast<unsigned long long*>(r->status + 2);
}

}  // namespace

namespace bits {

int resolve_launch(const bits_ref* ref, const bits_launch* in, LaunchCfg* out) {
    LaunchCfg c{1024u, 2u, ref->depth, 0u, BITS_PATH_PLAIN};
    if (in) {
        if (in->block) c.block = in->block;
        if (in->qpl) c.qpl = in->qpl;
        if (in->depth != 0xFFFFFFFFu) c.depth = in->depth < ref->depth ? in->depth : ref->depth;
        c.grid = in->grid;
    }
    const uint32_t path = in ? in->path : BITS_PATH_AUTO;
    if (path == BITS_PATH_AUTO) c.path = ref->learned ? BITS_PATH_LEARNED : BITS_PATH_PLAIN;
    else if (path == BITS_PATH_PLAIN || path == BITS_PATH_LEARNED || path == BITS_PATH_TIERED) c.path = path;
    else return BITS_E_ARG;
    if (c.path == BITS_PATH_LEARNED && !ref->learned) return BITS_E_ARG;
    if (c.block != 256 && c.block != 512 && c.block != 1024) return BITS_E_ARG;
    if (c.qpl != 1 && c.qpl != 2 && c.qpl != 4) return BITS_E_ARG;
    // the per-wave scratch of the learned and tiered paths grows with qpl: step
    // the block down until one workgroup's LDS fits the device
    while (c.path != BITS_PATH_PLAIN && c.block > 256 &&
           count_lds_bytes(c.path, c.depth, (int)c.qpl, c.block) + 1024 > device_lds_per_block())
        c.block >>= 1;
    if (c.path == BITS_PATH_TIERED && count_lds_bytes(c.path, c.depth, (int)c.qpl, c.block) > device_lds_per_block())
        return BITS_E_ARG;
    *out = c;
    return BITS_OK;
}

SearchArgs make_search_args(const bits_ref* ref, const LaunchCfg& cfg) {
    SearchArgs sa{};
    sa.bs = ref->bs;
    sa.be = ref->be;
    sa.tree = ref->tree;
    sa.rmi = (const bits_rmi_model*)ref->rmi;
    sa.hs = ref->heads;
    sa.he = ref->heads ? ref->heads + heads_len(ref->n) : nullptr;
    sa.status = ref->status;
    sa.fallbacks = fallback_counter(ref);
    sa.n = (uint32_t)ref->n;
    sa.tree_stride = 1u << ref->depth;
    sa.depth = cfg.depth;
    return sa;
}

}  // namespace bits

extern "C" {

int bits_version(void) { return 1; }

const char* bits_strerror(int status) {
    switch (status) {
        case BITS_OK: return "ok";
        case BITS_E_ARG: return "invalid argument";
        case BITS_E_INTERVAL: return "interval with start > end";
        case BITS_E_CHROM: return "interval outside its chromosome or genome too large";
        case BITS_E_WORKSPACE: return "workspace too small";
        case BITS_E_HIP: return "HIP runtime error";
        case BITS_E_UNSUPPORTED: return "unsupported device or parameter";
        default: return "unknown status";
    }
}

int bits_get_status(const uint32_t* d_status, void* stream, uint32_t* status_out) {
    if (!d_status || !status_out) return BITS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    BITS_CHECK_HIP(hipStreamSynchronize(s));
    uint32_t v = 0;
    BITS_CHECK_HIP(hipMemcpy(&v, d_status, sizeof(v), hipMemcpyDeviceToHost));
    *status_out = v;
    return BITS_OK;
}

int bits_clear_status(uint32_t* d_status, void* stream) {
    if (!d_status) return BITS_E_ARG;
    BITS_CHECK_HIP(launch_fill_u32(d_status, 1, 0u, (hipStream_t)stream));
    return BITS_OK;
}

int bits_project(const uint32_t* chrom_len, uint32_t n_chrom, const uint32_t* d_chrom, const uint32_t* d_lstart,
                 const uint32_t* d_lend, uint64_t n, uint32_t* d_start, uint32_t* d_end, uint32_t* d_status,
                 void* stream) {
    if (!chrom_len || n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    if (n && (!d_chrom || !d_lstart || !d_lend || !d_start || !d_end)) return BITS_E_ARG;
    uint64_t g = 0;
    for (uint32_t c = 0; c < n_chrom; ++c) g += chrom_len[c];
    if (g > 0xFFFFFFFFull) return BITS_E_CHROM;
    BITS_CHECK_HIP(launch_project(chrom_len, n_chrom, d_chrom, d_lstart, d_lend, n, d_start, d_end, d_status,
                                  (hipStream_t)stream));
    return BITS_OK;
}

int bits_ref_bytes(uint64_t n, uint32_t depth, int learned, size_t* bytes) {
    if (!bytes || n > 0xFFFFFFFFull) return BITS_E_ARG;
    if (learned && n > 0x7FFFFFFFull) return BITS_E_ARG;
    *bytes = ref_layout(n, clamp_depth(n, depth), learned).total;
    return BITS_OK;
}

int bits_ref_init(void* d_block, size_t block_bytes, uint64_t n, uint32_t depth, int learned, bits_ref* ref) {
    if (!d_block || !ref || n > 0xFFFFFFFFull) return BITS_E_ARG;
    if (learned && n > 0x7FFFFFFFull) return BITS_E_ARG;
    const uint32_t d = clamp_depth(n, depth);
    const RefLayout L = ref_layout(n, d, learned);
    if (block_bytes < L.total) return BITS_E_WORKSPACE;
    if (((uintptr_t)d_block & 255u) != 0) return BITS_E_ARG;
    char* b = (char*)d_block;
    memset(ref, 0, sizeof(*ref));
    ref->n = n;
    ref->depth = d;
    ref->learned = learned ? 1u : 0u;
    ref->status = (uint32_t*)(b + L.status);
    ref->tree = (uint32_t*)(b + L.tree);
    ref->rmi = learned ? (void*)(b + L.rmi) : nullptr;
    ref->heads = (uint32_t*)(b + L.heads);
    ref->bs = (uint32_t*)(b + L.bs);
    ref->be = (uint32_t*)(b + L.be);
    ref->block = d_block;
    ref->block_bytes = block_bytes;
    return BITS_OK;
}

int bits_sort_ref_workspace(uint64_t n, size_t* bytes) {
    if (!bytes || n > 0xFFFFFFFFull) return BITS_E_ARG;
    const uint64_t ns[2] = {n, n};
    *bytes = std::max(sort_workspace_bytes(ns, 2), rmi_workspace_bytes());
    return BITS_OK;
}

int bits_sort_refs_workspace(const uint64_t* n, uint32_t n_ref, size_t* bytes) {
    if (!bytes || (n_ref && !n)) return BITS_E_ARG;
    std::vector<uint64_t> ns(2 * (size_t)n_ref);
    for (uint32_t j = 0; j < n_ref; ++j) {
        if (n[j] > 0xFFFFFFFFull) return BITS_E_ARG;
        ns[2 * j] = ns[2 * j + 1] = n[j];
    }
    *bytes = std::max(sort_workspace_bytes(ns.data(), 2 * n_ref), rmi_workspace_bytes());
    return BITS_OK;
}

// Builds the rest of a reference index from its sorted arrays; the status
// block was cleared before the sort.
static int finish_ref(const bits_ref* r, const bits_train& tr, void* ws, hipStream_t s) {
    if (r->n) {
        // keys past n up to the end of the last 128-byte line read as +inf
        const uint64_t pad = ((r->n + 31) & ~31ull) - r->n;
        BITS_CHECK_HIP(launch_fill_u32(r->bs + r->n, pad, 0xFFFFFFFFu, s));
        BITS_CHECK_HIP(launch_fill_u32(r->be + r->n, pad, 0xFFFFFFFFu, s));
        BITS_CHECK_HIP(launch_build_tree(r->bs, r->n, r->depth, r->tree, s));
        BITS_CHECK_HIP(launch_build_tree(r->be, r->n, r->depth, r->tree + ((size_t)1 << r->depth), s));
    } else {
        BITS_CHECK_HIP(launch_fill_u32(r->tree, (uint64_t)2 << r->depth, 0u, s));
    }
    uint32_t* he = r->heads + heads_len(r->n);
    if (r->learned && r->n) {   // the learned build's pass over the keys also writes the heads
        bits_rmi_model* m = (bits_rmi_model*)r->rmi;
        return launch_rmi_build2(r->bs, r->be, r->n, m, m + 1, r->heads, he, tr, ws, s);
    }
    BITS_CHECK_HIP(launch_build_heads(r->bs, r->n, r->heads, s));
    BITS_CHECK_HIP(launch_build_heads(r->be, r->n, he, s));
    if (r->learned) BITS_CHECK_HIP(launch_fill_u32((uint32_t*)r->rmi, 2 * sizeof(bits_rmi_model) / 4, 0u, s));
    return BITS_OK;
}

int bits_sort_ref(const uint32_t* d_b_start, const uint32_t* d_b_end, const bits_ref* ref, void* d_ws,
                  size_t ws_bytes, const bits_train* train, void* stream) {
    if (!ref_ok(ref)) return BITS_E_ARG;
    if (ref->n && (!d_b_start || !d_b_end || !d_ws)) return BITS_E_ARG;
    size_t need = 0;
    bits_sort_ref_workspace(ref->n, &need);
    if (ref->n && ws_bytes < need) return BITS_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    BITS_CHECK_HIP(launch_fill_u32(ref->status, kStatusBytes / 4, 0u, s));
    if (ref->n) {
        SortSeg segs[2] = {{d_b_start, ref->bs, ref->n}, {d_b_end, ref->be, ref->n}};
        const int rc = launch_sort(segs, 2, d_ws, ws_bytes, s);
        if (rc != BITS_OK) return rc;
        BITS_CHECK_HIP(launch_sort_report(d_ws, ref->status, s));
    }
    return finish_ref(ref, train_defaults(train), d_ws, s);
}

int bits_sort_refs(const uint32_t* const* d_b_start, const uint32_t* const* d_b_end, const bits_ref* refs,
                   uint32_t n_ref, void* d_ws, size_t ws_bytes, const bits_train* train, void* stream) {
    if (n_ref == 0) return BITS_OK;
    if (!d_b_start || !d_b_end || !refs || !d_ws) return BITS_E_ARG;
    std::vector<uint64_t> ns(n_ref);
    std::vector<SortSeg> segs;
    segs.reserve(2 * (size_t)n_ref);
    for (uint32_t j = 0; j < n_ref; ++j) {
        if (!ref_ok(&refs[j])) return BITS_E_ARG;
        if (refs[j].n && (!d_b_start[j] || !d_b_end[j])) return BITS_E_ARG;
        ns[j] = refs[j].n;
        segs.push_back({d_b_start[j], refs[j].bs, refs[j].n});
        segs.push_back({d_b_end[j], refs[j].be, refs[j].n});
    }
    size_t need = 0;
    bits_sort_refs_workspace(ns.data(), n_ref, &need);
    if (ws_bytes < need) return BITS_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t j = 0; j < n_ref; ++j) BITS_CHECK_HIP(launch_fill_u32(refs[j].status, kStatusBytes / 4, 0u, s));
    int rc = launch_sort(segs.data(), (uint32_t)segs.size(), d_ws, ws_bytes, s);
    if (rc != BITS_OK) return rc;
    for (uint32_t j = 0; j < n_ref; ++j) BITS_CHECK_HIP(launch_sort_report(d_ws, refs[j].status, s));
    const bits_train tr = train_defaults(train);
    for (uint32_t j = 0; j < n_ref; ++j) {
        rc = finish_ref(&refs[j], tr, d_ws, s);
        if (rc != BITS_OK) return rc;
    }
    return BITS_OK;
}

int bits_rmi_info(const bits_ref* ref, void* stream, bits_rmi_stats* out) {
    if (!ref_ok(ref) || !out || !ref->learned) return BITS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    BITS_CHECK_HIP(hipStreamSynchronize(s));
    std::vector<bits_rmi_model> host(2);
    BITS_CHECK_HIP(hipMemcpy(host.data(), ref->rmi, 2 * sizeof(bits_rmi_model), hipMemcpyDeviceToHost));
    unsigned long long fb = 0;
    BITS_CHECK_HIP(hipMemcpy(&fb, fallback_counter(ref), sizeof(fb), hipMemcpyDeviceToHost));
    double wsum = 0.0, lsum = 0.0;
    uint64_t nonempty = 0;
    uint32_t wmax = 0, empty = 0;
    for (int a = 0; a < 2; ++a)
        for (uint32_t l = 0; l < BITS_RMI_LEAVES; ++l) {
            const bits_rmi_leaf& L = host[a].leaf[l];
            if (L.a[1].h[1] == 0) {   // cnt
                ++empty;
                continue;
            }
            const uint32_t err = L.a[3].h[0];
            const uint32_t w = (err & 0xFFFFu) + (err >> 16) + 1u;
            float loss;
            memcpy(&loss, &L.a[3].h[1], sizeof(loss));
            wsum += w;
            lsum += loss;
            wmax = std::max(wmax, w);
            ++nonempty;
        }
    out->mean_window = nonempty ? wsum / (double)nonempty : 0.0;
    out->max_window = wmax;
    out->empty_leaves = empty;
    out->mean_loss = nonempty ? lsum / (double)nonempty : 0.0;
    out->fallbacks = fb;
    return BITS_OK;
}

static int check_queries(const bits_ref* ref, const uint32_t* as, const uint32_t* ae, uint64_t na) {
    if (!ref_ok(ref)) return BITS_E_ARG;
    if (na && (!as || !ae)) return BITS_E_ARG;
    return BITS_OK;
}

int bits_count_per_query(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                         uint32_t* d_counts, uint64_t* d_total, const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (na && !d_counts) return BITS_E_ARG;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* tot = (unsigned long long*)d_total;
    if (tot) BITS_CHECK_HIP(launch_fill_u64(tot, 1, 0ull, s));
    if (ref->n == 0) {
        BITS_CHECK_HIP(launch_fill_u32(d_counts, na, 0u, s));
        return BITS_OK;
    }
    BITS_CHECK_HIP(launch_count(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, na, d_counts, tot, s));
    return BITS_OK;
}

int bits_count(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
               uint64_t* d_total, const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (!d_total) return BITS_E_ARG;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* tot = (unsigned long long*)d_total;
    BITS_CHECK_HIP(launch_fill_u64(tot, 1, 0ull, s));
    if (ref->n == 0) return BITS_OK;
    BITS_CHECK_HIP(launch_count(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, na, nullptr, tot, s));
    return BITS_OK;
}

int bits_mc_workspace(uint64_t na, size_t* bytes) {
    if (!bytes || na > 0xFFFFFFFFull) return BITS_E_ARG;
    *bytes = 4 * align256((size_t)na * sizeof(uint32_t)) + 2 * align256(BITS_MAX_CHROM * sizeof(uint32_t));
    return BITS_OK;
}

}  // extern "C"

namespace {

// The body of bits_mc_pvalue and bits_mc_pvalue_noalloc: d_ws is the query
// table (bits_mc_workspace(na) bytes), from the caller or the library's own
// device array.
int mc_pvalue_impl(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                   const uint32_t* chrom_len, uint32_t n_chrom, uint64_t seed, uint64_t s0, uint64_t s1,
                   void* d_ws, size_t ws_bytes, uint64_t* d_totals, uint64_t* d_observed, uint64_t* d_n_ge,
                   uint64_t* d_n_le, const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (s1 < s0 || !chrom_len || n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    if (!d_observed || !d_n_ge || !d_n_le || (s1 > s0 && !d_totals)) return BITS_E_ARG;
    const uint64_t ns = s1 - s0;
    if (na > 0xFFFFFFFFull) return BITS_E_ARG;
    if (na && ns > ~0ull / na) return BITS_E_ARG;   // counter g = s * na + i must not wrap
    if (na && s1 > (~0ull - na) / na) return BITS_E_ARG;
    uint64_t g = 0;
    for (uint32_t c = 0; c < n_chrom; ++c) g += chrom_len[c];
    if (g > 0xFFFFFFFFull) return BITS_E_CHROM;
    size_t need = 0;
    bits_mc_workspace(na, &need);
    if (na && (!d_ws || ws_bytes < need)) return BITS_E_WORKSPACE;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    if (cfg.path == BITS_PATH_TIERED) return BITS_E_ARG;   // a counting-only path
    hipStream_t s = (hipStream_t)stream;
    auto* totals = (unsigned long long*)d_totals;
    auto* obs = (unsigned long long*)d_observed;
    BITS_CHECK_HIP(launch_fill_u64(totals, ns, 0ull, s));
    BITS_CHECK_HIP(launch_fill_u64(obs, 1, 0ull, s));
    if (na && ref->n) {
        const size_t stride = align256((size_t)na * sizeof(uint32_t));
        const size_t cstride = align256(BITS_MAX_CHROM * sizeof(uint32_t));
        char* w = (char*)d_ws;
        McTable tab;
        tab.off = (uint32_t*)w;
        tab.span = (uint32_t*)(w + stride);
        tab.len = (uint32_t*)(w + 2 * stride);
        tab.idx = (uint32_t*)(w + 3 * stride);
        tab.hist = (uint32_t*)(w + 4 * stride);
        tab.cursor = (uint32_t*)(w + 4 * stride + cstride);
        BITS_CHECK_HIP(launch_mc_prepare(d_a_start, d_a_end, na, chrom_len, n_chrom, tab, ref->status, s));
        BITS_CHECK_HIP(launch_mc(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, tab, na, seed, s0, ns, totals,
                                 obs, s));
    }
    BITS_CHECK_HIP(launch_mc_tail(totals, ns, obs, (unsigned long long*)d_n_ge, (unsigned long long*)d_n_le, s));
    return BITS_OK;
}

// Query table of bits_mc_pvalue_noalloc for up to BITS_NOALLOC_MAX_QUERIES
// queries.  In host code `scratch` only names the symbol: its device address
// (one per GPU) comes from hipGetSymbolAddress, taken once per device.
constexpr size_t kNoallocBytes =
    4 * ((BITS_NOALLOC_MAX_QUERIES * sizeof(uint32_t) + 255) & ~(size_t)255) +
    2 * ((BITS_MAX_CHROM * sizeof(uint32_t) + 255) & ~(size_t)255);
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch`, looked up on its first use.  The
// stream must belong to the current device.
int noalloc_scratch(void* stream, void** out) {
    int dev = 0;
    BITS_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return BITS_E_ARG;
    if (stream) {
        int sdev = -1;
        BITS_CHECK_HIP(hipStreamGetDevice((hipStream_t)stream, &sdev));
        if (sdev != dev) return BITS_E_ARG;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        BITS_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return BITS_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BITS_OK;
}

}  // namespace

extern "C" {

int bits_mc_pvalue(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                   const uint32_t* chrom_len, uint32_t n_chrom, uint64_t seed, uint64_t s0, uint64_t s1,
                   void* d_ws, size_t ws_bytes, uint64_t* d_totals, uint64_t* d_observed, uint64_t* d_n_ge,
                   uint64_t* d_n_le, const bits_launch* launch, void* stream) {
    return mc_pvalue_impl(ref, d_a_start, d_a_end, na, chrom_len, n_chrom, seed, s0, s1, d_ws, ws_bytes, d_totals,
                          d_observed, d_n_ge, d_n_le, launch, stream);
}

int bits_mc_pvalue_noalloc(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                           const uint32_t* chrom_len, uint32_t n_chrom, uint64_t seed, uint64_t s0, uint64_t s1,
                           uint64_t* d_totals, uint64_t* d_observed, uint64_t* d_n_ge, uint64_t* d_n_le,
                           const bits_launch* launch, void* stream) {
    if (na > BITS_NOALLOC_MAX_QUERIES) return BITS_E_WORKSPACE;
    size_t need = 0;
    int rc = bits_mc_workspace(na, &need);
    if (rc != BITS_OK) return rc;
    if (need > kNoallocBytes) return BITS_E_WORKSPACE;
    void* ws = nullptr;
    rc = noalloc_scratch(stream, &ws);
    if (rc != BITS_OK) return rc;
    return mc_pvalue_impl(ref, d_a_start, d_a_end, na, chrom_len, n_chrom, seed, s0, s1, ws, kNoallocBytes, d_totals,
                          d_observed, d_n_ge, d_n_le, launch, stream);
}

// ---------------------------------------------------------------- Monte-Carlo binned by region

namespace {
// Stage timing of bits_mc_binned (off unless bits_mc_binned_timing(1)): four
// events per pass of the last call, created on first use and kept.
struct BinTiming {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;   // 4 per pass
    size_t used = 0;              // events recorded by the last call
};
BinTiming& bin_timing() {
    static BinTiming t;
    return t;
}
}  // namespace

int bits_mc_binned_timing(int enable) {
    BinTiming& t = bin_timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.on = enable != 0;
    t.used = 0;
    return BITS_OK;
}

int bits_mc_binned_stage_ms(float* ms) {
    if (!ms) return BITS_E_ARG;
    BinTiming& t = bin_timing();
    std::lock_guard<std::mutex> g(t.mu);
    ms[0] = ms[1] = ms[2] = 0.0f;
    if (!t.used) return BITS_OK;
    BITS_CHECK_HIP(hipEventSynchronize(t.ev[t.used - 1]));
    for (size_t b = 0; b + 4 <= t.used; b += 4) {
        for (int k = 0; k < 3; ++k) {
            float x = 0.0f;
            BITS_CHECK_HIP(hipEventElapsedTime(&x, t.ev[b + k], t.ev[b + k + 1]));
            ms[k] += x;
        }
    }
    return BITS_OK;
}

namespace {
struct BinWsLayout {
    BinLayout L;
    size_t table, rs, re, flag, offsets, tiles, cell_region, desc, seg_start, seg_cnt, partial, packed, recs, total;
};

bool bin_ws_layout(uint64_t na, uint64_t n, const uint32_t* chrom_len, uint32_t n_chrom, uint32_t batch,
                   BinWsLayout* W) {
    if (!bin_layout(chrom_len, n_chrom, n, &W->L)) return false;
    const uint64_t nc = W->L.ncells, nr = W->L.nreg_max;
    size_t o = 0;
    W->table = o;
    o += 4 * align256((size_t)na * sizeof(uint32_t)) + 2 * align256(BITS_MAX_CHROM * sizeof(uint32_t));
    W->rs = o; o = align256(o + nc * sizeof(uint32_t));
    W->re = o; o = align256(o + nc * sizeof(uint32_t));
    W->flag = o; o = align256(o + nc * sizeof(uint32_t));
    W->offsets = o; o = align256(o + (nc + 1) * sizeof(uint64_t));
    W->tiles = o; o = align256(o + scan_tiles(nc) * sizeof(uint64_t));
    W->cell_region = o; o = align256(o + nc * sizeof(uint32_t));
    W->desc = o; o = align256(o + (nr + 1) * 16);
    W->seg_start = o; o = align256(o + (size_t)batch * nr * sizeof(uint32_t));
    W->seg_cnt = o; o = align256(o + (size_t)batch * nr * sizeof(uint32_t));
    W->partial = o; o = align256(o + (size_t)batch * nr * W->L.splits * sizeof(uint64_t));
    W->packed = o; o = align256(o + (size_t)na * 8);
    W->recs = o; o = align256(o + (size_t)batch * na * 8);
    W->total = o;
    return true;
}
}  // namespace

int bits_mc_binned_workspace(uint64_t na, uint64_t n, const uint32_t* chrom_len, uint32_t n_chrom, uint32_t batch,
                             size_t* bytes) {
    if (!bytes || !chrom_len || n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    if (na > 0xFFFFFFFFull || n > 0xFFFFFFFFull || batch == 0 || batch > BITS_MC_BIN_MAX_BATCH) return BITS_E_ARG;
    BinWsLayout W;
    if (!bin_ws_layout(na, n, chrom_len, n_chrom, batch, &W)) return BITS_E_CHROM;
    *bytes = W.total;
    return BITS_OK;
}

int bits_mc_binned(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                   const uint32_t* chrom_len, uint32_t n_chrom, uint64_t seed, uint64_t s0, uint64_t s1,
                   uint32_t batch, void* d_ws, size_t ws_bytes, uint64_t* d_totals, uint64_t* d_observed,
                   uint64_t* d_n_ge, uint64_t* d_n_le, const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (s1 < s0 || !chrom_len || n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    if (!d_observed || !d_n_ge || !d_n_le || (s1 > s0 && !d_totals)) return BITS_E_ARG;
    if (batch == 0 || batch > BITS_MC_BIN_MAX_BATCH) return BITS_E_ARG;
    const uint64_t ns = s1 - s0;
    if (na > 0xFFFFFFFFull) return BITS_E_ARG;
    if (na && ns > ~0ull / na) return BITS_E_ARG;   // counter g = s * na + i must not wrap
    if (na && s1 > (~0ull - na) / na) return BITS_E_ARG;
    uint64_t g = 0;
    for (uint32_t c = 0; c < n_chrom; ++c) g += chrom_len[c];
    if (g > 0xFFFFFFFFull) return BITS_E_CHROM;
    BinWsLayout W;
    if (!bin_ws_layout(na, ref->n, chrom_len, n_chrom, batch, &W)) return BITS_E_CHROM;
    if (na && ref->n && (!d_ws || ws_bytes < W.total)) return BITS_E_WORKSPACE;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    if (cfg.path == BITS_PATH_TIERED) return BITS_E_ARG;   // a counting-only path
    hipStream_t s = (hipStream_t)stream;
    auto* totals = (unsigned long long*)d_totals;
    auto* obs = (unsigned long long*)d_observed;
    BITS_CHECK_HIP(launch_fill_u64(totals, ns, 0ull, s));
    BITS_CHECK_HIP(launch_fill_u64(obs, 1, 0ull, s));
    if (na && ref->n) {
        char* w = (char*)d_ws;
        const size_t stride = align256((size_t)na * sizeof(uint32_t));
        const size_t cstride = align256(BITS_MAX_CHROM * sizeof(uint32_t));
        McTable tab;
        tab.off = (uint32_t*)(w + W.table);
        tab.span = (uint32_t*)(w + W.table + stride);
        tab.len = (uint32_t*)(w + W.table + 2 * stride);
        tab.idx = (uint32_t*)(w + W.table + 3 * stride);
        tab.hist = (uint32_t*)(w + W.table + 4 * stride);
        tab.cursor = (uint32_t*)(w + W.table + 4 * stride + cstride);
        BinWs bw;
        bw.rs = (uint32_t*)(w + W.rs);
        bw.re = (uint32_t*)(w + W.re);
        bw.flag = (uint32_t*)(w + W.flag);
        bw.offsets = (uint64_t*)(w + W.offsets);
        bw.scan_tiles = (uint64_t*)(w + W.tiles);
        bw.cell_region = (uint32_t*)(w + W.cell_region);
        bw.desc = w + W.desc;
        bw.seg_start = (uint32_t*)(w + W.seg_start);
        bw.seg_cnt = (uint32_t*)(w + W.seg_cnt);
        bw.partial = (unsigned long long*)(w + W.partial);
        bw.recs = w + W.recs;
        bw.packed = w + W.packed;
        bw.nreg_max = (uint32_t)W.L.nreg_max;
        bw.splits = W.L.splits;
        BITS_CHECK_HIP(launch_mc_prepare(d_a_start, d_a_end, na, chrom_len, n_chrom, tab, ref->status, s));
        BITS_CHECK_HIP(launch_mc(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, tab, na, seed, s0, 0, totals,
                                 obs, s));
        if (W.L.ncells && ns) {   // a genome of length 0 holds no legal placement
            BITS_CHECK_HIP(launch_bin_regions(chrom_len, n_chrom, ref->bs, ref->be, ref->n, bw, ref->status, s));
            BITS_CHECK_HIP(launch_bin_pack(tab, na, bw, s));
        }
        BinTiming& tm = bin_timing();
        std::unique_lock<std::mutex> tl(tm.mu);
        tm.used = 0;
        // a pass indexes its records in 32 bits: at most (2^32 - 1) / na shuffles
        const uint64_t pass = na ? std::min<uint64_t>(batch, 0xFFFFFFFFull / na) : batch;
        for (uint64_t sb = s0; W.L.ncells && sb < s1; sb += pass) {
            const uint32_t nb = (uint32_t)((s1 - sb) < pass ? (s1 - sb) : pass);
            hipEvent_t* ev = nullptr;
            if (tm.on) {
                while (tm.ev.size() < tm.used + 4) {
                    hipEvent_t e;
                    BITS_CHECK_HIP(hipEventCreate(&e));
                    tm.ev.push_back(e);
                }
                ev = tm.ev.data() + tm.used;
                tm.used += 4;
            }
            BITS_CHECK_HIP(launch_bin_batch(chrom_len, n_chrom, tab, na, ref->bs, ref->be, ref->n, seed, sb, nb, bw,
                                            totals + (sb - s0), s, ev));
        }
    }
    BITS_CHECK_HIP(launch_mc_tail(totals, ns, obs, (unsigned long long*)d_n_ge, (unsigned long long*)d_n_le, s));
    return BITS_OK;
}

// ---------------------------------------------------------------- enumeration

namespace {
struct EnumLayout {
    size_t starts, ends, ids, total;
};
EnumLayout enum_layout(uint64_t n) {
    EnumLayout L;
    size_t o = 0;
    L.starts = o; o = align256(o + (size_t)n * sizeof(uint32_t));
    L.ends = o; o = align256(o + (size_t)n * sizeof(uint32_t));
    L.ids = o; o = align256(o + (size_t)n * sizeof(uint32_t));
    L.total = o;
    return L;
}
}  // namespace

int bits_enum_index_bytes(uint64_t n, size_t* bytes) {
    if (!bytes || n > 0xFFFFFFFFull) return BITS_E_ARG;
    *bytes = enum_layout(n).total;
    return BITS_OK;
}

int bits_enum_index_workspace(uint64_t n, size_t* bytes) {
    if (!bytes || n > 0xFFFFFFFFull) return BITS_E_ARG;
    const uint32_t vm = 2;
    *bytes = sort_workspace_bytes(&n, 1, &vm);
    return BITS_OK;
}

int bits_enum_index_build(const uint32_t* d_b_start, const uint32_t* d_b_end, uint64_t n, void* d_index,
                          size_t index_bytes, void* d_ws, size_t ws_bytes, void* stream) {
    if (n > 0xFFFFFFFFull || !d_index || ((uintptr_t)d_index & 255u)) return BITS_E_ARG;
    if (n && (!d_b_start || !d_b_end || !d_ws)) return BITS_E_ARG;
    const EnumLayout L = enum_layout(n);
    if (index_bytes < L.total) return BITS_E_WORKSPACE;
    if (!n) return BITS_OK;
    size_t need = 0;
    bits_enum_index_workspace(n, &need);
    if (ws_bytes < need) return BITS_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)d_index;
    uint32_t* starts = (uint32_t*)(b + L.starts);
    uint32_t* ends = (uint32_t*)(b + L.ends);
    uint32_t* ids = (uint32_t*)(b + L.ids);
    SortSeg seg{d_b_start, starts, n, 2u, nullptr, ids};
    const int rc = launch_sort(&seg, 1, d_ws, ws_bytes, s);
    if (rc != BITS_OK) return rc;
    BITS_CHECK_HIP(launch_gather_u32(d_b_end, ids, n, ends, s));
    return BITS_OK;
}

int bits_scan_workspace(uint64_t n, size_t* bytes) {
    if (!bytes) return BITS_E_ARG;
    *bytes = align256((size_t)std::max<uint64_t>(scan_tiles(n), 1) * sizeof(uint64_t));
    return BITS_OK;
}

int bits_scan_counts(const uint32_t* d_counts, uint64_t n, uint64_t* d_offsets, void* d_ws, size_t ws_bytes,
                     void* stream) {
    if (!d_offsets || (n && (!d_counts || !d_ws))) return BITS_E_ARG;
    size_t need = 0;
    bits_scan_workspace(n, &need);
    if (n && ws_bytes < need) return BITS_E_WORKSPACE;
    BITS_CHECK_HIP(launch_scan_counts(d_counts, n, d_offsets, (uint64_t*)d_ws, (hipStream_t)stream));
    return BITS_OK;
}

int bits_enum_counts(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                     uint32_t* d_counts, uint32_t* d_first, uint64_t* d_offsets, void* d_ws, size_t ws_bytes,
                     const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (na > 0xFFFFFFFFull || !d_offsets || (na && (!d_counts || !d_first))) return BITS_E_ARG;
    size_t need = 0;
    bits_scan_workspace(na, &need);
    if (na && (!d_ws || ws_bytes < need)) return BITS_E_WORKSPACE;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (na) {
        if (ref->n) {
            BITS_CHECK_HIP(launch_count(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, na, d_counts, nullptr, s,
                                        d_first));
        } else {
            BITS_CHECK_HIP(launch_fill_u32(d_counts, na, 0u, s));
            BITS_CHECK_HIP(launch_fill_u32(d_first, na, 0u, s));
        }
    }
    BITS_CHECK_HIP(launch_scan_counts(d_counts, na, d_offsets, (uint64_t*)d_ws, s));
    return BITS_OK;
}

int bits_enumerate(const void* d_index, uint64_t n, const uint32_t* d_a_start, const uint32_t* d_a_end,
                   uint64_t na, const uint32_t* d_counts, const uint32_t* d_first, const uint64_t* d_offsets,
                   uint32_t* d_pair_a, uint32_t* d_pair_b, uint64_t max_pairs, uint32_t* d_status, void* stream) {
    if (n > 0xFFFFFFFFull || na > 0xFFFFFFFFull) return BITS_E_ARG;
    if (!na) return BITS_OK;
    if (!d_a_start || !d_a_end || !d_counts || !d_offsets) return BITS_E_ARG;
    if (max_pairs && (!d_pair_a || !d_pair_b)) return BITS_E_ARG;
    if (n && (!d_index || ((uintptr_t)d_index & 255u))) return BITS_E_ARG;
    if (!n) return BITS_OK;   // every count is 0
    const EnumLayout L = enum_layout(n);
    const char* b = (const char*)d_index;
    BITS_CHECK_HIP(launch_enumerate((const uint32_t*)(b + L.starts), (const uint32_t*)(b + L.ends),
                                    (const uint32_t*)(b + L.ids), (uint32_t)n, d_a_start, d_a_end, na, d_counts,
                                    d_first, d_offsets, d_pair_a, d_pair_b, max_pairs, d_status,
                                    (hipStream_t)stream));
    return BITS_OK;
}

// ---------------------------------------------------------------- paper orientation

namespace {
struct ResortWs {
    size_t tab, status, s_in, e_in, s_out, e_out, sort, total;
    size_t seg;   // bytes of one round's keys
};
ResortWs resort_ws(uint64_t nb, uint32_t batch) {
    ResortWs W;
    size_t o = 0;
    const size_t col = align256((size_t)nb * sizeof(uint32_t));
    W.seg = (size_t)nb * sizeof(uint32_t);
    W.tab = o; o += 4 * col + 2 * align256(BITS_MAX_CHROM * sizeof(uint32_t));
    W.status = o; o += 256;   // status word used when the caller passes none
    const size_t keys = align256((size_t)batch * W.seg);
    W.s_in = o; o += keys;
    W.e_in = o; o += keys;
    W.s_out = o; o += keys;
    W.e_out = o; o += keys;
    W.sort = o;
    std::vector<uint64_t> ns(2 * (size_t)batch, nb);
    o += align256(sort_workspace_bytes(ns.data(), 2 * batch));
    W.total = o;
    return W;
}
}  // namespace

int bits_mc_resort_workspace(uint64_t nb, uint32_t batch, size_t* bytes) {
    if (!bytes || nb > 0xFFFFFFFFull || batch == 0 || batch > 4096) return BITS_E_ARG;
    *bytes = resort_ws(nb, batch).total;
    return BITS_OK;
}

int bits_mc_resort(const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na, const uint32_t* d_b_start,
                   const uint32_t* d_b_end, uint64_t nb, const uint32_t* chrom_len, uint32_t n_chrom, uint64_t seed,
                   uint64_t s0, uint64_t s1, uint32_t batch, void* d_ws, size_t ws_bytes, uint64_t* d_totals,
                   uint64_t* d_observed, uint64_t* d_n_ge, uint64_t* d_n_le, uint32_t* d_status, void* stream) {
    if (nb > 0xFFFFFFFFull || s1 < s0 || batch == 0 || batch > 4096) return BITS_E_ARG;
    if (!chrom_len || n_chrom == 0 || n_chrom > BITS_MAX_CHROM) return BITS_E_ARG;
    if (!d_observed || !d_n_ge || !d_n_le || (s1 > s0 && !d_totals)) return BITS_E_ARG;
    if ((na && (!d_a_start || !d_a_end)) || (nb && (!d_b_start || !d_b_end))) return BITS_E_ARG;
    const uint64_t ns = s1 - s0;
    if (nb && s1 > (~0ull - nb) / nb) return BITS_E_ARG;   // counter g = s * nb + j must not wrap
    uint64_t g = 0;
    for (uint32_t c = 0; c < n_chrom; ++c) g += chrom_len[c];
    if (g > 0xFFFFFFFFull) return BITS_E_CHROM;
    const ResortWs W = resort_ws(nb, batch);
    if (nb && (!d_ws || ws_bytes < W.total || ((uintptr_t)d_ws & 255u))) return BITS_E_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    auto* totals = (unsigned long long*)d_totals;
    auto* obs = (unsigned long long*)d_observed;
    BITS_CHECK_HIP(launch_fill_u64(totals, ns, 0ull, s));
    BITS_CHECK_HIP(launch_fill_u64(obs, 1, 0ull, s));
    if (nb && na) {
        char* w = (char*)d_ws;
        const size_t col = align256((size_t)nb * sizeof(uint32_t)), cstride = align256(BITS_MAX_CHROM * 4);
        McTable tab;
        tab.off = (uint32_t*)(w + W.tab);
        tab.span = (uint32_t*)(w + W.tab + col);
        tab.len = (uint32_t*)(w + W.tab + 2 * col);
        tab.idx = (uint32_t*)(w + W.tab + 3 * col);
        tab.hist = (uint32_t*)(w + W.tab + 4 * col);
        tab.cursor = (uint32_t*)(w + W.tab + 4 * col + cstride);
        uint32_t* S_in = (uint32_t*)(w + W.s_in);
        uint32_t* E_in = (uint32_t*)(w + W.e_in);
        uint32_t* S_out = (uint32_t*)(w + W.s_out);
        uint32_t* E_out = (uint32_t*)(w + W.e_out);
        void* sort_ws = w + W.sort;
        const size_t sort_bytes = W.total - W.sort;
        // B's per-interval table (chromosome offset, legal starts, length, index), computed once
        uint32_t* status = d_status ? d_status : (uint32_t*)(w + W.status);
        BITS_CHECK_HIP(launch_mc_prepare(d_b_start, d_b_end, nb, chrom_len, n_chrom, tab, status, s));
        auto run = [&](uint64_t first, uint32_t rounds, bool identity, unsigned long long* out) -> int {
            BITS_CHECK_HIP(launch_place_rounds(tab, d_b_start, nb, seed, first, rounds, identity, S_in, E_in, s));
            std::vector<SortSeg> segs;
            segs.reserve(2 * (size_t)rounds);
            for (uint32_t r = 0; r < rounds; ++r) {
                segs.push_back({S_in + (size_t)r * nb, S_out + (size_t)r * nb, nb});
                segs.push_back({E_in + (size_t)r * nb, E_out + (size_t)r * nb, nb});
            }
            const int rc = launch_sort(segs.data(), 2 * rounds, sort_ws, sort_bytes, s);
            if (rc != BITS_OK) return rc;
            BITS_CHECK_HIP(launch_sort_report(sort_ws, status, s));
            BITS_CHECK_HIP(launch_count_rounds(S_out, E_out, nb, rounds, d_a_start, d_a_end, na, out, status, s));
            return BITS_OK;
        };
        int rc = run(0, 1, true, obs);
        if (rc != BITS_OK) return rc;
        for (uint64_t b = 0; b < ns; b += batch) {
            const uint32_t r = (uint32_t)std::min<uint64_t>(batch, ns - b);
            rc = run(s0 + b, r, false, totals + b);
            if (rc != BITS_OK) return rc;
        }
    }
    BITS_CHECK_HIP(launch_mc_tail(totals, ns, obs, (unsigned long long*)d_n_ge, (unsigned long long*)d_n_le, s));
    return BITS_OK;
}

double bits_pvalue(uint64_t n_ge, uint64_t n_shuffles) {
    return (1.0 + (double)n_ge) / ((double)n_shuffles + 1.0);
}

double bits_pvalue_lower(uint64_t n_le, uint64_t n_shuffles) {
    return (1.0 + (double)n_le) / ((double)n_shuffles + 1.0);
}

double bits_pvalue_two_sided(uint64_t n_ge, uint64_t n_le, uint64_t n_shuffles) {
    const double p = 2.0 * std::min(bits_pvalue(n_ge, n_shuffles), bits_pvalue_lower(n_le, n_shuffles));
    return p < 1.0 ? p : 1.0;
}

int bits_mc_median(const uint64_t* d_totals, uint64_t n, uint64_t* d_lo, uint64_t* d_hi, void* stream) {
    if (!d_totals || !d_lo || !d_hi || n == 0 || n > 0xFFFFFFFFull) return BITS_E_ARG;
    BITS_CHECK_HIP(launch_select_u64((const unsigned long long*)d_totals, n, (n - 1) / 2, n / 2,
                                     (unsigned long long*)d_lo, (unsigned long long*)d_hi, (hipStream_t)stream));
    return BITS_OK;
}

double bits_enrichment(uint64_t observed, uint64_t median_lo, uint64_t median_hi) {
    const double median = ((double)median_lo + (double)median_hi) * 0.5;
    return std::log2((double)observed / median);
}

int bits_decide(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                uint32_t* d_found, uint64_t* d_witness, const bits_launch* launch, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (!d_found || !d_witness) return BITS_E_ARG;
    LaunchCfg cfg;
    rc = resolve_launch(ref, launch, &cfg);
    if (rc != BITS_OK) return rc;
    if (cfg.path == BITS_PATH_TIERED) return BITS_E_ARG;   // a counting-only path
    hipStream_t s = (hipStream_t)stream;
    BITS_CHECK_HIP(launch_fill_u32(d_found, 1, 0u, s));
    BITS_CHECK_HIP(launch_fill_u64((unsigned long long*)d_witness, 1, ~0ull, s));
    if (ref->n == 0) return BITS_OK;
    BITS_CHECK_HIP(launch_decide(make_search_args(ref, cfg), cfg, d_a_start, d_a_end, na, d_found,
                                 (unsigned long long*)d_witness, s));
    return BITS_OK;
}

// ---------------------------------------------------------------- batch

struct bits_batch_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
struct BatchWs {
    size_t refs, qs, items, wg, total;
};
BatchWs batch_ws(uint32_t n_ref, uint32_t n_q, uint64_t n_items, uint32_t n_wg) {
    BatchWs w;
    size_t o = 0;
    w.refs = o; o = align256(o + sizeof(BatchRef) * n_ref);
    w.qs = o; o = align256(o + sizeof(BatchQuery) * n_q);
    w.items = o; o = align256(o + sizeof(BatchItem) * n_items);
    w.wg = o; o = align256(o + sizeof(uint32_t) * ((size_t)n_wg + 1));
    w.total = o;
    return w;
}
constexpr uint32_t kMaxBatchWg = 256u * 16u;
}  // namespace

int bits_batch_workspace(const uint64_t* na, uint32_t n_q, uint32_t n_ref, size_t* bytes) {
    if (!bytes || (n_q && !na)) return BITS_E_ARG;
    uint64_t tiles = 0;
    for (uint32_t i = 0; i < n_q; ++i) tiles += (na[i] + 255) / 256;   // smallest tile: 256 x 1
    *bytes = batch_ws(n_ref, n_q, tiles * n_ref, kMaxBatchWg).total;
    return BITS_OK;
}

int bits_batch_create(const bits_ref* refs, uint32_t n_ref, const uint32_t* const* d_a_start,
                      const uint32_t* const* d_a_end, const uint64_t* na, uint32_t n_q, uint64_t* d_pair_totals,
                      void* d_ws, size_t ws_bytes, const bits_launch* launch, void* stream, bits_batch_plan** plan) {
    if (!plan || !refs || !d_a_start || !d_a_end || !na || !d_pair_totals || !d_ws || !n_ref || !n_q)
        return BITS_E_ARG;
    *plan = nullptr;
    uint32_t max_depth = 0;
    bool all_learned = true;
    for (uint32_t j = 0; j < n_ref; ++j) {
        if (!ref_ok(&refs[j])) return BITS_E_ARG;
        max_depth = std::max(max_depth, refs[j].depth);
        all_learned = all_learned && refs[j].learned;
    }
    for (uint32_t i = 0; i < n_q; ++i) {
        if (na[i] && (!d_a_start[i] || !d_a_end[i])) return BITS_E_ARG;
        if (na[i] > 0xFFFFFFFFull) return BITS_E_ARG;
    }
    LaunchCfg cfg{1024u, 2u, max_depth, 0u, all_learned ? BITS_PATH_LEARNED : BITS_PATH_PLAIN};
    if (launch) {
        if (launch->block) cfg.block = launch->block;
        if (launch->qpl) cfg.qpl = launch->qpl;
        if (launch->depth != 0xFFFFFFFFu) cfg.depth = std::min(launch->depth, max_depth);
        cfg.grid = launch->grid;
        if (launch->path == BITS_PATH_PLAIN || launch->path == BITS_PATH_LEARNED) cfg.path = launch->path;
        else if (launch->path != BITS_PATH_AUTO) return BITS_E_ARG;
    }
    if (cfg.path == BITS_PATH_LEARNED && !all_learned) return BITS_E_ARG;
    if ((cfg.block != 256 && cfg.block != 512 && cfg.block != 1024) || (cfg.qpl != 1 && cfg.qpl != 2 && cfg.qpl != 4))
        return BITS_E_ARG;
    // the learned path's per-wave scratch grows with qpl: step the block down until it fits
    while (cfg.path == BITS_PATH_LEARNED && cfg.block > 256 &&
           search_lds_bytes(true, 0, (int)cfg.qpl, cfg.block) + 1024 > device_lds_per_block())
        cfg.block >>= 1;
    if (cfg.path == BITS_PATH_LEARNED) cfg.depth = 0;
    const uint32_t tile = cfg.block * cfg.qpl;

    // Work list ordered by reference, then query set, then tile.
    std::vector<BatchItem> items;
    std::vector<double> cost;
    for (uint32_t j = 0; j < n_ref; ++j) {
        const double per_q = std::log2((double)refs[j].n + 2.0) + 8.0;
        for (uint32_t i = 0; i < n_q; ++i)
            for (uint64_t b = 0; b < na[i]; b += tile) {
                const uint32_t c = (uint32_t)std::min<uint64_t>(tile, na[i] - b);
                items.push_back({i, j, (uint32_t)b, c});
                cost.push_back(c * per_q);
            }
    }
    uint32_t n_wg = cfg.grid ? cfg.grid : (uint32_t)device_cu_count() * (uint32_t)batch_blocks_per_cu(cfg, cfg.depth);
    n_wg = std::max(1u, std::min({n_wg, kMaxBatchWg, (uint32_t)std::max<size_t>(items.size(), 1)}));
    const BatchWs W = batch_ws(n_ref, n_q, items.size(), n_wg);
    if (ws_bytes < W.total) return BITS_E_WORKSPACE;
    // Contiguous partition of the work list with near-equal cost per workgroup.
    std::vector<uint32_t> wg(n_wg + 1, (uint32_t)items.size());
    double total = 0.0;
    for (double c : cost) total += c;
    wg[0] = 0;
    double acc = 0.0;
    uint32_t w = 1;
    for (size_t k = 0; k < items.size() && w < n_wg; ++k) {
        acc += cost[k];
        while (w < n_wg && acc >= total * w / n_wg) wg[w++] = (uint32_t)(k + 1);
    }
    std::vector<BatchRef> rtab(n_ref);
    for (uint32_t j = 0; j < n_ref; ++j) {
        const bits_ref& r = refs[j];
        const bool L = cfg.path == BITS_PATH_LEARNED;
        rtab[j] = {r.bs, r.be, r.tree, L ? (const bits_rmi_model*)r.rmi : nullptr, L ? r.heads : nullptr,
                   L ? r.heads + heads_len(r.n) : nullptr, fallback_counter(&r), (uint32_t)r.n, 1u << r.depth,
                   std::min(r.depth, cfg.depth), 0u};
    }
    std::vector<BatchQuery> qtab(n_q);
    for (uint32_t i = 0; i < n_q; ++i) qtab[i] = {d_a_start[i], d_a_end[i], na[i]};
    hipStream_t s = (hipStream_t)stream;
    char* b = (char*)d_ws;
    BITS_CHECK_HIP(hipMemcpyAsync(b + W.refs, rtab.data(), sizeof(BatchRef) * n_ref, hipMemcpyHostToDevice, s));
    BITS_CHECK_HIP(hipMemcpyAsync(b + W.qs, qtab.data(), sizeof(BatchQuery) * n_q, hipMemcpyHostToDevice, s));
    if (!items.empty())
        BITS_CHECK_HIP(hipMemcpyAsync(b + W.items, items.data(), sizeof(BatchItem) * items.size(),
                                      hipMemcpyHostToDevice, s));
    BITS_CHECK_HIP(hipMemcpyAsync(b + W.wg, wg.data(), sizeof(uint32_t) * (n_wg + 1), hipMemcpyHostToDevice, s));
    BITS_CHECK_HIP(hipStreamSynchronize(s));

    bits_batch_plan* p = new (std::nothrow) bits_batch_plan();
    if (!p) return BITS_E_ARG;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete p;
        return BITS_E_HIP;
    }
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        ok = launch_fill_u64((unsigned long long*)d_pair_totals, (uint64_t)n_q * n_ref, 0ull, cs) == hipSuccess;
        ok = ok && launch_batch((const BatchRef*)(b + W.refs), (const BatchQuery*)(b + W.qs),
                                (const BatchItem*)(b + W.items), (const uint32_t*)(b + W.wg), n_wg, n_ref, cfg.depth,
                                cfg, (unsigned long long*)d_pair_totals, refs[0].status, cs) == hipSuccess;
        hipGraph_t g = nullptr;
        const bool ended = hipStreamEndCapture(cs, &g) == hipSuccess;
        ok = ok && ended && g;
        p->graph = g;
    }
    if (ok) ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(cs);
    if (!ok) {
        bits_batch_destroy(p);
        return BITS_E_HIP;
    }
    *plan = p;
    return BITS_OK;
}

int bits_batch_run(bits_batch_plan* plan, void* stream) {
    if (!plan || !plan->exec) return BITS_E_ARG;
    BITS_CHECK_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return BITS_OK;
}

int bits_batch_destroy(bits_batch_plan* plan) {
    if (!plan) return BITS_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return BITS_OK;
}

// ---------------------------------------------------------------- autotuner

int bits_autotune_count(const bits_ref* ref, const uint32_t* d_a_start, const uint32_t* d_a_end, uint64_t na,
                        uint64_t* d_total, uint32_t path, bits_launch* best, float* best_ms, void* stream) {
    int rc = check_queries(ref, d_a_start, d_a_end, na);
    if (rc != BITS_OK) return rc;
    if (!d_total || !best || !best_ms ||
        (path != BITS_PATH_PLAIN && path != BITS_PATH_LEARNED && path != BITS_PATH_TIERED))
        return BITS_E_ARG;
    if (path == BITS_PATH_LEARNED && !ref->learned) return BITS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    std::vector<bits_launch> cand;
    const uint32_t dmin = ref->depth > 8 ? 8 : ref->depth;
    for (uint32_t block : {256u, 512u, 1024u})
        for (uint32_t qpl : {1u, 2u, 4u}) {
            if (path == BITS_PATH_LEARNED) {
                cand.push_back({block, qpl, 0u, 0u, path});
            } else {
                for (uint32_t d = ref->depth + 1; d-- > dmin;) cand.push_back({block, qpl, d, 0u, path});
            }
        }
    hipEvent_t e0, e1;
    BITS_CHECK_HIP(hipEventCreate(&e0));
    BITS_CHECK_HIP(hipEventCreate(&e1));
    float bestt = 1e30f;
    bits_launch bl = cand.front();
    for (const bits_launch& c : cand) {
        rc = bits_count(ref, d_a_start, d_a_end, na, d_total, &c, stream);   // warm-up
        if (rc != BITS_OK) break;
        float tmin = 1e30f;
        for (int r = 0; r < 3; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = BITS_E_HIP; break; }
            rc = bits_count(ref, d_a_start, d_a_end, na, d_total, &c, stream);
            if (rc != BITS_OK) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = BITS_E_HIP; break; }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        if (rc != BITS_OK) break;
        if (tmin < bestt) {
            bestt = tmin;
            bl = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BITS_OK) return rc;
    *best = bl;
    *best_ms = bestt;
    return BITS_OK;
}

int bits_autotune_batch(const bits_ref* refs, uint32_t n_ref, const uint32_t* const* d_a_start,
                        const uint32_t* const* d_a_end, const uint64_t* na, uint32_t n_q, uint32_t path,
                        uint64_t* d_pair_totals, void* d_ws, size_t ws_bytes, bits_launch* best, float* best_ms,
                        void* stream) {
    if (!refs || !n_ref || !best || !best_ms || (path != BITS_PATH_PLAIN && path != BITS_PATH_LEARNED))
        return BITS_E_ARG;
    uint32_t max_depth = 0;
    for (uint32_t j = 0; j < n_ref; ++j) {
        if (!ref_ok(&refs[j])) return BITS_E_ARG;
        if (path == BITS_PATH_LEARNED && !refs[j].learned) return BITS_E_ARG;
        max_depth = std::max(max_depth, refs[j].depth);
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<bits_launch> cand;
    const uint32_t dmin = max_depth > 8 ? 8 : max_depth;
    for (uint32_t block : {256u, 512u, 1024u})
        for (uint32_t qpl : {1u, 2u, 4u}) {
            if (path == BITS_PATH_LEARNED) {
                cand.push_back({block, qpl, 0u, 0u, path});
            } else {
                for (uint32_t d = max_depth + 1; d-- > dmin;) cand.push_back({block, qpl, d, 0u, path});
            }
        }
    hipEvent_t e0, e1;
    BITS_CHECK_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BITS_E_HIP;
    }
    int rc = BITS_OK;
    float bestt = 1e30f;
    bits_launch bl = cand.front();
    for (const bits_launch& c : cand) {
        bits_batch_plan* plan = nullptr;
        rc = bits_batch_create(refs, n_ref, d_a_start, d_a_end, na, n_q, d_pair_totals, d_ws, ws_bytes, &c, stream,
                               &plan);
        if (rc != BITS_OK) break;
        rc = bits_batch_run(plan, stream);   // warm-up
        float tmin = 1e30f;
        for (int r = 0; r < 3 && rc == BITS_OK; ++r) {
            if (hipEventRecord(e0, s) != hipSuccess) { rc = BITS_E_HIP; break; }
            rc = bits_batch_run(plan, stream);
            if (rc != BITS_OK) break;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { rc = BITS_E_HIP; break; }
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        bits_batch_destroy(plan);
        if (rc != BITS_OK) break;
        if (tmin < bestt) {
            bestt = tmin;
            bl = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BITS_OK) return rc;
    *best = bl;
    *best_ms = bestt;
    return BITS_OK;
}

int bits_rmi_window(const bits_ref* ref, uint32_t which, const uint32_t* d_x, uint64_t n, uint32_t* d_lo,
                    uint32_t* d_hi, void* stream) {
    if (!ref_ok(ref) || !ref->learned || which > 1 || (n && (!d_x || !d_lo || !d_hi))) return BITS_E_ARG;
    if (!ref->n) return BITS_E_ARG;
    LaunchCfg cfg{256u, 1u, 0u, 0u, BITS_PATH_LEARNED};
    BITS_CHECK_HIP(launch_rmi_window(make_search_args(ref, cfg), which, d_x, n, d_lo, d_hi, (hipStream_t)stream));
    return BITS_OK;
}

int bits_rmi_leaf_grad(const float* d_u, const float* d_t, uint32_t m, const float* d_params, float* d_grad,
                       float* d_loss, void* stream) {
    if (m > BITS_RMI_MAX_POINTS || !d_params || !d_grad || !d_loss || (m && (!d_u || !d_t))) return BITS_E_ARG;
    BITS_CHECK_HIP(launch_rmi_leaf_grad(d_u, d_t, m, d_params, d_grad, d_loss, (hipStream_t)stream));
    return BITS_OK;
}

}  // extern "C"
