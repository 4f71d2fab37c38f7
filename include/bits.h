/*
 * bits.h -- C ABI of libbits.so: Binary Interval Search (BITS) on AMD
 * Instinct MI355X (gfx950).
 *
 * Method: Layer, Skadron, Robins, Hall, Quinlan, "Binary Interval Search
 * (BITS): A Scalable Algorithm for Counting Interval Intersections",
 * Bioinformatics 2012.  Section/algorithm references below are to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Intervals are closed, 0-based uint32 coordinates [start, end] with
 *    start <= end (Sec. 1.1: a and b intersect when a.start <= b.end and
 *    a.end >= b.start).  Sets are passed as two arrays (structure of arrays).
 *  - Pointers prefixed d_ (and every array argument unless marked "host") are
 *    DEVICE pointers on the current HIP device, owned by the caller.  The
 *    library never allocates device memory in these calls: scratch comes
 *    from caller-provided workspaces sized by the *_workspace functions.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *    compute call only enqueues work on it and returns; results are valid
 *    once the stream has reached that point.  Calls on one stream are
 *    ordered; two streams must not write the same outputs concurrently.
 *  - Return value: a bits_status.  Host-detectable argument errors return
 *    immediately without enqueuing anything.  Errors found while the kernels
 *    run (an interval with start > end, an interval that leaves its
 *    chromosome) set bits in a device status word, read by bits_get_status.
 *    Nothing aborts or throws across this boundary.
 *  - Counts are exact integers: per-query counts uint32 (<= |B| < 2^32),
 *    totals uint64.
 */
#ifndef BITS_H
#define BITS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bits_status {
    BITS_OK = 0,
    BITS_E_ARG = 1,          /* null pointer with n > 0, size or parameter out of range */
    BITS_E_INTERVAL = 2,     /* an interval with start > end (device-detected) */
    BITS_E_CHROM = 3,        /* an interval outside its chromosome, or genome >= 2^32 */
    BITS_E_WORKSPACE = 4,    /* caller buffer smaller than the *_workspace/_bytes size */
    BITS_E_HIP = 5,          /* a HIP runtime call failed */
    BITS_E_UNSUPPORTED = 6   /* no usable gfx950 device */
} bits_status;

/* Device status-word bits (OR-ed by kernels). */
#define BITS_FLAG_INTERVAL 0x1u   /* start > end seen */
#define BITS_FLAG_CHROM    0x2u   /* interval outside its chromosome */
#define BITS_FLAG_ENUM     0x4u   /* enumeration: a query's scan found fewer pairs than its
                                     count, or the pair buffer was too small */
#define BITS_FLAG_SORT     0x8u   /* radix sort: a tile gave up waiting for the digit counts
                                     of the tiles before it (never expected; the sorted
                                     output is then invalid) */

#define BITS_MAX_CHROM   256u     /* chromosomes per genome for projection / Monte-Carlo */
#define BITS_MC_BIN_MAX_BATCH 1024u /* shuffles per pass of bits_mc_binned */
#define BITS_NOALLOC_MAX_QUERIES (1u << 20) /* queries per call of bits_mc_pvalue_noalloc */
#define BITS_MAX_DEPTH   13u      /* Eytzinger top-tree levels held in LDS */
#define BITS_RMI_LEAVES  4096u    /* leaf models per learned index */
#define BITS_RMI_HIDDEN  16u      /* hidden ReLU units per leaf model */
#define BITS_RMI_PARAMS  49u      /* w1[16], b1[16], w2[16], b2 */
#define BITS_RMI_MAX_POINTS 2048u /* training points per leaf */

/* Search path selection for a call (bits_launch.path). */
#define BITS_PATH_AUTO    0u      /* learned index if the reference has one, else plain */
#define BITS_PATH_PLAIN   1u      /* LDS Eytzinger top tree + bisection in HBM */
#define BITS_PATH_LEARNED 2u      /* learned CDF index + error-window search over the line heads (needs learned ref) */
#define BITS_PATH_TIERED  3u      /* counting only: LDS top tree, then bisection over the
                                     32-key node tier (the line heads), then one 128-byte line;
                                     no model (the index the learned path is measured against) */

/* Launch shape of the search kernels.  A NULL bits_launch* means the
 * library defaults; bits_autotune_count picks one by timing. */
typedef struct bits_launch {
    uint32_t block;   /* threads per workgroup: 256, 512 or 1024 (0 = default 1024); the learned
                         path uses a smaller one when its LDS scratch would not fit */
    uint32_t qpl;     /* queries interleaved per lane: 1, 2 or 4 (0 = default 2) */
    uint32_t depth;   /* top-tree levels searched from LDS, <= the reference's depth
                         (0xFFFFFFFF = the reference's depth; 0 = no LDS tree) */
    uint32_t grid;    /* workgroups, 0 = one persistent wave of workgroups per CU slot */
    uint32_t path;    /* BITS_PATH_* */
} bits_launch;

/* Reference (database) index over B.  Filled by bits_ref_init from ONE
 * caller-allocated device block; every pointer below points into it.
 * Layout of the block (each region 256-byte aligned):
 *   status[64]   uint32: [0] status bits, [2..3] uint64 learned-path fallbacks
 *   tree         uint32[2][2^depth]: Eytzinger splitters of B_S then B_E,
 *                node k (1-based BFS order) at [k]; entry 0 unused
 *   rmi          (learned only) 2 x bits_rmi_model (128-byte header + 4096 leaves)
 *   heads        uint32[2][hl], line heads of B_S then B_E (the 32-key node tier):
 *                H[j] = K[32 j] (first key of each 128-byte line) for j < ceil(n/32),
 *                then 0xFFFFFFFF; hl = 32 * ceil((ceil(n/32) + 32) / 32)
 *   bs, be       uint32[n] each: sorted B_S and B_E (Sec. 2.1, Algorithm 2); the rest
 *                of each array's last 128-byte line is filled with 0xFFFFFFFF */
typedef struct bits_ref {
    uint64_t n;          /* |B|, < 2^32 */
    uint32_t depth;      /* top-tree depth built: min(requested, floor(log2 n)) */
    uint32_t learned;    /* 1 if the learned CDF index is present */
    uint32_t *bs;        /* device: sorted starts */
    uint32_t *be;        /* device: sorted ends */
    uint32_t *tree;      /* device: 2 * 2^depth splitters */
    void *rmi;           /* device: 2 bits_rmi_model (starts, ends) or NULL */
    uint32_t *heads;     /* device: line heads of B_S, then of B_E */
    uint32_t *status;    /* device: status word and counters */
    void *block;         /* device: base of the caller's block */
    size_t block_bytes;
} bits_ref;

/* One leaf of the learned CDF index: one 128-byte line.  Keys routed to the
 * leaf are the contiguous sorted range [rlo, rlo + cnt).  The model is
 *   y(u) = b2 + sum_j w2_j relu(w1_j u + b1_j),  j = 0..15,
 * u = (x - kmin) * kinv, predicted rank rlo + clamp(rint(y * cnt), 0, cnt).
 * w1, b1, w2 are stored as IEEE binary16 (fp32 arithmetic); kinv and b2 as
 * fp32 bit patterns.  The record is laid out for 4 lanes reading it with two
 * 16-byte loads each: lane q takes a[q] (bytes 16q..16q+15) and b[q]
 * (bytes 64+16q..), i.e. header words h[] and hidden units 4q..4q+3.
 *   a[0].h = {kmin, kmax}      kmin = 0xFFFFFFFF for an empty leaf
 *   a[1].h = {rlo, cnt}
 *   a[2].h = {kinv, b2}        kinv = 1 / max(1, kmax - kmin)
 *   a[3].h = {err_lo | err_hi << 16, loss}
 * err_lo / err_hi: largest over- / under-prediction of the rank over the
 * leaf's keys (capped at 65535; a capped window only causes a fallback). */
typedef struct bits_rmi_leaf {
    struct { uint32_t h[2]; uint16_t w1[4]; } a[4];
    struct { uint16_t b1[4]; uint16_t w2[4]; } b[4];
} bits_rmi_leaf;

/* Learned CDF index of one sorted array: root line routing to 4096 leaves. */
typedef struct bits_rmi_model {
    float root_a, root_b;    /* leaf = clamp(floor(fmaf(root_a, (float)x, root_b)), 0, 4095) */
    double fit_a, fit_b;     /* least-squares line rank ~ fit_a * key + fit_b (fp64) */
    uint64_t n;
    uint32_t pad[24];
    bits_rmi_leaf leaf[BITS_RMI_LEAVES];
} bits_rmi_model;

/* Training settings for the learned index (NULL = defaults). */
typedef struct bits_train {
    uint32_t epochs;      /* full-batch Adam steps per leaf (default 300; 0 = init only) */
    uint32_t max_points;  /* training points per leaf, stride-sampled (0 = default 256; above 2048 clamps to 2048) */
    float lr;             /* Adam step size (default 2e-3) */
    float beta1, beta2;   /* Adam moments (defaults 0.9, 0.999) */
} bits_train;

/* Summary of a learned index (host-side result of bits_rmi_info). */
typedef struct bits_rmi_stats {
    double mean_window;      /* mean err_lo + err_hi + 1 over non-empty leaves, both arrays */
    uint32_t max_window;
    uint32_t empty_leaves;
    double mean_loss;
    uint64_t fallbacks;      /* queries whose window failed verification since the last reset */
} bits_rmi_stats;

/* ---------------------------------------------------------------------- */
/* Library                                                                 */
/* ---------------------------------------------------------------------- */

/* ABI version (monotone integer). */
int bits_version(void);

/* Human-readable name of a bits_status. Never NULL. */
const char *bits_strerror(int status);

/* Waits for `stream`, then copies the device status word d_status (4 bytes)
 * into *status_out (BITS_FLAG_* bits).  Returns BITS_E_HIP on a runtime error. */
int bits_get_status(const uint32_t *d_status, void *stream, uint32_t *status_out);

/* Enqueues a zero fill of the device status word. */
int bits_clear_status(uint32_t *d_status, void *stream);

/* ---------------------------------------------------------------------- */
/* Projection (Sec. 2.1, "BITS solution to the counting problem"; Sec. 3.2) */
/* ---------------------------------------------------------------------- */

/* Maps chromosome-local intervals to the one-dimensional genome: global =
 * (sum of the lengths of chromosomes before c) + local.
 *   chrom_len  host, n_chrom lengths (n_chrom <= BITS_MAX_CHROM, sum < 2^32)
 *   d_chrom, d_lstart, d_lend   device, n each: chromosome id, local closed interval
 *   d_start, d_end              device, n each: output global interval
 *   d_status   device status word (nullable): BITS_FLAG_CHROM for a bad id or
 *              an interval past its chromosome's end, BITS_FLAG_INTERVAL for
 *              start > end.  Such intervals are written as given. */
int bits_project(const uint32_t *chrom_len, uint32_t n_chrom, const uint32_t *d_chrom,
                 const uint32_t *d_lstart, const uint32_t *d_lend, uint64_t n,
                 uint32_t *d_start, uint32_t *d_end, uint32_t *d_status, void *stream);

/* ---------------------------------------------------------------------- */
/* Reference index: sort (Algorithm 2), top tree, learned CDF model         */
/* ---------------------------------------------------------------------- */

/* Bytes of the device block for a reference of n intervals. */
int bits_ref_bytes(uint64_t n, uint32_t depth, int learned, size_t *bytes);

/* Host only: carves the caller's device block (at least bits_ref_bytes) into
 * *ref.  depth is clamped to min(depth, BITS_MAX_DEPTH, floor(log2 n)). */
int bits_ref_init(void *d_block, size_t block_bytes, uint64_t n, uint32_t depth, int learned,
                  bits_ref *ref);

/* Workspace bytes bits_sort_ref needs for n intervals. */
int bits_sort_ref_workspace(uint64_t n, size_t *bytes);

/* Builds the reference index from B (Algorithm 2's setup): B_S and B_E are
 * sorted ascending by an on-device LSD radix sort (8-bit digits, digits
 * constant over the whole input skipped), the Eytzinger top tree of each is
 * built, and if ref->learned the learned CDF index is trained on the device
 * and its per-leaf error windows measured.  Clears the status word (then
 * BITS_FLAG_SORT reports a sort that could not complete).
 *   d_b_start, d_b_end  device, ref->n each, unsorted (not modified)
 *   d_ws, ws_bytes      device workspace >= bits_sort_ref_workspace(n)
 *   train               host, NULL for defaults (ignored if not learned)
 * The intervals' start <= end is not checked here (starts and ends are sorted
 * independently); count calls check their queries. */
int bits_sort_ref(const uint32_t *d_b_start, const uint32_t *d_b_end, const bits_ref *ref,
                  void *d_ws, size_t ws_bytes, const bits_train *train, void *stream);

/* Several references in one segmented sort: refs[j] (host array) each with
 * its own block, inputs d_b_start[j], d_b_end[j] (host arrays of device
 * pointers).  Same semantics as bits_sort_ref for each j. */
int bits_sort_refs_workspace(const uint64_t *n, uint32_t n_ref, size_t *bytes);
int bits_sort_refs(const uint32_t *const *d_b_start, const uint32_t *const *d_b_end,
                   const bits_ref *refs, uint32_t n_ref, void *d_ws, size_t ws_bytes,
                   const bits_train *train, void *stream);

/* Waits for `stream` and summarises the learned index of ref into *out. */
int bits_rmi_info(const bits_ref *ref, void *stream, bits_rmi_stats *out);

/* ---------------------------------------------------------------------- */
/* Counting (Algorithm 1 ICount; Algorithm 2 Counter; Sec. 2.3)            */
/* ---------------------------------------------------------------------- */

/* Per-interval counting sub-problem (Sec. 1.1, problem 3): for each query
 * a_i, d_counts[i] = |{b in B : a_i.start <= b.end and a_i.end >= b.start}|
 * = upper_bound(B_S, a_i.end) - lower_bound(B_E, a_i.start).
 *   d_a_start, d_a_end  device, na each
 *   d_counts            device, na uint32, in query order
 *   d_total             device uint64 (nullable): sum of the counts (overwritten)
 *   launch              host, NULL for defaults
 * A query with start > end sets BITS_FLAG_INTERVAL in ref->status and counts 0. */
int bits_count_per_query(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end,
                         uint64_t na, uint32_t *d_counts, uint64_t *d_total,
                         const bits_launch *launch, void *stream);

/* Counting sub-problem (Sec. 1.1, problem 2; Algorithm 2): *d_total = sum of
 * the per-query counts, exact uint64 (overwritten). */
int bits_count(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end,
               uint64_t na, uint64_t *d_total, const bits_launch *launch, void *stream);

/* Decision (Sec. 1.1, sub-problem 1): *d_found = 1 if some a_i intersects
 * some interval of B, else 0.  Workgroups stop taking tiles of A once a hit
 * is seen.  *d_witness = an index i with count_i > 0 (the smallest among the
 * tiles that ran, so not necessarily the smallest overall), or 2^64 - 1.  A
 * query with start > end sets BITS_FLAG_INTERVAL in ref->status and is
 * skipped. */
int bits_decide(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end, uint64_t na,
                uint32_t *d_found, uint64_t *d_witness, const bits_launch *launch, void *stream);

/* ---------------------------------------------------------------------- */
/* Monte-Carlo significance (Sec. 3.2)                                      */
/* ---------------------------------------------------------------------- */

/* Workspace bytes bits_mc_pvalue needs for na queries (na < 2^32):
 * a per-query table of 16 bytes plus 2 KiB. */
int bits_mc_workspace(uint64_t na, size_t *bytes);

/* Shuffles the query set A against the fixed reference and counts, in one
 * persistent launch over all shuffles [s0, s1).  Shuffle s places query i at
 * a uniformly drawn legal start of its own chromosome, length kept:
 *   g = s * na + i;  (x0,x1,x2,x3) = Philox4x32-10(counter = (lo32 g, hi32 g, 0, 0),
 *                                                  key = (lo32 seed, hi32 seed))
 *   local = floor(((x1 << 32) | x0) * span / 2^64),  span = len_c - L + 1
 *   a'    = [off_c + local, off_c + local + L - 1]
 * (Philox-4x32-10: Salmon et al., SC'11.)
 *   chrom_len        host, n_chrom lengths of the genome A was projected on;
 *                    a query's chromosome is the one holding its start
 *   d_totals         device uint64[s1 - s0]: per-shuffle totals
 *   d_observed       device uint64: total of the unshuffled A
 *   d_n_ge, d_n_le   device uint64: #{s : T_s >= T_obs}, #{s : T_s <= T_obs}
 * The one-sided empirical p-value is bits_pvalue(n_ge, s1 - s0).  A query
 * outside its chromosome sets BITS_FLAG_CHROM and is left out of every total.
 * The queries are first grouped by chromosome in d_ws, and the shuffles run
 * over that table with one group of workgroups per part of the genome; with
 * the learned path, each search is the leaf model, one window of line heads
 * and one line of the sorted array.  na must be < 2^32 (BITS_E_ARG). */
int bits_mc_pvalue(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end,
                   uint64_t na, const uint32_t *chrom_len, uint32_t n_chrom, uint64_t seed,
                   uint64_t s0, uint64_t s1, void *d_ws, size_t ws_bytes, uint64_t *d_totals,
                   uint64_t *d_observed, uint64_t *d_n_ge, uint64_t *d_n_le,
                   const bits_launch *launch, void *stream);

/* bits_mc_pvalue without the caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, outputs, flags and
 * results bit for bit as bits_mc_pvalue, less d_ws and ws_bytes: the query
 * table lives in a device array of the library, about 16 MiB, that each GPU
 * the library runs on holds until the process ends.  Its device address is
 * looked up on the first call on a device; after that the call allocates
 * nothing and calls no allocating routine.
 *   na <= BITS_NOALLOC_MAX_QUERIES, else BITS_E_WORKSPACE (nothing enqueued)
 *   stream must belong to the current device, else BITS_E_ARG
 * Every call on one GPU shares that array (each call rebuilds the table it
 * reads, so nothing carries over): calls that overlap on one GPU, on
 * different streams or from different threads, race and give wrong totals. */
int bits_mc_pvalue_noalloc(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end,
                           uint64_t na, const uint32_t *chrom_len, uint32_t n_chrom, uint64_t seed,
                           uint64_t s0, uint64_t s1, uint64_t *d_totals, uint64_t *d_observed,
                           uint64_t *d_n_ge, uint64_t *d_n_le, const bits_launch *launch,
                           void *stream);

/* Workspace bytes of bits_mc_binned for na queries (na < 2^32) against a
 * reference of n intervals on the genome chrom_len[n_chrom], with `batch`
 * shuffles per pass (1 <= batch <= BITS_MC_BIN_MAX_BATCH): the query table
 * of bits_mc_workspace plus 8 bytes per query; about 24 bytes per cell of
 * the genome (cells of 2^S bp,
 * S >= 10 the least that leaves at most 8192 cells in every chromosome);
 * 16 + 8 * batch * (1 + splits) bytes per region (at most n_chrom + 2n / 8192
 * regions R; splits = min(16, ceil(2048 / R)) search workgroups per region);
 * and 8 * batch * na bytes of placement records.  BITS_E_CHROM if the
 * genome is 2^32 bp or more. */
int bits_mc_binned_workspace(uint64_t na, uint64_t n, const uint32_t *chrom_len, uint32_t n_chrom,
                             uint32_t batch, size_t *bytes);

/* The Monte-Carlo loop of bits_mc_pvalue (same shuffles, same Philox
 * stream, same outputs bit for bit), ordered by region of the genome
 * rather than by query.  Each chromosome is cut into cells; a region is a
 * run of cells holding about 8192 keys of B_S and B_E together.  Per pass
 * of `batch` shuffles (fewer if batch * na would reach 2^32, so that a pass
 * indexes its records in 32 bits):
 *   1. binning: the placements of every (shuffle, chromosome) are made,
 *      counted per region, made again and written as {start, end} records
 *      in region order (8 bytes per placement into d_ws);
 *   2. search: one workgroup per region stages the region's slices of B_S
 *      and B_E in LDS and counts every placement of the pass that starts in
 *      the region by two bisections there (Algorithm 1); ends past the
 *      region continue in HBM;
 *   3. the per-region sums are added to d_totals.
 * The total of each shuffle is a sum over its placements, so this order
 * gives the same totals.  The observed total uses the reference's own
 * search (launch: its path and shape; NULL = defaults).  Needs no learned
 * index.  Arguments, outputs and flags as bits_mc_pvalue; d_ws of
 * bits_mc_binned_workspace(na, ref->n, chrom_len, n_chrom, batch) bytes.
 * BITS_E_ARG for batch outside [1, BITS_MC_BIN_MAX_BATCH]. */
int bits_mc_binned(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end, uint64_t na,
                   const uint32_t *chrom_len, uint32_t n_chrom, uint64_t seed, uint64_t s0, uint64_t s1,
                   uint32_t batch, void *d_ws, size_t ws_bytes, uint64_t *d_totals, uint64_t *d_observed,
                   uint64_t *d_n_ge, uint64_t *d_n_le, const bits_launch *launch, void *stream);

/* Stage timing of bits_mc_binned, for profiling.  With timing on
 * (enable != 0; off by default), each later bits_mc_binned call records HIP
 * events on its stream around every pass's binning, search and reduction
 * kernels (recording only: nothing inside the call waits).
 * bits_mc_binned_stage_ms waits for the last call's events and writes the
 * summed milliseconds of its binning, search and reduction kernels to
 * ms[0], ms[1], ms[2] (zeros if nothing was recorded).  Calls that overlap
 * in time share one record. */
int bits_mc_binned_timing(int enable);
int bits_mc_binned_stage_ms(float *ms);

/* Workspace bytes of bits_mc_resort for |B| = nb and `batch` rounds per
 * sort launch (1 <= batch <= 4096): 16 bytes per interval of B, 16 bytes per
 * interval per round of the batch, and the segmented sort's workspace. */
int bits_mc_resort_workspace(uint64_t nb, uint32_t batch, size_t *bytes);

/* The Monte-Carlo loop in the paper's orientation (Sec. 3.2, Table 1): every
 * round randomises the DATABASE set B within its chromosomes (rule and
 * Philox stream of bits_mc_pvalue with the roles of A and B swapped: round s
 * places interval j of B with counter g = s * nb + j), sorts B_S and B_E
 * again on the device (segmented radix sort, `batch` rounds per launch) and
 * counts the fixed query set A against it by plain bisection.  The count is
 * symmetric in A and B, so the per-round totals equal bits_mc_pvalue's with
 * a reference built from A and B as the queries, which needs no per-round
 * sort; this entry point is the literal form, for comparison.
 *   d_a_*, na       the fixed query set A (projected; no end of 2^32 - 1)
 *   d_b_*, nb       the database set B (projected, < 2^32 intervals); an interval
 *                   outside its chromosome sets BITS_FLAG_CHROM in d_status and
 *                   is left out of every round and of the observed total
 *   outputs         as bits_mc_pvalue (d_status nullable) */
int bits_mc_resort(const uint32_t *d_a_start, const uint32_t *d_a_end, uint64_t na, const uint32_t *d_b_start,
                   const uint32_t *d_b_end, uint64_t nb, const uint32_t *chrom_len, uint32_t n_chrom, uint64_t seed,
                   uint64_t s0, uint64_t s1, uint32_t batch, void *d_ws, size_t ws_bytes, uint64_t *d_totals,
                   uint64_t *d_observed, uint64_t *d_n_ge, uint64_t *d_n_le, uint32_t *d_status, void *stream);

/* (1 + n_ge) / (n_shuffles + 1) as one IEEE fp64 division (host). */
double bits_pvalue(uint64_t n_ge, uint64_t n_shuffles);

/* Lower tail (depletion): (1 + n_le) / (n_shuffles + 1) (host). */
double bits_pvalue_lower(uint64_t n_le, uint64_t n_shuffles);

/* Two-sided: min(1, 2 min(upper, lower)) of the two one-sided values (host). */
double bits_pvalue_two_sided(uint64_t n_ge, uint64_t n_le, uint64_t n_shuffles);

/* Median of the per-shuffle totals (Sec. 3.3, Fig. 3): *d_lo = the
 * floor((n-1)/2)-th and *d_hi = the floor(n/2)-th smallest of d_totals[0..n)
 * (0-based; equal when n is odd), exact, by radix selection on the device.
 * The median is (lo + hi) / 2.  1 <= n < 2^32. */
int bits_mc_median(const uint64_t *d_totals, uint64_t n, uint64_t *d_lo, uint64_t *d_hi, void *stream);

/* Enrichment score of Sec. 3.3 / Fig. 3: log2(observed / median) with
 * median = (lo + hi) / 2, in IEEE fp64 on the host (an observed count of 0
 * gives -inf; a median of 0 gives +inf, or NaN when observed is 0 too). */
double bits_enrichment(uint64_t observed, uint64_t median_lo, uint64_t median_hi);

/* ---------------------------------------------------------------------- */
/* Enumeration (Sec. 1.1, sub-problem 4)                                    */
/* ---------------------------------------------------------------------- */

/* Bytes of an enumeration index over n intervals: uint32 starts[n], ends[n],
 * ids[n], each region 256-byte aligned (n < 2^32). */
int bits_enum_index_bytes(uint64_t n, size_t *bytes);

/* Workspace bytes of bits_enum_index_build for n intervals. */
int bits_enum_index_workspace(uint64_t n, size_t *bytes);

/* Enumeration index: B sorted by start (stable radix sort, so equal starts
 * keep their input order) with each interval's input index and end moved
 * along.  d_index is a caller block of bits_enum_index_bytes(n) bytes,
 * 256-byte aligned; d_b_start / d_b_end are not modified. */
int bits_enum_index_build(const uint32_t *d_b_start, const uint32_t *d_b_end, uint64_t n, void *d_index,
                          size_t index_bytes, void *d_ws, size_t ws_bytes, void *stream);

/* Workspace bytes of bits_scan_counts for n counts. */
int bits_scan_workspace(uint64_t n, size_t *bytes);

/* d_offsets[i] = d_counts[0] + ... + d_counts[i - 1] for i <= n (uint64), so
 * d_offsets[n] is the total: the output offsets of enumeration. */
int bits_scan_counts(const uint32_t *d_counts, uint64_t n, uint64_t *d_offsets, void *d_ws, size_t ws_bytes,
                     void *stream);

/* Step 1 of enumeration in one call: per-query counts (as bits_count_per_query),
 * d_first[i] = #{B_S <= a_i.end} (the first search of ICount, where the scan
 * of bits_enumerate starts) and d_offsets = bits_scan_counts(d_counts), so
 * d_offsets[na] is the number of pairs.  d_ws: bits_scan_workspace(na) bytes. */
int bits_enum_counts(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end, uint64_t na,
                     uint32_t *d_counts, uint32_t *d_first, uint64_t *d_offsets, void *d_ws, size_t ws_bytes,
                     const bits_launch *launch, void *stream);

/* Every intersecting pair (Sec. 1.1): for each query i, the indices b of
 * the intervals of B that intersect a_i are written to d_pair_b[o .. o + c)
 * with d_pair_a[.] = i, where o = d_offsets[i] and c = d_counts[i].  Within
 * a query, pairs come in order of decreasing start of b (equal starts:
 * decreasing index).  The scan of B sorted by start runs backwards from the
 * last start <= a_i.end and stops after c hits (Sec. 2.1: the count is the
 * stop condition); nested intervals cost extra steps.
 *   d_index     bits_enum_index_build's block for B (n intervals)
 *   d_counts    bits_count_per_query's (or bits_enum_counts's) counts of the same A
 *               against the same B
 *   d_first     bits_enum_counts's d_first, or NULL (then found here by bisection)
 *   d_offsets   bits_scan_counts of d_counts
 *   max_pairs   capacity of d_pair_a / d_pair_b; nothing is written at or past it
 *   d_status    device status word (nullable): BITS_FLAG_ENUM when a scan ends
 *               short of its count or a pair did not fit, BITS_FLAG_INTERVAL for
 *               a query with start > end and a non-zero count */
int bits_enumerate(const void *d_index, uint64_t n, const uint32_t *d_a_start, const uint32_t *d_a_end,
                   uint64_t na, const uint32_t *d_counts, const uint32_t *d_first, const uint64_t *d_offsets,
                   uint32_t *d_pair_a, uint32_t *d_pair_b, uint64_t max_pairs, uint32_t *d_status, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched pairs: many query sets x many references, one persistent launch  */
/* captured in a HIP graph (the many-pairs screen of Sec. 3.3).             */
/* ---------------------------------------------------------------------- */

typedef struct bits_batch_plan bits_batch_plan;   /* opaque host object */

/* Workspace bytes for a plan over n_q query sets of sizes na[] (host). */
int bits_batch_workspace(const uint64_t *na, uint32_t n_q, uint32_t n_ref, size_t *bytes);

/* Builds a plan that computes d_pair_totals[i * n_ref + j] = total count of
 * query set i against reference j for all pairs, as one zero-fill kernel and
 * one persistent kernel captured into a HIP graph.  Work items (pair, tile)
 * are ordered by reference so a workgroup re-stages the LDS top tree only
 * when its reference changes.  Uploads the work list into d_ws (synchronous
 * on `stream`).  refs and the query pointers are host arrays; the device
 * buffers they name must stay valid while the plan is used.
 * launch (nullable): block, qpl, depth, grid and path of the persistent
 * kernel.  path BITS_PATH_LEARNED searches every pair through its
 * reference's learned index (BITS_E_ARG unless every reference is learned);
 * BITS_PATH_AUTO (and launch = NULL) picks it when every reference is
 * learned, else the plain path.  The learned path's fallbacks are counted in
 * each reference's own counter; interval errors go to refs[0]'s status. */
int bits_batch_create(const bits_ref *refs, uint32_t n_ref, const uint32_t *const *d_a_start,
                      const uint32_t *const *d_a_end, const uint64_t *na, uint32_t n_q,
                      uint64_t *d_pair_totals, void *d_ws, size_t ws_bytes,
                      const bits_launch *launch, void *stream, bits_batch_plan **plan);

/* Replays the captured graph on `stream`. */
int bits_batch_run(bits_batch_plan *plan, void *stream);

/* Frees the host plan and its graph. */
int bits_batch_destroy(bits_batch_plan *plan);

/* ---------------------------------------------------------------------- */
/* Autotuner                                                               */
/* ---------------------------------------------------------------------- */

/* Times bits_count on the given queries for every candidate launch shape
 * (block 256/512/1024, qpl 1/2/4, LDS depth 8..ref->depth, the given path)
 * with HIP events and writes the fastest to *best and its time to *best_ms.
 * `path` is BITS_PATH_PLAIN, BITS_PATH_LEARNED or BITS_PATH_TIERED.  Writes d_total. */
int bits_autotune_count(const bits_ref *ref, const uint32_t *d_a_start, const uint32_t *d_a_end,
                        uint64_t na, uint64_t *d_total, uint32_t path, bits_launch *best,
                        float *best_ms, void *stream);

/* The batch plan's autotuner: builds a plan for every candidate launch shape
 * of the persistent kernel (block 256/512/1024, qpl 1/2/4, and on the plain
 * path LDS depth 8..max depth of the references), times its graph replay with
 * HIP events (one warm-up, best of three) and writes the fastest shape to
 * *best and its time to *best_ms.  Arguments as bits_batch_create; the
 * caller may pass a sample of each query set (a prefix) to bound the tuning
 * time.  Writes d_pair_totals; waits on `stream`. */
int bits_autotune_batch(const bits_ref *refs, uint32_t n_ref, const uint32_t *const *d_a_start,
                        const uint32_t *const *d_a_end, const uint64_t *na, uint32_t n_q, uint32_t path,
                        uint64_t *d_pair_totals, void *d_ws, size_t ws_bytes, bits_launch *best,
                        float *best_ms, void *stream);

/* ---------------------------------------------------------------------- */
/* Learned-model gradient (exposes the training kernel's own device code)   */
/* ---------------------------------------------------------------------- */

/* Loss and gradient of one leaf model over m points, computed by the same
 * device code the training kernel runs (fp32):
 *   loss = mean_i (y(u_i) - t_i)^2,  y(u) = b2 + sum_j w2_j relu(w1_j u + b1_j)
 *   d_u, d_t      device float[m], m <= BITS_RMI_MAX_POINTS (2048)
 *   d_params      device float[49]  (w1[16], b1[16], w2[16], b2)
 *   d_grad        device float[49];  d_loss device float[1] */
int bits_rmi_leaf_grad(const float *d_u, const float *d_t, uint32_t m, const float *d_params,
                       float *d_grad, float *d_loss, void *stream);

/* Search window of the learned index, computed by the same device code the
 * learned searches run (route, leaf model, error window): for each key
 * d_x[i], the window [d_lo[i], d_hi[i]] of ranks in which
 * lower_bound(array, d_x[i]) is searched, or d_lo[i] = d_hi[i] = that rank
 * when the leaf resolves it directly (x <= the leaf's smallest key or > its
 * largest).  which: 0 = sorted starts, 1 = sorted ends.  For every key of
 * the array the window holds its rank; other queries are verified by the
 * search itself.  The reference must be learned and non-empty. */
int bits_rmi_window(const bits_ref *ref, uint32_t which, const uint32_t *d_x, uint64_t n, uint32_t *d_lo,
                    uint32_t *d_hi, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BITS_H */
