/*
 * CPU oracle for Binary Interval Search (BITS) -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C (fp64 where floating point appears).  It
 * shares no code, header, table or helper with the HIP library: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load it.  The
 * product path never calls into this file.
 *
 * Citations are to Layer et al., "Binary Interval Search (BITS): A Scalable
 * Algorithm for Counting Interval Intersections", Bioinformatics 2012:
 *   Sec. 1.1  interval, intersection predicate, the pair set I(A,B)
 *   Sec. 2.1  the exclusion sets L, R and the identity |I| = first - last;
 *             Algorithm 1 (ICount) and Algorithm 2 (Counter); projection of
 *             <chrom,start,end> to one dimension by a per-chromosome offset
 *   Sec. 2.2  complexity O((|A|+|B|) log |B|)
 *   Sec. 3.2  Monte-Carlo significance by randomised placement
 * and to Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as
 * 1, 2, 3", SC'11 (Philox-4x32 with 10 rounds).
 *
 * Readings where the paper is silent (coordinate base, how a random word maps
 * to a start, the p-value convention, the learned-index loss) are listed in
 * the design notes of the repository; each function below states the one it
 * uses.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Projection (Sec. 2.1, counting paragraph; Sec. 3.2 setup description).   */
/* A chromosome-local interval becomes one-dimensional by adding the summed  */
/* length of all earlier chromosomes.  Coordinates are 0-based and closed.   */
/* Returns 0, or -1 when a chromosome id is out of range, an interval leaves */
/* its chromosome, or the genome does not fit in 32 bits.                    */
/* ------------------------------------------------------------------------ */
int oracle_genome_offsets(const uint32_t *len, uint32_t n_chrom, uint64_t *off)
{
    uint64_t acc = 0;
    for (uint32_t c = 0; c < n_chrom; ++c) {
        off[c] = acc;
        acc += len[c];
    }
    off[n_chrom] = acc;
    return acc <= 0xFFFFFFFFull ? 0 : -1;
}

int oracle_project(const uint32_t *len, uint32_t n_chrom, const uint32_t *chrom,
                   const uint32_t *lstart, const uint32_t *lend, uint64_t n,
                   uint32_t *gstart, uint32_t *gend)
{
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n_chrom + 1));
    if (!off) return -1;
    if (oracle_genome_offsets(len, n_chrom, off) != 0) { free(off); return -1; }
    int rc = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t c = chrom[i];
        if (c >= n_chrom || lstart[i] > lend[i] || lend[i] >= len[c]) { rc = -1; break; }
        gstart[i] = (uint32_t)(off[c] + lstart[i]);
        gend[i] = (uint32_t)(off[c] + lend[i]);
    }
    free(off);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sort (Algorithm 2, the two Sort steps): the C library's qsort.            */
/* ------------------------------------------------------------------------ */
static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return (a > b) - (a < b);
}

void oracle_sort_u32(uint32_t *a, uint64_t n)
{
    qsort(a, (size_t)n, sizeof(uint32_t), cmp_u32);
}

/* ------------------------------------------------------------------------ */
/* The definition (Sec. 1.1): a and b intersect when a.start <= b.end and    */
/* a.end >= b.start.  Brute force over every pair, O(|A||B|).                */
/* counts may be NULL; total may be NULL.                                    */
/* ------------------------------------------------------------------------ */
void oracle_count_bruteforce(const uint32_t *as, const uint32_t *ae, uint64_t na,
                             const uint32_t *bs, const uint32_t *be, uint64_t nb,
                             uint32_t *counts, uint64_t *total)
{
    uint64_t t = 0;
    for (uint64_t i = 0; i < na; ++i) {
        uint64_t c = 0;
        for (uint64_t j = 0; j < nb; ++j)
            if (as[i] <= be[j] && ae[i] >= bs[j]) ++c;
        if (counts) counts[i] = (uint32_t)c;
        t += c;
    }
    if (total) *total = t;
}

/* Enumeration (Sec. 1.1, sub-problem 4) by the same definition: every pair  */
/* (i, j) with a_i.start <= b_j.end and a_i.end >= b_j.start, in order of i  */
/* then j.  At most max_pairs pairs are written; returns how many exist.     */
uint64_t oracle_enumerate_bruteforce(const uint32_t *as, const uint32_t *ae, uint64_t na,
                                     const uint32_t *bs, const uint32_t *be, uint64_t nb,
                                     uint32_t *pa, uint32_t *pb, uint64_t max_pairs)
{
    uint64_t k = 0;
    for (uint64_t i = 0; i < na; ++i)
        for (uint64_t j = 0; j < nb; ++j)
            if (as[i] <= be[j] && ae[i] >= bs[j]) {
                if (k < max_pairs) {
                    pa[k] = (uint32_t)i;
                    pb[k] = (uint32_t)j;
                }
                ++k;
            }
    return k;
}

/* ------------------------------------------------------------------------ */
/* BSearch (Sec. 2.1).  The equations fix what the two searches return:      */
/*   last  = |L| = number of sorted ends   strictly below a.start            */
/*   first = |B| - |R| = number of sorted starts at or below a.end           */
/* Both are textbook bisections on a sorted array.                           */
/* ------------------------------------------------------------------------ */
uint64_t oracle_count_less(const uint32_t *sorted, uint64_t n, uint32_t x)
{
    uint64_t lo = 0, hi = n;              /* invariant: answer in [lo, hi] */
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (sorted[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

uint64_t oracle_count_le(const uint32_t *sorted, uint64_t n, uint32_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (sorted[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* ICount (Algorithm 1): c = first - last.  Requires start <= end. */
static uint64_t icount(const uint32_t *sbs, const uint32_t *sbe, uint64_t nb,
                       uint32_t a_start, uint32_t a_end)
{
    uint64_t first = oracle_count_le(sbs, nb, a_end);
    uint64_t last = oracle_count_less(sbe, nb, a_start);
    return first - last;
}

/* ------------------------------------------------------------------------ */
/* Counter (Algorithm 2) over already sorted B_S, B_E, split over threads    */
/* by disjoint query ranges; partial sums are added in thread order.         */
/* Returns -1 if some query has start > end (outside the definition).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint32_t *sbs, *sbe, *as, *ae;
    uint64_t nb, lo, hi;
    uint32_t *counts;
    uint64_t total;
    int bad;
} count_job;

static void *count_worker(void *p)
{
    count_job *j = (count_job *)p;
    uint64_t t = 0;
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        if (j->as[i] > j->ae[i]) { j->bad = 1; continue; }
        uint64_t c = icount(j->sbs, j->sbe, j->nb, j->as[i], j->ae[i]);
        if (j->counts) j->counts[i] = (uint32_t)c;
        t += c;
    }
    j->total = t;
    return NULL;
}

int oracle_count_sorted(const uint32_t *sbs, const uint32_t *sbe, uint64_t nb,
                        const uint32_t *as, const uint32_t *ae, uint64_t na,
                        uint32_t *counts, uint64_t *total, int threads)
{
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > na) threads = na ? (int)na : 1;
    count_job *jobs = (count_job *)calloc((size_t)threads, sizeof(count_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return -2; }
    for (int k = 0; k < threads; ++k) {
        count_job *j = &jobs[k];
        j->sbs = sbs; j->sbe = sbe; j->as = as; j->ae = ae; j->nb = nb;
        j->lo = na * (uint64_t)k / (uint64_t)threads;
        j->hi = na * (uint64_t)(k + 1) / (uint64_t)threads;
        j->counts = counts;
        if (threads > 1) pthread_create(&tid[k], NULL, count_worker, j);
        else count_worker(j);
    }
    uint64_t t = 0;
    int bad = 0;
    for (int k = 0; k < threads; ++k) {
        if (threads > 1) pthread_join(tid[k], NULL);
        t += jobs[k].total;
        bad |= jobs[k].bad;
    }
    if (total) *total = t;
    free(jobs); free(tid);
    return bad ? -1 : 0;
}

/* Counter (Algorithm 2) from unsorted B: build B_S and B_E, sort, count. */
int oracle_counter(const uint32_t *as, const uint32_t *ae, uint64_t na,
                   const uint32_t *bs, const uint32_t *be, uint64_t nb,
                   uint32_t *counts, uint64_t *total, int threads)
{
    uint32_t *sbs = (uint32_t *)malloc(sizeof(uint32_t) * (nb ? nb : 1));
    uint32_t *sbe = (uint32_t *)malloc(sizeof(uint32_t) * (nb ? nb : 1));
    if (!sbs || !sbe) { free(sbs); free(sbe); return -2; }
    memcpy(sbs, bs, sizeof(uint32_t) * nb);
    memcpy(sbe, be, sizeof(uint32_t) * nb);
    oracle_sort_u32(sbs, nb);
    oracle_sort_u32(sbe, nb);
    int rc = oracle_count_sorted(sbs, sbe, nb, as, ae, na, counts, total, threads);
    free(sbs); free(sbe);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Independent cross-check for totals: a linear merge ("sweep") of sorted    */
/* query endpoints against sorted database endpoints.  By the exclusion      */
/* identity, total = sum_a #{b.start <= a.end} - sum_a #{b.end < a.start}.   */
/* No bisection is used.  All four arrays must be sorted ascending.          */
/* ------------------------------------------------------------------------ */
uint64_t oracle_sweep_total(const uint32_t *sorted_a_start, const uint32_t *sorted_a_end, uint64_t na,
                            const uint32_t *sorted_b_start, const uint32_t *sorted_b_end, uint64_t nb)
{
    uint64_t starts_le = 0, ends_lt = 0, j = 0;
    for (uint64_t i = 0; i < na; ++i) {          /* a.end ascending */
        while (j < nb && sorted_b_start[j] <= sorted_a_end[i]) ++j;
        starts_le += j;
    }
    j = 0;
    for (uint64_t i = 0; i < na; ++i) {          /* a.start ascending */
        while (j < nb && sorted_b_end[j] < sorted_a_start[i]) ++j;
        ends_lt += j;
    }
    return starts_le - ends_lt;
}

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (Salmon et al., SC'11, Sec. 4): a 4-word counter and a     */
/* 2-word key.  Each of ten rounds multiplies words 0 and 2 by the two round */
/* multipliers, exchanges the word pairs and xors the high halves with the   */
/* other two words and the round key; the key advances by the two Weyl       */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint64_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = M0 * (uint64_t)x0;
        uint64_t p1 = M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Monte-Carlo randomisation (Sec. 3.2).  The paper only says each round     */
/* draws "random starts"; the reading used here:                             */
/*  - the query set A is re-placed, each interval inside its own chromosome, */
/*    length kept, uniformly over the len_c - L + 1 legal starts;            */
/*  - draw (s, i) uses Philox-4x32-10 with key = (lo32 seed, hi32 seed) and  */
/*    counter = (lo32 g, hi32 g, 0, 0), g = s * |A| + i;                     */
/*  - the 64-bit word u = out1:out0 maps to floor(u * span / 2^64).          */
/* The chromosome of a is the one whose projected range holds a.start.       */
/* ------------------------------------------------------------------------ */
static int chrom_of(const uint64_t *off, uint32_t n_chrom, uint32_t x)
{
    /* last c with off[c] <= x; linear scan, the genomes here are small */
    int c = -1;
    for (uint32_t k = 0; k < n_chrom; ++k)
        if (off[k] <= x) c = (int)k;
    return c;
}

int oracle_mc_prepare(const uint32_t *chrom_len, uint32_t n_chrom,
                      const uint32_t *as, const uint32_t *ae, uint64_t na,
                      uint32_t *off_out, uint32_t *span_out, uint32_t *len_out)
{
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n_chrom + 1));
    if (!off) return -2;
    if (oracle_genome_offsets(chrom_len, n_chrom, off) != 0) { free(off); return -1; }
    int rc = 0;
    for (uint64_t i = 0; i < na; ++i) {
        int c = chrom_of(off, n_chrom, as[i]);
        if (c < 0 || as[i] > ae[i] || (uint64_t)ae[i] >= off[c + 1]) { rc = -1; break; }
        uint64_t L = (uint64_t)ae[i] - as[i] + 1;
        off_out[i] = (uint32_t)off[c];
        len_out[i] = (uint32_t)L;
        span_out[i] = (uint32_t)(chrom_len[c] - L + 1);
    }
    free(off);
    return rc;
}

/* Start of shuffled interval i in shuffle s (global coordinate). */
static uint32_t mc_place(uint64_t seed, uint64_t s, uint64_t na, uint64_t i,
                         uint32_t off, uint32_t span)
{
    uint64_t g = s * na + i;
    uint32_t ctr[4] = {(uint32_t)g, (uint32_t)(g >> 32), 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    uint64_t u = ((uint64_t)r[1] << 32) | r[0];
    uint64_t local = (uint64_t)(((unsigned __int128)u * span) >> 64);
    return (uint32_t)(off + local);
}

void oracle_mc_placements(uint64_t seed, uint64_t s, uint64_t na,
                          const uint32_t *off, const uint32_t *span, uint32_t *start_out)
{
    for (uint64_t i = 0; i < na; ++i) start_out[i] = mc_place(seed, s, na, i, off[i], span[i]);
}

typedef struct {
    const uint32_t *sbs, *sbe, *off, *span, *len;
    uint64_t nb, na, seed, s_lo, s_hi, s0;
    uint64_t *totals;
} mc_job;

static void *mc_worker(void *p)
{
    mc_job *j = (mc_job *)p;
    for (uint64_t s = j->s_lo; s < j->s_hi; ++s) {
        uint64_t t = 0;
        for (uint64_t i = 0; i < j->na; ++i) {
            uint32_t st = mc_place(j->seed, s, j->na, i, j->off[i], j->span[i]);
            uint32_t en = st + j->len[i] - 1;
            t += icount(j->sbs, j->sbe, j->nb, st, en);
        }
        j->totals[s - j->s0] = t;
    }
    return NULL;
}

/* Per-shuffle totals for shuffles [s0, s1) against sorted B_S, B_E. */
int oracle_mc_totals(const uint32_t *sbs, const uint32_t *sbe, uint64_t nb,
                     const uint32_t *off, const uint32_t *span, const uint32_t *len, uint64_t na,
                     uint64_t seed, uint64_t s0, uint64_t s1, uint64_t *totals, int threads)
{
    if (s1 < s0) return -1;
    uint64_t ns = s1 - s0;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > ns) threads = ns ? (int)ns : 1;
    mc_job *jobs = (mc_job *)calloc((size_t)threads, sizeof(mc_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); return -2; }
    for (int k = 0; k < threads; ++k) {
        mc_job *j = &jobs[k];
        j->sbs = sbs; j->sbe = sbe; j->off = off; j->span = span; j->len = len;
        j->nb = nb; j->na = na; j->seed = seed; j->s0 = s0; j->totals = totals;
        j->s_lo = s0 + ns * (uint64_t)k / (uint64_t)threads;
        j->s_hi = s0 + ns * (uint64_t)(k + 1) / (uint64_t)threads;
        if (threads > 1) pthread_create(&tid[k], NULL, mc_worker, j);
        else mc_worker(j);
    }
    if (threads > 1)
        for (int k = 0; k < threads; ++k) pthread_join(tid[k], NULL);
    free(jobs); free(tid);
    return 0;
}

/* Tail counts: n_ge = #{T_s >= T_obs}, n_le = #{T_s <= T_obs}.  The paper  */
/* gives no p-value formula (Sec. 3.3 reports only log2(observed/median));   */
/* the reading used is p = (1 + n_ge) / (N + 1), computed by the caller.     */
void oracle_mc_tail(const uint64_t *totals, uint64_t n, uint64_t observed,
                    uint64_t *n_ge, uint64_t *n_le)
{
    uint64_t ge = 0, le = 0;
    for (uint64_t s = 0; s < n; ++s) {
        if (totals[s] >= observed) ++ge;
        if (totals[s] <= observed) ++le;
    }
    *n_ge = ge;
    *n_le = le;
}

/* Median of the per-shuffle totals, as used by the enrichment score of      */
/* Sec. 3.3 / Fig. 3: sort a copy, take the floor((n-1)/2)-th and the        */
/* floor(n/2)-th values (0-based); the median is their mean.  n >= 1.        */
static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

void oracle_mc_median(const uint64_t *totals, uint64_t n, uint64_t *lo, uint64_t *hi)
{
    uint64_t *c = (uint64_t *)malloc(n * sizeof(uint64_t));
    memcpy(c, totals, n * sizeof(uint64_t));
    qsort(c, n, sizeof(uint64_t), cmp_u64);
    *lo = c[(n - 1) / 2];
    *hi = c[n / 2];
    free(c);
}

/* Exact expectation of one shuffle's total under the uniform placement     */
/* above: a of length L on chromosome c intersects b (same chromosome) for   */
/* starts in [b.start - L + 1, b.end], of which those in [0, len_c - L] are  */
/* legal; E[T] = sum_a sum_b |legal hits| / span.  O(|A||B|), in fp64.       */
double oracle_mc_expected_total(const uint32_t *chrom_len, uint32_t n_chrom,
                                const uint32_t *as, const uint32_t *ae, uint64_t na,
                                const uint32_t *bs, const uint32_t *be, uint64_t nb)
{
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (n_chrom + 1));
    if (!off) return -1.0;
    oracle_genome_offsets(chrom_len, n_chrom, off);
    double e = 0.0;
    for (uint64_t i = 0; i < na; ++i) {
        int c = chrom_of(off, n_chrom, as[i]);
        int64_t L = (int64_t)ae[i] - as[i] + 1;
        int64_t maxs = (int64_t)chrom_len[c] - L;          /* last legal local start */
        double hits = 0.0;
        for (uint64_t j = 0; j < nb; ++j) {
            if (chrom_of(off, n_chrom, bs[j]) != c) continue;
            int64_t lb = (int64_t)bs[j] - (int64_t)off[c] - L + 1;
            int64_t ub = (int64_t)be[j] - (int64_t)off[c];
            if (lb < 0) lb = 0;
            if (ub > maxs) ub = maxs;
            if (ub >= lb) hits += (double)(ub - lb + 1);
        }
        e += hits / (double)(maxs + 1);
    }
    free(off);
    return e;
}

/* ------------------------------------------------------------------------ */
/* Learned CDF leaf model (not in the paper; an extension of the index).     */
/* One hidden layer of 16 ReLU units: y(u) = b2 + sum_j w2_j relu(w1_j u +   */
/* b1_j); loss = mean over m points of (y(u_i) - t_i)^2.  Parameters are the */
/* 49 floats [w1[16], b1[16], w2[16], b2].  Loss and gradient in fp64.       */
/* ------------------------------------------------------------------------ */
void oracle_rmi_forward(const float *p, const float *u, uint32_t m, double *y)
{
    for (uint32_t i = 0; i < m; ++i) {
        double acc = (double)p[48];
        for (int j = 0; j < 16; ++j) {
            double h = (double)p[j] * (double)u[i] + (double)p[16 + j];
            if (h > 0.0) acc += (double)p[32 + j] * h;
        }
        y[i] = acc;
    }
}

void oracle_rmi_loss_grad(const float *p, const float *u, const float *t, uint32_t m,
                          double *loss, double *grad)
{
    double L = 0.0;
    for (int k = 0; k < 49; ++k) grad[k] = 0.0;
    for (uint32_t i = 0; i < m; ++i) {
        double pre[16], y = (double)p[48];
        for (int j = 0; j < 16; ++j) {
            pre[j] = (double)p[j] * (double)u[i] + (double)p[16 + j];
            if (pre[j] > 0.0) y += (double)p[32 + j] * pre[j];
        }
        double r = y - (double)t[i];
        L += r * r;
        double dy = 2.0 * r / (double)m;
        grad[48] += dy;
        for (int j = 0; j < 16; ++j) {
            if (pre[j] > 0.0) {
                grad[32 + j] += dy * pre[j];
                double dh = dy * (double)p[32 + j];
                grad[j] += dh * (double)u[i];
                grad[16 + j] += dh;
            }
        }
    }
    *loss = m ? L / (double)m : 0.0;
}

/* Least-squares line rank ~ a*key + b over a sorted array, in fp64, using */
/* centred sums (two passes) so large coordinates do not cancel.            */
void oracle_linear_fit(const uint32_t *sorted, uint64_t n, double *a, double *b)
{
    if (n == 0) { *a = 0.0; *b = 0.0; return; }
    double mx = 0.0, my = 0.0;
    for (uint64_t i = 0; i < n; ++i) { mx += (double)sorted[i]; my += (double)i; }
    mx /= (double)n; my /= (double)n;
    double sxx = 0.0, sxy = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        double dx = (double)sorted[i] - mx;
        sxx += dx * dx;
        sxy += dx * ((double)i - my);
    }
    *a = sxx > 0.0 ? sxy / sxx : 0.0;
    *b = my - *a * mx;
}
