"""GPU parity of the decision sub-problem (Sec. 1.1) and of the Monte-Carlo
summary statistics (median of the per-shuffle totals, enrichment score of
Sec. 3.3) through the C ABI, against the oracle."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1208_3407_amd import bits, datagen  # noqa: E402

DEV = torch.device("cuda", 0)


def up(x, dtype=np.uint32):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=dtype))).to(DEV)


def down(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n", [1, 2, 3, 1000, 1001, 10_000, 65_537])
def test_median_of_totals(n):
    note("case: median n=%d" % n)
    r = np.random.default_rng(n)
    for hi in (3, 10**9, 2**63):
        t = r.integers(0, hi, n, dtype=np.uint64)
        lo_d, hi_d = bits.bits_mc_median(up(t, np.uint64))
        assert (int(down(lo_d)[0]), int(down(hi_d)[0])) == oracle.mc_median(t), hi


def test_median_and_enrichment_of_a_monte_carlo_run():
    """The summary of a real run: median of the device totals, the enrichment
    score and the tails, each against the oracle's own totals."""
    note("case: MC summary")
    lengths, A, B = datagen.w2_sets(seed=2, n_a=2000, n_b=40_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    exp = oracle.mc_totals(np.sort(b_s), np.sort(b_e), oracle.mc_prepare(lengths, a_s, a_e), 7, 0, 101, threads=8)
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": 10})
    mc = bits.bits_mc_pvalue(ref, up(a_s), up(a_e), lengths, 7, 0, 101)
    assert np.array_equal(down(mc.totals), exp)
    lo, hi = bits.bits_mc_median(mc.totals)
    lo, hi = int(down(lo)[0]), int(down(hi)[0])
    assert (lo, hi) == oracle.mc_median(exp)
    assert bits.bits_enrichment(obs, lo, hi) == oracle.enrichment(obs, lo, hi)
    ge, le = int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])
    assert bits.bits_pvalue_lower(le, 101) == (1.0 + le) / 102.0
    assert bits.bits_pvalue_two_sided(ge, le, 101) == min(1.0, 2.0 * min((1.0 + ge) / 102.0, (1.0 + le) / 102.0))


LAUNCHES = [{"path": bits.BITS_PATH_PLAIN}, {"path": bits.BITS_PATH_PLAIN, "block": 256, "qpl": 1, "grid": 3},
            {"path": bits.BITS_PATH_LEARNED}, {"path": bits.BITS_PATH_LEARNED, "block": 512, "qpl": 4}]


def check_decide(ref, a_s, a_e, b_s, b_e, lp):
    found, wit = bits.bits_decide(ref, up(a_s), up(a_e), launch=lp)
    f, w = int(down(found)[0]), int(down(wit)[0])
    ok = a_s <= a_e
    counts = oracle.counter(a_s[ok], a_e[ok], b_s, b_e)[0] if ok.any() else np.zeros(0, np.uint32)
    exp = bool(np.any(counts > 0))
    assert f == int(exp), lp
    if exp:
        idx = np.flatnonzero(ok)
        assert w < len(a_s) and ok[w] and counts[np.searchsorted(idx, w)] > 0, lp
    else:
        assert w == 2**64 - 1, lp


def test_decide():
    note("case: decide")
    r = np.random.default_rng(4)
    b_s = (r.integers(0, 10**6, 50_000) * 20).astype(np.uint32)        # starts at multiples of 20
    b_e = b_s + np.uint32(9)                                           # [20k, 20k + 9]
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": 10})
    gap_s = (r.integers(0, 10**6, 300_000) * 20 + 10).astype(np.uint32)  # [20k + 10, 20k + 19]: in the gaps
    gap_e = gap_s + np.uint32(9)
    for lp in LAUNCHES:
        note("  launch %s" % lp)
        check_decide(ref, gap_s, gap_e, b_s, b_e, lp)                  # no intersection anywhere
        hit_s, hit_e = gap_s.copy(), gap_e.copy()
        hit_s[-1], hit_e[-1] = b_e[7], b_e[7] + 5                     # only the last query touches one interval
        check_decide(ref, hit_s, hit_e, b_s, b_e, lp)
        check_decide(ref, b_s, b_e, b_s, b_e, lp)                      # everything intersects
        bad_s, bad_e = hit_s.copy(), hit_e.copy()
        bad_s[5], bad_e[5] = 100, 50                                   # start > end: skipped and flagged
        check_decide(ref, bad_s, bad_e, b_s, b_e, lp)
        assert bits.bits_get_status(ref) & bits.BITS_FLAG_INTERVAL
        bits.bits_clear_status(ref)
    # empty reference, empty query set
    empty = bits.bits_sort_ref(up(np.zeros(0)), up(np.zeros(0)))
    found, wit = bits.bits_decide(empty, up([1]), up([5]))
    assert int(down(found)[0]) == 0 and int(down(wit)[0]) == 2**64 - 1
    found, wit = bits.bits_decide(ref, up(np.zeros(0)), up(np.zeros(0)))
    assert int(down(found)[0]) == 0


@pytest.mark.parametrize("batch", [1, 7, 64])
def test_paper_orientation_resort(batch):
    """Sec. 3.2 as the paper runs it: B randomised and re-sorted every round,
    A fixed.  Per-round totals, observed and tails equal (1) the oracle with
    the shuffled set's table built from B and the sorted arrays from A, and
    (2) the fixed-reference Monte-Carlo path with A as the reference and B as
    the queries (no per-round sort); uneven batches of rounds."""
    note("case: paper orientation batch=%d" % batch)
    lengths, A, B = datagen.w2_sets(seed=6, n_a=30_000, n_b=3_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    s0, s1 = 3, 23
    exp = oracle.mc_totals(np.sort(a_s), np.sort(a_e), oracle.mc_prepare(lengths, b_s, b_e), 11, s0, s1, threads=8)
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    mc = bits.bits_mc_resort(up(a_s), up(a_e), up(b_s), up(b_e), lengths, 11, s0, s1, batch=batch)
    assert np.array_equal(down(mc.totals), exp)
    assert int(down(mc.observed)[0]) == obs
    assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == oracle.mc_tail(exp, obs)
    ref_a = bits.bits_sort_ref(up(a_s), up(a_e), learned=True, train={"epochs": 10})
    swapped = bits.bits_mc_pvalue(ref_a, up(b_s), up(b_e), lengths, 11, s0, s1)
    assert np.array_equal(down(swapped.totals), exp) and int(down(swapped.observed)[0]) == obs


def test_paper_orientation_interval_outside_chromosome():
    note("case: paper orientation, bad interval")
    lengths = np.array([1000, 2000], np.uint32)
    b_s = np.array([10, 990, 1500, 2500], np.uint32)     # interval 1 crosses the end of chromosome 0
    b_e = np.array([20, 1010, 1600, 2600], np.uint32)
    a_s = np.arange(0, 3000, 37).astype(np.uint32)
    a_e = a_s + np.uint32(30)
    st = torch.zeros(1, dtype=torch.uint32, device=DEV)
    mc = bits.bits_mc_resort(up(a_s), up(a_e), up(b_s), up(b_e), lengths, 5, 0, 9, batch=4, status=st)
    assert int(down(st)[0]) & bits.BITS_FLAG_CHROM
    keep = np.array([True, False, True, True])
    # the oracle's placements of all four intervals (counter g = 4 s + j; the bad
    # one gets a dummy table entry and is then dropped), counted against A
    off, span, ln = oracle.mc_prepare(lengths, b_s[keep], b_e[keep])
    off4 = np.array([off[0], 0, off[1], off[2]], np.uint32)
    span4 = np.array([span[0], 1, span[1], span[2]], np.uint32)
    len4 = np.array([ln[0], 1, ln[1], ln[2]], np.uint32)
    t = down(mc.totals)
    for s in range(9):
        st_ = oracle.mc_placements(5, s, off4, span4)[keep]
        en_ = st_ + len4[keep] - np.uint32(1)
        assert int(t[s]) == oracle.counter(a_s, a_e, st_, en_)[1], s
    assert int(down(mc.observed)[0]) == oracle.counter(a_s, a_e, b_s[keep], b_e[keep])[1]


def test_all_pairs_screen_small():
    """The all-pairs screen of Sec. 3.3 at a small scale (6 tracks, 36 pairs,
    15 rounds): observed counts of all pairs from one batch launch, and every
    pair's Monte-Carlo totals, median, enrichment and p-value, against the
    oracle pair by pair."""
    note("case: all-pairs screen, 6 tracks")
    from paper_1208_3407_amd import screen
    lengths, tracks = datagen.screen_sets(seed=3, n_tracks=6, size_range=(300, 6000))
    td = [bits.bits_project(lengths, up(T.chrom), up(T.start), up(T.end)) for T in tracks]
    to = [oracle.project(lengths, T.chrom, T.start, T.end) for T in tracks]
    refs = bits.bits_sort_refs(td)
    plan = bits.bits_batch_create(refs, td)
    observed = down(bits.bits_batch_run(plan)).reshape(6, 6)
    bits.bits_batch_destroy(plan)
    N = 15
    for i in range(6):
        prep = oracle.mc_prepare(lengths, to[i][0], to[i][1])
        for j in range(6):
            sbs, sbe = np.sort(to[j][0]), np.sort(to[j][1])
            obs = oracle.counter(to[i][0], to[i][1], to[j][0], to[j][1])[1]
            assert int(observed[i, j]) == obs, (i, j)
            exp_T = oracle.mc_totals(sbs, sbe, prep, screen.MC_SEED, 0, N)
            mc, lo, hi = screen.mc_pair(refs[j], td[i], lengths, N, batch=screen.pass_batch(len(tracks[i])))
            assert np.array_equal(down(mc.totals), exp_T), (i, j)
            s = screen.summarise(mc, lo, hi, N)
            olo, ohi = oracle.mc_median(exp_T)
            assert s["observed"] == obs and s["median"] == (olo + ohi) / 2
            ge, le = oracle.mc_tail(exp_T, obs)
            assert s["p_upper"] == oracle.pvalue(ge, N)
            e = oracle.enrichment(obs, olo, ohi)
            assert s["enrichment_log2"] == e or (np.isnan(e) and np.isnan(s["enrichment_log2"]))
