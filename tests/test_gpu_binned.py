"""GPU parity of the region-binned Monte-Carlo path (Sec. 3.2) through the C
ABI: per-shuffle totals, observed total and tails against the oracle and,
bit for bit, against the query-ordered path (bits_mc_pvalue), over uneven
batches of shuffles, region layouts that exercise the LDS slices, the
margin past a region's end, ends that continue in HBM, oversize regions
(duplicated keys) searched in HBM, empty chromosomes, and bad queries."""
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


def up(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint32))).to(DEV)


def down(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check(lengths, a_s, a_e, b_s, b_e, seed, s0, s1, batch, learned=False, against_pvalue=True):
    """bits_mc_binned against the oracle (and against bits_mc_pvalue on the same reference)."""
    exp = oracle.mc_totals(np.sort(b_s), np.sort(b_e), oracle.mc_prepare(lengths, a_s, a_e), seed, s0, s1,
                           threads=8)
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=learned, train={"epochs": 10})
    mc = bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, seed, s0, s1, batch=batch)
    got = down(mc.totals)
    assert np.array_equal(got, exp), np.flatnonzero(got != exp)[:10]
    assert int(down(mc.observed)[0]) == obs
    assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == oracle.mc_tail(exp, obs)
    assert bits.bits_get_status(ref) == 0
    if against_pvalue:
        pv = bits.bits_mc_pvalue(ref, up(a_s), up(a_e), lengths, seed, s0, s1)
        assert np.array_equal(down(pv.totals), got)
    return got


@pytest.mark.parametrize("batch", [1, 3, 64, 1024])
def test_binned_matches_oracle_w2(batch):
    """Multi-chromosome genome, clustered B (the Monte-Carlo recipe), uneven batches, s0 > 0."""
    note("case: binned w2 batch=%d" % batch)
    lengths, A, B = datagen.w2_sets(seed=2, n_a=3000, n_b=60_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    check(lengths, a_s, a_e, b_s, b_e, 7, 5, 22, batch, learned=batch == 64)


def test_binned_many_regions_and_long_queries():
    """One chromosome, dense B (many regions of ~8192 keys), queries up to 100 kbp
    long so that ends cross the staged margin and continue in HBM."""
    note("case: binned dense, long queries")
    r = np.random.default_rng(11)
    L = np.array([4_000_000], np.uint32)
    nb = 400_000
    b_s = r.integers(0, 3_990_000, nb).astype(np.uint32)
    b_e = b_s + r.integers(0, 2000, nb).astype(np.uint32)
    na = 2000
    a_s = r.integers(0, 3_800_000, na).astype(np.uint32)
    a_e = a_s + r.integers(0, 100_000, na).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 3, 0, 9, 4)


def test_binned_staged_chunks_and_direct_chromosomes():
    """A chromosome with about 500 regions (its second binning sweep goes through LDS
    in several chunks) beside one with few regions (records written one by one), in
    the same call; queries up to 50 kbp."""
    note("case: binned staged chunks + direct")
    r = np.random.default_rng(21)
    L = np.array([50_000_000, 2_000_000], np.uint32)
    nb = 2_000_000
    centres = r.integers(0, 49_000_000, 300)
    b_s = np.concatenate([r.integers(0, 49_990_000, nb // 2),
                          np.clip(centres[r.integers(0, 300, nb // 2)] + r.normal(0, 40_000, nb // 2), 0,
                                  49_990_000).astype(np.int64),
                          50_000_000 + r.integers(0, 1_990_000, 5000)]).astype(np.uint32)
    b_e = b_s + r.integers(0, 3000, len(b_s)).astype(np.uint32)
    na = 20_000
    a_s = np.concatenate([r.integers(0, 49_940_000, na), 50_000_000 + r.integers(0, 1_940_000, 2000)]).astype(np.uint32)
    a_e = a_s + r.integers(0, 50_000, len(a_s)).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 5, 3, 9, 4)


def test_binned_more_regions_than_staging_holds():
    """A chromosome with more regions than the staged binning's tables hold (about
    2200): its records are written one by one through the same kernel."""
    note("case: binned > 2048 regions on one chromosome")
    r = np.random.default_rng(22)
    L = np.array([200_000_000], np.uint32)
    nb = 9_000_000
    b_s = r.integers(0, 199_990_000, nb).astype(np.uint32)
    b_e = b_s + r.integers(0, 2000, nb).astype(np.uint32)
    na = 3000
    a_s = r.integers(0, 199_900_000, na).astype(np.uint32)
    a_e = a_s + r.integers(0, 20_000, na).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 8, 0, 4, 4, against_pvalue=False)


def test_binned_bucket_edges():
    """Keys in tight clusters separated by wide gaps (most buckets of a region empty, a few
    holding runs of equal keys) and queries whose starts and ends sit on keys, one before
    and one after them: the bucket tables' edges and the empty-bucket reads."""
    note("case: binned bucket edges")
    r = np.random.default_rng(31)
    L = np.array([30_000_000, 7_000_000], np.uint32)
    centres = np.sort(r.integers(0, 36_900_000, 400))
    b_s = np.concatenate([np.repeat(centres, r.integers(1, 40, len(centres))),
                          r.integers(0, 36_990_000, 5000)]).astype(np.int64)
    b_s = np.clip(b_s + r.integers(-3, 4, len(b_s)), 0, 36_990_000).astype(np.uint32)
    b_e = b_s + r.integers(0, 6, len(b_s)).astype(np.uint32)
    pick = r.integers(0, len(b_s), 4000)
    a_s = (b_s[pick].astype(np.int64) + r.integers(-1, 2, len(pick))).clip(0, 36_999_000).astype(np.uint32)
    a_e = (b_e[pick].astype(np.int64) + r.integers(-1, 2, len(pick)))
    a_e = np.maximum(a_e, a_s).astype(np.uint32)
    # keep every query inside its chromosome
    off = np.array([0, 30_000_000, 37_000_000], np.int64)
    c = np.searchsorted(off, a_s, side="right") - 1
    a_e = np.minimum(a_e.astype(np.int64), off[c + 1] - 1).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 13, 0, 24, 8)


@pytest.mark.parametrize("n_b", [100_000, 800_000])
@pytest.mark.parametrize("na", [5631, 5632, 5633, 11264, 11265])
def test_binned_group_sizes_around_one_chunk(n_b, na):
    """One 40 Mbp chromosome, so that each (shuffle, chromosome) group holds all na
    queries: groups of up to 5632 queries are placed once and written as one LDS chunk;
    one more query sends the group through the counting sweep and then two chunks (about
    200 regions, staged) or the one-by-one writes (about 25 regions)."""
    note("case: binned group of %d queries, n_b=%d" % (na, n_b))
    r = np.random.default_rng(na + n_b)
    L = np.array([40_000_000], np.uint32)
    b_s = r.integers(0, 39_990_000, n_b).astype(np.uint32)
    b_e = b_s + r.integers(0, 3000, n_b).astype(np.uint32)
    a_s = r.integers(0, 39_900_000, na).astype(np.uint32)
    a_e = a_s + r.integers(0, 20_000, na).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 17, 1, 8, 3)


def test_binned_oversize_region_and_empty_chromosomes():
    """Empty chromosomes between non-empty ones, 12,000 intervals of B on one
    coordinate (a region too large for LDS, searched in HBM), B keys past the
    genome's end, and a 1-bp chromosome."""
    note("case: binned oversize, empty chromosomes")
    r = np.random.default_rng(12)
    L = np.array([0, 500_000, 0, 0, 300_000, 1], np.uint32)
    b_s = np.concatenate([np.full(12_000, 1234, np.uint32), r.integers(0, 800_001, 20_000).astype(np.uint32),
                          np.full(10, 900_000, np.uint32)])
    b_e = b_s + r.integers(0, 50, len(b_s)).astype(np.uint32)
    a_s = np.concatenate([r.integers(0, 499_000, 300), r.integers(500_000, 799_000, 300), [800_000]]).astype(np.uint32)
    cap = np.where(a_s < 500_000, 499_999, np.where(a_s < 800_000, 799_999, 800_000))
    a_e = np.minimum(a_s + r.integers(0, 1000, len(a_s)), cap).astype(np.uint32)
    check(L, a_s, a_e, b_s, b_e, 9, 2, 12, 5)


def test_binned_w0_single_chromosome():
    """The small single-chromosome workload (10 Mbp, 1e4 x 1e4)."""
    note("case: binned w0")
    lengths, A, B = datagen.w0_sets(seed=1)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    check(lengths, a_s, a_e, b_s, b_e, 7, 0, 33, 16)


def test_binned_edges():
    """Empty shuffle range, empty query set, empty reference, a query outside its
    chromosome (flagged, left out), batch outside [1, 1024]."""
    note("case: binned edges")
    lengths, A, B = datagen.w2_sets(seed=3, n_a=500, n_b=5000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    ref = bits.bits_sort_ref(up(b_s), up(b_e))
    mc = bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, 7, 4, 4)
    assert len(mc.totals) == 0 and int(down(mc.observed)[0]) == oracle.counter(a_s, a_e, b_s, b_e)[1]
    assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == (0, 0)
    mc = bits.bits_mc_binned(ref, up(np.zeros(0)), up(np.zeros(0)), lengths, 7, 0, 5)
    assert down(mc.totals).tolist() == [0] * 5 and int(down(mc.observed)[0]) == 0
    empty = bits.bits_sort_ref(up(np.zeros(0)), up(np.zeros(0)))
    mc = bits.bits_mc_binned(empty, up(a_s), up(a_e), lengths, 7, 0, 5)
    assert down(mc.totals).tolist() == [0] * 5
    # the last query crosses the end of its chromosome: flagged and left out
    bad_s, bad_e = a_s.copy(), a_e.copy()
    off = np.concatenate([[0], np.cumsum(lengths.astype(np.uint64))])
    c = int(np.searchsorted(off, bad_s[-1], side="right") - 1)
    bad_e[-1] = np.uint32(off[c + 1] + 5)
    mc = bits.bits_mc_binned(ref, up(bad_s), up(bad_e), lengths, 7, 0, 6, batch=4)
    assert bits.bits_get_status(ref) & bits.BITS_FLAG_CHROM
    bits.bits_clear_status(ref)
    # the other queries keep their own counters g = s * na + i: the same totals as the
    # query-ordered path, which leaves the bad query out the same way
    pv = bits.bits_mc_pvalue(ref, up(bad_s), up(bad_e), lengths, 7, 0, 6)
    assert np.array_equal(down(mc.totals), down(pv.totals))
    assert int(down(mc.observed)[0]) == int(down(pv.observed)[0])
    bits.bits_clear_status(ref)
    for b in (0, 1025):
        with pytest.raises(bits.BitsError):
            bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, 7, 0, 5, batch=b)


def test_binned_at_monte_carlo_scale():
    """1e5 queries x 40 shuffles against 2e6 clustered intervals on the 24-chromosome
    genome: equal to the learned query-ordered path bit for bit, and to the oracle."""
    note("case: binned scale")
    lengths, A, B = datagen.w2_sets(seed=4, n_a=100_000, n_b=2_000_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    check(lengths, a_s, a_e, b_s, b_e, 7, 0, 40, 16, learned=True)


def test_binned_stage_timer():
    """The stage timer records one set of events per pass while on (positive times, the
    binning and search kernels of every pass summed) and nothing while off; the totals
    are the same either way."""
    note("case: binned stage timer")
    lengths, A, B = datagen.w2_sets(seed=5, n_a=2000, n_b=50_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    ref = bits.bits_sort_ref(up(b_s), up(b_e))
    plain = bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, 7, 0, 10, batch=4)
    bits.bits_mc_binned_timing(True)
    try:
        timed = bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, 7, 0, 10, batch=4)   # three passes
        st = bits.bits_mc_binned_stage_ms()
    finally:
        bits.bits_mc_binned_timing(False)
    assert st["place"] > 0.0 and st["search"] > 0.0 and st["reduce"] > 0.0
    assert np.array_equal(down(timed.totals), down(plain.totals))
    bits.bits_mc_binned(ref, up(a_s), up(a_e), lengths, 7, 0, 10, batch=4)
    assert bits.bits_mc_binned_stage_ms() == {"place": 0.0, "search": 0.0, "reduce": 0.0}
