"""Pins for the CPU oracle: each check ties it to something other than itself
(brute force from the definition, numpy library routines, an independent
merge, closed forms, invariants, an external Philox implementation, exact
expectations).  CPU only."""
import os
import shutil
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from paper_1208_3407_amd import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _np_count(a_s, a_e, b_s, b_e):
    """Library-routine count: numpy sort + searchsorted (right minus left)."""
    sbs, sbe = np.sort(b_s), np.sort(b_e)
    first = np.searchsorted(sbs, a_e, side="right")
    last = np.searchsorted(sbe, a_s, side="left")
    return (first - last).astype(np.int64)


def _read_golden(name):
    A, B, exp = [], [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "B":
                B.append((int(line[1]), int(line[2])))
            else:
                A.append((int(line[1]), int(line[2])))
                exp.append(int(line[3]))
    a = np.array(A, dtype=np.uint32).reshape(-1, 2)
    b = np.array(B, dtype=np.uint32).reshape(-1, 2)
    return a[:, 0], a[:, 1], b[:, 0], b[:, 1], np.array(exp)


def _rand_set(rng, n, hi=200, maxlen=40):
    s = rng.integers(0, hi, size=n)
    e = s + rng.integers(0, maxlen, size=n)
    return s.astype(np.uint32), e.astype(np.uint32)


# ---------------------------------------------------------------- counting

@settings(max_examples=200, deadline=None)
@given(st.integers(0, 2**31 - 1), st.integers(0, 64), st.integers(0, 64))
def test_bounds_count_equals_bruteforce(seed, na, nb):
    rng = np.random.default_rng(seed)
    a_s, a_e = _rand_set(rng, na)
    b_s, b_e = _rand_set(rng, nb)
    bc, bt = oracle.count_bruteforce(a_s, a_e, b_s, b_e)
    cc, ct = oracle.counter(a_s, a_e, b_s, b_e)
    assert np.array_equal(bc, cc) and bt == ct


@pytest.mark.parametrize("name", ["contained.txt", "touching.txt"])
def test_golden_fixtures(name):
    a_s, a_e, b_s, b_e, exp = _read_golden(name)
    c, t = oracle.counter(a_s, a_e, b_s, b_e)
    assert list(c) == list(exp) and t == int(exp.sum())
    bc, _ = oracle.count_bruteforce(a_s, a_e, b_s, b_e)
    assert list(bc) == list(exp)


def test_contained_defeats_single_search():
    """The fixture is one where a single search of B sorted by start for a.end
    (the rejected method of Sec. 2) finds a non-intersecting interval, while
    the true count is non-zero."""
    a_s, a_e, b_s, b_e, exp = _read_golden("contained.txt")
    order = np.argsort(b_s, kind="stable")
    j = np.searchsorted(b_s[order], a_e[0], side="right") - 1
    hit = b_s[order][j] <= a_e[0] and b_e[order][j] >= a_s[0]
    assert not hit and exp[0] == 1


def test_search_primitives_vs_numpy():
    rng = np.random.default_rng(3)
    arr = np.sort(rng.integers(0, 50, size=300).astype(np.uint32))
    for x in list(range(0, 52)) + [2**32 - 1]:
        assert oracle.count_less(arr, x) == int(np.searchsorted(arr, x, side="left"))
        assert oracle.count_le(arr, x) == int(np.searchsorted(arr, x, side="right"))
    assert oracle.count_less(np.zeros(0, np.uint32), 5) == 0


def test_counter_vs_numpy_library_w0():
    lengths, A, B = datagen.w0_sets()
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    c, t = oracle.counter(a_s, a_e, b_s, b_e, threads=4)
    ref = _np_count(a_s, a_e, b_s, b_e)
    assert np.array_equal(c.astype(np.int64), ref) and t == int(ref.sum())
    # brute force on the first 500 of each (definition of Sec. 1.1)
    bc, bt = oracle.count_bruteforce(a_s[:500], a_e[:500], b_s[:500], b_e[:500])
    cc, ct = oracle.counter(a_s[:500], a_e[:500], b_s[:500], b_e[:500])
    assert np.array_equal(bc, cc) and bt == ct
    # first 500 of A against all of B
    bc, _ = oracle.count_bruteforce(a_s[:500], a_e[:500], b_s, b_e)
    assert np.array_equal(bc, c[:500])


def test_counter_vs_numpy_and_sweep_genome_scale():
    lengths, A, B = datagen.w1_sets(n_a=200_000, n_b=300_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    c, t = oracle.counter(a_s, a_e, b_s, b_e, threads=4)
    ref = _np_count(a_s, a_e, b_s, b_e)
    assert np.array_equal(c.astype(np.int64), ref)
    assert oracle.sweep_total(a_s, a_e, b_s, b_e) == t
    assert t > 0


def test_threads_do_not_change_results():
    lengths, A, B = datagen.w1_sets(n_a=20_001, n_b=30_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    c1, t1 = oracle.counter(a_s, a_e, b_s, b_e, threads=1)
    c7, t7 = oracle.counter(a_s, a_e, b_s, b_e, threads=7)
    assert np.array_equal(c1, c7) and t1 == t7


def test_rejects_inverted_interval():
    with pytest.raises(ValueError):
        oracle.counter(np.array([5], np.uint32), np.array([4], np.uint32),
                       np.array([1], np.uint32), np.array([9], np.uint32))


def test_empty_inputs():
    z = np.zeros(0, np.uint32)
    c, t = oracle.counter(z, z, np.array([1], np.uint32), np.array([2], np.uint32))
    assert len(c) == 0 and t == 0
    c, t = oracle.counter(np.array([1], np.uint32), np.array([2], np.uint32), z, z)
    assert list(c) == [0] and t == 0


# ---------------------------------------------------------------- invariants

@settings(max_examples=60, deadline=None)
@given(st.integers(0, 2**31 - 1))
def test_invariants(seed):
    rng = np.random.default_rng(seed)
    a_s, a_e = _rand_set(rng, int(rng.integers(1, 80)), hi=1000, maxlen=80)
    b_s, b_e = _rand_set(rng, int(rng.integers(1, 80)), hi=1000, maxlen=80)
    c, t = oracle.counter(a_s, a_e, b_s, b_e)
    # I1 symmetry of totals
    assert oracle.counter(b_s, b_e, a_s, a_e)[1] == t
    # I2 per-query counts add up to the total
    assert int(c.astype(np.int64).sum()) == t
    # I3 self count: every interval meets itself, other pairs count twice
    _, tAA = oracle.counter(a_s, a_e, a_s, a_e)
    assert tAA >= len(a_s) and (tAA - len(a_s)) % 2 == 0
    # I5 shift invariance
    k = np.uint32(12345)
    assert np.array_equal(oracle.counter(a_s + k, a_e + k, b_s + k, b_e + k)[0], c)
    # I6 reflection x -> G-1-x (start and end swap roles)
    G = np.uint32(5000)
    rc, _ = oracle.counter(G - a_e, G - a_s, G - b_e, G - b_s)
    assert np.array_equal(rc, c)
    # I7 additivity over a split of B
    h = len(b_s) // 2
    c1, _ = oracle.counter(a_s, a_e, b_s[:h], b_e[:h])
    c2, _ = oracle.counter(a_s, a_e, b_s[h:], b_e[h:])
    assert np.array_equal(c1.astype(np.int64) + c2, c.astype(np.int64))
    # I8 bounds
    assert c.max() <= len(b_s)
    # I9 growing a query never loses intersections
    gc, _ = oracle.counter(a_s, a_e + np.uint32(7), b_s, b_e)
    assert np.all(gc >= c)


def test_disjoint_chromosomes_give_zero():
    lengths = datagen.genome_g24()
    r = datagen.rng_for(5, 0)
    A = datagen.uniform_set(r, lengths, datagen.lognormal_lengths(r, 3000, 200.0))
    B = datagen.uniform_set(r, lengths, datagen.lognormal_lengths(r, 3000, 200.0))
    A.chrom[:] = A.chrom % 12          # A on chromosomes 0..11
    B.chrom[:] = 12 + B.chrom % 12     # B on chromosomes 12..23
    A.end[:] = np.minimum(A.end, 40_000_000); A.start[:] = np.minimum(A.start, A.end)
    B.end[:] = np.minimum(B.end, 40_000_000); B.start[:] = np.minimum(B.start, B.end)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    assert oracle.counter(a_s, a_e, b_s, b_e)[1] == 0


# ---------------------------------------------------------------- closed forms

def test_closed_form_copies_and_spanning():
    b_s = np.full(17, 100, np.uint32)
    b_e = np.full(17, 200, np.uint32)
    c, _ = oracle.counter(np.array([150, 0, 201], np.uint32), np.array([150, 99, 300], np.uint32), b_s, b_e)
    assert list(c) == [17, 0, 0]
    lengths, A, B = datagen.w0_sets(n_a=10, n_b=777)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    c, _ = oracle.counter(np.array([0], np.uint32), np.array([9_999_999], np.uint32), b_s, b_e)
    assert list(c) == [777]


def test_closed_form_grid():
    M, w = 500, 7
    b_s = np.arange(M, dtype=np.uint32)
    b_e = b_s + np.uint32(w - 1)
    q = np.arange(0, M + w + 3, dtype=np.uint32)
    c, _ = oracle.counter(q, q, b_s, b_e)
    j_lo = np.maximum(q.astype(np.int64) - w + 1, 0)
    j_hi = np.minimum(q.astype(np.int64), M - 1)
    expect = np.maximum(j_hi - j_lo + 1, 0)
    assert np.array_equal(c.astype(np.int64), expect)


# ---------------------------------------------------------------- projection and data

def test_genome_g24_and_projection():
    lengths = datagen.genome_g24()
    assert int(lengths[0]) == 249_200_000 and int(lengths[23]) == 46_952_190
    off = oracle.genome_offsets(lengths)
    assert int(off[-1]) == 2_936_206_604
    assert np.array_equal(off[1:], np.cumsum(lengths.astype(np.uint64)))
    chrom = np.array([0, 1, 23, 23], np.uint32)
    ls = np.array([0, 5, 0, lengths[23] - 1], np.uint32)
    gs, ge = oracle.project(lengths, chrom, ls, ls)
    assert list(gs) == [0, 249_200_005, int(off[23]), 2_936_206_603]
    with pytest.raises(ValueError):
        oracle.project(lengths, np.array([0], np.uint32), np.array([0], np.uint32),
                       np.array([lengths[0]], np.uint32))


def test_sort_matches_numpy():
    r = np.random.default_rng(0)
    x = r.integers(0, 2**32, size=100_003, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(oracle.sort_u32(x), np.sort(x))


# ---------------------------------------------------------------- Philox

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Eng : rocrand_device::philox4x32_10_engine {
  uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  Eng e; unsigned a[6];
  while (std::scanf("%u %u %u %u %u %u", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
    uint4 r = e.rounds(uint4{a[0], a[1], a[2], a[3]}, uint2{a[4], a[5]});
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""


@pytest.fixture(scope="module")
def rocrand_rounds(tmp_path_factory):
    """External known-answer source: the installed rocRAND header's own
    Philox-4x32-10 rounds, compiled for the host.  Returns a function mapping
    a list of (ctr0, ctr1, ctr2, ctr3, key0, key1) to the four output words."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "probe.cpp"
    src.write_text(ROCRAND_PROBE)
    exe = d / "probe"
    subprocess.run([hipcc, "-O1", str(src), "-o", str(exe)], check=True, capture_output=True)

    def run(cases):
        inp = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
        out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
        got = [list(map(int, l.split())) for l in out.strip().splitlines()]
        assert len(got) == len(cases)
        return got
    return run


def test_philox_matches_rocrand_rounds(rocrand_rounds):
    """The oracle's Philox-4x32-10 equals rocRAND's rounds on the same
    (counter, key) pairs, all four words in use."""
    r = np.random.default_rng(11)
    cases = [[0] * 6, [0xFFFFFFFF] * 6] + r.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    for c, g in zip(cases, rocrand_rounds(cases)):
        assert list(oracle.philox4x32_10(c[:4], c[4:])) == g


@pytest.mark.parametrize("seed,s,na", [(7, 5_000_000, 1000), (2**40 + 12345, 4_294_967, 1001),
                                       (0xFFFFFFFFFFFFFFFF, 2**33 + 5, 977)])
def test_mc_placement_counter_past_2_pow_32(rocrand_rounds, seed, s, na):
    """Monte-Carlo draw (s, i) past the 32-bit counter range (Sec. 3.2's random
    starts, read as Philox-4x32-10 with counter (lo32 g, hi32 g, 0, 0),
    g = s * |A| + i, key (lo32 seed, hi32 seed), and start = off +
    floor(u * span / 2^64) with u = word1:word0): every placement of a shuffle
    whose counters all exceed 2^32 equals rocRAND's rounds on that counter,
    mapped to the range in Python integers."""
    assert s * na >= 2**32
    r = np.random.default_rng(s % 1000)
    off = r.integers(0, 2**31, size=na).astype(np.uint32)
    span = r.integers(1, 2**31, size=na).astype(np.uint32)
    span[:3] = [1, 2, 0x7FFFFFFF]
    got = oracle.mc_placements(seed, s, off, span)
    cases = []
    for i in range(na):
        g = s * na + i
        cases.append([g & 0xFFFFFFFF, g >> 32, 0, 0, seed & 0xFFFFFFFF, seed >> 32])
    words = rocrand_rounds(cases)
    for i, w in enumerate(words):
        u = (w[1] << 32) | w[0]
        assert int(got[i]) == int(off[i]) + ((u * int(span[i])) >> 64), i
    assert int(got[0]) == int(off[0])   # span 1: one legal start


# ---------------------------------------------------------------- Monte-Carlo

def _small_genome():
    return np.array([50, 80, 120, 33], np.uint32)


def test_mc_placement_range_and_uniformity():
    from scipy import stats
    lengths = _small_genome()
    off = oracle.genome_offsets(lengths)
    # one interval of length 11 on chromosome 2: 110 legal starts
    a_s = np.array([off[2] + 5], np.uint32)
    a_e = a_s + np.uint32(10)
    o, span, ln = oracle.mc_prepare(lengths, a_s, a_e)
    assert int(o[0]) == int(off[2]) and int(span[0]) == 120 - 11 + 1 and int(ln[0]) == 11
    starts = np.array([oracle.mc_placements(7, s, o, span)[0] for s in range(22_000)], np.int64)
    local = starts - int(off[2])
    assert local.min() >= 0 and local.max() <= 109
    hist = np.bincount(local, minlength=110)
    assert stats.chisquare(hist).pvalue > 1e-4
    assert hist.min() > 0


def test_mc_mean_matches_exact_expectation():
    lengths = _small_genome()
    off = oracle.genome_offsets(lengths).astype(np.int64)
    r = np.random.default_rng(2)
    def rand_set(n, maxlen):
        c = r.integers(0, 4, size=n)
        L = r.integers(1, maxlen + 1, size=n)
        s = r.integers(0, lengths[c].astype(np.int64) - L + 1)
        return (off[c] + s).astype(np.uint32), (off[c] + s + L - 1).astype(np.uint32)
    a_s, a_e = rand_set(40, 20)
    b_s, b_e = rand_set(60, 15)
    prep = oracle.mc_prepare(lengths, a_s, a_e)
    sbs, sbe = np.sort(b_s), np.sort(b_e)
    T = oracle.mc_totals(sbs, sbe, prep, 7, 0, 20_000, threads=4).astype(np.float64)
    E = oracle.mc_expected_total(lengths, a_s, a_e, b_s, b_e)
    se = T.std(ddof=1) / np.sqrt(len(T))
    assert abs(T.mean() - E) < 5 * se, (T.mean(), E, se)


def test_mc_split_ranges_and_tail():
    lengths, A, B = datagen.w2_sets(n_a=300, n_b=5000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    sbs, sbe = np.sort(b_s), np.sort(b_e)
    prep = oracle.mc_prepare(lengths, a_s, a_e)
    full = oracle.mc_totals(sbs, sbe, prep, 7, 0, 64, threads=3)
    halves = np.concatenate([oracle.mc_totals(sbs, sbe, prep, 7, 0, 29),
                             oracle.mc_totals(sbs, sbe, prep, 7, 29, 64)])
    assert np.array_equal(full, halves)
    # each shuffle total equals a plain count of the placed set
    for s in (0, 5, 63):
        st = oracle.mc_placements(7, s, prep[0], prep[1])
        _, t = oracle.counter(st, st + prep[2] - np.uint32(1), b_s, b_e)
        assert t == int(full[s])
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    ge, le = oracle.mc_tail(full, obs)
    assert ge == int((full >= obs).sum()) and le == int((full <= obs).sum())


def test_mc_enriched_set_has_smallest_pvalue():
    """A placed inside B's intervals on purpose: no shuffle reaches the
    observed total, so n_ge = 0 and p = 1/(N+1) exactly."""
    lengths, _, B = datagen.w2_sets(n_a=10, n_b=4000)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    a_s, a_e = b_s[:400].copy(), b_e[:400].copy()
    sbs, sbe = np.sort(b_s), np.sort(b_e)
    prep = oracle.mc_prepare(lengths, a_s, a_e)
    T = oracle.mc_totals(sbs, sbe, prep, 7, 0, 200, threads=4)
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    ge, _ = oracle.mc_tail(T, obs)
    assert ge == 0 and oracle.pvalue(ge, 200) == 1.0 / 201.0


def test_mc_rejects_interval_crossing_chromosome():
    lengths = _small_genome()
    with pytest.raises(ValueError):
        oracle.mc_prepare(lengths, np.array([45], np.uint32), np.array([55], np.uint32))


# ---------------------------------------------------------------- learned leaf model

def _params(rng):
    return rng.normal(0, 1, 49).astype(np.float32)


def test_rmi_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    p = _params(rng)
    u = rng.uniform(0, 1, 300).astype(np.float32)
    t = np.sort(rng.uniform(0, 1, 300)).astype(np.float32)
    loss, g = oracle.rmi_loss_grad(p, u, t)
    h = 1e-3
    for k in range(49):
        pp, pm = p.astype(np.float64).copy(), p.astype(np.float64).copy()
        pp[k] += h; pm[k] -= h
        # perturbation in fp64 through the fp32 interface: use values that are exact in fp32
        lp = oracle.rmi_loss_grad(pp.astype(np.float32), u, t)[0]
        lm = oracle.rmi_loss_grad(pm.astype(np.float32), u, t)[0]
        dp = float(pp.astype(np.float32)[k]) - float(pm.astype(np.float32)[k])
        fd = (lp - lm) / dp
        assert abs(fd - g[k]) <= 2e-3 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_rmi_forward_special_cases():
    u = np.linspace(0, 1, 11).astype(np.float32)
    p = np.zeros(49, np.float32)
    p[48] = 0.25                                    # constant network
    assert np.allclose(oracle.rmi_forward(p, u), 0.25)
    loss, g = oracle.rmi_loss_grad(p, u, np.zeros(11, np.float32))
    assert abs(loss - 0.0625) < 1e-12 and abs(g[48] - 0.5) < 1e-12
    p[:] = 0
    p[0], p[32] = 1.0, 1.0                          # y = relu(u) = identity on [0, 1]
    p[1], p[17], p[33] = 1.0, -0.5, -1.0            # minus relu(u - 0.5): flat after 0.5
    y = oracle.rmi_forward(p, u)
    assert np.allclose(y, np.minimum(u, 0.5), atol=1e-7)


def test_linear_fit_vs_polyfit():
    x = np.sort(np.random.default_rng(8).integers(0, 3_000_000_000, size=50_000).astype(np.uint32))
    a, b = oracle.linear_fit(x)
    pa, pb = np.polyfit(x.astype(np.float64), np.arange(len(x), dtype=np.float64), 1)
    assert abs(a - pa) <= 1e-9 * abs(pa) and abs(b - pb) <= 1e-6 * max(1.0, abs(pb))


def test_enumeration_oracle_golden(enum_golden):
    """Sub-problem 4 by the definition reproduces the hand-derived pair sets of
    a nested, tied fixture."""
    B, Q = enum_golden
    b = np.array(B, dtype=np.uint32)
    a = np.array([(s, e) for s, e, _, _ in Q], dtype=np.uint32)
    pa, pb = oracle.enumerate_bruteforce(a[:, 0], a[:, 1], b[:, 0], b[:, 1])
    for i, (_, _, st, _) in enumerate(Q):
        assert list(pb[pa == i]) == st, i


def test_enumeration_oracle_random():
    """Per query: every pair satisfies the closed predicate, none repeats, and
    the number of pairs equals the library-routine count (numpy searchsorted);
    the number of all pairs equals the independent endpoint sweep."""
    r = np.random.default_rng(42)
    for na, nb, span, ml in ((300, 500, 5_000, 60), (200, 2_000, 100_000, 3_000), (50, 40, 30, 0)):
        b_s = r.integers(0, span, nb).astype(np.uint32)
        b_e = b_s + r.integers(0, ml + 1, nb).astype(np.uint32)
        a_s = r.integers(0, span, na).astype(np.uint32)
        a_e = a_s + r.integers(0, ml + 1, na).astype(np.uint32)
        pa, pb = oracle.enumerate_bruteforce(a_s, a_e, b_s, b_e)
        assert np.all((a_s[pa] <= b_e[pb]) & (a_e[pa] >= b_s[pb]))
        assert len(np.unique(pa.astype(np.uint64) * nb + pb)) == len(pa)
        assert np.array_equal(np.bincount(pa, minlength=na), _np_count(a_s, a_e, b_s, b_e))
        assert len(pa) == oracle.sweep_total(a_s, a_e, b_s, b_e)


def test_median_and_enrichment_oracle():
    """The median of the totals equals numpy's median (library routine) on odd,
    even and tied samples; the enrichment score has its closed forms."""
    r = np.random.default_rng(3)
    for n in (1, 2, 3, 10, 999, 1000, 10_000):
        for hi in (5, 10**6, 2**50):
            t = r.integers(0, hi, n, dtype=np.uint64)
            lo_v, hi_v = oracle.mc_median(t)
            assert (lo_v + hi_v) / 2 == np.median(t.astype(np.float64))
            assert lo_v <= hi_v and np.sum(t < lo_v) <= (n - 1) // 2 < np.sum(t <= lo_v)
    assert oracle.enrichment(200, 100, 100) == 1.0
    assert oracle.enrichment(100, 99, 101) == 0.0
    assert oracle.enrichment(25, 100, 100) == -2.0
    assert oracle.enrichment(0, 3, 3) == -np.inf


def test_decision_oracle():
    """Sub-problem 1 is 'some count is non-zero': disjoint sets, one touching
    pair (closed intervals), and random sets against numpy searchsorted."""
    assert not oracle.decide([0, 20], [9, 29], [10, 30], [19, 39])
    assert oracle.decide([0, 20], [10, 29], [10, 30], [19, 39])
    r = np.random.default_rng(8)
    for _ in range(20):
        b_s = r.integers(0, 10**6, 50).astype(np.uint32)
        b_e = b_s + r.integers(0, 100, 50).astype(np.uint32)
        a_s = r.integers(0, 10**6, 30).astype(np.uint32)
        a_e = a_s + r.integers(0, 100, 30).astype(np.uint32)
        assert oracle.decide(a_s, a_e, b_s, b_e) == bool(np.any(_np_count(a_s, a_e, b_s, b_e) > 0))
