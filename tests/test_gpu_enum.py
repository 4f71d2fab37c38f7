"""GPU parity of enumeration (Sec. 1.1, sub-problem 4) through the C ABI:
the stable key-value sort behind the index, the count scan, and the pairs
themselves against the definition (brute-force oracle) and the hand-derived
golden fixture."""
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


def scan_order_ok(pb, b_s):
    """Within one query: decreasing start, equal starts by decreasing index."""
    if len(pb) < 2:
        return True
    s = b_s[pb].astype(np.int64)
    ds, di = np.diff(s), np.diff(pb.astype(np.int64))
    return bool(np.all((ds < 0) | ((ds == 0) & (di < 0))))


def enumerate_all(b_s, b_e, a_s, a_e, max_pairs=None, status=None, learned=False, with_first=True):
    """Step 1 (counts, first, offsets) and step 2 (pairs) through the C ABI;
    with_first=False lets the enumeration kernel find `first` by bisection."""
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=learned and len(b_s) > 0, train={"epochs": 20})
    counts, first, offsets = bits.bits_enum_counts(ref, up(a_s), up(a_e))
    assert np.array_equal(down(first), np.searchsorted(np.sort(b_s), a_e, side="right").astype(np.uint32))
    assert np.array_equal(down(offsets), np.concatenate([[0], np.cumsum(down(counts).astype(np.uint64))]))
    index = bits.bits_enum_index_build(up(b_s), up(b_e))
    pa, pb = bits.bits_enumerate(index, up(a_s), up(a_e), counts, offsets, first=first if with_first else None,
                                 max_pairs=max_pairs, status=status)
    return down(counts), down(offsets), index, down(pa), down(pb)


@pytest.mark.parametrize("n,span", [(1, 10), (4095, 1000), (16_384, 2**32), (16_385, 7), (70_001, 2**24),
                                    (300_000, 2**32), (5000, 1)])
def test_index_is_stable_sort_by_start(n, span):
    """The index is B_S sorted with each interval's input index carried along by
    a stable sort: equal to numpy's stable argsort (equal keys keep input order),
    across tile edges, skipped digit passes (span < 2^24) and all-equal keys."""
    note("case: index n=%d span=%d" % (n, span))
    r = np.random.default_rng(n + span % 97)
    b_s = r.integers(0, span, n, dtype=np.uint64).astype(np.uint32)
    b_e = b_s + r.integers(0, 100, n).astype(np.uint32)
    index = bits.bits_enum_index_build(up(b_s), up(b_e))
    order = np.argsort(b_s, kind="stable")
    assert np.array_equal(down(index.ids()), order.astype(np.uint32))
    assert np.array_equal(down(index.starts()), b_s[order])
    assert np.array_equal(down(index.ends()), b_e[order])


@pytest.mark.parametrize("n", [0, 1, 4095, 4096, 4097, 1_000_003])
def test_scan_counts(n):
    note("case: scan n=%d" % n)
    r = np.random.default_rng(n)
    c = r.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32) if n != 4097 else \
        np.full(n, 0xFFFFFFFF, np.uint32)
    off = down(bits.bits_scan_counts(up(c)))
    exp = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(c.astype(np.uint64), out=exp[1:])
    assert np.array_equal(off, exp)


def test_enumeration_golden(enum_golden):
    """Pairs and their backward-scan order on the hand-derived nested fixture."""
    note("case: enumeration golden")
    B, Q = enum_golden
    b = np.array(B, dtype=np.uint32)
    a = np.array([(s, e) for s, e, _, _ in Q], dtype=np.uint32)
    counts, offsets, _, pa, pb = enumerate_all(b[:, 0], b[:, 1], a[:, 0], a[:, 1])
    for i, (_, _, st, sc) in enumerate(Q):
        o, c = int(offsets[i]), int(counts[i])
        assert c == len(st)
        assert list(pa[o:o + c]) == [i] * c
        assert list(pb[o:o + c]) == sc, i


@pytest.mark.parametrize("case", range(6))
def test_enumeration_random_against_bruteforce(case):
    r = np.random.default_rng(500 + case)
    nb = int(r.choice([1, 31, 700, 5000, 12_000]))
    na = int(r.choice([1, 64, 999, 4000]))
    span = int(r.choice([100, 20_000, 10**6]))
    ml = int(r.choice([0, 5, 300, 20_000]))
    note("case %d: na=%d nb=%d span=%d maxlen=%d" % (case, na, nb, span, ml))
    b_s = r.integers(0, span, nb).astype(np.uint32)
    b_e = b_s + r.integers(0, ml + 1, nb).astype(np.uint32)
    a_s = r.integers(0, span, na).astype(np.uint32)
    a_e = a_s + r.integers(0, ml + 1, na).astype(np.uint32)
    ea, eb = oracle.enumerate_bruteforce(a_s, a_e, b_s, b_e)
    counts, offsets, _, pa, pb = enumerate_all(b_s, b_e, a_s, a_e, learned=case % 2 == 1,
                                               with_first=case % 3 != 2)
    assert np.array_equal(counts, np.bincount(ea, minlength=na).astype(np.uint32))
    assert int(offsets[-1]) == len(ea)
    assert np.array_equal(pa, np.repeat(np.arange(na, dtype=np.uint32), counts))
    for i in range(na):
        o, c = int(offsets[i]), int(counts[i])
        got = pb[o:o + c]
        assert np.array_equal(np.sort(got), eb[ea == i]), i
        assert scan_order_ok(got, b_s), i


def test_enumeration_at_scale_properties():
    """2e5 x 2e5 on the genome-scale recipe (uniform A, clustered mixture B):
    each query emits exactly count(a) distinct pairs that all satisfy the
    closed predicate, and count(a) is the oracle's, so the pair set is the
    exact one; the order within each query is the scan order."""
    note("case: enumeration at scale")
    lengths, A, B = datagen.w1_sets(seed=9, n_a=200_000, n_b=200_000)
    a_s, a_e = oracle.project(lengths, A.chrom, A.start, A.end)
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    exp_c, exp_t = oracle.counter(a_s, a_e, b_s, b_e, threads=8)
    counts, offsets, _, pa, pb = enumerate_all(b_s, b_e, a_s, a_e, learned=True)
    assert np.array_equal(counts, exp_c) and int(offsets[-1]) == exp_t
    assert np.array_equal(pa, np.repeat(np.arange(len(a_s), dtype=np.uint32), counts))
    assert np.all((a_s[pa] <= b_e[pb]) & (a_e[pa] >= b_s[pb]))
    key = pa.astype(np.uint64) * np.uint64(len(b_s)) + pb.astype(np.uint64)
    assert len(np.unique(key)) == len(key)
    # scan order: within a query, (start, index) strictly decreasing
    same = pa[1:] == pa[:-1]
    s0, s1 = b_s[pb[:-1]].astype(np.int64), b_s[pb[1:]].astype(np.int64)
    dec = (s1 < s0) | ((s1 == s0) & (pb[1:] < pb[:-1]))
    assert np.all(dec[same])


def test_enumeration_edges():
    note("case: enumeration edges")
    # empty B: every count is 0, nothing written
    counts, offsets, _, pa, pb = enumerate_all(np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                                               np.array([5, 9], np.uint32), np.array([6, 9], np.uint32))
    assert counts.tolist() == [0, 0] and offsets.tolist() == [0, 0, 0] and len(pa) == 0
    # a too-small pair buffer: nothing past it is written and the flag is raised
    b_s, b_e = np.array([0, 2, 4], np.uint32), np.array([10, 3, 5], np.uint32)
    a_s, a_e = np.array([1, 4], np.uint32), np.array([4, 4], np.uint32)
    st = torch.zeros(1, dtype=torch.uint32, device=DEV)
    counts, offsets, _, pa, pb = enumerate_all(b_s, b_e, a_s, a_e, max_pairs=3, status=st)
    assert counts.tolist() == [3, 2] and int(offsets[-1]) == 5 and len(pa) == 3
    assert int(down(st)[0]) & bits.BITS_FLAG_ENUM
    assert pa.tolist() == [0, 0, 0] and pb.tolist() == [2, 1, 0]
