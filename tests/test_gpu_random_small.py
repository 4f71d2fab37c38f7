"""Randomised GPU parity on many small seeded shapes: both search paths,
Monte-Carlo and batched pairs against the oracle, bit for bit.  Sizes cross
the 32-key line, the 4096-key sort tile and the learned index's 4096 leaves
(most leaves empty at these sizes), with heavy duplicates, point intervals
and touching endpoints."""
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1208_3407_amd import bits  # noqa: E402

DEV = torch.device("cuda", 0)
SIZES = [0, 1, 2, 31, 32, 33, 63, 64, 65, 127, 1000, 4095, 4096, 4097, 9000, 33_333]


def up(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint32))).to(DEV)


def down(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_set(r, n, span, maxlen):
    s = r.integers(0, span, size=n).astype(np.uint32)
    e = s + r.integers(0, maxlen + 1, size=n).astype(np.uint32)
    return s, e


@pytest.mark.parametrize("case", range(24))
def test_random_counts_both_paths(case):
    r = np.random.default_rng(1000 + case)
    nb = int(r.choice(SIZES))
    na = int(r.choice(SIZES[1:]))
    span = int(r.choice([50, 5_000, 10**6, 2**31]))
    maxlen = int(r.choice([0, 3, 100, 5_000]))
    print("case %d: na=%d nb=%d span=%d maxlen=%d" % (case, na, nb, span, maxlen), flush=True)
    sys.stdout.flush()
    b_s, b_e = rand_set(r, nb, span, maxlen)
    a_s, a_e = rand_set(r, na, span + maxlen, maxlen)
    exp, tot = oracle.counter(a_s, a_e, b_s, b_e, threads=4)
    learned = nb > 0
    ref = bits.bits_sort_ref(up(b_s), up(b_e), depth=int(r.integers(0, 14)), learned=learned,
                             train={"epochs": int(r.choice([0, 20]))})
    paths = [bits.BITS_PATH_PLAIN, bits.BITS_PATH_TIERED] + ([bits.BITS_PATH_LEARNED] if learned else [])
    for path in paths:
        for qpl in (1, 2, 4):
            lp = {"path": path, "qpl": qpl, "block": int(r.choice([256, 512, 1024]))}
            c, t = bits.bits_count_per_query(ref, up(a_s), up(a_e), launch=lp)
            assert np.array_equal(down(c), exp), lp
            assert int(down(t)[0]) == tot, lp
    assert bits.bits_get_status(ref) == 0


@pytest.mark.parametrize("case", range(6))
def test_random_monte_carlo(case):
    r = np.random.default_rng(2000 + case)
    lengths = r.integers(100, 5000, size=int(r.integers(1, 6))).astype(np.uint32)
    off = oracle.genome_offsets(lengths).astype(np.int64)

    def placed(n, maxlen):
        c = r.integers(0, len(lengths), size=n)
        L = r.integers(1, maxlen + 1, size=n)
        L = np.minimum(L, lengths[c].astype(np.int64))
        s = r.integers(0, lengths[c].astype(np.int64) - L + 1)
        return (off[c] + s).astype(np.uint32), (off[c] + s + L - 1).astype(np.uint32)

    na, nb = int(r.integers(1, 3000)), int(r.integers(1, 5000))
    a_s, a_e = placed(na, 60)
    b_s, b_e = placed(nb, 40)
    s0, s1 = int(r.integers(0, 50)), int(r.integers(50, 90))
    seed = int(r.integers(0, 2**63))
    print("case %d: na=%d nb=%d shuffles [%d,%d) seed=%d" % (case, na, nb, s0, s1, seed), flush=True)
    prep = oracle.mc_prepare(lengths, a_s, a_e)
    exp = oracle.mc_totals(np.sort(b_s), np.sort(b_e), prep, seed, s0, s1, threads=4)
    obs = oracle.counter(a_s, a_e, b_s, b_e)[1]
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": 10})
    for path in (bits.BITS_PATH_PLAIN, bits.BITS_PATH_LEARNED):
        mc = bits.bits_mc_pvalue(ref, up(a_s), up(a_e), lengths, seed, s0, s1, launch={"path": path})
        assert np.array_equal(down(mc.totals), exp), path
        assert int(down(mc.observed)[0]) == obs
        assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == oracle.mc_tail(exp, obs)


@pytest.mark.parametrize("learned", [False, True])
def test_random_batch_shapes(learned):
    r = np.random.default_rng(77)
    qsets = [rand_set(r, int(n), 10**6, 300) for n in (0, 1, 33, 5000, 70_000)]
    rsets = [rand_set(r, int(n), 10**6, 300) for n in (0, 1, 32, 4097, 50_000, 3)]
    refs = bits.bits_sort_refs([(up(s), up(e)) for s, e in rsets], learned=learned, train={"epochs": 5})
    for lp in ({"block": 256, "qpl": 2}, {"block": 1024, "qpl": 1}, {"block": 512, "qpl": 4, "grid": 3}):
        plan = bits.bits_batch_create(refs, [(up(s), up(e)) for s, e in qsets], launch=lp)
        got = down(bits.bits_batch_run(plan)).reshape(len(qsets), len(rsets))
        for i, (qs, qe) in enumerate(qsets):
            for j, (rs, re_) in enumerate(rsets):
                assert int(got[i, j]) == oracle.counter(qs, qe, rs, re_)[1], (lp, i, j)
        bits.bits_batch_destroy(plan)
