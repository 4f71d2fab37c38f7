"""GPU parity at the workloads' full sizes, against the oracle on every output:
all per-query counts (1e7 and 5e7 queries), every shuffle total of the two
Monte-Carlo workloads (10,000 x 1e5 and 1,000 x 1e6), the observed totals and
the tail counts and p-values recomputed from the oracle's own totals, and all
2,048 pair totals of the uneven batch.  Every launch shape the autotuner can
pick for the counting kernels is run at full size, so whichever shape
bench.py times is covered.  The oracle runs multithreaded (about 2e9
evaluations in all)."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1208_3407_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1208_3407_amd import bits  # noqa: E402

from bench import MC_BATCH  # noqa: E402  (bench's binned pass size)

DEV = torch.device("cuda", 0)
THREADS = 16


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def up(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def down(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def proj(lengths, S):
    gs, ge = bits.bits_project(lengths, up(S.chrom), up(S.start), up(S.end))
    return gs, ge


def count_shapes(ref, path):
    """Every launch shape bits_autotune_count tries for this reference and path."""
    out = []
    dmin = min(ref.depth, 8)
    for block in (256, 512, 1024):
        for qpl in (1, 2, 4):
            if path == bits.BITS_PATH_LEARNED:
                out.append({"block": block, "qpl": qpl, "depth": 0, "grid": 0, "path": path})
            else:
                for d in range(ref.depth, dmin - 1, -1):
                    out.append({"block": block, "qpl": qpl, "depth": d, "grid": 0, "path": path})
    return out


def check_all_shapes(ref, a_s, a_e, exp_dev, total):
    """Per-query counts equal the oracle's (compared on the device) and the
    total equals it, at every candidate shape of the three counting paths."""
    counts = torch.empty_like(exp_dev)
    tot = torch.empty(1, dtype=torch.uint64, device=DEV)
    n = 0
    for path in (bits.BITS_PATH_LEARNED, bits.BITS_PATH_PLAIN, bits.BITS_PATH_TIERED):
        for lp in count_shapes(ref, path):
            bits.bits_count_per_query(ref, a_s, a_e, launch=lp, counts=counts, total=tot)
            assert torch.equal(counts, exp_dev), lp
            assert int(down(tot)[0]) == total, lp
            n += 1
    return n


def oracle_sets(lengths, S):
    return oracle.project(lengths, S.chrom, S.start, S.end)


def check_mc(mc, exp_T, obs, N):
    """Totals, observed, tail counts and p-value against the oracle's own totals."""
    assert np.array_equal(down(mc.totals), exp_T)
    assert int(down(mc.observed)[0]) == obs
    ge, le = oracle.mc_tail(exp_T, obs)
    assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == (ge, le)
    assert bits.bits_pvalue(int(down(mc.n_ge)[0]), N) == oracle.pvalue(ge, N)


def test_w1_full_every_count():
    note("case: W1 full 1e7 x 1e7, every per-query count, every launch shape")
    lengths, A, B = datagen.w1_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True)
    oa_s, oa_e = oracle_sets(lengths, A)
    ob_s, ob_e = oracle_sets(lengths, B)
    t0 = time.time()
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    exp, total = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS)
    assert total == oracle.sweep_total(oa_s, oa_e, ob_s, ob_e)
    note("  oracle %.1f s" % (time.time() - t0))
    assert np.array_equal(down(ref.sorted_starts()), sbs) and np.array_equal(down(ref.sorted_ends()), sbe)
    n = check_all_shapes(ref, a_s, a_e, up(exp), total)
    note("  %d launch shapes equal the oracle on all 1e7 counts" % n)
    assert bits.bits_get_status(ref) == 0


def test_w2_full_monte_carlo_every_shuffle():
    note("case: W2 full, all 10,000 shuffles vs the oracle")
    lengths, A, B = datagen.w2_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True)
    N = 10_000
    oa_s, oa_e = oracle_sets(lengths, A)
    ob_s, ob_e = oracle_sets(lengths, B)
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    t0 = time.time()
    exp_T = oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, 0, N, threads=THREADS)
    obs = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS, per_query=False)[1]
    note("  oracle %.1f s for 1e9 evaluations" % (time.time() - t0))
    for lp in ({"block": 1024, "qpl": 1, "depth": 0, "grid": 0, "path": 2},
               {"block": 512, "qpl": 1, "depth": 0, "grid": 0, "path": 2},
               {"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 1}):
        check_mc(bits.bits_mc_pvalue(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, N, launch=lp), exp_T, obs, N)
    check_mc(bits.bits_mc_binned(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, N, batch=MC_BATCH), exp_T, obs, N)
    assert bits.bits_get_status(ref) == 0


def test_w3_full_batch_every_pair():
    note("case: W3 full 32 x 64 pairs, all 2,048 totals vs the oracle")
    lengths, Q, R = datagen.w3_sets()
    qd = [proj(lengths, S) for S in Q]
    rd = [proj(lengths, S) for S in R]
    refs = bits.bits_sort_refs(rd)
    plan = bits.bits_batch_create(refs, qd)
    got1 = down(bits.bits_batch_run(plan)).copy()
    got2 = down(bits.bits_batch_run(plan)).reshape(len(Q), len(R))
    assert np.array_equal(got1.reshape(len(Q), len(R)), got2)
    t0 = time.time()
    oq = [oracle_sets(lengths, S) for S in Q]
    exp = np.zeros((len(Q), len(R)), np.uint64)
    for j, S in enumerate(R):
        rs, re_ = oracle_sets(lengths, S)
        sbs, sbe = oracle.sort_u32(rs), oracle.sort_u32(re_)
        for i, (qs, qe) in enumerate(oq):
            exp[i, j] = oracle.count_sorted(sbs, sbe, qs, qe, threads=THREADS, per_query=False)[1]
    note("  oracle %.1f s" % (time.time() - t0))
    assert np.array_equal(got2, exp)
    bits.bits_batch_destroy(plan)


def test_w4_full_every_count_and_shuffle():
    note("case: W4 full 5e7 x 5e7, every count and launch shape; MC 1000 x 1e6 vs the oracle")
    lengths, A, B = datagen.w4_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 80})   # bench.py's training
    oa_s, oa_e = oracle_sets(lengths, A)
    ob_s, ob_e = oracle_sets(lengths, B)
    del A, B
    t0 = time.time()
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    exp, total = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS)
    note("  oracle counts %.1f s" % (time.time() - t0))
    assert np.array_equal(down(ref.sorted_starts()), sbs) and np.array_equal(down(ref.sorted_ends()), sbe)
    n = check_all_shapes(ref, a_s, a_e, up(exp), total)
    note("  %d launch shapes equal the oracle on all 5e7 counts" % n)
    del exp
    nmc, N = 1_000_000, 1000
    prep = oracle.mc_prepare(lengths, oa_s[:nmc], oa_e[:nmc])
    t0 = time.time()
    exp_T = oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, 0, N, threads=THREADS)
    obs = oracle.count_sorted(sbs, sbe, oa_s[:nmc], oa_e[:nmc], threads=THREADS, per_query=False)[1]
    note("  oracle Monte-Carlo %.1f s for 1e9 evaluations" % (time.time() - t0))
    # the region-binned path in bench.py's configuration (one pass of MC_BATCH shuffles), under
    # both observed-pass launches bench.py's tuner can pick, and the query-ordered paths
    for blk in (512, 1024):
        lp = {"block": blk, "qpl": 1, "depth": 0, "grid": 0, "path": 2}
        check_mc(bits.bits_mc_binned(ref, a_s[:nmc], a_e[:nmc], lengths, datagen.MC_SEED, 0, N, batch=MC_BATCH,
                                     launch=lp), exp_T, obs, N)
        check_mc(bits.bits_mc_pvalue(ref, a_s[:nmc], a_e[:nmc], lengths, datagen.MC_SEED, 0, N, launch=lp),
                 exp_T, obs, N)
    check_mc(bits.bits_mc_pvalue(ref, a_s[:nmc], a_e[:nmc], lengths, datagen.MC_SEED, 0, N,
                                 launch={"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 1}), exp_T, obs, N)
    assert bits.bits_get_status(ref) == 0


def test_binned_reference_past_2_pow_26():
    """A reference of 7e7 intervals (64 counts of n can pass 2^32, so the search
    kernel sums each 64-record step in 64 bits): every binned total equals the
    oracle's."""
    note("case: binned, n = 7e7")
    lengths, A, B = datagen.w4_sets(seed=3, n_a=20_000, n_b=70_000_000)
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e)
    mb = bits.bits_mc_binned(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, 12, batch=5)
    ob_s, ob_e = oracle_sets(lengths, B)
    del B
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    oa_s, oa_e = oracle_sets(lengths, A)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    exp_T = oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, 0, 12, threads=THREADS)
    obs = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS, per_query=False)[1]
    check_mc(mb, exp_T, obs, 12)
    assert bits.bits_get_status(ref) == 0


def test_monte_carlo_counter_past_2_pow_32():
    """Shuffles whose Philox counters g = s * |A| + i all exceed 2^32 (the
    counter's high word in use): the query-ordered plain and learned paths,
    the binned path and the paper's orientation (roles swapped: g = s * |B| + j)
    equal the oracle shuffle by shuffle."""
    note("case: Monte-Carlo counters past 2^32")
    lengths, A, B = datagen.w2_sets(seed=5, n_a=1000, n_b=200_000)
    oa_s, oa_e = oracle_sets(lengths, A)
    ob_s, ob_e = oracle_sets(lengths, B)
    s0, s1 = 5_000_000, 5_000_024
    assert s0 * len(oa_s) > 2**32
    a_s, a_e, b_s, b_e = up(oa_s), up(oa_e), up(ob_s), up(ob_e)
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    exp_T = oracle.mc_totals(sbs, sbe, oracle.mc_prepare(lengths, oa_s, oa_e), 2**33 + 7, s0, s1, threads=8)
    obs = oracle.count_sorted(sbs, sbe, oa_s, oa_e, per_query=False)[1]
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 20})
    for lp in ({"block": 1024, "qpl": 1, "depth": 0, "grid": 0, "path": 2},
               {"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 1}):
        check_mc(bits.bits_mc_pvalue(ref, a_s, a_e, lengths, 2**33 + 7, s0, s1, launch=lp), exp_T, obs, s1 - s0)
    for batch in (1, 7, 24):
        check_mc(bits.bits_mc_binned(ref, a_s, a_e, lengths, 2**33 + 7, s0, s1, batch=batch), exp_T, obs, s1 - s0)
    # the paper's orientation: the 1000-interval set randomised and re-sorted every round,
    # the 2e5-interval set fixed; the randomised set's counters are s * 1000 + j
    r0, r1 = 5_000_003, 5_000_013
    exp_R = oracle.mc_totals(sbs, sbe, oracle.mc_prepare(lengths, oa_s, oa_e), 2**33 + 7, r0, r1)
    mr = bits.bits_mc_resort(b_s, b_e, a_s, a_e, lengths, 2**33 + 7, r0, r1, batch=4)
    assert np.array_equal(down(mr.totals), exp_R)
    assert int(down(mr.observed)[0]) == obs
    assert bits.bits_get_status(ref) == 0
