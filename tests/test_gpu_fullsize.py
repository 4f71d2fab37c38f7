"""GPU parity at the workloads' full sizes, in the launch shapes bench.py
times.  The oracle recomputes sampled outputs one by one (per-query counts of
sampled queries, sampled shuffles, sampled pairs); totals are checked against
the oracle's independent endpoint merge; the rest through properties that
hold at any size (learned == plain, tail counts from the totals)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1208_3407_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1208_3407_amd import bits  # noqa: E402

from bench import RECORDED_LEARNED, RECORDED_MC, RECORDED_PLAIN  # noqa: E402  (bench's launch shapes)

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


def test_w1_full_per_query_sampled_and_total():
    note("case: W1 full 1e7 x 1e7")
    lengths, A, B = datagen.w1_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True)
    c_plain, t_plain = bits.bits_count_per_query(ref, a_s, a_e, launch=RECORDED_PLAIN)
    c_plain = down(c_plain).copy()
    c_learn, t_learn = bits.bits_count_per_query(ref, a_s, a_e, launch=RECORDED_LEARNED)
    assert np.array_equal(down(c_learn), c_plain)
    oa_s, oa_e = oracle.project(lengths, A.chrom, A.start, A.end)
    ob_s, ob_e = oracle.project(lengths, B.chrom, B.start, B.end)
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    idx = np.unique(np.concatenate([np.arange(1000), np.random.default_rng(0).integers(0, len(oa_s), 100_000),
                                    np.arange(len(oa_s) - 1000, len(oa_s))]))
    exp, _ = oracle.count_sorted(sbs, sbe, oa_s[idx], oa_e[idx], threads=THREADS)
    assert np.array_equal(c_plain[idx], exp)
    total = oracle.sweep_total(oa_s, oa_e, ob_s, ob_e)
    assert int(down(t_plain)[0]) == total and int(down(t_learn)[0]) == total
    assert int(c_plain.astype(np.uint64).sum()) == total
    assert bits.bits_get_status(ref) == 0


def test_w2_full_monte_carlo_sampled_shuffles():
    note("case: W2 full, 10,000 shuffles")
    lengths, A, B = datagen.w2_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True)
    N = 10_000
    mc = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, N, launch=RECORDED_MC)
    T = down(mc.totals).copy()
    obs, ge, le = int(down(mc.observed)[0]), int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])
    mcp = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, N, launch=RECORDED_PLAIN)
    assert np.array_equal(down(mcp.totals), T)
    oa_s, oa_e = oracle.project(lengths, A.chrom, A.start, A.end)
    ob_s, ob_e = oracle.project(lengths, B.chrom, B.start, B.end)
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    for s in (0, 1, 2, 4999, 9998, 9999):
        assert int(T[s]) == int(oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, s, s + 1)[0]), s
    assert obs == oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS, per_query=False)[1]
    assert (ge, le) == oracle.mc_tail(T, obs)
    assert bits.bits_pvalue(ge, N) == oracle.pvalue(ge, N)


def test_w3_full_batch_sampled_pairs():
    note("case: W3 full 32 x 64 pairs")
    lengths, Q, R = datagen.w3_sets()
    qd = [proj(lengths, S) for S in Q]
    rd = [proj(lengths, S) for S in R]
    refs = bits.bits_sort_refs(rd)
    plan = bits.bits_batch_create(refs, qd)
    got1 = down(bits.bits_batch_run(plan)).copy()
    got2 = down(bits.bits_batch_run(plan)).reshape(len(Q), len(R))
    assert np.array_equal(got1.reshape(len(Q), len(R)), got2)
    qsz = np.array([len(S) for S in Q])
    rsz = np.array([len(S) for S in R])
    pairs = {(int(np.argmax(qsz)), int(np.argmax(rsz))), (int(np.argmin(qsz)), int(np.argmin(rsz))),
             (int(np.argmax(qsz)), int(np.argmin(rsz))), (3, 17), (31, 63), (0, 0)}
    for i, j in sorted(pairs):
        qs, qe = oracle.project(lengths, Q[i].chrom, Q[i].start, Q[i].end)
        rs, re_ = oracle.project(lengths, R[j].chrom, R[j].start, R[j].end)
        sbs, sbe = oracle.sort_u32(rs), oracle.sort_u32(re_)
        exp = oracle.count_sorted(sbs, sbe, qs, qe, threads=THREADS, per_query=False)[1]
        assert int(got2[i, j]) == exp, (i, j)
    # every pair equals the single-pair entry point on the same reference
    for i in (0, 5, 31):
        for j in (0, 40, 63):
            assert int(down(bits.bits_count(refs[j], qd[i][0], qd[i][1]))[0]) == int(got2[i, j])
    bits.bits_batch_destroy(plan)


def test_w4_full_learned_vs_plain_and_sampled():
    note("case: W4 full 5e7 x 5e7 + MC 1000 x 1e6")
    lengths, A, B = datagen.w4_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True)
    c_learn, t_learn = bits.bits_count_per_query(ref, a_s, a_e, launch=RECORDED_LEARNED)
    c_learn = down(c_learn).copy()
    c_plain, t_plain = bits.bits_count_per_query(ref, a_s, a_e, launch=RECORDED_PLAIN)
    assert np.array_equal(down(c_plain), c_learn)
    oa_s, oa_e = oracle.project(lengths, A.chrom, A.start, A.end)
    ob_s, ob_e = oracle.project(lengths, B.chrom, B.start, B.end)
    del A, B
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    assert np.array_equal(down(ref.sorted_starts()), sbs)
    assert np.array_equal(down(ref.sorted_ends()), sbe)
    idx = np.random.default_rng(1).integers(0, len(oa_s), 200_000)
    exp, _ = oracle.count_sorted(sbs, sbe, oa_s[idx], oa_e[idx], threads=THREADS)
    assert np.array_equal(c_learn[idx], exp)
    _, total = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=THREADS, per_query=False)
    assert int(down(t_learn)[0]) == total and int(down(t_plain)[0]) == total
    nmc = 1_000_000
    mc = bits.bits_mc_pvalue(ref, a_s[:nmc], a_e[:nmc], lengths, datagen.MC_SEED, 0, 1000, launch=RECORDED_MC)
    T = down(mc.totals).copy()
    prep = oracle.mc_prepare(lengths, oa_s[:nmc], oa_e[:nmc])
    for s in (0, 1, 500, 999):
        assert int(T[s]) == int(oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, s, s + 1)[0]), s
    obs = oracle.count_sorted(sbs, sbe, oa_s[:nmc], oa_e[:nmc], threads=THREADS, per_query=False)[1]
    assert int(down(mc.observed)[0]) == obs
    assert (int(down(mc.n_ge)[0]), int(down(mc.n_le)[0])) == oracle.mc_tail(T, obs)
    # the region-binned path in bench.py's configuration (one pass of 1000 shuffles)
    from bench import MC_BATCH
    mb = bits.bits_mc_binned(ref, a_s[:nmc], a_e[:nmc], lengths, datagen.MC_SEED, 0, 1000, batch=MC_BATCH,
                             launch=RECORDED_MC)
    assert np.array_equal(down(mb.totals), T)
    assert int(down(mb.observed)[0]) == obs
    assert (int(down(mb.n_ge)[0]), int(down(mb.n_le)[0])) == oracle.mc_tail(T, obs)
    assert bits.bits_get_status(ref) == 0


def test_binned_reference_past_2_pow_26():
    """A reference of 7e7 intervals (64 counts of n can pass 2^32, so the search
    kernel sums each 64-record step in 64 bits): the binned totals equal the
    query-ordered plain path's, and sampled shuffles equal the oracle's."""
    note("case: binned, n = 7e7")
    lengths, A, B = datagen.w4_sets(seed=3, n_a=20_000, n_b=70_000_000)
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e)
    mb = bits.bits_mc_binned(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, 12, batch=5)
    mp = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, datagen.MC_SEED, 0, 12, launch=RECORDED_PLAIN)
    T = down(mb.totals).copy()
    assert np.array_equal(T, down(mp.totals))
    assert int(down(mb.observed)[0]) == int(down(mp.observed)[0])
    ob_s, ob_e = oracle.project(lengths, B.chrom, B.start, B.end)
    del B
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    oa_s, oa_e = oracle.project(lengths, A.chrom, A.start, A.end)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    for s in (0, 11):
        assert int(T[s]) == int(oracle.mc_totals(sbs, sbe, prep, datagen.MC_SEED, s, s + 1, threads=THREADS)[0]), s
    assert bits.bits_get_status(ref) == 0
