"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, on seeded synthetic inputs.  Counts, ranks, per-shuffle
totals and tail counts are integers and must be bit-exact."""
import sys

import numpy as np
import pytest

import oracle
from paper_1208_3407_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)
from paper_1208_3407_amd import bits  # noqa: E402  (loads libbits.so; raises if not built)

DEV = torch.device("cuda", 0)


def up(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint32))).to(DEV)


def down(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def project_both(lengths, S):
    gs, ge = bits.bits_project(lengths, up(S.chrom), up(S.start), up(S.end))
    os_, oe = oracle.project(lengths, S.chrom, S.start, S.end)
    assert np.array_equal(down(gs), os_) and np.array_equal(down(ge), oe)
    return gs, ge, os_, oe


LAUNCHES = [
    {"path": bits.BITS_PATH_PLAIN},
    {"path": bits.BITS_PATH_PLAIN, "block": 256, "qpl": 1, "depth": 0},
    {"path": bits.BITS_PATH_PLAIN, "block": 512, "qpl": 4, "depth": 9},
    {"path": bits.BITS_PATH_PLAIN, "block": 1024, "qpl": 2, "depth": 13, "grid": 7},
    {"path": bits.BITS_PATH_TIERED},
    {"path": bits.BITS_PATH_TIERED, "block": 256, "qpl": 4, "depth": 0},
    {"path": bits.BITS_PATH_TIERED, "block": 1024, "qpl": 1, "depth": 13, "grid": 5},
    {"path": bits.BITS_PATH_TIERED, "block": 1024, "qpl": 4, "depth": 13},
]


def test_w0_full_against_oracle_and_bruteforce():
    note("case: W0 10k x 10k")
    lengths, A, B = datagen.w0_sets()
    a_s, a_e, oa_s, oa_e = project_both(lengths, A)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e)
    assert np.array_equal(down(ref.sorted_starts()), oracle.sort_u32(ob_s))
    assert np.array_equal(down(ref.sorted_ends()), oracle.sort_u32(ob_e))
    exp, tot = oracle.counter(oa_s, oa_e, ob_s, ob_e)
    for lp in LAUNCHES:
        c, t = bits.bits_count_per_query(ref, a_s, a_e, launch=lp)
        assert np.array_equal(down(c), exp), lp
        assert int(down(t)[0]) == tot
        assert int(down(bits.bits_count(ref, a_s, a_e, launch=lp))[0]) == tot
    bc, bt = oracle.count_bruteforce(oa_s[:500], oa_e[:500], ob_s[:500], ob_e[:500])
    r5 = bits.bits_sort_ref(b_s[:500].contiguous(), b_e[:500].contiguous())
    c5, t5 = bits.bits_count_per_query(r5, a_s[:500].contiguous(), a_e[:500].contiguous())
    assert np.array_equal(down(c5), bc) and int(down(t5)[0]) == bt
    assert bits.bits_get_status(ref) == 0


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 70_001), (65_537, 4_099), (300_000, 500_000)])
def test_genome_scale_shapes_plain_and_learned(na, nb):
    note("case: W1 shape %d x %d" % (na, nb))
    lengths, A, B = datagen.w1_sets(seed=3, n_a=na, n_b=nb)
    a_s, a_e, oa_s, oa_e = project_both(lengths, A)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    exp, tot = oracle.counter(oa_s, oa_e, ob_s, ob_e, threads=8)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 60})
    assert np.array_equal(down(ref.sorted_starts()), np.sort(ob_s))
    assert np.array_equal(down(ref.sorted_ends()), np.sort(ob_e))
    for lp in LAUNCHES + [{"path": bits.BITS_PATH_LEARNED, "qpl": q} for q in (1, 2, 4)]:
        c, t = bits.bits_count_per_query(ref, a_s, a_e, launch=lp)
        assert np.array_equal(down(c), exp), lp
        assert int(down(t)[0]) == tot, lp
    assert bits.bits_get_status(ref) == 0


@pytest.mark.parametrize("n", [1, 31, 32, 33, 63, 64, 65, 1000, 4097, 70_001])
def test_learned_count_head_edges(n):
    """The learned count's head search at line and array edges: references of sizes around
    the 32-key line, queries whose ends sit on keys, one before and one after them, at
    coordinate 0 and at 2^32 - 1, against the oracle; trained and untrained models."""
    note("case: learned head edges n=%d" % n)
    r = np.random.default_rng(n)
    b_s = np.sort(r.integers(0, 2**32 - 2, n, dtype=np.uint64)).astype(np.uint32)
    b_s[: n // 3] = b_s[0]                       # a run of equal keys at the start
    b_e = np.minimum(b_s.astype(np.uint64) + r.integers(0, 1000, n), 2**32 - 2).astype(np.uint32)
    pick = r.integers(0, n, 3000)
    a_s = np.concatenate([b_e[pick].astype(np.int64) + r.integers(-1, 2, len(pick)), [0, 0, 2**32 - 2]])
    a_s = a_s.clip(0, 2**32 - 2).astype(np.uint32)
    a_e = np.concatenate([b_s[pick].astype(np.int64) + r.integers(-1, 2, len(pick)), [0, 2**32 - 2, 2**32 - 2]])
    a_e = np.maximum(a_e.clip(0, 2**32 - 2), a_s).astype(np.uint32)
    exp, tot = oracle.count_sorted(np.sort(b_s), np.sort(b_e), a_s, a_e)
    for epochs in (0, 40):
        ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": epochs})
        c, t = bits.bits_count_per_query(ref, up(a_s), up(a_e), launch={"path": 2})
        assert np.array_equal(down(c), exp), (n, epochs)
        assert int(down(t)[0]) == tot
        assert bits.bits_get_status(ref) == 0


def test_edge_cases():
    note("case: edge cases")
    z = torch.empty(0, dtype=torch.uint32, device=DEV)
    # empty reference
    ref0 = bits.bits_sort_ref(z, z)
    c, t = bits.bits_count_per_query(ref0, up([1, 5]), up([3, 9]))
    assert list(down(c)) == [0, 0] and int(down(t)[0]) == 0
    # empty queries
    ref1 = bits.bits_sort_ref(up([1, 2]), up([5, 6]))
    c, t = bits.bits_count_per_query(ref1, z, z)
    assert c.numel() == 0 and int(down(t)[0]) == 0
    # all keys equal (every digit constant: sort copies), duplicates
    ref2 = bits.bits_sort_ref(up([7] * 5000), up([7] * 5000), learned=True, train={"epochs": 5})
    for lp in ({"path": 1}, {"path": 2}, {"path": 3}):
        c, _ = bits.bits_count_per_query(ref2, up([0, 7, 8, 0]), up([6, 7, 9, 100]), launch=lp)
        assert list(down(c)) == [0, 5000, 0, 5000]
    # extreme coordinates: end = 2^32 - 1 and start = 0
    M = 0xFFFFFFFF
    bs, be = [0, 5, M - 1, M], [0, M, M, M]
    qs, qe = [0, M, 3, M - 1], [M, M, 4, M - 1]
    ref3 = bits.bits_sort_ref(up(bs), up(be), learned=True, train={"epochs": 5})
    exp, _ = oracle.count_bruteforce(qs, qe, bs, be)
    for lp in ({"path": 1}, {"path": 2}, {"path": 3}):
        c, _ = bits.bits_count_per_query(ref3, up(qs), up(qe), launch=lp)
        assert np.array_equal(down(c), exp), lp
    # golden fixtures (contained intervals, touching endpoints)
    import os
    gdir = os.path.join(os.path.dirname(__file__), "golden")
    for name in ("contained.txt", "touching.txt"):
        A, B, E = [], [], []
        for line in open(os.path.join(gdir, name)):
            f = line.split("#")[0].split()
            if not f:
                continue
            (B if f[0] == "B" else A).append((int(f[1]), int(f[2])))
            if f[0] == "A":
                E.append(int(f[3]))
        A, B = np.array(A, np.uint32), np.array(B, np.uint32)
        r = bits.bits_sort_ref(up(B[:, 0]), up(B[:, 1]))
        c, _ = bits.bits_count_per_query(r, up(A[:, 0]), up(A[:, 1]))
        assert list(down(c)) == E, name
    # inverted query interval: flagged, counted as zero
    c, _ = bits.bits_count_per_query(ref1, up([4, 1]), up([3, 2]))
    assert list(down(c)) == [0, 2]
    assert bits.bits_get_status(ref1) & bits.BITS_FLAG_INTERVAL


def test_heavy_duplicates_and_clustered_keys():
    note("case: duplicates")
    r = np.random.default_rng(9)
    nb = 200_000
    s = r.integers(0, 3000, size=nb).astype(np.uint32) * np.uint32(1000)
    e = s + r.integers(0, 4, size=nb).astype(np.uint32) * np.uint32(500)
    qs = r.integers(0, 3_000_000, size=50_000).astype(np.uint32)
    qe = qs + r.integers(0, 2000, size=50_000).astype(np.uint32)
    exp, tot = oracle.counter(qs, qe, s, e, threads=8)
    ref = bits.bits_sort_ref(up(s), up(e), learned=True, train={"epochs": 40})
    for lp in ({"path": 1}, {"path": 2}, {"path": 1, "depth": 4, "qpl": 4}):
        c, t = bits.bits_count_per_query(ref, up(qs), up(qe), launch=lp)
        assert np.array_equal(down(c), exp), lp
        assert int(down(t)[0]) == tot


@pytest.mark.parametrize("kind", ["descending", "top_byte_only", "low_byte_only", "few_distinct"])
def test_sort_key_patterns(kind):
    """The keys-only radix sort on patterns that stress single digit passes: a descending
    run, keys that differ only in the top or only in the low byte (the other passes are
    skipped), and a few distinct values (long equal-digit runs in every tile), at
    3 x 20480 + 5 keys, against numpy."""
    note("case: sort pattern %s" % kind)
    n = 3 * 20480 + 5
    r = np.random.default_rng(7)
    if kind == "descending":
        k = np.arange(n, 0, -1, dtype=np.uint64) * 65_537 % 2**32
    elif kind == "top_byte_only":
        k = (r.integers(0, 256, n, dtype=np.uint64) << 24) | 0x00ABCDEF
    elif kind == "low_byte_only":
        k = r.integers(0, 256, n, dtype=np.uint64) | 0x12345600
    else:
        k = r.choice(np.array([0, 1, 2**31, 2**32 - 1], np.uint64), n)
    k = k.astype(np.uint32)
    e = np.roll(k, 17)
    ref = bits.bits_sort_ref(up(k), up(e))
    assert np.array_equal(down(ref.sorted_starts()), np.sort(k))
    assert np.array_equal(down(ref.sorted_ends()), np.sort(e))
    assert bits.bits_get_status(ref) == 0


def test_segmented_sort_many_references():
    """Segments of every size class around the keys-only sort's 20480-key tile
    (one short of a tile, exactly one, one more, three and a ragged tail)."""
    note("case: segmented sort")
    r = np.random.default_rng(5)
    sizes = [0, 1, 4097, 20_479, 20_480, 20_481, 61_441, 100_000, 12_345]
    sets = []
    for n in sizes:
        a = r.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
        b = r.integers(0, 2**20, size=n, dtype=np.uint64).astype(np.uint32)
        sets.append((a, b))
    refs = bits.bits_sort_refs([(up(a), up(b)) for a, b in sets])
    for (a, b), ref in zip(sets, refs):
        assert np.array_equal(down(ref.sorted_starts()), oracle.sort_u32(a))
        assert np.array_equal(down(ref.sorted_ends()), oracle.sort_u32(b))


def test_monte_carlo_per_shuffle_totals():
    note("case: MC small")
    lengths, A, B = datagen.w2_sets(seed=1, n_a=3000, n_b=60_000)
    a_s, a_e, oa_s, oa_e = project_both(lengths, A)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    sbs, sbe = np.sort(ob_s), np.sort(ob_e)
    exp = oracle.mc_totals(sbs, sbe, prep, 7, 0, 40, threads=8)
    obs = oracle.counter(oa_s, oa_e, ob_s, ob_e)[1]
    ge, le = oracle.mc_tail(exp, obs)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 40})
    for lp in ({"path": 1}, {"path": 2}, {"path": 1, "qpl": 1, "block": 256}, {"path": 2, "qpl": 4}):
        mc = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, seed=7, s0=0, s1=40, launch=lp)
        assert np.array_equal(down(mc.totals), exp), lp
        assert int(down(mc.observed)[0]) == obs
        assert int(down(mc.n_ge)[0]) == ge and int(down(mc.n_le)[0]) == le
    # a shuffle range continues the same stream
    part = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, seed=7, s0=17, s1=40)
    assert np.array_equal(down(part.totals), exp[17:])
    assert bits.bits_pvalue(ge, 40) == (1.0 + ge) / 41.0
    assert bits.bits_get_status(ref) == 0


def test_monte_carlo_rejects_query_outside_chromosome():
    note("case: MC chrom flag")
    lengths = np.array([100, 200], np.uint32)
    b_s, b_e = np.array([0, 150, 100], np.uint32), np.array([10, 160, 299], np.uint32)
    ref = bits.bits_sort_ref(up(b_s), up(b_e))
    # query 0 crosses the end of chromosome 0; query 1 is valid
    mc = bits.bits_mc_pvalue(ref, up([95, 120]), up([105, 130]), lengths, seed=7, s0=0, s1=6)
    t = down(mc.totals)
    assert bits.bits_get_status(ref) & bits.BITS_FLAG_CHROM
    off1, span1, len1 = oracle.mc_prepare(lengths, np.array([120], np.uint32), np.array([130], np.uint32))
    off = np.array([0, off1[0]], np.uint32)
    span = np.array([1, span1[0]], np.uint32)
    for s in range(6):
        st = oracle.mc_placements(7, s, off, span)[1:2]     # counter g = 2 s + 1
        _, exp = oracle.counter(st, st + len1 - np.uint32(1), b_s, b_e)
        assert int(t[s]) == exp, s
    assert int(down(mc.observed)[0]) == oracle.counter(np.array([120], np.uint32), np.array([130], np.uint32),
                                                       b_s, b_e)[1]


def test_batch_pairs_graph_replay():
    note("case: batch")
    lengths, Q, R = datagen.w3_sets(seed=2, n_q=5, n_r=7, q_range=(10, 30_000), r_range=(100, 80_000))
    qd, qo = [], []
    for S in Q:
        s, e, os_, oe = project_both(lengths, S)
        qd.append((s, e))
        qo.append((os_, oe))
    rd, ro = [], []
    for S in R:
        s, e, os_, oe = project_both(lengths, S)
        rd.append((s, e))
        ro.append((os_, oe))
    refs = bits.bits_sort_refs(rd)
    exp = np.zeros((len(Q), len(R)), np.uint64)
    for i, (qs, qe) in enumerate(qo):
        for j, (rs, re_) in enumerate(ro):
            exp[i, j] = oracle.counter(qs, qe, rs, re_)[1]
    lrefs = bits.bits_sort_refs(rd, learned=True, train={"epochs": 10})
    for rr, lp in ((refs, None), (refs, {"block": 256, "qpl": 1, "depth": 5}), (refs, {"block": 1024, "qpl": 4}),
                   (lrefs, None), (lrefs, {"block": 512, "qpl": 2, "path": bits.BITS_PATH_LEARNED}),
                   (lrefs, {"block": 1024, "qpl": 4, "path": bits.BITS_PATH_LEARNED}),
                   (lrefs, {"block": 256, "qpl": 1, "depth": 13, "path": bits.BITS_PATH_PLAIN})):
        plan = bits.bits_batch_create(rr, qd, launch=lp)
        for rep in range(3):
            tot = bits.bits_batch_run(plan)
            got = down(tot).reshape(len(Q), len(R))
            assert np.array_equal(got, exp), (lp, rep)
            # eager work between replays
            bits.bits_count(rr[0], qd[0][0], qd[0][1])
            torch.cuda.synchronize()
        bits.bits_batch_destroy(plan)
    # the learned path needs every reference learned
    with pytest.raises(bits.BitsError):
        bits.bits_batch_create(refs, qd, launch={"path": bits.BITS_PATH_LEARNED})
    assert bits.bits_get_status(lrefs[0]) == 0


def test_batch_autotuner():
    """bits_autotune_batch times every candidate shape of the batch plan; the
    shape it returns gives the oracle's pair totals, on both paths."""
    note("case: batch autotuner")
    lengths, Q, R = datagen.w3_sets(seed=4, n_q=4, n_r=5, q_range=(100, 20_000), r_range=(1000, 60_000))
    qd = [bits.bits_project(lengths, up(S.chrom), up(S.start), up(S.end)) for S in Q]
    rd = [bits.bits_project(lengths, up(S.chrom), up(S.start), up(S.end)) for S in R]
    qo = [oracle.project(lengths, S.chrom, S.start, S.end) for S in Q]
    ro = [oracle.project(lengths, S.chrom, S.start, S.end) for S in R]
    exp = np.array([[oracle.counter(qs, qe, rs, re_)[1] for rs, re_ in ro] for qs, qe in qo], np.uint64)
    lrefs = bits.bits_sort_refs(rd, learned=True, train={"epochs": 10})
    for path in (bits.BITS_PATH_PLAIN, bits.BITS_PATH_LEARNED):
        best, ms = bits.bits_autotune_batch(lrefs, qd, path=path)
        assert ms > 0 and best.path == path and best.block in (256, 512, 1024) and best.qpl in (1, 2, 4)
        plan = bits.bits_batch_create(lrefs, qd, launch=best.as_dict())
        assert np.array_equal(down(bits.bits_batch_run(plan)).reshape(len(Q), len(R)), exp), best.as_dict()
        bits.bits_batch_destroy(plan)


def test_learned_gradient_matches_oracle():
    note("case: leaf gradient")
    r = np.random.default_rng(12)
    for m in (1, 100, 2048):
        p = r.normal(0, 1, 49).astype(np.float32)
        u = r.uniform(0, 1, m).astype(np.float32)
        t = np.sort(r.uniform(0, 1, m)).astype(np.float32)
        g, loss = bits.bits_rmi_leaf_grad(torch.from_numpy(u).to(DEV), torch.from_numpy(t).to(DEV),
                                          torch.from_numpy(p).to(DEV))
        lo, go = oracle.rmi_loss_grad(p, u, t)
        g = down(g).astype(np.float64)
        assert np.max(np.abs(g - go)) <= 1e-3 * np.max(np.abs(go)) + 1e-6, (m, g, go)
        assert abs(float(down(loss)[0]) - lo) <= 1e-4 * max(1.0, lo)


def test_learned_index_metadata():
    note("case: learned metadata")
    lengths, _, B = datagen.w1_sets(seed=4, n_a=1, n_b=400_000)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 100})
    raw = down(ref.rmi_bytes())
    for a, keys in enumerate((np.sort(ob_s), np.sort(ob_e))):
        base = a * bits.RMI_MODEL_BYTES
        hdr = raw[base:base + bits.RMI_HEADER_BYTES]
        fit_a, fit_b = np.frombuffer(hdr[8:24].tobytes(), np.float64)
        oa, ob = oracle.linear_fit(keys)
        assert abs(fit_a - oa) <= 1e-9 * abs(oa) and abs(fit_b - ob) <= 1e-6 * max(1.0, abs(ob))
        leaves = raw[base + bits.RMI_HEADER_BYTES: base + bits.RMI_MODEL_BYTES].reshape(4096, 128)
        u32 = leaves.copy().view(np.uint32)          # 32 words per leaf
        kmin, kmax, rlo, cnt = u32[:, 0], u32[:, 1], u32[:, 4].astype(np.int64), u32[:, 5].astype(np.int64)
        # leaves tile the rank range in order
        assert rlo[0] == 0 and rlo[-1] + cnt[-1] == len(keys)
        assert np.all(rlo[1:] == rlo[:-1] + cnt[:-1])
        nz = cnt > 0
        assert np.array_equal(kmin[nz], keys[rlo[nz]])
        assert np.array_equal(kmax[nz], keys[rlo[nz] + cnt[nz] - 1])
        assert np.all(kmin[~nz] == 0xFFFFFFFF)
        # kinv = 1 / max(1, kmax - kmin) in fp32
        kinv = u32[nz, 8].view(np.float32)
        span = np.maximum(kmax[nz].astype(np.int64) - kmin[nz], 1).astype(np.float32)
        assert np.array_equal(kinv, (np.float32(1.0) / span).astype(np.float32))
    info = bits.bits_rmi_info(ref)
    assert info["mean_window"] >= 1 and info["max_window"] >= 1


def test_learned_windows_hold_every_key():
    """The query path's window (bits_rmi_window runs the searches' own device
    code) must contain the lower-bound rank of every key of the array: this
    is what the per-leaf error windows promise, independently of the
    verification that keeps the searches exact."""
    note("case: learned windows")
    for seed, nb in ((4, 300_000), (5, 70_001)):
        lengths, _, B = datagen.w1_sets(seed=seed, n_a=1, n_b=nb)
        b_s, b_e, ob_s, ob_e = project_both(lengths, B)
        ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 50})
        for which, keys in ((0, np.sort(ob_s)), (1, np.sort(ob_e))):
            lo, hi = bits.bits_rmi_window(ref, which, up(keys))
            lo, hi = down(lo).astype(np.int64), down(hi).astype(np.int64)
            rank = np.searchsorted(keys, keys, side="left")
            bad = np.flatnonzero((rank < lo) | (rank > hi))
            assert bad.size == 0, (which, bad[:5], rank[bad[:5]], lo[bad[:5]], hi[bad[:5]])


def test_line_heads():
    """Line heads: the first key of every 128-byte line of each sorted array,
    then at least 32 entries of +inf up to whole lines."""
    note("case: line heads")
    for nb in (1, 31, 32, 33, 1000, 70_001):
        r = np.random.default_rng(nb)
        b_s = r.integers(0, 10**7, nb).astype(np.uint32)
        b_e = b_s + r.integers(0, 500, nb).astype(np.uint32)
        ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": 0})
        H = down(ref.heads())
        hl, m = ref.heads_len(), (nb + 31) // 32
        assert hl % 32 == 0 and hl - m >= 32
        for a, keys in enumerate((np.sort(b_s), np.sort(b_e))):
            assert np.array_equal(H[a, :m], keys[::32]), nb
            assert np.all(H[a, m:] == 0xFFFFFFFF), nb


def test_monte_carlo_grid_shapes():
    """The Monte-Carlo kernel splits its tiles over 8 workgroup groups (one
    per XCD) when the grid has >= 8 workgroups and runs one group otherwise;
    totals must not depend on either, nor on uneven groups."""
    note("case: MC grid shapes")
    lengths, A, B = datagen.w2_sets(seed=3, n_a=20_000, n_b=100_000)
    a_s, a_e, oa_s, oa_e = project_both(lengths, A)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    exp = oracle.mc_totals(np.sort(ob_s), np.sort(ob_e), prep, 11, 5, 17, threads=8)
    obs = oracle.counter(oa_s, oa_e, ob_s, ob_e)[1]
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 20})
    for grid in (1, 3, 8, 13, 64):
        for path in (bits.BITS_PATH_PLAIN, bits.BITS_PATH_LEARNED):
            lp = {"grid": grid, "path": path, "block": 256, "qpl": 1}
            note("  launch %s" % lp)
            mc = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, seed=11, s0=5, s1=17, launch=lp)
            assert np.array_equal(down(mc.totals), exp), lp
            assert int(down(mc.observed)[0]) == obs, lp
    assert bits.bits_get_status(ref) == 0


@pytest.mark.parametrize("b2", [0.0, 1.0])
def test_broken_model_stays_exact(b2):
    """Overwrite every leaf model with a constant (weights 0, b2 = 0 or 1,
    error bounds 0: every key is predicted at its leaf's first or last rank)
    in the caller-owned block.  Counts and Monte-Carlo totals must stay exact
    through the fallbacks (windowed path: verification -> bisection of the
    leaf; Monte-Carlo: head window miss -> bisection of the leaf's heads)."""
    note("case: broken model b2=%g" % b2)
    lengths, A, B = datagen.w2_sets(seed=5, n_a=4000, n_b=4_000_000)
    a_s, a_e, oa_s, oa_e = project_both(lengths, A)
    b_s, b_e, ob_s, ob_e = project_both(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 10})
    raw = ref.rmi_bytes()
    for a in range(2):
        base = a * bits.RMI_MODEL_BYTES + bits.RMI_HEADER_BYTES
        words = raw[base:base + 4096 * bits.RMI_LEAF_BYTES].view(torch.int32).view(4096, 32)
        for w in (2, 3, 6, 7, 10, 11, 14, 15):           # binary16 w1 of units 0..15
            words[:, w] = 0
        words[:, 16:32] = 0                              # binary16 b1 and w2
        words[:, 9] = int(np.float32(b2).view(np.int32))  # b2
        words[:, 12] = 0                                 # error bounds
    torch.cuda.synchronize()
    fb0 = bits.bits_rmi_info(ref)["fallbacks"]
    exp_c, exp_t = oracle.counter(oa_s, oa_e, ob_s, ob_e, threads=8)
    c, t = bits.bits_count_per_query(ref, a_s, a_e, launch={"path": bits.BITS_PATH_LEARNED})
    assert np.array_equal(down(c), exp_c) and int(down(t)[0]) == exp_t
    prep = oracle.mc_prepare(lengths, oa_s, oa_e)
    exp = oracle.mc_totals(np.sort(ob_s), np.sort(ob_e), prep, 7, 0, 6, threads=8)
    mc = bits.bits_mc_pvalue(ref, a_s, a_e, lengths, seed=7, s0=0, s1=6, launch={"path": bits.BITS_PATH_LEARNED})
    assert np.array_equal(down(mc.totals), exp)
    assert int(down(mc.observed)[0]) == exp_t
    assert bits.bits_rmi_info(ref)["fallbacks"] > fb0
    assert bits.bits_get_status(ref) == 0


def _mc_expected_with_left_out(lengths, a_s, a_e, ok, b_s, b_e, seed, s0, s1):
    """Per-shuffle totals by the oracle when the queries with ok = False are
    left out: placements of all queries from the oracle's stream (counter
    s * na + i; left-out queries get a dummy table entry), then a plain count
    of the placed kept queries."""
    off, span, ln = oracle.mc_prepare(lengths, a_s[ok], a_e[ok])
    na = len(a_s)
    off_all, span_all, len_all = np.zeros(na, np.uint32), np.ones(na, np.uint32), np.ones(na, np.uint32)
    off_all[ok], span_all[ok], len_all[ok] = off, span, ln
    out = []
    for s in range(s0, s1):
        st = oracle.mc_placements(seed, s, off_all, span_all)[ok]
        out.append(oracle.counter(st, st + len_all[ok] - np.uint32(1), b_s, b_e)[1])
    return np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_monte_carlo_sorted_items(block):
    """The learned Monte-Carlo kernel sorts each item's placements (tile of
    block/8 queries x up to 64 shuffles) before searching.  Shuffle counts that
    leave partial chunks and idle lanes (1, 7, 70), tiles that straddle
    chromosomes, and a run of queries outside their chromosome long enough to
    fill whole tiles: totals must still equal the oracle's."""
    note("case: MC sorted items block=%d" % block)
    r = np.random.default_rng(block)
    lengths = np.array([300_000, 50_000, 1_000, 200_000, 7_000], np.uint32)
    off = oracle.genome_offsets(lengths).astype(np.int64)
    na, nb = 3_000, 20_000

    def placed(n, maxlen):
        c = r.integers(0, len(lengths), size=n)
        L = np.minimum(r.integers(1, maxlen + 1, size=n), lengths[c].astype(np.int64))
        s = r.integers(0, lengths[c].astype(np.int64) - L + 1)
        return (off[c] + s).astype(np.uint32), (off[c] + s + L - 1).astype(np.uint32)
    a_s, a_e = placed(na, 400)
    b_s, b_e = placed(nb, 300)
    # queries 100..399 cross the end of chromosome 1 (left out, flagged)
    a_s[100:400] = np.uint32(off[2] - 10)
    a_e[100:400] = np.uint32(off[2] + 10)
    ok = np.ones(na, bool)
    ok[100:400] = False
    ref = bits.bits_sort_ref(up(b_s), up(b_e), learned=True, train={"epochs": 20})
    for s0, s1 in ((0, 1), (5, 12), (3, 73)):
        exp = _mc_expected_with_left_out(lengths, a_s, a_e, ok, b_s, b_e, 9, s0, s1)
        mc = bits.bits_mc_pvalue(ref, up(a_s), up(a_e), lengths, 9, s0, s1,
                                 launch={"path": bits.BITS_PATH_LEARNED, "block": block, "qpl": 1})
        assert np.array_equal(down(mc.totals), exp), (s0, s1)
        assert int(down(mc.observed)[0]) == oracle.counter(a_s[ok], a_e[ok], b_s, b_e)[1]
    assert bits.bits_get_status(ref) & bits.BITS_FLAG_CHROM
