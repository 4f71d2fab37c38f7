"""What the trained network gains, on the learned-index workload (B = 5e7
clustered, A = 5e7 uniform): the same counting kernel with (i) the trained
leaf models and (ii) the same models before training (knots at the sampled
quantiles, 0 epochs), against (iii) the index without a model (LDS top tree,
line-head tier, one line) and (iv) plain bisection.  All four give the
oracle's counts; training narrows the error windows the searches use; the
times are printed for the record (bench.py reports them in its `gain`
block)."""
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

DEV = torch.device("cuda", 0)


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def up(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def timed(fn, reps=3):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(reps):
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def test_trained_model_gain_w4():
    note("case: learned-index gain, W4 5e7 x 5e7")
    lengths, A, B = datagen.w4_sets()
    a_s, a_e = bits.bits_project(lengths, up(A.chrom), up(A.start), up(A.end))
    b_s, b_e = bits.bits_project(lengths, up(B.chrom), up(B.start), up(B.end))
    trained = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 80})
    init = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 0})
    # the oracle's counts of a sample, and its total
    oa_s, oa_e = oracle.project(lengths, A.chrom, A.start, A.end)
    ob_s, ob_e = oracle.project(lengths, B.chrom, B.start, B.end)
    del A, B
    sbs, sbe = oracle.sort_u32(ob_s), oracle.sort_u32(ob_e)
    idx = np.random.default_rng(5).integers(0, len(oa_s), 100_000)
    exp_sample, _ = oracle.count_sorted(sbs, sbe, oa_s[idx], oa_e[idx], threads=16)
    exp_total = oracle.count_sorted(sbs, sbe, oa_s, oa_e, threads=16, per_query=False)[1]
    counts = torch.empty(len(oa_s), dtype=torch.uint32, device=DEV)
    total = torch.empty(1, dtype=torch.uint64, device=DEV)
    paths = [("trained", trained, {"path": 2, "block": 1024, "qpl": 1}),
             ("init_only", init, {"path": 2, "block": 1024, "qpl": 1}),
             ("tiered_no_model", trained, {"path": 3, "block": 1024, "qpl": 1, "depth": 13}),
             ("plain", trained, {"path": 1, "block": 256, "qpl": 1, "depth": 13})]
    ref_counts, times, info = None, {}, {}
    for name, r, lp in paths:
        f0 = bits.bits_rmi_info(r)["fallbacks"]
        bits.bits_count_per_query(r, a_s, a_e, launch=lp, counts=counts, total=total)
        got = counts.cpu().numpy()
        assert np.array_equal(got[idx], exp_sample), name
        assert int(total.item()) == exp_total, name
        if ref_counts is None:
            ref_counts = counts.clone()
        else:
            assert torch.equal(counts, ref_counts), name
        st = bits.bits_rmi_info(r)
        info[name] = (st["mean_window"], st["max_window"], (st["fallbacks"] - f0) / (2.0 * len(oa_s)))
        times[name] = timed(lambda: bits.bits_count_per_query(r, a_s, a_e, launch=lp, counts=counts, total=total))
        note("  %-16s %7.2f ms  %.3g A-intervals/s  window mean %.1f max %d  fallbacks/search %.2g" % (
            name, times[name], len(oa_s) / (times[name] / 1e3), *info[name]))
    # training narrows the windows the windowed search has to cover
    assert info["trained"][0] < info["init_only"][0]
    note("  model over no-model index: %.2fx; over plain: %.2fx; trained over init-only: %.2fx" % (
        times["tiered_no_model"] / times["trained"], times["plain"] / times["trained"],
        times["init_only"] / times["trained"]))
    assert bits.bits_get_status(trained) == 0 and bits.bits_get_status(init) == 0
