"""Benchmark of the BITS hot path on one MI355X.

Workload (learned index at scale): B = 50,000,000 intervals (half uniform,
half around 20,000 Gaussian clusters, log-normal lengths median 200 bp) and
A = 50,000,000 uniform intervals on a 24-chromosome synthetic genome, plus a
Monte-Carlo run of 1,000 shuffles of the first 1,000,000 intervals of A.

One step is one pass of the whole hot path on inputs already resident in
HBM (chromosome-local coordinates):
  projection of A and B -> on-device radix sort of B_S and B_E, Eytzinger top
  trees, learned CDF index trained on the device -> per-query counts of all
  of A through the learned index -> 1,000 Monte-Carlo shuffles binned by
  genome region and counted in LDS (one pass of 1,000 shuffles), with the
  observed total and tail counts.
value = A-intervals counted per second over the step (50M queries + 1,000 x
1M shuffled queries per step).  Printed as one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

N_B = 50_000_000
N_A = 50_000_000
N_MC = 1_000_000
N_SHUF = 1_000
N_ENUM = 10_000_000   # A-intervals enumerated against the full B (outside the timed region)
MC_SEED = 7
MC_BATCH = 1000       # shuffles per pass of the binned Monte-Carlo path (8.2 GB workspace at 1e6 queries)
# Algorithmic HBM bytes per placement (one shuffled A-interval) of the binned Monte-Carlo kernels:
#   k_bin_place   reads the query's 8-byte {index, length} entry, writes its 8-byte {start, end} record;
#   k_bin_search  reads the record back (8 bytes); each region also stages its slices of B_S and B_E
#                 once per pass (4 bytes per key of both arrays, added per pass below).
BYTES_PER_PLACEMENT = {"k_bin_place": 16.0, "k_bin_search": 8.0}
# The query-ordered learned path (compared outside the timed region): the search through the line
# heads reads exactly one 128-byte line of B_S and one of B_E per evaluation.
BYTES_PER_EVAL_LEARNED = 256.0
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_bin_w4.json")
# launch shapes the autotuner picked on MI355X for this workload (used with --no-autotune)
RECORDED_LEARNED = {"block": 512, "qpl": 1, "depth": 0, "grid": 0, "path": 2}
RECORDED_PLAIN = {"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 1}
RECORDED_MC = {"block": 1024, "qpl": 1, "depth": 0, "grid": 0, "path": 2}
KERNEL_SOURCES = ["paper_1208_3407_amd/csrc/binned.hip", "paper_1208_3407_amd/csrc/bits_internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, placements_per_launch):
    """HBM bytes per launch of a binned kernel from the committed counter
    summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or kernel not in t.get("bytes_per_placement", {}):
        return None
    return float(t["bytes_per_placement"][kernel]) * placements_per_launch


def tune_mc(bits, ref, a_s, a_e, lengths, ws):
    """Monte-Carlo launch shape of the learned path: workgroup size by timing 64 shuffles."""
    import torch
    best, pick = 1e30, None
    for blk in (512, 1024):
        lp = {"block": blk, "qpl": 1, "depth": 0, "grid": 0, "path": 2}
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            bits.bits_mc_pvalue(ref, a_s, a_e, lengths, MC_SEED, 0, 64, launch=lp, workspace=ws)
            e1.record()
            e1.synchronize()
            t = e0.elapsed_time(e1)
            if t < best:
                best, pick = t, lp
    log("mc launch: %s (%.2f ms per 64 shuffles)" % (pick, best))
    return pick


def autotune(bits, ref, a_s, a_e, path, cache_key):
    cache_path = os.path.join(os.path.expanduser("~"), ".cache", "paper_1208_3407_amd", "autotune.json")
    try:
        with open(cache_path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    if cache_key in cache:
        return cache[cache_key]
    best, ms = bits.bits_autotune_count(ref, a_s, a_e, path)
    d = best.as_dict()
    cache[cache_key] = d
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    log("autotune path %d: %s (%.2f ms)" % (path, d, ms))
    return d


def cpu_baseline(lengths, A, B, threads):
    """The CPU oracle on a bounded sample of the same workload."""
    import oracle

    t0 = time.perf_counter()
    a_s, a_e = oracle.project(lengths, A.chrom[:8 * N_MC], A.start[:8 * N_MC], A.end[:8 * N_MC])
    b_s, b_e = oracle.project(lengths, B.chrom, B.start, B.end)
    sbs, sbe = oracle.sort_u32(b_s), oracle.sort_u32(b_e)
    t_setup = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, _ = oracle.count_sorted(sbs, sbe, a_s, a_e, threads=threads)
    t_count = time.perf_counter() - t1
    prep = oracle.mc_prepare(lengths, a_s[:N_MC], a_e[:N_MC])
    t2 = time.perf_counter()
    n_shuf = threads
    oracle.mc_totals(sbs, sbe, prep, MC_SEED, 0, n_shuf, threads=threads)
    t_mc = time.perf_counter() - t2
    n_evals = len(a_s) + n_shuf * N_MC
    # the same oracle on one thread (sequential BITS), on a smaller sample: 1e6 queries + 1 shuffle
    t3 = time.perf_counter()
    oracle.count_sorted(sbs, sbe, a_s[:N_MC], a_e[:N_MC], threads=1)
    oracle.mc_totals(sbs, sbe, prep, MC_SEED, 0, 1, threads=1)
    t_one = time.perf_counter() - t3
    return {
        "value": n_evals / (t_count + t_mc),
        "unit": "A-intervals/s",
        "cores": threads,
        "kind": "oracle",
        "value_1thread": 2 * N_MC / t_one,
        "sample_1thread": "the same oracle on 1 thread: counts of the first %d A-intervals and 1 Monte-Carlo "
                          "shuffle of the %d MC queries (%.2f s)" % (N_MC, N_MC, t_one),
        "sample": "oracle (C, -O2) on the same workload: projection + qsort of the full 5e7-interval B "
                  "(%.1f s, not in value), per-query counts of the first %d A-intervals on %d threads "
                  "(%.2f s) and %d Monte-Carlo shuffles of the 1e6 MC queries on %d threads (%.2f s); "
                  "value = %d evaluations / counting time" % (t_setup, len(a_s), threads, t_count, n_shuf, threads,
                                                              t_mc, n_evals),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the recorded best launch shapes instead of timing candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with a plain 1 GiB device copy (HBM byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (one process on one GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1208_3407_amd import bits, datagen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    t0 = time.time()
    lengths, A, B = datagen.w4_sets(seed=1, n_a=N_A, n_b=N_B)
    log("data %.1f s" % (time.time() - t0))

    def up(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    dA = [up(A.chrom), up(A.start), up(A.end)]
    dB = [up(B.chrom), up(B.start), up(B.end)]
    ref = bits.bits_ref_init(N_B, 13, learned=True)
    ws = bits._scratch(bits.bits_sort_ref_workspace(N_B), dev)
    mc_ws = bits._scratch(bits.bits_mc_workspace(N_MC), dev)
    bin_ws = bits._scratch(bits.bits_mc_binned_workspace(N_MC, N_B, lengths, MC_BATCH), dev)
    counts = torch.empty(N_A, dtype=torch.uint32, device=dev)
    total = torch.empty(1, dtype=torch.uint64, device=dev)
    mc_out = bits.MCResult(torch.empty(N_SHUF, dtype=torch.uint64, device=dev),
                           torch.empty(1, dtype=torch.uint64, device=dev),
                           torch.empty(1, dtype=torch.uint64, device=dev),
                           torch.empty(1, dtype=torch.uint64, device=dev))
    train = {"epochs": args.epochs}

    # launch shapes from the autotuner (outside the timed region)
    a_s, a_e = bits.bits_project(lengths, *dA)
    b_s, b_e = bits.bits_project(lengths, *dB)
    bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws)
    tag = "%s|nA=%d|nB=%d" % (torch.cuda.get_device_properties(0).gcnArchName, N_A, N_B)
    if args.no_autotune:
        lp_learned, lp_plain, lp_mc = dict(RECORDED_LEARNED), dict(RECORDED_PLAIN), dict(RECORDED_MC)
    else:
        lp_learned = autotune(bits, ref, a_s, a_e, bits.BITS_PATH_LEARNED, "learned|" + tag)
        lp_plain = autotune(bits, ref, a_s, a_e, bits.BITS_PATH_PLAIN, "plain|" + tag)
        lp_mc = tune_mc(bits, ref, a_s[:N_MC], a_e[:N_MC], lengths, mc_ws)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    mc_ms = []

    def step(record):
        a_s, a_e = bits.bits_project(lengths, *dA)
        b_s, b_e = bits.bits_project(lengths, *dB)
        if record:
            ev[0].record()
        bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws)
        if record:
            ev[1].record()
        bits.bits_count_per_query(ref, a_s, a_e, launch=lp_learned, counts=counts, total=total)
        if record:
            ev[2].record()
        bits.bits_mc_binned(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF, batch=MC_BATCH,
                            launch=lp_mc, workspace=bin_ws, out=mc_out)
        if record:
            ev[3].record()
        return a_s, a_e

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    phase = {"setup_ms": [], "count_ms": [], "mc_ms": []}
    stages = {"place": [], "search": [], "reduce": []}
    bits.bits_mc_binned_timing(True)    # HIP events around the binned kernels, on the stream they run on
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        ev[3].synchronize()
        phase["setup_ms"].append(ev[0].elapsed_time(ev[1]))
        phase["count_ms"].append(ev[1].elapsed_time(ev[2]))
        phase["mc_ms"].append(ev[2].elapsed_time(ev[3]))
        for k, v in bits.bits_mc_binned_stage_ms().items():
            stages[k].append(v)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    bits.bits_mc_binned_timing(False)
    ms_per_step = t_total * 1e3 / args.steps
    evals = N_A + N_SHUF * N_MC
    value = evals / (ms_per_step / 1e3)
    status = bits.bits_get_status(ref)
    learned_total = int(total.cpu().numpy()[0])
    mc_totals = mc_out.totals.cpu().numpy()

    # plain binary-search path on the same reference, outside the timed region
    a_s, a_e = bits.bits_project(lengths, *dA)
    def timed(fn, reps=3):
        best = 1e30
        for _ in range(reps):
            ev[4].record()
            fn()
            ev[5].record()
            ev[5].synchronize()
            best = min(best, ev[4].elapsed_time(ev[5]))
        return best
    t_plain = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch=lp_plain, counts=counts, total=total))
    plain_total = int(total.cpu().numpy()[0])
    t_learned = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch=lp_learned, counts=counts,
                                                        total=total))
    mc_plain = bits.MCResult(torch.empty(N_SHUF, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev))
    t_mc_plain = timed(lambda: bits.bits_mc_pvalue(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF,
                                                   launch=lp_plain, workspace=mc_ws, out=mc_plain), reps=1)
    mc_learned = bits.MCResult(torch.empty(N_SHUF, dtype=torch.uint64, device=dev),
                               torch.empty(1, dtype=torch.uint64, device=dev),
                               torch.empty(1, dtype=torch.uint64, device=dev),
                               torch.empty(1, dtype=torch.uint64, device=dev))
    t_mc_learned = timed(lambda: bits.bits_mc_pvalue(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF,
                                                     launch=lp_mc, workspace=mc_ws, out=mc_learned), reps=2)
    agree = (plain_total == learned_total) and np.array_equal(mc_plain.totals.cpu().numpy(), mc_totals)
    binned_agree = (np.array_equal(mc_learned.totals.cpu().numpy(), mc_totals)
                    and int(mc_learned.observed.item()) == int(mc_out.observed.item()))
    info = bits.bits_rmi_info(ref)

    # enumeration (sub-problem 4) of the first N_ENUM A-intervals against B, outside the timed region
    b_s, b_e = bits.bits_project(lengths, *dB)
    ea_s, ea_e = a_s[:N_ENUM], a_e[:N_ENUM]
    t_index = timed(lambda: bits.bits_enum_index_build(b_s, b_e), reps=2)
    index = bits.bits_enum_index_build(b_s, b_e)
    t_ecount = timed(lambda: bits.bits_enum_counts(ref, ea_s, ea_e, launch=lp_learned))
    e_counts, e_first, offsets = bits.bits_enum_counts(ref, ea_s, ea_e, launch=lp_learned)
    n_pairs = int(offsets[-1].item())
    e_status = torch.zeros(1, dtype=torch.uint32, device=dev)
    pairs = {}

    def run_enum():
        pairs["ab"] = bits.bits_enumerate(index, ea_s, ea_e, e_counts, offsets, first=e_first, max_pairs=n_pairs,
                                          status=e_status)
    t_enum = timed(run_enum)
    pa, pb = pairs["ab"]
    pick = torch.randint(0, max(n_pairs, 1), (min(n_pairs, 100_000),), device=dev)

    def gather_u32(t, idx):   # uint32 values at idx, as int64 (torch indexes int32, not uint32)
        return t.view(torch.int32)[idx].long() & 0xFFFFFFFF
    ia, ib = gather_u32(pa, pick), gather_u32(pb, pick)
    enum_ok = bool(int(e_status.item()) == 0 and
                   bool(((gather_u32(ea_s, ia) <= gather_u32(b_e, ib)) &
                         (gather_u32(ea_e, ia) >= gather_u32(b_s, ib))).all().item()))
    del pairs, pa, pb, index
    enumeration = {"a_intervals": N_ENUM, "pairs": n_pairs, "index_build_ms": t_index,
                   "counts_first_offsets_ms": t_ecount, "enumerate_ms": t_enum,
                   "pairs_per_s": n_pairs / (t_enum / 1e3),
                   "a_intervals_per_s": N_ENUM / ((t_ecount + t_enum) / 1e3),
                   "sampled_pairs_valid": enum_ok}

    # significance summary of the timed Monte-Carlo run (Sec. 3.2, Sec. 3.3) and the decision sub-problem
    m_lo, m_hi = bits.bits_mc_median(mc_out.totals)
    m_lo, m_hi = int(m_lo.item()), int(m_hi.item())
    obs, n_ge, n_le = int(mc_out.observed.item()), int(mc_out.n_ge.item()), int(mc_out.n_le.item())
    significance = {"observed": obs, "median": (m_lo + m_hi) / 2, "enrichment_log2": bits.bits_enrichment(obs, m_lo, m_hi),
                    "n_ge": n_ge, "n_le": n_le, "p_upper": bits.bits_pvalue(n_ge, N_SHUF),
                    "p_lower": bits.bits_pvalue_lower(n_le, N_SHUF),
                    "p_two_sided": bits.bits_pvalue_two_sided(n_ge, n_le, N_SHUF)}
    t_decide = timed(lambda: bits.bits_decide(ref, a_s, a_e, launch=lp_learned))
    significance["decide_ms"] = t_decide
    significance["decide_found"] = int(bits.bits_decide(ref, a_s, a_e, launch=lp_learned)[0].item())

    # the paper's Monte-Carlo orientation (B randomised and re-sorted every round) against this
    # library's fixed-index loop on the same draws: 1e6 x 1e6 intervals, 100 rounds
    n_po, r_po = 1_000_000, 100
    pa_s, pa_e, pb_s, pb_e = a_s[:n_po], a_e[:n_po], b_s[:n_po], b_e[:n_po]
    ref_po = bits.bits_sort_ref(pa_s, pa_e, learned=True, train=train)
    po = {}
    t_resort = timed(lambda: po.__setitem__("r", bits.bits_mc_resort(pa_s, pa_e, pb_s, pb_e, lengths, MC_SEED, 0,
                                                                     r_po)), reps=2)
    t_fixed = timed(lambda: po.__setitem__("f", bits.bits_mc_pvalue(ref_po, pb_s, pb_e, lengths, MC_SEED, 0, r_po)),
                    reps=2)
    paper_orientation = {"size": n_po, "rounds": r_po, "resort_ms_per_round": t_resort / r_po,
                         "fixed_index_ms_per_round": t_fixed / r_po,
                         "totals_equal": bool(torch.equal(po["r"].totals, po["f"].totals))}
    del ref_po, po

    # measured achievable HBM rate: a plain 1 GiB device copy (1 GiB read + 1 GiB written)
    cx = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cy = torch.empty_like(cx)
    t_copy = timed(lambda: cy.copy_(cx), reps=5)
    copy_gbs = 2.0 * (1 << 30) / (t_copy / 1e3) / 1e9
    del cx, cy
    mc_avg = float(np.mean(phase["mc_ms"]))
    stage_ms = {k: float(np.mean(v)) for k, v in stages.items()}
    # dominant binned kernel of the step and its algorithmic bytes per launch (one pass of MC_BATCH
    # shuffles; the step runs N_SHUF / MC_BATCH passes)
    passes = (N_SHUF + MC_BATCH - 1) // MC_BATCH
    placements = N_SHUF * N_MC // passes
    dom = "k_bin_place" if stage_ms["place"] >= stage_ms["search"] else "k_bin_search"
    dom_ms = (stage_ms["place"] if dom == "k_bin_place" else stage_ms["search"]) / passes
    dom_bytes = BYTES_PER_PLACEMENT[dom] * placements + (8.0 * N_B if dom == "k_bin_search" else 0.0)
    achieved = dom_bytes / (dom_ms / 1e3) / 1e9
    traffic = load_traffic(dom, placements)
    learned_achieved = BYTES_PER_EVAL_LEARNED * N_SHUF * N_MC / (t_mc_learned / 1e3) / 1e9
    result = {
        "metric": "A-intervals counted/s (learned vs binary-search index); MC shuffles/s",
        "value": value,
        "unit": "A-intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "learned index at scale: B=5e7 clustered, A=5e7 uniform, MC 1000 x 1e6 "
                               "(24-chromosome genome)",
                   "n_b": N_B, "n_a": N_A, "mc_queries": N_MC, "mc_shuffles": N_SHUF, "train_epochs": args.epochs,
                   "launch_learned": lp_learned, "launch_plain": lp_plain,
                   "mc": {"path": "binned by genome region", "batch": MC_BATCH, "observed_launch": lp_mc}},
        "phases_ms": {k: float(np.mean(v)) for k, v in phase.items()},
        "mc_stage_ms": stage_ms,
        "count_learned_aps": N_A / (t_learned / 1e3),
        "count_plain_aps": N_A / (t_plain / 1e3),
        "learned_speedup": t_plain / t_learned,
        "mc_shuffles_per_s": N_SHUF / (mc_avg / 1e3),
        "mc_shuffles_per_s_learned": N_SHUF / (t_mc_learned / 1e3),
        "mc_shuffles_per_s_plain": N_SHUF / (t_mc_plain / 1e3),
        "learned_equals_plain": bool(agree),
        "binned_equals_learned": bool(binned_agree),
        "rmi": info,
        "enumeration": enumeration,
        "significance": significance,
        "paper_orientation": paper_orientation,
        "status": status,
        "roofline": {"bound": "hbm", "kernel": dom + " (Monte-Carlo shuffles binned by genome region)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "peak_measured_copy": copy_gbs, "frac_of_measured": achieved / copy_gbs,
                     "traffic": traffic, "bytes_per_placement_model": BYTES_PER_PLACEMENT[dom],
                     "placements_per_launch": placements, "launch_ms": dom_ms,
                     "limiter": ("LDS and VALU issue (LDS busy and bank-conflict share in "
                                 "profiles/k_bin_w4_lds_counters.md)" if dom == "k_bin_search" else
                                 "partly written lines of the scattered records (profiles/k_bin_w4_hbm_counters.md)")},
        "roofline_learned_mc": {"bound": "hbm", "kernel": "k_mc_sorted (query-ordered learned-index Monte-Carlo, "
                                "outside the timed region)", "achieved": learned_achieved, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": learned_achieved / HBM_PEAK_GBS,
                                "bytes_per_eval_model": BYTES_PER_EVAL_LEARNED, "call_ms": t_mc_learned},
    }
    if not args.no_cpu_baseline:
        threads = max(1, min(16, os.cpu_count() or 1))
        result["cpu_baseline"] = cpu_baseline(lengths, A, B, threads)
    print(json.dumps(result), flush=True)
    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")


if __name__ == "__main__":
    main()
