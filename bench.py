"""Benchmark of the BITS hot path on one MI355X.

Workload (learned index at scale): B = 50,000,000 intervals (half uniform,
half around 20,000 Gaussian clusters, log-normal lengths median 200 bp) and
A = 50,000,000 uniform intervals on a 24-chromosome synthetic genome, plus a
Monte-Carlo run of 1,000 shuffles of the first 1,000,000 intervals of A.

One step is one pass of the whole hot path on inputs already resident in
HBM (chromosome-local coordinates):
  projection of A and B -> on-device radix sort of B_S and B_E, Eytzinger top
  trees, line heads, learned CDF index trained on the device -> per-query
  counts of all of A through the learned index -> 1,000 Monte-Carlo shuffles
  binned by genome region and counted in LDS (one pass of 1,000 shuffles),
  with the observed total and tail counts.
value = A-intervals counted per second over the step (50M queries + 1,000 x
1M shuffled queries per step).  Printed as one JSON line.

Outside the timed region the same run measures: the four counting paths on
the same reference (trained model, the model before training, the line-head
tier without a model, plain bisection), the query-ordered Monte-Carlo paths,
the other workloads (10k x 10k on one chromosome; 1e7 x 1e7; 1e5-query
Monte-Carlo with 10,000 shuffles against 1e6; the 32 x 64 uneven batch), a
1 GiB device copy as the measured HBM rate, and the CPU oracle on a bounded
sample (cpu_baseline).
"""
import argparse
import hashlib
import json
import math
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
TRAIN_EPOCHS = 80
TRAIN_POINTS = 128    # training points per leaf (the windows are as tight as with 256-2048; see the sweep)
# Algorithmic HBM bytes per placement (one shuffled A-interval) of the binned Monte-Carlo kernels:
#   k_bin_place   reads the query's 8-byte {index, length} entry, writes its 8-byte {start, end} record;
#   k_bin_search  reads the record back (8 bytes); each region also stages its slices of B_S and B_E
#                 once per pass (4 bytes per key of both arrays, added per pass below).
BYTES_PER_PLACEMENT = {"k_bin_place": 16.0, "k_bin_search": 8.0}
# The query-ordered learned path (compared outside the timed region): the search through the line
# heads reads exactly one 128-byte line of B_S and one of B_E per evaluation.
BYTES_PER_EVAL_LEARNED = 256.0
HBM_PEAK_GBS = 8000.0
# LDS: 128 bytes per clock per CU, 256 CUs, 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
# VALU: four 16-lane SIMDs per CU retire one wave64 instruction per clock between them
VALU_PEAK_G = 256 * 2.4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_bin_w4.json")
# launch shapes the autotuner picked on MI355X for this workload (used with --no-autotune)
RECORDED_LEARNED = {"block": 512, "qpl": 1, "depth": 0, "grid": 0, "path": 2}
RECORDED_PLAIN = {"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 1}
RECORDED_TIERED = {"block": 256, "qpl": 1, "depth": 13, "grid": 0, "path": 3}
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


def library_info(bits):
    with open(bits.LIB_PATH, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return {"path": os.path.relpath(bits.LIB_PATH, ROOT), "sha256": sha, "version": bits.bits_version()}


def load_counters(kernel, placements_per_launch):
    """HBM bytes and LDS instructions per launch of a binned kernel from the committed
    counter summary, if it was taken on the current kernel source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None, None
    if t.get("kernel_hash") != kernel_hash():
        return None, None
    b = t.get("bytes_per_placement", {}).get(kernel)
    lds = t.get("lds_instructions_per_placement", {}).get(kernel)
    return (None if b is None else float(b) * placements_per_launch,
            None if lds is None else float(lds) * placements_per_launch)


def load_valu(kernel, placements_per_launch):
    """VALU wave-instructions per launch of a binned kernel from the committed counter
    summary, if it was taken on the current kernel source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    v = t.get("valu_instructions_per_placement", {}).get(kernel)
    return None if v is None else float(v) * placements_per_launch


def host_cpu():
    """The host's CPU model and the thread count the oracle may use: the process's
    CPU share (cgroup quota, else its affinity mask), as the host allots it."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
            if q != "max":
                quota = int(q) / int(period)
    except (OSError, ValueError):
        pass
    threads = aff if quota is None else max(1, min(aff, int(math.floor(quota))))
    return {"model": model, "os_cpu_count": os.cpu_count(), "affinity": aff, "cgroup_quota_cpus": quota,
            "threads": threads}


def cached_autotune(key, fn):
    cache_path = os.path.join(os.path.expanduser("~"), ".cache", "paper_1208_3407_amd", "autotune.json")
    try:
        with open(cache_path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    if key in cache:
        return cache[key]
    best, ms = fn()
    d = best.as_dict()
    cache[key] = d
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    except OSError:
        pass
    log("autotune %s: %s (%.2f ms)" % (key, d, ms))
    return d


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


def make_timer():
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=3):
        """Best of `reps` device times (ms) of fn on the current stream."""
        best = 1e30
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best
    return timed


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
        "sample": "oracle (C, gcc -O2) on the same workload: projection + qsort of the full 5e7-interval B "
                  "(%.1f s, not in value), per-query counts of the first %d A-intervals on %d threads "
                  "(%.2f s) and %d Monte-Carlo shuffles of the 1e6 MC queries on %d threads (%.2f s); "
                  "value = %d evaluations / counting time" % (t_setup, len(a_s), threads, t_count, n_shuf, threads,
                                                              t_mc, n_evals),
    }


def batch_model_bytes(na_list, nb_list):
    """Per-pair search bytes of the plain path's model: 8 bytes of query read per (query, reference)
    plus 2 x (h_mid + 1) lines of 128 bytes, h_mid = ceil(log_33(n / (2^13 * 32))) node levels below
    the LDS tree (0 when the reference's buckets are at most one node)."""
    total = 0.0
    for nb in nb_list:
        h = max(0, math.ceil(math.log(max(nb, 1) / (2 ** 13 * 32)) / math.log(33))) if nb > 2 ** 18 else 0
        total += sum(na_list) * (8.0 + 2 * (h + 1) * 128.0)
    return total


def other_configs(bits, dev, timed, train, which=("c0", "c1", "c2", "c3")):
    """The other workloads, each on its own data: small single-chromosome counts (c0), genome-scale
    counts (c1), the small-reference Monte-Carlo (c2) and the uneven batch of pairs (c3); `which`
    names the ones to run."""
    import torch

    from paper_1208_3407_amd import datagen

    def up(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)

    def proj(lengths, S):
        return bits.bits_project(lengths, up(S.chrom), up(S.start), up(S.end))

    out = {}
    if "c0" in which:
        out["c0"] = config_c0(bits, datagen, proj, timed, train)
    if "c1" in which:
        out["c1"] = config_c1(bits, datagen, proj, timed, train, dev)
    if "c2" in which:
        out["c2"] = config_c2(bits, datagen, proj, timed, train, dev)
    if "c3" in which:
        out["c3"] = config_c3(bits, datagen, proj, timed, train)
    return out


def config_c0(bits, datagen, proj, timed, train):
    """10k x 10k on one 10 Mbp chromosome: launch-latency bound."""
    lengths, A, B = datagen.w0_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    t_setup = timed(lambda: bits.bits_sort_ref(b_s, b_e, learned=True, train=train), reps=3)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train=train)
    c0 = {"workload": "10k x 10k on one 10 Mbp chromosome", "setup_ms": t_setup}
    for name, path in (("learned", 2), ("plain", 1), ("tiered", 3)):
        t = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch={"path": path}), reps=5)
        c0[name + "_ms"] = t
        c0[name + "_aps"] = len(A.start) / (t / 1e3)
    return c0


def config_c1(bits, datagen, proj, timed, train, dev):
    """1e7 x 1e7 on the 24-chromosome genome, each path at its autotuned launch."""
    import torch

    lengths, A, B = datagen.w1_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ws = bits._scratch(bits.bits_sort_ref_workspace(len(B.start)), dev)
    ref = bits.bits_ref_init(len(B.start), 13, learned=True)
    t_setup = timed(lambda: bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws), reps=3)
    c1 = {"workload": "1e7 x 1e7, 24 chromosomes", "setup_ms": t_setup}
    counts = torch.empty(len(A.start), dtype=torch.uint32, device=dev)
    total = torch.empty(1, dtype=torch.uint64, device=dev)
    totals = {}
    for name, path in (("learned", 2), ("plain", 1), ("tiered", 3)):
        lp = cached_autotune("c1|%s|%s" % (name, torch.cuda.get_device_properties(0).gcnArchName),
                             lambda: bits.bits_autotune_count(ref, a_s, a_e, path))
        t = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch=lp, counts=counts, total=total))
        totals[name] = int(total.item())
        c1[name + "_ms"] = t
        c1[name + "_aps"] = len(A.start) / (t / 1e3)
        c1[name + "_launch"] = lp
    c1["paths_equal"] = len(set(totals.values())) == 1
    return c1


def config_c2(bits, datagen, proj, timed, train, dev):
    """Monte-Carlo: 1e5 queries x 10,000 shuffles against 1e6, binned and query-ordered."""
    import torch

    lengths, A, B = datagen.w2_sets()
    a_s, a_e = proj(lengths, A)
    b_s, b_e = proj(lengths, B)
    ref = bits.bits_sort_ref(b_s, b_e, learned=True, train=train)
    N = 10_000
    bws = bits._scratch(bits.bits_mc_binned_workspace(len(A.start), len(B.start), lengths, MC_BATCH), dev)
    res = {}
    t_bin = timed(lambda: res.__setitem__("b", bits.bits_mc_binned(ref, a_s, a_e, lengths, MC_SEED, 0, N,
                                                                   batch=MC_BATCH, workspace=bws)), reps=2)
    t_q = timed(lambda: res.__setitem__("q", bits.bits_mc_pvalue(ref, a_s, a_e, lengths, MC_SEED, 0, N,
                                                                 launch=RECORDED_MC)), reps=1)
    return {"workload": "Monte-Carlo 1e5 queries x 10,000 shuffles against 1e6",
                 "binned_ms": t_bin, "binned_shuffles_per_s": N / (t_bin / 1e3),
                 "binned_aps": N * len(A.start) / (t_bin / 1e3),
                 "query_ordered_learned_ms": t_q, "query_ordered_shuffles_per_s": N / (t_q / 1e3),
                 "totals_equal": bool(torch.equal(res["b"].totals, res["q"].totals)),
                 "p_upper": bits.bits_pvalue(int(res["b"].n_ge.item()), N)}


def config_c3(bits, datagen, proj, timed, train):
    """The uneven batch: 32 query sets x 64 references, one graph-captured persistent launch."""
    import torch

    lengths, Q, R = datagen.w3_sets()
    qd = [proj(lengths, S) for S in Q]
    rd = [proj(lengths, S) for S in R]
    na = [len(S.start) for S in Q]
    nb = [len(S.start) for S in R]
    refs = bits.bits_sort_refs(rd, learned=True, train=train)
    sample = [(s[:max(1, n // 16)].contiguous(), e[:max(1, n // 16)].contiguous()) for (s, e), n in zip(qd, na)]
    evals = float(sum(na)) * len(R)
    c3 = {"workload": "uneven batch: 32 query sets (log-uniform 1e3..2e6) x 64 references (1e4..5e6)",
          "pairs": len(Q) * len(R), "query_intervals": sum(na), "reference_intervals": sum(nb),
          "pair_evaluations": evals}
    res = {}
    for name, path in (("learned", 2), ("plain", 1)):
        lp = cached_autotune("c3|%s|%s" % (name, torch.cuda.get_device_properties(0).gcnArchName),
                             lambda: bits.bits_autotune_batch(refs, sample, path=path))
        plan = bits.bits_batch_create(refs, qd, launch=lp)
        t = timed(lambda: bits.bits_batch_run(plan), reps=5)
        res[name] = bits.bits_batch_run(plan).clone()
        c3[name] = {"launch": lp, "replay_ms": t, "pair_aps": evals / (t / 1e3)}
        bits.bits_batch_destroy(plan)
    c3["paths_equal"] = bool(torch.equal(res["learned"], res["plain"]))
    mb = batch_model_bytes(na, nb)
    ach = mb / (c3["plain"]["replay_ms"] / 1e3) / 1e9
    c3["roofline_plain"] = {"bound": "hbm", "kernel": "k_batch (plain path)", "achieved": ach,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                            "model_bytes": mb, "traffic": None,
                            "model": "8 B query read + 2 x (h_mid + 1) x 128 B per (query, reference)"}
    return c3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads (outside the timed step)")
    ap.add_argument("--configs", default="c0,c1,c2,c3",
                    help="the other workloads to run, comma-separated (c0 small counts, c1 genome-scale counts, "
                         "c2 small-reference Monte-Carlo, c3 uneven batch)")
    ap.add_argument("--epochs", type=int, default=TRAIN_EPOCHS)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the recorded best launch shapes instead of timing candidates")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with a plain 1 GiB device copy (HBM byte-counter calibration)")
    args = ap.parse_args()
    which = [] if args.no_configs else [c for c in args.configs.split(",") if c]
    unknown = sorted(set(which) - {"c0", "c1", "c2", "c3"})
    if unknown:
        raise SystemExit("bench.py: unknown --configs entries %s (known: c0, c1, c2, c3)" % ", ".join(unknown))
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
    arch = torch.cuda.get_device_properties(0).gcnArchName
    timed = make_timer()

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

    def mc_result():
        return bits.MCResult(torch.empty(N_SHUF, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev),
                             torch.empty(1, dtype=torch.uint64, device=dev))
    mc_out = mc_result()
    train = {"epochs": args.epochs, "max_points": TRAIN_POINTS}

    # launch shapes from the autotuner (outside the timed region)
    a_s, a_e = bits.bits_project(lengths, *dA)
    b_s, b_e = bits.bits_project(lengths, *dB)
    bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws)
    tag = "%s|nA=%d|nB=%d" % (arch, N_A, N_B)
    if args.no_autotune:
        lp_learned, lp_plain, lp_tiered, lp_mc = (dict(RECORDED_LEARNED), dict(RECORDED_PLAIN),
                                                  dict(RECORDED_TIERED), dict(RECORDED_MC))
    else:
        lp_learned = cached_autotune("learned|" + tag, lambda: bits.bits_autotune_count(ref, a_s, a_e, 2))
        lp_plain = cached_autotune("plain|" + tag, lambda: bits.bits_autotune_count(ref, a_s, a_e, 1))
        lp_tiered = cached_autotune("tiered|" + tag, lambda: bits.bits_autotune_count(ref, a_s, a_e, 3))
        lp_mc = tune_mc(bits, ref, a_s[:N_MC], a_e[:N_MC], lengths, mc_ws)

    def step(ev=None):
        a_s, a_e = bits.bits_project(lengths, *dA)
        b_s, b_e = bits.bits_project(lengths, *dB)
        if ev:
            ev[0].record()
        bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws)
        if ev:
            ev[1].record()
        bits.bits_count_per_query(ref, a_s, a_e, launch=lp_learned, counts=counts, total=total)
        if ev:
            ev[2].record()
        bits.bits_mc_binned(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF, batch=MC_BATCH,
                            launch=lp_mc, workspace=bin_ws, out=mc_out)
        if ev:
            ev[3].record()
        return a_s, a_e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phase = {"setup_ms": [], "count_ms": [], "mc_ms": []}
    stages = {"place": [], "search": [], "reduce": []}
    # The timed steps run back to back with no host wait between them (events only); the
    # phase times are read once the last step has finished.
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    bits.bits_mc_binned_timing(True)    # HIP events around the binned kernels, on the stream they run on
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    for ev in evs:
        phase["setup_ms"].append(ev[0].elapsed_time(ev[1]))
        phase["count_ms"].append(ev[1].elapsed_time(ev[2]))
        phase["mc_ms"].append(ev[2].elapsed_time(ev[3]))
    # the binned kernels' stage times: the last timed step, and two more steps after the timed region
    for k, v in bits.bits_mc_binned_stage_ms().items():
        stages[k].append(v)
    for _ in range(2):
        step()
        torch.cuda.synchronize()
        for k, v in bits.bits_mc_binned_stage_ms().items():
            stages[k].append(v)
    bits.bits_mc_binned_timing(False)
    ms_per_step = t_total * 1e3 / args.steps
    evals = N_A + N_SHUF * N_MC
    value = evals / (ms_per_step / 1e3)
    status = bits.bits_get_status(ref)
    mc_totals = mc_out.totals.clone()
    info = bits.bits_rmi_info(ref)

    # ---- what the trained network gains: four counting paths on the same reference, outside the
    # timed region.  (i) the trained model (the step's index), (ii) the same model before training
    # (knots at the sampled quantiles, 0 epochs), (iii) no model: LDS tree, then bisection over the
    # line heads (the 32-key node tier), then one line, (iv) plain: LDS tree, then bisection.
    a_s, a_e = bits.bits_project(lengths, *dA)
    b_s, b_e = bits.bits_project(lengths, *dB)
    exp_counts = torch.empty_like(counts)
    t_plain = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch=lp_plain, counts=exp_counts,
                                                      total=total))
    plain_total = int(total.item())
    gain = {}

    def count_path(name, r, lp):
        f0 = bits.bits_rmi_info(r)["fallbacks"] if lp["path"] == 2 else 0
        bits.bits_count_per_query(r, a_s, a_e, launch=lp, counts=counts, total=total)
        exact = bool(torch.equal(counts, exp_counts)) and int(total.item()) == plain_total
        rec = {"launch": lp, "exact_vs_plain": exact}
        if lp["path"] == 2:   # one call: two searches per query
            st = bits.bits_rmi_info(r)
            rec.update({"mean_window": st["mean_window"], "max_window": st["max_window"],
                        "fallbacks_per_search": (st["fallbacks"] - f0) / (2.0 * N_A)})
        t = timed(lambda: bits.bits_count_per_query(r, a_s, a_e, launch=lp, counts=counts, total=total))
        rec.update({"ms": t, "aps": N_A / (t / 1e3)})
        gain[name] = rec
    count_path("trained", ref, lp_learned)
    ref_init = bits.bits_sort_ref(b_s, b_e, learned=True, train={"epochs": 0, "max_points": TRAIN_POINTS})
    count_path("init_only", ref_init, lp_learned)
    del ref_init
    count_path("tiered_no_model", ref, lp_tiered)
    gain["plain"] = {"launch": lp_plain, "ms": t_plain, "aps": N_A / (t_plain / 1e3), "exact_vs_plain": True}
    gain["speedup_model_over_no_model"] = gain["tiered_no_model"]["ms"] / gain["trained"]["ms"]
    gain["speedup_model_over_plain"] = t_plain / gain["trained"]["ms"]
    gain["speedup_training"] = gain["init_only"]["ms"] / gain["trained"]["ms"]
    # training points per leaf: window against setup time (80 epochs)
    sweep = []
    for pts in (64, 128, 256, 1024, 2048):
        tr = {"epochs": args.epochs, "max_points": pts}
        ts = timed(lambda: bits.bits_sort_ref(b_s, b_e, learned=True, train=tr, ref=ref, workspace=ws), reps=2)
        st = bits.bits_rmi_info(ref)
        tc = timed(lambda: bits.bits_count_per_query(ref, a_s, a_e, launch=lp_learned, counts=counts, total=total))
        sweep.append({"max_points": pts, "setup_ms": ts, "count_ms": tc, "mean_window": st["mean_window"],
                      "max_window": st["max_window"]})
    gain["training_points_sweep"] = sweep
    bits.bits_sort_ref(b_s, b_e, learned=True, train=train, ref=ref, workspace=ws)   # back to the step's index

    # ---- query-ordered Monte-Carlo paths on the same draws (outside the timed region)
    mc_plain, mc_learned = mc_result(), mc_result()
    t_mc_plain = timed(lambda: bits.bits_mc_pvalue(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF,
                                                   launch=lp_plain, workspace=mc_ws, out=mc_plain), reps=1)
    t_mc_learned = timed(lambda: bits.bits_mc_pvalue(ref, a_s[:N_MC], a_e[:N_MC], lengths, MC_SEED, 0, N_SHUF,
                                                     launch=lp_mc, workspace=mc_ws, out=mc_learned), reps=2)
    agree = (plain_total == int(total.item())) and bool(torch.equal(mc_plain.totals, mc_totals))
    binned_agree = (bool(torch.equal(mc_learned.totals, mc_totals))
                    and int(mc_learned.observed.item()) == int(mc_out.observed.item()))

    # ---- enumeration (sub-problem 4) of the first N_ENUM A-intervals against B
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

    # ---- significance summary of the timed Monte-Carlo run (Sec. 3.2, Sec. 3.3) and the decision
    m_lo, m_hi = bits.bits_mc_median(mc_out.totals)
    m_lo, m_hi = int(m_lo.item()), int(m_hi.item())
    obs, n_ge, n_le = int(mc_out.observed.item()), int(mc_out.n_ge.item()), int(mc_out.n_le.item())
    significance = {"observed": obs, "median": (m_lo + m_hi) / 2, "enrichment_log2": bits.bits_enrichment(obs, m_lo, m_hi),
                    "n_ge": n_ge, "n_le": n_le, "p_upper": bits.bits_pvalue(n_ge, N_SHUF),
                    "p_lower": bits.bits_pvalue_lower(n_le, N_SHUF),
                    "p_two_sided": bits.bits_pvalue_two_sided(n_ge, n_le, N_SHUF)}
    significance["decide_ms"] = timed(lambda: bits.bits_decide(ref, a_s, a_e, launch=lp_learned))
    significance["decide_found"] = int(bits.bits_decide(ref, a_s, a_e, launch=lp_learned)[0].item())

    # ---- the paper's Monte-Carlo orientation (B randomised and re-sorted every round) against the
    # fixed-index loop on the same draws: 1e6 x 1e6 intervals, 100 rounds
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

    # ---- measured achievable HBM rate: a plain 1 GiB device copy (1 GiB read + 1 GiB written)
    cx = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cy = torch.empty_like(cx)
    t_copy = timed(lambda: cy.copy_(cx), reps=5)
    copy_gbs = 2.0 * (1 << 30) / (t_copy / 1e3) / 1e9
    del cx, cy

    # ---- rooflines of the binned Monte-Carlo kernels (one pass of MC_BATCH shuffles per launch)
    mc_avg = float(np.mean(phase["mc_ms"]))
    stage_ms = {k: float(np.mean(v)) for k, v in stages.items()}
    passes = (N_SHUF + MC_BATCH - 1) // MC_BATCH
    placements = N_SHUF * N_MC // passes
    dom = "k_bin_place" if stage_ms["place"] >= stage_ms["search"] else "k_bin_search"
    launch_ms = {"k_bin_place": stage_ms["place"] / passes, "k_bin_search": stage_ms["search"] / passes}
    design_bytes = {"k_bin_place": BYTES_PER_PLACEMENT["k_bin_place"] * placements,
                    "k_bin_search": BYTES_PER_PLACEMENT["k_bin_search"] * placements + 8.0 * N_B}
    achieved = design_bytes[dom] / (launch_ms[dom] / 1e3) / 1e9
    traffic, _ = load_counters(dom, placements)
    # the method's compulsory bytes for one pass of the loop: each reference slice staged once
    # (4 bytes per key of B_S and B_E) and the 8-byte query entry read once; a shuffled interval
    # itself is made in registers (no compulsory bytes per evaluation)
    compulsory = 8.0 * N_B + 8.0 * N_MC
    pass_ms = (stage_ms["place"] + stage_ms["search"] + stage_ms["reduce"]) / passes
    _, lds_instr = load_counters("k_bin_search", placements)
    lds_ach = None if lds_instr is None else lds_instr * 256.0 / (launch_ms["k_bin_search"] / 1e3) / 1e9
    valu_ach = {}
    for kname in ("k_bin_place", "k_bin_search"):
        instr = load_valu(kname, placements)
        valu_ach[kname] = None if instr is None else instr / (launch_ms[kname] / 1e3) / 1e9
    other = "k_bin_search" if dom == "k_bin_place" else "k_bin_place"
    learned_achieved = BYTES_PER_EVAL_LEARNED * N_SHUF * N_MC / (t_mc_learned / 1e3) / 1e9

    configs = other_configs(bits, dev, timed, train, which) if which else None

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
                   "train_points": TRAIN_POINTS,
                   "launch_learned": lp_learned, "launch_plain": lp_plain, "launch_tiered": lp_tiered,
                   "mc": {"path": "binned by genome region", "batch": MC_BATCH, "observed_launch": lp_mc}},
        "library": library_info(bits),
        "phases_ms": {k: float(np.mean(v)) for k, v in phase.items()},
        "mc_stage_ms": stage_ms,
        "count_learned_aps": gain["trained"]["aps"],
        "count_plain_aps": gain["plain"]["aps"],
        "count_tiered_aps": gain["tiered_no_model"]["aps"],
        "learned_speedup": gain["speedup_model_over_plain"],
        "learned_speedup_over_no_model": gain["speedup_model_over_no_model"],
        "gain": gain,
        "mc_shuffles_per_s": N_SHUF / (mc_avg / 1e3),
        "mc_shuffles_per_s_learned": N_SHUF / (t_mc_learned / 1e3),
        "mc_shuffles_per_s_plain": N_SHUF / (t_mc_plain / 1e3),
        "learned_equals_plain": bool(agree),
        "binned_equals_learned": bool(binned_agree),
        "rmi": info,
        "enumeration": enumeration,
        "significance": significance,
        "paper_orientation": paper_orientation,
        "configs": configs,
        "status": status,
        "roofline": {"bound": "hbm", "kernel": dom + " (Monte-Carlo shuffles binned by genome region)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes": "design bytes of the binned algorithm: %s per placement%s" % (
                         BYTES_PER_PLACEMENT[dom], " + 8 B per interval of B" if dom == "k_bin_search" else ""),
                     "placements_per_launch": placements, "launch_ms": launch_ms[dom],
                     "peak_measured_copy": copy_gbs, "frac_of_measured": achieved / copy_gbs,
                     "compulsory_bytes_per_pass": compulsory,
                     "frac_compulsory_per_pass": compulsory / (pass_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "limiter": ("VALU issue: the two bucket searches and the per-shuffle sums"
                                 if dom == "k_bin_search" else
                                 "VALU issue: two Philox draws per placement and the LDS ranking of each chunk; "
                                 "the record writes are about 1.6x the design bytes (partly written lines)")},
        "roofline_lds": {"bound": "lds", "kernel": "k_bin_search", "achieved": lds_ach, "peak": LDS_PEAK_GBS,
                         "unit": "GB/s", "frac": None if lds_ach is None else lds_ach / LDS_PEAK_GBS,
                         "launch_ms": launch_ms["k_bin_search"],
                         "bytes": "LDS instructions per launch (counters) x 256 B (64 lanes x 4 B)"},
        "roofline_valu": {"bound": "alu", "kernel": dom, "achieved": valu_ach[dom], "peak": VALU_PEAK_G,
                          "unit": "G wave-instructions/s",
                          "frac": None if valu_ach[dom] is None else valu_ach[dom] / VALU_PEAK_G,
                          "launch_ms": launch_ms[dom],
                          "bytes": "VALU wave-instructions per launch (counters); peak: one wave64 VALU "
                                   "instruction per CU per clock, 256 CUs, 2.4 GHz",
                          "other": {"kernel": other, "achieved": valu_ach[other], "launch_ms": launch_ms[other],
                                    "frac": None if valu_ach[other] is None else valu_ach[other] / VALU_PEAK_G}},
        "roofline_learned_mc": {"bound": "hbm", "kernel": "k_mc_sorted (query-ordered learned-index Monte-Carlo, "
                                "outside the timed region)", "achieved": learned_achieved, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": learned_achieved / HBM_PEAK_GBS,
                                "bytes_per_eval_model": BYTES_PER_EVAL_LEARNED, "call_ms": t_mc_learned},
    }
    if not args.no_cpu_baseline:
        cpu = host_cpu()
        result["cpu_baseline"] = cpu_baseline(lengths, A, B, cpu["threads"])
        result["cpu_baseline"]["host"] = cpu
    print(json.dumps(result), flush=True)
    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")


if __name__ == "__main__":
    main()
