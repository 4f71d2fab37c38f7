"""The all-pairs screen of Sec. 3.3 (Fig. 3) on one GPU: every pair (i, j) of
n annotation tracks, track i shuffled within its chromosomes against track j
held fixed, N Monte-Carlo rounds per pair; per pair the observed count, the
median of the shuffled counts, the enrichment log2(observed / median) and the
empirical p-values.  The paper ran 159 tracks (25,281 pairs) x 10,000 rounds
on one GPU.

Every step runs in libbits.so: the observed counts of all pairs are one
batch plan (one HIP-graph-captured persistent launch); each pair's Monte-Carlo
loop is bits_mc_binned (placements binned by region of track j, counted in
LDS), its median is bits_mc_median.

    python -m paper_1208_3407_amd.screen [--tracks 159] [--shuffles 10000] [--sample 3]

runs the observed counts of all pairs, and the Monte-Carlo loops of every
pair whose query is one of `--sample` tracks (seeded pick) at the full round
count; the full screen's time is extrapolated linearly in the number of
placements (sum over pairs of |track i| x rounds) from that sample, and is
labelled as extrapolated.  Prints a Markdown summary and one JSON line.
"""
import argparse
import json
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1208_3407_amd import bits, datagen  # noqa: E402

MC_SEED = 7
RECORD_BYTES_CAP = 4 << 30   # records of one binned pass stay under 4 GiB


def pass_batch(na: int) -> int:
    return int(max(1, min(1000, RECORD_BYTES_CAP // (8 * max(na, 1)))))


def mc_pair(ref, q, lengths, shuffles, batch, workspace=None):
    """Monte-Carlo loop of one pair: MCResult plus the (lo, hi) middle order statistics."""
    mc = bits.bits_mc_binned(ref, q[0], q[1], lengths, MC_SEED, 0, shuffles, batch=batch, workspace=workspace)
    lo, hi = bits.bits_mc_median(mc.totals)
    return mc, lo, hi


def summarise(mc, lo, hi, shuffles):
    obs, n_ge, n_le = int(mc.observed.item()), int(mc.n_ge.item()), int(mc.n_le.item())
    lo, hi = int(lo.item()), int(hi.item())
    return {"observed": obs, "median": (lo + hi) / 2, "enrichment_log2": bits.bits_enrichment(obs, lo, hi),
            "p_upper": bits.bits_pvalue(n_ge, shuffles), "p_lower": bits.bits_pvalue_lower(n_le, shuffles)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tracks", type=int, default=159)
    ap.add_argument("--shuffles", type=int, default=10_000)
    ap.add_argument("--sample", type=int, default=3, help="query tracks whose pairs run the full Monte-Carlo loop")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("needs the GPU")
    dev = torch.device("cuda", 0)
    lengths, tracks = datagen.screen_sets(n_tracks=args.tracks)

    def up(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    td = [bits.bits_project(lengths, up(T.chrom), up(T.start), up(T.end)) for T in tracks]
    sizes = np.array([len(T) for T in tracks], np.int64)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    e0.record()
    refs = bits.bits_sort_refs(td)
    e1.record()
    e1.synchronize()
    t_index = e0.elapsed_time(e1)
    plan = bits.bits_batch_create(refs, td)
    bits.bits_batch_run(plan)
    e0.record()
    observed = bits.bits_batch_run(plan)
    e1.record()
    e1.synchronize()
    t_observed = e0.elapsed_time(e1)
    observed = observed.view(len(td), len(refs)).cpu().numpy()
    bits.bits_batch_destroy(plan)

    pick = np.sort(np.random.default_rng(1).choice(len(td), size=min(args.sample, len(td)), replace=False))
    rows, t_mc = [], 0.0
    for i in pick:
        batch = pass_batch(int(sizes[i]))
        ws = bits._scratch(max(bits.bits_mc_binned_workspace(int(sizes[i]), int(sizes.max()), lengths, batch), 1), dev)
        mc_pair(refs[0], td[i], lengths, min(args.shuffles, 8), batch, ws)   # warm-up
        e0.record()
        res = [mc_pair(refs[j], td[i], lengths, args.shuffles, batch, ws) for j in range(len(refs))]
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1)
        t_mc += t
        for j, (mc, lo, hi) in enumerate(res):
            s = summarise(mc, lo, hi, args.shuffles)
            assert s["observed"] == int(observed[i, j])
            rows.append({"query": int(i), "reference": j, **s})
        print("query track %d (%d intervals): %d pairs x %d rounds in %.1f ms" % (i, sizes[i], len(refs),
                                                                                  args.shuffles, t),
              file=sys.stderr, flush=True)
        del ws, res
    n = len(td)
    placements_all = float(sizes.sum()) * n * args.shuffles
    placements_sample = float(sizes[pick].sum()) * n * args.shuffles
    t_full_s = (t_mc / 1e3) * placements_all / placements_sample + (t_index + t_observed) / 1e3
    enr = np.array([r["enrichment_log2"] for r in rows])
    summary = {
        "tracks": n, "pairs": n * n, "shuffles": args.shuffles, "intervals": int(sizes.sum()),
        "index_ms": t_index, "observed_all_pairs_ms": t_observed,
        "sample_query_tracks": [int(i) for i in pick], "sample_pairs": len(rows),
        "sample_placements": placements_sample, "sample_mc_ms": t_mc,
        "placements_per_s": placements_sample / (t_mc / 1e3),
        "full_screen_placements": placements_all, "full_screen_s_extrapolated": t_full_s,
        "sample_enrichment_log2": {"min": float(np.min(enr[np.isfinite(enr)])) if np.isfinite(enr).any() else None,
                                   "max": float(np.max(enr[np.isfinite(enr)])) if np.isfinite(enr).any() else None},
    }
    print("| Screen | Value |")
    print("|---|---|")
    print("| tracks / pairs | %d / %d |" % (n, n * n))
    print("| intervals over all tracks | %d |" % int(sizes.sum()))
    print("| index build (all tracks) | %.1f ms |" % t_index)
    print("| observed counts of all pairs (one graph launch) | %.1f ms |" % t_observed)
    print("| Monte-Carlo, %d sampled query tracks x %d references x %d rounds | %.1f s (%.3g placements/s) |" % (
        len(pick), n, args.shuffles, t_mc / 1e3, summary["placements_per_s"]))
    print("| full screen, %d pairs x %d rounds | ~%.0f s (extrapolated) |" % (n * n, args.shuffles, t_full_s))
    print(json.dumps({"screen": summary}))


if __name__ == "__main__":
    main()
