"""Table 1 replay: Monte-Carlo run time on the shapes of the paper's Table 1
(Sec. 3.2): set sizes 1e5, 1e6, 1e7 (|A| = |B| = size, uniform placements on
the 24-chromosome genome, log-normal lengths with median 200 bp) and 1, 100,
1000 and 10,000 Monte-Carlo rounds, on this GPU, in two orientations:

  resort  the paper's loop (bits_mc_resort): every round randomises the
          database set B, sorts it again and counts A against it;
  fixed   this library's loop (bits_mc_pvalue): the reference is built once
          from A (sort, line heads, learned index) and every round randomises
          B and searches it in A's index; the per-round totals are the same;
  binned  the same loop binned by genome region (bits_mc_binned): the
          placements of a batch of rounds are grouped by region of A's
          reference and counted in LDS; the per-round totals are the same.

A cell is setup (projection and sorting / index build) plus the rounds.
Rounds beyond a cap are timed on the cap and scaled linearly; such cells are
marked "~", as the paper marks its extrapolated cells.  Prints a Markdown
table and one JSON line.

    python -m paper_1208_3407_amd.table1 [--sizes 1e5,1e6,1e7] [--cap 1000]
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1208_3407_amd import bits, datagen  # noqa: E402

ROUNDS = [1, 100, 1000, 10_000]


def gpu_ms(fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1), out


def one_size(n, cap, seed=1):
    dev = torch.device("cuda", 0)
    lengths = datagen.genome_g24()
    sets = []
    for role in (1, 2):
        r = datagen.rng_for(seed, 5, role)
        sets.append(datagen.uniform_set(r, lengths, datagen.lognormal_lengths(r, n, 200.0)))
    A, B = sets

    def up(x):
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    dA = [up(A.chrom), up(A.start), up(A.end)]
    dB = [up(B.chrom), up(B.start), up(B.end)]
    batch = int(max(1, min(64, (1 << 26) // n)))
    ws_r = bits._scratch(bits.bits_mc_resort_workspace(n, batch), dev)
    ws_f = bits._scratch(bits.bits_mc_workspace(n), dev)
    bb = int(max(1, min(1000, (1 << 29) // n)))        # binned rounds per pass: records stay under 4 GiB
    ws_b = bits._scratch(bits.bits_mc_binned_workspace(n, n, lengths, bb), dev)
    # warm-up (loads kernels, sizes the caches)
    a_s, a_e = bits.bits_project(lengths, *dA)
    b_s, b_e = bits.bits_project(lengths, *dB)
    bits.bits_mc_resort(a_s, a_e, b_s, b_e, lengths, 7, 0, 2, batch=batch, workspace=ws_r)
    ref = bits.bits_sort_ref(a_s, a_e, learned=True)
    bits.bits_mc_pvalue(ref, b_s, b_e, lengths, 7, 0, 2, workspace=ws_f)
    bits.bits_mc_binned(ref, b_s, b_e, lengths, 7, 0, 2, batch=bb, workspace=ws_b)
    torch.cuda.synchronize()

    # setup: projection (+ the index build of the fixed orientation)
    t_proj, _ = gpu_ms(lambda: (bits.bits_project(lengths, *dA), bits.bits_project(lengths, *dB)))
    t_index, _ = gpu_ms(lambda: bits.bits_sort_ref(a_s, a_e, learned=True, ref=ref,
                                                   workspace=bits._scratch(bits.bits_sort_ref_workspace(n), dev)))
    rounds_timed = min(cap, ROUNDS[-1])
    t_resort, mr = gpu_ms(lambda: bits.bits_mc_resort(a_s, a_e, b_s, b_e, lengths, 7, 0, rounds_timed, batch=batch,
                                                      workspace=ws_r))
    t_fixed, mf = gpu_ms(lambda: bits.bits_mc_pvalue(ref, b_s, b_e, lengths, 7, 0, rounds_timed, workspace=ws_f))
    t_binned, mb = gpu_ms(lambda: bits.bits_mc_binned(ref, b_s, b_e, lengths, 7, 0, rounds_timed, batch=bb,
                                                      workspace=ws_b))
    same = bool(torch.equal(mr.totals, mf.totals)) and bool(torch.equal(mb.totals, mf.totals))
    per_r, per_f, per_b = t_resort / rounds_timed, t_fixed / rounds_timed, t_binned / rounds_timed
    row = {"size": n, "batch": batch, "binned_batch": bb, "rounds_timed": rounds_timed, "totals_equal": same,
           "setup_ms": {"projection": t_proj, "index": t_index},
           "per_round_ms": {"resort": per_r, "fixed": per_f, "binned": per_b}, "cells_s": {}}
    for r in ROUNDS:
        row["cells_s"][str(r)] = {
            "resort": (t_proj + r * per_r) / 1e3,
            "fixed": (t_proj + t_index + r * per_f) / 1e3,
            "binned": (t_proj + t_index + r * per_b) / 1e3,
            "extrapolated": r > rounds_timed}
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="1e5,1e6,1e7")
    ap.add_argument("--cap", type=int, default=1000, help="rounds actually timed per cell")
    args = ap.parse_args()
    if not torch.cuda.is_available():
        raise SystemExit("needs the GPU")
    rows = []
    for tok in args.sizes.split(","):
        n = int(float(tok))
        print("size %d ..." % n, file=sys.stderr, flush=True)
        rows.append(one_size(n, args.cap))
    print("| Size | Orientation | " + " | ".join("%d rounds" % r for r in ROUNDS) + " |")
    print("|---|---|" + "---|" * len(ROUNDS))
    for row in rows:
        for o, name in (("resort", "resort (paper's loop)"), ("fixed", "fixed index"), ("binned", "fixed index, binned")):
            cells = []
            for r in ROUNDS:
                c = row["cells_s"][str(r)]
                cells.append(("~" if c["extrapolated"] else "") + "%.3g" % c[o])
            print("| %.0e | %s | %s |" % (row["size"], name, " | ".join(cells)))
    print(json.dumps({"table1_replay": rows}))


if __name__ == "__main__":
    main()
