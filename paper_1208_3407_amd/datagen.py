"""Seeded synthetic interval sets for the BITS workloads.

This module only *samples* inputs.  It holds none of the method's arithmetic:
no projection to one dimension, no sorting, no counting, no random placement
used by the Monte-Carlo loop.  Every set is returned in chromosome-local,
0-based, closed coordinates as three uint32 arrays ``(chrom, start, end)``,
together with the genome's chromosome lengths; the HIP path and the CPU oracle
each project them with their own code.

The shapes follow the paper's workloads (Layer et al. 2012): Table 1 runs
Monte-Carlo rounds on sets of 1e5-1e7 intervals, Fig. 2 counts 1M/10M
alignment intervals against exons, Sec. 3.3 screens many pairs of annotation
tracks.  Those data sets (1000 Genomes alignments, RefSeq exons, ENCODE
tracks) are not available; uniform sets stand in for whole-genome alignments
and Gaussian-clustered sets for exome-capture alignments and exons.

Workloads (sizes, distributions and seeds):
  * W0  one 10,000,000 bp chromosome; A, B of 10,000 intervals each, starts
        uniform on [0, 9,999,000], lengths uniform on [100, 1000].
  * W1  24-chromosome genome with len_k = floor(249,200,000 * 0.93^k); A and
        B of 10M intervals, log-normal lengths (median 200, sigma 1, clipped
        to [20, 100,000]); A uniform; B half uniform, half drawn around 20,000
        Gaussian cluster centres (sigma 50 kbp).
  * W2  Monte-Carlo: A = 100,000 uniform (median length 500), B = 1,000,000
        half uniform / half clustered, 10,000 shuffles, Philox key 7.
  * W3  uneven batch: 32 query sets of log-uniform size in [1e3, 2e6], 64
        reference sets of log-uniform size in [1e4, 5e6].
  * W4  learned index at scale: B = 50M half uniform / half clustered,
        A = 50M uniform; Monte-Carlo over the first 1M of A, 1,000 shuffles.
  * S   the all-pairs screen of Sec. 3.3 (Fig. 3): 159 annotation tracks of
        log-uniform size in [1e3, 2e6], each half uniform / half clustered
        (shared cluster centres), every track both query and reference.
"""
from __future__ import annotations

import dataclasses

import numpy as np

N_CLUSTERS = 20_000
CLUSTER_SIGMA = 50_000.0
MC_SEED = 7


def rng_for(seed: int, *key: int) -> np.random.Generator:
    """Independent, reproducible stream for (seed, key...)."""
    return np.random.default_rng(np.random.SeedSequence(int(seed), spawn_key=tuple(int(k) for k in key)))


def genome_one(length: int = 10_000_000) -> np.ndarray:
    return np.array([length], dtype=np.uint32)


def genome_g24() -> np.ndarray:
    """Chromosome k has floor(249,200,000 * 93^k / 100^k) bp, k = 0..23 (exact integers)."""
    return np.array([249_200_000 * 93 ** k // 100 ** k for k in range(24)], dtype=np.uint32)


@dataclasses.dataclass
class IntervalSet:
    chrom: np.ndarray   # uint32 chromosome index
    start: np.ndarray   # uint32 chromosome-local start (0-based, closed)
    end: np.ndarray     # uint32 chromosome-local end   (inclusive)

    def __len__(self) -> int:
        return int(self.chrom.shape[0])

    def head(self, n: int) -> "IntervalSet":
        return IntervalSet(self.chrom[:n].copy(), self.start[:n].copy(), self.end[:n].copy())


def lognormal_lengths(rng: np.random.Generator, n: int, median: float, sigma: float = 1.0,
                      lo: int = 20, hi: int = 100_000) -> np.ndarray:
    z = rng.standard_normal(n)
    return np.clip(np.rint(np.exp(np.log(median) + sigma * z)), lo, hi).astype(np.int64)


def _pick_chrom(rng: np.random.Generator, lengths: np.ndarray, n: int) -> np.ndarray:
    p = lengths.astype(np.float64) / float(lengths.astype(np.float64).sum())
    return rng.choice(len(lengths), size=n, p=p).astype(np.int64)


def uniform_set(rng: np.random.Generator, lengths: np.ndarray, L: np.ndarray) -> IntervalSet:
    """Start position uniform over the genome; an interval that would run past
    its chromosome's end keeps its length and moves left."""
    n = len(L)
    lens = lengths.astype(np.int64)
    c = _pick_chrom(rng, lengths, n)
    pos = rng.integers(0, lens[c])
    s = np.minimum(pos, lens[c] - L)
    return IntervalSet(c.astype(np.uint32), s.astype(np.uint32), (s + L - 1).astype(np.uint32))


def cluster_centres(rng: np.random.Generator, lengths: np.ndarray, k: int = N_CLUSTERS):
    lens = lengths.astype(np.int64)
    c = _pick_chrom(rng, lengths, k)
    mu = rng.integers(0, lens[c])
    return c, mu


def clustered_set(rng: np.random.Generator, lengths: np.ndarray, L: np.ndarray, centres) -> IntervalSet:
    """Each interval picks a centre and lands at rint(mu + 50 kbp * z), kept
    inside the centre's chromosome with its length intact."""
    cc, mu = centres
    n = len(L)
    lens = lengths.astype(np.int64)
    j = rng.integers(0, len(cc), size=n)
    c = cc[j]
    p = np.rint(mu[j] + CLUSTER_SIGMA * rng.standard_normal(n)).astype(np.int64)
    s = np.clip(p, 0, lens[c] - L)
    return IntervalSet(c.astype(np.uint32), s.astype(np.uint32), (s + L - 1).astype(np.uint32))


def mixture_set(rng: np.random.Generator, lengths: np.ndarray, L: np.ndarray, centres) -> IntervalSet:
    """First floor(n/2) intervals uniform, the rest clustered."""
    h = len(L) // 2
    u = uniform_set(rng, lengths, L[:h])
    c = clustered_set(rng, lengths, L[h:], centres)
    return IntervalSet(np.concatenate([u.chrom, c.chrom]), np.concatenate([u.start, c.start]),
                       np.concatenate([u.end, c.end]))


# --------------------------------------------------------------------------
# Workload builders.  Stream keys: (workload, role) so every set is
# independent of the sizes of the others.
# --------------------------------------------------------------------------

def w0_sets(seed: int = 1, n_a: int = 10_000, n_b: int = 10_000):
    lengths = genome_one()

    def one(role, n):
        r = rng_for(seed, 0, role)
        s = r.integers(0, 10_000_000 - 1000 + 1, size=n)
        L = r.integers(100, 1000 + 1, size=n)
        return IntervalSet(np.zeros(n, np.uint32), s.astype(np.uint32), (s + L - 1).astype(np.uint32))

    return lengths, one(0, n_a), one(1, n_b)


def w1_sets(seed: int = 1, n_a: int = 10_000_000, n_b: int = 10_000_000, median_a: float = 200.0,
            workload: int = 1):
    lengths = genome_g24()
    centres = cluster_centres(rng_for(seed, workload, 9), lengths)
    ra = rng_for(seed, workload, 0)
    A = uniform_set(ra, lengths, lognormal_lengths(ra, n_a, median_a))
    rb = rng_for(seed, workload, 1)
    B = mixture_set(rb, lengths, lognormal_lengths(rb, n_b, 200.0), centres)
    return lengths, A, B


def w2_sets(seed: int = 1, n_a: int = 100_000, n_b: int = 1_000_000):
    return w1_sets(seed, n_a, n_b, median_a=500.0, workload=2)


def w3_sizes(seed: int = 1, n_q: int = 32, n_r: int = 64, q_range=(1_000, 2_000_000),
             r_range=(10_000, 5_000_000)):
    r = rng_for(seed, 3, 8)
    q = np.rint(np.exp(r.uniform(np.log(q_range[0]), np.log(q_range[1]), n_q))).astype(np.int64)
    b = np.rint(np.exp(r.uniform(np.log(r_range[0]), np.log(r_range[1]), n_r))).astype(np.int64)
    return q, b


def w3_sets(seed: int = 1, n_q: int = 32, n_r: int = 64, q_range=(1_000, 2_000_000),
            r_range=(10_000, 5_000_000)):
    lengths = genome_g24()
    centres = cluster_centres(rng_for(seed, 3, 9), lengths)
    qs, rs = w3_sizes(seed, n_q, n_r, q_range, r_range)
    queries, refs = [], []
    for i, n in enumerate(qs):
        r = rng_for(seed, 3, 100 + i)
        queries.append(uniform_set(r, lengths, lognormal_lengths(r, int(n), 200.0)))
    for j, n in enumerate(rs):
        r = rng_for(seed, 3, 1000 + j)
        refs.append(mixture_set(r, lengths, lognormal_lengths(r, int(n), 200.0), centres))
    return lengths, queries, refs


def w4_sets(seed: int = 1, n_a: int = 50_000_000, n_b: int = 50_000_000):
    return w1_sets(seed, n_a, n_b, median_a=200.0, workload=4)


def screen_sets(seed: int = 1, n_tracks: int = 159, size_range=(1_000, 2_000_000)):
    """Tracks of the all-pairs screen: sizes log-uniform in size_range, each a
    half-uniform / half-clustered mixture around shared centres."""
    lengths = genome_g24()
    centres = cluster_centres(rng_for(seed, 6, 9), lengths)
    r = rng_for(seed, 6, 8)
    sizes = np.rint(np.exp(r.uniform(np.log(size_range[0]), np.log(size_range[1]), n_tracks))).astype(np.int64)
    tracks = []
    for i, n in enumerate(sizes):
        ri = rng_for(seed, 6, 100 + i)
        tracks.append(mixture_set(ri, lengths, lognormal_lengths(ri, int(n), 200.0), centres))
    return lengths, tracks
