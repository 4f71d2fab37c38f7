"""CPU oracle for BITS -- TEST INFRASTRUCTURE ONLY.

A ctypes view of ``liboracle.so`` (plain C, see ``oracle.c``).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg use it; the product path
(the HIP library and its binding) never imports this package.

Citations: Layer et al., Bioinformatics 2012 (BITS) -- Sec. 1.1 (definition),
Sec. 2.1 (Algorithms 1 and 2, projection), Sec. 3.2 (Monte-Carlo); Salmon et
al., SC'11 (Philox-4x32-10).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c_u64 = ctypes.c_uint64
_c_u32 = ctypes.c_uint32


def lib():
    """Load liboracle.so, building it with gcc when it is absent."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_genome_offsets.argtypes = [_u32p, _c_u32, _u64p]
        L.oracle_project.argtypes = [_u32p, _c_u32, _u32p, _u32p, _u32p, _c_u64, _u32p, _u32p]
        L.oracle_sort_u32.argtypes = [_u32p, _c_u64]
        L.oracle_sort_u32.restype = None
        L.oracle_count_bruteforce.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _c_u64,
                                              ctypes.c_void_p, ctypes.POINTER(_c_u64)]
        L.oracle_count_bruteforce.restype = None
        L.oracle_enumerate_bruteforce.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _c_u64,
                                                  ctypes.c_void_p, ctypes.c_void_p, _c_u64]
        L.oracle_enumerate_bruteforce.restype = _c_u64
        L.oracle_count_less.argtypes = [_u32p, _c_u64, _c_u32]
        L.oracle_count_less.restype = _c_u64
        L.oracle_count_le.argtypes = [_u32p, _c_u64, _c_u32]
        L.oracle_count_le.restype = _c_u64
        L.oracle_count_sorted.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _c_u64,
                                          ctypes.c_void_p, ctypes.POINTER(_c_u64), ctypes.c_int]
        L.oracle_counter.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _c_u64,
                                     ctypes.c_void_p, ctypes.POINTER(_c_u64), ctypes.c_int]
        L.oracle_sweep_total.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _c_u64]
        L.oracle_sweep_total.restype = _c_u64
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_mc_prepare.argtypes = [_u32p, _c_u32, _u32p, _u32p, _c_u64, _u32p, _u32p, _u32p]
        L.oracle_mc_placements.argtypes = [_c_u64, _c_u64, _c_u64, _u32p, _u32p, _u32p]
        L.oracle_mc_placements.restype = None
        L.oracle_mc_totals.argtypes = [_u32p, _u32p, _c_u64, _u32p, _u32p, _u32p, _c_u64,
                                       _c_u64, _c_u64, _c_u64, _u64p, ctypes.c_int]
        L.oracle_mc_tail.argtypes = [_u64p, _c_u64, _c_u64, ctypes.POINTER(_c_u64),
                                     ctypes.POINTER(_c_u64)]
        L.oracle_mc_tail.restype = None
        L.oracle_mc_median.argtypes = [_u64p, _c_u64, ctypes.POINTER(_c_u64), ctypes.POINTER(_c_u64)]
        L.oracle_mc_median.restype = None
        L.oracle_mc_expected_total.argtypes = [_u32p, _c_u32, _u32p, _u32p, _c_u64,
                                               _u32p, _u32p, _c_u64]
        L.oracle_mc_expected_total.restype = ctypes.c_double
        L.oracle_rmi_forward.argtypes = [_f32p, _f32p, _c_u32, _f64p]
        L.oracle_rmi_forward.restype = None
        L.oracle_rmi_loss_grad.argtypes = [_f32p, _f32p, _f32p, _c_u32,
                                           ctypes.POINTER(ctypes.c_double), _f64p]
        L.oracle_rmi_loss_grad.restype = None
        L.oracle_linear_fit.argtypes = [_u32p, _c_u64, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]
        L.oracle_linear_fit.restype = None
        _LIB = L
    return _LIB


def _u32(x):
    return np.ascontiguousarray(x, dtype=np.uint32)


def genome_offsets(lengths):
    """Offsets of each chromosome in the projected 1-D genome (n_chrom + 1 values)."""
    lengths = _u32(lengths)
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    if lib().oracle_genome_offsets(lengths, len(lengths), off) != 0:
        raise ValueError("genome does not fit in 32-bit coordinates")
    return off


def project(lengths, chrom, lstart, lend):
    """Projection to global closed coordinates (Sec. 2.1)."""
    lengths, chrom, lstart, lend = _u32(lengths), _u32(chrom), _u32(lstart), _u32(lend)
    gs = np.empty(len(chrom), dtype=np.uint32)
    ge = np.empty(len(chrom), dtype=np.uint32)
    if lib().oracle_project(lengths, len(lengths), chrom, lstart, lend, len(chrom), gs, ge) != 0:
        raise ValueError("interval outside its chromosome or bad chromosome id")
    return gs, ge


def sort_u32(a):
    """Ascending copy of a uint32 array (qsort)."""
    out = np.array(a, dtype=np.uint32, copy=True)
    lib().oracle_sort_u32(out, len(out))
    return out


def count_bruteforce(a_start, a_end, b_start, b_end):
    """Per-query counts and total straight from the definition (Sec. 1.1)."""
    a_start, a_end, b_start, b_end = map(_u32, (a_start, a_end, b_start, b_end))
    counts = np.zeros(len(a_start), dtype=np.uint32)
    total = _c_u64(0)
    lib().oracle_count_bruteforce(a_start, a_end, len(a_start), b_start, b_end, len(b_start),
                                  counts.ctypes.data, ctypes.byref(total))
    return counts, int(total.value)


def enumerate_bruteforce(a_start, a_end, b_start, b_end):
    """Every intersecting pair (i, j) straight from the definition (Sec. 1.1,
    sub-problem 4), in order of i then j: two uint32 arrays."""
    a_start, a_end, b_start, b_end = map(_u32, (a_start, a_end, b_start, b_end))
    f = lib().oracle_enumerate_bruteforce
    k = int(f(a_start, a_end, len(a_start), b_start, b_end, len(b_start), None, None, 0))
    pa = np.zeros(max(k, 1), dtype=np.uint32)
    pb = np.zeros(max(k, 1), dtype=np.uint32)
    f(a_start, a_end, len(a_start), b_start, b_end, len(b_start), pa.ctypes.data, pb.ctypes.data, k)
    return pa[:k], pb[:k]


def count_less(sorted_arr, x):
    return int(lib().oracle_count_less(_u32(sorted_arr), len(sorted_arr), int(x)))


def count_le(sorted_arr, x):
    return int(lib().oracle_count_le(_u32(sorted_arr), len(sorted_arr), int(x)))


def count_sorted(sorted_bs, sorted_be, a_start, a_end, threads=1, per_query=True):
    """ICount over already sorted B_S, B_E (Algorithms 1 and 2)."""
    sorted_bs, sorted_be, a_start, a_end = map(_u32, (sorted_bs, sorted_be, a_start, a_end))
    counts = np.zeros(len(a_start), dtype=np.uint32) if per_query else None
    total = _c_u64(0)
    rc = lib().oracle_count_sorted(sorted_bs, sorted_be, len(sorted_bs), a_start, a_end,
                                   len(a_start), counts.ctypes.data if per_query else None,
                                   ctypes.byref(total), int(threads))
    if rc != 0:
        raise ValueError("query interval with start > end")
    return counts, int(total.value)


def counter(a_start, a_end, b_start, b_end, threads=1):
    """Counter(A, B) (Algorithm 2): sort B_S and B_E, then ICount every query."""
    a_start, a_end, b_start, b_end = map(_u32, (a_start, a_end, b_start, b_end))
    counts = np.zeros(len(a_start), dtype=np.uint32)
    total = _c_u64(0)
    rc = lib().oracle_counter(a_start, a_end, len(a_start), b_start, b_end, len(b_start),
                              counts.ctypes.data, ctypes.byref(total), int(threads))
    if rc != 0:
        raise ValueError("query interval with start > end")
    return counts, int(total.value)


def sweep_total(a_start, a_end, b_start, b_end):
    """Total by linear merges of sorted endpoints (independent of bisection)."""
    sa, ea, sb, eb = (sort_u32(x) for x in (a_start, a_end, b_start, b_end))
    return int(lib().oracle_sweep_total(sa, ea, len(sa), sb, eb, len(sb)))


def philox4x32_10(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_u32(ctr), _u32(key), out)
    return out


def mc_prepare(lengths, a_start, a_end):
    """Per-query (chromosome offset, number of legal starts, length)."""
    lengths, a_start, a_end = map(_u32, (lengths, a_start, a_end))
    n = len(a_start)
    off = np.zeros(n, dtype=np.uint32)
    span = np.zeros(n, dtype=np.uint32)
    ln = np.zeros(n, dtype=np.uint32)
    if lib().oracle_mc_prepare(lengths, len(lengths), a_start, a_end, n, off, span, ln) != 0:
        raise ValueError("query interval outside a chromosome")
    return off, span, ln


def mc_placements(seed, s, off, span):
    out = np.zeros(len(off), dtype=np.uint32)
    lib().oracle_mc_placements(int(seed), int(s), len(off), _u32(off), _u32(span), out)
    return out


def mc_totals(sorted_bs, sorted_be, prep, seed, s0, s1, threads=1):
    off, span, ln = prep
    out = np.zeros(max(0, s1 - s0), dtype=np.uint64)
    rc = lib().oracle_mc_totals(_u32(sorted_bs), _u32(sorted_be), len(sorted_bs), off, span, ln,
                                len(off), int(seed), int(s0), int(s1), out, int(threads))
    if rc != 0:
        raise ValueError("bad shuffle range")
    return out


def mc_tail(totals, observed):
    totals = np.ascontiguousarray(totals, dtype=np.uint64)
    ge, le = _c_u64(0), _c_u64(0)
    lib().oracle_mc_tail(totals, len(totals), int(observed), ctypes.byref(ge), ctypes.byref(le))
    return int(ge.value), int(le.value)


def mc_median(totals):
    """(lo, hi): the two middle order statistics of the totals (equal for odd n)."""
    t = np.ascontiguousarray(totals, dtype=np.uint64)
    lo, hi = _c_u64(0), _c_u64(0)
    lib().oracle_mc_median(t, len(t), ctypes.byref(lo), ctypes.byref(hi))
    return int(lo.value), int(hi.value)


def enrichment(observed, lo, hi):
    """Sec. 3.3 / Fig. 3: log2(observed / median), median = (lo + hi) / 2."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return float(np.log2(np.float64(observed) / ((np.float64(lo) + np.float64(hi)) * 0.5)))


def decide(a_start, a_end, b_start, b_end):
    """Sec. 1.1 sub-problem 1: does any pair intersect?  By the definition."""
    return count_bruteforce(a_start, a_end, b_start, b_end)[1] > 0


def pvalue(n_ge, n_shuffles):
    """One-sided empirical p-value (1 + n_ge) / (N + 1) as an fp64 division."""
    return (1.0 + float(n_ge)) / (float(n_shuffles) + 1.0)


def mc_expected_total(lengths, a_start, a_end, b_start, b_end):
    lengths, a_start, a_end, b_start, b_end = map(_u32, (lengths, a_start, a_end, b_start, b_end))
    return float(lib().oracle_mc_expected_total(lengths, len(lengths), a_start, a_end,
                                                len(a_start), b_start, b_end, len(b_start)))


def rmi_forward(params, u):
    params = np.ascontiguousarray(params, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    y = np.zeros(len(u), dtype=np.float64)
    lib().oracle_rmi_forward(params, u, len(u), y)
    return y


def rmi_loss_grad(params, u, t):
    params = np.ascontiguousarray(params, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    g = np.zeros(49, dtype=np.float64)
    loss = ctypes.c_double(0.0)
    lib().oracle_rmi_loss_grad(params, u, t, len(u), ctypes.byref(loss), g)
    return float(loss.value), g


def linear_fit(sorted_arr):
    a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    lib().oracle_linear_fit(_u32(sorted_arr), len(sorted_arr), ctypes.byref(a), ctypes.byref(b))
    return float(a.value), float(b.value)
