"""CPU checks of the C ABI: libbits.so loads, exports every entry point that
include/bits.h declares, and rejects bad host-side arguments before touching
a device.  No compute call is made here."""
import ctypes
import os
import re

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bits.h")
LIB = os.path.join(ROOT, "paper_1208_3407_amd", "libbits.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bits_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbits.so is not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_host_only_entry_points(lib):
    assert lib.bits_version() >= 1
    lib.bits_strerror.restype = ctypes.c_char_p
    assert lib.bits_strerror(4) == b"workspace too small"
    lib.bits_pvalue.restype = ctypes.c_double
    lib.bits_pvalue.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    assert lib.bits_pvalue(0, 9999) == 1.0 / 10000.0
    assert lib.bits_pvalue(3, 99) == 4.0 / 100.0
    sz = ctypes.c_size_t(0)
    assert lib.bits_ref_bytes(ctypes.c_uint64(1000), 13, 1, ctypes.byref(sz)) == 0 and sz.value > 8000
    assert lib.bits_ref_bytes(ctypes.c_uint64(2**33), 13, 0, ctypes.byref(sz)) == 1
    assert lib.bits_sort_ref_workspace(ctypes.c_uint64(10**6), ctypes.byref(sz)) == 0 and sz.value > 8 * 10**6
    assert lib.bits_mc_workspace(ctypes.c_uint64(100), ctypes.byref(sz)) == 0 and sz.value >= 1200


def test_ref_init_carves_block_on_host(lib):
    class Ref(ctypes.Structure):
        _fields_ = [("n", ctypes.c_uint64), ("depth", ctypes.c_uint32), ("learned", ctypes.c_uint32),
                    ("bs", ctypes.c_void_p), ("be", ctypes.c_void_p), ("tree", ctypes.c_void_p),
                    ("rmi", ctypes.c_void_p), ("heads", ctypes.c_void_p), ("status", ctypes.c_void_p),
                    ("block", ctypes.c_void_p), ("block_bytes", ctypes.c_size_t)]
    sz = ctypes.c_size_t(0)
    assert lib.bits_ref_bytes(ctypes.c_uint64(100), 13, 0, ctypes.byref(sz)) == 0
    r = Ref()
    base = 1 << 20    # a fake, 256-aligned address: ref_init only computes offsets
    assert lib.bits_ref_init(ctypes.c_void_p(base), sz, ctypes.c_uint64(100), 13, 0, ctypes.byref(r)) == 0
    assert r.depth == 6                      # floor(log2 100)
    assert r.status == base and r.tree > base and r.be > r.bs > r.tree
    assert r.be + 400 <= base + sz.value
    assert lib.bits_ref_init(ctypes.c_void_p(base), ctypes.c_size_t(sz.value - 1), ctypes.c_uint64(100), 13, 0,
                             ctypes.byref(r)) == 4
    assert lib.bits_ref_init(ctypes.c_void_p(base + 4), sz, ctypes.c_uint64(100), 13, 0, ctypes.byref(r)) == 1
    # a plain reference has no models but keeps the line heads (the 32-key node tier)
    hl = ((100 + 31) // 32 + 32 + 31) // 32 * 32
    assert r.rmi is None and r.heads > r.tree and r.bs >= r.heads + 2 * hl * 4 and r.heads % 256 == 0
    # learned: rmi (2 models of 128 + 4096 * 128 bytes), then the two line-head
    # arrays (ceil(n/32) heads + >= 32 padding, whole 128-byte lines), then B_S, B_E
    n = 100_000
    assert lib.bits_ref_bytes(ctypes.c_uint64(n), 13, 1, ctypes.byref(sz)) == 0
    assert lib.bits_ref_init(ctypes.c_void_p(base), sz, ctypes.c_uint64(n), 13, 1, ctypes.byref(r)) == 0
    hl = ((n + 31) // 32 + 32 + 31) // 32 * 32
    assert r.learned == 1 and r.heads >= r.rmi + 2 * (128 + 4096 * 128)
    assert r.bs >= r.heads + 2 * hl * 4 and r.heads % 256 == 0
    assert r.be + 4 * n <= base + sz.value


def test_bad_arguments_rejected_before_any_device_work(lib):
    # null reference / null query pointers with n > 0 -> BITS_E_ARG (1)
    assert lib.bits_count(None, None, None, ctypes.c_uint64(5), None, None, None) == 1
    assert lib.bits_count_per_query(None, None, None, ctypes.c_uint64(5), None, None, None, None) == 1
    lens = (ctypes.c_uint32 * 2)(10, 20)
    assert lib.bits_project(lens, 0, None, None, None, ctypes.c_uint64(0), None, None, None, None) == 1
    big = (ctypes.c_uint32 * 2)(0xF0000000, 0xF0000000)
    assert lib.bits_project(big, 2, None, None, None, ctypes.c_uint64(0), None, None, None, None) == 3
    assert lib.bits_rmi_leaf_grad(None, None, 5000, None, None, None, None) == 1
    assert lib.bits_batch_create(None, 0, None, None, None, 0, None, None, ctypes.c_size_t(0), None, None, None) == 1


def test_host_statistics(lib):
    """Host-side helpers of the Monte-Carlo statistics: tails and enrichment
    against closed forms and the oracle's definition (no device needed)."""
    import math
    import oracle
    lib.bits_pvalue_lower.restype = ctypes.c_double
    lib.bits_pvalue_lower.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.bits_pvalue_two_sided.restype = ctypes.c_double
    lib.bits_pvalue_two_sided.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.bits_enrichment.restype = ctypes.c_double
    lib.bits_enrichment.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    assert lib.bits_pvalue_lower(0, 9999) == 1.0 / 10000.0
    assert lib.bits_pvalue_two_sided(0, 9999, 9999) == 2.0 / 10000.0
    assert lib.bits_pvalue_two_sided(9999, 9999, 9999) == 1.0
    assert lib.bits_pvalue_two_sided(4, 99, 99) == 2.0 * 5.0 / 100.0
    assert lib.bits_enrichment(200, 100, 100) == 1.0
    assert lib.bits_enrichment(7, 7, 7) == 0.0
    assert lib.bits_enrichment(0, 5, 5) == -math.inf
    assert lib.bits_enrichment(5, 0, 0) == math.inf
    for obs, lo, hi in ((123456, 1000, 1003), (1, 2**40, 2**40 + 1), (10**12, 7, 8)):
        assert lib.bits_enrichment(obs, lo, hi) == oracle.enrichment(obs, lo, hi)


def test_binned_monte_carlo_host_checks(lib):
    """bits_mc_binned_workspace's size against the layout the header states,
    its argument checks, and the stage timer's host side (nothing recorded yet)."""
    from paper_1208_3407_amd import datagen
    lens = datagen.genome_g24().astype(np.uint32)
    cl = lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    na, n, batch = 1_000_000, 50_000_000, 1000
    sz, mc = ctypes.c_size_t(0), ctypes.c_size_t(0)
    U64 = ctypes.c_uint64
    assert lib.bits_mc_binned_workspace(U64(na), U64(n), cl, len(lens), batch, ctypes.byref(sz)) == 0
    assert lib.bits_mc_workspace(U64(na), ctypes.byref(mc)) == 0
    shift = 10
    while -(-int(lens.max()) // (1 << shift)) > 8192:
        shift += 1
    cells = int(sum(-(-int(x) // (1 << shift)) for x in lens))
    regions = min(cells, len(lens) + 2 * n // 8192)
    floor_bytes = mc.value + 8 * na + 8 * batch * na + (16 + 16 * batch) * regions + 24 * cells
    assert floor_bytes <= sz.value <= floor_bytes + 4 * cells + 64 * 1024
    small = ctypes.c_size_t(0)
    assert lib.bits_mc_binned_workspace(U64(na), U64(n), cl, len(lens), 256, ctypes.byref(small)) == 0
    assert small.value < sz.value
    for b in (0, 1025):
        assert lib.bits_mc_binned_workspace(U64(na), U64(n), cl, len(lens), b, ctypes.byref(sz)) == 1
    assert lib.bits_mc_binned_workspace(U64(2**32), U64(n), cl, len(lens), 8, ctypes.byref(sz)) == 1
    big = (ctypes.c_uint32 * 2)(0xF0000000, 0xF0000000)
    assert lib.bits_mc_binned_workspace(U64(na), U64(n), big, 2, 8, ctypes.byref(sz)) == 3
    assert lib.bits_mc_binned(None, None, None, U64(5), cl, len(lens), U64(7), U64(0), U64(4), 8, None,
                              ctypes.c_size_t(0), None, None, None, None, None, None) == 1
    ms = (ctypes.c_float * 3)(1.0, 1.0, 1.0)
    assert lib.bits_mc_binned_stage_ms(None) == 1
    assert lib.bits_mc_binned_timing(0) == 0 and lib.bits_mc_binned_stage_ms(ms) == 0
    assert list(ms) == [0.0, 0.0, 0.0]


def test_monte_carlo_wrappers_refuse_mismatched_buffers():
    """The binding's Monte-Carlo wrappers refuse query arrays of different
    lengths, an inverted shuffle range and output buffers the kernels would
    overrun, before any call into the library."""
    import torch
    from paper_1208_3407_amd import bits
    a = torch.zeros(10, dtype=torch.uint32)
    u64 = lambda n: torch.zeros(n, dtype=torch.uint64)   # noqa: E731
    ok = bits.MCResult(u64(8), u64(1), u64(1), u64(1))
    bits._check_mc_args(a, a, 2, 10, ok)
    bits._check_mc_args(a, a, 5, 5, None)
    with pytest.raises(bits.BitsError, match="differ in length"):
        bits._check_mc_args(a, a[:9], 0, 8, ok)
    with pytest.raises(bits.BitsError, match="s1 < s0"):
        bits._check_mc_args(a, a, 9, 8, None)
    with pytest.raises(bits.BitsError, match="totals holds 7"):
        bits._check_mc_args(a, a, 0, 8, bits.MCResult(u64(7), u64(1), u64(1), u64(1)))
    with pytest.raises(bits.BitsError, match="n_le holds 0"):
        bits._check_mc_args(a, a, 0, 8, bits.MCResult(u64(8), u64(1), u64(1), u64(0)))
    with pytest.raises(bits.BitsError, match="uint64"):
        bits._check_mc_args(a, a, 0, 8, bits.MCResult(torch.zeros(8, dtype=torch.int32), u64(1), u64(1), u64(1)))
    with pytest.raises(bits.BitsError, match="uint64"):
        bits._check_mc_args(a, a, 0, 4, bits.MCResult(u64(16)[::2], u64(1), u64(1), u64(1)))


def test_noalloc_monte_carlo_limit_checked_on_host(lib):
    """bits_mc_pvalue_noalloc refuses more queries than its device array
    holds before it looks at anything else (no device is touched)."""
    U64 = ctypes.c_uint64
    lim = int(re.search(r"#define BITS_NOALLOC_MAX_QUERIES \(1u << (\d+)\)", open(HEADER).read()).group(1))
    lens = (ctypes.c_uint32 * 1)(1000)
    assert lib.bits_mc_pvalue_noalloc(None, None, None, U64((1 << lim) + 1), lens, 1, U64(7), U64(0), U64(4),
                                      None, None, None, None, None, None) == 4
    assert lib.bits_mc_pvalue_noalloc(None, None, None, U64(2**40), lens, 1, U64(7), U64(0), U64(4),
                                      None, None, None, None, None, None) == 4
