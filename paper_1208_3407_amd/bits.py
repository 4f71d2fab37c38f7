"""Thin Python binding of libbits.so (include/bits.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies device memory (tensors on the current HIP device) and the
current stream.  The functions carry the C entry points' names.  There is no
CPU fallback: importing this module raises if ``libbits.so`` has not been
built, and every call raises if no GPU is present or the library reports an
error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbits.so")

BITS_OK = 0
BITS_FLAG_INTERVAL = 0x1
BITS_FLAG_CHROM = 0x2
BITS_FLAG_ENUM = 0x4
BITS_MAX_DEPTH = 13
BITS_NOALLOC_MAX_QUERIES = 1 << 20
BITS_PATH_AUTO, BITS_PATH_PLAIN, BITS_PATH_LEARNED, BITS_PATH_TIERED = 0, 1, 2, 3
DEPTH_FROM_REF = 0xFFFFFFFF

_u32, _u64, _vp, _sz = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t


class bits_launch(ctypes.Structure):
    _fields_ = [("block", _u32), ("qpl", _u32), ("depth", _u32), ("grid", _u32), ("path", _u32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class bits_ref(ctypes.Structure):
    _fields_ = [("n", _u64), ("depth", _u32), ("learned", _u32), ("bs", _vp), ("be", _vp), ("tree", _vp),
                ("rmi", _vp), ("heads", _vp), ("status", _vp), ("block", _vp), ("block_bytes", _sz)]


class bits_train(ctypes.Structure):
    _fields_ = [("epochs", _u32), ("max_points", _u32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float)]


class bits_rmi_stats(ctypes.Structure):
    _fields_ = [("mean_window", ctypes.c_double), ("max_window", _u32), ("empty_leaves", _u32),
                ("mean_loss", ctypes.c_double), ("fallbacks", _u64)]


# byte layout of one learned model (bits_rmi_model): 128-byte header + 4096 leaves of 128 bytes
RMI_HEADER_BYTES = 128
RMI_LEAF_BYTES = 128
RMI_LEAVES = 4096
RMI_MODEL_BYTES = RMI_HEADER_BYTES + RMI_LEAVES * RMI_LEAF_BYTES


class BitsError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbits.so is not built (run __graft_entry__.build() or "
                          "python -m paper_1208_3407_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sig = {
        "bits_version": ([], ctypes.c_int),
        "bits_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "bits_get_status": ([_vp, _vp, P(_u32)], ctypes.c_int),
        "bits_clear_status": ([_vp, _vp], ctypes.c_int),
        "bits_project": ([P(_u32), _u32, _vp, _vp, _vp, _u64, _vp, _vp, _vp, _vp], ctypes.c_int),
        "bits_ref_bytes": ([_u64, _u32, ctypes.c_int, P(_sz)], ctypes.c_int),
        "bits_ref_init": ([_vp, _sz, _u64, _u32, ctypes.c_int, P(bits_ref)], ctypes.c_int),
        "bits_sort_ref_workspace": ([_u64, P(_sz)], ctypes.c_int),
        "bits_sort_ref": ([_vp, _vp, P(bits_ref), _vp, _sz, P(bits_train), _vp], ctypes.c_int),
        "bits_sort_refs_workspace": ([P(_u64), _u32, P(_sz)], ctypes.c_int),
        "bits_sort_refs": ([P(_vp), P(_vp), P(bits_ref), _u32, _vp, _sz, P(bits_train), _vp], ctypes.c_int),
        "bits_rmi_info": ([P(bits_ref), _vp, P(bits_rmi_stats)], ctypes.c_int),
        "bits_count_per_query": ([P(bits_ref), _vp, _vp, _u64, _vp, _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_count": ([P(bits_ref), _vp, _vp, _u64, _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_mc_workspace": ([_u64, P(_sz)], ctypes.c_int),
        "bits_mc_pvalue": ([P(bits_ref), _vp, _vp, _u64, P(_u32), _u32, _u64, _u64, _u64, _vp, _sz, _vp, _vp,
                            _vp, _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_mc_pvalue_noalloc": ([P(bits_ref), _vp, _vp, _u64, P(_u32), _u32, _u64, _u64, _u64, _vp, _vp, _vp,
                                    _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_pvalue": ([_u64, _u64], ctypes.c_double),
        "bits_batch_workspace": ([P(_u64), _u32, _u32, P(_sz)], ctypes.c_int),
        "bits_batch_create": ([P(bits_ref), _u32, P(_vp), P(_vp), P(_u64), _u32, _vp, _vp, _sz, P(bits_launch),
                               _vp, P(_vp)], ctypes.c_int),
        "bits_batch_run": ([_vp, _vp], ctypes.c_int),
        "bits_batch_destroy": ([_vp], ctypes.c_int),
        "bits_autotune_count": ([P(bits_ref), _vp, _vp, _u64, _vp, _u32, P(bits_launch), P(ctypes.c_float), _vp],
                                ctypes.c_int),
        "bits_autotune_batch": ([P(bits_ref), _u32, P(_vp), P(_vp), P(_u64), _u32, _u32, _vp, _vp, _sz,
                                 P(bits_launch), P(ctypes.c_float), _vp], ctypes.c_int),
        "bits_rmi_leaf_grad": ([_vp, _vp, _u32, _vp, _vp, _vp, _vp], ctypes.c_int),
        "bits_rmi_window": ([P(bits_ref), _u32, _vp, _u64, _vp, _vp, _vp], ctypes.c_int),
        "bits_enum_index_bytes": ([_u64, P(_sz)], ctypes.c_int),
        "bits_enum_index_workspace": ([_u64, P(_sz)], ctypes.c_int),
        "bits_enum_index_build": ([_vp, _vp, _u64, _vp, _sz, _vp, _sz, _vp], ctypes.c_int),
        "bits_scan_workspace": ([_u64, P(_sz)], ctypes.c_int),
        "bits_scan_counts": ([_vp, _u64, _vp, _vp, _sz, _vp], ctypes.c_int),
        "bits_mc_resort_workspace": ([_u64, _u32, P(_sz)], ctypes.c_int),
        "bits_mc_binned_workspace": ([_u64, _u64, P(_u32), _u32, _u32, P(_sz)], ctypes.c_int),
        "bits_mc_binned_timing": ([ctypes.c_int], ctypes.c_int),
        "bits_mc_binned_stage_ms": ([P(ctypes.c_float)], ctypes.c_int),
        "bits_mc_binned": ([P(bits_ref), _vp, _vp, _u64, P(_u32), _u32, _u64, _u64, _u64, _u32, _vp, _sz, _vp, _vp,
                            _vp, _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_mc_resort": ([_vp, _vp, _u64, _vp, _vp, _u64, P(_u32), _u32, _u64, _u64, _u64, _u32, _vp, _sz, _vp,
                            _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
        "bits_pvalue_lower": ([_u64, _u64], ctypes.c_double),
        "bits_pvalue_two_sided": ([_u64, _u64, _u64], ctypes.c_double),
        "bits_mc_median": ([_vp, _u64, _vp, _vp, _vp], ctypes.c_int),
        "bits_enrichment": ([_u64, _u64, _u64], ctypes.c_double),
        "bits_decide": ([P(bits_ref), _vp, _vp, _u64, _vp, _vp, P(bits_launch), _vp], ctypes.c_int),
        "bits_enum_counts": ([P(bits_ref), _vp, _vp, _u64, _vp, _vp, _vp, _vp, _sz, P(bits_launch), _vp],
                             ctypes.c_int),
        "bits_enumerate": ([_vp, _u64, _vp, _vp, _u64, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


_lib = _load()


def _check(rc: int, what: str):
    if rc != BITS_OK:
        raise BitsError("%s: %s (status %d)" % (what, _lib.bits_strerror(rc).decode(), rc))


def _device() -> torch.device:
    if not torch.cuda.is_available():
        raise BitsError("no GPU: libbits.so runs on an AMD Instinct (gfx950) device only")
    return torch.device("cuda", torch.cuda.current_device())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _u32_dev(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise BitsError("%s must be a device tensor" % name)
    if t.dtype == torch.int32:
        t = t.view(torch.uint32)
    if t.dtype != torch.uint32:
        raise BitsError("%s must be uint32 (or int32 reinterpreted), got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise BitsError("%s must be contiguous" % name)
    return t


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _scratch(nbytes: int, dev) -> torch.Tensor:
    """Caller-owned device bytes, 256-byte aligned (a view into a slightly larger tensor)."""
    nbytes = max(int(nbytes), 1)
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-raw.data_ptr()) % 256
    return raw[off:off + nbytes]


def bits_version() -> int:
    return int(_lib.bits_version())


def bits_strerror(status: int) -> str:
    return _lib.bits_strerror(int(status)).decode()


def bits_get_status(status_tensor_or_ref, stream=None) -> int:
    t = status_tensor_or_ref
    ptr = t.c.status if isinstance(t, Ref) else t.data_ptr()
    out = _u32(0)
    _check(_lib.bits_get_status(ctypes.c_void_p(ptr), _stream(stream), ctypes.byref(out)), "bits_get_status")
    return int(out.value)


def bits_clear_status(status_tensor_or_ref, stream=None):
    t = status_tensor_or_ref
    ptr = t.c.status if isinstance(t, Ref) else t.data_ptr()
    _check(_lib.bits_clear_status(ctypes.c_void_p(ptr), _stream(stream)), "bits_clear_status")


def _host_u32(values) -> ctypes.Array:
    vals = [int(v) for v in values]
    return (_u32 * len(vals))(*vals)


def bits_project(chrom_len, chrom, lstart, lend, status: Optional[torch.Tensor] = None, stream=None):
    """Projection of chromosome-local intervals to the 1-D genome (device)."""
    dev = _device()
    chrom, lstart, lend = (_u32_dev(x, n) for x, n in ((chrom, "chrom"), (lstart, "lstart"), (lend, "lend")))
    n = chrom.numel()
    gs = torch.empty(n, dtype=torch.uint32, device=dev)
    ge = torch.empty(n, dtype=torch.uint32, device=dev)
    cl = _host_u32(chrom_len)
    _check(_lib.bits_project(cl, len(cl), _ptr(chrom), _ptr(lstart), _ptr(lend), n, _ptr(gs), _ptr(ge),
                             _ptr(status), _stream(stream)), "bits_project")
    return gs, ge


@dataclass
class Ref:
    """A reference index: the caller-owned device block and its descriptor."""
    c: bits_ref
    block: torch.Tensor

    @property
    def n(self) -> int:
        return int(self.c.n)

    @property
    def depth(self) -> int:
        return int(self.c.depth)

    @property
    def learned(self) -> bool:
        return bool(self.c.learned)

    def _view(self, addr: int, count: int, dtype) -> torch.Tensor:
        off = addr - self.block.data_ptr()
        item = torch.tensor([], dtype=dtype).element_size()
        return self.block[off:off + count * item].view(dtype)

    def sorted_starts(self) -> torch.Tensor:
        return self._view(self.c.bs, self.n, torch.uint32) if self.n else torch.empty(0, dtype=torch.uint32)

    def sorted_ends(self) -> torch.Tensor:
        return self._view(self.c.be, self.n, torch.uint32) if self.n else torch.empty(0, dtype=torch.uint32)

    def tree(self) -> torch.Tensor:
        return self._view(self.c.tree, 2 << self.depth, torch.uint32)

    def heads_len(self) -> int:
        """Entries of one line-head array (learned references)."""
        return ((self.n + 31) // 32 + 32 + 31) // 32 * 32

    def heads(self) -> torch.Tensor:
        """Line heads [2, heads_len]: first key of every 128-byte line of B_S, B_E."""
        if not self.learned:
            raise BitsError("the reference has no learned index")
        return self._view(self.c.heads, 2 * self.heads_len(), torch.uint32).view(2, -1)

    def rmi_bytes(self) -> torch.Tensor:
        if not self.learned:
            raise BitsError("reference has no learned index")
        return self._view(self.c.rmi, 2 * RMI_MODEL_BYTES, torch.uint8)

    def status_words(self) -> torch.Tensor:
        return self._view(self.c.status, 64, torch.uint32)


def bits_ref_bytes(n: int, depth: int = BITS_MAX_DEPTH, learned: bool = False) -> int:
    out = _sz(0)
    _check(_lib.bits_ref_bytes(int(n), int(depth), int(bool(learned)), ctypes.byref(out)), "bits_ref_bytes")
    return int(out.value)


def bits_ref_init(n: int, depth: int = BITS_MAX_DEPTH, learned: bool = False, block: Optional[torch.Tensor] = None) -> Ref:
    dev = _device()
    nbytes = bits_ref_bytes(n, depth, learned)
    if block is None:
        block = _scratch(nbytes, dev)
    c = bits_ref()
    _check(_lib.bits_ref_init(ctypes.c_void_p(block.data_ptr()), block.numel() * block.element_size(), int(n),
                              int(depth), int(bool(learned)), ctypes.byref(c)), "bits_ref_init")
    return Ref(c, block)


def _train(train: Optional[dict]):
    if train is None:
        return None
    t = bits_train(int(train.get("epochs", 300)), int(train.get("max_points", 256)), float(train.get("lr", 2e-3)),
                   float(train.get("beta1", 0.9)), float(train.get("beta2", 0.999)))
    return ctypes.byref(t)


def bits_sort_ref_workspace(n: int) -> int:
    out = _sz(0)
    _check(_lib.bits_sort_ref_workspace(int(n), ctypes.byref(out)), "bits_sort_ref_workspace")
    return int(out.value)


def bits_sort_ref(b_start, b_end, depth: int = BITS_MAX_DEPTH, learned: bool = False, train: Optional[dict] = None,
                  ref: Optional[Ref] = None, workspace: Optional[torch.Tensor] = None, stream=None) -> Ref:
    """Sorts B_S and B_E on the device, builds the top tree (and the learned index)."""
    dev = _device()
    b_start, b_end = _u32_dev(b_start, "b_start"), _u32_dev(b_end, "b_end")
    if b_start.numel() != b_end.numel():
        raise BitsError("b_start and b_end differ in length")
    n = b_start.numel()
    if ref is None:
        ref = bits_ref_init(n, depth, learned)
    if workspace is None:
        workspace = _scratch(bits_sort_ref_workspace(n), dev)
    _check(_lib.bits_sort_ref(_ptr(b_start), _ptr(b_end), ctypes.byref(ref.c), _ptr(workspace),
                              workspace.numel(), _train(train), _stream(stream)), "bits_sort_ref")
    ref._keepalive = workspace  # the kernels may still be reading it on the stream
    return ref


def bits_sort_refs(sets: Sequence[Tuple[torch.Tensor, torch.Tensor]], depth: int = BITS_MAX_DEPTH,
                   learned: bool = False, train: Optional[dict] = None, stream=None) -> List[Ref]:
    """Sorts several references in one segmented sort."""
    dev = _device()
    sets = [(_u32_dev(s, "b_start"), _u32_dev(e, "b_end")) for s, e in sets]
    refs = [bits_ref_init(s.numel(), depth, learned) for s, _ in sets]
    k = len(sets)
    ns = (_u64 * k)(*[s.numel() for s, _ in sets])
    out = _sz(0)
    _check(_lib.bits_sort_refs_workspace(ns, k, ctypes.byref(out)), "bits_sort_refs_workspace")
    ws = _scratch(out.value, dev)
    starts = (_vp * k)(*[_ptr(s).value for s, _ in sets])
    ends = (_vp * k)(*[_ptr(e).value for _, e in sets])
    arr = (bits_ref * k)(*[r.c for r in refs])
    _check(_lib.bits_sort_refs(starts, ends, arr, k, _ptr(ws), ws.numel(), _train(train), _stream(stream)),
           "bits_sort_refs")
    for r in refs:
        r._keepalive = ws
    return refs


def _launch(launch) -> Optional[bits_launch]:
    if launch is None:
        return None
    if isinstance(launch, bits_launch):
        return launch
    return bits_launch(int(launch.get("block", 0)), int(launch.get("qpl", 0)),
                       int(launch.get("depth", DEPTH_FROM_REF)), int(launch.get("grid", 0)),
                       int(launch.get("path", BITS_PATH_AUTO)))


def _lp(launch):
    lp = _launch(launch)
    return ctypes.byref(lp) if lp is not None else None


def bits_count_per_query(ref: Ref, a_start, a_end, launch=None, counts: Optional[torch.Tensor] = None,
                         total: Optional[torch.Tensor] = None, stream=None):
    """Per-interval counts (uint32[na]) and their uint64 total (1-element tensor)."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    na = a_start.numel()
    if a_end.numel() != na:
        raise BitsError("a_start and a_end differ in length")
    if counts is None:
        counts = torch.empty(na, dtype=torch.uint32, device=dev)
    if total is None:
        total = torch.empty(1, dtype=torch.uint64, device=dev)
    _check(_lib.bits_count_per_query(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), na, _ptr(counts),
                                     ctypes.c_void_p(total.data_ptr()), _lp(launch), _stream(stream)),
           "bits_count_per_query")
    return counts, total


def bits_count(ref: Ref, a_start, a_end, launch=None, total: Optional[torch.Tensor] = None, stream=None):
    """Total count (uint64, 1-element device tensor)."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    if a_end.numel() != a_start.numel():
        raise BitsError("a_start and a_end differ in length")
    if total is None:
        total = torch.empty(1, dtype=torch.uint64, device=dev)
    _check(_lib.bits_count(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), a_start.numel(),
                           ctypes.c_void_p(total.data_ptr()), _lp(launch), _stream(stream)), "bits_count")
    return total


def bits_mc_workspace(na: int) -> int:
    out = _sz(0)
    _check(_lib.bits_mc_workspace(int(na), ctypes.byref(out)), "bits_mc_workspace")
    return int(out.value)


@dataclass
class MCResult:
    totals: torch.Tensor     # uint64[s1 - s0]
    observed: torch.Tensor   # uint64[1]
    n_ge: torch.Tensor       # uint64[1]
    n_le: torch.Tensor       # uint64[1]


def _check_mc_args(a_start: torch.Tensor, a_end: torch.Tensor, s0: int, s1: int, out: Optional["MCResult"]):
    """Host-side checks shared by the Monte-Carlo wrappers: equal query array
    lengths, a shuffle range with s0 <= s1, and caller-supplied outputs large
    enough for the kernels to write (uint64, contiguous, totals >= s1 - s0)."""
    if a_end.numel() != a_start.numel():
        raise BitsError("a_start and a_end differ in length")
    if int(s1) < int(s0):
        raise BitsError("shuffle range [s0, s1) has s1 < s0")
    if out is None:
        return
    for name, t, need in (("totals", out.totals, int(s1) - int(s0)), ("observed", out.observed, 1),
                          ("n_ge", out.n_ge, 1), ("n_le", out.n_le, 1)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.uint64 or not t.is_contiguous():
            raise BitsError("out.%s must be a contiguous uint64 tensor" % name)
        if t.numel() < need:
            raise BitsError("out.%s holds %d values, needs %d" % (name, t.numel(), need))


def bits_mc_pvalue(ref: Ref, a_start, a_end, chrom_len, seed: int, s0: int, s1: int, launch=None,
                   workspace: Optional[torch.Tensor] = None, out: Optional[MCResult] = None, stream=None) -> MCResult:
    """Monte-Carlo shuffles [s0, s1) of A against the reference, in one persistent launch."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    _check_mc_args(a_start, a_end, s0, s1, out)
    na = a_start.numel()
    if workspace is None:
        workspace = _scratch(bits_mc_workspace(na), dev)
    if out is None:
        out = MCResult(torch.empty(max(s1 - s0, 0), dtype=torch.uint64, device=dev),
                       torch.empty(1, dtype=torch.uint64, device=dev), torch.empty(1, dtype=torch.uint64, device=dev),
                       torch.empty(1, dtype=torch.uint64, device=dev))
    cl = _host_u32(chrom_len)
    _check(_lib.bits_mc_pvalue(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), na, cl, len(cl), int(seed), int(s0),
                               int(s1), _ptr(workspace), workspace.numel(), _ptr(out.totals),
                               ctypes.c_void_p(out.observed.data_ptr()), ctypes.c_void_p(out.n_ge.data_ptr()),
                               ctypes.c_void_p(out.n_le.data_ptr()), _lp(launch), _stream(stream)), "bits_mc_pvalue")
    out._keepalive = workspace
    return out


def bits_mc_pvalue_noalloc(ref: Ref, a_start, a_end, chrom_len, seed: int, s0: int, s1: int, out: MCResult,
                           launch=None, stream=None) -> MCResult:
    """bits_mc_pvalue with its query table in the library's own device array (no workspace,
    no allocation in the call); `out` is required (its tensors are the call's outputs)."""
    _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    if out is None:
        raise BitsError("bits_mc_pvalue_noalloc: out is required")
    _check_mc_args(a_start, a_end, s0, s1, out)
    if a_start.numel() > BITS_NOALLOC_MAX_QUERIES:
        raise BitsError("bits_mc_pvalue_noalloc: at most %d queries" % BITS_NOALLOC_MAX_QUERIES)
    cl = _host_u32(chrom_len)
    _check(_lib.bits_mc_pvalue_noalloc(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), a_start.numel(), cl, len(cl),
                                       int(seed), int(s0), int(s1), _ptr(out.totals),
                                       ctypes.c_void_p(out.observed.data_ptr()), ctypes.c_void_p(out.n_ge.data_ptr()),
                                       ctypes.c_void_p(out.n_le.data_ptr()), _lp(launch), _stream(stream)),
           "bits_mc_pvalue_noalloc")
    return out


def bits_mc_binned_workspace(na: int, n: int, chrom_len, batch: int) -> int:
    out = _sz(0)
    cl = _host_u32(chrom_len)
    _check(_lib.bits_mc_binned_workspace(int(na), int(n), cl, len(cl), int(batch), ctypes.byref(out)),
           "bits_mc_binned_workspace")
    return int(out.value)


def bits_mc_binned(ref: Ref, a_start, a_end, chrom_len, seed: int, s0: int, s1: int, batch: int = 256,
                   launch=None, workspace: Optional[torch.Tensor] = None, out: Optional[MCResult] = None,
                   stream=None) -> MCResult:
    """Monte-Carlo shuffles [s0, s1) of A against the reference, binned by genome region and
    counted in LDS, `batch` shuffles per pass; same totals as bits_mc_pvalue."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    _check_mc_args(a_start, a_end, s0, s1, out)
    na = a_start.numel()
    if workspace is None:
        workspace = _scratch(bits_mc_binned_workspace(na, ref.n, chrom_len, batch), dev)
    if out is None:
        out = MCResult(torch.empty(max(s1 - s0, 1), dtype=torch.uint64, device=dev)[:max(s1 - s0, 0)],
                       torch.empty(1, dtype=torch.uint64, device=dev), torch.empty(1, dtype=torch.uint64, device=dev),
                       torch.empty(1, dtype=torch.uint64, device=dev))
    cl = _host_u32(chrom_len)
    _check(_lib.bits_mc_binned(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), na, cl, len(cl), int(seed), int(s0),
                               int(s1), int(batch), _ptr(workspace), workspace.numel(), _ptr(out.totals),
                               ctypes.c_void_p(out.observed.data_ptr()), ctypes.c_void_p(out.n_ge.data_ptr()),
                               ctypes.c_void_p(out.n_le.data_ptr()), _lp(launch), _stream(stream)), "bits_mc_binned")
    out._keepalive = workspace
    return out


def bits_mc_binned_timing(enable: bool) -> None:
    _check(_lib.bits_mc_binned_timing(1 if enable else 0), "bits_mc_binned_timing")


def bits_mc_binned_stage_ms() -> dict:
    """Device milliseconds of the last timed bits_mc_binned call, per stage."""
    ms = (ctypes.c_float * 3)()
    _check(_lib.bits_mc_binned_stage_ms(ms), "bits_mc_binned_stage_ms")
    return {"place": float(ms[0]), "search": float(ms[1]), "reduce": float(ms[2])}


def bits_mc_resort_workspace(nb: int, batch: int) -> int:
    n = _sz(0)
    _check(_lib.bits_mc_resort_workspace(nb, batch, ctypes.byref(n)), "bits_mc_resort_workspace")
    return n.value


def bits_mc_resort(a_start, a_end, b_start, b_end, chrom_len, seed: int, s0: int, s1: int, batch: int = 64,
                   workspace: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                   stream=None) -> "MCResult":
    """The paper's Monte-Carlo orientation: B randomised and re-sorted every round, A fixed."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    b_start, b_end = _u32_dev(b_start, "b_start"), _u32_dev(b_end, "b_end")
    nb = b_start.numel()
    if a_end.numel() != a_start.numel() or b_end.numel() != nb:
        raise BitsError("start and end arrays differ in length")
    if workspace is None:
        workspace = _scratch(bits_mc_resort_workspace(nb, batch), dev)
    lens = _host_u32(chrom_len)
    ns = s1 - s0
    out = MCResult(torch.empty(max(ns, 1), dtype=torch.uint64, device=dev)[:ns],
                   torch.empty(1, dtype=torch.uint64, device=dev), torch.empty(1, dtype=torch.uint64, device=dev),
                   torch.empty(1, dtype=torch.uint64, device=dev))
    _check(_lib.bits_mc_resort(_ptr(a_start), _ptr(a_end), a_start.numel(), _ptr(b_start), _ptr(b_end), nb, lens,
                               len(lens), seed, s0, s1, batch, _ptr(workspace), workspace.numel(),
                               _ptr(out.totals), _ptr(out.observed), _ptr(out.n_ge), _ptr(out.n_le), _ptr(status),
                               _stream(stream)), "bits_mc_resort")
    return out


def bits_pvalue_lower(n_le: int, n_shuffles: int) -> float:
    return float(_lib.bits_pvalue_lower(n_le, n_shuffles))


def bits_pvalue_two_sided(n_ge: int, n_le: int, n_shuffles: int) -> float:
    return float(_lib.bits_pvalue_two_sided(n_ge, n_le, n_shuffles))


def bits_mc_median(totals: torch.Tensor, stream=None):
    """(lo, hi) middle order statistics of the uint64 per-shuffle totals (1-element device tensors)."""
    dev = _device()
    if not totals.is_cuda or totals.dtype != torch.uint64 or not totals.is_contiguous():
        raise BitsError("totals must be a contiguous uint64 device tensor")
    lo = torch.empty(1, dtype=torch.uint64, device=dev)
    hi = torch.empty(1, dtype=torch.uint64, device=dev)
    _check(_lib.bits_mc_median(_ptr(totals), totals.numel(), _ptr(lo), _ptr(hi), _stream(stream)), "bits_mc_median")
    return lo, hi


def bits_enrichment(observed: int, median_lo: int, median_hi: int) -> float:
    return float(_lib.bits_enrichment(observed, median_lo, median_hi))


def bits_decide(ref: Ref, a_start, a_end, launch=None, stream=None):
    """Decision (1-element uint32 found, 1-element uint64 witness) device tensors."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    if a_end.numel() != a_start.numel():
        raise BitsError("a_start and a_end differ in length")
    found = torch.empty(1, dtype=torch.uint32, device=dev)
    witness = torch.empty(1, dtype=torch.uint64, device=dev)
    _check(_lib.bits_decide(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), a_start.numel(), _ptr(found),
                            _ptr(witness), _lp(launch), _stream(stream)), "bits_decide")
    return found, witness


def bits_pvalue(n_ge: int, n_shuffles: int) -> float:
    return float(_lib.bits_pvalue(int(n_ge), int(n_shuffles)))


class BatchPlan:
    def __init__(self, handle, totals, workspace, keep):
        self.handle = handle
        self.totals = totals
        self.workspace = workspace
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None):
            _lib.bits_batch_destroy(self.handle)
            self.handle = None


def bits_batch_workspace(na: Sequence[int], n_ref: int) -> int:
    k = len(na)
    arr = (_u64 * k)(*[int(x) for x in na])
    out = _sz(0)
    _check(_lib.bits_batch_workspace(arr, k, int(n_ref), ctypes.byref(out)), "bits_batch_workspace")
    return int(out.value)


def bits_batch_create(refs: Sequence[Ref], queries: Sequence[Tuple[torch.Tensor, torch.Tensor]], launch=None,
                      stream=None) -> BatchPlan:
    """Plan over all (query set, reference) pairs, captured in a HIP graph."""
    dev = _device()
    queries = [(_u32_dev(s, "a_start"), _u32_dev(e, "a_end")) for s, e in queries]
    nq, nr = len(queries), len(refs)
    na = [s.numel() for s, _ in queries]
    ws = _scratch(bits_batch_workspace(na, nr), dev)
    totals = torch.empty(nq * nr, dtype=torch.uint64, device=dev)
    rarr = (bits_ref * nr)(*[r.c for r in refs])
    sp = (_vp * nq)(*[_ptr(s).value for s, _ in queries])
    ep = (_vp * nq)(*[_ptr(e).value for _, e in queries])
    nav = (_u64 * nq)(*na)
    h = _vp(0)
    _check(_lib.bits_batch_create(rarr, nr, sp, ep, nav, nq, ctypes.c_void_p(totals.data_ptr()), _ptr(ws),
                                  ws.numel(), _lp(launch), _stream(stream), ctypes.byref(h)), "bits_batch_create")
    return BatchPlan(h, totals, ws, (list(refs), queries))


def bits_batch_run(plan: BatchPlan, stream=None) -> torch.Tensor:
    _check(_lib.bits_batch_run(plan.handle, _stream(stream)), "bits_batch_run")
    return plan.totals


def bits_batch_destroy(plan: BatchPlan):
    if plan.handle:
        _check(_lib.bits_batch_destroy(plan.handle), "bits_batch_destroy")
        plan.handle = None


def bits_autotune_count(ref: Ref, a_start, a_end, path: int = BITS_PATH_PLAIN, stream=None):
    """Fastest launch shape for bits_count on these queries (timed with HIP events)."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    total = torch.empty(1, dtype=torch.uint64, device=dev)
    best = bits_launch()
    ms = ctypes.c_float(0.0)
    _check(_lib.bits_autotune_count(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), a_start.numel(),
                                    ctypes.c_void_p(total.data_ptr()), int(path), ctypes.byref(best),
                                    ctypes.byref(ms), _stream(stream)), "bits_autotune_count")
    return best, float(ms.value)


def bits_autotune_batch(refs: Sequence[Ref], queries: Sequence[Tuple[torch.Tensor, torch.Tensor]],
                        path: int = BITS_PATH_PLAIN, stream=None):
    """Fastest launch shape of the batch plan over these (query set, reference) pairs:
    every candidate shape's graph replay timed with HIP events.  Pass a prefix of each
    query set to bound the tuning time."""
    dev = _device()
    queries = [(_u32_dev(s, "a_start"), _u32_dev(e, "a_end")) for s, e in queries]
    nq, nr = len(queries), len(refs)
    na = [s.numel() for s, _ in queries]
    ws = _scratch(bits_batch_workspace(na, nr), dev)
    totals = torch.empty(nq * nr, dtype=torch.uint64, device=dev)
    rarr = (bits_ref * nr)(*[r.c for r in refs])
    sp = (_vp * nq)(*[_ptr(s).value for s, _ in queries])
    ep = (_vp * nq)(*[_ptr(e).value for _, e in queries])
    nav = (_u64 * nq)(*na)
    best = bits_launch()
    ms = ctypes.c_float(0.0)
    _check(_lib.bits_autotune_batch(rarr, nr, sp, ep, nav, nq, int(path), ctypes.c_void_p(totals.data_ptr()),
                                    _ptr(ws), ws.numel(), ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
           "bits_autotune_batch")
    return best, float(ms.value)

def bits_rmi_info(ref: Ref, stream=None) -> dict:
    st = bits_rmi_stats()
    _check(_lib.bits_rmi_info(ctypes.byref(ref.c), _stream(stream), ctypes.byref(st)), "bits_rmi_info")
    return {"mean_window": st.mean_window, "max_window": int(st.max_window), "empty_leaves": int(st.empty_leaves),
            "mean_loss": st.mean_loss, "fallbacks": int(st.fallbacks)}


def bits_rmi_leaf_grad(u: torch.Tensor, t: torch.Tensor, params: torch.Tensor, stream=None):
    """Loss and gradient of one leaf model, by the training kernel's device code."""
    dev = _device()
    for x, nm in ((u, "u"), (t, "t"), (params, "params")):
        if not x.is_cuda or x.dtype != torch.float32 or not x.is_contiguous():
            raise BitsError("%s must be a contiguous float32 device tensor" % nm)
    grad = torch.empty(49, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    _check(_lib.bits_rmi_leaf_grad(_ptr(u), _ptr(t), u.numel(), _ptr(params), _ptr(grad), _ptr(loss),
                                   _stream(stream)), "bits_rmi_leaf_grad")
    return grad, loss


def bits_rmi_window(ref: Ref, which: int, x, stream=None):
    """Learned-path search windows [lo, hi] for keys x (device code of the searches)."""
    dev = _device()
    x = _u32_dev(x, "x")
    lo = torch.empty(x.numel(), dtype=torch.uint32, device=dev)
    hi = torch.empty(x.numel(), dtype=torch.uint32, device=dev)
    _check(_lib.bits_rmi_window(ctypes.byref(ref.c), int(which), _ptr(x), x.numel(), _ptr(lo), _ptr(hi),
                                _stream(stream)), "bits_rmi_window")
    return lo, hi


# ---------------------------------------------------------------- enumeration

@dataclass
class EnumIndex:
    """B sorted by start with each interval's end and input index (caller-owned block)."""
    n: int
    block: torch.Tensor

    def _region(self, k: int) -> torch.Tensor:
        stride = (self.n * 4 + 255) // 256 * 256
        return self.block[k * stride:k * stride + self.n * 4].view(torch.uint32)

    def starts(self) -> torch.Tensor:
        return self._region(0)

    def ends(self) -> torch.Tensor:
        return self._region(1)

    def ids(self) -> torch.Tensor:
        return self._region(2)


def bits_enum_index_build(b_start, b_end, stream=None) -> EnumIndex:
    """Enumeration index over B (stable sort by start; ends and input indices moved along)."""
    dev = _device()
    b_start, b_end = _u32_dev(b_start, "b_start"), _u32_dev(b_end, "b_end")
    n = b_start.numel()
    if b_end.numel() != n:
        raise BitsError("b_start and b_end differ in length")
    nb, nw = _sz(0), _sz(0)
    _check(_lib.bits_enum_index_bytes(n, ctypes.byref(nb)), "bits_enum_index_bytes")
    _check(_lib.bits_enum_index_workspace(n, ctypes.byref(nw)), "bits_enum_index_workspace")
    block = _scratch(nb.value, dev)
    ws = _scratch(nw.value, dev)
    _check(_lib.bits_enum_index_build(_ptr(b_start), _ptr(b_end), n, _ptr(block), nb.value, _ptr(ws), nw.value,
                                      _stream(stream)), "bits_enum_index_build")
    return EnumIndex(n, block)


def bits_scan_counts(counts, stream=None) -> torch.Tensor:
    """uint64[n + 1] exclusive prefix sums of uint32 counts; the last entry is the total."""
    dev = _device()
    counts = _u32_dev(counts, "counts")
    n = counts.numel()
    nw = _sz(0)
    _check(_lib.bits_scan_workspace(n, ctypes.byref(nw)), "bits_scan_workspace")
    ws = _scratch(nw.value, dev)
    offsets = torch.empty(n + 1, dtype=torch.uint64, device=dev)
    _check(_lib.bits_scan_counts(_ptr(counts), n, _ptr(offsets), _ptr(ws), nw.value, _stream(stream)),
           "bits_scan_counts")
    return offsets


def bits_enum_counts(ref: Ref, a_start, a_end, launch=None, stream=None):
    """Enumeration step 1: (counts uint32[na], first uint32[na], offsets uint64[na + 1])."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    na = a_start.numel()
    if a_end.numel() != na:
        raise BitsError("a_start and a_end differ in length")
    counts = torch.empty(na, dtype=torch.uint32, device=dev)
    first = torch.empty(na, dtype=torch.uint32, device=dev)
    offsets = torch.empty(na + 1, dtype=torch.uint64, device=dev)
    nw = _sz(0)
    _check(_lib.bits_scan_workspace(na, ctypes.byref(nw)), "bits_scan_workspace")
    ws = _scratch(nw.value, dev)
    _check(_lib.bits_enum_counts(ctypes.byref(ref.c), _ptr(a_start), _ptr(a_end), na, _ptr(counts), _ptr(first),
                                 _ptr(offsets), _ptr(ws), nw.value, _lp(launch), _stream(stream)), "bits_enum_counts")
    return counts, first, offsets


def bits_enumerate(index: EnumIndex, a_start, a_end, counts, offsets, first: Optional[torch.Tensor] = None,
                   max_pairs: Optional[int] = None, status: Optional[torch.Tensor] = None, stream=None):
    """Every intersecting pair: (pair_a, pair_b) uint32 device tensors of length offsets[-1]
    (or max_pairs), query i's pairs at [offsets[i], offsets[i] + counts[i]).  `first` from
    bits_enum_counts saves the kernel its own search."""
    dev = _device()
    a_start, a_end = _u32_dev(a_start, "a_start"), _u32_dev(a_end, "a_end")
    counts = _u32_dev(counts, "counts")
    na = a_start.numel()
    if a_end.numel() != na or counts.numel() != na or offsets.numel() != na + 1:
        raise BitsError("a_start, a_end, counts and offsets disagree in length")
    if first is not None:
        first = _u32_dev(first, "first")
        if first.numel() != na:
            raise BitsError("first must have one entry per query")
    if max_pairs is None:
        max_pairs = int(offsets[-1].item())
    pa = torch.empty(max(max_pairs, 0), dtype=torch.uint32, device=dev)
    pb = torch.empty_like(pa)
    _check(_lib.bits_enumerate(_ptr(index.block) if index.n else ctypes.c_void_p(0), index.n, _ptr(a_start),
                               _ptr(a_end), na, _ptr(counts), _ptr(first), _ptr(offsets), _ptr(pa), _ptr(pb),
                               max_pairs,
                               _ptr(status), _stream(stream)), "bits_enumerate")
    return pa, pb
