"""Python binding of the MI355X divide-and-conquer sampler (libdcs.so).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  torch supplies device memory and streams.  Importing works
without a GPU; calling anything that needs the library raises if
``_lib/libdcs.so`` has not been built (``python paper_1610_05141_amd/build.py``
or ``__graft_entry__.build()``) -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "DcsError", "lib", "sample", "sample_noalloc", "sample_replacement", "sample_bernoulli", "sample_part",
    "sample_segments", "sample_wholerange", "sample_edges_gnm", "sample_edges_gnp",
    "synchronize",
    "workspace_size", "bernoulli_capacity_hint", "Batch", "Online", "Server", "profile_enable",
    "profile_read", "profile_kinds", "debug_primitive", "debug_plan", "debug_leaf_capacity",
    "debug_lookback_help", "debug_bernoulli_list", "debug_leaf_kernels",
    "tune_set", "tune_get", "tune_reset",
    "EXPORTED_SYMBOLS", "LIB_PATH",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdcs.so")

DCS_OK, DCS_EINVAL, DCS_ENOMEM, DCS_EHIP, DCS_EOVERFLOW, DCS_EDEVICE, DCS_ENOTSUP = range(7)
# Static scratch of dcs_sample_noalloc per device (DCS_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 64 << 20

# Every symbol declared in include/dcs.h.
EXPORTED_SYMBOLS = (
    "dcs_sample", "dcs_sample_ex", "dcs_sample_noalloc", "dcs_sample_replacement", "dcs_sample_replacement_ex",
    "dcs_sample_bernoulli", "dcs_sample_bernoulli_ex", "dcs_bernoulli_capacity_hint",
    "dcs_sample_part", "dcs_sample_segments", "dcs_sample_wholerange", "dcs_sample_edges_gnm", "dcs_sample_edges_gnp",
    "dcs_workspace_size", "dcs_batch_create", "dcs_batch_run", "dcs_batch_destroy",
    "dcs_batch_total", "dcs_synchronize", "dcs_status_string", "dcs_profile_enable",
    "dcs_profile_read", "dcs_profile_kinds", "dcs_debug_primitive", "dcs_server_create", "dcs_server_submit",
    "dcs_server_submit_schedule", "dcs_server_poll", "dcs_server_release", "dcs_server_drain",
    "dcs_server_stats_read", "dcs_server_destroy", "dcs_server_now", "dcs_server_copy_out",
    "dcs_tune_set", "dcs_tune_get", "dcs_tune_reset", "dcs_debug_leaf_capacity",
    "dcs_debug_plan", "dcs_debug_lookback_help", "dcs_debug_bernoulli_list",
    "dcs_debug_leaf_kernels", "dcs_online_create", "dcs_online_counts", "dcs_online_next",
    "dcs_online_destroy",
)


class DcsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        msg = lib().dcs_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} (status {code})")


class _Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n0", ctypes.c_uint32),
                ("dense_ratio", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("N", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("out_offset", ctypes.c_uint64), ("variant", ctypes.c_uint32),
                ("n0", ctypes.c_uint32), ("dense_ratio", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("N", ctypes.c_uint64), ("seed", ctypes.c_uint64),
                ("variant", ctypes.c_uint32), ("n0", ctypes.c_uint32)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("samples", ctypes.c_uint64),
                ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("max_s", ctypes.c_double), ("span_s", ctypes.c_double),
                ("batches", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libdcs.so (raises FileNotFoundError if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with `python paper_1610_05141_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, i32, dbl, vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                  ctypes.c_double, ctypes.c_void_p)
        pp = ctypes.POINTER(_Params)
        sig = {
            "dcs_sample": (i32, [u64, u64, u64, vp, vp]),
            "dcs_sample_ex": (i32, [u64, u64, u64, pp, vp, vp, ctypes.c_size_t, vp]),
            "dcs_sample_noalloc": (i32, [u64, u64, u64, pp, vp, vp]),
            "dcs_sample_replacement": (i32, [u64, u64, u64, vp, vp]),
            "dcs_sample_replacement_ex": (i32, [u64, u64, u64, pp, vp, vp, ctypes.c_size_t, vp]),
            "dcs_sample_bernoulli": (i32, [dbl, u64, u64, vp, u64, vp, vp]),
            "dcs_sample_bernoulli_ex": (i32, [dbl, u64, u64, pp, vp, u64, vp, vp,
                                              ctypes.c_size_t, vp]),
            "dcs_bernoulli_capacity_hint": (u64, [dbl, u64]),
            "dcs_sample_part": (i32, [i32, u64, u64, u64, pp, u32, u64, vp, u64, vp, vp]),
            "dcs_sample_segments": (i32, [u64, vp, u64, u64, pp, vp, vp, vp]),
            "dcs_sample_wholerange": (i32, [u64, u64, u64, pp, vp, vp]),
            "dcs_sample_edges_gnm": (i32, [u64, u64, u64, pp, vp, vp]),
            "dcs_sample_edges_gnp": (i32, [u64, dbl, u64, pp, vp, u64, vp, vp]),
            "dcs_workspace_size": (i32, [i32, u64, u64, dbl, pp, ctypes.POINTER(ctypes.c_size_t)]),
            "dcs_batch_create": (i32, [ctypes.POINTER(_Instance), u32, ctypes.POINTER(vp),
                                       ctypes.POINTER(u32)]),
            "dcs_batch_run": (i32, [vp, vp, i32, vp]),
            "dcs_batch_destroy": (i32, [vp]),
            "dcs_batch_total": (u64, [vp]),
            "dcs_synchronize": (i32, [vp]),
            "dcs_status_string": (ctypes.c_char_p, [i32]),
            "dcs_profile_enable": (i32, [i32]),
            "dcs_profile_read": (i32, [i32, ctypes.POINTER(dbl), ctypes.POINTER(u64)]),
            "dcs_profile_kinds": (i32, [u32]),
            "dcs_debug_primitive": (i32, [i32, vp, vp, vp, u64, u64, u64, u64, u64, vp]),
            "dcs_server_create": (i32, [u64, u32, u32, i32, ctypes.POINTER(vp)]),
            "dcs_server_submit": (i32, [vp, ctypes.POINTER(_Request), dbl, ctypes.POINTER(u64)]),
            "dcs_server_submit_schedule": (i32, [vp, ctypes.POINTER(_Request),
                                                 ctypes.POINTER(dbl), u64, ctypes.POINTER(u64)]),
            "dcs_server_poll": (i32, [vp, u64, ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.POINTER(u64)), ctypes.POINTER(dbl)]),
            "dcs_server_release": (i32, [vp, u64]),
            "dcs_server_drain": (i32, [vp]),
            "dcs_server_stats_read": (i32, [vp, ctypes.POINTER(_ServerStats)]),
            "dcs_server_destroy": (i32, [vp]),
            "dcs_server_now": (dbl, []),
            "dcs_server_copy_out": (i32, [vp, u64, vp, vp]),
            "dcs_tune_set": (i32, [i32, u32, i32, u32]),
            "dcs_tune_get": (i32, [i32, u32, ctypes.POINTER(i32), ctypes.POINTER(u32)]),
            "dcs_tune_reset": (i32, []),
            "dcs_debug_leaf_capacity": (i32, [u64, i32, ctypes.POINTER(u32)]),
            "dcs_debug_plan": (i32, [i32, u64, u64, pp, ctypes.POINTER(u64)]),
            "dcs_debug_lookback_help": (i32, [u32]),
            "dcs_debug_bernoulli_list": (i32, [u32]),
            "dcs_debug_leaf_kernels": (i32, [i32]),
            "dcs_online_create": (i32, [i32, u64, u64, u64, pp, u32, vp, ctypes.POINTER(vp)]),
            "dcs_online_counts": (i32, [vp, u64, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]),
            "dcs_online_next": (i32, [vp, u64, u64, vp, u64, ctypes.POINTER(u64), vp]),
            "dcs_online_destroy": (i32, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        # launch geometry from the committed tuning table (never changes a sample)
        from . import autotune
        autotune.apply_table(L)
    return _lib


def _check(rc: int, what: str) -> None:
    if rc != DCS_OK:
        raise DcsError(rc, what)


def _params(n0, dense_ratio):
    if n0 is None and dense_ratio is None:
        return None
    return ctypes.byref(_Params(ctypes.sizeof(_Params), n0 or 0, dense_ratio or 0, 0))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _out_tensor(out, n: int):
    import torch
    if out is None:
        return torch.empty(max(n, 0), dtype=torch.int64, device="cuda")
    if out.dtype not in (torch.int64, torch.uint64) or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous int64 CUDA tensor")
    if out.numel() < n:
        raise ValueError(f"out holds {out.numel()} elements, {n} needed")
    return out


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def sample(n: int, N: int, seed: int, out=None, stream=None, n0=None, dense_ratio=None,
           workspace=None):
    """n distinct values of 1..N, ascending, into an int64 CUDA tensor."""
    out = _out_tensor(out, n)
    ws, wsb = (_ptr(workspace), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (ctypes.c_void_p(0), 0)
    rc = lib().dcs_sample_ex(n, N, seed, _params(n0, dense_ratio), _ptr(out), ws, wsb,
                             _stream_handle(stream))
    _check(rc, "dcs_sample_ex")
    return out


def sample_noalloc(n: int, N: int, seed: int, out, stream=None, n0=None, dense_ratio=None):
    """As sample(), into a caller tensor, with the library's static scratch:
    the call allocates no device memory (DcsError DCS_ENOMEM if the sample
    needs more than NOALLOC_SCRATCH_BYTES of workspace)."""
    out = _out_tensor(out, n)
    rc = lib().dcs_sample_noalloc(n, N, seed, _params(n0, dense_ratio), _ptr(out),
                                  _stream_handle(stream))
    _check(rc, "dcs_sample_noalloc")
    return out


def sample_replacement(n: int, N: int, seed: int, out=None, stream=None, n0=None,
                       workspace=None):
    """n independent uniform values of 1..N, sorted, repeats kept."""
    out = _out_tensor(out, n)
    ws, wsb = (_ptr(workspace), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (ctypes.c_void_p(0), 0)
    rc = lib().dcs_sample_replacement_ex(n, N, seed, _params(n0, None), _ptr(out), ws, wsb,
                                         _stream_handle(stream))
    _check(rc, "dcs_sample_replacement_ex")
    return out


def sample_part(n: int, N: int, seed: int, depth: int, index: int, out=None, capacity=None,
                count_rank=None, variant: int = 0, stream=None, n0=None, dense_ratio=None):
    """Part `index` of the depth-`depth` cut of the sample (variant 0: without
    replacement, 1: with replacement).  Returns (out, count_rank): out holds
    the part's values from element 0 when they fit `capacity`; count_rank is
    a 2-element int64 CUDA tensor (count, rank in the full sample)."""
    import torch
    if capacity is None:
        capacity = out.numel() if out is not None else n
    out = _out_tensor(out, capacity)
    if count_rank is None:
        count_rank = torch.zeros(2, dtype=torch.int64, device="cuda")
    rc = lib().dcs_sample_part(variant, n, N, seed, _params(n0, dense_ratio), depth, index,
                               _ptr(out), capacity, _ptr(count_rank), _stream_handle(stream))
    _check(rc, "dcs_sample_part")
    return out, count_rank


def sample_segments(n: int, lengths, seed: int, out=None, counts=None, stream=None, n0=None,
                    dense_ratio=None):
    """n distinct elements of the concatenation of segments of the given
    lengths (a host sequence), ascending as elements of 1..sum(lengths)
    (Sec. 4.3).  Returns (out, counts): counts is a K-element int64 CUDA
    tensor with each segment's number of values."""
    import numpy as np
    import torch
    L = np.ascontiguousarray(np.asarray(lengths, dtype=np.uint64))
    out = _out_tensor(out, n)
    if counts is None:
        counts = torch.empty(max(L.size, 1), dtype=torch.int64, device="cuda")
    rc = lib().dcs_sample_segments(n, ctypes.c_void_p(L.ctypes.data), L.size, seed,
                                   _params(n0, dense_ratio), _ptr(out), _ptr(counts),
                                   _stream_handle(stream))
    _check(rc, "dcs_sample_segments")
    return out, counts


def sample_wholerange(n: int, N: int, seed: int, out=None, stream=None, n0=None):
    """n distinct values of 1..N (N <= 2^32, n/N not below about 2^-10),
    ascending, by Algorithm B over the whole range with the repair on the
    device (Sec. 2, 4.7, 5)."""
    out = _out_tensor(out, n)
    rc = lib().dcs_sample_wholerange(n, N, seed, _params(n0, None), _ptr(out),
                                     _stream_handle(stream))
    _check(rc, "dcs_sample_wholerange")
    return out


def _edge_tensor(out, m: int):
    import torch
    if out is None:
        return torch.empty((max(m, 0), 2), dtype=torch.int32, device="cuda")
    if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() or \
            out.numel() < 2 * m:
        raise ValueError(f"out must be a contiguous int32 CUDA tensor of {2 * m} elements")
    return out


def sample_edges_gnm(n_vertices: int, m: int, seed: int, out=None, stream=None, n0=None):
    """G(n, m): m distinct edges (u, v), v < u < n_vertices, as an (m, 2) int32
    CUDA tensor in increasing (u, v) order (values are below 2^31 for any
    n_vertices the library accepts)."""
    out = _edge_tensor(out, m)
    rc = lib().dcs_sample_edges_gnm(n_vertices, m, seed, _params(n0, None), _ptr(out),
                                    _stream_handle(stream))
    _check(rc, "dcs_sample_edges_gnm")
    return out


def sample_edges_gnp(n_vertices: int, p: float, seed: int, out=None, capacity=None, count=None,
                     stream=None, n0=None):
    """G(n, p): each pair an edge with probability p.  Returns (edges, count):
    edges is an (capacity, 2) int32 CUDA tensor whose first min(count,
    capacity) rows hold the edges; count a 1-element int64 CUDA tensor."""
    import torch
    N = n_vertices * (n_vertices - 1) // 2
    if capacity is None:
        capacity = out.numel() // 2 if out is not None else bernoulli_capacity_hint(p, N)
    out = _edge_tensor(out, capacity)
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = lib().dcs_sample_edges_gnp(n_vertices, float(p), seed, _params(n0, None), _ptr(out),
                                    capacity, _ptr(count), _stream_handle(stream))
    _check(rc, "dcs_sample_edges_gnp")
    return out, count


def bernoulli_capacity_hint(p: float, N: int) -> int:
    return int(lib().dcs_bernoulli_capacity_hint(float(p), N))


def sample_bernoulli(p: float, N: int, seed: int, out=None, capacity=None, count=None,
                     stream=None, n0=None, workspace=None):
    """Bernoulli(p) sample of 1..N.  Returns (out, count) tensors; count is a
    1-element int64 CUDA tensor with the true number of hits."""
    import torch
    if capacity is None:
        capacity = out.numel() if out is not None else bernoulli_capacity_hint(p, N)
    out = _out_tensor(out, capacity)
    if count is None:
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws, wsb = (_ptr(workspace), workspace.numel() * workspace.element_size()) \
        if workspace is not None else (ctypes.c_void_p(0), 0)
    rc = lib().dcs_sample_bernoulli_ex(float(p), N, seed, _params(n0, None), _ptr(out), capacity,
                                       _ptr(count), ws, wsb, _stream_handle(stream))
    _check(rc, "dcs_sample_bernoulli_ex")
    return out, count


def synchronize(stream=None) -> None:
    """Wait for the stream; raise DcsError if a kernel latched an error."""
    _check(lib().dcs_synchronize(_stream_handle(stream)), "dcs_synchronize")


def workspace_size(variant: int, n: int, N: int, p: float = 0.0, n0=None, dense_ratio=None) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().dcs_workspace_size(variant, n, N, float(p), _params(n0, dense_ratio),
                                    ctypes.byref(b)), "dcs_workspace_size")
    return int(b.value)


@dataclass
class InstanceSpec:
    n: int
    N: int
    seed: int
    out_offset: int
    variant: int = 0
    n0: int = 0
    dense_ratio: int = 0


class Online:
    """Online sampling in sorted order (Sec. 4.1): the sample of `sample`
    (variant 0) or `sample_replacement` (variant 1) as the 2^depth parts of
    the depth-`depth` cut, whose roots are computed once, produced in runs of
    consecutive parts."""

    def __init__(self, n: int, N: int, seed: int, depth: int, variant: int = 0, n0=None,
                 dense_ratio=None, stream=None):
        self.depth = depth
        self.parts = 1 << depth
        h = ctypes.c_void_p()
        _check(lib().dcs_online_create(variant, n, N, seed, _params(n0, dense_ratio), depth,
                                       _stream_handle(stream), ctypes.byref(h)),
               "dcs_online_create")
        self._h = h

    def counts(self, first: int = 0, count=None):
        """(counts, ranks) of parts [first, first + count) as numpy arrays."""
        import numpy as np
        count = self.parts - first if count is None else count
        c = np.zeros(max(count, 1), dtype=np.uint64)
        r = np.zeros(max(count, 1), dtype=np.uint64)
        _check(lib().dcs_online_counts(self._h, first, count,
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                       r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "dcs_online_counts")
        return c[:count], r[:count]

    def next(self, first: int, count: int, out, stream=None) -> int:
        """Parts [first, first + count) into out (a device int64 tensor);
        returns the number of values written."""
        w = ctypes.c_uint64(0)
        _check(lib().dcs_online_next(self._h, first, count, _ptr(out), out.numel(),
                                     ctypes.byref(w), _stream_handle(stream)), "dcs_online_next")
        return int(w.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().dcs_online_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances sampled by one launch sequence."""

    def __init__(self, instances):
        arr = (_Instance * len(instances))()
        for i, s in enumerate(instances):
            arr[i] = _Instance(s.n, s.N, s.seed, s.out_offset, s.variant, s.n0, s.dense_ratio, 0)
        h = ctypes.c_void_p(0)
        bad = ctypes.c_uint32(0)
        rc = lib().dcs_batch_create(arr, len(instances), ctypes.byref(h), ctypes.byref(bad))
        if rc != DCS_OK:
            raise DcsError(rc, f"dcs_batch_create (instance {bad.value})")
        self._h = h
        self.total = int(lib().dcs_batch_total(h))

    def run(self, out, use_graph: bool = False, stream=None) -> None:
        _check(lib().dcs_batch_run(self._h, _ptr(out), 1 if use_graph else 0,
                                   _stream_handle(stream)), "dcs_batch_run")

    def close(self) -> None:
        if self._h:
            lib().dcs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True) -> None:
    _check(lib().dcs_profile_enable(1 if on else 0), "dcs_profile_enable")


def tune_set(variant: int, log2_n: int, cut_bias: int, leaf_wgs_per_cu: int) -> None:
    """Launch geometry of size class (variant, floor(log2 n)); never changes a sample."""
    _check(lib().dcs_tune_set(variant, log2_n, cut_bias, leaf_wgs_per_cu), "dcs_tune_set")


def tune_get(variant: int, log2_n: int):
    """(cut_bias, leaf_wgs_per_cu) of a size class."""
    cb, w = ctypes.c_int32(0), ctypes.c_uint32(0)
    _check(lib().dcs_tune_get(variant, log2_n, ctypes.byref(cb), ctypes.byref(w)), "dcs_tune_get")
    return int(cb.value), int(w.value)


def tune_reset() -> None:
    _check(lib().dcs_tune_reset(), "dcs_tune_reset")


def debug_plan(variant: int, n: int, N: int, n0: int = 0, dense_ratio: int = 0) -> dict:
    """The plan of a tree call (host only): cut depth, tree threads, DFS
    stack entries per thread, leaf-job capacity, proven bound on leaf jobs,
    and whether the second round is planned."""
    info = (ctypes.c_uint64 * 6)()
    _check(lib().dcs_debug_plan(variant, n, N, _params(n0, dense_ratio), info), "dcs_debug_plan")
    return {"cut": int(info[0]), "threads": int(info[1]), "stack_depth": int(info[2]),
            "leaf_cap": int(info[3]), "leaf_bound": int(info[4]),
            "second_round": bool(info[5])}


def debug_lookback_help(polls: int) -> None:
    """Test hook: Bernoulli look-backs count a silent predecessor chunk
    themselves after `polls` polls (0: the default)."""
    _check(lib().dcs_debug_lookback_help(int(polls)), "dcs_debug_lookback_help")


def debug_leaf_kernels(mask: int) -> None:
    """Test hook: the specialised leaf kernels a single-instance tree call
    leaves out (bit 0 dense, bit 1 small, bit 2 one-pass; their leaves then
    run in the general work-group kernel); a negative mask restores the
    default choice."""
    _check(lib().dcs_debug_leaf_kernels(int(mask)), "dcs_debug_leaf_kernels")


def debug_bernoulli_list(words: int) -> None:
    """Test hook: double-precision Bernoulli chunks keep `words` hit
    positions in LDS (1-1024: the one-wave kernel, more: the work-group
    kernel; 0: the default size)."""
    _check(lib().dcs_debug_bernoulli_list(int(words)), "dcs_debug_bernoulli_list")


def debug_leaf_capacity(capacity: int, reset_boost: bool = False) -> int:
    """Test hook: plan later tree calls with `capacity` leaf-job slots per
    instance and the device's second round (0: normal planning).  Returns the
    multiplier of the expected-case capacity in effect (raised after a call
    ran out of slots in both rounds), then resets it to 1 if asked."""
    b = ctypes.c_uint32(0)
    _check(lib().dcs_debug_leaf_capacity(int(capacity), 1 if reset_boost else 0,
                                         ctypes.byref(b)), "dcs_debug_leaf_capacity")
    return int(b.value)


def profile_kinds(kinds=None):
    """Time only the given kernel kinds (an iterable of ints; None = all)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << int(k) for k in kinds)
    _check(lib().dcs_profile_kinds(mask), "dcs_profile_kinds")


def profile_read(kind: int):
    """(total milliseconds, launches) of kernel kind 0 reset, 1 tree, 2 leaf
    stage (all leaf kernels), 3 Bernoulli, 4 leaf kernel of the sparse and
    with-replacement jobs over power-of-two ranges, 5 work-group leaf kernel
    of the other jobs, 6 one-wave dense leaf kernel, 7 edge decoding, 8
    segment splits, 9 / 10 / 11 whole-range B count / repair / write, 12
    one-wave leaf kernel of jobs of at most 1024 values, 13 one-pass kernel
    of sparse jobs expected to repeat, accumulated since profile_enable (read
    after synchronize)."""
    ms = ctypes.c_double(0)
    n = ctypes.c_uint64(0)
    _check(lib().dcs_profile_read(kind, ctypes.byref(ms), ctypes.byref(n)), "dcs_profile_read")
    return float(ms.value), int(n.value)


def debug_primitive(op: int, x, x2, y, p0=0, p1=0, p2=0, p3=0, stream=None) -> None:
    count = y.numel() if op != 8 else y.numel() // 4
    rc = lib().dcs_debug_primitive(op, _ptr(x), _ptr(x2), _ptr(y), count, p0, p1, p2, p3,
                                   _stream_handle(stream))
    _check(rc, "dcs_debug_primitive")


class Server:
    """Continuous-batching sampling server (see dcs_server_* in include/dcs.h)."""

    def __init__(self, arena_bytes: int, max_batch: int = 1024, n_streams: int = 4,
                 auto_release: bool = False):
        h = ctypes.c_void_p(0)
        _check(lib().dcs_server_create(arena_bytes, max_batch, n_streams,
                                       1 if auto_release else 0, ctypes.byref(h)),
               "dcs_server_create")
        self._h = h

    @staticmethod
    def now() -> float:
        return float(lib().dcs_server_now())

    def submit(self, n: int, N: int, seed: int, variant: int = 0, n0: int = 0,
               arrival_s: float = -1.0) -> int:
        tk = ctypes.c_uint64(0)
        r = _Request(n, N, seed, variant, n0)
        _check(lib().dcs_server_submit(self._h, ctypes.byref(r), float(arrival_s),
                                       ctypes.byref(tk)), "dcs_server_submit")
        return int(tk.value)

    def submit_schedule(self, requests, arrival_s) -> int:
        """requests: iterable of (n, N, seed[, variant[, n0]]); arrival times on
        the server clock.  Returns the first ticket; tickets are consecutive."""
        reqs = list(requests)
        arr = (_Request * len(reqs))()
        for i, r in enumerate(reqs):
            r = tuple(r) + (0,) * (5 - len(r))
            arr[i] = _Request(*r)
        times = (ctypes.c_double * len(reqs))(*[float(t) for t in arrival_s])
        first = ctypes.c_uint64(0)
        _check(lib().dcs_server_submit_schedule(self._h, arr, times, len(reqs),
                                                ctypes.byref(first)),
               "dcs_server_submit_schedule")
        return int(first.value)

    def poll(self, ticket: int):
        """(state, device pointer or 0, latency seconds)."""
        st = ctypes.c_int32(0)
        ptr = ctypes.POINTER(ctypes.c_uint64)()
        lat = ctypes.c_double(0)
        _check(lib().dcs_server_poll(self._h, ticket, ctypes.byref(st), ctypes.byref(ptr),
                                     ctypes.byref(lat)), "dcs_server_poll")
        addr = ctypes.cast(ptr, ctypes.c_void_p).value or 0
        return int(st.value), addr, float(lat.value)

    def result(self, ticket: int, n: int, stream=None):
        """The request's output copied into a new int64 CUDA tensor."""
        import torch
        out = torch.empty(n, dtype=torch.int64, device="cuda")
        _check(lib().dcs_server_copy_out(self._h, ticket, _ptr(out), _stream_handle(stream)),
               "dcs_server_copy_out")
        return out

    def release(self, ticket: int) -> None:
        _check(lib().dcs_server_release(self._h, ticket), "dcs_server_release")

    def drain(self) -> None:
        _check(lib().dcs_server_drain(self._h), "dcs_server_drain")

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().dcs_server_stats_read(self._h, ctypes.byref(st)), "dcs_server_stats_read")
        return {k: getattr(st, k) for k, _ in _ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            lib().dcs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
