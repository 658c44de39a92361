"""CPU oracle for the divide-and-conquer sampler -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``dcs_oracle.c`` with gcc, contraction off) through ctypes and shares no code
with the HIP library in ``paper_1610_05141_amd``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "dcs_oracle.c")

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-shared", "-fvisibility=hidden", "-Wall", "-Wextra"]

# Stream purposes (same meaning as the library's; restated here on purpose).
P_SPLIT, P_LEAF, P_BERN, P_REPAIR, P_BCHUNK, P_WRSPLIT, P_WRLEAF = 1, 2, 3, 4, 5, 6, 7
P_SEGSPLIT, P_SEGSEED = 8, 9
P_WCHUNK, P_WREPAIR = 10, 11

DEFAULT_N0 = 4096
DEFAULT_DENSE_RATIO = 16


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (idempotent unless ``force``)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC_PATH, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = configure(ctypes.CDLL(LIB_PATH))
    return _lib


def configure(L: ctypes.CDLL) -> ctypes.CDLL:
    """Declare the argument and result types of a loaded oracle library."""
    if True:
        u64, u32, i32, dbl, flt = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                   ctypes.c_double, ctypes.c_float)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        p32 = ctypes.POINTER(ctypes.c_uint32)
        sig = {
            "dcs_ref_sample": (i32, [u64, u64, u64, u32, u32, p64]),
            "dcs_ref_sample_window": (i32, [u64, u64, u64, u32, u32, u64, u64, p64]),
            "dcs_ref_replacement": (i32, [u64, u64, u64, u32, p64]),
            "dcs_ref_replacement_window": (i32, [u64, u64, u64, u32, u64, u64, p64]),
            "dcs_ref_part": (i32, [i32, u64, u64, u64, u32, u32, u32, u64, p64, u64, p64,
                                   p64]),
            "dcs_ref_bernoulli": (i32, [dbl, u64, u64, u32, p64, u64, p64]),
            "dcs_ref_edge_pair": (None, [u64, p64]),
            "dcs_ref_edges_gnm": (i32, [u64, u64, u64, u32, p32]),
            "dcs_ref_edges_gnp": (i32, [u64, dbl, u64, u32, p32, u64, p64]),
            "dcs_ref_bernoulli_chunks": (i32, [dbl, u64, u64, u32, u64, u64, p64, u64, p64]),
            "dcs_ref_bernoulli_chunk_len": (u64, [dbl, u32]),
            "dcs_ref_philox": (None, [p32, p32, p32]),
            "dcs_ref_stream_word": (u32, [u64, u64, u32, u32, u64]),
            "dcs_ref_stream_draw64": (u64, [u64, u64, u32, u32, u64]),
            "dcs_ref_range_map": (ctypes.c_int64, [u32, u64]),
            "dcs_ref_log64": (dbl, [dbl]),
            "dcs_ref_log1p64": (dbl, [dbl]),
            "dcs_ref_log32": (flt, [flt]),
            "dcs_ref_u32_geom": (flt, [u32]),
            "dcs_ref_lnfact_diff": (dbl, [u64, u64]),
            "dcs_ref_hyp": (u64, [u64, u64, u64, u64, u64]),
            "dcs_ref_bin": (u64, [u64, u64, u64, u64, u64]),
            "dcs_ref_hyp_mode": (u64, [u64, u64, u64]),
            "dcs_ref_bin_mode": (u64, [u64, u64, u64]),
            "dcs_ref_tree_stats": (i32, [u64, u64, u64, u32, p64]),
            "dcs_ref_log32_batch": (None, [ctypes.c_void_p, u64, ctypes.c_void_p]),
            "dcs_ref_log64_batch": (None, [ctypes.c_void_p, u64, ctypes.c_void_p]),
            "dcs_ref_log1p64_batch": (None, [ctypes.c_void_p, u64, ctypes.c_void_p]),
            "dcs_ref_lnfact_diff_batch": (None, [ctypes.c_void_p, ctypes.c_void_p, u64,
                                                 ctypes.c_void_p]),
            "dcs_ref_hyp_batch": (None, [u64, u64, u64, u64, u64, u64, p64]),
            "dcs_ref_bin_batch": (None, [u64, u64, u64, u64, u64, u64, p64]),
            "dcs_ref_range_map_counts": (None, [u64, p64, p64]),
            "dcs_ref_segment_tree": (i32, [u64, p64, u64, u64, p64, p64]),
            "dcs_ref_sample_wholerange": (i32, [u64, u64, u64, u32, p64, p32]),
            "dcs_ref_wholerange_hits": (i32, [u64, u64, u64, u32, u32, p64, u64, p64]),
            "dcs_ref_sample_segments": (i32, [u64, p64, u64, u64, u32, u32, p64, p64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
    return L


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def sample(n: int, N: int, seed: int, n0: int = DEFAULT_N0,
           dense_ratio: int = DEFAULT_DENSE_RATIO) -> np.ndarray:
    """n distinct values of 1..N, ascending (Algorithm R, Fig. 1)."""
    out = np.empty(n, dtype=np.uint64)
    _check(lib().dcs_ref_sample(n, N, seed, n0, dense_ratio, _p64(out)), "sample")
    return out


def sample_window(n: int, N: int, seed: int, start: int, count: int,
                  n0: int = DEFAULT_N0, dense_ratio: int = DEFAULT_DENSE_RATIO) -> np.ndarray:
    """out[start:start+count] of ``sample(n, N, seed)``, visiting only the
    subtrees whose output overlaps the window."""
    out = np.empty(count, dtype=np.uint64)
    _check(lib().dcs_ref_sample_window(n, N, seed, n0, dense_ratio, start, count, _p64(out)),
           "sample_window")
    return out


def replacement(n: int, N: int, seed: int, n0: int = DEFAULT_N0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(lib().dcs_ref_replacement(n, N, seed, n0, _p64(out)), "replacement")
    return out


def replacement_window(n: int, N: int, seed: int, start: int, count: int,
                       n0: int = DEFAULT_N0) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _check(lib().dcs_ref_replacement_window(n, N, seed, n0, start, count, _p64(out)),
           "replacement_window")
    return out


def part(variant: int, n: int, N: int, seed: int, depth: int, index: int,
         n0: int = DEFAULT_N0, dense_ratio: int = DEFAULT_DENSE_RATIO,
         capacity: int | None = None) -> tuple:
    """Part `index` of the depth-`depth` cut of ``sample`` (variant 0) or
    ``replacement`` (variant 1), Sec. 4.1 online sampling: returns
    (values, count, rank); values is None when count exceeds capacity."""
    cap = n if capacity is None else capacity
    out = np.empty(max(cap, 1), dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    rank = np.zeros(1, dtype=np.uint64)
    rc = lib().dcs_ref_part(variant, n, N, seed, n0, dense_ratio, depth, index, _p64(out), cap,
                            _p64(cnt), _p64(rank))
    count, r = int(cnt[0]), int(rank[0])
    if rc == 4:  # overflow: the part does not fit
        return None, count, r
    _check(rc, "part")
    return out[:count].copy(), count, r


def _lengths(lengths) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(lengths, dtype=np.uint64))


def segment_tree(n: int, lengths, seed: int) -> tuple:
    """The two passes of Sec. 4.3 over the binomial tree of the segments:
    (sums, counts), each indexed by heap id 1 .. 2^(D+1)-1 (entry 0 unused;
    node (level j, subtree a) has id 2^(D-j) + a, D = ceil(log2 K))."""
    L = _lengths(lengths)
    D = max(0, (len(L) - 1).bit_length())
    sums = np.zeros(2 << D, dtype=np.uint64)
    cnt = np.zeros(2 << D, dtype=np.uint64)
    _check(lib().dcs_ref_segment_tree(n, _p64(L), len(L), seed, _p64(sums), _p64(cnt)),
           "segment_tree")
    return sums, cnt


def sample_segments(n: int, lengths, seed: int, n0: int = DEFAULT_N0,
                    dense_ratio: int = DEFAULT_DENSE_RATIO) -> tuple:
    """n distinct values of 1..sum(lengths), ascending, computed segment by
    segment (Sec. 4.3, uneven universe): returns (values, per-segment
    counts)."""
    L = _lengths(lengths)
    out = np.empty(max(n, 1), dtype=np.uint64)
    counts = np.zeros(max(len(L), 1), dtype=np.uint64)
    _check(lib().dcs_ref_sample_segments(n, _p64(L), len(L), seed, n0, dense_ratio, _p64(out),
                                         _p64(counts)), "sample_segments")
    return out[:n].copy(), counts[:len(L)].copy()


def sample_wholerange(n: int, N: int, seed: int, n0: int = DEFAULT_N0) -> tuple:
    """n of 1..N by Algorithm B over the whole range with the repair (Sec. 2,
    Sec. 4.7, Sec. 5's GPU variant): (values, accepted attempt)."""
    out = np.empty(max(n, 1), dtype=np.uint64)
    att = (ctypes.c_uint32 * 1)()
    _check(lib().dcs_ref_sample_wholerange(n, N, seed, n0, _p64(out), att),
           "sample_wholerange")
    return out[:n].copy(), int(att[0])


def wholerange_hits(n: int, N: int, seed: int, attempt: int = 0, n0: int = DEFAULT_N0,
                    cap: int = 0) -> tuple:
    """(n', first min(n', cap) hit positions + 1) of one attempt."""
    out = np.empty(max(cap, 1), dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    _check(lib().dcs_ref_wholerange_hits(n, N, seed, n0, attempt, _p64(out), cap, _p64(cnt)),
           "wholerange_hits")
    c = int(cnt[0])
    return c, out[:min(c, cap)].copy()


def edge_pair(k: int) -> tuple:
    """(u, v), v < u, of edge index k = u(u-1)/2 + v (Sec. 7 random graphs)."""
    out = np.zeros(2, dtype=np.uint64)
    lib().dcs_ref_edge_pair(k, _p64(out))
    return int(out[0]), int(out[1])


def edges_gnm(n_vertices: int, m: int, seed: int, n0: int = DEFAULT_N0) -> np.ndarray:
    """G(n, m) edge list, (m, 2) uint32 rows (u, v), in increasing order."""
    uv = np.zeros((max(m, 1), 2), dtype=np.uint32)
    _check(lib().dcs_ref_edges_gnm(n_vertices, m, seed, n0,
                                   uv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
           "edges_gnm")
    return uv[:m]


def edges_gnp(n_vertices: int, p: float, seed: int, n0: int = DEFAULT_N0,
              capacity: int = 1 << 20) -> np.ndarray:
    """G(n, p) edge list (all of it; capacity must hold it)."""
    uv = np.zeros((max(capacity, 1), 2), dtype=np.uint32)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().dcs_ref_edges_gnp(n_vertices, float(p), seed, n0,
                                 uv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), capacity,
                                 _p64(cnt))
    _check(rc, "edges_gnp")
    return uv[: int(cnt[0])].copy()


def bernoulli(p: float, N: int, seed: int, n0: int = DEFAULT_N0,
              capacity: int | None = None) -> np.ndarray:
    if capacity is None:
        capacity = int(N * p + 10 * (N * p * (1 - p)) ** 0.5 + 64) if p < 1 else N
    out = np.empty(max(capacity, 1), dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().dcs_ref_bernoulli(float(p), N, seed, n0, _p64(out), capacity, _p64(cnt))
    _check(rc, "bernoulli")
    return out[: int(cnt[0])].copy()


def bernoulli_chunks(p: float, N: int, seed: int, chunk_lo: int, chunk_hi: int,
                     n0: int = DEFAULT_N0, capacity: int = 1 << 20) -> np.ndarray:
    out = np.empty(capacity, dtype=np.uint64)
    cnt = np.zeros(1, dtype=np.uint64)
    rc = lib().dcs_ref_bernoulli_chunks(float(p), N, seed, n0, chunk_lo, chunk_hi,
                                        _p64(out), capacity, _p64(cnt))
    _check(rc, "bernoulli_chunks")
    return out[: int(cnt[0])].copy()


def bernoulli_chunk_len(p: float, n0: int = DEFAULT_N0) -> int:
    return int(lib().dcs_ref_bernoulli_chunk_len(float(p), n0))


def philox(ctr, key) -> tuple:
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().dcs_ref_philox(c, k, o)
    return tuple(o)


def stream_word(seed, node_id, purpose, attempt, t) -> int:
    return int(lib().dcs_ref_stream_word(seed, node_id, purpose, attempt, t))


def stream_draw64(seed, node_id, purpose, attempt, t) -> int:
    return int(lib().dcs_ref_stream_draw64(seed, node_id, purpose, attempt, t))


def range_map(w: int, s: int) -> int:
    return int(lib().dcs_ref_range_map(w, s))


def log64(x: float) -> float:
    return lib().dcs_ref_log64(x)


def log1p64(x: float) -> float:
    return lib().dcs_ref_log1p64(x)


def log32(x: float) -> float:
    return lib().dcs_ref_log32(x)


def u32_geom(w: int) -> float:
    return lib().dcs_ref_u32_geom(w)


def lnfact_diff(a: int, b: int) -> float:
    return lib().dcs_ref_lnfact_diff(a, b)


def hyp(n: int, M: int, N: int, seed: int, node_id: int) -> int:
    return int(lib().dcs_ref_hyp(n, M, N, seed, node_id))


def hyp_mode(n: int, M: int, N: int) -> int:
    return int(lib().dcs_ref_hyp_mode(n, M, N))


def bin_mode(n: int, l: int, Nv: int) -> int:
    return int(lib().dcs_ref_bin_mode(n, l, Nv))


def binom(n: int, l: int, Nv: int, seed: int, node_id: int) -> int:
    return int(lib().dcs_ref_bin(n, l, Nv, seed, node_id))


def tree_stats(n: int, N: int, seed: int, n0: int = DEFAULT_N0) -> tuple:
    st = np.zeros(3, dtype=np.uint64)
    _check(lib().dcs_ref_tree_stats(n, N, seed, n0, _p64(st)), "tree_stats")
    return int(st[0]), int(st[1]), int(st[2])


def log32_batch(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib().dcs_ref_log32_batch(x.ctypes.data, x.size, y.ctypes.data)
    return y


def log64_batch(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().dcs_ref_log64_batch(x.ctypes.data, x.size, y.ctypes.data)
    return y


def log1p64_batch(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().dcs_ref_log1p64_batch(x.ctypes.data, x.size, y.ctypes.data)
    return y


def lnfact_diff_batch(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    y = np.empty(a.size, dtype=np.float64)
    lib().dcs_ref_lnfact_diff_batch(a.ctypes.data, b.ctypes.data, a.size, y.ctypes.data)
    return y


def hyp_batch(n: int, M: int, N: int, seed: int, id0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().dcs_ref_hyp_batch(n, M, N, seed, id0, count, _p64(out))
    return out


def binom_batch(n: int, l: int, Nv: int, seed: int, id0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().dcs_ref_bin_batch(n, l, Nv, seed, id0, count, _p64(out))
    return out


def range_map_counts(s: int) -> tuple:
    counts = np.zeros(s, dtype=np.uint64)
    voids = np.zeros(1, dtype=np.uint64)
    lib().dcs_ref_range_map_counts(s, _p64(counts), _p64(voids))
    return counts, int(voids[0])
