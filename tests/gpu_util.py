"""Helpers shared by the GPU tests (test infrastructure)."""
import sys

import numpy as np
import pytest


def dcs():
    """The HIP library's binding; fails the test (never skips) when the
    built library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1610_05141_amd as m
    m.lib()  # raises FileNotFoundError if libdcs.so was not built
    return m


def announce(msg: str) -> None:
    """Print and flush what the next GPU step is, so a failing run names it."""
    print(f"[gpu-step] {msg}", flush=True)
    sys.stdout.flush()


def to_np_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def first_mismatch(a: np.ndarray, b: np.ndarray) -> str:
    if a.shape != b.shape:
        return f"shape {a.shape} vs {b.shape}"
    bad = np.nonzero(a != b)[0]
    if bad.size == 0:
        return "identical"
    i = int(bad[0])
    return f"{bad.size} mismatches, first at {i}: {int(a[i])} vs {int(b[i])}"
