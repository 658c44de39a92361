"""The sample never depends on launch geometry (GPU): different numbers of
leaf work-groups and different Algorithm P cut depths give identical bytes,
equal to the oracle's.  Also a race detector: any order dependence inside a
work-group or between work-groups would show up as a difference."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.gpu_util import announce, dcs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = [  # (variant, n, N, seed, n0)
    ("wor", 1 << 20, 1 << 32, 1, 4096),
    ("wor", 300000, 700000, 3, 1024),
    ("wor", 40000, 2**41 + 5, 4, 256),
    ("wr", 200000, 3 * 10**6 + 1, 5, 512),
]

SCRIPT = r"""
import hashlib, sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import paper_1610_05141_amd as dcs
for variant, n, N, seed, n0 in {cases!r}:
    f = dcs.sample if variant == "wor" else dcs.sample_replacement
    out = f(n, N, seed, n0=n0)
    dcs.synchronize()
    print(hashlib.sha256(out.cpu().numpy().tobytes()).hexdigest(), flush=True)
"""


def _run(env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    print(f"[gpu-step] geometry {env_extra}", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, cases=CASES)],
                       env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    return r.stdout.split()


def test_launch_geometry_invariance(ref):
    want = []
    for variant, n, N, seed, n0 in CASES:
        v = ref.sample(n, N, seed, n0=n0) if variant == "wor" else ref.replacement(n, N, seed, n0=n0)
        want.append(hashlib.sha256(v.astype(np.int64).tobytes()).hexdigest())
    for env in [{}, {"DCS_LEAF_GRID": "1"}, {"DCS_LEAF_GRID": "7"},
                {"DCS_LEAF_GRID": "5000"}, {"DCS_CUT_BIAS": "-4"},
                {"DCS_CUT_BIAS": "3"}, {"DCS_LEAF_GRID": "13", "DCS_CUT_BIAS": "-20"}]:
        assert _run(env) == want, env


def test_tuning_table_geometry_invariance(ref):
    """Entries of the library's tuning table (what the autotuner sets) change
    the launch geometry of a size class, never its sample."""
    import torch
    from tests.gpu_util import dcs, to_np_u64
    m = dcs()
    cases = [(0, 1 << 20, 1 << 32, 1), (0, 300000, 700000, 3), (1, 200000, 3 * 10**6 + 1, 5)]
    saved = {}
    try:
        for variant, n, N, seed in cases:
            k = n.bit_length() - 1
            saved[(variant, k)] = m.tune_get(variant, k)
            want = ref.sample(n, N, seed) if variant == 0 else ref.replacement(n, N, seed)
            for cb, w in [(-2, 1), (2, 3), (0, 2), (-16, 1), (5, 64)]:
                print(f"[gpu-step] tuned geometry variant={variant} n={n} cut_bias={cb} wgs={w}",
                      flush=True)
                m.tune_set(variant, k, cb, w)
                f = m.sample if variant == 0 else m.sample_replacement
                got = to_np_u64(f(n, N, seed))
                m.synchronize()
                assert np.array_equal(got, want), (variant, n, cb, w)
    finally:
        for (variant, k), (cb, w) in saved.items():
            m.tune_set(variant, k, cb, w)


def test_profile_kinds_times_only_the_selected_kernels():
    """dcs_profile_kinds: with only kind 4 selected, a sample records launches
    of the power-of-two leaf kernel and none of the tree or the other leaf
    kernels; with every kind selected and every leaf kernel launched, all of
    them.  By default this sparse sample (density 2^-18) launches no
    one-wave dense, one-wave small or one-pass kernel: its tree cannot
    plausibly hold their leaves."""
    m = dcs()
    announce("profile kinds")
    n, N = 1 << 18, 1 << 36
    try:
        m.profile_kinds([4])
        m.profile_enable(True)
        m.sample(n, N, 5)
        m.synchronize()
        assert m.profile_read(4)[1] == 1
        assert all(m.profile_read(k)[1] == 0 for k in (0, 1, 2, 5, 6))
        m.profile_kinds(None)
        m.debug_leaf_kernels(0)
        m.profile_enable(True)
        m.sample(n, N, 5)
        m.synchronize()
        assert all(m.profile_read(k)[1] == 1 for k in (0, 1, 2, 4, 5, 6, 12, 13))
        m.debug_leaf_kernels(-1)
        m.profile_enable(True)
        m.sample(n, N, 5)
        m.synchronize()
        assert all(m.profile_read(k)[1] == 1 for k in (0, 1, 2, 4, 5))
        assert all(m.profile_read(k)[1] == 0 for k in (6, 12, 13))
    finally:
        m.debug_leaf_kernels(-1)
        m.profile_kinds(None)
        m.profile_enable(False)
