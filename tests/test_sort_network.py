"""The leaf kernel's in-bucket sort (CPU): the comparator table compiled
into the kernel is a sorting network for 16 inputs and its first 19
comparators one for 8 (0-1 principle, exhaustive), and two passes of
W-key windows at offsets 0 and W/2 sort any bucket-ordered sequence whose
buckets hold at most W/2 + 1 keys."""
import os
import random
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1610_05141_amd", "csrc", "dcs_kernels.hip")


def _network():
    text = open(SRC).read()
    body = re.search(r"kNet16\[63\]\[2\]\s*=\s*\{(.*?)\};", text, re.S).group(1)
    pairs = [(int(a), int(b)) for a, b in re.findall(r"\{\s*(\d+)\s*,\s*(\d+)\s*\}", body)]
    assert len(pairs) == 63
    return pairs


def _sorts_all_01(pairs, w):
    x = ((np.arange(1 << w)[:, None] >> np.arange(w)[None, :]) & 1).astype(np.uint8)
    for a, b in pairs:
        lo, hi = np.minimum(x[:, a], x[:, b]), np.maximum(x[:, a], x[:, b])
        x[:, a], x[:, b] = lo, hi
    return bool((np.diff(x.astype(np.int8), axis=1) >= 0).all())


def test_network_16_sorts_every_01_input():
    pairs = _network()
    assert all(0 <= a < b < 16 for a, b in pairs)
    assert _sorts_all_01(pairs, 16)


def test_first_19_comparators_sort_8():
    pairs = _network()[:19]
    assert all(b < 8 for _, b in pairs)
    assert _sorts_all_01(pairs, 8)
    # and 18 would not do
    assert not _sorts_all_01(pairs[:18], 8)


def _two_pass(arr, w):
    n = len(arr)
    a = list(arr) + [0xFFFFFFFF] * (2 * w)
    for off in (0, w // 2):
        for w0 in range(off, n, w):
            a[w0:w0 + w] = sorted(a[w0:w0 + w])
    return a[:n]


def _bucketed(rng, n, kb, shift, cap):
    keys = [rng.randrange(1 << kb) for _ in range(n)]
    buckets = {}
    for x in keys:
        buckets.setdefault(x >> shift, []).append(x)
    arr = []
    for b in sorted(buckets):
        v = buckets[b]
        rng.shuffle(v)
        arr += v
    return keys, arr, max((len(v) for v in buckets.values()), default=0)


def test_two_pass_windows_sort_small_buckets():
    rng = random.Random(12)
    for w, cap in ((8, 5), (16, 9)):
        done = 0
        for _ in range(4000):
            n = rng.randint(0, 400)
            kb = rng.randint(13, 32)
            keys, arr, cmax = _bucketed(rng, n, kb, kb - 12, cap)
            if cmax <= cap:
                assert _two_pass(arr, w) == sorted(keys)
                done += 1
        assert done > 1000
        # a bucket of the largest size at every position relative to the windows
        for start in range(0, 3 * w):
            for c in range(1, cap + 1):
                arr = list(range(start)) + [start + c - 1 - i for i in range(c)] + \
                    list(range(start + c, start + c + 2 * w))
                assert _two_pass(arr, w) == sorted(arr), (w, start, c)


def test_two_pass_windows_can_fail_beyond_the_bound():
    # a bucket of W/2 + 2 keys straddling both window grids is not always sorted
    w = 8
    start = 3
    c = w // 2 + 2
    arr = list(range(start)) + [start + c - 1 - i for i in range(c)] + list(range(start + c, 40))
    assert _two_pass(arr, w) != sorted(arr)
