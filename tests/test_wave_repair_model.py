"""Host model of how the one-wave dense leaf chooses its repair values (CPU).

The dense leaf (Algorithm B, Sec. 2) removes the first r distinct values of
the REPAIR stream mapped into [0, n').  The wave kernel takes stream words 64
at a time, lane m holding word 64j + m of a 256-word Philox round; lanes
whose value is not yet removed set its bit with an atomic OR, lanes that
find the bit already set by another lane of the same step resolve the tie to
the lowest lane holding that value, a ballot ranks the first occurrences,
and the bits of first occurrences past the r-th are cleared again.  The
order in which the hardware serves the atomics of one step is not fixed;
this model plays the step with random service orders and checks that the
removed set is always the first r distinct values in stream order (the
definition the oracle implements).
"""
import random

import pytest


def first_distinct(values, r):
    """Definition: the first r distinct non-void values in stream order."""
    seen, out = set(), []
    for v in values:
        if v is None or v in seen:
            continue
        seen.add(v)
        out.append(v)
        if len(out) == r:
            break
    return set(out)


def wave_select(values, r, rng):
    """The kernel's selection, one 64-word step at a time; the atomics of a
    step are served in a random order."""
    mask, have, base = set(), 0, 0
    while have < r:
        for _j in range(4):
            if have >= r:
                break
            words = values[base:base + 64]
            words += [None] * (64 - len(words))
            base += 64
            fresh = [v is not None and v not in mask for v in words]
            # atomic OR in some order: the first served lane of a value sees
            # the bit clear, the others see it set
            served = set()
            raced = [False] * 64
            for lane in rng.sample(range(64), 64):
                if fresh[lane]:
                    if words[lane] in served:
                        raced[lane] = True
                    served.add(words[lane])
            mask |= served
            later = [False] * 64
            pending = {lane for lane in range(64) if raced[lane]}
            while pending:
                s = min(pending)
                same = [m for m in range(64) if fresh[m] and words[m] == words[s]]
                first = min(same)
                for m in same:
                    if m != first:
                        later[m] = True
                pending -= set(same)
            firsts = [fresh[m] and not later[m] for m in range(64)]
            need = r - have
            rank = 0
            for m in range(64):
                if firsts[m]:
                    if rank >= need:
                        mask.discard(words[m])
                    rank += 1
            have += min(rank, need)
    return mask


@pytest.mark.parametrize("range_size,r,void_rate", [
    (100, 30, 0.0),      # many repeats inside one step
    (4000, 200, 0.0),    # the typical leaf: ~3 sqrt(n) removals from ~4000 hits
    (64, 63, 0.0),       # nearly every value removed
    (5, 5, 0.3),         # tiny range with void words
    (3000, 150, 0.45),   # many void words (non-power-of-two n')
    (1, 1, 0.0),
])
def test_wave_selection_is_first_distinct(range_size, r, void_rate):
    rng = random.Random(range_size * 1000 + r)
    for _trial in range(300):
        n_words = 64 * 4 * (1 + (4 * r) // 64 + 40)
        values = [None if rng.random() < void_rate else rng.randrange(range_size)
                  for _ in range(n_words)]
        want = first_distinct(values, r)
        assert len(want) == r
        for _order in range(3):
            assert wave_select(values, r, rng) == want


def test_selection_ignores_repeats_of_removed_values():
    # a value removed in an earlier step repeats in a later step: not counted again
    values = [7] * 64 + [7, 8] + [None] * 62 + [9] * 64
    rng = random.Random(1)
    assert wave_select(values, 3, rng) == {7, 8, 9}
    assert wave_select(values, 2, rng) == {7, 8}
