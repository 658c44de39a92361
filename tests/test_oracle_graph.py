"""Pins for the oracle's random-graph samplers (CPU only; Sec. 7: G(n, m) is
a sample without replacement of the n(n-1)/2 possible edges, G(n, p) a
Bernoulli sample of them).  Edge index k is the pair (u, v), v < u, with
k = u(u-1)/2 + v: checked against enumeration of all pairs in that order
and against the triangular numbers at both ends of every row u."""
import numpy as np
import pytest

MAX_VERTICES = 94906266  # largest n with n(n-1)/2 <= 2^52


def test_edge_pair_enumerates_pairs_in_order(ref):
    k = 0
    for u in range(1, 300):
        for v in range(u):
            assert ref.edge_pair(k) == (u, v), k
            k += 1


@pytest.mark.parametrize("u", [2, 3, 1000, 2**20 + 7, 2**26, 2**26 + 12345, MAX_VERTICES - 1])
def test_edge_pair_at_row_ends(ref, u):
    first = u * (u - 1) // 2           # (u, 0)
    last = u * (u + 1) // 2 - 1        # (u, u - 1)
    assert ref.edge_pair(first) == (u, 0)
    assert ref.edge_pair(last) == (u, u - 1)
    assert ref.edge_pair(first - 1) == (u - 1, u - 2)


def _pack(e):
    return e[:, 0].astype(np.int64) << 32 | e[:, 1].astype(np.int64)


@pytest.mark.parametrize("n,m,seed", [(1000, 5000, 3), (50, 1225, 4), (2, 1, 5), (3000, 1, 6),
                                      (MAX_VERTICES, 3000, 7)])
def test_gnm_is_the_decoded_sample(ref, n, m, seed):
    e = ref.edges_gnm(n, m, seed)
    N = n * (n - 1) // 2
    idx = ref.sample(m, N, seed)
    want = np.array([ref.edge_pair(int(k) - 1) for k in idx], dtype=np.uint64)
    assert (e.astype(np.uint64) == want).all()
    assert (e[:, 1] < e[:, 0]).all() and (e[:, 0] < n).all()
    key = _pack(e)
    assert (np.diff(key) > 0).all()  # distinct edges in increasing (u, v) order


def test_gnm_complete_graph(ref):
    e = ref.edges_gnm(50, 1225, 9)  # m = n(n-1)/2: every pair once
    want = [(u, v) for u in range(1, 50) for v in range(u)]
    assert [tuple(int(x) for x in r) for r in e] == want


def test_gnp_degenerate_and_count(ref):
    assert len(ref.edges_gnp(100, 0.0, 1)) == 0
    full = ref.edges_gnp(60, 1.0, 1)
    assert [tuple(int(x) for x in r) for r in full] == [(u, v) for u in range(1, 60)
                                                         for v in range(u)]
    n, p = 3000, 0.01
    e = ref.edges_gnp(n, p, 2)
    N = n * (n - 1) // 2
    z = (len(e) - N * p) / np.sqrt(N * p * (1 - p))
    assert abs(z) < 5
    assert (np.diff(_pack(e)) > 0).all() and (e[:, 1] < e[:, 0]).all()
