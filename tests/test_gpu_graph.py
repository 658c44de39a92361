"""Random graphs G(n, m) and G(n, p) on the GPU (Sec. 7), through the C ABI:
edge lists equal to the oracle's bit for bit, and at 2^28 edges on 2^26
vertices, windows compared with the oracle's decoded sample plus order and
range properties over the whole list."""
import numpy as np
import pytest

from tests.gpu_util import announce, dcs, first_mismatch

pytestmark = pytest.mark.gpu

MAX_VERTICES = 94906266  # largest n with n(n-1)/2 <= 2^52 (the G(n, p) bound)
MAX_VERTICES_GNM = 3037000500  # largest n with n(n-1)/2 <= 2^62 (the G(n, m) bound)


def _np_edges(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n,m,seed", [
    (1000, 5000, 3),
    (50, 1225, 4),              # complete graph
    (2, 1, 5),
    (100000, 1 << 20, 6),       # ~2e-4 of all pairs, non-power-of-two universe
    (1 << 16, 1 << 20, 8),      # pairs of 2^16 vertices
    (MAX_VERTICES, 20000, 7),   # 2^52 pairs
    (1 << 30, 1 << 20, 10),     # 2^30 vertices: about 2^59 pairs
    (MAX_VERTICES_GNM, 30000, 11),  # largest universe of G(n, m)
    (3000, 0, 9),               # no edges
])
def test_gnm_matches_oracle(ref, n, m, seed):
    mod = dcs()
    announce(f"gnm n={n} m={m} seed={seed}")
    e = mod.sample_edges_gnm(n, m, seed)
    mod.synchronize()
    got = _np_edges(e).reshape(-1, 2)[:m]
    want = ref.edges_gnm(n, m, seed)
    assert np.array_equal(got, want), first_mismatch(got.ravel(), want.ravel())


@pytest.mark.parametrize("n,p,seed", [(2000, 0.01, 4), (300, 0.5, 5), (60, 1.0, 6),
                                      (100, 0.0, 7), (20000, 2e-4, 8)])
def test_gnp_matches_oracle(ref, n, p, seed):
    mod = dcs()
    announce(f"gnp n={n} p={p} seed={seed}")
    e, cnt = mod.sample_edges_gnp(n, p, seed)
    mod.synchronize()
    c = int(cnt.item())
    got = _np_edges(e).reshape(-1, 2)[:c]
    want = ref.edges_gnp(n, p, seed)
    assert c == len(want)
    assert np.array_equal(got, want), first_mismatch(got.ravel(), want.ravel())


def test_gnm_2p28_edges_on_2p26_vertices(ref):
    import torch
    mod = dcs()
    n, m, seed = 1 << 26, 1 << 28, 7
    N = n * (n - 1) // 2
    announce("gnm 2^28 edges on 2^26 vertices")
    e = mod.sample_edges_gnm(n, m, seed)
    mod.synchronize()
    for s in (0, m // 3, m - 4096):
        idx = ref.sample_window(m, N, seed, s, 4096)
        want = np.array([ref.edge_pair(int(k) - 1) for k in idx], dtype=np.uint32)
        got = _np_edges(e[s:s + 4096])
        assert np.array_equal(got, want), f"window {s}: {first_mismatch(got.ravel(), want.ravel())}"
    u = e[:, 0].to(torch.int64)
    v = e[:, 1].to(torch.int64)
    assert bool((v < u).all()) and bool((u < n).all()) and bool((v >= 0).all())
    key = u * n + v
    assert bool((key[1:] > key[:-1]).all())


def test_graphs_without_pairs(ref):
    """n_vertices 0 and 1 have no pairs: G(n, m) with m = 0, G(n, p) empty."""
    mod = dcs()
    announce("graphs without pairs")
    for nv in (0, 1):
        e = mod.sample_edges_gnm(nv, 0, 1)
        assert e.shape[0] == 0
        e, cnt = mod.sample_edges_gnp(nv, 0.5, 1)
        mod.synchronize()
        assert int(cnt.item()) == 0
