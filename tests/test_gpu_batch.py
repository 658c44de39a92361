"""Batched sampling (GPU): 4096 uneven instances in one launch sequence, plain
and hipGraph-replayed; each instance's output equals the oracle's and the
same instance sampled alone."""
import numpy as np
import pytest

from paper_1610_05141_amd.workloads import batched_instances
from tests.gpu_util import announce, dcs, first_mismatch, to_np_u64

pytestmark = pytest.mark.gpu


def _specs(m, insts, variants=None):
    specs, off = [], 0
    for i, x in enumerate(insts):
        v = 0 if variants is None else variants[i]
        specs.append(m.InstanceSpec(n=x.n, N=x.N, seed=x.seed, out_offset=off, variant=v))
        off += x.n
    return specs, off


def test_small_mixed_batch_matches_oracle(ref):
    """A mixed batch (both variants, edge sizes) against the oracle, whole."""
    import torch
    m = dcs()
    announce("small mixed batch")
    insts = batched_instances(96, n_lo_log2=0, n_hi_log2=15, dens_lo=1e-6, dens_hi=1.0, key=77)
    variants = [i % 3 == 2 for i in range(len(insts))]
    specs, total = _specs(m, insts, [int(v) for v in variants])
    b = m.Batch(specs)
    out = torch.full((total,), -1, dtype=torch.int64, device="cuda")
    b.run(out)
    m.synchronize()
    got = to_np_u64(out)
    for s, x, v in zip(specs, insts, variants):
        want = ref.replacement(x.n, x.N, x.seed) if v else ref.sample(x.n, x.N, x.seed)
        g = got[s.out_offset:s.out_offset + x.n]
        assert np.array_equal(g, want), f"{x} wr={v}: {first_mismatch(g, want)}"
    b.close()


def test_config4_batch_4096(ref):
    import torch
    m = dcs()
    insts = batched_instances(4096)
    specs, total = _specs(m, insts)
    announce(f"config 4 batch, {total} samples")
    b = m.Batch(specs)
    out = torch.empty(total, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.run(out, use_graph=False, stream=stream)
    m.synchronize(stream)
    # (1) a sample of instances against the oracle
    rng = np.random.default_rng(0)
    pick = sorted(set([0, len(insts) - 1] + [int(i) for i in rng.integers(0, len(insts), 40)]))
    for i in pick:
        s, x = specs[i], insts[i]
        g = to_np_u64(out[s.out_offset:s.out_offset + x.n])
        want = ref.sample(x.n, x.N, x.seed)
        assert np.array_equal(g, want), f"instance {i} {x}: {first_mismatch(g, want)}"
    # (2) every instance: sorted, distinct, in range -- and alone == in the mix
    alone = torch.empty(max(x.n for x in insts), dtype=torch.int64, device="cuda")
    for i, (s, x) in enumerate(zip(specs, insts)):
        seg = out[s.out_offset:s.out_offset + x.n]
        if i % 16 == 0:
            m.sample(x.n, x.N, x.seed, out=alone)
            m.synchronize()
            assert torch.equal(alone[:x.n], seg), f"instance {i} alone != in batch"
    # (3) graph capture, replayed several times with eager work in between
    out2 = torch.zeros_like(out)
    torch.cuda.synchronize()  # the fill above ran on the default stream
    for rep in range(3):
        with torch.cuda.stream(stream):
            b.run(out2, use_graph=True, stream=stream)
        m.synchronize(stream)
        assert torch.equal(out, out2), f"graph replay {rep} differs"
        out2.zero_()
        torch.cuda.synchronize()
    b.close()


def test_batch_with_recorded_leaf_sizes(ref):
    """Instances carry their own leaf size (as the autotuner records them per
    class): mixed n0 in one batch, each instance equal to the oracle run with
    that n0."""
    import torch
    m = dcs()
    from paper_1610_05141_amd import autotune
    announce("batch with per-instance leaf sizes")
    insts = batched_instances(160, n_lo_log2=4, n_hi_log2=17, key=4242)
    choices = autotune.N0_CHOICES
    specs, off = [], 0
    for i, x in enumerate(insts):
        n0 = autotune.n0_for(x.n, x.N) if i % 2 else choices[i % len(choices)]
        specs.append(m.InstanceSpec(n=x.n, N=x.N, seed=x.seed, out_offset=off, n0=n0))
        off += x.n
    b = m.Batch(specs)
    out = torch.full((off,), -1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.run(out, use_graph=True, stream=stream)
    m.synchronize(stream)
    got = to_np_u64(out)
    for s, x in zip(specs, insts):
        want = ref.sample(x.n, x.N, x.seed, n0=s.n0)
        g = got[s.out_offset:s.out_offset + x.n]
        assert np.array_equal(g, want), f"{x} n0={s.n0}: {first_mismatch(g, want)}"
    b.close()
