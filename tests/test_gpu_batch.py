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


def _bench_batch_specs(m):
    """The batched workload exactly as the benchmark builds it: 4096
    instances, each with the leaf size the autotuner recorded for its class
    (floor(log2 n), dense or sparse)."""
    from paper_1610_05141_amd import autotune
    insts = batched_instances(4096)
    table = autotune.load_table()
    specs, off = [], 0
    for x in insts:
        specs.append(m.InstanceSpec(n=x.n, N=x.N, seed=x.seed, out_offset=off,
                                    n0=autotune.n0_for(x.n, x.N, table)))
        off += x.n
    return insts, specs, off


def _check_instances_sorted_in_range(out, specs, insts):
    """On the GPU: every instance strictly increasing, first value >= 1 and
    last <= N (hence all values distinct and in 1..N)."""
    import torch
    total = out.numel()
    starts = torch.tensor([s.out_offset for s in specs], dtype=torch.int64, device="cuda")
    ends = torch.tensor([s.out_offset + x.n - 1 for s, x in zip(specs, insts)],
                        dtype=torch.int64, device="cuda")
    Ns = torch.tensor([x.N for x in insts], dtype=torch.int64, device="cuda")
    assert bool((out[starts] >= 1).all()), "a first value below 1"
    assert bool((out[ends] <= Ns).all()), "a last value above its N"
    first = torch.zeros(total, dtype=torch.bool, device="cuda")
    first[starts] = True  # positions where a new instance begins
    step = 1 << 27
    for a in range(0, total - 1, step):
        b = min(total - 1, a + step)
        ok = (out[a + 1:b + 1] > out[a:b]) | first[a + 1:b + 1]
        if not bool(ok.all()):
            j = a + 1 + int(torch.nonzero(~ok)[0].item())
            raise AssertionError(f"not strictly increasing at output {j}")


def test_config4_batch_as_benchmarked(ref):
    """The benchmark's batch (recorded leaf sizes, hipGraph capture and
    replay).  Checked: (1) every instance sorted, distinct and in 1..N, on the
    GPU; (2) every instance equal to the same instance sampled alone by a
    plain call with the same leaf size; (3) at least 256 instances, covering
    every (floor(log2 n), dense/sparse, n0) class present, equal to the
    oracle with that leaf size; (4) three more graph replays, with eager work
    in between, equal to the first."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    m = dcs()
    insts, specs, total = _bench_batch_specs(m)
    announce(f"config 4 batch as benchmarked, {total} samples, graph replay")
    b = m.Batch(specs)
    out = torch.zeros(total, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        b.run(out, use_graph=True, stream=stream)  # capture + first replay
    m.synchronize(stream)
    _check_instances_sorted_in_range(out, specs, insts)
    # (2) alone == in the batch, all 4096 (plain calls, as the benchmark's
    # per-instance leg makes them)
    announce("config 4: every instance alone")
    alone = torch.zeros_like(out)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        for s, x in zip(specs, insts):
            m.sample(x.n, x.N, x.seed, out=alone[s.out_offset:s.out_offset + x.n],
                     stream=stream, n0=s.n0)
    m.synchronize(stream)
    if not torch.equal(out, alone):
        for i, (s, x) in enumerate(zip(specs, insts)):
            seg = slice(s.out_offset, s.out_offset + x.n)
            assert torch.equal(out[seg], alone[seg]), f"instance {i} {x} n0={s.n0}: batch != alone"
    del alone
    # (3) the oracle on >= 256 instances covering every class
    classes = {}
    for i, (s, x) in enumerate(zip(specs, insts)):
        key = (x.n.bit_length() - 1, 16 * x.n >= x.N, s.n0)
        classes.setdefault(key, []).append(i)
    pick = set()
    for idx in classes.values():
        pick.update([idx[0], idx[-1]])
    rng = np.random.default_rng(4)
    while len(pick) < 256:
        pick.add(int(rng.integers(0, len(insts))))
    pick = sorted(pick)
    announce(f"config 4: oracle on {len(pick)} instances, {len(classes)} classes")
    with ThreadPoolExecutor(max_workers=8) as ex:
        wants = list(ex.map(lambda i: ref.sample(insts[i].n, insts[i].N, insts[i].seed,
                                                 n0=specs[i].n0), pick))
    for i, want in zip(pick, wants):
        s, x = specs[i], insts[i]
        g = to_np_u64(out[s.out_offset:s.out_offset + x.n])
        assert np.array_equal(g, want), f"instance {i} {x} n0={s.n0}: {first_mismatch(g, want)}"
    # (4) replays of the captured graph, eager work in between
    out2 = torch.zeros_like(out)
    for rep in range(3):
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            b.run(out2, use_graph=True, stream=stream)
        m.synchronize(stream)
        assert torch.equal(out, out2), f"graph replay {rep} differs"
        out2.fill_(-1)
        m.sample(1000, 1 << 20, rep)  # eager library work between replays
        m.synchronize()
    b.close()


def test_config4_batch_n0_4096_eager(ref):
    """The same 4096 instances at the default leaf size, eager launches:
    a sample of instances against the oracle."""
    import torch
    m = dcs()
    insts = batched_instances(4096)
    specs, total = _specs(m, insts)
    announce(f"config 4 batch at n0=4096, {total} samples")
    b = m.Batch(specs)
    out = torch.empty(total, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.run(out, use_graph=False, stream=stream)
    m.synchronize(stream)
    _check_instances_sorted_in_range(out, specs, insts)
    rng = np.random.default_rng(0)
    pick = sorted(set([0, len(insts) - 1] + [int(i) for i in rng.integers(0, len(insts), 40)]))
    for i in pick:
        s, x = specs[i], insts[i]
        g = to_np_u64(out[s.out_offset:s.out_offset + x.n])
        want = ref.sample(x.n, x.N, x.seed)
        assert np.array_equal(g, want), f"instance {i} {x}: {first_mismatch(g, want)}"
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
