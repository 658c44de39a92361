"""Benchmark: n = 2^30 distinct values of 1..2^48 (seed 7), sorted uint64,
one MI355X; also the batched path against per-instance plain launches on
4096 uneven instances, and serving latency (p50/p99) under Poisson arrivals.

One step = one full sample (tree kernel + leaf kernel) into a resident 8 GiB
output buffer.  Prints one JSON line: samples/s, the leaf kernel's achieved
HBM-write bandwidth against the 8 TB/s peak (algorithmic bytes: 8 B per
sample written, nothing read), and the CPU oracle timed on a bounded window
of the same sample on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
N_SAMPLE = 1 << 30
UNIVERSE = 1 << 48
SEED = 7
N0 = 4096
BYTES_PER_SAMPLE = 8


# HBM bytes per launch of each configuration's dominant kernel, from rocprofv3
# FETCH_SIZE and WRITE_SIZE passes scaled by the same counters on a 1 GiB copy
# (x2.0 and x1.0; the profile summaries under profiles/ give the commands and
# raw figures), next to the kernel's algorithmic bytes.  They describe the
# kernels as built from the sources with this digest and are reported only
# while the sources still match it.
TRAFFIC_SOURCES_SHA256 = "431c57e9dcd1f5baf469f65b8ad6f8d117199f33f06d809519e880a0cee3b159"
LEAF_TRAFFIC = {  # k_leaf_pow2, n = 2^30 of N = 2^48
    "fetch_bytes": 70_600_684,      # 34473.0 KiB FETCH_SIZE x 2.0
    "write_bytes": 8_877_810_144,   # 8669736.5 KiB WRITE_SIZE x 1.0
}
CONFIG_TRAFFIC = {
    "c1_wor_2^20_of_2^32": {"kernel": "k_leaf_pow2", "fetch_bytes": 655_498,
        "write_bytes": 12_126_592, "algorithmic_bytes": 8_388_608},
    "c2b_wor_dense_2^29_of_2^30": {"kernel": "k_leaf_dense", "fetch_bytes": 38_021_868,
        "write_bytes": 4_831_421_120, "algorithmic_bytes": 4_294_967_296},
    "c3a_bernoulli_p0.01_of_2^36": {"kernel": "k_bern_wave", "fetch_bytes": 228_354_369,
        "write_bytes": 5_894_884_217, "algorithmic_bytes": 5_497_618_384},
    "c3b_wr_2^28_of_2^40": {"kernel": "k_leaf_pow2", "fetch_bytes": 23_125_584,
        "write_bytes": 2_228_530_617, "algorithmic_bytes": 2_147_483_648},
    "c2b_wholerange_B_2^29_of_2^30": {"kernel": "k_wb_write", "fetch_bytes": 171_987_807,
        "write_bytes": 4_669_660_403, "algorithmic_bytes": 4_362_099_332},
}
KERNEL_SOURCES = ("dcs_kernels.hip", "dcs_kernels.hpp", "dcs_device.hpp")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1610_05141_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    if TRAFFIC_SOURCES_SHA256 != kernel_sources_digest():
        return None
    return LEAF_TRAFFIC["fetch_bytes"] + LEAF_TRAFFIC["write_bytes"]


def config_traffic(name: str):
    """Recorded HBM bytes of a configuration's dominant kernel, or None when
    none were taken or the kernel sources have changed since."""
    t = CONFIG_TRAFFIC.get(name)
    if t is None or TRAFFIC_SOURCES_SHA256 != kernel_sources_digest():
        return None
    return dict(t, traffic_bytes=t["fetch_bytes"] + t["write_bytes"],
                traffic_over_algorithmic=(t["fetch_bytes"] + t["write_bytes"])
                / t["algorithmic_bytes"])


def host_description() -> dict:
    """What the CPU baseline ran on: logical CPUs, those this process may
    use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def cpu_baseline(gpu_out, budget_s: float = 12.0, max_threads: int = 16):
    """The oracle (plain C) on a window of the same sample, sized to about
    `budget_s` seconds on one thread; then the same window on all usable
    cores (up to `max_threads`), split into consecutive sub-windows that
    each thread computes on its own (each visits only the subtrees that
    overlap it, so the pieces concatenate to the same values); also checks
    the GPU's values there."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.build()
    # calibrate on a small window, then size the timed one
    t0 = time.perf_counter()
    oracle.sample_window(N_SAMPLE, UNIVERSE, SEED, 0, 1 << 20)
    rate = (1 << 20) / max(time.perf_counter() - t0, 1e-6)
    count = int(min(N_SAMPLE, max(1 << 20, rate * budget_s)))
    start = (N_SAMPLE - count) // 2
    t0 = time.perf_counter()
    want = oracle.sample_window(N_SAMPLE, UNIVERSE, SEED, start, count)
    dt1 = time.perf_counter() - t0
    threads = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    bounds = [start + count * k // threads for k in range(threads + 1)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        pieces = list(ex.map(lambda k: oracle.sample_window(
            N_SAMPLE, UNIVERSE, SEED, bounds[k], bounds[k + 1] - bounds[k]), range(threads)))
    dtn = time.perf_counter() - t0
    same = bool(np.array_equal(np.concatenate(pieces), want))
    got = gpu_out[start:start + count].cpu().numpy().view(np.uint64)
    return {
        "value": count / dtn,
        "unit": "samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"window of {count} consecutive outputs (offset {start}) of the same "
                  f"n=2^30, N=2^48, seed=7 sample: {dtn:.2f} s on {threads} threads "
                  f"(consecutive sub-windows), {dt1:.1f} s on one thread",
        "single_thread": {"value": count / dt1, "unit": "samples/s", "cores": 1},
        "threads_match_single": same,
        "host": host_description(),
        "matches_gpu": bool(np.array_equal(got, want)),
    }


def bench_batched(dcs, reps: int = 3, plain: bool = True):
    """4096 uneven instances (n log-uniform in [2^8, 2^22], density in
    [1e-6, 0.5], seeds 0..4095): one hipGraph-replayed batch vs one plain
    dcs_sample call per instance on one stream (synchronized once)."""
    import torch
    from paper_1610_05141_amd import autotune
    from paper_1610_05141_amd.workloads import batched_instances
    insts = batched_instances(4096)
    table = autotune.load_table()
    specs, off = [], 0
    for x in insts:
        n0 = autotune.n0_for(x.n, x.N, table)  # the autotuner's recorded leaf size
        specs.append(dcs.InstanceSpec(n=x.n, N=x.N, seed=x.seed, out_offset=off, n0=n0))
        off += x.n
    total = off
    out = torch.empty(total, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    b = dcs.Batch(specs)
    with torch.cuda.stream(stream):
        b.run(out, use_graph=True, stream=stream)  # capture + first replay
    dcs.synchronize(stream)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(reps):
            b.run(out, use_graph=True, stream=stream)
    dcs.synchronize(stream)
    batched_s = (time.perf_counter() - t0) / reps
    if not plain:  # the batch alone (e.g. under a counter profiler)
        b.close()
        del out
        torch.cuda.empty_cache()
        return {"samples": total, "batched_ms": batched_s * 1e3,
                "batched_samples_per_s": total / batched_s}
    # plain: one call per instance into the same buffer
    with torch.cuda.stream(stream):
        for s_, x in zip(specs, insts):
            dcs.sample(x.n, x.N, x.seed, out=out[s_.out_offset:s_.out_offset + x.n], stream=stream,
                       n0=s_.n0)
    dcs.synchronize(stream)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for s_, x in zip(specs, insts):
            dcs.sample(x.n, x.N, x.seed, out=out[s_.out_offset:s_.out_offset + x.n], stream=stream,
                       n0=s_.n0)
    dcs.synchronize(stream)
    plain_s = time.perf_counter() - t0
    b.close()
    del out
    torch.cuda.empty_cache()
    return {
        "workload": "4096 instances, n log-uniform in [2^8, 2^22], n/N log-uniform in "
                    "[1e-6, 0.5], seeds 0..4095, without replacement",
        "samples": total,
        "batched_ms": batched_s * 1e3,
        "batched_samples_per_s": total / batched_s,
        "plain_ms": plain_s * 1e3,
        "speedup_vs_plain": plain_s / batched_s,
        "leaf_sizes": {str(k): sum(1 for s_ in specs if s_.n0 == k)
                       for k in sorted({s_.n0 for s_ in specs})},
        "tuning_table": "paper_1610_05141_amd/tune_table.json" if table else None,
    }


OTHER_CONFIGS = [
    ("c1_wor_2^20_of_2^32", "wor", (1 << 20, 1 << 32, 1)),
    ("c2b_wor_dense_2^29_of_2^30", "wor", (1 << 29, 1 << 30, 7)),
    ("c3a_bernoulli_p0.01_of_2^36", "bern", (0.01, 1 << 36, 7)),
    ("c3b_wr_2^28_of_2^40", "wr", (1 << 28, 1 << 40, 7)),
    # the same dense workload as c2b by whole-range Algorithm B with the repair
    # on the device (Sec. 5's GPU variant), for comparison with the tree
    ("c2b_wholerange_B_2^29_of_2^30", "wb", (1 << 29, 1 << 30, 7)),
]


def bench_other_configs(dcs, reps: int = 5, only=None):
    """Throughput of the other configurations (same timing method: K calls,
    inputs resident, kernel durations from HIP events on the launch stream).
    `only`: names (or name prefixes such as "c3a") to restrict to."""
    import torch
    res = {}
    stream = torch.cuda.current_stream()
    cases = [c for c in OTHER_CONFIGS
             if only is None or any(c[0] == o or c[0].startswith(o + "_") for o in only)]
    for name, kind, args in cases:
        if kind == "bern":
            p, N, seed = args
            cap = dcs.bernoulli_capacity_hint(p, N)
            out = torch.empty(cap, dtype=torch.int64, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            run = lambda: dcs.sample_bernoulli(p, N, seed, out=out, capacity=cap, count=cnt,
                                               stream=stream)
            kernels = {"k_bern": 3}
        elif kind == "wb":
            n, N, seed = args
            out = torch.empty(n, dtype=torch.int64, device="cuda")
            run = lambda: dcs.sample_wholerange(n, N, seed, out=out, stream=stream)
            kernels = {"k_wb_count": 9, "k_wb_mid": 10, "k_wb_write": 11}
        else:
            n, N, seed = args
            out = torch.empty(n, dtype=torch.int64, device="cuda")
            f = dcs.sample if kind == "wor" else dcs.sample_replacement
            run = lambda: f(n, N, seed, out=out, stream=stream)
            kernels = {"k_leaf_pow2": 4, "k_leaf_mixed": 5, "k_leaf_dense": 6,
                       "k_leaf_small": 12, "k_leaf_once": 13}
        run()
        dcs.synchronize(stream)
        # calls of small samples last tens of microseconds: time more of them
        creps = reps if kind in ("bern", "wb") or args[0] >= (1 << 24) else 40 * reps
        t0 = time.perf_counter()
        for _ in range(creps):
            run()
        dcs.synchronize(stream)
        dt = (time.perf_counter() - t0) / creps
        # kernel durations from `reps` more calls, with HIP events around
        # every kernel (outside the timed calls, whose launches they would slow)
        dcs.profile_enable(True)
        for _ in range(reps):
            run()
        dcs.synchronize(stream)
        avgs = {}
        for kname, kind_id in kernels.items():
            k_ms, k_n = dcs.profile_read(kind_id)
            # whole-range B enqueues a second attempt that returns at once:
            # report its kernels per call
            avgs[kname] = k_ms / (reps if kind == "wb" else max(k_n, 1))
        t_ms, t_n = dcs.profile_read(1)
        dcs.profile_enable(False)
        samples = int(cnt.item()) if kind == "bern" else args[0]
        dom = max(avgs, key=avgs.get)
        k_avg = avgs[dom]
        res[name] = {
            "samples": samples,
            "ms_per_call": dt * 1e3,
            "samples_per_s": samples / dt,
            "dominant_kernel": dom,
            "dominant_kernel_ms": k_avg,
            "kernels_ms": avgs,
            "dominant_kernel_write_GBs": 8 * samples / (k_avg * 1e-3) / 1e9 if k_avg > 0 else None,
            "tree_ms": (t_ms / t_n) if t_n else None,
            "traffic": config_traffic(name),
        }
        del out
        torch.cuda.empty_cache()
    return res


def time_calls(dcs, run, reps, stream, kinds=()):
    """(seconds per call, {kind: (ms, launches)}, the last call's result):
    `reps` calls back to back with no HIP events, then, for the kernel
    durations of `kinds`, `reps` more with events around every kernel (the
    events slow the launches of short calls, so they stay out of the timing)."""
    dcs.synchronize(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        last = run()
    dcs.synchronize(stream)
    dt = (time.perf_counter() - t0) / reps
    prof = {}
    if kinds:
        dcs.profile_enable(True)
        for _ in range(reps):
            run()
        dcs.synchronize(stream)
        prof = {k: dcs.profile_read(k) for k in kinds}
        dcs.profile_enable(False)
    return dt, prof, last


def bench_parts(dcs, depths=(4, 8), reps: int = 3):
    """Online sampling in parts (Sec. 4.1): the n = 2^30 of 2^48 sample
    produced part by part, all 2^d parts of the depth-d cut in order, into
    one reused buffer (a streaming consumer's memory bound), against the
    whole sample in one call."""
    import torch
    stream = torch.cuda.current_stream()
    n, N, seed = N_SAMPLE, UNIVERSE, SEED
    res = {"workload": f"without-replacement sample n=2^30 of N=2^48, seed={seed}, "
                       "streamed part by part"}
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    dcs.sample(n, N, seed, out=out, stream=stream, n0=N0)
    dcs.synchronize(stream)
    t0 = time.perf_counter()
    for _ in range(reps):
        dcs.sample(n, N, seed, out=out, stream=stream, n0=N0)
    dcs.synchronize(stream)
    plain_ms = (time.perf_counter() - t0) / reps * 1e3
    del out
    torch.cuda.empty_cache()
    res["plain_ms"] = plain_ms
    cr = torch.zeros(2, dtype=torch.int64, device="cuda")
    for d in depths:
        per = n >> d
        cap = per + per // 8 + (1 << 16)
        buf = torch.empty(cap, dtype=torch.int64, device="cuda")

        def sweep():
            for g in range(1 << d):
                dcs.sample_part(n, N, seed, d, g, out=buf, capacity=cap, count_rank=cr,
                                stream=stream, n0=N0)

        sweep()
        dt, prof, _ = time_calls(dcs, sweep, reps, stream, (1, 2))
        (t_ms, t_n), (l_ms, l_n) = prof[1], prof[2]
        count, rank = (int(x) for x in cr.cpu())
        res[f"depth_{d}"] = {
            "parts": 1 << d,
            "buffer_bytes": 8 * cap,
            "ms_all_parts": dt * 1e3,
            "ms_per_part": dt * 1e3 / (1 << d),
            "samples_per_s": n / dt,
            "tree_ms_per_part": t_ms / max(t_n, 1),
            "leaf_ms_per_part": l_ms / max(l_n, 1),
            "vs_one_call": plain_ms / (dt * 1e3),
            "last_part_ends_at_n": count + rank == n,
        }
        del buf
        torch.cuda.empty_cache()
    # Sessions: the part roots computed once, then runs of `run` consecutive
    # parts per call into one reused buffer (its size: the largest run).
    for d, run in ((8, 1), (8, 16), (12, 256)):
        t0 = time.perf_counter()
        o = dcs.Online(n, N, seed, d, n0=N0, stream=stream)
        create_ms = (time.perf_counter() - t0) * 1e3
        counts, _ = o.counts()
        cap = max(int(counts[g:g + run].sum()) for g in range(0, 1 << d, run))
        buf = torch.empty(cap, dtype=torch.int64, device="cuda")

        def sweep():
            total = 0
            for g in range(0, 1 << d, run):
                total += o.next(g, run, buf, stream=stream)
            return total

        sweep()
        dt, prof, total = time_calls(dcs, sweep, reps, stream, (1, 2))
        (t_ms, t_n), (l_ms, l_n) = prof[1], prof[2]
        calls = (1 << d) // run
        res[f"session_depth_{d}_run_{run}"] = {
            "parts": 1 << d,
            "parts_per_call": run,
            "buffer_bytes": 8 * cap,
            "create_ms": create_ms,
            "ms_all_parts": dt * 1e3,
            "ms_per_call": dt * 1e3 / calls,
            "samples_per_s": n / dt,
            "tree_ms_per_call": t_ms / max(t_n, 1),
            "leaf_ms_per_call": l_ms / max(l_n, 1),
            "vs_one_call": plain_ms / (dt * 1e3),
            "all_values": total == n,
        }
        o.close()
        del buf
        torch.cuda.empty_cache()
    return res


def bench_segments(dcs, reps: int = 5):
    """Uneven universe (Sec. 4.3): n = 2^28 of the concatenation of 4096
    segments with sizes log-uniform in [2^16, 2^40] (about 2^48 elements),
    against the plain sample of n of the same N; the segment-split kernel,
    tree and leaf stage timed with HIP events."""
    import torch
    from paper_1610_05141_amd import workloads
    stream = torch.cuda.current_stream()
    L = workloads.segment_lengths(4096, 16, 40)
    n, N, seed = 1 << 28, sum(L), SEED
    res = {"workload": f"n=2^28 of {len(L)} segments, sizes log-uniform in [2^16, 2^40], "
                       f"N={N}, seed={seed}"}
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    cnt = torch.empty(len(L), dtype=torch.int64, device="cuda")
    cases = {
        "segments": (lambda: dcs.sample_segments(n, L, seed, out=out, counts=cnt, stream=stream),
                     {"split_ms": 8, "tree_ms": 1, "leaf_stage_ms": 2}),
        "plain_same_n_N": (lambda: dcs.sample(n, N, seed, out=out, stream=stream),
                           {"tree_ms": 1, "leaf_stage_ms": 2}),
    }
    for name, (run, kinds) in cases.items():
        run()
        dt, prof, _ = time_calls(dcs, run, reps, stream, tuple(kinds.values()))
        r = {"ms_per_call": dt * 1e3, "samples_per_s": n / dt}
        for key, kind in kinds.items():
            k_ms, k_n = prof[kind]
            r[key] = k_ms / max(k_n, 1)
        res[name] = r
    d = out[1:] - out[:-1]
    res["invariants_ok"] = bool((d > 0).all()) and int(out[0]) >= 1 and int(out[-1]) <= N
    del out, cnt, d
    torch.cuda.empty_cache()
    return res


def bench_graph(dcs, reps: int = 5):
    """Random graphs (Sec. 7): G(n, m) with m = 2^28 edges on n = 2^26
    vertices, and G(n, p) on the same vertices with p = 2^-23 (2^28 edges
    expected): whole-call edges/s, and the in-place index decoding kernel
    against HBM (8 B read + 8 B written per edge)."""
    import torch
    stream = torch.cuda.current_stream()
    n, m, seed = 1 << 26, 1 << 28, 7
    p = 2.0 ** -23
    res = {"workload": f"G(n, m) and G(n, p) on n=2^26 vertices, m=2^28, p=2^-23, seed={seed}"}
    e = torch.empty((m, 2), dtype=torch.int32, device="cuda")
    N = n * (n - 1) // 2
    cap = dcs.bernoulli_capacity_hint(p, N)
    eg = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    # G(n, m) on 2^30 vertices: about 2^59 pairs, beyond 2^53
    n_big, m_big = 1 << 30, 1 << 24
    cases = {
        "gnm": (lambda: dcs.sample_edges_gnm(n, m, seed, out=e, stream=stream), None),
        "gnp": (lambda: dcs.sample_edges_gnp(n, p, seed, out=eg, capacity=cap, count=cnt,
                                             stream=stream), cnt),
        "gnm_2^30_vertices_2^24_edges": (
            lambda: dcs.sample_edges_gnm(n_big, m_big, seed, out=e[:m_big], stream=stream),
            m_big),
    }
    for name, (run, count) in cases.items():
        run()
        dt, prof, _ = time_calls(dcs, run, reps, stream, (7,))
        d_ms, d_n = prof[7]
        edges = m if count is None else (count if isinstance(count, int) else int(count.item()))
        dec = d_ms / max(d_n, 1)
        res[name] = {
            "edges": edges,
            "ms_per_call": dt * 1e3,
            "edges_per_s": edges / dt,
            "decode_kernel_ms": dec,
            "decode_GBs": 16 * edges / (dec * 1e-3) / 1e9 if dec > 0 else None,
        }
    del e, eg
    torch.cuda.empty_cache()
    return res


def bench_serving(dcs, rate: float = 20000.0, warm: int = 10000, timed: int = 100000):
    """Open-loop Poisson arrivals at `rate`/s of instances drawn like the
    batched workload (n capped at 2^24), admitted by output footprint under a
    64 GiB arena; latency from scheduled arrival to completion."""
    from paper_1610_05141_amd.workloads import batched_instances, poisson_arrivals
    insts = batched_instances(warm + timed, n_cap_log2=24, key=0xC5)
    srv = dcs.Server(arena_bytes=64 << 30, max_batch=4096, n_streams=4, auto_release=True)
    reqs = [(x.n, x.N, x.seed) for x in insts]
    t0 = dcs.Server.now() + 0.05
    arr = [t0 + t for t in poisson_arrivals(len(reqs), rate, key=0xC5)]
    srv.submit_schedule(reqs[:warm], arr[:warm])
    srv.drain()
    warm_stats = srv.stats()
    srv.close()
    # fresh server for the timed part so that the statistics hold only it
    srv = dcs.Server(arena_bytes=64 << 30, max_batch=4096, n_streams=4, auto_release=True)
    t1 = dcs.Server.now() + 0.05
    base = arr[warm]
    srv.submit_schedule(reqs[warm:], [t1 + (t - base) for t in arr[warm:]])
    srv.drain()
    st = srv.stats()
    srv.close()
    return {
        "workload": f"Poisson {rate:.0f} req/s, n log-uniform in [2^8, 2^22], density "
                    "[1e-6, 0.5], 64 GiB admission cap, without replacement",
        "requests": st["completed"],
        "warmup_requests": warm_stats["completed"],
        "p50_ms": st["p50_s"] * 1e3,
        "p99_ms": st["p99_s"] * 1e3,
        "max_ms": st["max_s"] * 1e3,
        "samples_per_s": st["samples"] / st["span_s"] if st["span_s"] > 0 else None,
        "offered_samples_per_s": rate * (sum(r[0] for r in reqs[warm:]) / max(timed, 1)),
        "batches": st["batches"],
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for counter scaling)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-parts", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-segments", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="batched: time the batch without the per-instance plain calls")
    ap.add_argument("--only", default=None,
                    help="comma list of other configurations (c1, c2b, c3a, c3b, batched, "
                         "parts, graph, segments, serving) to run alone, e.g. under a profiler; "
                         "prints their lines only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampler shards across GPUs without communication)", file=sys.stderr)
        return 2

    import torch
    import paper_1610_05141_amd as dcs

    torch.cuda.set_device(0)

    def copy_calibration():
        # 1 GiB fill (writes 2^30 B) then 1 GiB copy (reads and writes 2^30 B)
        a = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
        b = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
        b.fill_(1)
        a.copy_(b)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    if args.only:
        if args.copy_calibration:
            copy_calibration()
        names = args.only.split(",")
        res = {}
        other = [x for x in names if x not in ("batched", "serving", "parts", "graph", "segments")]
        if other:
            res.update(bench_other_configs(dcs, reps=args.steps, only=other))
        if "batched" in names:
            res["batched"] = bench_batched(dcs, plain=not args.batched_only)
        if "parts" in names:
            res["parts"] = bench_parts(dcs)
        if "graph" in names:
            res["graph"] = bench_graph(dcs)
        if "segments" in names:
            res["segments"] = bench_segments(dcs)
        if "serving" in names:
            res["serving"] = bench_serving(dcs)
        print(json.dumps(res), flush=True)
        return 0
    stream = torch.cuda.current_stream()
    out = torch.empty(N_SAMPLE, dtype=torch.int64, device="cuda")
    print(f"[bench] warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        dcs.sample(N_SAMPLE, UNIVERSE, SEED, out=out, stream=stream, n0=N0)
    dcs.synchronize(stream)

    if args.copy_calibration:
        copy_calibration()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    # inside the timed steps only the roofline kernel carries HIP events
    dcs.profile_kinds([4])
    dcs.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dcs.sample(N_SAMPLE, UNIVERSE, SEED, out=out, stream=stream, n0=N0)
    dcs.synchronize(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    leaf_ms, leaf_n = dcs.profile_read(4)     # the power-of-two leaf kernel
    # the other kernels' durations, from a few untimed steps with every kind timed
    dcs.profile_kinds(None)
    dcs.profile_enable(True)
    for _ in range(3):
        dcs.sample(N_SAMPLE, UNIVERSE, SEED, out=out, stream=stream, n0=N0)
    dcs.synchronize(stream)
    stage_ms, stage_n = dcs.profile_read(2)
    mixed_ms, mixed_n = dcs.profile_read(5)   # work-group leaf kernel of the other kinds
    dense_ms, dense_n = dcs.profile_read(6)   # one-wave dense leaf kernel
    small_ms, small_n = dcs.profile_read(12)  # one-wave small leaf kernel
    once_ms, once_n = dcs.profile_read(13)    # one-pass kernel of repeating sparse leaves
    tree_ms, tree_n = dcs.profile_read(1)
    reset_ms, reset_n = dcs.profile_read(0)
    dcs.profile_enable(False)

    ms_per_step = elapsed * 1e3 / args.steps
    value = N_SAMPLE * args.steps / elapsed
    leaf_avg_ms = leaf_ms / max(leaf_n, 1)
    achieved = BYTES_PER_SAMPLE * N_SAMPLE / (leaf_avg_ms * 1e-3) / 1e9

    # properties that hold at any size, checked on the timed output
    d = out[1:] - out[:-1]
    props_ok = bool((d > 0).all()) and int(out[0]) >= 1 and int(out[-1]) <= UNIVERSE
    del d

    rec = {
        "metric": "samples/s (n=2^30 of N=2^48, sorted uint64, without replacement)",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "without-replacement sample, n=2^30 of N=2^48, seed=7, n0=4096",
                   "n": N_SAMPLE, "N": UNIVERSE, "seed": SEED, "n0": N0,
                   "output_bytes": BYTES_PER_SAMPLE * N_SAMPLE},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic(),
            "kernel": "k_leaf_pow2",
            "kernel_avg_ms": leaf_avg_ms,
        },
        "geometry": {"cut_bias,leaf_wgs_per_cu": list(dcs.tune_get(0, 30))},
        "kernels_ms_per_step": {"reset": reset_ms / max(reset_n, 1),
                                "tree": tree_ms / max(tree_n, 1),
                                "k_leaf_pow2": leaf_avg_ms,
                                "k_leaf_mixed": mixed_ms / max(mixed_n, 1),
                                "k_leaf_dense": dense_ms / max(dense_n, 1),
                                "k_leaf_small": small_ms / max(small_n, 1),
                                "k_leaf_once": once_ms / max(once_n, 1),
                                "leaf_stage": stage_ms / max(stage_n, 1)},
        "whole_step_write_GBs": BYTES_PER_SAMPLE * N_SAMPLE / (ms_per_step * 1e-3) / 1e9,
        "invariants_ok": props_ok,
    }
    del out
    torch.cuda.empty_cache()
    if not args.no_configs:
        print("[bench] other configurations", file=sys.stderr, flush=True)
        rec["configs"] = bench_other_configs(dcs)
    if not args.no_batched:
        print("[bench] batched vs plain", file=sys.stderr, flush=True)
        rec["batched"] = bench_batched(dcs)
    if not args.no_parts:
        print("[bench] online parts", file=sys.stderr, flush=True)
        rec["parts"] = bench_parts(dcs)
    if not args.no_graph:
        print("[bench] random graphs", file=sys.stderr, flush=True)
        rec["graph"] = bench_graph(dcs)
    if not args.no_segments:
        print("[bench] uneven universe", file=sys.stderr, flush=True)
        rec["segments"] = bench_segments(dcs)
    if not args.no_serving:
        print("[bench] serving", file=sys.stderr, flush=True)
        rec["serving"] = bench_serving(dcs)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out = torch.empty(N_SAMPLE, dtype=torch.int64, device="cuda")
        dcs.sample(N_SAMPLE, UNIVERSE, SEED, out=out, stream=stream, n0=N0)
        dcs.synchronize(stream)
        rec["cpu_baseline"] = cpu_baseline(out)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
