#!/usr/bin/env python3
"""Benchmark of the batched dice-roll hot path on one MI355X.

The timed step is one pass of the flat dice stream: 2^28 u32 bounds uniform
in [1, 2^16) (seed 7) rolled k per 64-bit word (brr_dice, Theorem 1 chain +
Algorithm 3 acceptance), inputs resident in HBM. k = 1..4 are all timed; the
headline is the fastest batched k (2..4) unless --k fixes one, and k = 1
(the single-roll multiply-and-reject form) is reported beside it, with the
same stream at word width 32, in the division form of Sec. 2.1 (one roll of
the bound product, dice by successive remainders) and with bounds below
2^12. Secondary workloads report shuffled elements per second: 65,536
shuffles of 256 elements, 20,000 ragged shuffles (also autotuned,
exhaustively and by the learned model), one 10,000-element shuffle and one
2^26-element shuffle, each batched (shuffle_6), unbatched (k = 1) and with
the division-based pairs of the paper's comparison (naive shuffle_2),
shuffle_6 and k = 1 again on ChaCha20 words, and the L = 32 cost-model
schedule on 32-bit words; and the serving loop's latency under Poisson
load.

Prints one JSON line. Timing: HIP events recorded on the stream the kernels
are launched on (torch's current stream), K steps after W warmup steps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
COUNT = 1 << 28
BYTES_PER_ROLL = 8  # 4 B bound read + 4 B die written
KNOWN_BOUND = 65535  # the known-bounds stream: one bound, 65535^4 < 2^64

# Context, not a target: the paper's speed ratios of shuffle_6 over an
# unbatched Fisher-Yates shuffle of 64-bit elements on CPUs, ranges over its
# array sizes (Experiments section, speed-ratio figure and its discussion).
# The GPU ratios beside them are the secondary workloads' speedup_k6_vs_k1
# (Philox words: the fast generator) and chacha20_speedup_k6_vs_k1.
PAPER_CPU_SPEEDUPS = {
    "Intel Xeon Gold 6338 (3.2 GHz)": {"Lehmer128": [1.4, 1.8], "PCG64": [1.8, 2.5],
                                       "ChaCha": [2.9, 4.7]},
    "Apple M2 (3.49 GHz)": {"Lehmer128": [1.5, 2.3], "PCG64": [1.9, 2.6], "ChaCha": [2.6, 3.9]},
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dice.hip", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2408_06213_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(k):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current dice kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "dice_stream_2p28_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("per_k", {}).get(str(k))
    return None if ent is None else ent.get("bytes_per_launch")


def time_launches(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def launch_stats(fn, launches=20):
    """Per-launch times (HIP events around each launch on the launch
    stream): median, min, mean, and whether the min is within 10% of the
    mean."""
    import statistics

    import torch

    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(launches)]
    for a, b in ev:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    t = [a.elapsed_time(b) for a, b in ev]
    mean = sum(t) / len(t)
    return {"launches": launches, "median_ms": statistics.median(t), "min_ms": min(t),
            "mean_ms": mean, "min_within_10pct_of_mean": min(t) >= 0.9 * mean}


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def serving(brr, workloads, up, rates=(1000, 2000, 4000, 8000, 16000, 32000, 64000), count=400,
            clients=64, max_inflight=128, nstreams=32):
    """Poisson arrivals at each rate: requests (shuffle or sample, n
    log-uniform in [2^4, 2^22], u64 payload, m <= n/10) from `clients`
    independent clients (request i belongs to session i mod clients; a
    session's requests run in order) are submitted at their arrival times to
    a continuous-batching server; p50/p99 latency from submission to
    completion, and the throughput achieved."""
    import numpy as np

    out = []
    for rate in rates:
        reqs = workloads.serving_requests(count, rate, seed=5)
        bufs = []
        for r in reqs:
            d = up(np.arange(r["n"], dtype=np.uint64))
            o = up(np.zeros(r["m"], np.uint64)) if r["kind"] == "sample" else None
            bufs.append((d, o))
        torch_sync()
        srv = brr.Server(hbm_budget=8 << 30, max_inflight=max_inflight, nstreams=nstreams, seed=11)
        t0 = time.perf_counter()
        for i, (r, (d, o)) in enumerate(zip(reqs, bufs)):
            while time.perf_counter() - t0 < r["t"]:
                pass
            kind = brr.BRR_REQ_SAMPLE if r["kind"] == "sample" else brr.BRR_REQ_SHUFFLE
            srv.submit(kind, d, r["n"], 8, session=i % clients, m=r["m"], out=o)
        srv.drain()
        st = srv.stats()
        srv.close()
        out.append({"offered_req_per_s": rate, "requests": count, "clients": clients,
                    "p50_us": st["p50_us"], "p99_us": st["p99_us"], "mean_us": st["mean_us"],
                    "req_per_s": st["requests_per_s"], "elems_per_s": st["elements_per_s"],
                    "peak_inflight": st["peak_inflight"]})
        del bufs
    return out


def tuned_ragged(brr, workloads, up, steps):
    """The 20,000 ragged shuffles under the plan's default (shuffle_6), the
    exhaustive tuner's pick and the learned tuner's pick (model trained here
    on measured times of random batches; it times the default and its top 3
    of ~100 candidates), each re-timed as the median of 15 single runs with
    its spread; and the model's held-out evaluation on 8 fresh random
    batches (rank correlation, quality against exhaustive tuning, gain over
    the default beside the spread)."""
    import numpy as np

    from paper_2408_06213_amd import learned

    sizes = workloads.ragged_sizes(20000, seed=3)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes)
    d, d_off = up(data), up(off)
    s6 = brr.brr_schedule_paper(6)

    def retime(sched, wave_max):
        med, spread = learned.time_median(brr, off, d, d_off, sizes.size, 4, sched, wave_max, 15)
        return {"ms": med, "spread": spread}

    res = {"default": retime(s6, 512)}
    t0 = time.perf_counter()
    full = brr.Plan(off, 4)
    rep = full.autotune(d, d_off, 1, 0)
    res["exhaustive"] = {"timed": rep.candidates, "tune_s": time.perf_counter() - t0,
                         "schedule": rep.schedule.steps(), "wave_max": rep.mapping.wave_max,
                         **retime(rep.schedule, rep.mapping.wave_max)}
    full.close()
    rng = np.random.default_rng(11)
    t0 = time.perf_counter()
    X, y, _ = learned.collect(brr, up, rng, nbatch=16, ncand=40)
    net, loss = learned.train(brr, up, X, y, steps=4000, lr=3e-3, hidden=64)
    train_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = brr.Plan(off, 4)
    rep = brr.brr_plan_autotune_learned(plan, net, 3, d, d_off, 1, 0)
    res["learned"] = {"timed": rep.candidates, "tune_s": time.perf_counter() - t0,
                      "train_samples": int(X.shape[0]), "train_s": train_s, "train_mse": loss,
                      "target_variance": float(np.var(y)),
                      "schedule": rep.schedule.steps(), "wave_max": rep.mapping.wave_max,
                      **retime(rep.schedule, rep.mapping.wave_max)}
    plan.close()
    for k in ("exhaustive", "learned"):
        g = res["default"]["ms"] / res[k]["ms"]
        res[k]["gain_vs_default"] = g
        res[k]["gain_beyond_2x_spread"] = bool(
            g > 1 + 2 * max(res[k]["spread"], res["default"]["spread"]))
    rows = learned.evaluate(brr, up, net, rng, nbatch=8, reps=5)
    gain = np.array([r["gain_learned_vs_default"] for r in rows])
    spread = np.array([max(r["learned_spread"], r["default_spread"]) for r in rows])
    res["held_out"] = {
        "batches": len(rows),
        "mean_spearman": float(np.mean([r["spearman"] for r in rows])),
        "learned_vs_exhaustive_mean": float(np.mean([r["learned_vs_exhaustive"] for r in rows])),
        "learned_vs_exhaustive_min": float(np.min([r["learned_vs_exhaustive"] for r in rows])),
        "gain_vs_default": [float(x) for x in gain],
        "spread": [float(x) for x in spread],
        "gains_beyond_2x_spread": int(np.sum(gain > 1 + 2 * spread)),
        "timed_learned_vs_exhaustive": [rows[0]["learned_timed"], rows[0]["exhaustive_timed"]],
    }
    net.close()
    return res


def cpu_baseline(brr, workloads, up, bounds_np, head_out, k_head):
    """The oracle on every host core: the whole 2^28-roll headline stream
    (its groups split over the cores; also one thread alone), and the equal
    and ragged shuffle batches (shuffles split over the cores). Each oracle
    output is compared bit for bit with the GPU's output of the same
    workload (the headline stream as timed; one fresh shuffle_6 run of each
    batch)."""
    import numpy as np

    import oracle

    threads = oracle.host_threads()
    t0 = time.perf_counter()
    err, want = oracle.dice_stream(oracle.STREAM_MULTIPLY, bounds_np, k_head, 7, 0, threads=threads)
    dt = time.perf_counter() - t0
    assert err == 0
    exact = {"dice_stream_2p28": bool(np.array_equal(head_out, want))}
    del want
    t0 = time.perf_counter()
    err, _ = oracle.dice(bounds_np, k_head, 7, 0)
    dt1 = time.perf_counter() - t0
    assert err == 0
    base = {
        "value": COUNT / dt,
        "unit": "rolls/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"the whole 2^28-roll stream at k={k_head}, plain C oracle, its group range "
                  f"split over {threads} threads ({dt:.2f} s)",
        "host": host_cpu(),
        "one_thread": {"value": COUNT / dt1, "seconds": dt1},
        "secondary": {},
    }
    s6 = oracle.schedule_paper(6)
    batches = (("equal_65536x256_u32", np.full(65536, 256, dtype=np.uint64)),
               ("ragged_20000_u32", workloads.ragged_sizes(20000, seed=3)))
    for tag, sizes in batches:
        off = workloads.csr_offsets(sizes)
        data = workloads.iota_segments(sizes)
        d, d_off = up(data), up(off)
        plan = brr.Plan(off, 4)
        brr.check(brr.brr_shuffle_batched(d, d_off, sizes.size, 4, plan, 1, 0))
        got = d.cpu().numpy()
        plan.close()
        del d, d_off
        t0 = time.perf_counter()
        assert oracle.shuffle_batched_threads(data, off, s6, 1, 0, threads=threads) == 0
        dt = time.perf_counter() - t0
        exact[tag] = bool(np.array_equal(got, data))
        base["secondary"][tag] = {"elems_per_s": data.size / dt, "seconds": dt, "cores": threads,
                                  "sample": "the whole batch, shuffle_6, shuffles split over "
                                            f"{threads} threads"}
    return base, exact


def pmc_pass(brr, workloads, up):
    """For counter runs: a plain copy of 2^28 int32 (1 GiB read, 1 GiB written)
    and one 2^28-roll dice stream per k = 1..4, then the other forms and word
    streams once each."""
    import numpy as np
    import torch

    a = torch.arange(COUNT, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.bitwise_or(a, 0, out=b)
    torch.cuda.synchronize()
    del a, b
    bounds = up(workloads.dice_bounds(COUNT, seed=7))
    out = torch.empty(COUNT, dtype=torch.uint32, device="cuda")
    for k in (1, 2, 3, 4):
        brr.check(brr.brr_dice(bounds, out, COUNT, k, 7, 0))
    # the other forms and word streams once each, after the headline kernels
    for k in (1, 2, 3, 4):
        brr.check(brr.brr_dice_div(bounds, out, COUNT, k, 7, 0))
        brr.check(brr.brr_dice_chacha(bounds, out, COUNT, k, 7, 0))
    for k in (1, 2):
        brr.check(brr.brr_dice32(bounds, out, COUNT, k, 7, 0))
    torch.cuda.synchronize()
    print(json.dumps({"pmc_pass": "copy + dice k=1..4, then the division form, ChaCha20 words "
                                  "(k=1..4) and 32-bit words (k=1, 2)",
                      "source_hash": kernel_source_hash()}))


def ceilings(brr, torch):
    """Measured context for the roofline: a plain elementwise pass over the
    stream's bytes (1 GiB read + 1 GiB written, torch's own kernel), a bare
    copy of the same bytes in the fastest copy shape measured, and the
    rate at which the vector ALUs chain dice (Theorem 1 steps with no memory
    traffic and no word generation)."""
    a = torch.arange(COUNT, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    ms = time_launches(lambda: torch.bitwise_or(a, 0, out=b), 10, 2)
    copy_bps = brr.brr_probe_copy_rate(a, b, 4 * COUNT, 10)
    del a, b
    torch.cuda.empty_cache()
    return {"elementwise_GBps": BYTES_PER_ROLL * COUNT / (ms * 1e-3) / 1e9,
            "elementwise_kernel": "torch.bitwise_or over 2^28 int32 (1 GiB in, 1 GiB out)",
            "copy_probe_GBps": copy_bps / 1e9,
            "copy_probe_kernel": "brr_probe_copy_rate: 1 GiB copied, one 16-byte "
                                 "nontemporal vector per lane (the fastest copy shape "
                                 "measured), read + written bytes",
            "frac_of_copy_probe": None,
            "chain_dice_per_s": brr.brr_probe_chain_rate(4096)}


def torch_sync():
    import torch

    torch.cuda.synchronize()


def ragged_classes(brr, workloads, up, steps):
    """The 20,000 ragged shuffles split by the plan's size class (one lane
    per array up to 256 elements; one wavefront up to 512; workgroups of
    256, 256, 512 and 1,024 threads up to 2,048, 4,096, 8,192 and 16,384; one
    workgroup in peels beyond), each class timed alone as its own batch
    (shuffle_6, its own plan and graph): the time each class costs when
    nothing runs beside it, against the whole batch (where the classes
    overlap on forked streams)."""
    import numpy as np

    import torch

    sizes = workloads.ragged_sizes(20000, seed=3)
    bounds = [(2, 256, "lane"), (257, 512, "wavefront"), (513, 2048, "wg256x8"),
              (2049, 4096, "wg256x16"), (4097, 8192, "wg512x16"), (8193, 16384, "wg1024x16"),
              (16385, 1 << 20, "peel")]
    res = {}
    # the whole batch first, on memory torch takes fresh from the device
    torch.cuda.empty_cache()
    off = workloads.csr_offsets(sizes)
    d, d_off = up(workloads.iota_segments(sizes)), up(off)
    plan = brr.Plan(off, 4)
    whole_ms = time_launches(
        lambda: brr.check(brr.brr_shuffle_batched(d, d_off, sizes.size, 4, plan, 1, 0)),
        max(steps, 10), 3)
    plan.close()
    del d, d_off
    for lo, hi, name in bounds:
        sub = sizes[(sizes >= lo) & (sizes <= hi)]
        if sub.size == 0:
            continue
        off = workloads.csr_offsets(sub)
        d, d_off = up(workloads.iota_segments(sub)), up(off)
        plan = brr.Plan(off, 4)
        ms = time_launches(lambda: brr.check(brr.brr_shuffle_batched(d, d_off, sub.size, 4, plan, 1, 0)),
                           max(steps, 10), 3)
        plan.close()
        res[name] = {"arrays": int(sub.size), "elements": int(sub.sum()), "ms": ms,
                     "elems_per_s": float(sub.sum()) / (ms * 1e-3),
                     "hbm_frac": 8 * float(sub.sum()) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
        del d, d_off
    res["whole_batch_ms"] = whole_ms
    res["sum_of_classes_ms"] = sum(v["ms"] for v in res.values() if isinstance(v, dict))
    return res


def sample_sweep(brr, up, steps):
    """Samples without replacement far smaller than their array: time and
    device scratch against m, beside the full shuffle of the same array
    (n = 2^22 u64, the serving workload's largest, and n = 2^26 u32)."""
    import numpy as np
    import torch

    s6 = brr.brr_schedule_paper(6)
    res = {}
    for n, dt, ms in ((1 << 22, np.uint64, (4194, 41943, 419430)), (1 << 26, np.uint32, (6710886,))):
        eb = np.dtype(dt).itemsize
        d = up(np.arange(n, dtype=dt))
        rows = {}
        for m in ms:
            o = torch.empty(m * eb, dtype=torch.uint8, device="cuda")
            f = lambda: brr.check(brr.brr_sample(d, n, m, eb, o, s6, 5, 0))
            t = time_launches(f, max(5, steps), 2)
            # host time of one call (argument checks, scratch, launches)
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            f()
            host_ms = (time.perf_counter() - h0) * 1e3
            torch.cuda.synchronize()
            rows[str(m)] = {"ms": t, "sampled_per_s": m / (t * 1e-3), "host_ms_per_call": host_ms,
                            "scratch_bytes": brr.brr_scratch_bytes(n, m, eb)}
            del o
        t = time_launches(lambda: brr.check(brr.brr_shuffle(d, n, eb, s6, 5, 0)), max(3, steps // 2), 1)
        res[f"n_{n}_{np.dtype(dt).name}"] = {
            "samples": rows,
            "full_shuffle": {"ms": t, "scratch_bytes": brr.brr_scratch_bytes(n, 0, eb)}}
        del d
        torch.cuda.empty_cache()
    return res


def fresh_calls(brr, d, d_off, off, count, steps):
    """Calls per second of one plan, every call with a new instance base (a
    caller streaming batches), with the graph (captured once, arguments
    bound per call) and with direct launches; the captures made."""
    import torch

    res = {}
    for name, use_graph in (("graph", 1), ("direct", 0)):
        plan = brr.Plan(off, 4)
        m = plan.mapping()
        m.use_graph = use_graph
        brr.check(plan.set_mapping(m), "set_mapping")
        inst = [0]

        def f():
            inst[0] += count
            brr.check(brr.brr_shuffle_batched(d, d_off, count, 4, plan, 1, inst[0]))

        ms = time_launches(f, max(steps, 20), 2)
        res[name] = {"ms_per_call": ms, "calls_per_s": 1e3 / ms, "captures": plan.captures()}
        plan.close()
        torch.cuda.synchronize()
    res["graph_speedup"] = res["direct"]["ms_per_call"] / res["graph"]["ms_per_call"]
    return res


def secondary(brr, workloads, up, steps, only=None):
    import numpy as np

    out = {}
    s6 = brr.brr_schedule_paper(6)
    s1 = brr.brr_schedule_paper(1)
    # the paper's comparisons: unbatched (k1) and two dice by division (naive2);
    # shuffle_6 and k1 again on ChaCha20 words (its slow generator); the
    # L = 32 cost-model schedule on 32-bit words
    cc6 = brr.brr_schedule.from_steps(s6.steps(), tail=True, u_tail=720,
                                      words=brr.BRR_WORDS_CHACHA20)
    cc1 = brr.brr_schedule.from_steps(s1.steps(), tail=bool(s1.tail), u_tail=s1.u_tail,
                                      words=brr.BRR_WORDS_CHACHA20)
    l32 = brr.brr_schedule_from_costs(6, l32=True)
    scheds = (("k6", s6), ("k1", s1), ("naive2", brr.brr_schedule_naive2()),
              ("k6_chacha20", cc6), ("k1_chacha20", cc1), ("costs_l32", l32))

    def batched(sizes, tag):
        off = workloads.csr_offsets(sizes)
        data = workloads.iota_segments(sizes)
        # enough copies of the batch, used in turn, that a step never finds
        # its data in the 256 MB last-level cache
        sets = min(8, max(1, -(-(512 << 20) // data.nbytes)))
        ds, d_off = [up(data) for _ in range(sets)], up(off)
        res = {"buffer_sets": sets}
        variants = list(scheds)
        if tag.startswith("ragged"):  # the same plan launched without its hip graph
            variants.append(("k6_no_graph", s6))
        for name, sched in variants:
            plans = [brr.Plan(off, 4, sched) for _ in range(sets)]
            if name.endswith("no_graph"):
                for plan in plans:
                    m = plan.mapping()
                    m.use_graph = 0
                    brr.check(plan.set_mapping(m), "set_mapping")
            turn = [0]

            def f():
                i = turn[0] % sets
                turn[0] += 1
                brr.check(brr.brr_shuffle_batched(ds[i], d_off, sizes.size, 4, plans[i], 1, 0))

            ms = time_launches(f, max(steps, sets), max(2, sets))
            res[name] = {"ms": ms, "elems_per_s": data.size / (ms * 1e-3)}
            for plan in plans:
                plan.close()
        res["speedup_k6_vs_k1"] = res["k1"]["ms"] / res["k6"]["ms"]
        res["speedup_k6_vs_naive2"] = res["naive2"]["ms"] / res["k6"]["ms"]
        res["chacha20_speedup_k6_vs_k1"] = res["k1_chacha20"]["ms"] / res["k6_chacha20"]["ms"]
        if "k6_no_graph" in res:
            res["graph_speedup_k6"] = res["k6_no_graph"]["ms"] / res["k6"]["ms"]
        if tag.startswith("ragged"):
            res["calls_fresh_instance"] = fresh_calls(brr, ds[0], d_off, off, sizes.size, steps)
        res["hbm_frac_k6"] = 2 * 4 * data.size / (res["k6"]["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS
        out[tag] = res

    # samples first: after the other workloads' allocations, the 2^26 sample's
    # random gathers from its array have run up to 8x slower in the same
    # process (its kernels alone, not the host side), cause not found
    if only in (None, "sample"):
        out["sample_sparse"] = sample_sweep(brr, up, steps)
    if only in (None, "equal"):
        batched(np.full(65536, 256, dtype=np.uint64), "equal_65536x256_u32")
    if only in (None, "ragged"):
        batched(workloads.ragged_sizes(20000, seed=3), "ragged_20000_u32")

    singles = ((10000, "single_10000_u32", "single10000"), (1 << 26, "single_2p26_u32", "single2p26"))
    for n, tag, key in singles:
        if only not in (None, key):
            continue
        a = up(np.arange(n, dtype=np.uint32))
        res = {}
        for name, sched in scheds:
            f = lambda: brr.check(brr.brr_shuffle(a, n, 4, sched, 42, 0))
            ms = time_launches(f, max(3, steps // 2), 1)
            res[name] = {"ms": ms, "elems_per_s": n / (ms * 1e-3)}
        res["speedup_k6_vs_k1"] = res["k1"]["ms"] / res["k6"]["ms"]
        res["speedup_k6_vs_naive2"] = res["naive2"]["ms"] / res["k6"]["ms"]
        res["chacha20_speedup_k6_vs_k1"] = res["k1_chacha20"]["ms"] / res["k6_chacha20"]["ms"]
        out[tag] = res
    if only in (None, "ragged_classes"):
        out["ragged_20000_u32_classes"] = ragged_classes(brr, workloads, up, steps)
    if only in (None, "tuned"):
        out["ragged_20000_u32_tuned"] = tuned_ragged(brr, workloads, up, steps)
    if only in (None, "serving"):
        out["serving_u64"] = serving(brr, workloads, up)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", default="best",
                    help="dice per word of the headline stream: 1..4, or 'best' (fastest of 2..4)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--only", choices=["equal", "ragged", "single10000", "single2p26", "serving",
                                       "tuned", "sample", "ragged_classes", "pmc"],
                    help="run one shuffle workload only (for profiling); prints its timings")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the batched dice and shuffle kernels have no multi-GPU path in this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2408_06213_amd import brr, workloads

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    if args.only == "pmc":
        pmc_pass(brr, workloads, up)
        return
    if args.only:
        # a plain copy of known size first: counter runs scale each kernel's
        # FETCH_SIZE / WRITE_SIZE by what the counters read for it
        a = torch.arange(COUNT, dtype=torch.int32, device=dev)
        torch.bitwise_or(a, 0, out=torch.empty_like(a))
        torch.cuda.synchronize()
        del a
        torch.cuda.empty_cache()
        print(json.dumps(secondary(brr, workloads, up, args.steps, args.only)), flush=True)
        return

    bounds_np = workloads.dice_bounds(COUNT, seed=7)
    bounds = up(bounds_np)
    out = torch.empty(COUNT, dtype=torch.uint32, device=dev)

    def step(k):
        return lambda: brr.check(brr.brr_dice(bounds, out, COUNT, k, 7, 0), "brr_dice")

    # steady state before any timing: without it the first kernel timed runs
    # while clocks and the memory system are still ramping (k = 1 read about
    # 20% slow when it was timed first)
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        for _ in range(10):
            step(2)()
        torch.cuda.synchronize()

    ms_k = {k: time_launches(step(k), args.steps, args.warmup) for k in (1, 2, 3, 4)}
    # the same stream on 32-bit words (two dice per word fit: every bound
    # is below 2^16); and a stream of bounds below 2^12, under the L = 32
    # threshold n_2 = 20724 of Table 2, at both widths
    ms_32 = {k: time_launches(lambda k=k: brr.check(brr.brr_dice32(bounds, out, COUNT, k, 7, 0),
                                                    "brr_dice32"), args.steps, args.warmup)
             for k in (1, 2)}
    # the division form of Sec. 2.1 on the same stream (same words, dice by
    # successive remainders)
    ms_div = {k: time_launches(lambda k=k: brr.check(brr.brr_dice_div(bounds, out, COUNT, k, 7, 0),
                                                     "brr_dice_div"), args.steps, args.warmup)
              for k in (1, 2, 3, 4)}
    # known bounds (Algorithm 2: one bound, threshold computed once): the
    # stream only writes, 4 B per roll, so its roofline is the write roofline
    ms_const = {k: time_launches(lambda k=k: brr.check(brr.brr_dice_const(KNOWN_BOUND, out, COUNT, k,
                                                                          7, 0),
                                                       "brr_dice_const"), args.steps, args.warmup)
                for k in (1, 2, 3, 4)}
    # ChaCha20 words (the paper's slow generator): batching saves words
    ms_cc = {k: time_launches(lambda k=k: brr.check(brr.brr_dice_chacha(bounds, out, COUNT, k, 7, 0),
                                                    "brr_dice_chacha"), args.steps, args.warmup)
             for k in (1, 2, 3, 4)}
    small = up(workloads.dice_bounds(COUNT, seed=8, high=1 << 12))
    ms_small = {f"L{L}_k{k}": time_launches(
        lambda L=L, k=k: brr.check((brr.brr_dice32 if L == 32 else brr.brr_dice)(
            small, out, COUNT, k, 8, 0), "dice"), args.steps, args.warmup)
        for L, k in ((64, 1), (64, 2), (32, 1), (32, 2))}
    # ChaCha20 words on these bounds: k = 4 rarely rerolls here
    ms_small.update({f"chacha20_k{k}": time_launches(
        lambda k=k: brr.check(brr.brr_dice_chacha(small, out, COUNT, k, 8, 0), "brr_dice_chacha"),
        args.steps, args.warmup) for k in (1, 2, 3, 4)})
    del small
    brr.check(brr.brr_sync_status(), "device status")
    k_head = min((2, 3, 4), key=lambda k: ms_k[k]) if args.k == "best" else int(args.k)
    ms = ms_k[k_head]
    head_stats = launch_stats(step(k_head))
    # the headline stream as the timed launches wrote it, for the bit-exact
    # comparison with the oracle
    step(k_head)()
    head_out = out.cpu().numpy()
    value = COUNT / (ms * 1e-3)
    achieved = BYTES_PER_ROLL * COUNT / (ms * 1e-3) / 1e9
    traffic = measured_traffic(k_head)

    rec = {
        "metric": "dice rolls/s and shuffled elems/s, batched vs k=1 on GPU, bit-exact; % roofline",
        "value": value,
        "unit": "rolls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"flat dice stream: 2^28 u32 bounds uniform in [1,2^16) (seed 7), "
                        f"k={k_head} dice per 64-bit Philox4x32-10 word"
                        + (" (fastest of k=2..4)" if args.k == "best" else ""),
            "count": COUNT,
            "k": k_head,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
        },
        "k_sweep": {str(k): {"ms": v, "rolls_per_s": COUNT / (v * 1e-3),
                             "hbm_frac": BYTES_PER_ROLL * COUNT / (v * 1e-3) / 1e9 / PEAK_HBM_GBS}
                    for k, v in ms_k.items()},
        "speedup_vs_k1": ms_k[1] / ms,
        # per-launch spread of the headline kernel, and the share of the HBM
        # peak its written bytes alone take (1 GiB of dice per launch; it
        # reads as much again, which the roofline above counts)
        "headline_launch_stats": head_stats,
        "headline_written_bytes_frac": (COUNT * 4) / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "l32_sweep": {str(k): {"ms": v, "rolls_per_s": COUNT / (v * 1e-3),
                               "hbm_frac": BYTES_PER_ROLL * COUNT / (v * 1e-3) / 1e9 / PEAK_HBM_GBS}
                      for k, v in ms_32.items()},
        "bounds_below_2p12": {key: {"ms": v, "rolls_per_s": COUNT / (v * 1e-3)}
                              for key, v in ms_small.items()},
        "chacha20_sweep": {str(k): {"ms": v, "rolls_per_s": COUNT / (v * 1e-3),
                                    "speedup_vs_k1": ms_cc[1] / v,
                                    "hbm_frac": BYTES_PER_ROLL * COUNT / (v * 1e-3) / 1e9 / PEAK_HBM_GBS}
                           for k, v in ms_cc.items()},
        "division_form_sweep": {str(k): {"ms": v, "rolls_per_s": COUNT / (v * 1e-3),
                                         "multiply_form_speedup": v / ms_k[k]}
                                for k, v in ms_div.items()},
        "known_bounds_sweep": {
            "bound": KNOWN_BOUND,
            **{str(k): {"ms": v, "rolls_per_s": COUNT / (v * 1e-3),
                        "write_GBps": 4 * COUNT / (v * 1e-3) / 1e9,
                        "hbm_write_frac": 4 * COUNT / (v * 1e-3) / 1e9 / PEAK_HBM_GBS}
               for k, v in ms_const.items()},
            "speedup_best_vs_k1": ms_const[1] / min(ms_const[k] for k in (2, 3, 4)),
            "best_k": min((2, 3, 4), key=lambda k: ms_const[k]),
            "best_hbm_write_frac": 4 * COUNT / (min(ms_const[k] for k in (2, 3, 4)) * 1e-3) / 1e9
                                   / PEAK_HBM_GBS,
        },
        "ceilings": ceilings(brr, torch),
    }
    rec["ceilings"]["frac_of_copy_probe"] = achieved / rec["ceilings"]["copy_probe_GBps"]
    del out, bounds
    torch.cuda.empty_cache()

    if not args.no_secondary:
        rec["secondary"] = secondary(brr, workloads, up, max(5, args.steps // 2))
        rec["secondary"]["paper_cpu_speedups"] = PAPER_CPU_SPEEDUPS

    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["bit_exact"] = cpu_baseline(brr, workloads, up, bounds_np, head_out,
                                                             k_head)
        if not all(rec["bit_exact"].values()):
            print(json.dumps(rec), flush=True)
            sys.exit("bench: a GPU output differs from the oracle: " + json.dumps(rec["bit_exact"]))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
