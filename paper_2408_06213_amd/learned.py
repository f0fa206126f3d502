"""Training data and training for the learned plan-cost model.

A sample is (features of a batch under a schedule and wavefront-tier limit,
log of the measured milliseconds of one batched shuffle). Features come from
brr_plan_features, times from HIP events around brr_shuffle_batched on a
device copy, training from brr_mlp_train: every step runs in libbrr.
"""
from __future__ import annotations

import math

import numpy as np


def candidate_configs(brr):
    """(schedule, wave_max) pairs: the paper's schedules and cost-model ones
    (kmax 3..8, several generator/division cost ratios) under wavefront-tier
    limits 64..512 -- the same family the autotuner searches."""
    scheds = [brr.brr_schedule_paper(k) for k in (6, 2, 1)]
    for kmax in range(3, 9):
        for c_rng, c_div in ((2, 16), (1, 16), (4, 16), (8, 16), (2, 64)):
            s = brr.brr_schedule_from_costs(kmax, c_rng, c_div, pow2=True, smooth=True)
            if all(s.steps() != o.steps() for o in scheds):
                scheds.append(s)
    return [(s, w) for s in scheds for w in (64, 128, 256, 512)]


def random_batch(rng, max_total=1 << 22):
    lo = rng.uniform(3, 13)
    hi = rng.uniform(lo + 1, 20)
    mean_n = 2 ** ((lo + hi) / 2)
    count = int(np.clip(max_total / mean_n * rng.uniform(0.2, 1.0), 4, 60000))
    return np.floor(2 ** rng.uniform(lo, hi, size=count)).astype(np.uint64)


def time_config(brr, off, work, d_off, count, eb, sched, wave_max, reps=2):
    import torch

    plan = brr.Plan(off, eb, sched)
    m = plan.mapping()
    m.wave_max = wave_max
    m.use_graph = 0
    brr.check(plan.set_mapping(m))
    run = lambda: brr.check(brr.brr_shuffle_batched(work, d_off, count, eb, plan, 1, 0))
    run()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    torch.cuda.synchronize()
    plan.close()
    return e0.elapsed_time(e1) / reps


def collect(brr, up, rng, nbatch, ncand=None, eb=4):
    """Features and log-times of random batches under random candidates
    (all candidates when ncand is None). Returns X, y, groups (batch ids)."""
    from . import workloads

    cands = candidate_configs(brr)
    X, y, groups = [], [], []
    for b in range(nbatch):
        sizes = random_batch(rng)
        off = workloads.csr_offsets(sizes)
        dtype = np.uint32 if eb == 4 else np.uint64
        work = up(workloads.iota_segments(sizes, dtype))
        d_off = up(off)
        pick = range(len(cands)) if ncand is None else rng.choice(len(cands), ncand, replace=False)
        for c in pick:
            sched, wm = cands[c]
            ms = time_config(brr, off, work, d_off, sizes.size, eb, sched, wm)
            X.append(brr.brr_plan_features(off, eb, sched, wm))
            y.append(math.log(ms))
            groups.append(b)
        del work
    return np.array(X, np.float32), np.array(y, np.float32), np.array(groups)


def train(brr, up, X, y, steps=3000, lr=3e-3, hidden=64, seed=0):
    net = brr.MLP(X.shape[1], hidden, seed)
    loss = net.train(up(X), up(y), X.shape[0], steps, lr)
    return net, loss


def predict(brr, up, net, X):
    import torch

    d_y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    net.forward(up(X), X.shape[0], d_y)
    torch.cuda.synchronize()
    return d_y.cpu().numpy()
