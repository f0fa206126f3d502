"""Training data, training and held-out evaluation of the learned plan-cost
model.

A sample is (features of a batch under a schedule and wavefront-tier limit,
log of the measured milliseconds of one batched shuffle less the batch's
mean over its candidates). Features come from
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


def collect(brr, up, rng, nbatch, ncand=None, eb=4, reps=5):
    """Features and targets of random batches under random candidates (all
    candidates when ncand is None). A target is the log of the candidate's
    time (median of `reps` single runs) less the mean log time of the
    batch's candidates: the tuner only ranks the candidates of one batch, so
    the model learns how a configuration's time differs from the batch's
    typical one rather than the batch size's far larger effect. Returns X,
    y, groups (batch ids)."""
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
        logs = []
        for c in pick:
            sched, wm = cands[c]
            ms = time_median(brr, off, work, d_off, sizes.size, eb, sched, wm, reps)[0]
            X.append(brr.brr_plan_features(off, eb, sched, wm))
            logs.append(math.log(ms))
            groups.append(b)
        mean = sum(logs) / len(logs)
        y.extend(v - mean for v in logs)
        del work
    return np.array(X, np.float32), np.array(y, np.float32), np.array(groups)


def time_median(brr, off, work, d_off, count, eb, sched, wave_max, reps):
    """Median and the (max - min) / median spread of `reps` single timed
    runs of one configuration (one untimed run first)."""
    import torch

    plan = brr.Plan(off, eb, sched)
    m = plan.mapping()
    m.wave_max = wave_max
    m.use_graph = 0
    brr.check(plan.set_mapping(m))
    run = lambda: brr.check(brr.brr_shuffle_batched(work, d_off, count, eb, plan, 1, 0))
    run()
    s = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(s)
        run()
        b.record(s)
    torch.cuda.synchronize()
    plan.close()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    med = float(np.median(t))
    return med, float((t.max() - t.min()) / med)


def evaluate(brr, up, net, rng, nbatch=8, reps=7, top=3, eb=4):
    """Held-out evaluation of the trained model on nbatch fresh random
    batches. For each: every candidate configuration timed (median of `reps`
    single runs); the model's Spearman rank correlation between predicted
    and measured times over the candidates; the learned tuner's pick
    (brr_plan_autotune_learned, which times the default and the model's
    `top` candidates) and the exhaustive tuner's pick (brr_plan_autotune,
    about 30 candidates), both re-timed with `reps` runs beside the
    shuffle_6 default, with their spreads. Returns a list of per-batch
    records."""
    from scipy.stats import spearmanr

    from . import workloads

    cands = candidate_configs(brr)
    rows = []
    dtype = np.uint32 if eb == 4 else np.uint64
    for b in range(nbatch):
        sizes = random_batch(rng)
        off = workloads.csr_offsets(sizes)
        work = up(workloads.iota_segments(sizes, dtype))
        d_off = up(off)
        meas = [time_median(brr, off, work, d_off, sizes.size, eb, sc, wm, reps)[0]
                for sc, wm in cands]
        feats = np.array([brr.brr_plan_features(off, eb, sc, wm) for sc, wm in cands], np.float32)
        pred = predict(brr, up, net, feats)
        rho = float(spearmanr(pred, meas).correlation)
        s6 = brr.brr_schedule_paper(6)
        default = time_median(brr, off, work, d_off, sizes.size, eb, s6, 512, reps)
        plan = brr.Plan(off, eb)
        rep = brr.brr_plan_autotune_learned(plan, net, top, work, d_off, 1, 0)
        learned = time_median(brr, off, work, d_off, sizes.size, eb, rep.schedule,
                              rep.mapping.wave_max, reps)
        plan.close()
        plan = brr.Plan(off, eb)
        rep_x = plan.autotune(work, d_off, 1, 0)
        exhaustive = time_median(brr, off, work, d_off, sizes.size, eb, rep_x.schedule,
                                 rep_x.mapping.wave_max, reps)
        plan.close()
        rows.append({"count": int(sizes.size), "elements": int(off[-1]),
                     "spearman": rho, "best_measured_ms": float(min(meas)),
                     "default_ms": default[0], "default_spread": default[1],
                     "learned_ms": learned[0], "learned_spread": learned[1],
                     "learned_timed": int(rep.candidates),
                     "exhaustive_ms": exhaustive[0], "exhaustive_spread": exhaustive[1],
                     "exhaustive_timed": int(rep_x.candidates),
                     "gain_learned_vs_default": default[0] / learned[0],
                     "learned_vs_exhaustive": exhaustive[0] / learned[0]})
        del work
    return rows


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
