"""Serving with continuous batching: every request's result equals the
oracle's for its (session, place in session) instance, whatever mix,
interleaving, stream count or budget it ran under, and equals what the same
request gives alone."""
import numpy as np
import pytest

from conftest import say, to_dev, to_host

pytestmark = pytest.mark.gpu

SESSION_SHIFT = 40


def make_requests(seed, count):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(2 ** rng.uniform(1, 18))
        kind = "sample" if rng.random() < 0.5 else "shuffle"
        m = int(rng.integers(1, max(1, n // 10) + 1)) if kind == "sample" else n
        dtype = np.uint64 if rng.random() < 0.7 else np.uint32
        data = rng.integers(0, 2**31, size=n).astype(dtype)
        reqs.append(dict(kind=kind, n=n, m=m, data=data, session=int(rng.integers(0, 5))))
    # requests that run no shuffle kernel still take their instance, and one
    # large enough for the sorting path of the device-wide tier
    big = (1 << 21) + 7
    reqs[3] = dict(kind="shuffle", n=1, m=1, data=np.array([5], np.uint64), session=reqs[3]["session"])
    reqs[7] = dict(kind="sample", n=1, m=1, data=np.array([9], np.uint32), session=reqs[7]["session"])
    reqs[11] = dict(kind="shuffle", n=big, m=big, data=rng.integers(0, 2**31, size=big).astype(np.uint32),
                    session=reqs[11]["session"])
    return reqs


def run_mix(gpu, reqs, order, **cfg):
    srv = gpu.Server(**cfg)
    bufs = {}
    ids = {}
    for i in order:
        r = reqs[i]
        d = to_dev(r["data"])
        out = to_dev(np.zeros(r["m"], r["data"].dtype)) if r["kind"] == "sample" else None
        bufs[i] = (d, out)
        kind = gpu.BRR_REQ_SAMPLE if r["kind"] == "sample" else gpu.BRR_REQ_SHUFFLE
        ids[i] = srv.submit(kind, d, r["n"], r["data"].itemsize, r["session"], r["m"], out)
    for i in order:
        srv.wait(ids[i])
    counters = {s: srv.counter(s) for s in {r["session"] for r in reqs}}
    stats = srv.stats()
    srv.close()
    results = {i: to_host(out if out is not None else d) for i, (d, out) in bufs.items()}
    return results, counters, stats


def expected(orc, reqs, order, seed, sched=None):
    """Oracle result of each request at instance session * 2^40 + j, where j
    counts the earlier submissions of its session."""
    s6 = sched if sched is not None else orc.schedule_paper(6)
    seen = {}
    want = {}
    for i in order:
        r = reqs[i]
        j = seen.get(r["session"], 0)
        seen[r["session"]] = j + 1
        inst = (r["session"] << SESSION_SHIFT) + j
        if r["kind"] == "sample" and r["n"] == 1:
            err, out = 0, r["data"].copy()
        elif r["kind"] == "sample":
            err, out = orc.sample(r["data"], r["m"], s6, seed, inst)
        else:
            out = r["data"].copy()
            err = orc.shuffle(out, s6, seed, inst)
        assert err == 0
        want[i] = out
    return want, seen


def test_server_results_match_oracle_in_any_mix(gpu, orc):
    reqs = make_requests(1, 60)
    # same order within each session, different interleaving across sessions
    order_a = list(range(len(reqs)))
    by_session = {}
    for i in order_a:
        by_session.setdefault(reqs[i]["session"], []).append(i)
    order_b = []
    for s in sorted(by_session, reverse=True):
        order_b += by_session[s]
    want, seen = expected(orc, reqs, order_a, seed=99)
    say("server mix A")
    got_a, counters_a, stats_a = run_mix(gpu, reqs, order_a, seed=99, nstreams=8, max_inflight=32)
    say("server mix B")
    got_b, counters_b, _ = run_mix(gpu, reqs, order_b, seed=99, nstreams=3, max_inflight=4,
                                   hbm_budget=1 << 20)
    for i in range(len(reqs)):
        assert np.array_equal(got_a[i], want[i]), i
        assert np.array_equal(got_b[i], want[i]), i
    assert counters_a == seen == counters_b
    assert stats_a["completed"] == len(reqs) and stats_a["p99_us"] >= stats_a["p50_us"] > 0


def test_server_request_alone_equals_in_mix(gpu, orc):
    """Every request of a mix, run alone in a fresh server at the same
    (session, j) (its j earlier requests of the session replaced by
    one-element shuffles, which take an instance and move nothing), gives
    bit for bit the result it gave in the mix; both equal the oracle's."""
    reqs = make_requests(3, 40)
    order = list(range(len(reqs)))
    say("server mix for alone-vs-mix")
    mixed, _, stats = run_mix(gpu, reqs, order, seed=17, nstreams=4, max_inflight=32)
    assert stats["peak_inflight"] > 1  # the mix did overlap
    want, _ = expected(orc, reqs, order, seed=17)
    seen = {}
    for i in order:
        r = reqs[i]
        j = seen.get(r["session"], 0)
        seen[r["session"]] = j + 1
        say("server alone", i, r["kind"], r["n"], "session", r["session"], "j", j)
        srv = gpu.Server(seed=17, nstreams=2, max_inflight=4)
        pads = [to_dev(np.zeros(1, np.uint32)) for _ in range(j)]
        for pad in pads:
            srv.submit(gpu.BRR_REQ_SHUFFLE, pad, 1, 4, r["session"])
        d = to_dev(r["data"])
        out = to_dev(np.zeros(r["m"], r["data"].dtype)) if r["kind"] == "sample" else None
        kind = gpu.BRR_REQ_SAMPLE if r["kind"] == "sample" else gpu.BRR_REQ_SHUFFLE
        srv.wait(srv.submit(kind, d, r["n"], r["data"].itemsize, r["session"], r["m"], out))
        srv.drain()
        assert srv.counter(r["session"]) == j + 1
        srv.close()
        alone = to_host(out if out is not None else d)
        assert np.array_equal(alone, mixed[i]), i
        assert np.array_equal(alone, want[i]), i


def test_server_budget_limits_footprint(gpu):
    say("server budget")
    srv = gpu.Server(hbm_budget=64 << 20, max_inflight=16, nstreams=4, seed=3)
    bufs = []
    ids = []
    for s in range(12):
        d = to_dev(np.arange(1 << 20, dtype=np.uint32))  # needs ~28 MB of scratch each
        bufs.append(d)
        ids.append(srv.submit(gpu.BRR_REQ_SHUFFLE, d, 1 << 20, 4, session=s))
    srv.drain()
    st = srv.stats()
    srv.close()
    assert st["completed"] == 12
    assert 0 < st["peak_footprint"] <= 64 << 20
    for d in bufs:  # each is a permutation
        assert np.array_equal(np.sort(to_host(d)), np.arange(1 << 20, dtype=np.uint32))


@pytest.mark.parametrize("words", ["chacha", "l32"])
def test_server_other_word_streams(gpu, orc, words):
    """A server whose schedule reads ChaCha20 words (shuffle_6) or 32-bit
    words (Table 2's L = 32 schedule) serves what the oracle computes with
    that schedule."""
    if words == "chacha":
        steps = gpu.brr_schedule_paper(6).steps()
        gs = gpu.brr_schedule.from_steps(steps, tail=True, u_tail=720,
                                         words=gpu.BRR_WORDS_CHACHA20)
        os_ = orc.Schedule.from_segments(steps, tail=True, u_tail=720, words=orc.WORDS_CHACHA20)
    else:
        gs = gpu.brr_schedule_from_costs(4, pow2=False, smooth=False, l32=True)
        os_ = orc.Schedule.from_segments(gs.steps(), tail=bool(gs.tail), u_tail=gs.u_tail,
                                         words=orc.WORDS_PHILOX32)
    reqs = make_requests(2, 30)
    order = list(range(len(reqs)))
    want, seen = expected(orc, reqs, order, seed=5, sched=os_)
    say("server", words)
    got, counters, _ = run_mix(gpu, reqs, order, seed=5, nstreams=4, max_inflight=8, sched=gs)
    for i in order:
        assert np.array_equal(got[i], want[i]), (words, i)
    assert counters == seen
