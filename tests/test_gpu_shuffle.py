"""GPU parity of shuffles, batched shuffles and samples with the CPU oracle:
bit-exact permutations, through the C ABI."""
import numpy as np
import pytest

from conftest import say, to_dev, to_host
from paper_2408_06213_amd import workloads

pytestmark = pytest.mark.gpu

LDS_SIZES = [2, 3, 4, 5, 6, 7, 8, 13, 64, 100, 255, 256, 257, 511, 512, 513, 1000, 4096, 10000,
             16383, 16384]
# device-wide tier: counting up to 2^21 positions, radix sort above
GLOBAL_SIZES = [16385, 20000, 65536, 100003, 1 << 20, 1 << 21, (1 << 21) + 5]


def both_schedules(gpu, orc, max_k):
    return gpu.brr_schedule_paper(max_k), orc.schedule_paper(max_k)


def gpu_shuffle(gpu, data_np, sched, seed, inst):
    d = to_dev(data_np)
    gpu.check(gpu.brr_shuffle(d, data_np.size, data_np.itemsize, sched, seed, inst), "brr_shuffle")
    assert gpu.brr_sync_status() == 0
    return to_host(d)


@pytest.mark.parametrize("max_k", [6, 2, 1])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("tier", ["lds", "global"])
def test_shuffle_parity(gpu, orc, max_k, dtype, tier):
    gs, os_ = both_schedules(gpu, orc, max_k)
    sizes = LDS_SIZES if tier == "lds" else GLOBAL_SIZES
    for n in sizes:
        say("shuffle", tier, max_k, np.dtype(dtype).name, n)
        a = np.arange(n, dtype=dtype) * 3 + 1
        got = gpu_shuffle(gpu, a, gs, seed=1234, inst=n)
        want = a.copy()
        assert orc.shuffle(want, os_, 1234, n) == 0
        assert np.array_equal(got, want), (tier, max_k, n)


def test_shuffle_config_10000(gpu, orc):
    """A[i] = i, n = 10,000, seed 42: shuffle_6 and the unbatched form."""
    for max_k in (6, 1):
        gs, os_ = both_schedules(gpu, orc, max_k)
        say("shuffle n=10000 seed 42", max_k)
        a = np.arange(10000, dtype=np.uint32)
        got = gpu_shuffle(gpu, a, gs, seed=42, inst=0)
        want = a.copy()
        assert orc.shuffle(want, os_, 42, 0) == 0
        assert np.array_equal(got, want)


def test_shuffle_custom_schedules(gpu, orc):
    """Schedules other than the paper's: larger batches at small sizes (up to
    8 dice below 146 elements, 7-dice last batch) and exact-product guards."""
    steps = [(2**19, 2, 2**60), (26573, 3, 0), (3225, 4, 0), (815, 5, 0), (305, 6, 0), (146, 7, 0),
             (8, 8, 0)]
    gs = gpu.brr_schedule.from_steps(steps, tail=True, u_tail=0)
    os_ = orc.Schedule.from_segments(steps, tail=True, u_tail=0)
    for n in (9, 100, 147, 1000, 16384, 50000):
        say("shuffle custom", n)
        a = np.arange(n, dtype=np.uint32)
        got = gpu_shuffle(gpu, a, gs, seed=77, inst=1)
        want = a.copy()
        assert orc.shuffle(want, os_, 77, 1) == 0
        assert np.array_equal(got, want), n


def test_shuffle_trivial_sizes(gpu):
    import torch

    d = torch.arange(1, dtype=torch.int32, device="cuda")
    assert gpu.brr_shuffle(d, 1, 4, None, 1, 0) == 0
    assert gpu.brr_shuffle(d, 0, 4, None, 1, 0) == 0
    assert int(d[0]) == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_sample_parity(gpu, orc, dtype):
    s6g, s6o = both_schedules(gpu, orc, 6)
    rng = np.random.default_rng(9)
    cases = [(2, 1), (2, 2), (5, 5), (5, 4), (10, 3), (256, 25), (1000, 1), (10000, 1000),
             (16384, 16384), (16384, 1638), (16385, 1638), (100003, 10000), (1 << 20, 104857),
             (1 << 20, 1), (70000, 69999), (70000, 70000), (3000000, 300000),
             ((1 << 21) + 1, 1)]
    for n, m in cases:
        say("sample", np.dtype(dtype).name, n, m)
        data = rng.integers(0, 2**31, size=n).astype(dtype)
        d = to_dev(data)
        out = to_dev(np.zeros(m, dtype))
        gpu.check(gpu.brr_sample(d, n, m, data.itemsize, out, s6g, 31, n), "brr_sample")
        assert gpu.brr_sync_status() == 0
        err, want = orc.sample(data, m, s6o, 31, n)
        assert err == 0
        assert np.array_equal(to_host(out), want), (n, m)
        assert np.array_equal(to_host(d), data)  # input untouched


@pytest.mark.slow
@pytest.mark.parametrize("n,dtype,ms", [((1 << 26) + 3, np.uint32, (1, 999, ((1 << 26) + 3) // 10)),
                                       (1 << 22, np.uint64, (1, 4194, (1 << 22) // 10,
                                                             (1 << 22) - 1, 1 << 22))])
def test_sparse_sample_parity(gpu, orc, n, dtype, ms):
    """Samples far smaller than their array (the sparse path: only the m
    steps and the positions they touch) and up to the whole array, against
    the oracle's partial shuffle of a copy; the input stays untouched."""
    s6g, s6o = both_schedules(gpu, orc, 6)
    data = (np.arange(n, dtype=np.uint64) * 0x9E3779B97F4A7C15 % (1 << 63)).astype(dtype)
    d = to_dev(data)
    for m in ms:
        say("sparse sample", np.dtype(dtype).name, n, m)
        out = to_dev(np.zeros(m, dtype))
        gpu.check(gpu.brr_sample(d, n, m, data.itemsize, out, s6g, 41, m), "brr_sample")
        assert gpu.brr_sync_status() == 0
        err, want = orc.sample(data, m, s6o, 41, m)
        assert err == 0
        assert np.array_equal(to_host(out), want), (n, m)
    assert np.array_equal(to_host(d), data)


def run_batched(gpu, sizes, dtype, seed, inst_base, plan=True, graph=True, reps=1, sched=None,
                **mapping):
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes, dtype)
    d = to_dev(data)
    d_off = to_dev(off)
    p = None
    if plan:
        p = gpu.Plan(off, data.itemsize, sched)
        m = p.mapping()
        m.use_graph = int(graph)
        for key, v in mapping.items():
            setattr(m, key, v)
        gpu.check(p.set_mapping(m), "set_mapping")
    results = []
    for _ in range(reps):
        d.copy_(to_dev(data))
        gpu.check(gpu.brr_shuffle_batched(d, d_off, len(sizes), data.itemsize, p, seed, inst_base),
                  "brr_shuffle_batched")
        assert gpu.brr_sync_status() == 0
        results.append(to_host(d))
    if p is not None:
        p.close()
    return data, off, results


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_batched_ragged_parity(gpu, orc, graph, dtype):
    rng = np.random.default_rng(5)
    sizes = np.concatenate([[0, 1, 2, 3, 512, 513, 16384, 16385],
                            np.floor(2 ** rng.uniform(1, 16.2, size=300))]).astype(np.uint64)
    say("batched ragged", graph, np.dtype(dtype).name)
    data, off, results = run_batched(gpu, sizes, dtype, seed=3, inst_base=1000, graph=graph, reps=3)
    want = data.copy()
    assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 3, 1000) == 0
    for got in results:  # every replay of the graph is checked
        assert np.array_equal(got, want)


def test_batched_without_plan(gpu, orc):
    sizes = np.array([7, 300, 5000, 40000, 2, 64], dtype=np.uint64)
    say("batched no plan")
    data, off, results = run_batched(gpu, sizes, np.uint32, seed=8, inst_base=0, plan=False)
    want = data.copy()
    assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 8, 0) == 0
    assert np.array_equal(results[0], want)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("max_k", [6, 2, 1, "costs", "wide", "deep"])
def test_batched_lane_tier(gpu, orc, dtype, max_k):
    """One lane per shuffle: every size up to the tier's limit, ragged and in
    runs of equal sizes (both copy paths), with a partly filled last block of
    lanes, under several schedules ("wide":
    up to 8 dice with exact-product guards, so that about one batch in 2^8
    is rejected at n = 256; "deep": batches of 9 and 10 dice)."""
    cap = 256
    rng = np.random.default_rng(21)
    # runs of equal sizes give blocks of lanes whose arrays are contiguous
    sizes = np.concatenate([np.arange(cap + 1), np.full(150, 37), rng.integers(0, cap + 1, size=131),
                            np.full(70, cap), [cap + 1, 600]]).astype(np.uint64)
    if max_k == "costs":
        sg = gpu.brr_schedule_from_costs(6, 25.0, 40.0, pow2=False, smooth=True)
        so = orc.Schedule.from_segments(sg.steps(), tail=bool(sg.tail), u_tail=sg.u_tail)
    elif max_k in ("wide", "deep"):
        steps = ([(305, 1, 0), (146, 7, 0), (8, 8, 0)] if max_k == "wide"
                 else [(120, 1, 0), (40, 9, 0), (11, 10, 0)])
        sg = gpu.brr_schedule.from_steps(steps, tail=True, u_tail=0)
        so = orc.Schedule.from_segments(steps, tail=True, u_tail=0)
    else:
        sg, so = both_schedules(gpu, orc, max_k)
    say("batched lane tier", np.dtype(dtype).name, max_k)
    data, off, results = run_batched(gpu, sizes, dtype, seed=31, inst_base=11, reps=2, sched=sg,
                                     lane_max=cap)
    want = data.copy()
    assert orc.shuffle_batched(want, off, so, 31, 11) == 0
    for got in results:
        assert np.array_equal(got, want)


def test_lane_mapping_limits(gpu):
    off = workloads.csr_offsets(np.array([3, 4], dtype=np.uint64))
    for eb in (4, 8):
        p = gpu.Plan(off, eb)
        m = p.mapping()
        m.lane_max = 257
        assert p.set_mapping(m) == gpu.BRR_EINVAL
        m.lane_max = 256
        assert p.set_mapping(m) == 0
        p.close()


@pytest.mark.slow
@pytest.mark.parametrize("lane_max", [0, 256])
def test_batched_equal_size_full(gpu, orc, lane_max):
    """65,536 shuffles of n = 256 (values 0..255), seed 1, instance = id."""
    sizes = np.full(65536, 256, dtype=np.uint64)
    say("batched 65536 x 256, lane_max", lane_max)
    data, off, results = run_batched(gpu, sizes, np.uint32, seed=1, inst_base=0, reps=2,
                                     lane_max=lane_max)
    want = data.copy()
    assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 1, 0) == 0
    for got in results:
        assert np.array_equal(got, want)


def test_plan_rebinds_while_running(gpu, orc):
    """A plan called again with another buffer and instance before its last
    run has finished (no synchronization between calls): each replay must
    read its own arguments, never a later call's. Every tier is present
    (lane, LDS classes, peel, device-wide); every result equals the
    oracle's."""
    sizes = np.array([256, 100, 2048, 4097, 16384, 16385, 65536, 70001, 5, (1 << 20) + 1],
                     dtype=np.uint64)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes, np.uint32)
    d_off = to_dev(off)
    bufs = [to_dev(data) for _ in range(4)]
    plan = gpu.Plan(off, 4)
    say("plan rebinds while running", int(sizes.sum()))
    for r, d in enumerate(bufs):
        gpu.check(gpu.brr_shuffle_batched(d, d_off, len(sizes), 4, plan, 5, 100 + r),
                  "brr_shuffle_batched")
    assert gpu.brr_sync_status() == 0
    got = [to_host(d) for d in bufs]
    plan.close()
    for r in range(4):
        want = data.copy()
        assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 5, 100 + r) == 0
        assert np.array_equal(got[r], want), r


@pytest.mark.slow
def test_plan_replays_without_recapture(gpu, orc):
    """100 calls of one plan, each with a fresh buffer and instance base,
    enqueued behind a long-running kernel: the plan captures its graph once
    (on the first call, made beforehand) and no call waits on the host (the
    calls return while the kernel ahead of them still runs). Every tier is
    present; all 100 results equal the oracle's."""
    import time

    import torch

    sizes = np.array([256, 100, 300, 2048, 4097, 16384, 16385, 65536, 70001, 5, (1 << 20) + 1, 17],
                     dtype=np.uint64)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes, np.uint32)
    d_off = to_dev(off)
    calls = 100
    bufs = [to_dev(data) for _ in range(calls + 1)]
    plan = gpu.Plan(off, 4)
    say("plan replays: first call")
    gpu.check(gpu.brr_shuffle_batched(bufs[0], d_off, len(sizes), 4, plan, 9, 0))
    torch.cuda.synchronize()
    assert plan.captures() == 1
    say("plan replays: 100 calls behind a long kernel")
    s = torch.cuda.current_stream()
    torch.cuda._sleep(400_000_000)  # on the order of 0.2 s
    busy = torch.cuda.Event()
    busy.record(s)
    t0 = time.perf_counter()
    for c in range(1, calls + 1):
        gpu.check(gpu.brr_shuffle_batched(bufs[c], d_off, len(sizes), 4, plan, 9, 1000 * c))
    host_s = time.perf_counter() - t0
    still_running = not busy.query()
    torch.cuda.synchronize()
    print("host seconds for", calls, "calls:", host_s, "sleep still running:", still_running)
    assert still_running, host_s
    assert plan.captures() == 1
    assert gpu.brr_sync_status() == 0
    plan.close()
    s6 = orc.schedule_paper(6)
    for c in [0] + list(range(1, calls + 1)):
        want = data.copy()
        assert orc.shuffle_batched_threads(want, off, s6, 9, 1000 * c) == 0
        assert np.array_equal(to_host(bufs[c]), want), c


@pytest.mark.slow
def test_batched_ragged_full(gpu, orc):
    """20,000 shuffles, n log-uniform in [16, 65536) (seed 3), u32 payload."""
    sizes = workloads.ragged_sizes(20000, seed=3)
    say("batched ragged 20000", int(sizes.sum()))
    data, off, results = run_batched(gpu, sizes, np.uint32, seed=3, inst_base=0)
    want = data.copy()
    assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 3, 0) == 0
    assert np.array_equal(results[0], want)


@pytest.mark.slow
def test_shuffle_2_26(gpu, orc):
    n = 1 << 26
    s6g, s6o = both_schedules(gpu, orc, 6)
    say("shuffle 2^26")
    a = np.arange(n, dtype=np.uint32)
    got = gpu_shuffle(gpu, a, s6g, seed=42, inst=0)
    want = a.copy()
    assert orc.shuffle(want, s6o, 42, 0) == 0
    assert np.array_equal(got, want)


@pytest.mark.slow
def test_shuffle_2_27_plus_3(gpu, orc):
    """2^27 + 3 positions: 28-bit sort keys, sorted in three passes of
    10-bit digits (2^26 takes 9-bit digits, 2^21 + 5 8-bit ones)."""
    n = (1 << 27) + 3
    s6g, s6o = both_schedules(gpu, orc, 6)
    say("shuffle 2^27 + 3")
    a = np.arange(n, dtype=np.uint32)
    got = gpu_shuffle(gpu, a, s6g, seed=43, inst=2)
    want = a.copy()
    assert orc.shuffle(want, s6o, 43, 2) == 0
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("wave_max", [512, 100])
def test_batched_tier_boundaries(gpu, orc, dtype, wave_max):
    """Sizes on both sides of every size-class limit: lane (256), wavefront
    (wave_max), the workgroup classes (2048, 4096, 8192, 16384), peel (2^20)
    and device-wide tiers in one batch."""
    sizes = np.array([256, 257, 100, 101, 512, 513, 2048, 2049, 4096, 4097, 8192, 8193, 16384,
                      16385, 16404, 32773, 65536, 100000, 1 << 20, (1 << 20) + 1, 2, 70001],
                     dtype=np.uint64)
    say("batched tier boundaries", np.dtype(dtype).name, wave_max)
    data, off, results = run_batched(gpu, sizes, dtype, seed=12, inst_base=7, reps=2,
                                     wave_max=wave_max)
    want = data.copy()
    assert orc.shuffle_batched(want, off, orc.schedule_paper(6), 12, 7) == 0
    for got in results:
        assert np.array_equal(got, want)


def test_single_calls_stay_asynchronous(gpu, orc):
    """Shuffles and samples that take scratch (above 16,384 elements), and a
    ChaCha20 dice stream, enqueued behind a long-running kernel return while
    that kernel still runs (their scratch is the stream's buffer, not a
    per-call allocation); the buffers then grow for a larger call, are
    released, and are taken again; every result equals the oracle's."""
    import time

    import torch

    s6g, s6o = both_schedules(gpu, orc, 6)
    sizes = [100003, (1 << 21) + 5, 40000]
    arrays = [np.arange(n, dtype=np.uint32) * 3 + 1 for n in sizes]
    devs = [to_dev(a) for a in arrays]
    n_s, m_s = 3000000, 300000
    src = np.arange(n_s, dtype=np.uint64) * 7
    d_src, d_out = to_dev(src), to_dev(np.zeros(m_s, np.uint64))
    bounds = workloads.dice_bounds(1 << 20, seed=3)
    d_b, d_o = to_dev(bounds), to_dev(np.zeros(1 << 20, np.uint32))
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    say("single calls behind a long kernel")
    torch.cuda._sleep(400_000_000)  # on the order of 0.2 s
    busy = torch.cuda.Event()
    busy.record(s)
    t0 = time.perf_counter()
    for i, (d, n) in enumerate(zip(devs, sizes)):
        gpu.check(gpu.brr_shuffle(d, n, 4, s6g, 5, i), "brr_shuffle")
    gpu.check(gpu.brr_sample(d_src, n_s, m_s, 8, d_out, s6g, 6, 0), "brr_sample")
    gpu.check(gpu.brr_dice_chacha(d_b, d_o, 1 << 20, 4, 7, 0), "brr_dice_chacha")
    host_s = time.perf_counter() - t0
    still_running = not busy.query()
    torch.cuda.synchronize()
    print("host seconds:", host_s, "sleep still running:", still_running)
    assert still_running, host_s
    assert gpu.brr_sync_status() == 0
    for i, (a, n) in enumerate(zip(arrays, sizes)):
        want = a.copy()
        assert orc.shuffle(want, s6o, 5, i) == 0
        assert np.array_equal(to_host(devs[i]), want), n
    err, want = orc.sample(src, m_s, s6o, 6, 0)
    assert err == 0 and np.array_equal(to_host(d_out), want)
    err, want = orc.dice_stream(orc.STREAM_CHACHA20, bounds, 4, 7, 0)
    assert err == 0 and np.array_equal(to_host(d_o), want)
    say("released scratch, then taken again")
    assert gpu.brr_release_scratch() == 0
    d = to_dev(arrays[0])
    gpu.check(gpu.brr_shuffle(d, sizes[0], 4, s6g, 5, 0), "brr_shuffle")
    assert gpu.brr_sync_status() == 0
    want = arrays[0].copy()
    assert orc.shuffle(want, s6o, 5, 0) == 0
    assert np.array_equal(to_host(d), want)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("which", ["k6", "k1", "chacha20"])
def test_peel_resident_boundaries(gpu, orc, dtype, which):
    """Peel-tier arrays around the size below which the rest of an array
    moves into LDS for its last peels (22,272 elements for u32; 11,136 for
    u64, so every u64 array of the tier starts in HBM), and far above it,
    under shuffle_6, k = 1 (more peels, one die per batch) and shuffle_6 on
    ChaCha20 words (the other kernel instantiation)."""
    sizes = np.array([16385, 22271, 22272, 22273, 26368, 30000, 44545, 65536, 100000, 1 << 20],
                     dtype=np.uint64)
    if which == "chacha20":
        gs, os_ = word_stream_schedules(gpu, orc, "chacha")
    else:
        gs, os_ = both_schedules(gpu, orc, 6 if which == "k6" else 1)
    say("peel resident boundaries", np.dtype(dtype).name, which)
    data, off, results = run_batched(gpu, sizes, dtype, seed=21, inst_base=3, sched=gs)
    want = data.copy()
    assert orc.shuffle_batched(want, off, os_, 21, 3) == 0
    assert np.array_equal(results[0], want)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_global_shuffle_unaligned(gpu, orc, dtype):
    """Single shuffles of the device-wide tier whose array does not start
    16-byte aligned (the element-by-element copy pass) beside aligned ones
    (16-byte vectors), with the elements around the array left untouched."""
    gs, os_ = both_schedules(gpu, orc, 6)
    for n in (16385, 100003, (1 << 21) + 5):
        for shift in (0, 1, 3):
            say("unaligned global shuffle", np.dtype(dtype).name, n, shift)
            a = np.arange(n + shift + 2, dtype=dtype) * 7 + 3
            d = to_dev(a)
            gpu.check(gpu.brr_shuffle(d[shift:shift + n], n, a.itemsize, gs, 77, n), "brr_shuffle")
            assert gpu.brr_sync_status() == 0
            got = to_host(d)
            want = a.copy()
            part = want[shift:shift + n].copy()
            assert orc.shuffle(part, os_, 77, n) == 0
            want[shift:shift + n] = part
            assert np.array_equal(got, want), (n, shift)


# ---------------------------------------------------------------------------
# The division form (BRR_FORM_DIVISION steps; the naive two-dice shuffle)
# ---------------------------------------------------------------------------

def naive2_schedules(gpu, orc):
    return gpu.brr_schedule_naive2(), orc.schedule_naive2()


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("tier", ["lds", "global"])
def test_naive2_shuffle_parity(gpu, orc, dtype, tier):
    gs, os_ = naive2_schedules(gpu, orc)
    assert gs.forms() == os_.forms() == [1, 1] and gs.steps() == os_.segments()
    sizes = LDS_SIZES if tier == "lds" else GLOBAL_SIZES
    for n in sizes:
        say("naive2 shuffle", tier, np.dtype(dtype).name, n)
        a = np.arange(n, dtype=dtype) * 5 + 2
        got = gpu_shuffle(gpu, a, gs, seed=4321, inst=n)
        want = a.copy()
        assert orc.shuffle(want, os_, 4321, n) == 0
        assert np.array_equal(got, want), (tier, n)


def test_mixed_form_schedule(gpu, orc):
    """Forms change from step to step: multiply, division, multiply with a
    guard, then the (multiply) tail batch."""
    steps = [(5000, 1, 0), (300, 2, 0), (6, 3, 2**57)]
    forms = [0, 1, 0]
    gs = gpu.brr_schedule.from_steps(steps, tail=True, u_tail=720, forms=forms)
    os_ = orc.Schedule.from_segments(steps, tail=True, u_tail=720, forms=forms)
    for n in (7, 301, 4000, 16384, 70000):
        say("mixed forms", n)
        a = np.arange(n, dtype=np.uint32)
        got = gpu_shuffle(gpu, a, gs, seed=9, inst=2)
        want = a.copy()
        assert orc.shuffle(want, os_, 9, 2) == 0
        assert np.array_equal(got, want), n
    bad = gpu.brr_schedule.from_steps([(1, 2, 0)], tail=False, forms=[2])
    assert gpu.brr_schedule_check(bad, 100) == gpu.BRR_EINVAL


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_naive2_batched_every_tier(gpu, orc, dtype):
    """Lane tier (every n up to 256), the wavefront and workgroup classes,
    peel and device-wide arrays, under the division-form schedule."""
    gs, os_ = naive2_schedules(gpu, orc)
    sizes = np.concatenate([np.arange(258), [511, 512, 513, 2049, 4097, 8193, 16384, 16385, 40000,
                                             (1 << 20), (1 << 20) + 1]]).astype(np.uint64)
    say("naive2 batched", np.dtype(dtype).name)
    data, off, results = run_batched(gpu, sizes, dtype, seed=19, inst_base=3, reps=2, sched=gs,
                                     lane_max=256)
    want = data.copy()
    assert orc.shuffle_batched(want, off, os_, 19, 3) == 0
    for got in results:
        assert np.array_equal(got, want)


def test_naive2_sample_parity(gpu, orc):
    gs, os_ = naive2_schedules(gpu, orc)
    rng = np.random.default_rng(10)
    for n, m in ((5, 5), (1000, 100), (16384, 1638), (100003, 10000), ((1 << 21) + 1, 1000)):
        say("naive2 sample", n, m)
        data = rng.integers(0, 2**31, size=n).astype(np.uint64)
        d = to_dev(data)
        out = to_dev(np.zeros(m, np.uint64))
        gpu.check(gpu.brr_sample(d, n, m, 8, out, gs, 33, n), "brr_sample")
        assert gpu.brr_sync_status() == 0
        err, want = orc.sample(data, m, os_, 33, n)
        assert err == 0 and np.array_equal(to_host(out), want), (n, m)


# ---------------------------------------------------------------------------
# The greedy largest-batch schedule (brr_schedule_kmax)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kcap", [4, 8])
def test_kmax_shuffle_parity(gpu, orc, kcap):
    gs, os_ = gpu.brr_schedule_kmax(kcap), orc.schedule_kmax(kcap)
    assert gs.steps() == os_.segments()
    for n in LDS_SIZES + [16385, 65538, 100003, (1 << 21) + 5, 2642247]:
        say("kmax shuffle", kcap, n)
        a = np.arange(n, dtype=np.uint32) * 7 + 3
        got = gpu_shuffle(gpu, a, gs, seed=555, inst=n)
        want = a.copy()
        assert orc.shuffle(want, os_, 555, n) == 0
        assert np.array_equal(got, want), (kcap, n)


def test_kmax_batched_every_tier(gpu, orc):
    gs, os_ = gpu.brr_schedule_kmax(8), orc.schedule_kmax(8)
    sizes = np.concatenate([np.arange(2, 258), [259, 260, 568, 569, 1627, 1628, 4097, 7133, 7134,
                                                16384, 16385, 65537, 65538, (1 << 20) + 1]])
    sizes = sizes.astype(np.uint64)
    say("kmax batched")
    data, off, results = run_batched(gpu, sizes, np.uint64, seed=41, inst_base=9, reps=2, sched=gs,
                                     lane_max=256)
    want = data.copy()
    assert orc.shuffle_batched(want, off, os_, 41, 9) == 0
    for got in results:
        assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# Other word streams: 32-bit halves (L = 32) and ChaCha20 words
# ---------------------------------------------------------------------------

def word_stream_schedules(gpu, orc, words):
    if words == "l32":  # Table 2's L = 32 column, exact thresholds
        gs = gpu.brr_schedule_from_costs(4, pow2=False, smooth=False, l32=True)
        os_ = orc.Schedule.from_segments(gs.steps(), tail=bool(gs.tail), u_tail=gs.u_tail,
                                         words=orc.WORDS_PHILOX32)
    else:  # shuffle_6 on ChaCha20 words
        steps = gpu.brr_schedule_paper(6).steps()
        gs = gpu.brr_schedule.from_steps(steps, tail=True, u_tail=720,
                                         words=gpu.BRR_WORDS_CHACHA20)
        os_ = orc.Schedule.from_segments(steps, tail=True, u_tail=720, words=orc.WORDS_CHACHA20)
    return gs, os_


@pytest.mark.parametrize("words", ["l32", "chacha"])
@pytest.mark.parametrize("tier", ["lds", "global"])
def test_word_stream_shuffle_parity(gpu, orc, words, tier):
    gs, os_ = word_stream_schedules(gpu, orc, words)
    sizes = LDS_SIZES if tier == "lds" else GLOBAL_SIZES
    for n in sizes:
        say("shuffle", words, tier, n)
        a = np.arange(n, dtype=np.uint64) * 11 + 5
        got = gpu_shuffle(gpu, a, gs, seed=808, inst=n)
        want = a.copy()
        assert orc.shuffle(want, os_, 808, n) == 0
        assert np.array_equal(got, want), (words, n)


@pytest.mark.parametrize("words", ["l32", "chacha"])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_word_stream_batched_every_tier(gpu, orc, words, dtype):
    gs, os_ = word_stream_schedules(gpu, orc, words)
    sizes = np.concatenate([np.arange(258), [511, 512, 513, 2049, 4097, 8193, 16384, 16385, 40000,
                                             (1 << 20), (1 << 20) + 1]]).astype(np.uint64)
    say("batched", words, np.dtype(dtype).name)
    data, off, results = run_batched(gpu, sizes, dtype, seed=27, inst_base=6, reps=2, sched=gs,
                                     lane_max=256)
    want = data.copy()
    assert orc.shuffle_batched(want, off, os_, 27, 6) == 0
    for got in results:
        assert np.array_equal(got, want)


@pytest.mark.parametrize("words", ["l32", "chacha"])
def test_word_stream_sample_parity(gpu, orc, words):
    gs, os_ = word_stream_schedules(gpu, orc, words)
    rng = np.random.default_rng(12)
    for n, m in ((5, 5), (1000, 100), (16384, 1638), (100003, 10000), ((1 << 21) + 1, 1000)):
        say("sample", words, n, m)
        data = rng.integers(0, 2**31, size=n).astype(np.uint32)
        d = to_dev(data)
        out = to_dev(np.zeros(m, np.uint32))
        gpu.check(gpu.brr_sample(d, n, m, 4, out, gs, 35, n), "brr_sample")
        assert gpu.brr_sync_status() == 0
        err, want = orc.sample(data, m, os_, 35, n)
        assert err == 0 and np.array_equal(to_host(out), want), (words, n, m)


def test_chacha_division_schedule(gpu, orc):
    """Division-form pairs on ChaCha20 words."""
    steps = [(1 << 32, 1, 0), (1, 2, 0)]
    gs = gpu.brr_schedule.from_steps(steps, tail=False, forms=[1, 1], words=gpu.BRR_WORDS_CHACHA20)
    os_ = orc.Schedule.from_segments(steps, tail=False, forms=[1, 1], words=orc.WORDS_CHACHA20)
    for n in (9, 5000, 70001):
        say("chacha division", n)
        a = np.arange(n, dtype=np.uint32)
        got = gpu_shuffle(gpu, a, gs, seed=3, inst=1)
        want = a.copy()
        assert orc.shuffle(want, os_, 3, 1) == 0
        assert np.array_equal(got, want), n
