"""GPU parity of the dice-stream kernels (brr_dice, brr_dice_const) with the
CPU oracle: bit-exact, through the C ABI."""
import numpy as np
import pytest

from conftest import say, to_dev, to_host
from paper_2408_06213_amd import workloads

pytestmark = pytest.mark.gpu

# bound width per k so that a group's product stays <= 2^64
BITS = {1: 32, 2: 32, 3: 21, 4: 16, 5: 12, 6: 10, 7: 9, 8: 8}


def run_dice(gpu, bounds_np, k, seed, inst, offset=0):
    n = bounds_np.size
    b = to_dev(np.concatenate([np.zeros(offset, np.uint32), bounds_np]))
    out = to_dev(np.zeros(n + offset, np.uint32))
    bp = b.data_ptr() + 4 * offset
    op = out.data_ptr() + 4 * offset
    gpu.check(gpu.brr_dice(bp, op, n, k, seed, inst), "brr_dice")
    st = gpu.brr_sync_status()
    return st, to_host(out)[offset:]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dice_parity_ragged_counts(gpu, orc, k):
    rng = np.random.default_rng(100 + k)
    for count in (1, 2, 3, 4 * k - 1, 4 * k, 4 * k + 1, 1000 + 7, 65536 + 3, 300001):
        say("dice", k, count)
        bounds = rng.integers(1, 1 << BITS[k], size=count, dtype=np.uint64).astype(np.uint32)
        st, got = run_dice(gpu, bounds, k, seed=11, inst=3)
        err, want = orc.dice(bounds, k, 11, 3)
        assert st == 0 and err == 0
        assert np.array_equal(got, want), (k, count)


@pytest.mark.parametrize("k", [1, 3, 4])
def test_dice_unaligned_buffers(gpu, orc, k):
    bounds = workloads.dice_bounds(5003, seed=2)
    say("dice unaligned", k)
    st, got = run_dice(gpu, bounds, k, seed=5, inst=0, offset=1)
    assert st == 0
    assert np.array_equal(got, orc.dice(bounds, k, 5, 0)[1])


def test_dice_rejection_heavy(gpu, orc):
    """Pairs with product 2^63 + 2^31 - 1 reject about half of all words."""
    bounds = np.tile(np.array([2**31 + 1, 2**32 - 1], np.uint32), 20000)
    say("dice rejection heavy")
    st, got = run_dice(gpu, bounds, 2, seed=1, inst=9)
    assert st == 0
    assert np.array_equal(got, orc.dice(bounds, 2, 1, 9)[1])


def test_dice_product_exactly_2_64(gpu, orc):
    bounds = np.tile(np.array([2**31, 2**31, 4], np.uint32), 777)
    say("dice product 2^64")
    st, got = run_dice(gpu, bounds, 3, seed=3, inst=0)
    assert st == 0
    assert np.array_equal(got, orc.dice(bounds, 3, 3, 0)[1])


def test_dice_device_errors(gpu):
    say("dice zero bound")
    b = workloads.dice_bounds(4096, seed=4)
    b[1234] = 0
    st, _ = run_dice(gpu, b, 4, seed=1, inst=0)
    assert st == gpu.BRR_EINVAL
    assert gpu.brr_sync_status() == gpu.BRR_OK  # cleared after being read
    say("dice overflow")
    b = np.full(4096, 2**32 - 1, np.uint32)
    st, _ = run_dice(gpu, b, 3, seed=1, inst=0)
    assert st == gpu.BRR_EOVERFLOW
    assert gpu.brr_sync_status() == gpu.BRR_OK


@pytest.mark.parametrize("bound,k,count", [(6, 4, 100003), (2**16 - 1, 4, 4099), (2**31 + 1, 2, 5000),
                                           (1, 3, 10), (2**32 - 1, 1, 3001), (10, 8, 1234),
                                           (2**16, 4, 999)])
def test_dice_const_parity(gpu, orc, bound, k, count):
    say("dice_const", bound, k, count)
    out = to_dev(np.zeros(count, np.uint32))
    gpu.check(gpu.brr_dice_const(bound, out, count, k, 21, 4), "brr_dice_const")
    err, want = orc.dice_const(bound, count, k, 21, 4)
    assert err == 0
    assert np.array_equal(to_host(out), want)
    # Algorithm 2 and Algorithm 3 agree on the device too
    st, got = run_dice(gpu, np.full(count, bound, np.uint32), k, 21, 4)
    assert st == 0 and np.array_equal(got, want)


def test_dice_const_overflow_rejected_on_host(gpu):
    out = to_dev(np.zeros(16, np.uint32))
    assert gpu.brr_dice_const(2**32 - 1, out, 16, 3, 1, 0) == gpu.BRR_EOVERFLOW


# ---------------------------------------------------------------------------
# Word width 32 (brr_dice32)
# ---------------------------------------------------------------------------

# bound width per k so that a group's product stays <= 2^32
BITS32 = {1: 32, 2: 16, 3: 10, 4: 8, 5: 6, 6: 5, 7: 4, 8: 4}


def run_dice32(gpu, bounds_np, k, seed, inst, offset=0):
    n = bounds_np.size
    b = to_dev(np.concatenate([np.zeros(offset, np.uint32), bounds_np]))
    out = to_dev(np.zeros(n + offset, np.uint32))
    gpu.check(gpu.brr_dice32(b.data_ptr() + 4 * offset, out.data_ptr() + 4 * offset, n, k, seed,
                             inst), "brr_dice32")
    st = gpu.brr_sync_status()
    return st, to_host(out)[offset:]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dice32_parity_ragged_counts(gpu, orc, k):
    """Bounds in the upper half of their width: products come near 2^32, so
    a good share of groups reroll (several times for some)."""
    rng = np.random.default_rng(300 + k)
    hi = 1 << BITS32[k]
    for count in (1, 3, 4 * k - 1, 4 * k + 1, 256 * k + 5, 1000 + 7, 65536 + 3, 300001):
        say("dice32", k, count)
        bounds = rng.integers(max(1, hi // 2), hi, size=count, dtype=np.uint64).astype(np.uint32)
        st, got = run_dice32(gpu, bounds, k, seed=13, inst=5)
        err, want = orc.dice32(bounds, k, 13, 5)
        assert st == 0 and err == 0
        assert np.array_equal(got, want), (k, count)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_dice32_unaligned_buffers(gpu, orc, k):
    rng = np.random.default_rng(400 + k)
    bounds = rng.integers(1, 1 << BITS32[k], size=5003, dtype=np.uint64).astype(np.uint32)
    say("dice32 unaligned", k)
    st, got = run_dice32(gpu, bounds, k, seed=5, inst=0, offset=1)
    assert st == 0
    assert np.array_equal(got, orc.dice32(bounds, k, 5, 0)[1])


def test_dice32_edge_cases(gpu, orc):
    # product exactly 2^32 (threshold 0)
    b = np.tile(np.array([2**16, 2**16], np.uint32), 999)
    st, got = run_dice32(gpu, b, 2, seed=3, inst=0)
    assert st == 0 and np.array_equal(got, orc.dice32(b, 2, 3, 0)[1])
    # the C2 stream's bounds at two dice per 32-bit word
    b = workloads.dice_bounds(100003, seed=7)
    st, got = run_dice32(gpu, b, 2, seed=7, inst=0)
    assert st == 0 and np.array_equal(got, orc.dice32(b, 2, 7, 0)[1])
    # errors reach the status word
    st, _ = run_dice32(gpu, np.array([2**16 + 1, 2**16] * 5, np.uint32), 2, 1, 0)
    assert st == gpu.BRR_EOVERFLOW
    st, _ = run_dice32(gpu, np.array([5, 0, 3, 4], np.uint32), 2, 1, 0)
    assert st == gpu.BRR_EINVAL
    assert gpu.brr_sync_status() == 0  # reading the status clears it


# ---------------------------------------------------------------------------
# The division form (brr_dice_div)
# ---------------------------------------------------------------------------

# bound width per k so that a group's product stays <= 2^64
BITS64 = {1: 32, 2: 32, 3: 21, 4: 16, 5: 12, 6: 10, 7: 9, 8: 8}


def run_dice_div(gpu, bounds_np, k, seed, inst, offset=0):
    n = bounds_np.size
    b = to_dev(np.concatenate([np.zeros(offset, np.uint32), bounds_np]))
    out = to_dev(np.zeros(n + offset, np.uint32))
    gpu.check(gpu.brr_dice_div(b.data_ptr() + 4 * offset, out.data_ptr() + 4 * offset, n, k, seed,
                               inst), "brr_dice_div")
    st = gpu.brr_sync_status()
    return st, to_host(out)[offset:]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dice_div_parity_ragged_counts(gpu, orc, k):
    """Bounds in the upper half of their width, so products come near 2^64
    and groups reroll."""
    rng = np.random.default_rng(500 + k)
    hi = 1 << BITS64[k]
    for count in (1, 3, 4 * k - 1, 256 * k + 5, 1000 + 7, 65536 + 3, 300001):
        say("dice_div", k, count)
        bounds = rng.integers(max(1, hi // 2), hi, size=count, dtype=np.uint64).astype(np.uint32)
        st, got = run_dice_div(gpu, bounds, k, seed=17, inst=6)
        err, want = orc.dice_div(bounds, k, 17, 6)
        assert st == 0 and err == 0
        assert np.array_equal(got, want), (k, count)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_dice_div_unaligned_buffers(gpu, orc, k):
    rng = np.random.default_rng(600 + k)
    bounds = rng.integers(1, 1 << BITS64[k], size=5003, dtype=np.uint64).astype(np.uint32)
    say("dice_div unaligned", k)
    st, got = run_dice_div(gpu, bounds, k, seed=5, inst=0, offset=1)
    assert st == 0
    assert np.array_equal(got, orc.dice_div(bounds, k, 5, 0)[1])


def test_dice_div_edge_cases(gpu, orc):
    # product exactly 2^64: V is the word itself
    b = np.full(4 * 999, 1 << 16, np.uint32)
    st, got = run_dice_div(gpu, b, 4, seed=3, inst=0)
    assert st == 0 and np.array_equal(got, orc.dice_div(b, 4, 3, 0)[1])
    # rejection-heavy pairs (product 2^63 + 2^31 - 1)
    b = np.tile(np.array([2**31 + 1, 2**32 - 1], np.uint32), 5000)
    st, got = run_dice_div(gpu, b, 2, seed=4, inst=1)
    assert st == 0 and np.array_equal(got, orc.dice_div(b, 2, 4, 1)[1])
    # the 2^28 stream's bounds (uniform below 2^16) at k = 2..4
    b = workloads.dice_bounds(100003, seed=7)
    for k in (2, 3, 4):
        st, got = run_dice_div(gpu, b, k, seed=7, inst=0)
        assert st == 0 and np.array_equal(got, orc.dice_div(b, k, 7, 0)[1]), k
    st, _ = run_dice_div(gpu, np.array([2**32 - 1] * 6, np.uint32), 3, 1, 0)
    assert st == gpu.BRR_EOVERFLOW
    st, _ = run_dice_div(gpu, np.array([5, 0, 3, 4], np.uint32), 2, 1, 0)
    assert st == gpu.BRR_EINVAL
    assert gpu.brr_sync_status() == 0


# ---------------------------------------------------------------------------
# ChaCha20 words (brr_dice_chacha)
# ---------------------------------------------------------------------------

def run_dice_chacha(gpu, bounds_np, k, seed, inst, offset=0):
    n = bounds_np.size
    b = to_dev(np.concatenate([np.zeros(offset, np.uint32), bounds_np]))
    out = to_dev(np.zeros(n + offset, np.uint32))
    gpu.check(gpu.brr_dice_chacha(b.data_ptr() + 4 * offset, out.data_ptr() + 4 * offset, n, k,
                                  seed, inst), "brr_dice_chacha")
    st = gpu.brr_sync_status()
    return st, to_host(out)[offset:]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dice_chacha_parity_ragged_counts(gpu, orc, k):
    """Bounds in the upper half of their width (rerolls); counts around the
    8-group lane tiles and the 256-lane blocks, short last groups."""
    rng = np.random.default_rng(700 + k)
    hi = 1 << BITS64[k]
    for count in (1, 3, 8 * k - 1, 8 * k + 1, 2048 * k + 5, 1000 + 7, 65536 + 3, 300001):
        say("dice_chacha", k, count)
        bounds = rng.integers(max(1, hi // 2), hi, size=count, dtype=np.uint64).astype(np.uint32)
        st, got = run_dice_chacha(gpu, bounds, k, seed=23, inst=4)
        err, want = orc.dice_chacha(bounds, k, 23, 4)
        assert st == 0 and err == 0
        assert np.array_equal(got, want), (k, count)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_dice_chacha_unaligned_buffers(gpu, orc, k):
    rng = np.random.default_rng(800 + k)
    bounds = rng.integers(1, 1 << BITS64[k], size=5003, dtype=np.uint64).astype(np.uint32)
    say("dice_chacha unaligned", k)
    st, got = run_dice_chacha(gpu, bounds, k, seed=6, inst=1, offset=1)
    assert st == 0
    assert np.array_equal(got, orc.dice_chacha(bounds, k, 6, 1)[1])


def test_dice_chacha_edge_cases(gpu, orc):
    b = np.full(4 * 999, 1 << 16, np.uint32)  # product 2^64
    st, got = run_dice_chacha(gpu, b, 4, seed=3, inst=0)
    assert st == 0 and np.array_equal(got, orc.dice_chacha(b, 4, 3, 0)[1])
    b = np.tile(np.array([2**31 + 1, 2**32 - 1], np.uint32), 5000)  # about half rejected
    st, got = run_dice_chacha(gpu, b, 2, seed=4, inst=1)
    assert st == 0 and np.array_equal(got, orc.dice_chacha(b, 2, 4, 1)[1])
    b = workloads.dice_bounds(100003, seed=7)
    for k in (1, 2, 3, 4):
        st, got = run_dice_chacha(gpu, b, k, seed=7, inst=0)
        assert st == 0 and np.array_equal(got, orc.dice_chacha(b, k, 7, 0)[1]), k
    st, _ = run_dice_chacha(gpu, np.array([2**32 - 1] * 6, np.uint32), 3, 1, 0)
    assert st == gpu.BRR_EOVERFLOW
    st, _ = run_dice_chacha(gpu, np.array([5, 0, 3, 4], np.uint32), 2, 1, 0)
    assert st == gpu.BRR_EINVAL
    assert gpu.brr_sync_status() == 0


# ---------------------------------------------------------------------------
# Known bounds (brr_dice_tuple, Algorithm 2)
# ---------------------------------------------------------------------------

def test_dice_tuple_parity(gpu, orc):
    cases = [([4, 6, 8, 20], 4001), ([2**31 + 1, 2**32 - 1], 100001), ([6], 777),
             ([3, 5, 7, 11, 13, 17, 19, 23], 8 * 4096 + 5), ([1 << 16] * 4, 4 * 3000),
             ([2**21 - 1, 2**21 - 3, 2**21 - 5], 3 * 70000 + 2), ([1, 1, 2], 1000)]
    for tup, count in cases:
        for offset in (0, 1):
            say("dice_tuple", tup, count, offset)
            out = to_dev(np.zeros(count + offset, np.uint32))
            gpu.check(gpu.brr_dice_tuple(tup, out.data_ptr() + 4 * offset, count, 21, 2),
                      "brr_dice_tuple")
            assert gpu.brr_sync_status() == 0
            err, want = orc.dice_tuple(tup, count, 21, 2)
            assert err == 0 and np.array_equal(to_host(out)[offset:], want), (tup, count)


def test_dice_tuple_equals_dice_on_tiled_bounds(gpu):
    """The known-threshold path and the general path agree on the device."""
    tup, count = [10, 12, 1000, 77], 50003
    tiled = to_dev(np.resize(np.array(tup, np.uint32), count))
    a = to_dev(np.zeros(count, np.uint32))
    b = to_dev(np.zeros(count, np.uint32))
    gpu.check(gpu.brr_dice_tuple(tup, a, count, 5, 9), "brr_dice_tuple")
    gpu.check(gpu.brr_dice(tiled, b, count, len(tup), 5, 9), "brr_dice")
    assert gpu.brr_sync_status() == 0
    assert np.array_equal(to_host(a), to_host(b))


# ---------------------------------------------------------------------------
# Full size: every 2^28-roll stream the benchmark times, in the launch
# configuration it times, compared whole with the oracle (its group range
# split over every host core)
# ---------------------------------------------------------------------------

FULL = 1 << 28


@pytest.fixture(scope="module")
def full_bounds():
    """The benchmark's two 2^28 bound streams: uniform in [1, 2^16) from
    seed 7, and uniform in [1, 2^12) from seed 8."""
    return {7: workloads.dice_bounds(FULL, seed=7), 8: workloads.dice_bounds(FULL, seed=8, high=1 << 12)}


FULL_CASES = ([("mul", k, 7) for k in (1, 2, 3, 4)] + [("div", k, 7) for k in (1, 2, 3, 4)]
              + [("chacha", k, 7) for k in (1, 2, 3, 4)] + [("l32", k, 7) for k in (1, 2)]
              + [("const", k, 7) for k in (1, 2, 3, 4)] + [("tuple", 4, 7)]
              + [("mul", k, 8) for k in (1, 2)] + [("l32", k, 8) for k in (1, 2)]
              + [("chacha", k, 8) for k in (1, 2, 3, 4)])


@pytest.mark.slow
@pytest.mark.parametrize("entry,k,seed", FULL_CASES)
def test_full_size_stream_whole(gpu, orc, full_bounds, entry, k, seed):
    """All 2^28 outputs bit for bit: brr_dice (k = 1..4), brr_dice_div,
    brr_dice_chacha, brr_dice32 and the known-bounds streams (one bound
    65535, Algorithm 2, k = 1..4; the tuple (6, 10, 12, 20)) on the seed-7
    bounds, and the seed-8 stream (bounds below 2^12) at both word widths
    and on ChaCha20 words. Known-bound streams are compared with Algorithm 3
    on the bounds written out (the two are equal: oracle pins)."""
    import torch

    say("full size whole", entry, k, seed)
    if entry == "const":
        bounds = np.full(FULL, 65535, np.uint32)
    elif entry == "tuple":
        tup = [6, 10, 12, 20]
        bounds = np.resize(np.array(tup, np.uint32), FULL)
    else:
        bounds = full_bounds[seed]
    out = torch.empty(FULL, dtype=torch.uint32, device="cuda")
    if entry == "const":
        gpu.check(gpu.brr_dice_const(65535, out, FULL, k, seed, 0), "brr_dice_const")
    elif entry == "tuple":
        gpu.check(gpu.brr_dice_tuple(tup, out, FULL, seed, 0), "brr_dice_tuple")
    else:
        b = to_dev(bounds)
        fn = {"mul": gpu.brr_dice, "div": gpu.brr_dice_div, "chacha": gpu.brr_dice_chacha,
              "l32": gpu.brr_dice32}[entry]
        gpu.check(fn(b, out, FULL, k, seed, 0), entry)
        del b
    assert gpu.brr_sync_status() == 0
    got = to_host(out)
    del out
    kind = {"mul": orc.STREAM_MULTIPLY, "const": orc.STREAM_MULTIPLY, "tuple": orc.STREAM_MULTIPLY,
            "div": orc.STREAM_DIVISION, "chacha": orc.STREAM_CHACHA20, "l32": orc.STREAM_L32}[entry]
    err, want = orc.dice_stream(kind, bounds, k, seed, 0)
    assert err == 0
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{entry} k={k}: {bad.size} of {FULL} rolls differ, first at {bad[0]}")


def test_dice_chacha_rare_heavy_groups(gpu, orc):
    """ChaCha20 dice, k = 2: small bounds (no rerolls) except one group in
    997 with product 2^63 + 2^31 - 1, rejected about half the time, so the
    reroll waves hold one or two groups each and try many attempts of a
    group side by side (a group's first accepted attempt must win)."""
    rng = np.random.default_rng(41)
    groups = (1 << 20) + 333
    bounds = rng.integers(1, 1 << 10, size=2 * groups, dtype=np.uint64).astype(np.uint32)
    heavy = np.arange(5, groups, 997)
    bounds[2 * heavy] = 2**31 + 1
    bounds[2 * heavy + 1] = 2**32 - 1
    say("dice_chacha rare heavy groups", groups)
    st, got = run_dice_chacha(gpu, bounds, 2, seed=17, inst=2)
    err, want = orc.dice_chacha(bounds, 2, 17, 2)
    assert st == 0 and err == 0
    assert np.array_equal(got, want)


@pytest.mark.slow
def test_dice_chacha_long_stream(gpu, orc):
    """ChaCha20 dice, k = 2, on 2^29 + 4101 * 1024 + 77 bounds uniform below
    2^31 (about 3% of the groups reroll, as in the 16-bit stream at k = 4):
    270535207 groups in 132098 blocks of 2048, the last one short, and
    reroll words past index 2^29."""
    import torch

    count = (1 << 29) + 4101 * 1024 + 77
    bounds = workloads.dice_bounds(count, seed=9, high=1 << 31)
    say("dice_chacha long stream", count)
    b = to_dev(bounds)
    out = torch.empty(count, dtype=torch.uint32, device="cuda")
    gpu.check(gpu.brr_dice_chacha(b, out, count, 2, 12, 3), "brr_dice_chacha")
    assert gpu.brr_sync_status() == 0
    del b
    got = to_host(out)
    del out
    err, want = orc.dice_stream(orc.STREAM_CHACHA20, bounds, 2, 12, 3)
    assert err == 0
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{bad.size} of {count} rolls differ, first at {bad[0]}")


def test_copy_probe_copies(gpu):
    """The roofline's copy probe moves the bytes it claims: dst equals src
    after it, with a ragged last tile (1 MiB + 48 bytes)."""
    nbytes = (1 << 20) + 48
    rng = np.random.default_rng(21)
    src_np = rng.integers(0, 2**32, size=nbytes // 4, dtype=np.uint32)
    src, dst = to_dev(src_np), to_dev(np.zeros_like(src_np))
    say("copy probe", nbytes)
    rate = gpu.brr_probe_copy_rate(src, dst, nbytes, 2)
    assert rate > 0
    assert np.array_equal(to_host(dst), src_np)
