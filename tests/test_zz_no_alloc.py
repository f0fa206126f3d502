"""brr_shuffle_noalloc, the entry point for callers that cannot allocate,
through the C ABI: its output against brr_shuffle's (the same arguments,
bit for bit) and the oracle's, over calls in a row on one device that share
its scratch array, each next one smaller than the one before."""
import numpy as np
import pytest

from conftest import say, to_dev, to_host


def test_noalloc_host_errors():
    """Rejected on the host, before any device work."""
    from paper_2408_06213_amd import brr

    assert brr.lib.brr_shuffle_noalloc(0x20000, 2**21 + 1, 4, None, 1, 0, None) == brr.BRR_EINVAL
    assert brr.lib.brr_shuffle_noalloc(0x20000, 2**32, 8, None, 1, 0, None) == brr.BRR_EINVAL
    assert brr.lib.brr_shuffle_noalloc(None, 10, 4, None, 1, 0, None) == brr.BRR_EINVAL
    assert brr.lib.brr_shuffle_noalloc(None, 1, 4, None, 1, 0, None) == brr.BRR_OK
    assert brr.lib.brr_shuffle_noalloc(0x20000, 10, 3, None, 1, 0, None) == brr.BRR_EINVAL
    assert brr.lib.brr_shuffle_noalloc(0x10004, 10, 8, None, 1, 0, None) == brr.BRR_EINVAL


def _inputs(n, dtype):
    return (np.arange(n, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(dtype)


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_noalloc_calls_in_a_row_match_shuffle(gpu, orc, dtype):
    """Four calls enqueued back to back on one stream (largest first: 2^21,
    the largest size allowed, then 100,003, 20,000 and 5,000 elements; the
    first three use the scratch array, the last runs in LDS), then the same
    four through brr_shuffle, which allocates its scratch. Every output is
    equal bit for bit, and equal to the oracle's."""
    eb = np.dtype(dtype).itemsize
    cases = ((2**21, 9, 3), (100_003, 9, 4), (20_000, 5, 1), (5_000, 5, 2))
    s6 = gpu.brr_schedule_paper(6)
    ins = [_inputs(n, dtype) for n, _, _ in cases]
    say("noalloc in a row", np.dtype(dtype).name, [c[0] for c in cases])
    mine = [to_dev(a) for a in ins]
    for d, (n, seed, inst) in zip(mine, cases):
        gpu.check(gpu.brr_shuffle_noalloc(d, n, eb, s6, seed, inst), "brr_shuffle_noalloc")
    say("noalloc reference calls")
    ref = [to_dev(a) for a in ins]
    for d, (n, seed, inst) in zip(ref, cases):
        gpu.check(gpu.brr_shuffle(d, n, eb, s6, seed, inst), "brr_shuffle")
    assert gpu.brr_sync_status() == 0
    for a, d, r, (n, seed, inst) in zip(ins, mine, ref, cases):
        got = to_host(d)
        assert np.array_equal(got, to_host(r)), n
        want = a.copy()
        assert orc.shuffle(want, orc.schedule_paper(6), seed, inst) == 0
        assert np.array_equal(got, want), n


@pytest.mark.gpu
def test_noalloc_repeated_call_and_other_schedules(gpu, orc):
    """The same arguments twice in a row give the same output (no state
    survives a call), under the unbatched and the division-pair schedules."""
    n = 300_001
    a = _inputs(n, np.uint32)
    for sched, osched in ((gpu.brr_schedule_paper(1), orc.schedule_paper(1)),
                          (gpu.brr_schedule_naive2(), orc.schedule_naive2())):
        say("noalloc twice", n)
        d1, d2 = to_dev(a), to_dev(a)
        gpu.check(gpu.brr_shuffle_noalloc(d1, n, 4, sched, 17, 0), "brr_shuffle_noalloc")
        gpu.check(gpu.brr_shuffle_noalloc(d2, n, 4, sched, 17, 0), "brr_shuffle_noalloc")
        assert gpu.brr_sync_status() == 0
        got = to_host(d1)
        assert np.array_equal(got, to_host(d2))
        want = a.copy()
        assert orc.shuffle(want, osched, 17, 0) == 0
        assert np.array_equal(got, want)
