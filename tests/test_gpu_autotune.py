"""Autotuning on the device: every tuned configuration is still bit-exact
with the oracle run under the schedule the plan reports."""
import numpy as np
import pytest

from conftest import say, to_dev, to_host
from paper_2408_06213_amd import workloads

pytestmark = pytest.mark.gpu


def test_dice_autotune(gpu):
    say("dice autotune")
    k, times = gpu.brr_dice_autotune(2**16 - 1, 1 << 22, with_times=True)
    assert 1 <= k <= 4 and set(times) == {1, 2, 3, 4}
    assert times[k] == min(times.values())
    assert gpu.brr_dice_autotune(2**16 - 1, 1 << 22) == k  # cached
    k2, t2 = gpu.brr_dice_autotune(2**31, 1 << 20, with_times=True)
    assert set(t2) == {1, 2} and k2 in (1, 2)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_plan_autotune_parity(gpu, orc, dtype):
    rng = np.random.default_rng(21)
    sizes = np.floor(2 ** rng.uniform(4, 16.5, size=400)).astype(np.uint64)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes, dtype)
    d, d_off = to_dev(data), to_dev(off)
    plan = gpu.Plan(off, data.itemsize)
    say("plan autotune", np.dtype(dtype).name)
    rep = plan.autotune(d, d_off, seed=5, inst_base=3)
    assert rep.candidates >= 10 and rep.ms_best <= rep.ms_default
    assert np.array_equal(to_host(d), data)  # tuning shuffles a copy
    sched = plan.schedule()
    assert sched.steps() == rep.schedule.steps()
    gpu.check(gpu.brr_shuffle_batched(d, d_off, sizes.size, data.itemsize, plan, 5, 3))
    assert gpu.brr_sync_status() == 0
    want = data.copy()
    osched = orc.Schedule.from_segments(sched.steps(), tail=bool(sched.tail), u_tail=sched.u_tail)
    assert orc.shuffle_batched(want, off, osched, 5, 3) == 0
    assert np.array_equal(to_host(d), want)
    plan.close()


@pytest.mark.parametrize("words", ["chacha", "l32"])
def test_plan_autotune_keeps_word_stream(gpu, orc, words):
    """Tuning picks batch sizes and the mapping, never the word stream: a
    plan on ChaCha20 or 32-bit words stays on it, and the tuned plan is
    bit-exact with the oracle under the schedule it reports."""
    rng = np.random.default_rng(22)
    sizes = np.floor(2 ** rng.uniform(4, 15.5, size=200)).astype(np.uint64)
    off = workloads.csr_offsets(sizes)
    data = workloads.iota_segments(sizes, np.uint32)
    d, d_off = to_dev(data), to_dev(off)
    if words == "chacha":
        w = gpu.BRR_WORDS_CHACHA20
        s0 = gpu.brr_schedule.from_steps(gpu.brr_schedule_paper(6).steps(), tail=True, u_tail=720,
                                         words=w)
    else:
        w = gpu.BRR_WORDS_PHILOX32
        s0 = gpu.brr_schedule_from_costs(4, pow2=False, smooth=False, l32=True)
    plan = gpu.Plan(off, 4, s0)
    say("plan autotune", words)
    rep = plan.autotune(d, d_off, seed=6, inst_base=1)
    sched = plan.schedule()
    assert sched.words == w and rep.candidates >= 2
    gpu.check(gpu.brr_shuffle_batched(d, d_off, sizes.size, 4, plan, 6, 1))
    assert gpu.brr_sync_status() == 0
    want = data.copy()
    osched = orc.Schedule.from_segments(sched.steps(), tail=bool(sched.tail), u_tail=sched.u_tail,
                                        forms=sched.forms(), words=int(sched.words))
    assert orc.shuffle_batched(want, off, osched, 6, 1) == 0
    assert np.array_equal(to_host(d), want)
    plan.close()
