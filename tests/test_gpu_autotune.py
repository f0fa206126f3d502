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
