"""The cost model of Sec. 6.1 and the schedules derived from it (host only)."""
import math

import pytest

from conftest import golden_rows


@pytest.fixture(scope="module")
def brr():
    from paper_2408_06213_amd import brr

    return brr


def test_cost_model_reproduces_table2(brr):
    want = {}
    for row in golden_rows("table2.txt"):
        k, L, nk = map(int, row.split())
        want.setdefault(L, {})[k] = nk
    assert brr.brr_cost_thresholds(64, 8) == want[64]
    assert brr.brr_cost_thresholds(32, 4) == want[32]


def test_cost_model_formula_points(brr):
    # small n: p1 and p2 vanish, so the cost is (c_rng + k) / k
    for k in (1, 2, 3, 6):
        assert brr.brr_cost_per_die(10, k) == pytest.approx((2 + k) / k, rel=1e-9)
    # exact terms at one point: n = 2^31, k = 2 (p1, p2 written out by hand)
    n = 2**31
    b = n * (n - 1)
    p1, p2 = b / 2**64, (2**64 % b) / 2**64
    want = ((2 + 2) / (1 - p2) + (16 + 1) * p1) / 2
    assert brr.brr_cost_per_die(n, 2) == pytest.approx(want, rel=1e-12)
    assert math.isinf(brr.brr_cost_per_die(2**33, 2))  # product above 2^64
    # thresholds are where the k-batch stops being cheaper than the (k-1)-batch
    for k, nk in brr.brr_cost_thresholds(64, 6).items():
        assert brr.brr_cost_per_die(nk, k) < brr.brr_cost_per_die(nk, k - 1)
        assert brr.brr_cost_per_die(nk + 1, k) >= brr.brr_cost_per_die(nk + 1, k - 1)


def test_cost_schedule_is_shuffle_6(brr):
    """Table 2 rounded down to powers of two, with guards n_k^k, is the
    paper's shuffle_6 schedule (Sec. 6.1, Sec. 7)."""
    got = brr.brr_schedule_from_costs(6, 2.0, 16.0, True)
    s6 = brr.brr_schedule_paper(6)
    assert got.steps() == s6.steps()
    assert got.tail == s6.tail and got.u_tail == s6.u_tail


@pytest.mark.parametrize("kmax", [2, 3, 4, 5, 7, 8])
def test_cost_schedules_are_valid(brr, kmax):
    s = brr.brr_schedule_from_costs(kmax, 2.0, 16.0, True)
    for n in (2, 3, 7, 100, 1000, 2**20, 2**31 - 1):
        assert brr.brr_schedule_check(s, n) == brr.BRR_OK, (kmax, n)
    assert max(k for _, k, _ in s.steps()) == kmax
