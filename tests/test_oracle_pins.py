"""Pins of the CPU oracle to what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Table 1), published known answers (Philox), closed forms
(Theorem 1's equal counts, the one-shot product), special cases that reduce
to another routine of the paper (k = 1 is Lemire's method; Algorithms 2 and 3
agree), invariants (permutations) and chi-square uniformity.
"""
import math

import numpy as np
import pytest
from scipy.stats import chi2

from conftest import golden_rows
from oracle import ref

TWO64 = 1 << 64


# ---------------------------------------------------------------------------
# Word source
# ---------------------------------------------------------------------------

def test_philox_known_answers(orc):
    rows = golden_rows("philox_kat.txt")
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row.split()]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_word_halves(orc):
    # word c is half (c mod 2) of Philox block c // 2 of counter (c//2, inst)
    seed, inst = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    for c in (0, 1, 2, 3, 1 << 33, (1 << 33) + 1):
        blk = c // 2
        x = orc.philox4x32_10([blk & 0xFFFFFFFF, blk >> 32, inst & 0xFFFFFFFF, inst >> 32],
                              [seed & 0xFFFFFFFF, seed >> 32])
        want = (x[0] | x[1] << 32) if c % 2 == 0 else (x[2] | x[3] << 32)
        assert orc.word(seed, inst, c) == want


# ---------------------------------------------------------------------------
# Theorem 1
# ---------------------------------------------------------------------------

def test_table1_worked_example(orc):
    rows = golden_rows("table1.txt")
    assert len(rows) == 16
    accepted = set()
    for row in rows:
        r0, two_r0, a1, r1, six_r1, a2, r2, rej = map(int, row.split())
        assert two_r0 == 2 * r0 and six_r1 == 6 * r1
        for impl in (orc.chain, ref.chain):
            a, rk = impl(4, [2, 6], r0)
            assert (a, rk) == ([a1, a2], r2)
        _, r_1 = orc.chain(4, [2], r0)
        assert r_1 == r1
        err, t = orc.threshold(4, [2, 6])
        assert err == 0 and t == 4
        assert (r2 < t) == bool(rej)
        if not rej:
            accepted.add((a1, a2))
    # every (coin, die) pair appears exactly once among the 12 accepted rows
    assert accepted == {(x, y) for x in range(2) for y in range(6)}


TUPLES = [
    (3,), (7,), (2, 6), (3, 5, 7), (2, 3, 4, 5), (5, 5), (1, 9), (9, 1, 1), (1,),
    (16, 16),            # product = 2^8  (t = 0 at L = 8)
    (4, 4, 16),          # product = 2^8
    (255,), (17, 15),    # product just below 2^8
    (11, 13, 17), (64, 64, 16), (6, 10, 15, 21),
]


@pytest.mark.parametrize("L", [8, 12, 16])
def test_theorem1_exhaustive(orc, L):
    """Every L-bit word: each accepted digit tuple occurs floor(2^L/b) times
    and exactly 2^L mod b words are rejected (Theorem 1 with Lemma 1)."""
    for bounds in TUPLES:
        b = math.prod(bounds)
        if b > (1 << L):
            continue
        err, t = orc.threshold(L, bounds)
        assert err == 0 and t == (1 << L) % b
        counts = {}
        rejects = 0
        for r0 in range(1 << L):
            a, rk = orc.chain(L, bounds, r0)
            assert all(0 <= ai < bi for ai, bi in zip(a, bounds))
            if rk >= t:
                counts[tuple(a)] = counts.get(tuple(a), 0) + 1
            else:
                rejects += 1
        assert rejects == (1 << L) % b
        assert len(counts) == b
        assert set(counts.values()) == {(1 << L) // b}
        if L <= 12:  # the big-integer reference agrees word for word
            rc, rr = ref.enumerate_all(L, list(bounds))
            assert rr == rejects and dict(rc) == counts


def test_chain_equals_one_shot_product_L64(orc):
    """(prod b) (x) r0 = (a, r_k) with a the mixed-radix value of the digits
    (the claim inside the proof of Theorem 1), at L = 64."""
    rng = np.random.default_rng(2408)
    for _ in range(400):
        k = int(rng.integers(1, 9))
        bounds = [int(x) for x in rng.integers(1, 1 << int(rng.integers(1, 33)), size=k)]
        if math.prod(bounds) > TWO64:
            continue
        r0 = int(rng.integers(0, TWO64, dtype=np.uint64))
        a, rk = orc.chain(64, bounds, r0)
        value, low = divmod(math.prod(bounds) * r0, TWO64)
        assert rk == low
        assert ref.mixed_radix(a, bounds) == value
        assert ref.digits(value, bounds) == a
    # a 64-bit bound (one die covering most of the word)
    a, rk = orc.chain(64, [TWO64 - 59], TWO64 - 1)
    assert (a[0], rk) == divmod((TWO64 - 59) * (TWO64 - 1), TWO64)


def test_threshold_L64(orc):
    for bounds in ([1], [2], [3], [6], [2**32 - 1, 2**32 - 1], [2**31, 2**31, 4], [TWO64 - 1],
                   [10**9, 10**9, 18]):
        err, t = orc.threshold(64, bounds)
        assert err == 0 and t == TWO64 % math.prod(bounds)
    assert orc.threshold(64, [2**32, 2**32, 2])[0] == 2   # product 2^65
    assert orc.threshold(64, [3, 0])[0] == 1              # zero bound


# ---------------------------------------------------------------------------
# Dice streams (Algorithms 2 and 3)
# ---------------------------------------------------------------------------

def _stream_words(orc, seed, inst, S, g):
    a = 0
    while True:
        yield orc.word(seed, inst, a * S + g)
        a += 1


def test_k1_dice_is_lemire(orc):
    """With one die per word the batched stream is Lemire's method (Sec. 2)."""
    rng = np.random.default_rng(5)
    bounds = np.concatenate([
        rng.integers(1, 1 << 32, size=300, dtype=np.uint64),
        rng.integers(1, 7, size=100, dtype=np.uint64),
        np.array([1, 2, 2**31, 2**31 + 1, 2**32 - 1], dtype=np.uint64)]).astype(np.uint32)
    err, out = orc.dice(bounds, 1, seed=99, inst=3)
    assert err == 0
    S = bounds.size
    for g, b in enumerate(bounds):
        x, _ = ref.lemire(64, int(b), _stream_words(orc, 99, 3, S, g))
        assert out[g] == x


def test_rejection_heavy_groups(orc):
    """Pairs (2^31+1, 2^32-1) have product 2^63 + 2^31 - 1, so about half of
    all words are rejected; every group must still follow Theorem 1 with the
    rerolls reading words a*S + g."""
    count = 400
    bounds = np.tile(np.array([2**31 + 1, 2**32 - 1], dtype=np.uint32), count // 2)
    err, out = orc.dice(bounds, 2, seed=1, inst=0)
    assert err == 0
    S = count // 2
    rerolled = 0
    for g in range(S):
        b = [2**31 + 1, 2**32 - 1]
        for att, r0 in enumerate(_stream_words(orc, 1, 0, S, g)):
            a, rk = ref.chain(64, b, r0)
            if rk >= TWO64 % (b[0] * b[1]):
                break
        rerolled += att > 0
        assert list(out[2 * g:2 * g + 2]) == a
    assert rerolled > S // 4


@pytest.mark.parametrize("k,bits", [(2, 32), (3, 21), (4, 16), (7, 9)])
def test_dice_groups_follow_theorem1(orc, k, bits):
    rng = np.random.default_rng(k)
    count = 1000 + k - 1  # last group short when k does not divide the count
    bounds = rng.integers(1, 1 << bits, size=count, dtype=np.uint64).astype(np.uint32)
    err, out = orc.dice(bounds, k, seed=7, inst=11)
    assert err == 0
    S = -(-count // k)
    for g in range(S):
        b = [int(x) for x in bounds[g * k:(g + 1) * k]]
        for r0 in _stream_words(orc, 7, 11, S, g):
            a, rk = ref.chain(64, b, r0)
            if ref.accept(64, b, rk):
                break
        assert list(out[g * k:g * k + len(b)]) == a
    assert np.all(out < bounds)


@pytest.mark.parametrize("bound,k,count", [(6, 4, 1001), (2**16 - 1, 4, 999), (2**31 + 1, 2, 500),
                                           (1, 3, 10), (2**32 - 1, 1, 300)])
def test_alg2_equals_alg3(orc, bound, k, count):
    """Known threshold (Algorithm 2) and unknown threshold (Algorithm 3)
    produce the same dice from the same words."""
    e1, a = orc.dice_const(bound, count, k, seed=5, inst=2)
    e2, b = orc.dice(np.full(count, bound, dtype=np.uint32), k, seed=5, inst=2)
    assert e1 == e2 == 0
    assert np.array_equal(a, b)


def test_dice_edge_cases(orc):
    # bound product exactly 2^64: threshold 0, every word accepted first time
    bounds = np.array([2**31, 2**31, 4], dtype=np.uint32)
    err, out = orc.dice(bounds, 3, seed=3, inst=0)
    assert err == 0
    a, _ = ref.chain(64, [2**31, 2**31, 4], orc.word(3, 0, 0))
    assert list(out) == a
    # product above 2^64
    assert orc.dice(np.array([2**32 - 1] * 3, dtype=np.uint32), 3, 1, 0)[0] == 2
    # zero bound
    assert orc.dice(np.array([5, 0, 7, 9], dtype=np.uint32), 2, 1, 0)[0] == 1
    # empty stream
    err, out = orc.dice(np.zeros(0, dtype=np.uint32), 4, 1, 0)
    assert err == 0 and out.size == 0


def test_dice_uniform_chi2(orc):
    """Digits of a k = 4 stream of 6-sided dice are uniform (chi-square)."""
    count = 400_000
    err, out = orc.dice_const(6, count, 4, seed=13, inst=0)
    assert err == 0
    hist = np.bincount(out, minlength=6)
    stat = float(((hist - count / 6) ** 2 / (count / 6)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 5)


# ---------------------------------------------------------------------------
# Dice streams at word width 32
# ---------------------------------------------------------------------------

TWO32 = 1 << 32


def _stream_words32(orc, seed, inst, S, g):
    a = 0
    while True:
        yield orc.word32(seed, inst, a * S + g)
        a += 1


def test_word32_is_halves_of_word64(orc):
    """The 32-bit stream reads each 64-bit word low half first."""
    for c in (0, 1, 2, 3, 10, 2**33 + 5):
        w = orc.word(21, 4, c)
        assert orc.word32(21, 4, 2 * c) == w & 0xFFFFFFFF
        assert orc.word32(21, 4, 2 * c + 1) == w >> 32


def test_chain_equals_one_shot_product_L32(orc):
    """Theorem 1's one-shot form at L = 32: (prod b) (x) r0 = (a, r_k)."""
    rng = np.random.default_rng(32)
    for _ in range(400):
        k = int(rng.integers(1, 9))
        bounds = [int(x) for x in rng.integers(1, 1 << int(rng.integers(1, 17)), size=k)]
        if math.prod(bounds) > TWO32:
            continue
        r0 = int(rng.integers(0, TWO32))
        a, rk = orc.chain(32, bounds, r0)
        value, low = divmod(math.prod(bounds) * r0, TWO32)
        assert rk == low and ref.digits(value, bounds) == a


def test_k1_dice32_is_lemire(orc):
    """One die per 32-bit word is Lemire's method at L = 32 (Sec. 2)."""
    rng = np.random.default_rng(6)
    bounds = np.concatenate([rng.integers(1, 1 << 32, size=300, dtype=np.uint64),
                             rng.integers(1, 7, size=100, dtype=np.uint64),
                             np.array([1, 2, 2**31, 2**31 + 1, 2**32 - 1], dtype=np.uint64)]
                            ).astype(np.uint32)
    err, out = orc.dice32(bounds, 1, seed=99, inst=3)
    assert err == 0
    S = bounds.size
    for g, b in enumerate(bounds):
        x, _ = ref.lemire(32, int(b), _stream_words32(orc, 99, 3, S, g))
        assert out[g] == x


@pytest.mark.parametrize("k,bits", [(2, 16), (3, 10), (4, 8), (8, 4)])
def test_dice32_groups_follow_theorem1(orc, k, bits):
    """Every group of an L = 32 stream is the Theorem 1 chain on the first
    accepted 32-bit word of its attempt sequence; at these widths products
    come near 2^32, so rejections are frequent."""
    rng = np.random.default_rng(100 + k)
    count = 1000 + k - 1
    bounds = rng.integers((1 << bits) // 2, 1 << bits, size=count, dtype=np.uint64).astype(np.uint32)
    err, out = orc.dice32(bounds, k, seed=7, inst=11)
    assert err == 0
    S = -(-count // k)
    rerolled = 0
    for g in range(S):
        b = [int(x) for x in bounds[g * k:(g + 1) * k]]
        for att, r0 in enumerate(_stream_words32(orc, 7, 11, S, g)):
            a, rk = ref.chain(32, b, r0)
            if ref.accept(32, b, rk):
                break
        rerolled += att > 0
        assert list(out[g * k:g * k + len(b)]) == a
    assert np.all(out < bounds)
    if k == 2:
        assert rerolled > S // 20


def test_dice32_edge_cases(orc):
    # product exactly 2^32: threshold 0, the first word always accepted
    err, out = orc.dice32(np.array([2**16, 2**16], dtype=np.uint32), 2, seed=3, inst=0)
    assert err == 0 and list(out) == ref.chain(32, [2**16, 2**16], orc.word32(3, 0, 0))[0]
    assert orc.dice32(np.array([2**16 + 1, 2**16], dtype=np.uint32), 2, 1, 0)[0] == 2
    assert orc.dice32(np.array([5, 0], dtype=np.uint32), 2, 1, 0)[0] == 1
    err, out = orc.dice32(np.zeros(0, dtype=np.uint32), 4, 1, 0)
    assert err == 0 and out.size == 0


def test_dice32_uniform_chi2(orc):
    """Digits of a k = 4 stream of 6-sided dice at L = 32 are uniform."""
    count = 200_000
    err, out = orc.dice32(np.full(count, 6, dtype=np.uint32), 4, seed=17, inst=0)
    assert err == 0
    hist = np.bincount(out, minlength=6)
    stat = float(((hist - count / 6) ** 2 / (count / 6)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 5)


# ---------------------------------------------------------------------------
# Shuffles (Algorithm 4 under the paper's schedules)
# ---------------------------------------------------------------------------

def test_s6_batch_counts(orc):
    s6 = orc.schedule_paper(6)
    for row in golden_rows("s6_batches.txt"):
        n, batches = map(int, row.split()[:2])
        assert orc.count_batches(n, n - 1, s6) == batches


def test_paper_schedules(orc):
    s6 = orc.schedule_paper(6)
    assert s6.segments() == [(2**30, 1, 0), (2**19, 2, 2**60), (2**14, 3, 2**57), (2**11, 4, 2**56),
                             (2**9, 5, 2**55), (6, 6, 2**54)]
    assert s6.tail == 1 and s6.u_tail == 720
    s1 = orc.schedule_paper(1)
    assert orc.count_batches(1000, 999, s1) == 999


def test_worked_shuffles(orc):
    for row in golden_rows("worked_shuffles.txt"):
        head, words, result = [p.split() for p in row.split("|")]
        sched = orc.schedule_paper(6 if head[0] == "s6" else 1)
        n = int(head[1])
        z = np.arange(n, dtype=np.uint64)
        assert orc.shuffle_words(z, sched, [int(w, 16) for w in words]) == 0
        assert list(z) == [int(x) for x in result], row


@pytest.mark.parametrize("max_k", [1, 2, 6])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_shuffle_is_permutation(orc, max_k, dtype):
    sched = orc.schedule_paper(max_k)
    for n in (0, 1, 2, 3, 5, 6, 7, 13, 256, 1000, 10000):
        z = np.arange(n, dtype=dtype)
        assert orc.shuffle(z, sched, seed=42, inst=n) == 0
        assert np.array_equal(np.sort(z), np.arange(n, dtype=dtype))
        if n >= 13:
            assert not np.array_equal(z, np.arange(n, dtype=dtype))


def _dice_for_shuffle(orc, n, sched, seed, inst):
    """Dice of the scheduled shuffle by the big-integer chain: returns the
    sequence j_{n-1}, ..., j_1 that Algorithm 1 consumes."""
    segs = sched.segments()
    batches = []
    i = n
    for thr, k, _ in segs:
        while i > thr:
            batches.append((i, k))
            i -= k
    if sched.tail and i > 1:
        batches.append((i, i - 1))
    S = len(batches)
    js = []
    for s, (i, k) in enumerate(batches):
        bounds = [i - l for l in range(k)]
        att = 0
        while True:
            a, rk = ref.chain(64, bounds, orc.word(seed, inst, att * S + s))
            if ref.accept(64, bounds, rk):
                break
            att += 1
        js.extend(a)
    return js


@pytest.mark.parametrize("max_k,n", [(1, 50), (2, 77), (6, 300), (6, 10000)])
def test_shuffle_is_fisher_yates(orc, max_k, n):
    """The batched shuffle is Algorithm 1 driven by the batch digits: digit
    a_i of the batch at size i serves step i-1, a_2 step i-2, and so on."""
    sched = orc.schedule_paper(max_k)
    z = np.arange(n, dtype=np.uint32)
    assert orc.shuffle(z, sched, seed=17, inst=4) == 0
    js = _dice_for_shuffle(orc, n, sched, 17, 4)
    assert list(z) == ref.fisher_yates(range(n), js)


def test_k1_shuffle_is_lemire_fisher_yates(orc):
    """Unbatched: step i rolls Lemire's method with bound i+1 (Sec. 2)."""
    n = 200
    sched = orc.schedule_paper(1)
    z = np.arange(n, dtype=np.uint64)
    assert orc.shuffle(z, sched, seed=8, inst=1) == 0
    S = n - 1
    js = [ref.lemire(64, i + 1, _stream_words(orc, 8, 1, S, s))[0]
          for s, i in enumerate(range(n - 1, 0, -1))]
    assert list(z) == ref.fisher_yates(range(n), js)


def test_upper_bound_never_changes_output(orc):
    """The bound u of Algorithm 4 only saves work: with every guard replaced
    by the exact product the output is identical."""
    s6 = orc.schedule_paper(6)
    exact = orc.Schedule.from_segments([(t, k, 0) for t, k, _ in s6.segments()], tail=True, u_tail=0)
    for n in (7, 100, 3000, 40000):
        a = np.arange(n, dtype=np.uint32)
        b = a.copy()
        assert orc.shuffle(a, s6, 9, n) == 0
        assert orc.shuffle(b, exact, 9, n) == 0
        assert np.array_equal(a, b)


def test_bad_schedules_rejected(orc):
    z = np.arange(100, dtype=np.uint32)
    # product of 20 dice at n = 100 exceeds 2^64
    bad = orc.Schedule.from_segments([(19, 20, 0)], tail=True, u_tail=0)
    assert orc.shuffle(z, bad, 1, 0) == 2
    # an upper bound smaller than the product it guards
    bad = orc.Schedule.from_segments([(6, 6, 1000)], tail=True, u_tail=720)
    assert orc.shuffle(z, bad, 1, 0) == 1
    # no tail and a last threshold above 1 leaves elements unshuffled
    bad = orc.Schedule.from_segments([(6, 6, 2**54)], tail=False)
    assert orc.shuffle(z, bad, 1, 0) == 1


def _perm_index4(rows):
    # lexicographic rank of each length-4 permutation row
    idx = np.zeros(rows.shape[0], dtype=np.int64)
    fact = [6, 2, 1, 1]
    for p in range(4):
        smaller = (rows[:, p + 1:] < rows[:, p:p + 1]).sum(axis=1)
        idx += smaller * fact[p]
    return idx


@pytest.mark.parametrize("max_k", [6, 1])
def test_chi2_all_24_permutations(orc, max_k):
    """10^7 shuffles of n = 4 (instances 0..10^7-1, seed 42): all 24
    permutations appear, chi-square with 23 dof at alpha = 1e-3."""
    trials = 10_000_000
    data = np.tile(np.arange(4, dtype=np.uint32), trials)
    offsets = np.arange(0, 4 * trials + 1, 4, dtype=np.uint64)
    assert orc.shuffle_batched(data, offsets, orc.schedule_paper(max_k), seed=42) == 0
    hist = np.bincount(_perm_index4(data.reshape(trials, 4)), minlength=24)
    assert hist.size == 24 and hist.min() > 0
    expected = trials / 24
    stat = float(((hist - expected) ** 2 / expected).sum())
    assert stat < chi2.ppf(1 - 1e-3, 23), stat


# ---------------------------------------------------------------------------
# Sampling without replacement (partial Fisher-Yates)
# ---------------------------------------------------------------------------

def test_sample_is_partial_shuffle_tail(orc):
    s6 = orc.schedule_paper(6)
    rng = np.random.default_rng(1)
    for n, m in ((10, 3), (1000, 100), (5000, 1), (70000, 7000), (12, 12), (12, 11), (9, 0)):
        data = rng.integers(0, 2**63, size=n, dtype=np.uint64)
        err, out = orc.sample(data, m, s6, seed=4, inst=n)
        assert err == 0
        z = data.copy()
        assert orc.partial_shuffle(z, m, s6, seed=4, inst=n) == 0
        assert np.array_equal(out, z[::-1][:m])
        assert len(set(out.tolist())) == m


def test_sample_of_n_minus_1_is_full_shuffle(orc):
    s6 = orc.schedule_paper(6)
    for n in (5, 64, 999):
        data = np.arange(n, dtype=np.uint32)
        err, out = orc.sample(data, n - 1, s6, seed=6, inst=0)
        full = data.copy()
        assert orc.shuffle(full, s6, seed=6, inst=0) == 0
        assert err == 0 and np.array_equal(out, full[::-1][:n - 1])


def test_sample_chi2_ordered_pairs(orc):
    """Ordered 2-samples of n = 5: all 20 outcomes equally likely."""
    s6 = orc.schedule_paper(6)
    data = np.arange(5, dtype=np.uint32)
    trials = 200_000
    hist = np.zeros(25, dtype=np.int64)
    for inst in range(trials):
        err, out = orc.sample(data, 2, s6, seed=77, inst=inst)
        hist[int(out[0]) * 5 + int(out[1])] += 1
    diag = hist.reshape(5, 5).diagonal()
    assert diag.sum() == 0
    cells = hist[hist > 0]
    assert cells.size == 20
    stat = float(((cells - trials / 20) ** 2 / (trials / 20)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 19)


def test_dice_group_equals_stream(orc):
    """The single-group entry (used to sample long streams) reproduces the
    whole-stream oracle group by group, short last group included."""
    rng = np.random.default_rng(77)
    for k, count in ((1, 301), (3, 1000), (4, 1003)):
        bounds = rng.integers(1, 1 << 16, size=count, dtype=np.uint32)
        err, out = orc.dice(bounds, k, 9, 2)
        assert err == 0
        S = -(-count // k)
        for g in range(S):
            e, got = orc.dice_group(bounds[g * k:(g + 1) * k], S, g, 9, 2)
            assert e == 0 and np.array_equal(got, out[g * k:(g + 1) * k])


# ---------------------------------------------------------------------------
# The division form (Sec. 2.1; the naive batched shuffle of Appendix A)
# ---------------------------------------------------------------------------

def test_k1_division_dice_is_lemire(orc):
    """One die per group: the division form is Lemire's method (Sec. 2)."""
    rng = np.random.default_rng(6)
    bounds = np.concatenate([rng.integers(1, 1 << 32, size=200, dtype=np.uint64),
                             np.array([1, 2, 2**31 + 1, 2**32 - 1], dtype=np.uint64)]).astype(np.uint32)
    err, out = orc.dice_div(bounds, 1, seed=21, inst=5)
    assert err == 0
    S = bounds.size
    for g, b in enumerate(bounds):
        assert out[g] == ref.lemire(64, int(b), _stream_words(orc, 21, 5, S, g))[0]


@pytest.mark.parametrize("k,bits", [(2, 32), (2, 16), (3, 21), (4, 16), (6, 10)])
def test_division_and_multiply_forms_share_the_value(orc, k, bits):
    """Both forms accept by Lemire's criterion on the same word (the chain's
    leftover is the low half of prod(b) * r, pinned above), so a group reads
    the same words in both and rolls the same value V below prod(b). The
    multiply form writes V with b_1's digit most significant, the division
    form with b_1's digit least significant (V mod b_1 first)."""
    rng = np.random.default_rng(100 + k)
    count = 600 * k + k - 1
    bounds = rng.integers(1, 1 << bits, size=count, dtype=np.uint64).astype(np.uint32)
    if bits == 32:  # rejection-heavy pairs as well
        bounds[: 200] = np.tile(np.array([2**31 + 1, 2**32 - 1], dtype=np.uint32), 100)
    e1, mul = orc.dice(bounds, k, seed=3, inst=9)
    e2, div = orc.dice_div(bounds, k, seed=3, inst=9)
    assert e1 == e2 == 0
    assert np.all(div < bounds)
    for g in range(-(-count // k)):
        b = [int(x) for x in bounds[g * k:(g + 1) * k]]
        a = [int(x) for x in mul[g * k:(g + 1) * k]]
        d = [int(x) for x in div[g * k:(g + 1) * k]]
        assert ref.mixed_radix(a, b) == ref.mixed_radix(d[::-1], b[::-1])
    if k >= 2:  # the forms differ as tuples
        assert not np.array_equal(mul, div)


def test_division_form_product_2_64(orc):
    """Four bounds of 2^16: the product is 2^64, every word is accepted and
    V is the word itself, so the dice are its 16-bit fields, least
    significant first."""
    bounds = np.full(8, 1 << 16, dtype=np.uint32)
    err, out = orc.dice_div(bounds, 4, seed=12, inst=1)
    assert err == 0
    for g in range(2):
        w = orc.word(12, 1, g)
        assert [int(x) for x in out[4 * g:4 * g + 4]] == [(w >> (16 * i)) & 0xFFFF for i in range(4)]


def test_division_form_two_dice_example(orc):
    """Sec. 2.1 with b_1 = b_2 = 6: the pair is the remainder and the
    quotient of one roll of a 36-sided die (all 36 pairs, uniform)."""
    count = 360_000
    err, out = orc.dice_div(np.full(count, 6, dtype=np.uint32), 2, seed=2, inst=0)
    assert err == 0
    pairs = out[0::2].astype(np.int64) + 6 * out[1::2].astype(np.int64)
    e36, big = orc.dice(np.full(count // 2, 36, dtype=np.uint32), 1, seed=2, inst=0)
    assert e36 == 0 and np.array_equal(pairs, big.astype(np.int64))
    hist = np.bincount(pairs, minlength=36)
    stat = float(((hist - count / 72) ** 2 / (count / 72)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 35)


def test_division_edge_cases(orc):
    assert orc.dice_div(np.array([2**32 - 1] * 3, dtype=np.uint32), 3, 1, 0)[0] == 2
    assert orc.dice_div(np.array([5, 0, 7, 9], dtype=np.uint32), 2, 1, 0)[0] == 1
    err, out = orc.dice_div(np.zeros(0, dtype=np.uint32), 3, 1, 0)
    assert err == 0 and out.size == 0
    rng = np.random.default_rng(4)
    bounds = rng.integers(1, 1 << 16, size=1003, dtype=np.uint32)
    err, out = orc.dice_div(bounds, 4, 9, 2)
    S = -(-bounds.size // 4)
    for g in range(S):
        e, got = orc.dice_div_group(bounds[4 * g:4 * g + 4], S, g, 9, 2)
        assert e == 0 and np.array_equal(got, out[4 * g:4 * g + 4])


def _division_dice_for_shuffle(orc, n, seed, inst):
    """Dice of the naive batched shuffle from big integers: batch s at size
    i rolls V below i (i - 1) by Lemire's method on words a*S + s; the die
    for step i-1 is V mod i and the die for step i-2 is V div i (a batch at
    i = 2 keeps one die)."""
    batches = []
    i = n
    while i > 1:
        batches.append((i, min(2, i - 1)))
        i -= 2
    S = len(batches)
    js = []
    for s, (i, k) in enumerate(batches):
        bound = i * (i - 1) if k == 2 else i
        V = ref.lemire(64, bound, _stream_words(orc, seed, inst, S, s))[0]
        js.extend([V % i, V // i] if k == 2 else [V])
    return js


@pytest.mark.parametrize("n", [2, 3, 4, 9, 100, 5001])
def test_naive2_shuffle_is_fisher_yates(orc, n):
    sched = orc.schedule_naive2()
    assert orc.count_batches(n, n - 1, sched) == n // 2
    z = np.arange(n, dtype=np.uint64)
    assert orc.shuffle(z, sched, seed=23, inst=n) == 0
    assert list(z) == ref.fisher_yates(range(n), _division_dice_for_shuffle(orc, n, 23, n))


def test_naive2_chi2_all_24_permutations(orc):
    trials = 2_000_000
    data = np.tile(np.arange(4, dtype=np.uint32), trials)
    offsets = np.arange(0, 4 * trials + 1, 4, dtype=np.uint64)
    assert orc.shuffle_batched(data, offsets, orc.schedule_naive2(), seed=43) == 0
    hist = np.bincount(_perm_index4(data.reshape(trials, 4)), minlength=24)
    assert hist.size == 24 and hist.min() > 0
    stat = float(((hist - trials / 24) ** 2 / (trials / 24)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 23), stat


def test_mixed_form_schedule_and_bad_form(orc):
    """Forms may change from segment to segment; an unknown form is an
    invalid schedule."""
    mixed = orc.Schedule.from_segments([(500, 1, 0), (100, 2, 0), (6, 3, 2**57)], tail=True,
                                       u_tail=720, forms=[0, 1, 0])
    z = np.arange(3000, dtype=np.uint32)
    assert orc.shuffle(z, mixed, 1, 0) == 0
    assert np.array_equal(np.sort(z), np.arange(3000, dtype=np.uint32))
    bad = orc.Schedule.from_segments([(1, 2, 0)], tail=False, forms=[2])
    assert orc.shuffle(np.arange(10, dtype=np.uint32), bad, 1, 0) == 1


# ---------------------------------------------------------------------------
# ChaCha20 words (counter mode), the paper's slow generator
# ---------------------------------------------------------------------------

def test_chacha_known_answers(orc):
    """RFC 8439 Sec. 2.1.1 (quarter round) and Sec. 2.3.2 (block function)."""
    for row in golden_rows("chacha20_rfc8439.txt"):
        kind, rest = row.split(None, 1)
        inp, outp = [[int(x, 16) for x in part.split()] for part in rest.split("|")]
        if kind == "quarter":
            assert orc.chacha_quarter(*inp) == outp
        else:
            assert orc.chacha_block(inp, 20) == outp


def test_chacha_word_layout(orc):
    """Word c is output words 2(c mod 8), 2(c mod 8)+1 of block c/8 of the
    state (constants, key = seed, 64-bit counter, 64-bit nonce = inst)."""
    seed, inst = 0x0123456789ABCDEF, 0xFEDCBA9876543210
    for blk in (0, 1, 2**32 + 5):
        st = [0x61707865, 0x3320646e, 0x79622d32, 0x6b206574, seed & 0xFFFFFFFF, seed >> 32,
              0, 0, 0, 0, 0, 0, blk & 0xFFFFFFFF, blk >> 32, inst & 0xFFFFFFFF, inst >> 32]
        out = orc.chacha_block(st, 20)
        for m in range(8):
            assert orc.word_chacha(seed, inst, 8 * blk + m) == out[2 * m] | (out[2 * m + 1] << 32)


def _chacha_words(orc, seed, inst, S, g):
    a = 0
    while True:
        yield orc.word_chacha(seed, inst, a * S + g)
        a += 1


def test_k1_chacha_dice_is_lemire(orc):
    rng = np.random.default_rng(8)
    bounds = np.concatenate([rng.integers(1, 1 << 32, size=200, dtype=np.uint64),
                             np.array([1, 2, 2**31 + 1, 2**32 - 1], dtype=np.uint64)]).astype(np.uint32)
    err, out = orc.dice_chacha(bounds, 1, seed=31, inst=2)
    assert err == 0
    for g, b in enumerate(bounds):
        assert out[g] == ref.lemire(64, int(b), _chacha_words(orc, 31, 2, bounds.size, g))[0]


@pytest.mark.parametrize("k,bits", [(2, 32), (3, 21), (4, 16)])
def test_chacha_dice_follow_theorem1(orc, k, bits):
    rng = np.random.default_rng(40 + k)
    count = 500 * k + k - 1
    bounds = rng.integers(1 << (bits - 1), 1 << bits, size=count, dtype=np.uint64).astype(np.uint32)
    err, out = orc.dice_chacha(bounds, k, seed=5, inst=8)
    assert err == 0
    S = -(-count // k)
    rerolled = 0
    for g in range(S):
        b = [int(x) for x in bounds[g * k:(g + 1) * k]]
        for att, r0 in enumerate(_chacha_words(orc, 5, 8, S, g)):
            a, rk = ref.chain(64, b, r0)
            if ref.accept(64, b, rk):
                break
        rerolled += att > 0
        assert list(out[g * k:g * k + len(b)]) == a
    if bits == 32:
        assert rerolled > 0


# ---------------------------------------------------------------------------
# Known-threshold specialisations (Algorithm 2) and the KMAX schedule
# ---------------------------------------------------------------------------

def _falling(n, k):
    return math.prod(range(n - k + 1, n + 1))


@pytest.mark.parametrize("kcap", [2, 4, 6, 8])
def test_kmax_schedule_thresholds(orc, kcap):
    """N_k is the largest n whose k-th falling power fits in 2^64 (checked
    with exact integers); k dice run while N_{k+1} < i <= N_k, each segment
    guarded by N_k^(falling k)."""
    s = orc.schedule_kmax(kcap)
    segs = s.segments()
    assert [k for _, k, _ in segs] == list(range(1, kcap + 1)) and s.tail == 1
    for idx, (thr, k, u) in enumerate(segs[:-1]):
        n = thr  # N_{k+1}
        assert _falling(n, k + 1) <= TWO64 < _falling(n + 1, k + 1), (k + 1, n)
        if k > 1:
            top = segs[idx - 1][0]  # N_k
            assert u == _falling(top, k)
    assert segs[-1][0] == kcap - 1


@pytest.mark.parametrize("kcap", [3, 8])
def test_kmax_batches_are_maximal(orc, kcap):
    """Walking the schedule: every batch fits (product <= 2^64) and, above
    the last segment, one more die would not fit or k is at its cap."""
    s = orc.schedule_kmax(kcap)
    segs = s.segments()
    for n in (5, 8, 9, 259, 260, 567, 568, 569, 1627, 1628, 7133, 7134, 65537, 65538, 100000):
        i = n
        for thr, k, _ in segs:
            while i > thr:
                assert _falling(i, k) <= TWO64
                assert k == kcap or _falling(i, k + 1) > TWO64, (n, i, k)
                i -= k
        assert i <= kcap - 1


@pytest.mark.parametrize("n", [2, 9, 300, 2000, 70000])
def test_kmax_shuffle_is_fisher_yates(orc, n):
    sched = orc.schedule_kmax(8)
    z = np.arange(n, dtype=np.uint32)
    assert orc.shuffle(z, sched, seed=29, inst=n) == 0
    assert list(z) == ref.fisher_yates(range(n), _dice_for_shuffle(orc, n, sched, 29, n))


def test_dice_tuple_is_alg3_on_the_tiled_bounds(orc):
    """A fixed tuple (threshold known, Algorithm 2) rolls what Algorithm 3
    rolls on the same bounds written out group by group, short last group
    included."""
    for tup, count in (([4, 6, 8, 20], 4001), ([2**31 + 1, 2**32 - 1], 999), ([6], 500),
                       ([3, 5, 7, 11, 13, 17, 19], 7 * 300 + 3)):
        err, got = orc.dice_tuple(tup, count, seed=14, inst=3)
        tiled = np.resize(np.array(tup, dtype=np.uint32), count)
        e2, want = orc.dice(tiled, len(tup), 14, 3)
        assert err == e2 == 0 and np.array_equal(got, want), tup
        assert np.all(got < tiled)


def test_dice_tuple_product_2_64_and_errors(orc):
    """Four bounds of 2^16: threshold 0 and the dice are the word's 16-bit
    fields, most significant first (Theorem 1's digit order)."""
    err, out = orc.dice_tuple([1 << 16] * 4, 8, seed=12, inst=1)
    assert err == 0
    for g in range(2):
        w = orc.word(12, 1, g)
        assert [int(x) for x in out[4 * g:4 * g + 4]] == [(w >> (48 - 16 * i)) & 0xFFFF for i in range(4)]
    assert orc.dice_tuple([2**32 - 1] * 3, 10, 1, 0)[0] == 2
    assert orc.dice_tuple([5, 0, 3], 10, 1, 0)[0] == 1


# ---------------------------------------------------------------------------
# Shuffles on other word streams: 32-bit halves (L = 32) and ChaCha20
# ---------------------------------------------------------------------------

# batch sizes of Table 2's L = 32 column (n_2, n_3, n_4), exact guards
L32_STEPS = [(20724, 1, 0), (581, 2, 0), (109, 3, 0), (4, 4, 0)]


def _dice_for_shuffle_words(orc, n, sched, L, word):
    """Dice of a scheduled shuffle on the word stream word(c) at width L,
    by the big-integer chain and Lemire's criterion at L."""
    batches = []
    i = n
    for thr, k, _ in sched.segments():
        while i > thr:
            batches.append((i, k))
            i -= k
    if sched.tail and i > 1:
        batches.append((i, i - 1))
    S = len(batches)
    js = []
    for s, (i, k) in enumerate(batches):
        bounds = [i - l for l in range(k)]
        att = 0
        while True:
            a, rk = ref.chain(L, bounds, word(att * S + s))
            if ref.accept(L, bounds, rk):
                break
            att += 1
        js.extend(a)
    return js


@pytest.mark.parametrize("n", [2, 5, 110, 600, 3000, 25000])
def test_l32_shuffle_is_fisher_yates(orc, n):
    sched = orc.Schedule.from_segments(L32_STEPS, tail=True, u_tail=0, words=orc.WORDS_PHILOX32)
    z = np.arange(n, dtype=np.uint32)
    assert orc.shuffle(z, sched, seed=37, inst=n) == 0
    js = _dice_for_shuffle_words(orc, n, sched, 32, lambda c: orc.word32(37, n, c))
    assert list(z) == ref.fisher_yates(range(n), js)


def test_l32_k1_shuffle_is_lemire_at_32(orc):
    n = 300
    sched = orc.Schedule.from_segments([(1, 1, 0)], tail=False, words=orc.WORDS_PHILOX32)
    z = np.arange(n, dtype=np.uint64)
    assert orc.shuffle(z, sched, seed=3, inst=7) == 0
    S = n - 1

    def words(s):
        a = 0
        while True:
            yield orc.word32(3, 7, a * S + s)
            a += 1
    js = [ref.lemire(32, i + 1, words(s))[0] for s, i in enumerate(range(n - 1, 0, -1))]
    assert list(z) == ref.fisher_yates(range(n), js)


@pytest.mark.parametrize("n", [3, 300, 20000])
def test_chacha_shuffle_is_fisher_yates(orc, n):
    s6 = orc.schedule_paper(6)
    sched = orc.Schedule.from_segments(s6.segments(), tail=True, u_tail=720, words=orc.WORDS_CHACHA20)
    z = np.arange(n, dtype=np.uint32)
    assert orc.shuffle(z, sched, seed=38, inst=n) == 0
    js = _dice_for_shuffle_words(orc, n, sched, 64, lambda c: orc.word_chacha(38, n, c))
    assert list(z) == ref.fisher_yates(range(n), js)


def test_word_stream_schedule_checks(orc):
    z = np.arange(30000, dtype=np.uint32)
    # at L = 32 a pair at 30000 elements (product about 9e8) fits, a triple does not
    ok = orc.Schedule.from_segments([(1, 2, 0)], tail=False, words=orc.WORDS_PHILOX32)
    assert orc.shuffle(z.copy(), ok, 1, 0) == 0
    over = orc.Schedule.from_segments([(2, 3, 0)], tail=True, u_tail=0, words=orc.WORDS_PHILOX32)
    assert orc.shuffle(z.copy(), over, 1, 0) == 2
    # the division form needs 64-bit words; unknown streams are invalid
    div32 = orc.Schedule.from_segments([(1, 2, 0)], tail=False, forms=[1], words=orc.WORDS_PHILOX32)
    assert orc.shuffle(z.copy(), div32, 1, 0) == 1
    bad = orc.Schedule.from_segments([(1, 1, 0)], tail=False, words=3)
    assert orc.shuffle(z.copy(), bad, 1, 0) == 1
    # ChaCha words with the division form are fine
    divcc = orc.Schedule.from_segments([(1, 2, 0)], tail=False, forms=[1], words=orc.WORDS_CHACHA20)
    zz = z.copy()
    assert orc.shuffle(zz, divcc, 1, 0) == 0 and np.array_equal(np.sort(zz), z)


@pytest.mark.parametrize("words", ["l32", "chacha"])
def test_word_stream_chi2_all_24_permutations(orc, words):
    if words == "l32":
        sched = orc.Schedule.from_segments(L32_STEPS, tail=True, u_tail=0, words=orc.WORDS_PHILOX32)
    else:
        sched = orc.Schedule.from_segments(orc.schedule_paper(6).segments(), tail=True, u_tail=720,
                                           words=orc.WORDS_CHACHA20)
    trials = 1_000_000
    data = np.tile(np.arange(4, dtype=np.uint32), trials)
    offsets = np.arange(0, 4 * trials + 1, 4, dtype=np.uint64)
    assert orc.shuffle_batched(data, offsets, sched, seed=47) == 0
    hist = np.bincount(_perm_index4(data.reshape(trials, 4)), minlength=24)
    assert hist.size == 24 and hist.min() > 0
    stat = float(((hist - trials / 24) ** 2 / (trials / 24)).sum())
    assert stat < chi2.ppf(1 - 1e-3, 23), stat


def test_stream_group_entries_equal_streams(orc):
    """The single-group entries used for full-size sampling reproduce the
    whole-stream oracles group by group (32-bit words, ChaCha20 words, the
    division form), short last group included."""
    rng = np.random.default_rng(78)
    for k, count in ((1, 301), (2, 1001), (3, 1000)):
        b16 = rng.integers(1, 1 << 16, size=count, dtype=np.uint32)
        b10 = rng.integers(1, 1 << 10, size=count, dtype=np.uint32)
        S = -(-count // k)
        cases = ((orc.dice32, orc.dice32_group, b10), (orc.dice_chacha, orc.dice_chacha_group, b16),
                 (orc.dice_div, orc.dice_div_group, b16))
        for stream, group, bounds in cases:
            err, out = stream(bounds, k, 9, 2)
            assert err == 0
            for g in range(S):
                e, got = group(bounds[g * k:(g + 1) * k], S, g, 9, 2)
                assert e == 0 and np.array_equal(got, out[g * k:(g + 1) * k]), (stream, k, g)


def test_dice_ranges_equal_streams(orc):
    """The group-range entry (whole streams on every host core) writes what
    the whole-stream oracles write, for each stream kind, over uneven
    splits that cut at arbitrary groups, short last group included; ranges
    past the end and empty ranges write nothing; an error in one group is
    reported and leaves the others written."""
    rng = np.random.default_rng(79)
    streams = ((orc.STREAM_MULTIPLY, orc.dice, 16), (orc.STREAM_DIVISION, orc.dice_div, 16),
               (orc.STREAM_CHACHA20, orc.dice_chacha, 16), (orc.STREAM_L32, orc.dice32, 8))
    for kind, whole, bits in streams:
        for k, count in ((1, 997), (2, 1001), (3, 3001), (4, 4003)):
            bounds = rng.integers(1, 1 << (bits if k < 4 else bits // 2), size=count,
                                  dtype=np.uint32)
            err, want = whole(bounds, k, 9, 2)
            assert err == 0
            S = -(-count // k)
            cuts = np.sort(rng.integers(0, S + 1, size=5))
            edges = [0, *cuts.tolist(), S + 7]
            got = np.full(count, 0xFFFFFFFF, np.uint32)
            for g0, g1 in zip(edges[:-1], edges[1:]):
                assert orc.dice_range(kind, bounds, got, k, g0, g1, 9, 2) == 0
            assert np.array_equal(got, want), (kind, k)
            for threads in (1, 3, 8):
                e, got = orc.dice_stream(kind, bounds, k, 9, 2, threads=threads)
                assert e == 0 and np.array_equal(got, want), (kind, k, threads)
    bounds = rng.integers(1, 1 << 16, size=100, dtype=np.uint32)
    bounds[37] = 0
    err, want = orc.dice(bounds, 2, 9, 2)
    assert err == orc.EINVAL
    e, got = orc.dice_stream(orc.STREAM_MULTIPLY, bounds, 2, 9, 2, threads=4)
    assert e == orc.EINVAL
    keep = np.ones(100, bool)
    keep[36:38] = False
    assert np.array_equal(got[keep], want[keep])


def test_threaded_batched_shuffle_equals_batched(orc):
    """shuffle_batched split over threads by shuffle ranges equals the
    single-threaded batch (instances inst_base + q kept)."""
    from paper_2408_06213_amd import workloads

    sizes = workloads.ragged_sizes(300, seed=3)
    off = workloads.csr_offsets(sizes)
    a = workloads.iota_segments(sizes)
    b = a.copy()
    s6 = orc.schedule_paper(6)
    assert orc.shuffle_batched(a, off, s6, 1, 5) == 0
    assert orc.shuffle_batched_threads(b, off, s6, 1, 5, threads=7) == 0
    assert np.array_equal(a, b)
