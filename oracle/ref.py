"""Width-generic big-integer forms of the paper's definitions (L-bit words).

TEST INFRASTRUCTURE (part of the oracle). Pure Python integers, so these are
exact at any word width L and only meant for small cases: exhaustive
enumeration at L = 4..16 and spot checks at L = 64.

Each function follows one passage of Brackett-Rozinsky and Lemire,
"Batched Ranged Random Integer Generation":
  full_mul      -- the full-width multiply of Sec. 1.1
  lemire        -- Lemire's single bounded roll and its criterion, Sec. 2
  mixed_radix   -- the value of a mixed-radix digit tuple, Sec. 3
  digits        -- digits by successive division by b_k, ..., b_1, Sec. 3
  chain         -- the multiply chain of Theorem 1, Sec. 4
  accept        -- Lemire's criterion on the batch leftover, Theorem 1
"""
from __future__ import annotations

from collections import Counter
from math import prod


def full_mul(L: int, b: int, r: int):
    """b (x) r = (x, y) with 2^L x + y = b r and 0 <= y < 2^L."""
    return divmod(b * r, 1 << L)


def lemire(L: int, b: int, words):
    """Lemire's method: (x, y) = b (x) r; accept x when y >= 2^L mod b, only
    computing that threshold when y < b. ``words`` yields fresh L-bit words.
    Returns (x, number of words used)."""
    used = 0
    for r in words:
        used += 1
        x, y = full_mul(L, b, r)
        if y >= b:
            return x, used
        t = (1 << L) % b  # the C idiom -b % b computes the same value
        if y >= t:
            return x, used
    raise RuntimeError("word source exhausted")


def chain(L: int, bounds, r0: int):
    """(a_i, r_i) = b_i (x) r_{i-1} for i = 1..k; returns ([a_1..a_k], r_k)."""
    a, r = [], r0
    for b in bounds:
        ai, r = full_mul(L, b, r)
        a.append(ai)
    return a, r


def threshold(L: int, bounds) -> int:
    return (1 << L) % prod(bounds)


def accept(L: int, bounds, rk: int) -> bool:
    return rk >= threshold(L, bounds)


def mixed_radix(a, bounds) -> int:
    """Value of digits (a_1..a_k), a_1 most significant, in base (b_1..b_k)."""
    v = 0
    for ai, bi in zip(a, bounds):
        v = v * bi + ai
    return v


def digits(v: int, bounds):
    """Mixed-radix digits of v < prod(bounds) by successive remainders of
    quotients, dividing by b_k first."""
    out = []
    for b in reversed(bounds):
        v, d = divmod(v, b)
        out.append(d)
    assert v == 0
    return list(reversed(out))


def enumerate_all(L: int, bounds):
    """Runs the Theorem 1 chain on every L-bit word. Returns (Counter of
    accepted digit tuples, number of rejected words)."""
    counts, rejects = Counter(), 0
    t = threshold(L, bounds)
    for r0 in range(1 << L):
        a, rk = chain(L, bounds, r0)
        if rk >= t:
            counts[tuple(a)] += 1
        else:
            rejects += 1
    return counts, rejects


def fisher_yates(arr, dice):
    """Algorithm 1 with the dice given: dice[idx] is j for i = n-1-idx."""
    z = list(arr)
    n = len(z)
    for idx, i in enumerate(range(n - 1, 0, -1)):
        j = dice[idx]
        assert 0 <= j <= i
        z[i], z[j] = z[j], z[i]
    return z
