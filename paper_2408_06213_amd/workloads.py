"""Seeded synthetic inputs for the workloads (no arithmetic of the method).

Both the HIP path and the CPU oracle read these arrays; nothing here rolls a
die or shuffles. numpy's PCG64 generator (``default_rng(seed)``) draws them.

  dice_bounds   -- flat dice stream: bounds uniform in [1, 2^16), u32
  ragged_sizes  -- batch of shuffles: n = floor(16 * 4096^U), U uniform in
                   [0, 1), i.e. log-uniform in [16, 65536)
  csr_offsets   -- CSR offsets of a size list (offsets[0] = 0)
  iota_segments -- payload A[off_q + i] = i for every segment
  serving_requests -- Poisson arrivals of shuffle/sample requests
"""
from __future__ import annotations

import numpy as np


def dice_bounds(count: int, seed: int = 7, low: int = 1, high: int = 1 << 16) -> np.ndarray:
    return np.random.default_rng(seed).integers(low, high, size=count, dtype=np.uint32)


def ragged_sizes(count: int, seed: int = 3, lo: int = 16, hi: int = 65536) -> np.ndarray:
    u = np.random.default_rng(seed).random(count)
    return np.floor(lo * (hi / lo) ** u).astype(np.uint64)


def csr_offsets(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(sizes, dtype=np.uint64), out=off[1:])
    return off


def iota_segments(sizes, dtype=np.uint32) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.int64)
    total = int(sizes.sum())
    starts = np.repeat(np.cumsum(sizes) - sizes, sizes)
    return (np.arange(total, dtype=np.int64) - starts).astype(dtype)


def serving_requests(count: int, rate_per_s: float, seed: int = 5, lo_log2: int = 4,
                     hi_log2: int = 22):
    """Poisson arrivals (exponential gaps, mean 1/rate), each a shuffle or a
    sample (1/2 each) of n log-uniform in [2^lo, 2^hi], m uniform in
    [1, max(1, n // 10)] for samples. Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    n = np.floor(2.0 ** rng.uniform(lo_log2, hi_log2, size=count)).astype(np.int64)
    is_sample = rng.random(count) < 0.5
    m = np.array([int(rng.integers(1, max(1, int(x) // 10) + 1)) for x in n])
    return [dict(t=float(t[i]), kind="sample" if is_sample[i] else "shuffle", n=int(n[i]),
                 m=int(m[i]) if is_sample[i] else int(n[i])) for i in range(count)]
