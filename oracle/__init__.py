"""CPU oracle for batched ranged random integer generation.

TEST INFRASTRUCTURE. Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package. The product
(``paper_2408_06213_amd``) never imports it, and the two share no code: the
only common dependency is the seeded input generator module, which holds none
of the method's arithmetic.

``liboracle.so`` is built from ``brr_oracle.c`` (plain C, gcc) by
:func:`build`; the wrappers below only marshal numpy arrays into it.
``ref`` holds the width-generic big-integer forms used for exhaustive checks.
"""
from __future__ import annotations

import concurrent.futures
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "brr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, EINVAL, EOVERFLOW = 0, 1, 2


def build() -> str:
    """Compile liboracle.so with gcc (plain C, -O2)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", LIB, SRC]
    subprocess.run(cmd, check=True)
    return LIB


FORM_MULTIPLY, FORM_DIVISION = 0, 1
WORDS_PHILOX64, WORDS_PHILOX32, WORDS_CHACHA20 = 0, 1, 2


class Schedule(ctypes.Structure):
    """A batch-size schedule: while more than thr[g] elements remain, roll
    batches of k[g] dice with upper bound u[g] (0 = exact product), their
    dice from Theorem 1 (form 0) or the division form of Sec. 2.1 (form 1);
    then, if ``tail``, one last batch of i-1 dice bounded by ``u_tail``."""

    _fields_ = [
        ("nseg", ctypes.c_uint32),
        ("tail", ctypes.c_uint32),
        ("thr", ctypes.c_uint64 * 16),
        ("k", ctypes.c_uint32 * 16),
        ("u", ctypes.c_uint64 * 16),
        ("u_tail", ctypes.c_uint64),
        ("form", ctypes.c_uint32 * 16),
        ("words", ctypes.c_uint32),
    ]

    def segments(self):
        return [(int(self.thr[g]), int(self.k[g]), int(self.u[g])) for g in range(self.nseg)]

    def forms(self):
        return [int(self.form[g]) for g in range(self.nseg)]

    @classmethod
    def from_segments(cls, segs, tail=True, u_tail=720, forms=None, words=WORDS_PHILOX64):
        s = cls()
        s.words = words
        s.nseg = len(segs)
        for g, (thr, k, u) in enumerate(segs):
            s.thr[g], s.k[g], s.u[g] = thr, k, u
            s.form[g] = forms[g] if forms else FORM_MULTIPLY
        s.tail = 1 if tail else 0
        s.u_tail = u_tail
        return s


def schedule_naive2() -> Schedule:
    """The division-based comparison shuffle of Appendix A: one die per
    batch above 2^32 elements, then batches of two dice in the division form
    while more than one element remains (no separate last batch)."""
    return Schedule.from_segments([(1 << 32, 1, 0), (1, 2, 0)], tail=False,
                                  forms=[FORM_DIVISION, FORM_DIVISION])


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        u64, u32, p = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [p, p, p]
        L.orc_philox4x32_10.restype = None
        L.orc_word.argtypes = [u64, u64, u64]
        L.orc_word.restype = u64
        L.orc_chain.argtypes = [ctypes.c_uint, p, ctypes.c_uint, u64, p]
        L.orc_chain.restype = u64
        L.orc_threshold.argtypes = [ctypes.c_uint, p, ctypes.c_uint, p]
        L.orc_threshold.restype = ctypes.c_int
        L.orc_dice.argtypes = [p, p, u64, ctypes.c_uint, u64, u64]
        L.orc_dice.restype = ctypes.c_int
        L.orc_dice_group.argtypes = [p, ctypes.c_uint, u64, u64, u64, u64, p]
        L.orc_dice_group.restype = ctypes.c_int
        L.orc_dice_div.argtypes = [p, p, u64, ctypes.c_uint, u64, u64]
        L.orc_dice_div.restype = ctypes.c_int
        L.orc_dice_div_group.argtypes = [p, ctypes.c_uint, u64, u64, u64, u64, p]
        L.orc_dice_div_group.restype = ctypes.c_int
        L.orc_chacha_quarter.argtypes = [p, p, p, p]
        L.orc_chacha_quarter.restype = None
        L.orc_chacha_block.argtypes = [p, ctypes.c_uint, p]
        L.orc_chacha_block.restype = None
        L.orc_word_chacha.argtypes = [u64, u64, u64]
        L.orc_word_chacha.restype = u64
        L.orc_dice_chacha.argtypes = [p, p, u64, ctypes.c_uint, u64, u64]
        L.orc_dice_chacha.restype = ctypes.c_int
        L.orc_dice32_group.argtypes = [p, ctypes.c_uint, u64, u64, u64, u64, p]
        L.orc_dice32_group.restype = ctypes.c_int
        L.orc_dice_chacha_group.argtypes = [p, ctypes.c_uint, u64, u64, u64, u64, p]
        L.orc_dice_chacha_group.restype = ctypes.c_int
        L.orc_dice32.argtypes = [p, p, u64, ctypes.c_uint, u64, u64]
        L.orc_dice32.restype = ctypes.c_int
        L.orc_word32.argtypes = [u64, u64, u64]
        L.orc_word32.restype = ctypes.c_uint32
        L.orc_dice_const.argtypes = [u32, p, u64, ctypes.c_uint, u64, u64]
        L.orc_dice_const.restype = ctypes.c_int
        L.orc_schedule_kmax.argtypes = [ctypes.c_uint, ctypes.POINTER(Schedule)]
        L.orc_schedule_kmax.restype = ctypes.c_int
        L.orc_dice_tuple.argtypes = [p, ctypes.c_uint, p, u64, u64, u64]
        L.orc_dice_tuple.restype = ctypes.c_int
        L.orc_schedule_paper.argtypes = [ctypes.c_int, ctypes.POINTER(Schedule)]
        L.orc_schedule_paper.restype = ctypes.c_int
        L.orc_count_batches.argtypes = [u64, u64, ctypes.POINTER(Schedule)]
        L.orc_count_batches.restype = u64
        L.orc_shuffle.argtypes = [p, u64, ctypes.c_uint, ctypes.POINTER(Schedule), u64, u64]
        L.orc_shuffle.restype = ctypes.c_int
        L.orc_shuffle_words.argtypes = [p, u64, ctypes.c_uint, ctypes.POINTER(Schedule), p, u64]
        L.orc_shuffle_words.restype = ctypes.c_int
        L.orc_shuffle_batched.argtypes = [p, p, u64, ctypes.c_uint, ctypes.POINTER(Schedule), u64, u64]
        L.orc_shuffle_batched.restype = ctypes.c_int
        L.orc_partial_shuffle.argtypes = [p, u64, u64, ctypes.c_uint, ctypes.POINTER(Schedule), u64, u64]
        L.orc_partial_shuffle.restype = ctypes.c_int
        L.orc_sample.argtypes = [p, u64, u64, ctypes.c_uint, p, ctypes.POINTER(Schedule), u64, u64]
        L.orc_sample.restype = ctypes.c_int
        L.orc_dice_range.argtypes = [ctypes.c_uint, p, p, u64, ctypes.c_uint, u64, u64, u64, u64]
        L.orc_dice_range.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------
# thin wrappers
# ----------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def word(seed: int, inst: int, c: int) -> int:
    return int(lib().orc_word(seed, inst, c))


def chain(L: int, bounds, r0: int):
    b = np.asarray(bounds, dtype=np.uint64).copy()
    a = np.zeros(max(1, len(b)), dtype=np.uint64)
    r = lib().orc_chain(L, _ptr(b), len(b), r0, _ptr(a))
    return [int(x) for x in a[: len(b)]], int(r)


def threshold(L: int, bounds):
    b = np.asarray(bounds, dtype=np.uint64).copy()
    t = np.zeros(1, dtype=np.uint64)
    err = lib().orc_threshold(L, _ptr(b), len(b), _ptr(t))
    return err, int(t[0])


def dice(bounds: np.ndarray, k: int, seed: int, inst: int = 0):
    bounds = np.ascontiguousarray(bounds, dtype=np.uint32)
    out = np.zeros(bounds.size, dtype=np.uint32)
    err = lib().orc_dice(_ptr(bounds), _ptr(out), bounds.size, k, seed, inst)
    return err, out


def dice_div(bounds: np.ndarray, k: int, seed: int, inst: int = 0):
    """The dice stream in the division form (Sec. 2.1): per group one value
    below the product of its bounds, digits as successive remainders."""
    bounds = np.ascontiguousarray(bounds, dtype=np.uint32)
    out = np.zeros(bounds.size, dtype=np.uint32)
    err = lib().orc_dice_div(_ptr(bounds), _ptr(out), bounds.size, k, seed, inst)
    return err, out


def dice_div_group(group_bounds, S: int, s: int, seed: int, inst: int = 0):
    b = np.ascontiguousarray(group_bounds, dtype=np.uint32)
    out = np.zeros(b.size, dtype=np.uint32)
    err = lib().orc_dice_div_group(_ptr(b), b.size, S, s, seed, inst, _ptr(out))
    return err, out


def chacha_quarter(a: int, b: int, c: int, d: int):
    v = [np.array([x], dtype=np.uint32) for x in (a, b, c, d)]
    lib().orc_chacha_quarter(*[_ptr(x) for x in v])
    return [int(x[0]) for x in v]


def chacha_block(state, rounds: int = 20):
    st = np.ascontiguousarray(state, dtype=np.uint32)
    out = np.zeros(16, dtype=np.uint32)
    lib().orc_chacha_block(_ptr(st), rounds, _ptr(out))
    return [int(x) for x in out]


def word_chacha(seed: int, inst: int, c: int) -> int:
    return int(lib().orc_word_chacha(seed, inst, c))


def dice_chacha(bounds: np.ndarray, k: int, seed: int, inst: int = 0):
    """The dice stream with ChaCha20 words (counter mode) in place of Philox."""
    bounds = np.ascontiguousarray(bounds, dtype=np.uint32)
    out = np.zeros(bounds.size, dtype=np.uint32)
    err = lib().orc_dice_chacha(_ptr(bounds), _ptr(out), bounds.size, k, seed, inst)
    return err, out


def dice32(bounds: np.ndarray, k: int, seed: int, inst: int = 0):
    """The dice stream at word width 32 (32-bit halves of the 64-bit words)."""
    bounds = np.ascontiguousarray(bounds, dtype=np.uint32)
    out = np.zeros(bounds.size, dtype=np.uint32)
    err = lib().orc_dice32(_ptr(bounds), _ptr(out), bounds.size, k, seed, inst)
    return err, out


def word32(seed: int, inst: int, c: int) -> int:
    return int(lib().orc_word32(seed, inst, c))


def dice_group(group_bounds, S: int, s: int, seed: int, inst: int = 0):
    """Dice of group s (of S) alone; group_bounds are its kk bounds."""
    b = np.ascontiguousarray(group_bounds, dtype=np.uint32)
    out = np.zeros(b.size, dtype=np.uint32)
    err = lib().orc_dice_group(_ptr(b), b.size, S, s, seed, inst, _ptr(out))
    return err, out


def dice32_group(group_bounds, S: int, s: int, seed: int, inst: int = 0):
    b = np.ascontiguousarray(group_bounds, dtype=np.uint32)
    out = np.zeros(b.size, dtype=np.uint32)
    err = lib().orc_dice32_group(_ptr(b), b.size, S, s, seed, inst, _ptr(out))
    return err, out


def dice_chacha_group(group_bounds, S: int, s: int, seed: int, inst: int = 0):
    b = np.ascontiguousarray(group_bounds, dtype=np.uint32)
    out = np.zeros(b.size, dtype=np.uint32)
    err = lib().orc_dice_chacha_group(_ptr(b), b.size, S, s, seed, inst, _ptr(out))
    return err, out


def dice_const(bound: int, count: int, k: int, seed: int, inst: int = 0):
    out = np.zeros(count, dtype=np.uint32)
    err = lib().orc_dice_const(bound, _ptr(out), count, k, seed, inst)
    return err, out


def schedule_paper(max_k: int) -> Schedule:
    s = Schedule()
    err = lib().orc_schedule_paper(max_k, ctypes.byref(s))
    if err:
        raise ValueError(f"no paper schedule for max_k={max_k}")
    return s


def schedule_kmax(kcap: int) -> Schedule:
    """The greedy largest-batch schedule with at most kcap dice per batch."""
    s = Schedule()
    if lib().orc_schedule_kmax(kcap, ctypes.byref(s)):
        raise ValueError(f"no KMAX schedule for kcap={kcap}")
    return s


def dice_tuple(tuple_bounds, count: int, seed: int, inst: int = 0):
    """Algorithm 2 for a fixed tuple of bounds: out[j] in [0, tuple[j mod k])."""
    t = np.ascontiguousarray(tuple_bounds, dtype=np.uint32)
    out = np.zeros(count, dtype=np.uint32)
    err = lib().orc_dice_tuple(_ptr(t), t.size, _ptr(out), count, seed, inst)
    return err, out


def count_batches(n: int, steps: int, sched: Schedule) -> int:
    return int(lib().orc_count_batches(n, steps, ctypes.byref(sched)))


def shuffle(data: np.ndarray, sched: Schedule, seed: int, inst: int = 0):
    """In-place scheduled batched Fisher-Yates shuffle of a u32/u64 array."""
    assert data.dtype in (np.uint32, np.uint64)
    return lib().orc_shuffle(_ptr(data), data.size, data.itemsize, ctypes.byref(sched), seed, inst)


def shuffle_words(data: np.ndarray, sched: Schedule, words):
    w = np.asarray(words, dtype=np.uint64).copy()
    return lib().orc_shuffle_words(_ptr(data), data.size, data.itemsize, ctypes.byref(sched),
                                   _ptr(w), w.size)


def shuffle_batched(data: np.ndarray, offsets: np.ndarray, sched: Schedule, seed: int,
                    inst_base: int = 0):
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    return lib().orc_shuffle_batched(_ptr(data), _ptr(offsets), offsets.size - 1, data.itemsize,
                                     ctypes.byref(sched), seed, inst_base)


def partial_shuffle(data: np.ndarray, m: int, sched: Schedule, seed: int, inst: int = 0):
    return lib().orc_partial_shuffle(_ptr(data), data.size, m, data.itemsize, ctypes.byref(sched),
                                     seed, inst)


def sample(data: np.ndarray, m: int, sched: Schedule, seed: int, inst: int = 0):
    out = np.zeros(m, dtype=data.dtype)
    err = lib().orc_sample(_ptr(data), data.size, m, data.itemsize, _ptr(out), ctypes.byref(sched),
                           seed, inst)
    return err, out


# ----------------------------------------------------------------------------
# whole streams and batches on every host core
# ----------------------------------------------------------------------------

STREAM_MULTIPLY, STREAM_DIVISION, STREAM_CHACHA20, STREAM_L32 = 0, 1, 2, 3


def host_threads() -> int:
    """Host threads the process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _split(total: int, parts: int):
    parts = max(1, min(parts, total)) if total else 1
    edges = [total * i // parts for i in range(parts + 1)]
    return list(zip(edges[:-1], edges[1:]))


def dice_range(kind: int, bounds: np.ndarray, out: np.ndarray, k: int, g0: int, g1: int,
               seed: int, inst: int = 0) -> int:
    """Groups g0..g1-1 of the stream of ``kind`` (STREAM_*) into ``out``."""
    return lib().orc_dice_range(kind, _ptr(bounds), _ptr(out), bounds.size, k, g0, g1, seed, inst)


def dice_stream(kind: int, bounds: np.ndarray, k: int, seed: int, inst: int = 0,
                threads: int | None = None):
    """The whole dice stream of ``kind`` (the output of dice, dice_div,
    dice_chacha or dice32), its group range split over ``threads`` host
    threads (default: every core this process may use). Returns (err, out)."""
    bounds = np.ascontiguousarray(bounds, dtype=np.uint32)
    out = np.zeros(bounds.size, dtype=np.uint32)
    S = -(-bounds.size // k) if k else 0
    threads = threads or host_threads()
    lib()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        errs = list(ex.map(lambda r: dice_range(kind, bounds, out, k, r[0], r[1], seed, inst),
                           _split(S, threads)))
    return next((e for e in errs if e), OK), out


def shuffle_batched_threads(data: np.ndarray, offsets: np.ndarray, sched: Schedule, seed: int,
                            inst_base: int = 0, threads: int | None = None) -> int:
    """shuffle_batched with its shuffles split over ``threads`` host threads
    (contiguous ranges of shuffles; shuffle q keeps instance inst_base + q)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    count = offsets.size - 1
    threads = threads or host_threads()
    L = lib()

    def part(r):
        q0, q1 = r
        op = offsets.ctypes.data + 8 * q0
        return L.orc_shuffle_batched(_ptr(data), ctypes.c_void_p(op), q1 - q0, data.itemsize,
                                     ctypes.byref(sched), seed, inst_base + q0)

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        errs = list(ex.map(part, _split(count, threads)))
    return next((e for e in errs if e), OK)
