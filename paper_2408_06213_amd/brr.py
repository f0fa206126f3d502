"""Thin ctypes binding of libbrr (include/brr.h), same names as the C ABI.

Argument marshalling only: every step of every operation runs in the HIP
kernels of libbrr.so. Device buffers are passed as torch tensors (their
data_ptr) or as raw integer addresses; streams default to torch's current
stream on the current device. There is no fallback: importing this module
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbrr.so")

BRR_OK, BRR_EINVAL, BRR_EOVERFLOW, BRR_ENOMEM, BRR_EHIP, BRR_EDEVICE = range(6)
BRR_MAX_STEPS = 16
BRR_MAX_K = 20

# every symbol include/brr.h declares
EXPORTS = (
    "brr_schedule_paper", "brr_schedule_batches", "brr_schedule_check",
    "brr_schedule_check_upto", "brr_shuffle_noalloc", "brr_scratch_bytes", "brr_plan_captures",
    "brr_release_scratch",
    "brr_dice",
    "brr_dice_const", "brr_shuffle", "brr_plan_create", "brr_plan_destroy",
    "brr_plan_get_mapping", "brr_plan_set_mapping", "brr_shuffle_batched", "brr_sample",
    "brr_sync_status", "brr_strerror", "brr_cost_per_die", "brr_cost_thresholds",
    "brr_schedule_from_costs", "brr_dice_autotune", "brr_plan_autotune", "brr_plan_get_schedule",
    "brr_server_create", "brr_server_submit", "brr_server_wait", "brr_server_drain",
    "brr_server_get_stats", "brr_server_reset_stats", "brr_server_session_counter",
    "brr_server_destroy", "brr_mlp_create", "brr_mlp_destroy", "brr_mlp_num_params",
    "brr_mlp_get_params", "brr_mlp_set_params", "brr_mlp_get_grads", "brr_mlp_forward",
    "brr_mlp_backward", "brr_mlp_adam_step", "brr_mlp_train", "brr_plan_features",
    "brr_plan_autotune_learned", "brr_probe_chain_rate", "brr_probe_copy_rate", "brr_dice32", "brr_dice_div",
    "brr_schedule_naive2", "brr_dice_chacha", "brr_dice_tuple", "brr_schedule_kmax",
)
BRR_PLAN_FEATURES = 16
BRR_REQ_SHUFFLE, BRR_REQ_SAMPLE = 1, 2


class BrrError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {brr_strerror(status)} (status {status})")


BRR_FORM_MULTIPLY, BRR_FORM_DIVISION = 0, 1
BRR_WORDS_PHILOX64, BRR_WORDS_PHILOX32, BRR_WORDS_CHACHA20 = 0, 1, 2


class brr_step(ctypes.Structure):
    _fields_ = [("n_above", ctypes.c_uint64), ("k", ctypes.c_uint32),
                ("form", ctypes.c_uint32), ("u0", ctypes.c_uint64)]


class brr_schedule(ctypes.Structure):
    _fields_ = [("nsteps", ctypes.c_uint32), ("tail", ctypes.c_uint32),
                ("u_tail", ctypes.c_uint64), ("step", brr_step * BRR_MAX_STEPS),
                ("words", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def steps(self):
        return [(int(s.n_above), int(s.k), int(s.u0)) for s in self.step[: self.nsteps]]

    def forms(self):
        return [int(s.form) for s in self.step[: self.nsteps]]

    @classmethod
    def from_steps(cls, steps, tail=True, u_tail=720, forms=None, words=0):
        s = cls()
        s.words = words
        s.nsteps = len(steps)
        for g, (above, k, u0) in enumerate(steps):
            s.step[g].n_above, s.step[g].k, s.step[g].u0 = above, k, u0
            s.step[g].form = forms[g] if forms else BRR_FORM_MULTIPLY
        s.tail = 1 if tail else 0
        s.u_tail = u_tail
        return s


class brr_mapping(ctypes.Structure):
    _fields_ = [("lane_max", ctypes.c_uint32), ("wave_max", ctypes.c_uint32),
                ("wg_threads", ctypes.c_uint32), ("use_graph", ctypes.c_uint32)]


class brr_tune_report(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_uint32), ("ms_best", ctypes.c_float),
                ("ms_default", ctypes.c_float), ("schedule", brr_schedule),
                ("mapping", brr_mapping)]


class brr_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("nstreams", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("schedule", ctypes.POINTER(brr_schedule))]


class brr_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("elem_bytes", ctypes.c_uint32),
                ("session", ctypes.c_uint64), ("d_data", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("m", ctypes.c_uint64), ("d_out", ctypes.c_void_p)]


class brr_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("elements", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("mean_us", ctypes.c_double), ("max_us", ctypes.c_double),
                ("wall_s", ctypes.c_double), ("requests_per_s", ctypes.c_double),
                ("elements_per_s", ctypes.c_double), ("peak_inflight", ctypes.c_uint32),
                ("peak_footprint", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # torch ships its own HIP runtime library. Loaded first, it is the one
    # libbrr binds to (same soname), so the library and the device memory
    # and streams torch hands it share one runtime; loaded the other way
    # round, the process would hold two runtimes and the library's could not
    # use the device.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    u64, u32, p, st = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
    sched_p = ctypes.POINTER(brr_schedule)
    sig = {
        "brr_schedule_paper": (st, [ctypes.c_int, sched_p]),
        "brr_schedule_naive2": (st, [sched_p]),
        "brr_schedule_kmax": (st, [u32, sched_p]),
        "brr_dice_tuple": (st, [p, u32, p, u64, u64, u64, p]),
        "brr_schedule_batches": (u64, [sched_p, u64, u64]),
        "brr_schedule_check": (st, [sched_p, u64]),
        "brr_schedule_check_upto": (st, [sched_p, u64]),
        "brr_dice": (st, [p, p, u64, u32, u64, u64, p]),
        "brr_dice_const": (st, [u32, p, u64, u32, u64, u64, p]),
        "brr_dice32": (st, [p, p, u64, u32, u64, u64, p]),
        "brr_dice_div": (st, [p, p, u64, u32, u64, u64, p]),
        "brr_dice_chacha": (st, [p, p, u64, u32, u64, u64, p]),
        "brr_shuffle": (st, [p, u64, u32, sched_p, u64, u64, p]),
        "brr_shuffle_noalloc": (st, [p, u64, u32, sched_p, u64, u64, p]),
        "brr_scratch_bytes": (u64, [u64, u64, u32]),
        "brr_release_scratch": (st, []),
        "brr_plan_create": (st, [ctypes.POINTER(p), p, u64, u32, sched_p]),
        "brr_plan_destroy": (None, [p]),
        "brr_plan_captures": (u32, [p]),
        "brr_plan_get_mapping": (st, [p, ctypes.POINTER(brr_mapping)]),
        "brr_plan_set_mapping": (st, [p, ctypes.POINTER(brr_mapping)]),
        "brr_shuffle_batched": (st, [p, p, u64, u32, p, u64, u64, p]),
        "brr_sample": (st, [p, u64, u64, u32, p, sched_p, u64, u64, p]),
        "brr_sync_status": (st, [p]),
        "brr_cost_per_die": (ctypes.c_double, [u64, u32, u32, ctypes.c_double, ctypes.c_double]),
        "brr_cost_thresholds": (st, [u32, u32, ctypes.c_double, ctypes.c_double, p]),
        "brr_schedule_from_costs": (st, [u32, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                         sched_p]),
        "brr_strerror": (ctypes.c_char_p, [st]),
        "brr_dice_autotune": (st, [u32, u64, p, ctypes.POINTER(u32), p]),
        "brr_plan_autotune": (st, [p, p, p, u64, u64, p, ctypes.POINTER(brr_tune_report)]),
        "brr_plan_get_schedule": (st, [p, sched_p]),
        "brr_server_create": (st, [ctypes.POINTER(p), ctypes.POINTER(brr_server_config)]),
        "brr_server_submit": (st, [p, ctypes.POINTER(brr_request), ctypes.POINTER(u64)]),
        "brr_server_wait": (st, [p, u64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
        "brr_server_drain": (st, [p, ctypes.c_double]),
        "brr_server_get_stats": (st, [p, ctypes.POINTER(brr_server_stats)]),
        "brr_server_reset_stats": (st, [p]),
        "brr_server_session_counter": (st, [p, u64, ctypes.POINTER(u64)]),
        "brr_server_destroy": (None, [p]),
        "brr_mlp_create": (st, [ctypes.POINTER(p), u32, u32, u64]),
        "brr_mlp_destroy": (None, [p]),
        "brr_mlp_num_params": (u64, [p]),
        "brr_mlp_get_params": (st, [p, p]),
        "brr_mlp_set_params": (st, [p, p]),
        "brr_mlp_get_grads": (st, [p, p]),
        "brr_mlp_forward": (st, [p, p, u32, p, p]),
        "brr_mlp_backward": (st, [p, p, p, u32, p, p]),
        "brr_mlp_adam_step": (st, [p, ctypes.c_float, p]),
        "brr_mlp_train": (st, [p, p, p, u32, u32, ctypes.c_float, ctypes.POINTER(ctypes.c_float), p]),
        "brr_plan_features": (st, [p, u64, u32, sched_p, u32, p]),
        "brr_plan_autotune_learned": (st, [p, p, u32, p, p, u64, u64, p,
                                           ctypes.POINTER(brr_tune_report)]),
        "brr_probe_chain_rate": (st, [u32, ctypes.POINTER(ctypes.c_double)]),
        "brr_probe_copy_rate": (st, [p, p, u64, u32, p, ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def _addr(x):
    """Device address of a tensor (data_ptr) or an integer address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _sched(s):
    return ctypes.byref(s) if s is not None else None


def check(status: int, what: str = "brr") -> None:
    if status != BRR_OK:
        raise BrrError(status, what)


def brr_strerror(status: int) -> str:
    return lib.brr_strerror(status).decode()


def brr_schedule_paper(max_k: int) -> brr_schedule:
    s = brr_schedule()
    check(lib.brr_schedule_paper(max_k, ctypes.byref(s)), "brr_schedule_paper")
    return s


def brr_schedule_kmax(kcap: int) -> brr_schedule:
    s = brr_schedule()
    check(lib.brr_schedule_kmax(kcap, ctypes.byref(s)), "brr_schedule_kmax")
    return s


def brr_dice_tuple(bounds_tuple, out, count: int, seed: int, inst: int = 0, stream=None) -> int:
    t = (ctypes.c_uint32 * len(bounds_tuple))(*[int(x) for x in bounds_tuple])
    return lib.brr_dice_tuple(t, len(bounds_tuple), _addr(out), count, seed, inst, _stream(stream))


def brr_schedule_naive2() -> brr_schedule:
    s = brr_schedule()
    check(lib.brr_schedule_naive2(ctypes.byref(s)), "brr_schedule_naive2")
    return s


def brr_schedule_batches(sched: brr_schedule, n: int, steps: int) -> int:
    return int(lib.brr_schedule_batches(ctypes.byref(sched), n, steps))


def brr_schedule_check(sched: brr_schedule, n: int) -> int:
    return lib.brr_schedule_check(ctypes.byref(sched), n)


def brr_schedule_check_upto(sched: brr_schedule, max_n: int) -> int:
    return lib.brr_schedule_check_upto(ctypes.byref(sched), max_n)


def brr_cost_per_die(n: int, k: int, L: int = 64, c_rng: float = 2.0, c_div: float = 16.0) -> float:
    return float(lib.brr_cost_per_die(n, k, L, c_rng, c_div))


def brr_cost_thresholds(L: int, kmax: int, c_rng: float = 2.0, c_div: float = 16.0):
    out = (ctypes.c_uint64 * (kmax + 1))()
    check(lib.brr_cost_thresholds(L, kmax, c_rng, c_div, out), "brr_cost_thresholds")
    return {k: int(out[k]) for k in range(2, kmax + 1)}


BRR_COSTS_POW2, BRR_COSTS_SMOOTH, BRR_COSTS_L32 = 1, 2, 4


def brr_schedule_from_costs(kmax: int, c_rng: float = 2.0, c_div: float = 16.0,
                            pow2: bool = True, smooth: bool = False,
                            l32: bool = False) -> brr_schedule:
    s = brr_schedule()
    flags = ((BRR_COSTS_POW2 if pow2 else 0) | (BRR_COSTS_SMOOTH if smooth else 0)
             | (BRR_COSTS_L32 if l32 else 0))
    check(lib.brr_schedule_from_costs(kmax, c_rng, c_div, flags, ctypes.byref(s)),
          "brr_schedule_from_costs")
    return s


def brr_dice(bounds, out, count: int, k: int, seed: int, inst: int = 0, stream=None) -> int:
    return lib.brr_dice(_addr(bounds), _addr(out), count, k, seed, inst, _stream(stream))


def brr_dice32(bounds, out, count: int, k: int, seed: int, inst: int = 0, stream=None) -> int:
    return lib.brr_dice32(_addr(bounds), _addr(out), count, k, seed, inst, _stream(stream))


def brr_dice_div(bounds, out, count: int, k: int, seed: int, inst: int = 0, stream=None) -> int:
    return lib.brr_dice_div(_addr(bounds), _addr(out), count, k, seed, inst, _stream(stream))


def brr_dice_chacha(bounds, out, count: int, k: int, seed: int, inst: int = 0, stream=None) -> int:
    return lib.brr_dice_chacha(_addr(bounds), _addr(out), count, k, seed, inst, _stream(stream))


def brr_dice_const(bound: int, out, count: int, k: int, seed: int, inst: int = 0,
                   stream=None) -> int:
    return lib.brr_dice_const(bound, _addr(out), count, k, seed, inst, _stream(stream))


def brr_shuffle(data, n: int, elem_bytes: int, sched=None, seed: int = 0, inst: int = 0,
                stream=None) -> int:
    return lib.brr_shuffle(_addr(data), n, elem_bytes, _sched(sched), seed, inst, _stream(stream))


def brr_shuffle_noalloc(data, n: int, elem_bytes: int, sched=None, seed: int = 0, inst: int = 0,
                        stream=None) -> int:
    return lib.brr_shuffle_noalloc(_addr(data), n, elem_bytes, _sched(sched), seed, inst,
                                   _stream(stream))


def brr_scratch_bytes(n: int, m: int, elem_bytes: int) -> int:
    return int(lib.brr_scratch_bytes(n, m, elem_bytes))


def brr_release_scratch() -> int:
    return lib.brr_release_scratch()


def brr_sample(data, n: int, m: int, elem_bytes: int, out, sched=None, seed: int = 0,
               inst: int = 0, stream=None) -> int:
    return lib.brr_sample(_addr(data), n, m, elem_bytes, _addr(out), _sched(sched), seed, inst,
                          _stream(stream))


class Plan:
    """Owns a brr_plan* (brr_plan_create / brr_plan_destroy)."""

    def __init__(self, h_offsets, elem_bytes: int, sched=None):
        import numpy as np

        off = np.ascontiguousarray(h_offsets, dtype=np.uint64)
        self.count = off.size - 1
        self.elem_bytes = elem_bytes
        self.ptr = ctypes.c_void_p()
        check(lib.brr_plan_create(ctypes.byref(self.ptr), off.ctypes.data_as(ctypes.c_void_p),
                                  self.count, elem_bytes, _sched(sched)), "brr_plan_create")

    def mapping(self) -> brr_mapping:
        m = brr_mapping()
        check(lib.brr_plan_get_mapping(self.ptr, ctypes.byref(m)), "brr_plan_get_mapping")
        return m

    def set_mapping(self, m: brr_mapping) -> int:
        return lib.brr_plan_set_mapping(self.ptr, ctypes.byref(m))

    def schedule(self) -> brr_schedule:
        out = brr_schedule()
        check(lib.brr_plan_get_schedule(self.ptr, ctypes.byref(out)), "brr_plan_get_schedule")
        return out

    def captures(self) -> int:
        return int(lib.brr_plan_captures(self.ptr))

    def autotune(self, data, d_offsets, seed: int = 0, inst_base: int = 0,
                 stream=None) -> brr_tune_report:
        rep = brr_tune_report()
        check(lib.brr_plan_autotune(self.ptr, _addr(data), _addr(d_offsets), seed, inst_base,
                                    _stream(stream), ctypes.byref(rep)), "brr_plan_autotune")
        return rep

    def close(self):
        if self.ptr:
            lib.brr_plan_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def brr_plan_create(h_offsets, elem_bytes: int, sched=None) -> Plan:
    return Plan(h_offsets, elem_bytes, sched)


def brr_plan_destroy(plan: Plan) -> None:
    plan.close()


def brr_shuffle_batched(data, d_offsets, count: int, elem_bytes: int, plan=None, seed: int = 0,
                        inst_base: int = 0, stream=None) -> int:
    pp = plan.ptr if plan is not None else None
    return lib.brr_shuffle_batched(_addr(data), _addr(d_offsets), count, elem_bytes, pp, seed,
                                   inst_base, _stream(stream))


def brr_dice_autotune(max_bound: int, count: int, stream=None, with_times: bool = False):
    k = ctypes.c_uint32()
    times = (ctypes.c_float * 9)() if with_times else None
    check(lib.brr_dice_autotune(max_bound, count, _stream(stream), ctypes.byref(k), times),
          "brr_dice_autotune")
    if with_times:
        return int(k.value), {i: float(times[i]) for i in range(1, 9) if times[i] > 0}
    return int(k.value)


def brr_plan_autotune(plan: Plan, data, d_offsets, seed: int = 0, inst_base: int = 0,
                      stream=None) -> brr_tune_report:
    return plan.autotune(data, d_offsets, seed, inst_base, stream)


def brr_plan_get_schedule(plan: Plan) -> brr_schedule:
    return plan.schedule()


class Server:
    """Owns a brr_server* (continuous batching of shuffle/sample requests)."""

    def __init__(self, hbm_budget: int = 4 << 30, max_inflight: int = 64, nstreams: int = 8,
                 seed: int = 0, sched=None):
        cfg = brr_server_config(hbm_budget, max_inflight, nstreams, seed,
                                ctypes.pointer(sched) if sched is not None else None)
        self.ptr = ctypes.c_void_p()
        check(lib.brr_server_create(ctypes.byref(self.ptr), ctypes.byref(cfg)), "brr_server_create")

    def submit(self, kind: int, data, n: int, elem_bytes: int, session: int = 0, m: int = 0,
               out=None) -> int:
        req = brr_request(kind, elem_bytes, session, _addr(data), n, m, _addr(out))
        rid = ctypes.c_uint64()
        check(lib.brr_server_submit(self.ptr, ctypes.byref(req), ctypes.byref(rid)),
              "brr_server_submit")
        return int(rid.value)

    def wait(self, rid: int, timeout_s: float = 60.0) -> float:
        lat = ctypes.c_double()
        check(lib.brr_server_wait(self.ptr, rid, timeout_s, ctypes.byref(lat)), "brr_server_wait")
        return float(lat.value)

    def drain(self, timeout_s: float = 120.0) -> None:
        check(lib.brr_server_drain(self.ptr, timeout_s), "brr_server_drain")

    def stats(self) -> dict:
        st = brr_server_stats()
        check(lib.brr_server_get_stats(self.ptr, ctypes.byref(st)), "brr_server_get_stats")
        return st.as_dict()

    def reset_stats(self) -> None:
        check(lib.brr_server_reset_stats(self.ptr), "brr_server_reset_stats")

    def counter(self, session: int) -> int:
        v = ctypes.c_uint64()
        check(lib.brr_server_session_counter(self.ptr, session, ctypes.byref(v)),
              "brr_server_session_counter")
        return int(v.value)

    def close(self):
        if self.ptr:
            lib.brr_server_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Owns a brr_mlp* (the learned plan-cost model)."""

    def __init__(self, n_in: int = BRR_PLAN_FEATURES, hidden: int = 64, seed: int = 0):
        self.n_in, self.hidden = n_in, hidden
        self.ptr = ctypes.c_void_p()
        check(lib.brr_mlp_create(ctypes.byref(self.ptr), n_in, hidden, seed), "brr_mlp_create")
        self.nparams = int(lib.brr_mlp_num_params(self.ptr))

    def params(self):
        import numpy as np

        out = np.zeros(self.nparams, np.float32)
        check(lib.brr_mlp_get_params(self.ptr, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, values):
        import numpy as np

        v = np.ascontiguousarray(values, dtype=np.float32)
        assert v.size == self.nparams
        check(lib.brr_mlp_set_params(self.ptr, v.ctypes.data_as(ctypes.c_void_p)))

    def grads(self):
        import numpy as np

        out = np.zeros(self.nparams, np.float32)
        check(lib.brr_mlp_get_grads(self.ptr, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def forward(self, d_x, batch: int, d_y, stream=None) -> None:
        check(lib.brr_mlp_forward(self.ptr, _addr(d_x), batch, _addr(d_y), _stream(stream)),
              "brr_mlp_forward")

    def backward(self, d_x, d_t, batch: int, d_loss=None, stream=None) -> None:
        check(lib.brr_mlp_backward(self.ptr, _addr(d_x), _addr(d_t), batch, _addr(d_loss),
                                   _stream(stream)), "brr_mlp_backward")

    def adam_step(self, lr: float, stream=None) -> None:
        check(lib.brr_mlp_adam_step(self.ptr, lr, _stream(stream)), "brr_mlp_adam_step")

    def train(self, d_x, d_t, batch: int, steps: int, lr: float, stream=None) -> float:
        loss = ctypes.c_float()
        check(lib.brr_mlp_train(self.ptr, _addr(d_x), _addr(d_t), batch, steps, lr,
                                ctypes.byref(loss), _stream(stream)), "brr_mlp_train")
        return float(loss.value)

    def close(self):
        if self.ptr:
            lib.brr_mlp_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def brr_plan_features(h_offsets, elem_bytes: int, sched=None, wave_max: int = 512):
    import numpy as np

    off = np.ascontiguousarray(h_offsets, dtype=np.uint64)
    out = np.zeros(BRR_PLAN_FEATURES, np.float32)
    check(lib.brr_plan_features(off.ctypes.data_as(ctypes.c_void_p), off.size - 1, elem_bytes,
                                _sched(sched), wave_max, out.ctypes.data_as(ctypes.c_void_p)),
          "brr_plan_features")
    return out


def brr_plan_autotune_learned(plan: Plan, model: MLP, top: int, data, d_offsets, seed: int = 0,
                              inst_base: int = 0, stream=None) -> brr_tune_report:
    rep = brr_tune_report()
    check(lib.brr_plan_autotune_learned(plan.ptr, model.ptr, top, _addr(data), _addr(d_offsets),
                                        seed, inst_base, _stream(stream), ctypes.byref(rep)),
          "brr_plan_autotune_learned")
    return rep


def brr_sync_status(stream=None) -> int:
    return lib.brr_sync_status(_stream(stream))


def brr_probe_chain_rate(iters: int = 4096) -> float:
    """Dice per second the vector ALUs can chain (no memory, no word generation)."""
    out = ctypes.c_double()
    check(lib.brr_probe_chain_rate(iters, ctypes.byref(out)), "brr_probe_chain_rate")
    return out.value


def brr_probe_copy_rate(src, dst, nbytes: int, reps: int = 10, stream=None) -> float:
    """Bytes per second (read + written) of a bare copy with the dice stream's
    access pattern, src -> dst, nbytes each."""
    out = ctypes.c_double()
    check(lib.brr_probe_copy_rate(_addr(src), _addr(dst), nbytes, reps, _stream(stream),
                                  ctypes.byref(out)), "brr_probe_copy_rate")
    return out.value
