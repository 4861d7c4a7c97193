"""Thin ctypes binding of libsa.so (include/sa.h).

Argument marshalling only: every step of the annealing runs in the library's HIP kernels.  PyTorch
is used for device memory (output tensors) and streams.  Importing this module does not load the
library; the first call does, and raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsa.so")

OK, EINVAL, ERANGE, EUNSUPPORTED, ENOMEM, EDEVICE, EBUSY, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
METROPOLIS, HEAT_BATH, OPT_METROPOLIS, HEAT_BATH_CLOSED = 0, 1, 2, 3
RULE_NAMES = {METROPOLIS: "metropolis", HEAT_BATH: "heat_bath", OPT_METROPOLIS: "otm",
              HEAT_BATH_CLOSED: "heat_bath_closed"}


class SAError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"libsa status {code}: {message}")
        self.code = code


class sa_instance(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_terms", C.c_int64), ("term_ptr", C.c_void_p),
                ("factor_var", C.c_void_p), ("coef", C.c_void_p)]


class sa_bounds(C.Structure):
    _fields_ = [("lower", C.c_void_p), ("upper", C.c_void_p)]


class sa_schedule(C.Structure):
    _fields_ = [("n_sweeps", C.c_int32), ("beta", C.c_void_p)]


class sa_opts(C.Structure):
    _fields_ = [("instance_id", C.c_uint32), ("hip_stream", C.c_void_p), ("device_buffers", C.c_int32),
                ("sweep_begin", C.c_int32), ("sweep_end", C.c_int32), ("init_states", C.c_void_p),
                ("otm_r", C.c_double), ("waves_per_replica", C.c_int32), ("otm_enum_max", C.c_int32),
                ("trace_hashes", C.c_void_p), ("lanes_per_update", C.c_int32)]


class sa_plan_info(C.Structure):
    _fields_ = [("n_vars", C.c_int32), ("n_terms", C.c_int64), ("n_incidences", C.c_int64),
                ("n_factor_slots", C.c_int64), ("max_exponent", C.c_int32), ("max_width", C.c_int32),
                ("device_bytes", C.c_int64), ("coef_bits", C.c_int32), ("arith_bits", C.c_int32),
                ("dense", C.c_int32)]


class sa_launch_info(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("groups", C.c_int32), ("lds_bytes", C.c_int32),
                ("state_in_lds", C.c_int32), ("kernel_variant", C.c_int32),
                ("waves_per_replica", C.c_int32), ("n_windows", C.c_int32),
                ("lanes_per_update", C.c_int32), ("n_levels", C.c_int32)]


class sa_problem(C.Structure):
    _fields_ = [("inst", sa_instance), ("bounds", sa_bounds), ("sched", sa_schedule), ("rule", C.c_int32),
                ("n_reads", C.c_int32), ("seed", C.c_uint64), ("instance_id", C.c_uint32)]


class sa_result(C.Structure):
    _fields_ = [("states", C.c_void_p), ("energies", C.c_void_p), ("status", C.c_int32)]


class sa_batch_opts(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("use_graph", C.c_int32), ("hip_stream", C.c_void_p),
                ("waves_per_group", C.c_int32), ("groups", C.c_int32)]


class sa_batch_info(C.Structure):
    _fields_ = [("n_problems", C.c_int32), ("n_tasks", C.c_int64), ("total_updates", C.c_int64),
                ("waves_per_group", C.c_int32), ("groups", C.c_int32), ("slot_bytes", C.c_int32),
                ("kernel_maxe", C.c_int32), ("kernel_bits", C.c_int32), ("state_bits", C.c_int32),
                ("graph", C.c_int32), ("max_team", C.c_int32), ("policy", C.c_double),
                ("tune_ms", C.c_double)]


class sa_server_opts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_size_t), ("max_slots", C.c_int32), ("chunk_sweeps", C.c_int32),
                ("prep_threads", C.c_int32)]


class sa_timing(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("updates", C.c_uint64), ("status", C.c_int32)]


class sa_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("canceled", C.c_int64),
                ("failed", C.c_int64), ("active", C.c_int64), ("queued", C.c_int64), ("chunks", C.c_int64),
                ("updates", C.c_int64), ("mem_in_use", C.c_size_t), ("elapsed_s", C.c_double),
                ("plans_reused", C.c_int64)]


_lib = None


def lib():
    """Load libsa.so; raises if it was not built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_uint32
        P = C.POINTER
        L.sa_anneal.argtypes = [P(sa_instance), P(sa_bounds), P(sa_schedule), i32, i32, u64, vp, vp]
        L.sa_anneal_ex.argtypes = L.sa_anneal.argtypes + [P(sa_opts)]
        L.sa_anneal_noalloc.argtypes = L.sa_anneal.argtypes + [P(sa_opts)]
        L.sa_opts_default.argtypes = [P(sa_opts)]
        L.sa_opts_default.restype = None
        L.sa_plan_create.argtypes = [P(sa_instance), P(sa_bounds), i32, P(vp)]
        L.sa_plan_run.argtypes = [vp, P(sa_schedule), i32, u64, vp, vp, P(sa_opts)]
        L.sa_plan_destroy.argtypes = [vp]
        L.sa_plan_destroy.restype = None
        L.sa_plan_get_info.argtypes = [vp, P(sa_plan_info)]
        L.sa_plan_last_launch.argtypes = [vp, P(sa_launch_info)]
        L.sa_auto_schedule.argtypes = [P(sa_instance), P(sa_bounds), i32, vp]
        L.sa_energy.argtypes = [P(sa_instance), P(sa_bounds), i32, vp, vp]
        L.sa_batch_create.argtypes = [P(sa_problem), i32, P(sa_batch_opts), P(vp)]
        L.sa_batch_run.argtypes = [vp]
        L.sa_batch_wait.argtypes = [vp]
        L.sa_batch_results.argtypes = [vp, P(sa_result)]
        L.sa_batch_get_info.argtypes = [vp, P(sa_batch_info)]
        L.sa_batch_destroy.argtypes = [vp]
        L.sa_batch_destroy.restype = None
        L.sa_anneal_batch.argtypes = [P(sa_problem), i32, P(sa_result), P(sa_batch_opts)]
        L.sa_server_create.argtypes = [P(sa_server_opts), P(vp)]
        L.sa_server_submit.argtypes = [vp, P(sa_problem), P(sa_result), P(C.c_uint64)]
        L.sa_server_submit_plan.argtypes = [vp, vp, P(sa_schedule), i32, u64, u32, P(sa_result), P(C.c_uint64)]
        L.sa_server_poll.argtypes = [vp, C.c_uint64, P(i32), P(sa_timing)]
        L.sa_server_wait.argtypes = [vp, C.c_uint64, P(sa_timing)]
        L.sa_server_cancel.argtypes = [vp, C.c_uint64]
        L.sa_server_get_stats.argtypes = [vp, P(sa_server_stats)]
        L.sa_server_destroy.argtypes = [vp]
        L.sa_server_destroy.restype = None
        L.sa_last_error.argtypes = []
        L.sa_last_error.restype = C.c_char_p
        L.sa_version.argtypes = []
        for name in ("sa_anneal", "sa_anneal_ex", "sa_anneal_noalloc", "sa_plan_create", "sa_plan_run", "sa_plan_get_info",
                     "sa_plan_last_launch", "sa_auto_schedule", "sa_energy", "sa_version",
                     "sa_batch_create", "sa_batch_run", "sa_batch_wait", "sa_batch_results",
                     "sa_batch_get_info", "sa_anneal_batch", "sa_server_create", "sa_server_submit",
                     "sa_server_submit_plan", "sa_server_poll", "sa_server_wait", "sa_server_cancel",
                     "sa_server_get_stats"):
            getattr(L, name).restype = i32
        _lib = L
    return _lib


def last_error() -> str:
    return lib().sa_last_error().decode(errors="replace")


def _check(rc: int, what: str):
    if rc != OK:
        raise SAError(rc, f"{what}: {last_error()}")


def _p(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())  # torch tensor


class _Marshalled:
    """Keeps the numpy arrays of a problem alive while the C structs point at them."""

    def __init__(self, problem):
        self.tp = np.ascontiguousarray(problem.term_ptr, np.int64)
        self.fv = np.ascontiguousarray(problem.factor_var, np.int32)
        self.cf = np.ascontiguousarray(problem.coef, np.int64)
        self.lo = np.ascontiguousarray(problem.lower, np.int32)
        self.up = np.ascontiguousarray(problem.upper, np.int32)
        self.n = int(problem.n_vars)
        self.inst = sa_instance(self.n, int(self.cf.shape[0]), _p(self.tp), _p(self.fv), _p(self.cf))
        self.bounds = sa_bounds(_p(self.lo), _p(self.up))


def _schedule(n_sweeps: int, beta):
    if beta is None:
        return sa_schedule(int(n_sweeps), None), None
    b = np.ascontiguousarray(beta, np.float64)
    if int(n_sweeps) != b.shape[0]:
        raise ValueError("len(beta) must equal n_sweeps")
    return sa_schedule(int(b.shape[0]), _p(b)), b


def make_opts(instance_id=0, stream=None, device_buffers=False, sweep_begin=0, sweep_end=0,
              init_states=None, otm_r=-1.0, waves_per_replica=0, otm_enum_max=0,
              trace_hashes=None, lanes_per_update=0) -> sa_opts:
    o = sa_opts()
    lib().sa_opts_default(C.byref(o))
    o.instance_id = int(instance_id) & 0xFFFFFFFF
    o.hip_stream = stream
    o.device_buffers = 1 if device_buffers else 0
    o.sweep_begin = int(sweep_begin)
    o.sweep_end = int(sweep_end)
    o.init_states = _p(init_states)
    o.otm_r = float(otm_r)
    o.waves_per_replica = int(waves_per_replica)
    o.otm_enum_max = int(otm_enum_max)
    o.trace_hashes = _p(trace_hashes)
    o.lanes_per_update = int(lanes_per_update)
    return o


def anneal(problem, rule: int, n_sweeps: int, n_reads: int, seed: int, beta=None, instance_id=0,
           sweep_begin=0, sweep_end=0, init_states=None, otm_r=-1.0):
    """One-shot annealing with host buffers; returns (states int32[n_reads, N], energies int64)."""
    m = _Marshalled(problem)
    sched, keep = _schedule(n_sweeps, beta)
    z = np.zeros((n_reads, m.n), np.int32)
    e = np.zeros(n_reads, np.int64)
    zi = None if init_states is None else np.ascontiguousarray(init_states, np.int32)
    opts = make_opts(instance_id, None, False, sweep_begin, sweep_end, zi, otm_r)
    rc = lib().sa_anneal_ex(C.byref(m.inst), C.byref(m.bounds), C.byref(sched), int(rule), int(n_reads),
                            int(seed) & 0xFFFFFFFFFFFFFFFF, _p(z), _p(e), C.byref(opts))
    _check(rc, "sa_anneal_ex")
    return z, e


def anneal_device(problem, rule: int, n_sweeps: int, n_reads: int, seed: int, z_out, e_out, beta=None,
                  stream=None, instance_id=0, sweep_begin=0, sweep_end=0, init_states=None, otm_r=-1.0,
                  waves_per_replica=0, trace=None, no_alloc=False, lanes_per_update=0):
    """sa_anneal_ex (or, with no_alloc=True, sa_anneal_noalloc) writing into device tensors z_out
    (int32 [n_reads, N]) and e_out (int64 [n_reads]); returns once the work is queued."""
    m = _Marshalled(problem)
    assert z_out.is_cuda and e_out.is_cuda and z_out.is_contiguous() and e_out.is_contiguous()
    assert z_out.numel() == n_reads * m.n and e_out.numel() == n_reads
    assert z_out.dtype.itemsize == 4 and e_out.dtype.itemsize == 8
    sched, keep = _schedule(n_sweeps, beta)
    opts = make_opts(instance_id, stream, True, sweep_begin, sweep_end, init_states, otm_r,
                     waves_per_replica, trace_hashes=trace, lanes_per_update=lanes_per_update)
    fn = lib().sa_anneal_noalloc if no_alloc else lib().sa_anneal_ex
    rc = fn(C.byref(m.inst), C.byref(m.bounds), C.byref(sched), int(rule), int(n_reads),
            int(seed) & 0xFFFFFFFFFFFFFFFF, _p(z_out), _p(e_out), C.byref(opts))
    _check(rc, "sa_anneal_noalloc" if no_alloc else "sa_anneal_ex")


def auto_schedule(problem, n_sweeps: int) -> np.ndarray:
    m = _Marshalled(problem)
    beta = np.zeros(n_sweeps, np.float64)
    _check(lib().sa_auto_schedule(C.byref(m.inst), C.byref(m.bounds), int(n_sweeps), _p(beta)),
           "sa_auto_schedule")
    return beta


def energy(problem, states) -> np.ndarray:
    m = _Marshalled(problem)
    z = np.ascontiguousarray(states, np.int32).reshape(-1, m.n)
    out = np.zeros(z.shape[0], np.int64)
    _check(lib().sa_energy(C.byref(m.inst), C.byref(m.bounds), int(z.shape[0]), _p(z), _p(out)),
           "sa_energy")
    return out


class Plan:
    """A canonical instance packed in device memory for one rule (sa_plan)."""

    def __init__(self, problem, rule: int):
        m = _Marshalled(problem)
        h = C.c_void_p()
        _check(lib().sa_plan_create(C.byref(m.inst), C.byref(m.bounds), int(rule), C.byref(h)),
               "sa_plan_create")
        self.h = h
        self.n = m.n
        self.rule = int(rule)

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.sa_plan_destroy(self.h)
            self.h = None

    __del__ = close

    def info(self) -> dict:
        i = sa_plan_info()
        _check(lib().sa_plan_get_info(self.h, C.byref(i)), "sa_plan_get_info")
        return {f: getattr(i, f) for f, _ in sa_plan_info._fields_}

    def last_launch(self) -> dict:
        i = sa_launch_info()
        _check(lib().sa_plan_last_launch(self.h, C.byref(i)), "sa_plan_last_launch")
        return {f: getattr(i, f) for f, _ in sa_launch_info._fields_}

    def run_device(self, n_sweeps, n_reads, seed, z_out, e_out, beta=None, stream=None,
                   instance_id=0, sweep_begin=0, sweep_end=0, init_states=None, otm_r=-1.0,
                   waves_per_replica=0, otm_enum_max=0, trace=None, lanes_per_update=0):
        """Queue a run writing into device tensors z_out (int32 [n_reads, N]) and e_out (int64);
        trace, when given, is a device tensor of n_reads * (sweep_end - sweep_begin) 64-bit words
        that receives the state hash after every sweep."""
        assert z_out.is_cuda and e_out.is_cuda
        assert z_out.dtype.itemsize == 4 and e_out.dtype.itemsize == 8
        assert z_out.numel() == n_reads * self.n and e_out.numel() == n_reads
        assert z_out.is_contiguous() and e_out.is_contiguous()
        if init_states is not None:
            assert init_states.is_cuda and init_states.numel() == n_reads * self.n
        if trace is not None:
            s1 = sweep_end if sweep_end > 0 else n_sweeps
            assert trace.is_cuda and trace.dtype.itemsize == 8 and trace.is_contiguous()
            assert trace.numel() == n_reads * (s1 - sweep_begin)
        sched, keep = _schedule(n_sweeps, beta)
        opts = make_opts(instance_id, stream, True, sweep_begin, sweep_end, init_states, otm_r,
                         waves_per_replica, otm_enum_max, trace, lanes_per_update)
        rc = lib().sa_plan_run(self.h, C.byref(sched), int(n_reads), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               _p(z_out), _p(e_out), C.byref(opts))
        _check(rc, "sa_plan_run")

    def run(self, n_sweeps, n_reads, seed, beta=None, instance_id=0, sweep_begin=0, sweep_end=0,
            init_states=None, otm_r=-1.0, waves_per_replica=0, trace=False, lanes_per_update=0):
        """Run with host buffers; returns (states, energies), and with trace=True also the state
        hash after every sweep (uint64 [n_reads, sweep_end - sweep_begin])."""
        sched, keep = _schedule(n_sweeps, beta)
        z = np.zeros((n_reads, self.n), np.int32)
        e = np.zeros(n_reads, np.int64)
        zi = None if init_states is None else np.ascontiguousarray(init_states, np.int32)
        s1 = sweep_end if sweep_end > 0 else n_sweeps
        h = np.zeros((n_reads, s1 - sweep_begin), np.uint64) if trace else None
        opts = make_opts(instance_id, None, False, sweep_begin, sweep_end, zi, otm_r, waves_per_replica,
                         trace_hashes=h if trace and h.size else None, lanes_per_update=lanes_per_update)
        rc = lib().sa_plan_run(self.h, C.byref(sched), int(n_reads), int(seed) & 0xFFFFFFFFFFFFFFFF,
                               _p(z), _p(e), C.byref(opts))
        _check(rc, "sa_plan_run")
        return (z, e, h) if trace else (z, e)


class Batch:
    """Many problems annealed by one persistent launch (sa_batch).

    items: sequence of objects with .problem, .rule, .n_sweeps, .n_reads, .seed, .instance_id and
    .beta (None for the automatic schedule), e.g. inputs.Workload."""

    def __init__(self, items, autotune=False, use_graph=False, stream=None, waves_per_group=0, groups=0):
        self.items = list(items)
        n = len(self.items)
        self._keep = []
        probs = (sa_problem * n)()
        for i, w in enumerate(self.items):
            m = _Marshalled(w.problem)
            sched, b = _schedule(w.n_sweeps, w.beta)
            self._keep.append((m, b))
            probs[i] = sa_problem(m.inst, m.bounds, sched, int(w.rule), int(w.n_reads),
                                  int(w.seed) & 0xFFFFFFFFFFFFFFFF, int(w.instance_id) & 0xFFFFFFFF)
        opts = sa_batch_opts(1 if autotune else 0, 1 if use_graph else 0, stream, int(waves_per_group),
                             int(groups))
        h = C.c_void_p()
        _check(lib().sa_batch_create(probs, n, C.byref(opts), C.byref(h)), "sa_batch_create")
        self.h = h
        self._keep = None  # problems are copied by the library

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.sa_batch_destroy(self.h)
            self.h = None

    __del__ = close

    def run(self):
        _check(lib().sa_batch_run(self.h), "sa_batch_run")

    def wait(self):
        _check(lib().sa_batch_wait(self.h), "sa_batch_wait")

    def results(self):
        n = len(self.items)
        res = (sa_result * n)()
        bufs = []
        for i, w in enumerate(self.items):
            z = np.zeros((w.n_reads, w.problem.n_vars), np.int32)
            e = np.zeros(w.n_reads, np.int64)
            bufs.append((z, e))
            res[i] = sa_result(_p(z), _p(e), 0)
        _check(lib().sa_batch_results(self.h, res), "sa_batch_results")
        return bufs

    def info(self) -> dict:
        i = sa_batch_info()
        _check(lib().sa_batch_get_info(self.h, C.byref(i)), "sa_batch_get_info")
        return {f: getattr(i, f) for f, _ in sa_batch_info._fields_}


class Server:
    """Continuous-batching server (sa_server).  submit() copies the problem; results land in
    host buffers owned by this object and are returned by result()."""

    def __init__(self, mem_budget_bytes=0, max_slots=0, chunk_sweeps=0, prep_threads=0):
        o = sa_server_opts(int(mem_budget_bytes), int(max_slots), int(chunk_sweeps), int(prep_threads))
        h = C.c_void_p()
        _check(lib().sa_server_create(C.byref(o), C.byref(h)), "sa_server_create")
        self.h = h
        self._out = {}

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.sa_server_destroy(self.h)
            self.h = None

    __del__ = close

    def submit(self, w) -> int:
        """w: object with .problem, .rule, .n_sweeps, .n_reads, .seed, .instance_id, .beta."""
        m = _Marshalled(w.problem)
        sched, keep = _schedule(w.n_sweeps, w.beta)
        prob = sa_problem(m.inst, m.bounds, sched, int(w.rule), int(w.n_reads),
                          int(w.seed) & 0xFFFFFFFFFFFFFFFF, int(w.instance_id) & 0xFFFFFFFF)
        z = np.zeros((w.n_reads, w.problem.n_vars), np.int32)
        e = np.zeros(w.n_reads, np.int64)
        res = sa_result(_p(z), _p(e), 0)
        t = C.c_uint64()
        _check(lib().sa_server_submit(self.h, C.byref(prob), C.byref(res), C.byref(t)), "sa_server_submit")
        self._out[t.value] = (z, e)
        return t.value

    def submit_plan(self, plan, n_sweeps, n_reads, seed, instance_id=0, beta=None) -> int:
        sched, keep = _schedule(n_sweeps, beta)
        z = np.zeros((n_reads, plan.n), np.int32)
        e = np.zeros(n_reads, np.int64)
        res = sa_result(_p(z), _p(e), 0)
        t = C.c_uint64()
        _check(lib().sa_server_submit_plan(self.h, plan.h, C.byref(sched), int(n_reads),
                                           int(seed) & 0xFFFFFFFFFFFFFFFF, int(instance_id) & 0xFFFFFFFF,
                                           C.byref(res), C.byref(t)), "sa_server_submit_plan")
        self._out[t.value] = (z, e)
        return t.value

    @staticmethod
    def _timing(t):
        return {f: getattr(t, f) for f, _ in sa_timing._fields_}

    def poll(self, ticket):
        done = C.c_int32()
        t = sa_timing()
        _check(lib().sa_server_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(t)), "sa_server_poll")
        return bool(done.value), self._timing(t)

    def wait(self, ticket):
        """Blocks until done; returns the request's timing (status inside)."""
        t = sa_timing()
        lib().sa_server_wait(self.h, C.c_uint64(ticket), C.byref(t))
        return self._timing(t)

    def result(self, ticket):
        return self._out[ticket]

    def cancel(self, ticket):
        _check(lib().sa_server_cancel(self.h, C.c_uint64(ticket)), "sa_server_cancel")

    def stats(self) -> dict:
        st = sa_server_stats()
        _check(lib().sa_server_get_stats(self.h, C.byref(st)), "sa_server_get_stats")
        return {f: getattr(st, f) for f, _ in sa_server_stats._fields_}


EXPORTED = ["sa_anneal", "sa_anneal_ex", "sa_anneal_noalloc", "sa_opts_default", "sa_plan_create", "sa_plan_run",
            "sa_plan_destroy", "sa_plan_get_info", "sa_plan_last_launch", "sa_auto_schedule",
            "sa_energy", "sa_last_error", "sa_version", "sa_batch_create", "sa_batch_run", "sa_batch_wait",
            "sa_batch_results", "sa_batch_get_info", "sa_batch_destroy", "sa_anneal_batch",
            "sa_server_create", "sa_server_submit", "sa_server_submit_plan", "sa_server_poll",
            "sa_server_wait", "sa_server_cancel", "sa_server_get_stats", "sa_server_destroy"]
