"""ctypes binding of the CPU oracle (``oracle/sa_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py``.  The GPU library never loads it and shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsa_oracle.so")
SRC_PATH = os.path.join(HERE, "sa_oracle.c")

OK, EINVAL, ERANGE, EUNSUPPORTED, ENOMEM, EINTERNAL = 0, -1, -2, -3, -4, -8
METROPOLIS, HEAT_BATH, OPT_METROPOLIS, HEAT_BATH_CLOSED = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, so FP64 expressions round as written)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
           "-shared", "-pthread", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        p, i32, i64, u32, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.sao_poly_build.argtypes = [i32, i64, p, p, p, p, p, C.POINTER(C.c_void_p)]
        L.sao_poly_build.restype = C.c_int
        L.sao_poly_free.argtypes = [p]
        L.sao_poly_free.restype = None
        L.sao_poly_n_terms.argtypes = [p]
        L.sao_poly_n_terms.restype = i64
        L.sao_poly_n_pairs.argtypes = [p]
        L.sao_poly_n_pairs.restype = i64
        L.sao_poly_max_exponent.argtypes = [p]
        L.sao_poly_max_exponent.restype = i32
        L.sao_poly_export.argtypes = [p, p, p, p, p]
        L.sao_poly_export.restype = C.c_int
        L.sao_energy.argtypes = [p, p, p]
        L.sao_energy.restype = C.c_int
        L.sao_delta.argtypes = [p, p, i32, i32, p]
        L.sao_delta.restype = C.c_int
        L.sao_schedule.argtypes = [p, i32, p, p, p]
        L.sao_schedule.restype = C.c_int
        L.sao_philox.argtypes = [p, p, p]
        L.sao_philox.restype = None
        L.sao_anneal.argtypes = [p, C.c_int, p, i32, i32, i32, i32, u64, u32, dbl, C.c_int, C.c_int,
                                 p, p, p]
        L.sao_anneal.restype = C.c_int
        L.sao_anneal_reads.argtypes = [p, C.c_int, p, i32, i32, i32, i32, p, u64, u32, dbl, C.c_int,
                                       C.c_int, p, p, p, p]
        L.sao_anneal_reads.restype = C.c_int
        L.sao_single_step.argtypes = [p, C.c_int, p, i32, i32, dbl, dbl, i32, u64, u32, p]
        L.sao_single_step.restype = C.c_int
        L.sao_state_hash.argtypes = [i32, p]
        L.sao_state_hash.restype = u64
        L.sao_mix64.argtypes = [u64]
        L.sao_mix64.restype = u64
        L.sao_explain_step.argtypes = [p, C.c_int, p, i32, i32, u32, dbl, dbl, u64, u32, C.POINTER(StepInfo)]
        L.sao_explain_step.restype = C.c_int
        L.sao_default_threads.argtypes = []
        L.sao_default_threads.restype = C.c_int
        _lib = L
    return _lib


class StepInfo(C.Structure):
    """What one update computed (``sao_step_info``)."""
    _fields_ = [("v", C.c_int64), ("dE", C.c_int64), ("accepted", C.c_int32), ("branch", C.c_int32),
                ("U", C.c_double), ("threshold", C.c_double), ("total", C.c_double),
                ("c_prev", C.c_double), ("c_at", C.c_double), ("margin", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def default_threads() -> int:
    return int(lib().sao_default_threads())


class Poly:
    """Canonical polynomial held by the oracle."""

    def __init__(self, problem):
        L = lib()
        self._keep = (np.ascontiguousarray(problem.term_ptr, np.int64),
                      np.ascontiguousarray(problem.factor_var, np.int32),
                      np.ascontiguousarray(problem.coef, np.int64),
                      np.ascontiguousarray(problem.lower, np.int32),
                      np.ascontiguousarray(problem.upper, np.int32))
        tp, fv, cf, lo, up = self._keep
        h = C.c_void_p()
        rc = L.sao_poly_build(int(problem.n_vars), int(cf.shape[0]), _ptr(tp), _ptr(fv), _ptr(cf),
                              _ptr(lo), _ptr(up), C.byref(h))
        if rc != OK:
            raise OracleError(rc, "canonicalisation")
        self.h = h
        self.n = int(problem.n_vars)
        self.lower = lo
        self.upper = up

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.sao_poly_free(h)
            self.h = None

    @property
    def n_terms(self) -> int:
        return int(lib().sao_poly_n_terms(self.h))

    @property
    def max_exponent(self) -> int:
        return int(lib().sao_poly_max_exponent(self.h))

    def canonical_terms(self):
        """List of (coef, ((var, exp), ...)) in the oracle's canonical order."""
        nt = self.n_terms
        npairs = int(lib().sao_poly_n_pairs(self.h))
        tptr = np.zeros(nt + 1, np.int64)
        var = np.zeros(max(npairs, 1), np.int32)
        ex = np.zeros(max(npairs, 1), np.int32)
        cf = np.zeros(max(nt, 1), np.int64)
        lib().sao_poly_export(self.h, _ptr(tptr), _ptr(var), _ptr(ex), _ptr(cf))
        return [(int(cf[t]), tuple((int(var[q]), int(ex[q])) for q in range(tptr[t], tptr[t + 1])))
                for t in range(nt)]

    def energy(self, z) -> int:
        z = np.ascontiguousarray(z, np.int32)
        out = np.zeros(1, np.int64)
        rc = lib().sao_energy(self.h, _ptr(z), _ptr(out))
        if rc != OK:
            raise OracleError(rc, "energy")
        return int(out[0])

    def delta(self, z, k, v) -> int:
        z = np.ascontiguousarray(z, np.int32)
        out = np.zeros(1, np.int64)
        rc = lib().sao_delta(self.h, _ptr(z), int(k), int(v), _ptr(out))
        if rc != OK:
            raise OracleError(rc, "delta")
        return int(out[0])

    def schedule(self, n_sweeps):
        beta = np.zeros(n_sweeps, np.float64)
        ti, tf = C.c_double(), C.c_double()
        rc = lib().sao_schedule(self.h, int(n_sweeps), _ptr(beta), C.byref(ti), C.byref(tf))
        if rc != OK:
            raise OracleError(rc, "schedule")
        return beta, ti.value, tf.value

    def anneal(self, rule, beta, n_reads, seed, instance_id=0, s_begin=0, s_end=None,
               otm_r=-1.0, cache_mode=0, n_threads=0, z_init=None, trace=False):
        """Final states and tracked energies of reads 0..n_reads-1; with trace=True also the state
        hash after every sweep of the run (n_reads x (s_end - s_begin), uint64)."""
        return self.anneal_reads(rule, beta, np.arange(n_reads, dtype=np.uint32), seed, instance_id,
                                 otm_r, cache_mode, n_threads, s_begin=s_begin, s_end=s_end,
                                 z_init=z_init, trace=trace)

    def anneal_reads(self, rule, beta, read_ids, seed, instance_id=0, otm_r=-1.0, cache_mode=0,
                     n_threads=0, s_begin=0, s_end=None, z_init=None, trace=False):
        """Chains of the given read ids only (rows in the order of read_ids)."""
        beta = np.ascontiguousarray(beta, np.float64)
        ids = np.ascontiguousarray(read_ids, np.uint32)
        n = int(ids.shape[0])
        z = np.zeros((n, self.n), np.int32)
        e = np.zeros(n, np.int64)
        S = int(beta.shape[0])
        s_end = S if s_end is None else int(s_end)
        zi = None if z_init is None else np.ascontiguousarray(z_init, np.int32).reshape(n, self.n)
        h = np.zeros((n, max(s_end - int(s_begin), 0)), np.uint64) if trace else None
        rc = lib().sao_anneal_reads(self.h, int(rule), _ptr(beta), S, int(s_begin), s_end, n, _ptr(ids),
                                    int(seed) & 0xFFFFFFFFFFFFFFFF, int(instance_id) & 0xFFFFFFFF,
                                    float(otm_r), int(cache_mode), int(n_threads), _ptr(zi), _ptr(z),
                                    _ptr(e), _ptr(h) if trace and h.size else None)
        if rc != OK:
            raise OracleError(rc, "anneal_reads")
        return (z, e, h) if trace else (z, e)

    def explain_step(self, rule, z, k, s, read, beta, r_opt, seed, instance_id=0) -> dict:
        """The update of variable k at sweep s of read `read` from state z: drawn or proposed value,
        its energy change, the uniform number, the decision threshold and its margin."""
        z = np.ascontiguousarray(z, np.int32)
        info = StepInfo()
        rc = lib().sao_explain_step(self.h, int(rule), _ptr(z), int(k), int(s), int(read) & 0xFFFFFFFF,
                                    float(beta), float(r_opt), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                    int(instance_id) & 0xFFFFFFFF, C.byref(info))
        if rc != OK:
            raise OracleError(rc, "explain_step")
        return info.as_dict()

    def single_step(self, rule, z, k, s, beta, r_opt, n_reads, seed, instance_id=0):
        z = np.ascontiguousarray(z, np.int32)
        v = np.zeros(n_reads, np.int32)
        rc = lib().sao_single_step(self.h, int(rule), _ptr(z), int(k), int(s), float(beta),
                                   float(r_opt), int(n_reads), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                   int(instance_id) & 0xFFFFFFFF, _ptr(v))
        if rc != OK:
            raise OracleError(rc, "single_step")
        return v


def state_hash(z) -> int:
    """Hash of one state (``sao_state_hash``)."""
    z = np.ascontiguousarray(z, np.int32).reshape(-1)
    return int(lib().sao_state_hash(int(z.shape[0]), _ptr(z)))


def mix64(x: int) -> int:
    """The state hash's mixing function (``sao_mix64``)."""
    return int(lib().sao_mix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def philox(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().sao_philox(_ptr(c), _ptr(k), _ptr(o))
    return o
