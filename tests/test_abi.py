"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (these paths return before the first HIP call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w ]+?\**\s*\b(sa_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    L = sa.lib()
    names = declared_functions()
    assert "sa_anneal" in names and "sa_plan_run" in names and len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert L.sa_version() >= 100


def test_binding_covers_declared_functions():
    assert set(declared_functions()) == set(sa.EXPORTED)


def test_server_creation_without_a_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    _expect(sa.EDEVICE, lambda: sa.Server())


def _expect(code, fn):
    with pytest.raises(sa.SAError) as e:
        fn()
    assert e.value.code == code, e.value


def test_invalid_arguments_are_rejected_on_the_host():
    good = I.from_terms(3, [(1, [0, 1]), (-2, [2, 2])], -2, 2)
    _expect(sa.EINVAL, lambda: sa.Plan(I.from_terms(2, [(1, [0, 1])], [0, 3], [1, 2]), sa.METROPOLIS))
    _expect(sa.EINVAL, lambda: sa.Plan(I.from_terms(2, [(1, [0, 5])], 0, 1), sa.METROPOLIS))
    empty = I.Problem(2, np.array([0, 0], np.int64), np.zeros(0, np.int32), np.array([1], np.int64),
                      np.zeros(2, np.int32), np.ones(2, np.int32))
    _expect(sa.EINVAL, lambda: sa.Plan(empty, sa.METROPOLIS))
    _expect(sa.EINVAL, lambda: sa.Plan(good, 7))
    wide = I.from_terms(1, [(1, [0])], -2 ** 31, 2 ** 31 - 1)
    _expect(sa.EINVAL, lambda: sa.Plan(wide, sa.METROPOLIS))
    lim = 2 ** 62
    _expect(sa.ERANGE, lambda: sa.Plan(I.from_terms(1, [(lim // 4, [0, 0])], -2, 2), sa.METROPOLIS))
    five = I.from_terms(2, [(1, [0] * 5), (1, [0, 1])], -1, 1)
    _expect(sa.EUNSUPPORTED, lambda: sa.Plan(five, sa.OPT_METROPOLIS))
    _expect(sa.EUNSUPPORTED, lambda: sa.Plan(I.from_terms(1, [(1, [0] * 17)], -1, 1), sa.HEAT_BATH))
    _expect(sa.EINVAL, lambda: sa.anneal(good, sa.METROPOLIS, 0, 4, 1))
    _expect(sa.EINVAL, lambda: sa.anneal(good, sa.METROPOLIS, 3, 0, 1))
    _expect(sa.EINVAL, lambda: sa.anneal(good, sa.METROPOLIS, 2, 1, 1, beta=[1.0, float("nan")]))
    _expect(sa.EINVAL, lambda: sa.anneal(good, sa.METROPOLIS, 2, 1, 1, beta=[1.0, -1.0]))
    _expect(sa.EINVAL, lambda: sa.anneal(good, sa.METROPOLIS, 2, 1, 1, beta=[1.0, 2.0],
                                         init_states=np.full(3, 5, np.int32)))
    fixed = I.from_terms(2, [(3, [0, 1])], 1, 1)
    _expect(sa.EINVAL, lambda: sa.auto_schedule(fixed, 10))
    assert "bound" in sa.last_error() or "range" in sa.last_error() or sa.last_error()


def test_auto_schedule_matches_oracle():
    for prob in (I.cfg3_huio(n=300, m=3000).problem, I.cfg2_sparse_quio(n=500).problem,
                 I.cfg1_dense_quio().problem, I.fully_connected(40, 3, 5), I.multilinear(30, 4, 2)):
        lib_beta = sa.auto_schedule(prob, 200)
        ora_beta, _, _ = oracle.Poly(prob).schedule(200)
        np.testing.assert_allclose(lib_beta, ora_beta, rtol=1e-13, atol=0)


def test_auto_schedule_worked_example():
    # single variable z in [0,3], E = 2 z^2 - z: dE_max = 21, dE_min = 1 (Sec. 3.4)
    import math
    beta = sa.auto_schedule(I.from_terms(1, [(2, [0, 0]), (-1, [0])], 0, 3), 5)
    assert beta[0] == pytest.approx(math.log(2.0) / 21.0, rel=1e-15)
    assert beta[-1] == pytest.approx(math.log(1000.0), rel=1e-14)


def test_batch_rejects_bad_problems_on_the_host():
    w = I.cfg4_batch(n_instances=2, n_reads=2, n_sweeps=3, n_min=20, n_max=30)
    w[1].n_reads = 0
    _expect(sa.EINVAL, lambda: sa.Batch(w))
    big = I.Workload(I.erdos_renyi_quio(50_000, 2.0, -1, 1, 1, 1, np.random.Generator(np.random.PCG64(1))),
                     sa.METROPOLIS, 2, 2, 1)
    _expect(sa.EUNSUPPORTED, lambda: sa.Batch([big]))
    w = I.cfg4_batch(n_instances=2, n_reads=2, n_sweeps=3, n_min=20, n_max=30)
    w[0].beta = np.array([1.0, -2.0, 1.0])
    _expect(sa.EINVAL, lambda: sa.Batch(w))
