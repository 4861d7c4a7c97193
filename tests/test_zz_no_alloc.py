"""GPU: sa_anneal_noalloc (staging in a static device area, no device allocation) gives the results
of sa_anneal_ex with the same arguments, through the C ABI, on two calls in a row (the second with
a smaller problem, which reuses the area the first one filled)."""
import numpy as np
import pytest

from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)


def run(prob, rule, n_sweeps, n_reads, seed, beta=None, no_alloc=False, trace=False, instance_id=0):
    import torch
    z = torch.empty((n_reads, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(n_reads, dtype=torch.int64, device="cuda")
    h = torch.empty(n_reads * n_sweeps, dtype=torch.int64, device="cuda") if trace else None
    stream = torch.cuda.current_stream().cuda_stream
    sa.anneal_device(prob, rule, n_sweeps, n_reads, seed, z, e, beta=beta, stream=stream,
                     instance_id=instance_id, trace=h, no_alloc=no_alloc)
    torch.cuda.synchronize()
    out = [z.cpu().numpy(), e.cpu().numpy()]
    if trace:
        out.append(h.cpu().numpy())
    return out


def test_no_alloc_equals_anneal_ex_on_two_calls():
    big = I.cfg2_sparse_quio(n=3000).problem                     # heat bath, 16 cooperating waves
    small = I.cfg3_huio(n=300, m=3000).problem                    # HUIO, smaller than the first
    calls = [("big heat bath", big, sa.HEAT_BATH, 30, 48, 5),
             ("small otm", small, sa.OPT_METROPOLIS, 25, 20, 6)]
    for label, prob, rule, sweeps, reads, seed in calls:
        say(label, "no-alloc")
        za, ea, ha = run(prob, rule, sweeps, reads, seed, no_alloc=True, trace=True, instance_id=3)
        say(label, "anneal_ex")
        zb, eb, hb = run(prob, rule, sweeps, reads, seed, no_alloc=False, trace=True, instance_id=3)
        assert np.array_equal(za, zb) and np.array_equal(ea, eb), label
        assert np.array_equal(ha, hb), label


def test_no_alloc_takes_the_windows_when_the_round_records_do_not_fit():
    # 40,000 variables: the Metropolis quad kernel's round-major record copy (about 20 KB per round
    # of 16 updates) would take over 50 MB, beyond the 32 MiB area, while the instance fits: the
    # automatic choice takes the windows, whose results are the quad kernel's (sa_anneal_ex)
    prob = I.random_huio(40_000, 60_000, [2, 3], -4, 4, 3, np.random.Generator(np.random.PCG64(9)))
    plan = sa.Plan(prob, sa.METROPOLIS)
    import torch
    z = torch.empty((2, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(2, dtype=torch.int64, device="cuda")
    plan.run_device(3, 2, 7, z, e, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert plan.last_launch()["lanes_per_update"] == 4 and plan.last_launch()["n_levels"] > 0
    plan.close()
    say("big HUIO", "no-alloc")
    za, ea = run(prob, sa.METROPOLIS, 3, 2, 7, no_alloc=True)
    say("big HUIO", "anneal_ex")
    zb, eb = run(prob, sa.METROPOLIS, 3, 2, 7, no_alloc=False)
    assert np.array_equal(za, zb) and np.array_equal(ea, eb)


def test_no_alloc_rejects_host_outputs_and_oversize_problems():
    prob = I.cfg3_huio(n=200, m=2000).problem
    m = sa._Marshalled(prob)
    sched, _ = sa._schedule(5, None)
    z = np.zeros((2, prob.n_vars), np.int32)
    e = np.zeros(2, np.int64)
    import ctypes as C
    opts = sa.make_opts(device_buffers=False)
    rc = sa.lib().sa_anneal_noalloc(C.byref(m.inst), C.byref(m.bounds), C.byref(sched), 0, 2, 1,
                                    sa._p(z), sa._p(e), C.byref(opts))
    assert rc == sa.EINVAL and "device_buffers" in sa.last_error()
    # 1.5 million pair terms: their packed records alone exceed the 32 MiB area
    import torch
    huge = I.random_huio(100_000, 1_500_000, [2], -3, 3, 3, np.random.Generator(np.random.PCG64(1)))
    zt = torch.empty((1, huge.n_vars), dtype=torch.int32, device="cuda")
    et = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(sa.SAError) as ex:
        sa.anneal_device(huge, sa.METROPOLIS, 1, 1, 1, zt, et, no_alloc=True)
    assert ex.value.code == sa.ENOMEM and "bytes of staging" in str(ex.value)
