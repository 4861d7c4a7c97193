"""GPU: the continuous-batching server.  Every served result must equal the same problem annealed
alone (and the oracle), whatever the chunk size, the memory budget or the other requests."""
import time

import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa
from tests import parity
from tests.test_gpu_parity import explainer

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-server]", *a, flush=True)


def requests(n=10, sweeps=40, reads=5):
    items = I.cfg4_batch(n_instances=n, n_reads=reads, n_sweeps=sweeps, n_min=30, n_max=600,
                         w_min=2, w_max=200)
    for i, w in enumerate(items):
        w.instance_id = 1000 + i
        if i % 3 == 0:
            w.beta = oracle.Poly(w.problem).schedule(sweeps)[0]
        if i % 5 == 4:
            w.rule = sa.HEAT_BATH_CLOSED   # closed-form draws for linear variables, in the mix too
    return items


def alone(w):
    import torch
    plan = sa.Plan(w.problem, w.rule)
    z = torch.empty((w.n_reads, w.problem.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(w.n_reads, dtype=torch.int64, device="cuda")
    plan.run_device(w.n_sweeps, w.n_reads, w.seed, z, e, beta=w.beta,
                    stream=torch.cuda.current_stream().cuda_stream, instance_id=w.instance_id,
                    waves_per_replica=1)
    torch.cuda.synchronize()
    plan.close()
    return z.cpu().numpy(), e.cpu().numpy()


def serve(items, **kw):
    srv = sa.Server(**kw)
    tickets = [srv.submit(w) for w in items]
    timings = [srv.wait(t) for t in tickets]
    out = [srv.result(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    return out, timings, stats


@pytest.mark.parametrize("chunk", [1, 7, 1000])
def test_served_results_equal_alone(chunk):
    items = requests()
    say("chunk", chunk)
    out, timings, stats = serve(items, chunk_sweeps=chunk)
    say("stats", stats)
    assert all(t["status"] == sa.OK for t in timings)
    assert stats["completed"] == len(items)
    for i, w in enumerate(items):
        z, e = alone(w)
        assert np.array_equal(out[i][0], z) and np.array_equal(out[i][1], e), f"request {i}"
    w = items[2]
    P = oracle.Poly(w.problem)
    beta = w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]
    zo, eo = P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id)
    parity.check("served request 2", w.n_reads,
                 lambda i: out[2][1][i] == eo[i] and np.array_equal(out[2][0][i], zo[i]),
                 explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id, G=1))


def test_memory_budget_admission():
    items = requests(n=8, sweeps=20, reads=4)
    # a budget that holds only a few requests at a time: everything still completes, identically
    out, timings, stats = serve(items, mem_budget_bytes=2_000_000, chunk_sweeps=5, max_slots=3)
    for i, w in enumerate(items):
        assert timings[i]["status"] == sa.OK
        z, e = alone(w)
        assert np.array_equal(out[i][0], z) and np.array_equal(out[i][1], e)
    srv = sa.Server(mem_budget_bytes=100_000)
    big = I.Workload(I.erdos_renyi_quio(20_000, 3.0, -3, 3, 3, 3, np.random.Generator(np.random.PCG64(2))),
                     sa.METROPOLIS, 5, 4, 1)
    with pytest.raises(sa.SAError) as ex:
        srv.submit(big)                      # states alone exceed the budget
    assert ex.value.code == sa.ENOMEM
    mid = I.Workload(I.erdos_renyi_quio(5_000, 3.0, -3, 3, 3, 3, np.random.Generator(np.random.PCG64(3))),
                     sa.METROPOLIS, 5, 4, 1)
    t = srv.submit(mid)                      # fits the states, not the packed instance as well
    assert srv.wait(t)["status"] == sa.ENOMEM
    srv.close()


def test_repeated_instances_share_a_cached_plan():
    # requests over the same instance (different seeds and ids) reuse one prepared plan; results
    # are still those of each request alone
    base = I.cfg3_huio(rule="otm", n=300, m=3000, n_sweeps=30, n_reads=4)
    items = []
    for i in range(9):
        w = I.Workload(base.problem, sa.OPT_METROPOLIS if i % 3 else sa.HEAT_BATH, 30, 4, 100 + i, 500 + i)
        items.append(w)
    out, timings, stats = serve(items, chunk_sweeps=10)
    say("stats", stats)
    assert all(t["status"] == sa.OK for t in timings)
    # two rules, two plans; at most one extra build per preparer racing on the same instance
    assert stats["plans_reused"] >= len(items) - 2 - 4
    for i, w in enumerate(items):
        z, e = alone(w)
        assert np.array_equal(out[i][0], z) and np.array_equal(out[i][1], e), f"request {i}"


def test_cancel_leaves_others_untouched():
    items = requests(n=6, sweeps=30, reads=4)
    long = I.cfg3_huio(rule="otm", n=1500, m=15000, n_sweeps=100000, n_reads=8)
    long.instance_id = 77
    srv = sa.Server(chunk_sweeps=10)
    tl = srv.submit(long)
    ts = [srv.submit(w) for w in items]
    time.sleep(0.5)
    srv.cancel(tl)
    for i, t in enumerate(ts):
        assert srv.wait(t)["status"] == sa.OK
        z, e = alone(items[i])
        assert np.array_equal(srv.result(t)[0], z) and np.array_equal(srv.result(t)[1], e)
    assert srv.wait(tl)["status"] == sa.ECANCELED
    assert srv.stats()["canceled"] == 1
    srv.close()


def test_shared_plan_requests():
    w = I.cfg3_huio(rule="metropolis", n=400, m=4000, n_sweeps=25, n_reads=6)
    plan = sa.Plan(w.problem, w.rule)
    srv = sa.Server(chunk_sweeps=6)
    tickets = [srv.submit_plan(plan, w.n_sweeps, w.n_reads, w.seed, instance_id=k) for k in range(5)]
    for k, t in enumerate(tickets):
        assert srv.wait(t)["status"] == sa.OK
        w.instance_id = k
        z, e = alone(w)
        assert np.array_equal(srv.result(t)[0], z) and np.array_equal(srv.result(t)[1], e)
    srv.close()
    plan.close()


def test_served_wide_heat_bath_alone_and_in_mix():
    # dense W = 2001 heat-bath requests (the serving mix's type B, smaller N) and a W > 2048 one,
    # served with HUIO requests: each equals its plain launch alone and the oracle
    r = np.random.Generator(np.random.PCG64(23))
    wide = [I.Workload(I.dense_quio(192, -1000, 1000, 10, 10, r), sa.HEAT_BATH, 3, 4, 31, 3001),
            I.Workload(I.random_huio(100, 400, [1, 2], -1400, 1400, 2, r), sa.HEAT_BATH, 3, 3, 32, 3002),
            I.Workload(I.erdos_renyi_quio(150, 5.0, -600, 600, 6, 6, r), sa.HEAT_BATH, 5, 4, 33, 3003)]
    items = requests(n=6, sweeps=20, reads=4) + wide
    out, timings, stats = serve(items, chunk_sweeps=2)
    assert all(t["status"] == sa.OK for t in timings)
    for k, w in enumerate(wide):
        i = len(items) - len(wide) + k
        solo, _, _ = serve([w], chunk_sweeps=1)
        assert np.array_equal(out[i][0], solo[0][0]) and np.array_equal(out[i][1], solo[0][1]), "mix vs alone"
        z, e = alone(w)
        assert np.array_equal(out[i][0], z) and np.array_equal(out[i][1], e), f"wide request {k} vs plain"
        P = oracle.Poly(w.problem)
        beta = P.schedule(w.n_sweeps)[0]
        zo, eo = P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id)
        parity.check(f"wide request {k}", w.n_reads,
                     lambda j: out[i][1][j] == eo[j] and np.array_equal(out[i][0][j], zo[j]),
                     explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id, G=1))


def test_cfg5_served_mix_all_reads():
    # 64 requests of the serving stream (HUIO and dense N = 4096, W = 2001 heat bath; sweeps cut
    # to 100 and 2) served together with staggered arrivals; every read against the oracle's stored
    # results
    from tests.golden import make_full_size as M
    ws = M.cfg5_workloads()
    gold = M.read("cfg5")
    srv = sa.Server(chunk_sweeps=10)
    tickets = []
    for k, w in enumerate(ws):
        tickets.append(srv.submit(w))
        if k % 8 == 7:
            time.sleep(0.05)
    for w, t in zip(ws, tickets):
        assert srv.wait(t)["status"] == sa.OK
        z, e = srv.result(t)
        hdr, eo, ho = gold[f"cfg5-req{w.instance_id}"]
        P = oracle.Poly(w.problem)
        assert all(int(e[j]) == P.energy(z[j]) for j in range(w.n_reads))
        hg = parity.state_hashes(z)
        beta = M.schedule(P, w)
        parity.check(f"cfg5 request {w.instance_id}", w.n_reads,
                     lambda j: e[j] == eo[j] and hg[j] == ho[j],
                     explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id, G=1))
    say("stats", srv.stats())
    srv.close()
