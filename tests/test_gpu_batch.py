"""GPU: the batched form (one persistent launch over many problems) gives, problem by problem,
exactly the results of plain per-instance launches of the same kernels (one wavefront per update),
and those match the oracle at the parity bar (tests/parity.py)."""
import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa
from tests import parity
from tests.test_gpu_parity import explainer

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-batch]", *a, flush=True)


def mixed_items(n=18, sweeps=30, reads=6):
    """Uneven sizes, widths, orders and rules, drawn like the 512-instance batch but small."""
    items = I.cfg4_batch(n_instances=n, n_reads=reads, n_sweeps=sweeps, n_min=20, n_max=700,
                         w_min=2, w_max=300)
    r = np.random.Generator(np.random.PCG64(8))
    items.append(I.Workload(I.dense_quio(160, -30, 30, 10, 10, r), sa.HEAT_BATH, sweeps, reads, 5, 901))
    items.append(I.Workload(I.dense_quio(70, -4, 4, 400, 50, r), sa.OPT_METROPOLIS, sweeps, reads, 6, 902))
    # closed-form heat bath: all variables linear, and mixed with squared variables
    items.append(I.Workload(I.erdos_renyi_quio(300, 6.0, -40, 40, 10, 20, r), sa.HEAT_BATH_CLOSED, sweeps,
                            reads, 7, 903))
    items.append(I.Workload(I.random_huio(120, 600, [1, 2, 3], -6, 9, 5, r), sa.HEAT_BATH_CLOSED, sweeps,
                            reads, 8, 904))
    # explicit schedules for some problems, automatic for the others
    for i, w in enumerate(items):
        if i % 4 == 0:
            w.beta = oracle.Poly(w.problem).schedule(sweeps)[0]
    return items


def per_instance(w):
    """A plain launch of the problem alone, one wavefront per update (the batch's update code)."""
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


def oracle_run(w):
    P = oracle.Poly(w.problem)
    beta = w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]
    return P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id)


def vs_oracle(label, w, z, e):
    """Results of problem w against the oracle at the parity bar; a parted read is traced through
    plain launches of the same update code."""
    P = oracle.Poly(w.problem)
    beta = w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]
    zo, eo = P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id)
    parity.check(label, w.n_reads, lambda i: e[i] == eo[i] and np.array_equal(z[i], zo[i]),
                 explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id, G=1))


@pytest.mark.parametrize("mode", ["plain", "graph", "autotune"])
def test_batch_equals_per_instance_and_oracle(mode):
    items = mixed_items()
    say("batch", mode, [(w.problem.n_vars, int(w.problem.upper[0] - w.problem.lower[0] + 1), w.rule)
                        for w in items])
    b = sa.Batch(items, autotune=(mode == "autotune"), use_graph=(mode == "graph"))
    say("info", b.info())
    assert b.info()["state_bits"] == 16
    b.run()
    got = b.results()
    for i, w in enumerate(items):
        zp, ep = per_instance(w)
        assert np.array_equal(got[i][0], zp) and np.array_equal(got[i][1], ep), f"problem {i} vs plain"
        if i % 3 == 0 or w.rule == sa.HEAT_BATH_CLOSED:
            vs_oracle(f"{mode} problem {i}", w, got[i][0], got[i][1])
    b.close()


def test_batch_wide_heat_bath_ranges():
    # heat-bath problems wider than 512 values take the batch kernel's recompute path (weights
    # evaluated again in the selection); 2048 < W takes it in plain launches too.  Sparse and dense
    # QUIO (the served dense requests have W = 2001), linear and squared variables.
    r = np.random.Generator(np.random.PCG64(21))
    items = [
        I.Workload(I.erdos_renyi_quio(300, 6.0, -400, 400, 10, 10, r), sa.HEAT_BATH, 8, 4, 11, 1),   # W 801
        I.Workload(I.dense_quio(256, -1000, 1000, 10, 10, r), sa.HEAT_BATH, 3, 4, 12, 2),        # W 2001, dense
        I.Workload(I.random_huio(120, 500, [1, 2, 3], -1500, 1500, 2, r), sa.HEAT_BATH, 4, 3, 13, 3),  # W 3001
        I.Workload(I.erdos_renyi_quio(200, 4.0, -1200, 1300, 5, 5, r), sa.HEAT_BATH_CLOSED, 6, 4, 14, 4),
        I.Workload(I.dense_quio(96, -700, 700, 8, 8, r), sa.HEAT_BATH_CLOSED, 4, 4, 15, 5),       # squares: enum
        I.Workload(I.cfg3_huio(n=200, m=2000).problem, sa.OPT_METROPOLIS, 10, 4, 16, 6),
    ]
    for mode in ("plain", "graph"):
        say("wide batch", mode)
        b = sa.Batch(items, use_graph=(mode == "graph"))
        b.run()
        got = b.results()
        b.close()
        for i, w in enumerate(items):
            zp, ep = per_instance(w)
            assert np.array_equal(got[i][0], zp) and np.array_equal(got[i][1], ep), f"{mode} problem {i} vs plain"
            if mode == "plain":
                vs_oracle(f"wide problem {i}", w, got[i][0], got[i][1])


def test_cfg4_full_batch_sampled_problems_all_reads():
    # the 512-problem batch in the benchmark's configuration (autotuned geometry, graph replay);
    # every read of a seeded sample of 40 problems against the oracle's stored results
    from tests.golden import make_full_size as M
    items, ids = M.cfg4_sample()
    gold = M.read("cfg4")
    say("cfg4 full batch", len(items), "problems")
    b = sa.Batch(items, autotune=True, use_graph=True)
    say("info", b.info())
    b.run()
    got = b.results()
    b.close()
    for i in ids:
        w = items[i]
        hdr, eo, ho = gold[f"cfg4-item{i}"]
        z, e = got[i]
        P = oracle.Poly(w.problem)
        assert all(int(e[j]) == P.energy(z[j]) for j in range(w.n_reads))
        hg = parity.state_hashes(z)
        beta = M.schedule(P, w)
        parity.check(f"cfg4 item {i}", w.n_reads, lambda j: e[j] == eo[j] and hg[j] == ho[j],
                     explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id, G=1))


def test_graph_replays_are_identical_with_eager_work_between():
    import torch
    items = mixed_items(n=10, sweeps=15, reads=4)
    b = sa.Batch(items, use_graph=True)
    ref = None
    for rep in range(3):
        say("replay", rep)
        b.run()
        got = b.results()
        # unrelated eager work on the device between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
        torch.cuda.synchronize()
        assert float(x.sum().item()) > 0
        if ref is None:
            ref = got
        else:
            for (za, ea), (zb, eb) in zip(ref, got):
                assert np.array_equal(za, zb) and np.array_equal(ea, eb)
    zp, ep = per_instance(items[3])
    assert np.array_equal(ref[3][0], zp) and np.array_equal(ref[3][1], ep)
    b.close()


def test_batch_geometry_does_not_change_results():
    items = mixed_items(n=8, sweeps=12, reads=5)
    outs = []
    for groups in (64, 7, 512):
        say("geometry", groups)
        b = sa.Batch(items, groups=groups)
        b.run()
        outs.append(b.results())
        b.close()
    for other in outs[1:]:
        for (za, ea), (zb, eb) in zip(outs[0], other):
            assert np.array_equal(za, zb) and np.array_equal(ea, eb)


def test_batch_with_wide_bounds_uses_32bit_states():
    items = mixed_items(n=6, sweeps=10, reads=4)
    r = np.random.Generator(np.random.PCG64(17))
    wide = I.erdos_renyi_quio(300, 4.0, -40_000, 40_000, 3, 3, r, name="wide")
    items.append(I.Workload(wide, sa.METROPOLIS, 10, 4, 99, 1234))
    b = sa.Batch(items)
    assert b.info()["state_bits"] == 32
    b.run()
    got = b.results()
    for i in (0, len(items) - 1):
        zp, ep = per_instance(items[i])
        assert np.array_equal(got[i][0], zp) and np.array_equal(got[i][1], ep)
    b.close()
