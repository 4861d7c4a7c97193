"""GPU: the batched form (one persistent launch over many problems) gives, problem by problem,
exactly the per-instance results, which match the oracle."""
import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa

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
    import torch
    plan = sa.Plan(w.problem, w.rule)
    z = torch.empty((w.n_reads, w.problem.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(w.n_reads, dtype=torch.int64, device="cuda")
    plan.run_device(w.n_sweeps, w.n_reads, w.seed, z, e, beta=w.beta,
                    stream=torch.cuda.current_stream().cuda_stream, instance_id=w.instance_id)
    torch.cuda.synchronize()
    plan.close()
    return z.cpu().numpy(), e.cpu().numpy()


def oracle_run(w):
    P = oracle.Poly(w.problem)
    beta = w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]
    return P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id)


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
            zo, eo = oracle_run(w)
            assert np.array_equal(got[i][0], zo) and np.array_equal(got[i][1], eo), f"problem {i} vs oracle"
    b.close()


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
