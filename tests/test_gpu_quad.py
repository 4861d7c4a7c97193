"""GPU: the quad kernel (one update per four lanes over the sweep's dependency levels) against the
oracle, for the heat bath, Metropolis and the optimal transition.  Its heat-bath cumulative weights
are added in value order, the oracle's order, so reads part only where an exponential's last bit
decides a draw; the bar is tests/parity.py's."""
import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa
from tests import parity

pytestmark = pytest.mark.gpu

HB = [sa.HEAT_BATH, sa.HEAT_BATH_CLOSED]


def say(*a):
    print("[gpu-quad]", *a, flush=True)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def quad_run(prob, rule, beta, n_reads, seed, instance_id=0, init=None, s0=0, s1=0, trace=False, lanes=4,
             otm_r=-1.0):
    import torch
    plan = sa.Plan(prob, rule)
    z = torch.empty((n_reads, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(n_reads, dtype=torch.int64, device="cuda")
    zi = None if init is None else torch.as_tensor(np.ascontiguousarray(init, np.int32), device="cuda")
    n_traced = (s1 if s1 > 0 else len(beta)) - s0
    h = torch.empty(n_reads * n_traced, dtype=torch.int64, device="cuda") if trace else None
    plan.run_device(len(beta), n_reads, seed, z, e, beta=beta, stream=torch.cuda.current_stream().cuda_stream,
                    instance_id=instance_id, init_states=zi, sweep_begin=s0, sweep_end=s1, trace=h,
                    lanes_per_update=lanes, otm_r=otm_r)
    torch.cuda.synchronize()
    launch = plan.last_launch()
    plan.close()
    assert launch["lanes_per_update"] == lanes
    out = (z.cpu().numpy(), e.cpu().numpy(), launch)
    if trace:
        out += (h.cpu().numpy().view(np.uint64).reshape(n_reads, n_traced),)
    return out


def vs_oracle(label, prob, rule, beta, n_reads, seed, instance_id=0, otm_r=-1.0):
    P = oracle.Poly(prob)
    zg, eg, launch = quad_run(prob, rule, beta, n_reads, seed, instance_id, otm_r=otm_r)
    zo, eo = P.anneal(rule, beta, n_reads, seed, instance_id, otm_r=otm_r)
    assert all(int(eg[i]) == P.energy(zg[i]) for i in range(n_reads))

    def explain(i):
        _, _, _, h = quad_run(prob, rule, beta, i + 1, seed, instance_id, trace=True, otm_r=otm_r)

        def after(s, z):
            zz, _, _ = quad_run(prob, rule, beta, i + 1, seed, instance_id, init=np.tile(z, (i + 1, 1)),
                                s0=s, s1=s + 1, otm_r=otm_r)
            return zz[i]
        return parity.localise(P, rule, beta, seed, instance_id, i, h[i], after, otm_r=otm_r)
    parity.check(f"{label} {launch}", n_reads, lambda i: eg[i] == eo[i] and np.array_equal(zg[i], zo[i]),
                 explain)


def uneven(p):
    """The terms of p over 300 variables whose widths run through 7..23 (bounds i % 7 - 12 .. i % 11)."""
    n = np.arange(300, dtype=np.int32)
    return I.Problem(300, p.term_ptr, p.factor_var, p.coef, n % 7 - 12, n % 11)


def hub_huio(r):
    """HUIO of 200 variables where variable 0 sits in about 150 terms and variable 1 in about 70
    (rows longer than the 64 records per update that the Metropolis / optimal-transition kernel
    loads one round ahead), some of them with four other factors."""
    base = I.random_huio(200, 500, [2, 3], -6, 6, 4, r)
    terms = [(int(base.coef[t]), base.factor_var[base.term_ptr[t]:base.term_ptr[t + 1]].tolist())
             for t in range(len(base.coef))]
    for _ in range(150):
        terms.append((int(r.integers(-4, 5)) or 1, [0, int(r.integers(2, 200))]))
    for _ in range(60):
        terms.append((int(r.integers(-4, 5)) or 1, [1, 1, int(r.integers(2, 200))]))
    for _ in range(10):
        terms.append((int(r.integers(-2, 3)) or 1, [1] + [int(x) for x in r.integers(2, 200, size=4)]))
    return I.from_terms(200, terms, -6, 6)


def cases():
    r = rng(4040)
    yield "er_w101_n3000", I.cfg2_sparse_quio(n=3000).problem, 30, 48
    yield "er_w2", I.erdos_renyi_quio(500, 6.0, 0, 1, 5, 5, r), 25, 32
    yield "er_w7_n900", I.erdos_renyi_quio(900, 8.0, -3, 3, 10, 10, r), 25, 32
    yield "er_w33", I.erdos_renyi_quio(700, 5.0, -16, 16, 10, 10, r), 25, 32
    yield "er_w64", I.erdos_renyi_quio(700, 5.0, -32, 31, 10, 10, r), 25, 32
    yield "er_w128", I.erdos_renyi_quio(600, 4.0, -64, 63, 7, 7, r), 20, 24
    # the factored weights at the most places past the range their classes allow (98 of 104,
    # 60 of 64), and beside the enumeration of quadratic variables in one launch (width 101)
    yield "er_w98", I.erdos_renyi_quio(700, 6.0, -49, 48, 9, 9, r), 25, 32
    # mean degree 1: a few levels of over a thousand variables, several batches of rounds each
    yield "er_w101_big_levels", I.erdos_renyi_quio(3000, 1.0, -50, 50, 9, 9, r), 20, 16
    yield "er_w60", I.erdos_renyi_quio(700, 6.0, -30, 29, 9, 9, r), 25, 32
    yield "squares_w101", I.random_huio(700, 2100, [1, 2], -50, 50, 4, r), 25, 32
    squares = I.random_huio(800, 2400, [1, 2], -20, 20, 6, r)      # z_i^2 terms: enumeration
    yield "squares_w41", squares, 25, 32
    fixed = I.erdos_renyi_quio(400, 6.0, -8, 9, 8, 8, r)
    fixed.lower[::5] = 3
    fixed.upper[::5] = 3
    yield "fixed_vars_w18", fixed, 20, 16
    yield "wide_coefs_64bit", I.random_huio(300, 900, [1, 2], -60, 60, 20000, r), 15, 16
    yield "single_variable", I.from_terms(1, [(3, [0, 0]), (-7, [0])], -5, 6), 30, 8
    yield "hub_rows", hub_huio(r), 20, 16
    yield "uneven_widths", uneven(I.erdos_renyi_quio(300, 5.0, -4, 4, 6, 6, r))
    # the factored weights with no place past the range (104 of 104) and at the most places the
    # 32-value class allows (120 of 128)
    yield "er_w104", I.erdos_renyi_quio(600, 5.0, -52, 51, 9, 9, r), 25, 32
    yield "er_w120", I.erdos_renyi_quio(500, 5.0, -60, 59, 8, 8, r), 25, 32


@pytest.mark.parametrize("case", list(cases()), ids=lambda c: c[0])
def test_quad_kernel_against_the_oracle(case):
    name, prob, sweeps, reads = case if len(case) == 4 else (*case, 20, 16)
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(sweeps)
    for rule in HB:
        say(name, sa.RULE_NAMES[rule], f"N={prob.n_vars} S={sweeps} R={reads}")
        vs_oracle(f"{name}/{sa.RULE_NAMES[rule]}", prob, rule, beta, reads, 600 + rule, instance_id=5)


def mo_cases():
    r = rng(4141)
    yield "huio_w101_deg4", I.cfg3_huio(n=400, m=4000).problem, 25, 48
    yield "huio_powers_w17", I.random_huio(300, 1500, [1, 2, 3, 4], -8, 8, 5, r), 25, 32
    yield "er_w7", I.erdos_renyi_quio(600, 8.0, -3, 3, 10, 10, r), 25, 32
    yield "squares_w41", I.random_huio(500, 1500, [1, 2], -20, 20, 6, r), 25, 32
    yield "er_w128", I.erdos_renyi_quio(400, 4.0, -64, 63, 7, 7, r), 20, 24
    yield "wide_coefs_64bit", I.random_huio(300, 900, [1, 2, 3], -60, 60, 20000, r), 15, 16
    yield "ml_p5_long_terms", I.multilinear(120, 5, 2), 25, 16
    fixed = I.random_huio(300, 1200, [2, 3], -5, 6, 4, r)
    fixed.lower[::4] = 1
    fixed.upper[::4] = 1
    yield "fixed_vars", fixed, 20, 16
    yield "single_variable", I.from_terms(1, [(3, [0, 0]), (-7, [0])], -5, 6), 30, 8
    yield "hub_rows", hub_huio(r), 20, 16
    yield "uneven_widths", uneven(I.random_huio(300, 1200, [1, 2, 3], -4, 4, 5, r)), 20, 16
    # squared terms with coefficients in {-1, 0, 1}: many values share the smallest dE, so the
    # optimal transition's lowest-value rule decides often (the argmin from the vertex's neighbours)
    yield "squares_ties_w61", I.random_huio(400, 1200, [1, 2], -30, 30, 1, r), 25, 32


@pytest.mark.parametrize("case", list(mo_cases()), ids=lambda c: c[0])
def test_quad_metropolis_and_optimal_transition_against_the_oracle(case):
    name, prob, sweeps, reads = case
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(sweeps)
    for rule, r in ((sa.METROPOLIS, -1.0), (sa.OPT_METROPOLIS, -1.0), (sa.OPT_METROPOLIS, 1.0)):
        say(name, sa.RULE_NAMES[rule], f"r={r} N={prob.n_vars} S={sweeps} R={reads}")
        vs_oracle(f"{name}/{sa.RULE_NAMES[rule]}/r={r}", prob, rule, beta, reads, 700 + rule, instance_id=6, otm_r=r)


@pytest.mark.parametrize("kind", ["heat_bath", "metropolis_otm"])
def test_quad_trace_resume_and_determinism(kind):
    prob = I.cfg2_sparse_quio(n=2000).problem if kind == "heat_bath" else I.cfg3_huio(n=600, m=6000).problem
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(20)
    for rule in (HB if kind == "heat_bath" else (sa.METROPOLIS, sa.OPT_METROPOLIS)):
        say(kind, sa.RULE_NAMES[rule], "trace, resume at sweep 7, repeat")
        z, e, _, h = quad_run(prob, rule, beta, 16, 9, trace=True)
        _, _, ho = P.anneal(rule, beta, 16, 9, trace=True)
        assert np.array_equal(h, ho)
        z1, _, _ = quad_run(prob, rule, beta, 16, 9, s1=7)
        z2, e2, _ = quad_run(prob, rule, beta, 16, 9, init=z1, s0=7)
        assert np.array_equal(z2, z) and np.array_equal(e2, e)
        z3, e3, _ = quad_run(prob, rule, beta, 16, 9)
        assert np.array_equal(z3, z) and np.array_equal(e3, e)


def test_quad_is_chosen_automatically_for_the_sparse_workload_and_rejected_elsewhere():
    prob = I.cfg2_sparse_quio(n=10_000, n_sweeps=2).problem
    beta = sa.auto_schedule(prob, 2)
    _, _, launch = quad_run(prob, sa.HEAT_BATH, beta, 4, 1, lanes=4)
    import torch
    plan = sa.Plan(prob, sa.HEAT_BATH)
    z = torch.empty((4, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(4, dtype=torch.int64, device="cuda")
    plan.run_device(2, 4, 1, z, e, beta=beta, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert plan.last_launch()["lanes_per_update"] == 4
    plan.close()
    r = rng(1)
    for prob, rule in [(I.dense_quio(80, -5, 5, 5, 5, r), sa.HEAT_BATH),
                       (I.erdos_renyi_quio(200, 4.0, -100, 100, 5, 5, r), sa.HEAT_BATH),
                       (I.erdos_renyi_quio(200, 4.0, -100, 100, 5, 5, r), sa.OPT_METROPOLIS),
                       (I.from_terms(2, [(1, [0, 0, 0, 0, 0]), (2, [0, 1])], -3, 3), sa.METROPOLIS),
                       (I.from_terms(3, [(1, [0, 0, 0]), (2, [1, 2]), (-1, [0, 1])], -3, 3), sa.HEAT_BATH)]:
        with pytest.raises(sa.SAError) as ex:
            quad_run(prob, rule, np.full(2, 0.1), 2, 1)
        assert ex.value.code == sa.EINVAL
