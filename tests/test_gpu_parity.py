"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

The bar is bit-exactness of every compared read's final state and int64 energy: both sides follow
the same Philox stream, exact integer energy differences and the same FP64 formulas, so any
difference is a defect (or an exp() ulp difference at an acceptance threshold, which the failure
message would show as a single diverging read).  Small cases compare every read; the measured
configurations are run at full size on the GPU, in the launch configuration the benchmark uses,
and a seeded sample of their reads is recomputed by the oracle one by one.
"""
import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa

pytestmark = pytest.mark.gpu

RULES = [sa.METROPOLIS, sa.HEAT_BATH, sa.OPT_METROPOLIS, sa.HEAT_BATH_CLOSED]


def say(*a):
    print("[gpu-parity]", *a, flush=True)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gpu_run(prob, rule, beta, n_reads, seed, instance_id=0, otm_r=-1.0, init=None, s0=0, s1=0, G=0,
            otm_enum_max=0):
    import torch
    plan = sa.Plan(prob, rule)
    z = torch.empty((n_reads, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(n_reads, dtype=torch.int64, device="cuda")
    zi = None if init is None else torch.as_tensor(np.ascontiguousarray(init, np.int32), device="cuda")
    plan.run_device(len(beta), n_reads, seed, z, e, beta=beta,
                    stream=torch.cuda.current_stream().cuda_stream, instance_id=instance_id,
                    otm_r=otm_r, init_states=zi, sweep_begin=s0, sweep_end=s1, waves_per_replica=G,
                    otm_enum_max=otm_enum_max)
    torch.cuda.synchronize()
    launch = plan.last_launch()
    plan.close()
    return z.cpu().numpy(), e.cpu().numpy(), launch


def assert_same(zg, eg, zo, eo, label):
    bad = [i for i in range(len(eo)) if eg[i] != eo[i] or not np.array_equal(zg[i], zo[i])]
    if bad:
        i = bad[0]
        diff = np.nonzero(zg[i] != zo[i])[0][:8]
        pytest.fail(f"{label}: {len(bad)}/{len(eo)} reads differ; first read {i}: E gpu {eg[i]} "
                    f"oracle {eo[i]}; first differing variables {diff.tolist()}")


def small_cases():
    r = rng(42)
    yield "huio_powers_n150", I.random_huio(150, 900, [1, 2, 3, 4], -7, 9, 5, r), 60, 48, RULES
    yield "cfg1_dense_n100_s200", I.cfg1_dense_quio().problem, 200, 16, RULES
    yield "cfg2_like_n1000", I.cfg2_sparse_quio(n=1000).problem, 40, 64, RULES
    yield "cfg3_like_n300", I.cfg3_huio(n=300, m=3000).problem, 100, 128, RULES
    yield "ml_p30_u1_long_terms", I.multilinear(100, 30, 1), 50, 16, RULES
    yield "fc_p8_u2_high_power", I.fully_connected(30, 8, 2), 60, 16, [sa.METROPOLIS, sa.HEAT_BATH,
                                                                      sa.HEAT_BATH_CLOSED]
    yield "binary_qubo_n200", I.dense_quio(200, 0, 1, 5, 5, r), 40, 32, RULES
    yield "wide_w2001_regs", I.erdos_renyi_quio(64, 6.0, -1000, 1000, 10, 10, r), 12, 8, RULES
    yield "wide_w5001_recompute", I.dense_quio(40, -2500, 2500, 3, 3, r), 6, 4, [sa.HEAT_BATH,
                                                                                   sa.HEAT_BATH_CLOSED]
    yield "linear_w2000001", I.erdos_renyi_quio(80, 5.0, -10 ** 6, 10 ** 6, 3, 3, r), 30, 16, [sa.HEAT_BATH_CLOSED]
    fixed = I.random_huio(90, 300, [1, 2, 3], -4, 4, 4, r)
    fixed.lower[::7] = 2
    fixed.upper[::7] = 2
    yield "fixed_and_unused_vars", I.Problem(fixed.n_vars + 5, fixed.term_ptr, fixed.factor_var,
                                             fixed.coef, np.r_[fixed.lower, [-3] * 5],
                                             np.r_[fixed.upper, [3] * 5]), 30, 16, RULES
    yield "single_variable", I.from_terms(1, [(3, [0, 0]), (-7, [0])], -5, 6), 50, 64, RULES
    yield "dense_int32_couplings_n70", I.dense_quio(70, -20, 20, 1000, 1000, r), 40, 24, RULES
    yield "dense_no_diagonal_n150", I.fully_connected(150, 1, 3), 30, 16, RULES
    yield "many_reads_n50", I.random_huio(50, 200, [2, 3], -3, 3, 3, r), 20, 2048, RULES
    # sparse form with one variable in 300+ terms: its row spans six 64-record chunks (the first
    # chunk prefetched, the rest loaded four at a time, lanes past the end on the zero record)
    hub = I.random_huio(400, 1600, [1, 2, 3], -6, 6, 4, r)
    hub_terms = list(hub.terms()) + [(int(c), [0, i]) for i, c in zip(range(1, 301), r.integers(1, 6, 300))]
    hub_terms += [(2, [0, 5, 9]), (-3, [7, 7, 0]), (1, [0, 0])]
    yield "hub_rows_over_256", I.from_terms(400, hub_terms, -6, 6), 40, 32, RULES
    # coefficients above 2^31 (|z| <= 2000, degree 4): the 64-bit kernels' full 64-bit path
    yield "huio_wide_64bit_coefs", I.random_huio(60, 240, [1, 2, 3, 4], -2000, 2000, 5, r), 10, 8, RULES


@pytest.mark.parametrize("case", list(small_cases()), ids=lambda c: c[0])
def test_small_instances_all_reads(case):
    name, prob, sweeps, reads, rules = case
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(sweeps)
    for rule in rules:
        say(name, sa.RULE_NAMES[rule], f"N={prob.n_vars} S={sweeps} R={reads}")
        zg, eg, launch = gpu_run(prob, rule, beta, reads, seed=1234 + rule, instance_id=3)
        zo, eo = P.anneal(rule, beta, reads, seed=1234 + rule, instance_id=3)
        assert_same(zg, eg, zo, eo, f"{name}/{sa.RULE_NAMES[rule]} {launch}")


@pytest.mark.parametrize("rule", RULES)
def test_cooperating_waves_match_sequential_sweep(rule):
    # G waves per replica update the variables of a window (no shared term) at the same time;
    # the result must equal the sequential index-order sweep for every G
    r = rng(55)
    # a path (each variable couples to the next): most windows hold one variable
    path = I.from_terms(300, [(int(c), [i, i + 1]) for i, c in enumerate(r.integers(-9, 10, 299))]
                        + [(1, [i]) for i in range(0, 300, 7)], -4, 4)
    cases = [("dense", I.dense_quio(90, -5, 5, 10, 10, r)),
             ("er_quio", I.erdos_renyi_quio(700, 5.0, -20, 20, 10, 10, r)),
             ("huio_powers", I.random_huio(400, 1200, [1, 2, 3, 4], -6, 6, 4, r)),
             ("ml_long", I.multilinear(150, 7, 2)),
             ("path", path)]
    for name, prob in cases:
        P = oracle.Poly(prob)
        beta, _, _ = P.schedule(25)
        zo, eo = P.anneal(rule, beta, 12, seed=31)
        for G in (1, 2, 4, 8, 16):
            say("windows", name, sa.RULE_NAMES[rule], "G", G)
            zg, eg, launch = gpu_run(prob, rule, beta, 12, seed=31, G=G)
            # 16 waves only for the variants built that way; the others fall back to 8
            assert launch["waves_per_replica"] == G or (G == 16 and launch["waves_per_replica"] == 8)
            if G == 16 and name == "er_quio":
                assert launch["waves_per_replica"] == 16
            assert_same(zg, eg, zo, eo, f"{name}/{sa.RULE_NAMES[rule]}/G={G} {launch}")


def test_degenerate_instances():
    # terms that cancel (no canonical term: every dE is 0), every variable fixed (no update), and
    # the widest range the ABI accepts (u - l = 2^31 - 2) with one read and one or three sweeps
    cancel = I.from_terms(4, [(3, [0, 1]), (-3, [1, 0]), (2, [2, 2]), (-2, [2, 2])], -3, 4)
    fixed = I.from_terms(3, [(3, [0, 1]), (-2, [1, 2, 2])], 2, 2)
    wide = I.from_terms(2, [(1, [0]), (1, [0, 1]), (-1, [1])], [-2 ** 30, -3], [2 ** 30 - 2, 3])
    beta5 = np.linspace(0.1, 2.0, 5)
    cases = [("cancelling_terms", cancel, beta5, 3, RULES), ("all_fixed", fixed, beta5, 2, RULES),
             ("widest_range_one_sweep", wide, np.array([1e-9]), 1,
              [sa.METROPOLIS, sa.OPT_METROPOLIS, sa.HEAT_BATH_CLOSED]),
             ("widest_range_three_sweeps", wide, np.array([1e-9, 1e-6, 1e-3]), 4,
              [sa.METROPOLIS, sa.OPT_METROPOLIS, sa.HEAT_BATH_CLOSED])]
    for name, prob, beta, reads, rules in cases:
        P = oracle.Poly(prob)
        for rule in rules:
            say("degenerate", name, sa.RULE_NAMES[rule])
            zg, eg, launch = gpu_run(prob, rule, beta, reads, seed=9)
            zo, eo = P.anneal(rule, beta, reads, seed=9)
            assert_same(zg, eg, zo, eo, f"{name}/{sa.RULE_NAMES[rule]} {launch}")
    zg, eg, _ = gpu_run(fixed, sa.HEAT_BATH, beta5, 2, seed=9)
    assert (zg == 2).all() and (eg == -4).all()


def random_instances():
    # seeded small instances across the kernels' paths: narrow and wide ranges (32-bit and 64-bit
    # energy differences, 32-bit and 64-bit coefficients), linear and power terms, fixed
    # variables, short and long rows, exponents up to 4 (every rule takes them)
    r = rng(2718)
    for i in range(24):
        n = int(r.integers(1, 70))
        span = int([1, 3, 20, 300, 5000][i % 5])
        lo = int(r.integers(-span, 1))
        hi = lo + int(r.integers(0, 2 * span + 1))
        prob = I.tiny_random(r, n, lo, hi, int(r.integers(1, 4 * n + 2)), int(r.integers(1, 5)),
                             jmax=int([3, 9, 200][i % 3]), name=f"random{i}")
        prob.lower[r.random(n) < 0.1] = hi    # some variables fixed
        yield f"random{i}_n{n}_w{hi - lo + 1}", prob


@pytest.mark.parametrize("case", list(random_instances()), ids=lambda c: c[0])
def test_random_instances_all_reads(case):
    name, prob = case
    P = oracle.Poly(prob)
    try:
        beta, _, _ = P.schedule(12)
    except oracle.OracleError:
        # no energy scale for the automatic schedule (every variable fixed): a given one
        beta = np.geomspace(0.01, 2.0, 12)
    for rule in RULES:
        say(name, sa.RULE_NAMES[rule])
        zg, eg, launch = gpu_run(prob, rule, beta, 9, seed=404 + rule, instance_id=7)
        zo, eo = P.anneal(rule, beta, 9, seed=404 + rule, instance_id=7)
        assert_same(zg, eg, zo, eo, f"{name}/{sa.RULE_NAMES[rule]} {launch}")


def test_cfg1_full_all_reads():
    w = I.cfg1_dense_quio()
    P = oracle.Poly(w.problem)
    say("cfg1 full", w.name)
    zg, eg, _ = gpu_run(w.problem, w.rule, w.beta, w.n_reads, w.seed)
    zo, eo = P.anneal(w.rule, w.beta, w.n_reads, w.seed)
    assert_same(zg, eg, zo, eo, "cfg1")


def test_state_outside_lds():
    # N * 4 bytes above the 160 KiB LDS of a CU: states live in device memory
    prob = I.erdos_renyi_quio(45_000, 3.0, -5, 5, 10, 10, rng(9))
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(3)
    for rule in RULES:
        say("state_outside_lds", sa.RULE_NAMES[rule])
        zg, eg, launch = gpu_run(prob, rule, beta, 4, seed=5)
        assert launch["state_in_lds"] == 0
        zo, eo = P.anneal(rule, beta, 4, seed=5)
        assert_same(zg, eg, zo, eo, f"outside-LDS/{sa.RULE_NAMES[rule]}")


@pytest.mark.parametrize("rule", RULES)
def test_resume_from_device_states(rule):
    prob = I.cfg3_huio(n=200, m=2000).problem
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(30)
    say("resume", sa.RULE_NAMES[rule])
    z_full, e_full, _ = gpu_run(prob, rule, beta, 32, seed=8)
    z_a, _, _ = gpu_run(prob, rule, beta, 32, seed=8, s1=11)
    z_b, e_b, _ = gpu_run(prob, rule, beta, 32, seed=8, init=z_a, s0=11)
    assert_same(z_b, e_b, z_full, e_full, "resume vs uninterrupted")
    zo, eo = P.anneal(rule, beta, 32, seed=8)
    assert_same(z_full, e_full, zo, eo, "uninterrupted vs oracle")


def test_otm_fixed_r():
    prob = I.cfg3_huio(n=250, m=2500).problem
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(25)
    say("otm r override")
    z0, e0, _ = gpu_run(prob, sa.OPT_METROPOLIS, beta, 32, seed=2, otm_r=0.0)
    zm, em, _ = gpu_run(prob, sa.METROPOLIS, beta, 32, seed=2)
    assert_same(z0, e0, zm, em, "OTM r=0 vs Metropolis")
    for r in (0.5, 1.0):
        zg, eg, _ = gpu_run(prob, sa.OPT_METROPOLIS, beta, 32, seed=2, otm_r=r)
        zo, eo = P.anneal(sa.OPT_METROPOLIS, beta, 32, seed=2, otm_r=r)
        assert_same(zg, eg, zo, eo, f"OTM r={r}")


def test_otm_stationary_point_argmin_matches_enumeration():
    # ranges wider than the enumeration limit take the argmin from the stationary points of the
    # degree <= 4 energy difference; it must be the oracle's enumerated argmin (ties to the
    # smallest value) in every step.  otm_enum_max = 1 forces the path on narrow ranges too.
    r = rng(91)
    cases = [("huio_quartic_w6001", I.random_huio(60, 240, [1, 2, 3, 4], -3000, 3000, 3, r), 20, 16, -1.0, 0),
             ("fc_p4_w4001", I.fully_connected(20, 4, 2000), 12, 8, -1.0, 0),
             ("fc_p3_w20001", I.fully_connected(12, 3, 10000), 12, 8, 0.7, 0),
             ("forced_narrow_ranges", I.cfg3_huio(n=300, m=3000).problem, 30, 32, -1.0, 1),
             ("forced_quartic_w81", I.random_huio(80, 400, [1, 2, 3, 4], -40, 40, 5, r), 30, 32, -1.0, 1),
             ("square_ties", I.from_terms(2, [(3, [0, 0]), (1, [1, 1]), (-1, [0, 1])], -5000, 5000),
              40, 32, 1.0, 0)]
    for name, prob, sweeps, reads, r_fixed, enum_max in cases:
        P = oracle.Poly(prob)
        beta, _, _ = P.schedule(sweeps)
        say("otm stationary", name)
        zg, eg, launch = gpu_run(prob, sa.OPT_METROPOLIS, beta, reads, seed=17, otm_r=r_fixed,
                                 otm_enum_max=enum_max)
        zo, eo = P.anneal(sa.OPT_METROPOLIS, beta, reads, seed=17, otm_r=r_fixed)
        assert_same(zg, eg, zo, eo, f"{name} {launch}")


def test_energy_kernel_and_one_shot_api():
    r = rng(3)
    for dense in (I.dense_quio(130, -50, 50, 10, 10, r), I.dense_quio(75, -9, 9, 500, 30, r)):
        assert sa.Plan(dense, sa.METROPOLIS).info()["dense"] == 1
        Pd = oracle.Poly(dense)
        st = r.integers(dense.lower, dense.upper + 1, size=(9, dense.n_vars)).astype(np.int32)
        assert [int(x) for x in sa.energy(dense, st)] == [Pd.energy(s) for s in st]
    prob = I.cfg3_huio(n=400, m=4000).problem
    P = oracle.Poly(prob)
    states = r.integers(prob.lower, prob.upper + 1, size=(37, prob.n_vars)).astype(np.int32)
    say("sa_energy")
    e = sa.energy(prob, states)
    assert [int(x) for x in e] == [P.energy(s) for s in states]
    beta, _, _ = P.schedule(20)
    say("sa_anneal host buffers")
    z, en = sa.anneal(prob, sa.HEAT_BATH, 20, 24, seed=6, beta=beta, instance_id=9)
    zo, eo = P.anneal(sa.HEAT_BATH, beta, 24, seed=6, instance_id=9)
    assert_same(z, en, zo, eo, "one-shot")
    za, ea = sa.anneal(prob, sa.OPT_METROPOLIS, 20, 8, seed=6)   # automatic schedule
    zo, eo = P.anneal(sa.OPT_METROPOLIS, P.schedule(20)[0], 8, seed=6)
    assert_same(za, ea, zo, eo, "one-shot auto schedule")


def test_repeat_runs_are_identical():
    prob = I.cfg2_sparse_quio(n=2000).problem
    beta = sa.auto_schedule(prob, 30)
    say("determinism")
    a = gpu_run(prob, sa.HEAT_BATH, beta, 64, seed=11)
    b = gpu_run(prob, sa.HEAT_BATH, beta, 64, seed=11)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------------------------------------
# Full-size measured configurations: every read checked for E == E(z); a seeded sample of reads
# recomputed by the oracle.
# ------------------------------------------------------------------------------------------------

def full_size(w, n_sample, label):
    P = oracle.Poly(w.problem)
    beta = w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]
    say(label, "GPU full run", w.name)
    zg, eg, launch = gpu_run(w.problem, w.rule, beta, w.n_reads, w.seed, w.instance_id)
    say(label, "launch", launch)
    for i in range(0, w.n_reads, max(1, w.n_reads // 64)):
        assert int(eg[i]) == P.energy(zg[i]), f"{label}: tracked energy of read {i} is not E(z)"
    ids = np.sort(rng(77).choice(w.n_reads, size=n_sample, replace=False)).astype(np.uint32)
    say(label, "oracle sample", ids.tolist())
    zo, eo = P.anneal_reads(w.rule, beta, ids, w.seed, w.instance_id)
    assert_same(zg[ids], eg[ids], zo, eo, f"{label} sampled reads")


def test_cfg2_full_size_sampled():
    full_size(I.cfg2_sparse_quio(), 8, "cfg2")


def test_cfg2_closed_form_full_size_sampled():
    w = I.cfg2_sparse_quio()
    w.rule = sa.HEAT_BATH_CLOSED
    full_size(w, 16, "cfg2-closed")


@pytest.mark.parametrize("rule", ["otm", "metropolis"])
def test_cfg3_full_size_sampled(rule):
    full_size(I.cfg3_huio(rule=rule), 24, f"cfg3-{rule}")
