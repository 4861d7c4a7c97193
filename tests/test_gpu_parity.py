"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Both sides follow the same Philox stream, exact integer energy differences and FP64 decisions of
the same formulas, so a read's final state and energy agree unless a floating-point decision lies
within rounding of a flip (an exp() ulp, or the order in which heat-bath weights are added).  The
bar (tests/parity.py): at least 99.9 % of the compared reads identical, and every read that parts
traced to its first sweep and variable by per-sweep state hashes, where the oracle's decision
must be within rounding of a flip.  Small cases compare every read; the measured configurations
are run at full size in the benchmark's launch configuration and compared read by read with the
oracle's stored results (tests/golden/full_size_*.txt) or a live oracle sample.
"""
import numpy as np
import pytest

import oracle
from paper_2511_17245_amd import inputs as I
from paper_2511_17245_amd import sa
from tests import parity

pytestmark = pytest.mark.gpu

RULES = [sa.METROPOLIS, sa.HEAT_BATH, sa.OPT_METROPOLIS, sa.HEAT_BATH_CLOSED]


def say(*a):
    print("[gpu-parity]", *a, flush=True)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gpu_run(prob, rule, beta, n_reads, seed, instance_id=0, otm_r=-1.0, init=None, s0=0, s1=0, G=0,
            otm_enum_max=0, trace=False):
    import torch
    plan = sa.Plan(prob, rule)
    z = torch.empty((n_reads, prob.n_vars), dtype=torch.int32, device="cuda")
    e = torch.empty(n_reads, dtype=torch.int64, device="cuda")
    zi = None if init is None else torch.as_tensor(np.ascontiguousarray(init, np.int32), device="cuda")
    n_traced = (s1 if s1 > 0 else len(beta)) - s0
    h = torch.empty(n_reads * n_traced, dtype=torch.int64, device="cuda") if trace else None
    plan.run_device(len(beta), n_reads, seed, z, e, beta=beta,
                    stream=torch.cuda.current_stream().cuda_stream, instance_id=instance_id,
                    otm_r=otm_r, init_states=zi, sweep_begin=s0, sweep_end=s1, waves_per_replica=G,
                    otm_enum_max=otm_enum_max, trace=h)
    torch.cuda.synchronize()
    launch = plan.last_launch()
    plan.close()
    out = (z.cpu().numpy(), e.cpu().numpy(), launch)
    if trace:
        out += (h.cpu().numpy().view(np.uint64).reshape(n_reads, n_traced),)
    return out


def assert_same(zg, eg, zo, eo, label):
    """Bit-exact equality of two GPU runs (same kernels, same stream: nothing may differ)."""
    bad = [i for i in range(len(eo)) if eg[i] != eo[i] or not np.array_equal(zg[i], zo[i])]
    if bad:
        i = bad[0]
        diff = np.nonzero(zg[i] != zo[i])[0][:8]
        pytest.fail(f"{label}: {len(bad)}/{len(eo)} reads differ; first read {i}: E {eg[i]} vs "
                    f"{eo[i]}; first differing variables {diff.tolist()}")


def explainer(prob, P, rule, beta, seed, instance_id=0, otm_r=-1.0, G=0, otm_enum_max=0):
    """explain(i) for parity.check: traces read i of this GPU launch against the oracle."""
    def explain(i):
        kw = dict(instance_id=instance_id, otm_r=otm_r, G=G, otm_enum_max=otm_enum_max)
        _, _, _, h = gpu_run(prob, rule, beta, i + 1, seed, trace=True, **kw)

        def after(s, z):
            zz, _, _ = gpu_run(prob, rule, beta, i + 1, seed, init=np.tile(z, (i + 1, 1)), s0=s, s1=s + 1, **kw)
            return zz[i]
        return parity.localise(P, rule, beta, seed, instance_id, i, h[i], after, otm_r)
    return explain


def vs_oracle(label, prob, P, rule, beta, zg, eg, zo, eo, seed, instance_id=0, otm_r=-1.0, G=0,
              otm_enum_max=0):
    """GPU reads (zg, eg) against the oracle's (zo, eo) at the parity bar."""
    parity.check(label, len(eo), lambda i: eg[i] == eo[i] and np.array_equal(zg[i], zo[i]),
                 explainer(prob, P, rule, beta, seed, instance_id, otm_r, G, otm_enum_max))


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
    # the serving stream's dense heat-bath shape (width 2001, squared variables) over a longer
    # schedule: most late draws have only a few lanes of nonzero weight
    yield "dense_w2001_cold", I.dense_quio(48, -1000, 1000, 10, 10, r), 40, 8, [sa.HEAT_BATH]


@pytest.mark.parametrize("case", list(small_cases()), ids=lambda c: c[0])
def test_small_instances_all_reads(case):
    name, prob, sweeps, reads, rules = case
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(sweeps)
    for rule in rules:
        say(name, sa.RULE_NAMES[rule], f"N={prob.n_vars} S={sweeps} R={reads}")
        zg, eg, launch = gpu_run(prob, rule, beta, reads, seed=1234 + rule, instance_id=3)
        zo, eo = P.anneal(rule, beta, reads, seed=1234 + rule, instance_id=3)
        vs_oracle(f"{name}/{sa.RULE_NAMES[rule]} {launch}", prob, P, rule, beta, zg, eg, zo, eo,
                  1234 + rule, instance_id=3)


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
            vs_oracle(f"{name}/{sa.RULE_NAMES[rule]}/G={G} {launch}", prob, P, rule, beta, zg, eg, zo, eo,
                      31, G=G)


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
            vs_oracle(f"{name}/{sa.RULE_NAMES[rule]} {launch}", prob, P, rule, beta, zg, eg, zo, eo, 9)
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
        vs_oracle(f"{name}/{sa.RULE_NAMES[rule]} {launch}", prob, P, rule, beta, zg, eg, zo, eo,
                  404 + rule, instance_id=7)


def test_cfg1_full_all_reads():
    w = I.cfg1_dense_quio()
    P = oracle.Poly(w.problem)
    say("cfg1 full", w.name)
    zg, eg, _ = gpu_run(w.problem, w.rule, w.beta, w.n_reads, w.seed)
    zo, eo = P.anneal(w.rule, w.beta, w.n_reads, w.seed)
    vs_oracle("cfg1", w.problem, P, w.rule, w.beta, zg, eg, zo, eo, w.seed)
    assert all(int(eg[i]) == P.energy(zg[i]) for i in range(w.n_reads))


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
        vs_oracle(f"outside-LDS/{sa.RULE_NAMES[rule]}", prob, P, rule, beta, zg, eg, zo, eo, 5)


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
    vs_oracle("uninterrupted vs oracle", prob, P, rule, beta, z_full, e_full, zo, eo, 8)


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
        vs_oracle(f"OTM r={r}", prob, P, sa.OPT_METROPOLIS, beta, zg, eg, zo, eo, 2, otm_r=r)


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
        vs_oracle(f"{name} {launch}", prob, P, sa.OPT_METROPOLIS, beta, zg, eg, zo, eo, 17, otm_r=r_fixed,
                  otm_enum_max=enum_max)


def _quartic_terms(var, c):
    """Terms c[m] z_var^m, m = 1..4 (zero coefficients left out)."""
    return [(int(c[m]), [var] * m) for m in range(1, 5) if c[m] != 0]


def _expand(roots_sq, scale=1, tilt=0):
    """Coefficients of scale * prod_{r in roots_sq} (v - r)^2 + tilt * v (two roots: a quartic)."""
    poly = [1]
    for r in roots_sq:
        for _ in range(2):
            nxt = [0] * (len(poly) + 1)
            for i, a in enumerate(poly):
                nxt[i] -= r * a
                nxt[i + 1] += a
            poly = nxt
    c = [scale * a for a in poly] + [0] * (5 - len(poly))
    c[1] += tilt
    return c


def _bound(terms, lo, hi):
    M = [max(abs(a), abs(b)) for a, b in zip(lo, hi)]
    tot = 0
    for coef, vs in terms:
        t = abs(coef)
        for v in vs:
            t *= M[v]
        tot += t
    return tot


def test_otm_wide_argmin_on_adversarial_quartics():
    # The optimal transition over ranges wider than the enumeration limit (forward-difference sign
    # changes, exact by construction) on quartics built to defeat approximate root finding: equal
    # double minima (ties to the lower one), nearly double minima tilted by +-1, concave quartics
    # (minimum at an end), coefficients summing to just under the 2^62 energy bound, and a
    # quadratic over a range of 2^31 - 1 values whose minimiser is known in closed form.  At r = 1
    # every step takes the argmin, so after the first sweep each variable sits at the minimiser of
    # its own quartic; the oracle enumerates the range.
    r = rng(92)
    M = 6000
    terms, expect = [], []
    for v in range(12):
        kind = v % 4
        a, b = sorted(int(x) for x in r.integers(-M + 10, M - 10, size=2))
        if kind == 0:                       # (v-a)^2 (v-b)^2: equal minima at a and b, tie -> a
            c, want = _expand([a, b]), a
        elif kind == 1:                     # (v-a)^2 (v-a-1)^2 + t v
            t = int(r.integers(-1, 2))
            c = _expand([a, a + 1], tilt=t)
            want = a if t >= 0 else a + 1
        elif kind == 2:                     # -(v-a)^2 (v-b)^2: concave ends; the larger end value
            c, want = _expand([a, b], scale=-1), None
        else:                               # double minimum at one point
            c, want = _expand([a, a]), a
        terms += _quartic_terms(v, c)
        expect.append(want)
    lo, hi = [-M] * 12, [M] * 12
    assert _bound(terms, lo, hi) < 2 ** 62
    quartics = I.from_terms(12, terms, lo, hi, name="adversarial quartics")
    # near the bound: one variable, a double well (c4 > 0, c2 < 0, c1 and c3 of random sign) whose
    # terms take random shares of 0.98 * 2^62 at the range's ends
    Mb = 9000
    s4, s2, s3 = r.uniform(0.40, 0.55), r.uniform(0.35, 0.42), r.uniform(0.0, 0.02)
    share = [0.98 - s4 - s2 - s3, s2, s3, s4]
    sign = [0, int(r.choice([-1, 1])), -1, int(r.choice([-1, 1])), 1]
    c = [0] + [max(1, int(share[m - 1] * 2 ** 62) // Mb ** m) * sign[m] for m in range(1, 5)]
    near = I.from_terms(1, _quartic_terms(0, c), -Mb, Mb, name="quartic at the bound")
    assert 0.9 * 2 ** 62 < _bound(_quartic_terms(0, c), [-Mb], [Mb]) < 2 ** 62
    beta = np.full(3, 0.5)
    for name, prob, want in (("adversarial quartics", quartics, expect), ("quartic at the bound", near, [None])):
        P = oracle.Poly(prob)
        say("otm adversarial", name)
        zg, eg, launch = gpu_run(prob, sa.OPT_METROPOLIS, beta, 16, seed=5, otm_r=1.0)
        zo, eo = P.anneal(sa.OPT_METROPOLIS, beta, 16, seed=5, otm_r=1.0)
        assert np.array_equal(zg, zo) and np.array_equal(eg, eo), name
        for k, w in enumerate(want):
            if w is not None:
                assert np.all(zg[:, k] == w), (name, k, w, zg[:, k])
    # the widest range: E = z^2 - 2 t z over [-(2^30 - 1), 2^30 - 1] (2^31 - 1 values): argmin t,
    # and for a tilt of exactly half a step both t and t + 1 give the same energy: the lower wins
    t = 123456789
    for c1, want in ((-2 * t, t), (-(2 * t + 1), t)):
        huge = I.from_terms(1, [(1, [0, 0]), (c1, [0])], -(2 ** 30 - 1), 2 ** 30 - 1, name="huge quadratic")
        say("otm huge range", c1)
        zg, eg, launch = gpu_run(huge, sa.OPT_METROPOLIS, np.full(2, 0.5), 8, seed=6, otm_r=1.0)
        assert np.all(zg[:, 0] == want), zg[:, 0]
        assert np.all(eg == want * want + c1 * want)


def test_dense_coefficient_cache_equals_the_row_product():
    # A dense QUIO annealed one wavefront per replica keeps the coefficient cache c1 of Sec. 3.2 in
    # LDS, updated on every accepted move; two wavefronts per replica recompute the row product at
    # every visit.  Both must give the same reads (same integers), and every tracked energy must be
    # the energy of its final state, for each rule and for int8 and int32 couplings.
    r = rng(93)
    cases = [("int8_w16", I.dense_quio(100, 0, 15, 10, 10, r)),
             ("int32_w41", I.dense_quio(300, -20, 20, 3000, 700, r)),
             ("n1024_w3", I.dense_quio(1024, -1, 1, 20, 20, r))]
    for name, prob in cases:
        P = oracle.Poly(prob)
        beta, _, _ = P.schedule(40)
        for rule in (sa.METROPOLIS, sa.HEAT_BATH, sa.OPT_METROPOLIS):
            say("dense cache", name, sa.RULE_NAMES[rule])
            zc, ec, lc = gpu_run(prob, rule, beta, 24, seed=13, G=1)
            assert lc["kernel_variant"] // 1000 % 10 == 5, lc          # the cached variant ran
            zr, er, lr = gpu_run(prob, rule, beta, 24, seed=13, G=2)
            assert lr["kernel_variant"] // 1000 % 10 != 5, lr
            assert_same(zc, ec, zr, er, f"{name} {sa.RULE_NAMES[rule]} cache vs row product")
            assert all(int(ec[i]) == P.energy(zc[i]) for i in range(24))


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
    vs_oracle("one-shot", prob, P, sa.HEAT_BATH, beta, z, en, zo, eo, 6, instance_id=9)
    za, ea = sa.anneal(prob, sa.OPT_METROPOLIS, 20, 8, seed=6)   # automatic schedule
    zo, eo = P.anneal(sa.OPT_METROPOLIS, P.schedule(20)[0], 8, seed=6)
    vs_oracle("one-shot auto schedule", prob, P, sa.OPT_METROPOLIS, P.schedule(20)[0], za, ea, zo, eo, 6)


def test_repeat_runs_are_identical():
    prob = I.cfg2_sparse_quio(n=2000).problem
    beta = sa.auto_schedule(prob, 30)
    say("determinism")
    a = gpu_run(prob, sa.HEAT_BATH, beta, 64, seed=11)
    b = gpu_run(prob, sa.HEAT_BATH, beta, 64, seed=11)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ------------------------------------------------------------------------------------------------
# Full-size measured configurations, in the benchmark's launch configuration: every read checked
# for E == E(z) and compared with the oracle's stored result for that read
# (tests/golden/make_full_size.py wrote them with the oracle alone).
# ------------------------------------------------------------------------------------------------

def full_size(name):
    from tests.golden import make_full_size as M
    gold = M.read(name)
    for label, w in M.workloads(name):
        hdr, eo, ho = gold[label]
        P = oracle.Poly(w.problem)
        beta = M.schedule(P, w)
        assert hdr["beta_sha256"] == M.beta_sha(beta), f"{label}: stored results were made with another schedule"
        say(label, "GPU full run", w.name)
        zg, eg, launch = gpu_run(w.problem, w.rule, beta, w.n_reads, w.seed, w.instance_id)
        say(label, "launch", launch)
        bad = [i for i in range(w.n_reads) if int(eg[i]) != P.energy(zg[i])]
        assert not bad, f"{label}: tracked energy is not E(z) for reads {bad[:8]}"
        hg = parity.state_hashes(zg)
        parity.check(label, w.n_reads, lambda i: eg[i] == eo[i] and hg[i] == ho[i],
                     explainer(w.problem, P, w.rule, beta, w.seed, w.instance_id))


def test_cfg2_full_size_all_reads():
    full_size("cfg2")


def test_cfg2_closed_form_full_size_all_reads():
    full_size("cfg2-closed")


@pytest.mark.parametrize("rule", ["otm", "metropolis"])
def test_cfg3_full_size_all_reads(rule):
    full_size(f"cfg3-{rule}")


def test_traced_hashes_match_the_oracle():
    # the per-sweep state hashes of the GPU (trace_hashes) equal the oracle's, every rule
    r = rng(606)
    prob = I.random_huio(120, 700, [1, 2, 3], -6, 8, 4, r)
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(15)
    for rule in RULES:
        say("trace", sa.RULE_NAMES[rule])
        zg, eg, _, hg = gpu_run(prob, rule, beta, 10, seed=3, instance_id=2, trace=True)
        zo, eo, ho = P.anneal(rule, beta, 10, seed=3, instance_id=2, trace=True)
        assert np.array_equal(hg, ho), sa.RULE_NAMES[rule]
        # a resumed range reports the hashes of its own sweeps
        z1, _, _ = gpu_run(prob, rule, beta, 10, seed=3, instance_id=2, s1=6)
        _, _, _, h2 = gpu_run(prob, rule, beta, 10, seed=3, instance_id=2, init=z1, s0=6, trace=True)
        assert np.array_equal(h2, ho[:, 6:])
    # host-buffer form of the option
    plan = sa.Plan(prob, sa.HEAT_BATH)
    z, e, h = plan.run(15, 10, 3, beta=beta, instance_id=2, trace=True)
    plan.close()
    _, _, ho = P.anneal(sa.HEAT_BATH, beta, 10, seed=3, instance_id=2, trace=True)
    assert np.array_equal(h, ho)


def test_localisation_finds_a_planted_parting():
    # the tracing machinery itself: a run restarted at sweep 4 from a state that differs in one
    # variable parts from the unperturbed chain; the GPU's per-sweep hashes follow the perturbed
    # chain exactly (as the oracle runs it), so the first differing hash names the sweep where the
    # chains part
    r = rng(607)
    prob = I.erdos_renyi_quio(200, 4.0, -9, 9, 5, 5, r)
    P = oracle.Poly(prob)
    beta, _, _ = P.schedule(10)
    rule = sa.METROPOLIS
    z4, _ = P.anneal(rule, beta, 1, seed=8, s_end=4)
    z_alt = z4.copy()
    z_alt[0, 7] = -9 if z_alt[0, 7] != -9 else 9
    _, _, _, hg = gpu_run(prob, rule, beta, 1, seed=8, init=z_alt, s0=4, trace=True)
    _, _, ho_alt = P.anneal(rule, beta, 1, seed=8, s_begin=4, z_init=z_alt, trace=True)
    _, _, ho = P.anneal(rule, beta, 1, seed=8, trace=True)
    assert np.array_equal(hg, ho_alt)
    parted = np.nonzero(hg[0] != ho[0, 4:])[0]
    assert parted.size > 0
    # localise() reports that first sweep and the first differing variable after it
    def after(s, z):
        zz, _, _ = gpu_run(prob, rule, beta, 1, seed=8, init=z_alt if s == 4 else z[None, :], s0=s, s1=s + 1)
        return zz[0]
    info = parity.localise(P, rule, beta, 8, 0, 0, np.r_[ho[0, :4], hg[0]], after)
    assert info is not None and info["sweep"] == 4 + int(parted[0])
