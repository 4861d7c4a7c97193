"""Seeded synthetic problem generators.

This module is shared by the GPU path's tests/bench and by the CPU oracle's
tests.  It only *draws* problems (raw, unmerged polynomial terms plus integer
bounds); it holds none of the annealing arithmetic.  Everything is driven by
``numpy.random.Generator(PCG64(seed))`` so that a (generator, seed) pair names
an input exactly.

Raw problem format (the C ABI's ``sa_instance`` + ``sa_bounds``):

* ``term_ptr``  int64[n_terms + 1]: term t owns ``factor_var[term_ptr[t]:term_ptr[t+1]]``.
* ``factor_var`` int32: the variable indices of the term's factors; a power
  z_i^m is written as index i repeated m times.  Order inside a term is free and
  equal multisets may repeat (both sides merge them, Sec. 2 of the paper).
* ``coef`` int64[n_terms]: the term's integer coefficient (zeros allowed).
* ``lower``/``upper`` int32[n_vars]: the integer box l_i <= z_i <= u_i.

The workloads follow the paper's benchmark families (Sec. 4: fully connected,
multilinear and random-interaction models, with coefficients scaled to
integers) and the five measured configurations: dense QUIO N=100, sparse
Erdos-Renyi QUIO N=10^4, random HUIO N=2000, a 512-instance mixed batch and a
Poisson request stream.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

GEN_SEED_BASE = 251117245      # generator seed of workload c is GEN_SEED_BASE + c
PHILOX_SEED_BASE = 0x5A000000  # annealing (Philox key) seed of workload c is PHILOX_SEED_BASE + c


@dataclasses.dataclass
class Problem:
    """A raw integer polynomial problem: E(z) = sum_t coef[t] * prod(z[f] for f in term t)."""

    n_vars: int
    term_ptr: np.ndarray
    factor_var: np.ndarray
    coef: np.ndarray
    lower: np.ndarray
    upper: np.ndarray
    name: str = ""

    def __post_init__(self):
        self.term_ptr = np.ascontiguousarray(self.term_ptr, dtype=np.int64)
        self.factor_var = np.ascontiguousarray(self.factor_var, dtype=np.int32)
        self.coef = np.ascontiguousarray(self.coef, dtype=np.int64)
        self.lower = np.ascontiguousarray(self.lower, dtype=np.int32)
        self.upper = np.ascontiguousarray(self.upper, dtype=np.int32)

    @property
    def n_terms(self) -> int:
        return int(self.coef.shape[0])

    @property
    def n_factors(self) -> int:
        return int(self.factor_var.shape[0])

    def terms(self):
        """Yield (coef, tuple_of_factor_vars) for every raw term (slow; small problems only)."""
        for t in range(self.n_terms):
            a, b = int(self.term_ptr[t]), int(self.term_ptr[t + 1])
            yield int(self.coef[t]), tuple(int(x) for x in self.factor_var[a:b])


def from_terms(n_vars: int, terms: Sequence, lower, upper, name: str = "") -> Problem:
    """Build a Problem from a list of (coef, [var, var, ...]) pairs."""
    ptr = [0]
    fv: List[int] = []
    cf: List[int] = []
    for c, vs in terms:
        fv.extend(int(v) for v in vs)
        ptr.append(len(fv))
        cf.append(int(c))
    lo = np.broadcast_to(np.asarray(lower, dtype=np.int32), (n_vars,)).copy()
    up = np.broadcast_to(np.asarray(upper, dtype=np.int32), (n_vars,)).copy()
    return Problem(n_vars, np.asarray(ptr, np.int64), np.asarray(fv, np.int32),
                   np.asarray(cf, np.int64), lo, up, name)


def _assemble(n_vars, blocks, lower, upper, name) -> Problem:
    """blocks: list of (coef[M], factors[M, d]) with a fixed degree d per block."""
    ptrs, fvs, cfs = [], [], []
    off = 0
    for coef, fac in blocks:
        coef = np.asarray(coef, np.int64)
        fac = np.asarray(fac, np.int32)
        m, d = fac.shape
        ptrs.append(off + d * np.arange(m, dtype=np.int64))
        fvs.append(fac.reshape(-1))
        cfs.append(coef)
        off += m * d
    term_ptr = np.concatenate(ptrs + [np.asarray([off], np.int64)])
    lo = np.broadcast_to(np.asarray(lower, np.int32), (n_vars,)).copy()
    up = np.broadcast_to(np.asarray(upper, np.int32), (n_vars,)).copy()
    return Problem(n_vars, term_ptr, np.concatenate(fvs), np.concatenate(cfs), lo, up, name)


def _uniform_int(rng, lo, hi, size, nonzero=False):
    """Integers uniform on {lo..hi} (or on {lo..hi} minus {0} when nonzero)."""
    if not nonzero:
        return rng.integers(lo, hi + 1, size=size, dtype=np.int64)
    vals = np.array([v for v in range(lo, hi + 1) if v != 0], np.int64)
    return vals[rng.integers(0, len(vals), size=size)]


# ----------------------------------------------------------------------------------------------
# Problem families
# ----------------------------------------------------------------------------------------------

def dense_quio(n, lo, hi, jmax, hmax, rng, name="dense_quio") -> Problem:
    """One coefficient per unordered pair i <= j (diagonal z_i^2 included) plus a linear term
    per variable; all iid uniform integers (QUIO, Sec. 2)."""
    iu, ju = np.triu_indices(n)
    jc = _uniform_int(rng, -jmax, jmax, iu.shape[0])
    hc = _uniform_int(rng, -hmax, hmax, n)
    return _assemble(n, [(hc, np.arange(n).reshape(n, 1)),
                         (jc, np.stack([iu, ju], axis=1))], lo, hi, name)


def erdos_renyi_quio(n, mean_degree, lo, hi, jmax, hmax, rng, name="er_quio") -> Problem:
    """Sparse QUIO on an Erdos-Renyi graph G(n, p = mean_degree/(n-1)); no diagonal terms, so
    the energy is multilinear in every variable."""
    n_pairs = n * (n - 1) // 2
    p = mean_degree / (n - 1)
    m = int(rng.binomial(n_pairs, p))
    flat = np.sort(rng.choice(n_pairs, size=m, replace=False))
    # invert the row-major enumeration of pairs (i < j)
    i = (n - 2 - np.floor(np.sqrt(-8.0 * flat + 4.0 * n * (n - 1) - 7) / 2.0 - 0.5)).astype(np.int64)
    start = i * (2 * n - i - 1) // 2
    j = flat - start + i + 1
    bad = (j <= i) | (j >= n)
    if np.any(bad):  # floating-point edge of the inversion; repair exactly
        for q in np.nonzero(bad)[0]:
            f = int(flat[q])
            ii = 0
            while (ii + 1) * (2 * n - ii - 2) // 2 <= f:
                ii += 1
            i[q] = ii
            j[q] = f - ii * (2 * n - ii - 1) // 2 + ii + 1
    jc = _uniform_int(rng, -jmax, jmax, m, nonzero=True)
    hc = _uniform_int(rng, -hmax, hmax, n)
    return _assemble(n, [(hc, np.arange(n).reshape(n, 1)),
                         (jc, np.stack([i, j], axis=1))], lo, hi, name)


def random_huio(n, n_monomials, degrees, lo, hi, jmax, rng, name="random_huio",
                nonzero=False) -> Problem:
    """Random HUIO: each monomial draws its degree uniformly from `degrees` and that many variable
    indices uniformly *with replacement* (so powers z_i^m occur), with an iid integer coefficient
    (the random-interaction model of Sec. 4)."""
    degs = np.asarray(degrees)[rng.integers(0, len(degrees), size=n_monomials)]
    blocks = []
    for d in sorted(set(int(x) for x in degs)):
        cnt = int(np.sum(degs == d))
        fac = rng.integers(0, n, size=(cnt, d), dtype=np.int64)
        blocks.append((_uniform_int(rng, -jmax, jmax, cnt, nonzero=nonzero), fac))
    return _assemble(n, blocks, lo, hi, name)


def fully_connected(n, p, u, name=None) -> Problem:
    """Fully connected model of Sec. 4 scaled to integer coefficients by S = u^max(p,2):
    p >= 2: E = -u^(p-2) sum_{i<j} z_i z_j - sum_i z_i^p;  p = 1: E = -sum_{i<j} z_i z_j - u sum_i z_i,
    with -u <= z_i <= u.  Ground-state energy -S N(N+1)/2."""
    iu, ju = np.triu_indices(n, k=1)
    if p >= 2:
        pair_c = -(u ** (p - 2))
        self_c = -1
    else:
        pair_c = -1
        self_c = -u
    blocks = [(np.full(iu.shape[0], pair_c, np.int64), np.stack([iu, ju], axis=1)),
              (np.full(n, self_c, np.int64), np.repeat(np.arange(n).reshape(n, 1), p, axis=1))]
    return _assemble(n, blocks, -u, u, name or f"fc_p{p}_u{u}")


def fully_connected_scale(p, u) -> int:
    return u ** max(p, 2)


def multilinear(n, p, u, name=None) -> Problem:
    """Multilinear model of Sec. 4 with periodic boundary, scaled by u^p:
    E = -sum_i z_i z_{i+1} ... z_{i+p-1}, -u <= z_i <= u.  Ground-state energy -N u^p."""
    idx = (np.arange(n).reshape(n, 1) + np.arange(p).reshape(1, p)) % n
    return _assemble(n, [(np.full(n, -1, np.int64), idx)], -u, u, name or f"ml_p{p}_u{u}")


def random_interaction(n, p, u, n_terms, rng, kmax=100, name=None) -> Problem:
    """Random-interaction model of Sec. 4 with integer coefficients: n_terms monomials of degree p,
    indices drawn with repetition, coefficient uniform on {-kmax..kmax} minus {0}."""
    fac = rng.integers(0, n, size=(n_terms, p), dtype=np.int64)
    return _assemble(n, [(_uniform_int(rng, -kmax, kmax, n_terms, nonzero=True), fac)],
                     -u, u, name or f"ri_p{p}_u{u}")


# ----------------------------------------------------------------------------------------------
# Measured configurations
# ----------------------------------------------------------------------------------------------

RULES = {"metropolis": 0, "heat_bath": 1, "otm": 2, "heat_bath_closed": 3}


@dataclasses.dataclass
class Workload:
    problem: Problem
    rule: int
    n_sweeps: int
    n_reads: int
    seed: int
    instance_id: int = 0
    beta: Optional[np.ndarray] = None   # explicit schedule, or None for the automatic one
    name: str = ""


def cfg1_beta(n_sweeps: int) -> np.ndarray:
    """The dense configuration's given schedule, geometric from beta 0.01 to 10 over n_sweeps."""
    s = np.arange(n_sweeps, dtype=np.float64)
    return 0.01 * np.power(1000.0, s / max(n_sweeps - 1, 1))


def cfg1_dense_quio() -> Workload:
    """Dense QUIO, N=100, z in [0,15], J_ij (i<=j) and h_i uniform on {-10..10}; Metropolis with
    geometric beta 0.01 -> 10 over 1000 sweeps, 16 reads."""
    rng = np.random.Generator(np.random.PCG64(GEN_SEED_BASE + 1))
    prob = dense_quio(100, 0, 15, 10, 10, rng, name="cfg1_dense_quio_n100")
    beta = cfg1_beta(1000)
    return Workload(prob, RULES["metropolis"], 1000, 16, PHILOX_SEED_BASE + 1, 0, beta,
                    "dense QUIO N=100 [0,15] Metropolis 1000 sweeps 16 reads")


def cfg2_sparse_quio(n=10_000, n_sweeps=2000, n_reads=256) -> Workload:
    """Sparse QUIO, N=10^4, z in [-50,50], Erdos-Renyi mean degree 8, J in {-10..10}\\{0},
    h in {-20..20}; heat bath, automatic schedule, 2000 sweeps, 256 reads."""
    rng = np.random.Generator(np.random.PCG64(GEN_SEED_BASE + 2))
    prob = erdos_renyi_quio(n, 8.0, -50, 50, 10, 20, rng, name=f"cfg2_er_quio_n{n}")
    return Workload(prob, RULES["heat_bath"], n_sweeps, n_reads, PHILOX_SEED_BASE + 2, 0, None,
                    f"sparse ER QUIO N={n} [-50,50] deg 8 heat bath {n_sweeps} sweeps {n_reads} reads")


def cfg3_huio(rule="otm", n=2000, m=20_000, n_sweeps=1000, n_reads=1024) -> Workload:
    """HUIO, N=2000, z in [0,100], 20,000 monomials of degree 2-4 drawn with replacement,
    J in {-5..5}; OTM or Metropolis, automatic schedule, 1000 sweeps, 1024 reads."""
    rng = np.random.Generator(np.random.PCG64(GEN_SEED_BASE + 3))
    prob = random_huio(n, m, [2, 3, 4], 0, 100, 5, rng, name=f"cfg3_huio_n{n}")
    return Workload(prob, RULES[rule], n_sweeps, n_reads, PHILOX_SEED_BASE + 3, 0, None,
                    f"HUIO N={n} [0,100] {m} monomials deg 2-4 {rule} {n_sweeps} sweeps {n_reads} reads")


def cfg4_batch(n_instances=512, n_reads=32, n_sweeps=1000, n_min=50, n_max=5000,
               w_min=2, w_max=1000) -> List[Workload]:
    """Mixed batch: instance i has N log-uniform in [50,5000] and width W log-uniform in [2,1000]
    (bounds -floor(W/2) .. -floor(W/2)+W-1); even i is ER QUIO (degree 8, J, h in {-10..10}),
    odd i is HUIO (10 N monomials of degree 2-4 with replacement, J in {-10..10}); the rule
    cycles Metropolis / heat bath / OTM with i; automatic schedule, 1000 sweeps, 32 reads."""
    rng = np.random.Generator(np.random.PCG64(GEN_SEED_BASE + 4))
    out = []
    for i in range(n_instances):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        w = int(round(math.exp(rng.uniform(math.log(w_min), math.log(w_max)))))
        lo = -(w // 2)
        hi = lo + w - 1
        if i % 2 == 0:
            prob = erdos_renyi_quio(n, min(8.0, n - 1.0), lo, hi, 10, 10, rng, name=f"b{i}_quio")
        else:
            prob = random_huio(n, 10 * n, [2, 3, 4], lo, hi, 10, rng, name=f"b{i}_huio")
        out.append(Workload(prob, i % 3, n_sweeps, n_reads, PHILOX_SEED_BASE + 4, i, None,
                            f"batch item {i}"))
    return out


_DENSE_POOL = {}


def cfg5_request(req_id: int, dense_n=4096, dense_pool=4) -> Workload:
    """Request `req_id` of the serving stream: 90% are HUIO drawn as the N=2000 config (rule OTM
    for even ids, Metropolis for odd ids; 16 reads, 1000 sweeps); 10% are dense QUIO N=4096,
    z in [-1000,1000], J and h in {-10..10}, heat bath, 16 reads, 100 sweeps.  Dense requests draw
    their instance from a pool of `dense_pool` seeded instances (their own seed and instance id
    still make every request a distinct run)."""
    rng = np.random.Generator(np.random.PCG64([GEN_SEED_BASE + 5, req_id]))
    if rng.uniform() < 0.9:
        prob = random_huio(2000, 20_000, [2, 3, 4], 0, 100, 5, rng, name=f"req{req_id}_huio")
        rule = RULES["otm"] if req_id % 2 == 0 else RULES["metropolis"]
        return Workload(prob, rule, 1000, 16, PHILOX_SEED_BASE + 5 + req_id, req_id, None, f"req {req_id} A")
    key = (dense_n, req_id % dense_pool)
    if key not in _DENSE_POOL:
        drng = np.random.Generator(np.random.PCG64([GEN_SEED_BASE + 5, 1 << 40, key[1]]))
        _DENSE_POOL[key] = dense_quio(dense_n, -1000, 1000, 10, 10, drng, name=f"dense{key[1]}")
    return Workload(_DENSE_POOL[key], RULES["heat_bath"], 100, 16, PHILOX_SEED_BASE + 5 + req_id, req_id,
                    None, f"req {req_id} B")


def cfg5_arrivals(n_requests: int, rate_per_s: float, seed=0x5A0005A0) -> np.ndarray:
    """Poisson arrival times (seconds) of the serving stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n_requests))


def tiny_random(rng, n, lo, hi, n_terms, max_deg, jmax=5, name="tiny") -> Problem:
    """Small random polynomial for exhaustive tests: n variables, n_terms monomials of degree
    1..max_deg drawn with replacement (powers allowed), coefficients in {-jmax..jmax}."""
    terms = []
    for _ in range(n_terms):
        d = int(rng.integers(1, max_deg + 1))
        terms.append((int(rng.integers(-jmax, jmax + 1)), rng.integers(0, n, size=d).tolist()))
    return from_terms(n, terms, lo, hi, name)
