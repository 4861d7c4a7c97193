"""The stored full-size oracle results (tests/golden/full_size_*.txt) are current and correct.

Each file records the sha256 of the oracle source and of the inverse-temperature array it was
made with; a change of either makes the file stale (regenerate it with the command in its
header).  A few reads of each file are recomputed by the oracle here."""
import numpy as np
import pytest

import oracle
from tests.golden import make_full_size as M

NAMES = ["cfg2", "cfg2-closed", "cfg3-otm", "cfg3-metropolis", "cfg4", "cfg5"]


@pytest.mark.parametrize("name", NAMES)
def test_stored_results_are_current(name):
    gold = M.read(name)
    labels = [label for label, _ in M.workloads(name)]
    assert sorted(gold) == sorted(labels)
    for label, w in M.workloads(name):
        hdr, e, h = gold[label]
        assert hdr["oracle_sha256"] == M.oracle_sha(), f"{name}: made with another oracle source"
        assert int(hdr["reads"]) == w.n_reads == len(e) == len(h)
        assert int(hdr["sweeps"]) == w.n_sweeps and int(hdr["rule"]) == w.rule
        P = oracle.Poly(w.problem)
        assert hdr["beta_sha256"] == M.beta_sha(M.schedule(P, w))


@pytest.mark.parametrize("name", ["cfg2-closed", "cfg3-otm", "cfg3-metropolis", "cfg5"])
def test_stored_results_recompute(name):
    # a seeded sample of reads recomputed one by one (cfg2's enumeration costs ~20 s per read and
    # is left to the full regeneration)
    gold = M.read(name)
    pairs = M.workloads(name)
    r = np.random.Generator(np.random.PCG64(31))
    for label, w in [pairs[int(i)] for i in r.choice(len(pairs), size=min(3, len(pairs)), replace=False)]:
        hdr, e, h = gold[label]
        P = oracle.Poly(w.problem)
        ids = np.sort(r.choice(w.n_reads, size=2, replace=False)).astype(np.uint32)
        z, en = P.anneal_reads(w.rule, M.schedule(P, w), ids, w.seed, w.instance_id)
        for j, i in enumerate(ids):
            assert int(en[j]) == int(e[i]) and oracle.state_hash(z[j]) == int(h[i]), (label, int(i))
