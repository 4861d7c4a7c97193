#!/usr/bin/env python3
"""Writes the oracle's results for the full-size measured workloads (tests/golden/full_size_*.txt).

Calls only the oracle (oracle/) and the seeded input generators; nothing here touches the GPU
library.  Each file records, per read, the tracked final energy and the state hash of the final
state (sum_k mix(k 2^32 + z_k) modulo 2^64, oracle.state_hash), together with the sha256 of the
oracle source and of the inverse-temperature array it was made with, so that a stale file is
detected (tests/test_golden_files.py).

    python tests/golden/make_full_size.py cfg2 cfg2-closed cfg3-otm cfg3-metropolis cfg4 cfg5
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2511_17245_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# problems of the 512-problem batch whose reads are all recomputed (a seeded sample)
CFG4_SAMPLE = 40
# requests of the serving stream recomputed, with their sweep counts cut so that the oracle's work
# stays within minutes: HUIO requests run 100 sweeps, dense heat-bath requests 2
CFG5_REQUESTS = 64
CFG5_SWEEPS = {"A": 100, "B": 2}


def oracle_sha() -> str:
    with open(os.path.join(ROOT, "oracle", "sa_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def beta_sha(beta) -> str:
    return hashlib.sha256(np.ascontiguousarray(beta, np.float64).tobytes()).hexdigest()


def cfg4_sample():
    items = I.cfg4_batch()
    r = np.random.Generator(np.random.PCG64(0x5A0004))
    ids = np.sort(r.choice(len(items), size=CFG4_SAMPLE, replace=False))
    return items, [int(i) for i in ids]


def cfg5_workloads():
    out = []
    for rid in range(CFG5_REQUESTS):
        w = I.cfg5_request(rid)
        kind = w.name.split()[-1]
        w.n_sweeps = CFG5_SWEEPS[kind]
        out.append(w)
    return out


def workloads(name):
    """(label, workload) pairs of a configuration, as the tests run them."""
    if name == "cfg2":
        return [("cfg2", I.cfg2_sparse_quio())]
    if name == "cfg2-closed":
        w = I.cfg2_sparse_quio()
        w.rule = I.RULES["heat_bath_closed"]
        return [("cfg2-closed", w)]
    if name in ("cfg3-otm", "cfg3-metropolis"):
        return [(name, I.cfg3_huio(rule=name.split("-")[1]))]
    if name == "cfg4":
        items, ids = cfg4_sample()
        return [(f"cfg4-item{i}", items[i]) for i in ids]
    if name == "cfg5":
        return [(f"cfg5-req{w.instance_id}", w) for w in cfg5_workloads()]
    raise SystemExit(f"unknown configuration {name}")


def schedule(P, w):
    return w.beta if w.beta is not None else P.schedule(w.n_sweeps)[0]


def write(name):
    path = os.path.join(HERE, f"full_size_{name}.txt")
    lines = [f"# oracle results for {name}: per read, tracked final energy and final-state hash",
             f"# command: python tests/golden/make_full_size.py {name}",
             f"# oracle sha256 {oracle_sha()}"]
    for label, w in workloads(name):
        t0 = time.time()
        P = oracle.Poly(w.problem)
        beta = schedule(P, w)
        z, e = P.anneal(w.rule, beta, w.n_reads, w.seed, w.instance_id, cache_mode=1)
        assert all(int(e[i]) == P.energy(z[i]) for i in range(w.n_reads))
        lines.append(f"workload {label} rule {w.rule} reads {w.n_reads} sweeps {w.n_sweeps} seed {w.seed} "
                     f"instance {w.instance_id} n {w.problem.n_vars} beta_sha256 {beta_sha(beta)}")
        for i in range(w.n_reads):
            lines.append(f"{i} {int(e[i])} {oracle.state_hash(z[i]):016x}")
        print(f"{label}: {w.n_reads} reads in {time.time() - t0:.1f} s", flush=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read(name):
    """{label: (header dict, energies int64[reads], hashes uint64[reads])} of a stored file."""
    path = os.path.join(HERE, f"full_size_{name}.txt")
    out, cur = {}, None
    meta = {}
    with open(path) as f:
        for line in f:
            if line.startswith("# oracle sha256"):
                meta["oracle_sha256"] = line.split()[-1]
            elif line.startswith("#"):
                continue
            elif line.startswith("workload"):
                tok = line.split()
                hdr = dict(zip(tok[2::2], tok[3::2]))
                hdr.update(meta)
                cur = tok[1]
                out[cur] = (hdr, [], [])
            else:
                i, e, h = line.split()
                out[cur][1].append(int(e))
                out[cur][2].append(int(h, 16))
    return {k: (h, np.array(e, np.int64), np.array(hs, np.uint64)) for k, (h, e, hs) in out.items()}


if __name__ == "__main__":
    for n in sys.argv[1:]:
        write(n)
