"""Read-by-read comparison of GPU runs with the oracle, at the parity bar of the tests.

A read is identical when its final state and tracked energy are equal on both sides.  Both sides
follow the same Philox stream and exact integer energy differences, so reads can part only where
floating point decides: an acceptance threshold exp(-beta dE), or a heat-bath cumulative weight
C_v against U * total, whose last bits depend on the exponential routine and (heat bath) on the
order in which the weights are added.  The bar: at least 99.9 % of the compared reads identical,
and every read that parts is traced to its first sweep (per-sweep state hashes) and variable (the
first differing value after that sweep), where the oracle's decision must lie within rounding of
a flip.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle

# a parted update's decision must lie this close to a flip (relative to the heat-bath total, or
# absolute against the acceptance probability): a few units in the last place of the sums
FLIP_MARGIN = 1e-12


def say(*a):
    print("[parity]", *a, flush=True)


def allowed_partings(n_reads: int) -> int:
    """Reads that may part at the 99.9 % bar."""
    return int(math.floor(0.001 * n_reads))


def r_of(s: int, n_sweeps: int, otm_r: float) -> float:
    if otm_r >= 0:
        return otm_r
    return s / (n_sweeps - 1) if n_sweeps > 1 else 0.0


def localise(P, rule, beta, seed, instance_id, read, gpu_hashes, gpu_after_sweep, otm_r=-1.0):
    """First (sweep, variable) at which read `read` parts, with the oracle's view of that update.

    gpu_hashes: the GPU's state hash after every sweep of this read.  gpu_after_sweep(s, z): the
    GPU's state of this read after sweep s started from state z.  Returns None when the hashes
    never differ (then the parting is not a floating-point decision)."""
    S = len(beta)
    _, _, h = P.anneal_reads(rule, beta, [read], seed, instance_id, otm_r=otm_r, trace=True)
    diff = np.nonzero(np.asarray(gpu_hashes, np.uint64) != h[0])[0]
    if diff.size == 0:
        return None
    s = int(diff[0])
    zb, _ = P.anneal_reads(rule, beta, [read], seed, instance_id, otm_r=otm_r, s_end=s)
    za, _ = P.anneal_reads(rule, beta, [read], seed, instance_id, otm_r=otm_r, s_begin=s, s_end=s + 1,
                           z_init=zb)
    zg = np.asarray(gpu_after_sweep(s, zb[0]))
    bad = np.nonzero(zg != za[0])[0]
    if bad.size == 0:
        return None
    k = int(bad[0])
    z_at = zb[0].copy()
    z_at[:k] = za[0][:k]
    info = P.explain_step(rule, z_at, k, s, read, beta[s], r_of(s, S, otm_r), seed, instance_id)
    info.update(sweep=s, var=k, gpu_v=int(zg[k]), oracle_v=int(za[0][k]))
    return info


def check(label, n_reads, same, explain=None):
    """same(i): read i identical on both sides.  explain(i): localise's record for a parted read.
    Fails unless >= 99.9 % of the reads are identical and each parted read is a rounding-level
    decision."""
    parted = [i for i in range(n_reads) if not same(i)]
    say(label, f"{n_reads - len(parted)}/{n_reads} reads identical")
    if not parted:
        return parted
    notes = []
    for i in parted[:8]:
        info = explain(i) if explain else None
        notes.append((i, info))
        say(label, "read", i, "parted:", info)
    if len(parted) > allowed_partings(n_reads):
        pytest.fail(f"{label}: {len(parted)}/{n_reads} reads part (at most {allowed_partings(n_reads)} "
                    f"allowed); first: {notes[:3]}")
    for i, info in notes:
        if info is None or not (info["margin"] < FLIP_MARGIN):
            pytest.fail(f"{label}: read {i} parts at a decision that is not within rounding: {info}")
    return parted


def state_hashes(z) -> np.ndarray:
    """The oracle's state hash of every row of z."""
    z = np.ascontiguousarray(z, np.int32)
    return np.array([oracle.state_hash(row) for row in z], np.uint64)
