"""Brute-force helpers for the tests: exact Python-integer arithmetic straight from the raw
(unmerged) terms of a problem.  They share nothing with either implementation."""
import itertools
import math

import numpy as np


def energy_raw(problem, z):
    """E(z) = sum over raw terms of coef * prod z[f] (Python big integers)."""
    E = 0
    for c, fs in problem.terms():
        prod = c
        for f in fs:
            prod *= int(z[f])
        E += prod
    return E


def all_states(problem):
    ranges = [range(int(l), int(u) + 1) for l, u in zip(problem.lower, problem.upper)]
    return itertools.product(*ranges)


def ground_energy(problem):
    return min(energy_raw(problem, z) for z in all_states(problem))


def boltzmann(problem, beta):
    """Exact Boltzmann distribution over all states: (states list, probabilities array)."""
    states = list(all_states(problem))
    E = np.array([energy_raw(problem, z) for z in states], dtype=np.float64)
    w = np.exp(-beta * (E - E.min()))
    return states, w / w.sum()


def deltas(problem, z, k):
    """dE(v) = E(z with z_k = v) - E(z) for every v in [l_k, u_k] (brute force)."""
    z = list(int(x) for x in z)
    e0 = energy_raw(problem, z)
    out = {}
    for v in range(int(problem.lower[k]), int(problem.upper[k]) + 1):
        z2 = list(z)
        z2[k] = v
        out[v] = energy_raw(problem, z2) - e0
    return out


def chi2_pvalue(observed_counts, expected_probs, min_expected=5.0):
    """Pearson chi-square p-value, pooling cells with small expectation into one cell."""
    from scipy import stats
    obs = np.asarray(observed_counts, np.float64)
    prob = np.asarray(expected_probs, np.float64)
    if np.any(obs[prob <= 0] > 0):
        return 0.0
    obs = obs[prob > 0]
    prob = prob[prob > 0]
    n = obs.sum()
    exp = prob * n
    big = exp >= min_expected
    o = list(obs[big])
    e = list(exp[big])
    if (~big).any():
        o.append(obs[~big].sum())
        e.append(exp[~big].sum())
    o = np.array(o)
    e = np.array(e)
    if len(o) < 2:
        return 1.0
    e = e * (o.sum() / e.sum())
    return float(stats.chisquare(o, e).pvalue)
